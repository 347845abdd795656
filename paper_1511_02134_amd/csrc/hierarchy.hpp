// Host-side construction of the refined hierarchy: mesh validation, per-macro
// layout, interface vertices (face / edge / corner primitives) with their
// neighbour tables and stencils, workgroup tile tables and the level-0
// system.  Pure C++; the device upload lives in hhg.hip.
#pragma once
#include <array>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/hhg.h"
#include "hhg_internal.hpp"

namespace hhg {

struct MacroInfo {
    int o[3];        // origin (integer macro coordinates of vertex 0)
    int ax[3];       // Kuhn path axes a, b, c
    double nu;
    int8_t bc[4];    // tag of the face opposite vertex f
    // linear part of the macro's affine map from lattice to physical
    // coordinates: a lattice displacement d moves the point by F d (identity
    // on Kuhn lattices without physical coordinates)
    double F[3][3];
};

struct MeshInfo {
    std::vector<MacroInfo> macros;
    int ext[3];      // bounding box extents (macro units), origin at 0
    bool project;    // pressure has a null space (no natural face)
    bool slip = false;   // some face is free-slip (tag 3)
    bool general;    // physical coordinates given: general 15-point A and C
    bool holes;      // some lattice points of the bounding box lie in no macro
    // the coupled velocity blocks of the records (ST_A2, ST_DINV) hold the
    // Laplace form delta_kl A: general meshes with a_1 run the point-block
    // velocity kernels, which read every tap
    bool lap_blocks = false;
};

bool validate_mesh(const hhg_mesh* mesh, MeshInfo* out, std::string* err);

// (macro, zero-pattern of the barycentric coordinates) of every macro closure
// that contains a vertex; vertices with equal keys have equal stencils and
// equal neighbour routing.
using Key = std::vector<std::pair<int32_t, int32_t>>;

struct HostLevel {
    int R = 0, n = 0, nm = 0;
    int64_t mstride = 0, len = 0;
    int lat[3] = {0, 0, 0};
    int64_t N = 0;
    std::vector<int32_t> slab_base;
    std::vector<Tile> vtiles, ctiles;
    // interface vertices, sorted by (colour, Dirichlet flag, primary slot)
    int32_t nif = 0;
    std::vector<int32_t> if_self, if_nb, if_sid, if_cptr, if_copy, if_flag;
    std::vector<int64_t> if_lat;
    int32_t col_start[5] = {0, 0, 0, 0, 0};
    int32_t vel_end[4] = {0, 0, 0, 0};
    int32_t slip_beg[4] = {0, 0, 0, 0};   // first free-slip vertex of colour c
    std::vector<Key> keys;                 // interface stencil id - nm -> key
    std::vector<double> st;                // (nm + keys) * ST_SIZE
    std::vector<double> st_vol_global;     // nm * ST_SIZE, volume stencils in global order
    std::vector<double> gst;               // nm * 16 * GR_SIZE
    std::vector<int32_t> slot_node;        // [len] lattice node or -1 (padding)
    std::vector<int32_t> node_slot;        // [N] primary slot
    std::vector<int32_t> node_sid;         // [N] stencil id (interface) or -(m+1) (volume of m)
    std::vector<int8_t> node_dir;          // [N] velocity Dirichlet
    std::vector<int8_t> node_slip;         // [N] free-slip (velocity tangential)
    std::vector<int32_t> rif_fine;         // [nif] index in the finer level's interface list
    // [15][nif] fine slots that the restriction sums at each interface vertex:
    // the coincident vertex, then its 14 neighbours (-1 where the finer
    // level's neighbour table points back at the vertex: no neighbour)
    std::vector<int32_t> rif_tap;
    // compact mirror of x: entries 0..nif-1 are the interface vertices (in
    // list order), entries nif.. the volume vertices they couple to (halo)
    int32_t ncomp = 0;
    std::vector<int32_t> if_tap;           // [14][nif] mirror index of each neighbour
    std::vector<int32_t> halo_slot;        // [ncomp - nif] slot of each halo vertex
    std::vector<int32_t> comp_of_slot;     // [len] mirror index of a slot or -1
    // hybrid ordering (primitive classes, Section 3.4): interface vertices
    // grouped by class (0 macro vertex, 1 edge, 2 face) and colour, the
    // velocity-free ones and all of them; hyb_off[12 * kind + 4 * class +
    // colour] .. [+1] delimit a group in hyb_list (kind 0 velocity, 1
    // pressure); hyb_mask[t] bit g-1: tap g reaches another primitive of t's
    // class (read from the class's starting values)
    std::vector<int32_t> hyb_list;
    int32_t hyb_off[26] = {0};
    std::vector<int32_t> hyb_mask;
    int64_t nfree = 0;                     // free velocity vertices
    int64_t nnodes = 0;                    // vertices (N minus the lattice points of a hole)
};

// Slot of macro-local vertex (i, j, k): tetrahedral slabs k; slab k (m = n-k)
// holds rows j = 0..m of Q_j = ceil((m+1-j)/4) quads, split by i mod 4 into
// four sub-arrays of S = sum_j Q_j entries, each listing the even rows, then
// the odd rows (the device kernels address it with the same formulas).
inline int32_t R4(int32_t L) {
    int32_t a = L >> 2, b = L & 3;
    return 4 * (a + 1) * (2 * a + b);
}
inline int32_t parity_prefix_h(int32_t m, int32_t j) {
    const int32_t J = j >> 1, A = m + 4 - (j & 1);
    const int32_t E = (J + 1) >> 1, O = J >> 1;
    return E * (A >> 2) - ((E * (E - 1)) >> 1) + O * ((A - 2) >> 2) - ((O * (O - 1)) >> 1);
}
inline int32_t row_off_h(int32_t m, int32_t j) {
    return (j & 1) ? parity_prefix_h(m, ((m >> 1) << 1) + 2) + parity_prefix_h(m, j)
                   : parity_prefix_h(m, j);
}
inline int64_t local_slot(const HostLevel& L, int m, int i, int j, int k) {
    int mm = L.n - k;
    return (int64_t)m * L.mstride + L.slab_base[k] + row_off_h(mm, j) + (i & 3) * (R4(mm + 1) >> 2) +
           (i >> 2);
}

bool build_level(const MeshInfo& mi, int R, int block_order, HostLevel* out, std::string* err);
bool compute_stencils(const MeshInfo& mi, HostLevel* L, std::string* err);
void link_levels(HostLevel* coarse, const HostLevel& fine);

// Level-0 system in compact numbering: free velocity vertices x 3, then the
// pressure of every vertex.  Vertices are numbered in lattice order, skipping
// the lattice points of a hole.
struct CoarseHost {
    int32_t nfv = 0, N = 0, nd = 0;
    std::vector<int32_t> node_lat;  // [N] lattice index of each vertex
    std::vector<int32_t> rowptr, col;
    std::vector<double> val;
    std::vector<double> ainv;       // [nfv][nfv] inverse of the free-free A block
    std::vector<double> pdinv;      // [N] 1 / (sum |T|/4/nu_T)
    std::vector<double> sinv;       // [N][N] inverse of the Schur complement
                                    // B A^-1 B^T + C (+ a rank-one term on the
                                    // pressure null space), symmetric
    // direct solver: the level-0 matrix bordered by the mean constraint
    // sum_i m_i p_i = 0 when the pressure has a null space, [nb][nb] row
    // major, nb = nd (+ 1); the device inverts it at set-up
    int32_t nb = 0;
    std::vector<double> kb;
    std::vector<double> a2inv;      // D form: [3 nfv][3 nfv] inverse of the coupled
                                    // free velocity block
    std::vector<double> mass;       // [N] int phi_i
    std::vector<int32_t> vel_node;  // [nfv] vertex of each compact velocity vertex
    int32_t nslip = 0;              // free-slip vertices among them
    std::vector<int32_t> node_slot; // [N]
    std::vector<int32_t> node_cptr, node_copy;   // every slot of each vertex
};
constexpr int COARSE_DIRECT_MAX = 16384;   // level-0 unknowns (the staged b0 of the direct solve fits the LDS)
// direct: the bordered matrix (kb); schur: the dense Schur complement
// inverse (sinv) of the MINRES preconditioner; dform: coupled velocity rows
bool build_coarse(const MeshInfo& mi, const HostLevel& L0, bool direct, bool schur, bool dform,
                  CoarseHost* out, std::string* err);

}  // namespace hhg
