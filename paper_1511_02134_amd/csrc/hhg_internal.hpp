// Internal data structures of the hierarchy shared by the host builder and the
// device kernels.  Not part of the public ABI.
#pragma once
#include <cstdint>

namespace hhg {

// --- stencil record ----------------------------------------------------------
// One record per (level, stencil id).  Taps: index 0 is the centre, 1..14 the
// neighbours.  Volume stencils (id < number of macros) use the macro-local
// offset order below; interface stencils use the global direction order.
// All blocks come from the P1 element matrices of Section 2.1 summed over the
// fine tetrahedra around the vertex:
//   A     a_1 (viscosity weighted), scalar block of the velocity
//   C     c_l (PSPG, delta h_T^2 / nu_T)
//   M     consistent mass
//   B_k   pressure row, velocity column component k:  b(phi_y e_k, phi_x)
//   BT_k  velocity row component k, pressure column:   b(phi_x e_k, phi_y)
//   G_k   pressure row, forcing column component k:    g_l for f = phi_y e_k
//   GT_k  forcing row component k, pressure column (transpose of G_k)
constexpr int ST_A = 0;
constexpr int ST_C = 15;
constexpr int ST_M = 30;
constexpr int ST_B = 45;
constexpr int ST_BT = 90;
constexpr int ST_G = 135;
constexpr int ST_GT = 180;
constexpr int ST_INVA = 225;   // 1 / A[0]
constexpr int ST_INVC = 226;   // 1 / C[0]
constexpr int ST_MASS = 227;   // int phi_x (row sum of M)
constexpr int ST_MASSNU = 228; // sum over the tetrahedra T around x of (|T|/4) / nu_T
// D form a_2 = 2 <nu D(u), D(v)>: the velocity block couples the components;
// block (k, l) of 15 taps at ST_A2 + 15 (3 k + l) is delta_kl A + E^{kl} with
// E^{kl} = sum_T nu_T |T| d_l phi_x d_k phi_y (x the row vertex, y the tap),
// and the inverse of the 3x3 centre block (row major) follows.
constexpr int ST_A2 = 232;
constexpr int ST_DINV = 367;
// mass-conservative normal of a free-slip vertex (Section 6.1): -(B^T 1)
// over the record's velocity rows, normalised (interface records; zero where
// B^T 1 vanishes)
constexpr int ST_NRM = 376;
constexpr int ST_SIZE = 379;

// Per-macro one-sided stencils for the viscosity gradient: the part of A, C
// and G that comes from the fine tetrahedra of one macro only, at unit
// viscosity, for each of the 16 zero-patterns of the barycentric coordinates
// (bit z set <=> lambda_z = 0; pattern 0 = interior), macro-local order.
constexpr int GR_A = 0;
constexpr int GR_C = 15;
constexpr int GR_G = 30;
constexpr int GR_A2 = 75;      // D form: the 9 coupled blocks of a_2 (block (k, l) at 15 (3 k + l))
constexpr int GR_SIZE = 210;

// Local offsets (di, dj, dk) of the 14 neighbours in macro index space, where
// a vertex (i, j, k) of a macro with origin O and Kuhn path axes (a, b, c) is
// O + (i+j+k) e_a + (j+k) e_b + k e_c.
//   1 ( 1, 0, 0) = +e_a        2 (-1, 0, 0) = -e_a
//   3 (-1, 1, 0) = +e_b        4 ( 1,-1, 0) = -e_b
//   5 ( 0, 1, 0) = +e_a+e_b    6 ( 0,-1, 0) = -(e_a+e_b)
//   7 ( 0,-1, 1) = +e_c        8 ( 0, 1,-1) = -e_c
//   9 (-1, 0, 1) = +e_b+e_c   10 ( 1, 0,-1) = -(e_b+e_c)
//  11 ( 0, 0, 1) = +e_a+e_b+e_c  12 ( 0, 0,-1)
//  13 ( 1,-1, 1) = +e_a+e_c   14 (-1, 1,-1)
// A and C couple only +-e_a, +-e_b, +-e_c (taps 1,2,3,4,7,8) on Kuhn meshes.
// Global direction order (interface stencils and neighbour tables):
//   1 +x  2 -x  3 +y  4 -y  5 +z  6 -z  7 +(x+y)  8 -(x+y)  9 +(y+z)
//  10 -(y+z)  11 +(x+z)  12 -(x+z)  13 +(x+y+z)  14 -(x+y+z)
// A and C couple only taps 1..6 in this order.

// Volume tile: one 256-lane workgroup over the fold of a slab of one macro.
struct Tile {
    int32_t macro;  // < 0: empty tile (XCD padding)
    int32_t k;      // slab
    int32_t t0;     // first lane of the tile in the slab's fold
    int32_t W;      // fold width (quads per row pair)
    int32_t nat;    // index in natural (macro, slab, lane) order; reductions
                    // write their partial sums there, so sums do not depend
                    // on the workgroup order
};

// Device view of one level (all pointers into the workspace).
template <typename T>
struct LevelDev {
    int32_t n;             // 2^R
    int32_t nm;            // macros
    int64_t mstride;       // slots per macro
    int64_t len;           // nm * mstride (values per field)
    const int32_t* slab_base;  // [n+2]
    const Tile* vtiles;    // interior tiles (launch order)
    int32_t n_vtiles;      // including padding
    int32_t nv_nat;        // interior tiles without padding (partials of the
                           // interface blocks follow them)
    const Tile* ctiles;    // closure tiles (launch order)
    int32_t n_ctiles;
    // interface vertices (every vertex on a macro face, edge or corner)
    int32_t nif;
    const int32_t* if_self;  // [nif] primary slot
    const int32_t* if_nb;    // [14][nif] neighbour slots (global direction order)
    const int32_t* if_sid;   // [nif] stencil id
    const int32_t* if_cptr;  // [nif+1]
    const int32_t* if_copy;  // all slots of the vertex
    const int32_t* if_flag;  // bit 0: velocity Dirichlet, bit 1: free-slip (u . n = 0)
    int32_t col_start[5];    // interface range of each colour
    int32_t vel_end[4];      // end of velocity-free vertices inside colour c
    int32_t slip_beg[4];     // start of the free-slip vertices inside colour c
                             // (free, Dirichlet and free-slip vertices follow
                             // each other in every colour)
    const T* st;             // stencil records
    const T* gst;            // gradient one-sided stencils [nm][16][GR_SIZE]
    // restriction of coarse interface vertices (this level as the coarse one):
    // [15][nif] fine slots summed at each vertex, the coincident one first
    // (-1: no neighbour in that direction)
    const int32_t* rif_tap;
    const T* macro_nu;       // [nm]
    // compact mirror of the smoothed iterate x: interface vertices (list
    // order) then their volume neighbours; field f of entry e is cx[f * cstride + e]
    int32_t ncomp;
    int64_t cstride;
    const int32_t* if_tap;       // [14][nif] mirror index of each neighbour
    const int32_t* halo_slot;    // [ncomp - nif]
    const int32_t* comp_of_slot; // [len] mirror index of a slot or -1
    T* cx;
};

}  // namespace hhg
