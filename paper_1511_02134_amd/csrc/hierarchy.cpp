// Host-side construction of the refined hierarchy (see hierarchy.hpp).
//
// Geometry.  Every macro is a Kuhn tetrahedron v0, v0+e_a, v0+e_a+e_b,
// v0+e_a+e_b+e_c of the integer lattice.  Uniform 1->8 refinement (Section
// 2.1) of such a tetrahedron R times produces the Kuhn triangulation of the
// lattice with spacing 2^-R restricted to the macro; a refined vertex with
// barycentric coordinates (n-i-j-k, i, j, k)/n, n = 2^R, is stored at the
// macro-local index (i, j, k).  The stencils are the P1 element matrices of
// a_1, b, c_l and g_l (Section 2.1) summed over the 24 lattice tetrahedra
// around a vertex, each weighted with the viscosity of the macro it lies in.
#include "hierarchy.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

namespace hhg {

namespace {

constexpr double DELTA = 1.0 / 12.0;  // PSPG parameter delta_T (Section 2.1)

// global direction order (see hhg_internal.hpp)
const int GDIR[15][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                         {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {0, 1, 1},
                         {0, -1, -1}, {1, 0, 1},  {-1, 0, -1}, {1, 1, 1},  {-1, -1, -1}};
// macro-local offsets (di, dj, dk)
const int LOFF[15][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {-1, 1, 0}, {1, -1, 0},
                         {0, 1, 0},  {0, -1, 0}, {0, -1, 1}, {0, 1, -1}, {-1, 0, 1},
                         {1, 0, -1}, {0, 0, 1},  {0, 0, -1}, {1, -1, 1}, {-1, 1, -1}};

int gdir_index(int dx, int dy, int dz) {
    for (int g = 0; g < 15; ++g)
        if (GDIR[g][0] == dx && GDIR[g][1] == dy && GDIR[g][2] == dz) return g;
    return -1;
}

// global vector of a macro-local offset
void local_to_vec(const MacroInfo& m, const int l[3], int v[3]) {
    v[0] = v[1] = v[2] = 0;
    v[m.ax[0]] += l[0] + l[1] + l[2];
    v[m.ax[1]] += l[1] + l[2];
    v[m.ax[2]] += l[2];
}

// change of the barycentric coordinates (lambda_0..3, in lattice units) of a
// macro under the global displacement d (integer or fractional)
void dlambda(const MacroInfo& m, const double d[3], double dl[4]) {
    double da = d[m.ax[0]], db = d[m.ax[1]], dc = d[m.ax[2]];
    dl[0] = -da;
    dl[1] = da - db;
    dl[2] = db - dc;
    dl[3] = dc;
}

// local (i,j,k) of global lattice point X in macro m at level n; false if X is
// outside the macro closure
bool global_to_local(const MacroInfo& m, int n, const int X[3], int* i, int* j, int* k) {
    int D[3] = {X[0] - m.o[0] * n, X[1] - m.o[1] * n, X[2] - m.o[2] * n};
    int a = D[m.ax[0]], b = D[m.ax[1]], c = D[m.ax[2]];
    *k = c;
    *j = b - c;
    *i = a - b;
    return *i >= 0 && *j >= 0 && *k >= 0 && a <= n;
}

// gradients of the barycentric coordinates and volume of a tetrahedron
void tet_geom(const double P[4][3], double G[4][3], double* vol) {
    double J[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) J[r][c] = P[r + 1][c] - P[0][c];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    // x = P0 + J^T xi  =>  xi = J^-T (x - P0): grad xi_r = row r of J^-T = column r of J^-1
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) G[r + 1][c] = inv[c][r];
    for (int c = 0; c < 3; ++c) G[0][c] = -(G[1][c] + G[2][c] + G[3][c]);
    *vol = std::fabs(det) / 6.0;
}

// The 24 lattice tetrahedra around a vertex: for every cube corner offset e
// and axis permutation s, the Kuhn tetrahedron c, c+e_s0, c+e_s0+e_s1, c+1
// with c = X - e contains X iff e is one of its path points.
struct Incident {
    int off[4][3];   // vertex offsets relative to X (lattice units)
    int a;           // local index of X in the tetrahedron
};
std::vector<Incident> incident_tets() {
    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    std::vector<Incident> out;
    for (int s = 0; s < 6; ++s) {
        int path[4][3] = {{0, 0, 0}};
        for (int q = 1; q < 4; ++q) {
            for (int c = 0; c < 3; ++c) path[q][c] = path[q - 1][c];
            path[q][perms[s][q - 1]] += 1;
        }
        for (int a = 0; a < 4; ++a) {
            Incident t;
            t.a = a;
            for (int q = 0; q < 4; ++q)
                for (int c = 0; c < 3; ++c) t.off[q][c] = path[q][c] - path[a][c];
            out.push_back(t);
        }
    }
    return out;
}

// Adds the element contributions of one tetrahedron to the stencil record of
// its vertex a (global direction order).  nu_A multiplies a_1, wC the PSPG
// weight delta h_T^2 / nu_T is divided by nu_C.  F is the linear part of the
// affine map of the macro the tetrahedron lies in (lattice to physical).
void add_element(double* rec, const Incident& t, const double F[3][3], double h, double nuA,
                 double nuC, double nuM, bool full) {
    double P[4][3], G[4][3], vol;
    for (int q = 0; q < 4; ++q)
        for (int r = 0; r < 3; ++r)
            P[q][r] = (F[r][0] * t.off[q][0] + F[r][1] * t.off[q][1] + F[r][2] * t.off[q][2]) * h;
    tet_geom(P, G, &vol);
    const int a = t.a;
    const double h2 = std::pow(vol, 2.0 / 3.0);       // h_T^2, h_T = |T|^(1/3)
    const double wC = DELTA * h2 / nuC;
    for (int b = 0; b < 4; ++b) {
        int g = gdir_index(t.off[b][0], t.off[b][1], t.off[b][2]);
        double gg = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
        rec[ST_A + g] += nuA * vol * gg;
        rec[ST_C + g] += wC * vol * gg;
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l)
                rec[ST_A2 + 15 * (3 * k + l) + g] +=
                    nuA * vol * ((k == l ? gg : 0.0) + G[a][l] * G[b][k]);
        if (!full) {
            for (int k = 0; k < 3; ++k) rec[ST_G + 15 * k + g] += -wC * (vol / 4.0) * G[a][k];
            continue;
        }
        rec[ST_M + g] += vol / 20.0 * (a == b ? 2.0 : 1.0);
        for (int k = 0; k < 3; ++k) {
            rec[ST_B + 15 * k + g] += -(vol / 4.0) * G[b][k];
            rec[ST_BT + 15 * k + g] += -(vol / 4.0) * G[a][k];
            rec[ST_G + 15 * k + g] += -wC * (vol / 4.0) * G[a][k];
            rec[ST_GT + 15 * k + g] += -wC * (vol / 4.0) * G[b][k];
        }
    }
    if (full) {
        rec[ST_MASS] += vol / 4.0;
        rec[ST_MASSNU] += vol / 4.0 / nuM;
    }
}

// The coupled blocks of the Laplace form: block (k, l) = delta_kl A.
void laplace_blocks(double* rec) {
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l)
            for (int g = 0; g < 15; ++g) rec[ST_A2 + 15 * (3 * k + l) + g] = k == l ? rec[ST_A + g] : 0.0;
}

void finish_record(double* rec) {
    rec[ST_INVA] = rec[ST_A] != 0.0 ? 1.0 / rec[ST_A] : 0.0;
    rec[ST_INVC] = rec[ST_C] != 0.0 ? 1.0 / rec[ST_C] : 0.0;
    // inverse of the (symmetric positive definite) 3x3 centre block of A_2
    double m[3][3];
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) m[k][l] = rec[ST_A2 + 15 * (3 * k + l)];
    const double c00 = m[1][1] * m[2][2] - m[1][2] * m[2][1];
    const double c01 = m[1][2] * m[2][0] - m[1][0] * m[2][2];
    const double c02 = m[1][0] * m[2][1] - m[1][1] * m[2][0];
    const double det = m[0][0] * c00 + m[0][1] * c01 + m[0][2] * c02;
    double* inv = rec + ST_DINV;
    if (det == 0.0) {
        for (int q = 0; q < 9; ++q) inv[q] = 0.0;
        return;
    }
    const double id = 1.0 / det;
    inv[0] = c00 * id;
    inv[1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) * id;
    inv[2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) * id;
    inv[3] = c01 * id;
    inv[4] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) * id;
    inv[5] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) * id;
    inv[6] = c02 * id;
    inv[7] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) * id;
    inv[8] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) * id;
}

// global-order record -> macro-local order (blocks of 15 taps)
void to_local(const MacroInfo& m, const double* g, double* l, int nblocks) {
    int perm[15];
    for (int q = 0; q < 15; ++q) {
        int v[3];
        local_to_vec(m, LOFF[q], v);
        perm[q] = gdir_index(v[0], v[1], v[2]);
    }
    for (int b = 0; b < nblocks; ++b)
        for (int q = 0; q < 15; ++q) l[15 * b + q] = g[15 * b + perm[q]];
}

// A and C must couple only the axis directions (global taps 1..6); clears
// round-off on the others and reports a geometry error otherwise.
bool clean_axis_only(double* blk, std::string* err) {
    double scale = std::fabs(blk[0]);
    for (int g = 7; g < 15; ++g) {
        if (std::fabs(blk[g]) > 1e-12 * scale) {
            if (err) *err = "stencil couples non-axis neighbours (mesh is not a Kuhn lattice)";
            return false;
        }
        blk[g] = 0.0;
    }
    return true;
}

}  // namespace

// ---------------------------------------------------------------------------
bool validate_mesh(const hhg_mesh* mesh, MeshInfo* out, std::string* err) {
    if (!mesh || !mesh->xyz || !mesh->tet || !mesh->face_bc) {
        *err = "mesh or one of xyz/tet/face_bc is NULL";
        return false;
    }
    if (mesh->nv < 4 || mesh->nt < 1) {
        *err = "mesh needs nv >= 4 and nt >= 1";
        return false;
    }
    const int nv = mesh->nv, nt = mesh->nt;
    std::vector<std::array<int, 3>> V(nv);
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    for (int v = 0; v < nv; ++v)
        for (int c = 0; c < 3; ++c) {
            double x = mesh->xyz[3 * v + c];
            if (!std::isfinite(x) || x != std::floor(x) || std::fabs(x) > 1e6) {
                *err = "macro vertex coordinates must be integers";
                return false;
            }
            V[v][c] = (int)x;
        }
    out->macros.resize(nt);
    for (int t = 0; t < nt; ++t) {
        MacroInfo& m = out->macros[t];
        int id[4];
        for (int q = 0; q < 4; ++q) {
            id[q] = mesh->tet[4 * t + q];
            if (id[q] < 0 || id[q] >= nv) {
                *err = "tet vertex id out of range";
                return false;
            }
        }
        bool used[3] = {false, false, false};
        for (int q = 0; q < 3; ++q) {
            int d[3], nz = 0, ax = -1;
            for (int c = 0; c < 3; ++c) {
                d[c] = V[id[q + 1]][c] - V[id[q]][c];
                if (d[c] != 0) {
                    ++nz;
                    ax = c;
                }
            }
            if (nz != 1 || d[ax] != 1 || used[ax]) {
                *err = "tet " + std::to_string(t) +
                       " is not in Kuhn path order (consecutive vertices must differ by "
                       "distinct positive unit steps)";
                return false;
            }
            used[ax] = true;
            m.ax[q] = ax;
        }
        for (int c = 0; c < 3; ++c) {
            m.o[c] = V[id[0]][c];
            lo[c] = std::min(lo[c], m.o[c]);
            hi[c] = std::max(hi[c], m.o[c] + 1);
        }
        double nu = mesh->nu ? mesh->nu[t] : 1.0;
        if (!std::isfinite(nu) || nu <= 0.0) {
            *err = "viscosity must be finite and positive";
            return false;
        }
        // affine map to physical space: column ax[q] of F is the physical
        // edge from path vertex q to q + 1
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) m.F[r][c] = r == c ? 1.0 : 0.0;
        if (mesh->phys) {
            for (int q = 0; q < 3; ++q)
                for (int r = 0; r < 3; ++r) {
                    const double a = mesh->phys[3 * id[q + 1] + r], b = mesh->phys[3 * id[q] + r];
                    if (!std::isfinite(a) || !std::isfinite(b)) {
                        *err = "physical coordinates must be finite";
                        return false;
                    }
                    m.F[r][m.ax[q]] = a - b;
                }
            const double (*F)[3] = m.F;
            const double det = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                               F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                               F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
            if (!(det > 0.0)) {
                *err = "macro " + std::to_string(t) +
                       " is degenerate or inverted by its physical coordinates";
                return false;
            }
        }
        m.nu = nu;
        for (int f = 0; f < 4; ++f) {
            int8_t b = mesh->face_bc[4 * t + f];
            if (b < 0 || b > 3) {
                *err = "face_bc entries must be 0, 1, 2 or 3";
                return false;
            }
            m.bc[f] = b;
        }
    }
    for (int c = 0; c < 3; ++c) {
        if (lo[c] != 0) {
            *err = "mesh bounding box must start at the origin";
            return false;
        }
        out->ext[c] = hi[c];
    }
    // conforming: faces are shared by exactly two macros (tag 0) or lie on
    // the boundary (tag 1 or 2).  Without physical coordinates the macros
    // tile their bounding box (every Kuhn tetrahedron has volume 1/6) and the
    // boundary faces lie on its planes; with them the box may hold a hole.
    out->general = mesh->phys != nullptr;
    out->holes = false;
    if (!mesh->phys && (int64_t)nt != 6LL * out->ext[0] * out->ext[1] * out->ext[2]) {
        *err = "macro tetrahedra do not tile their bounding box";
        return false;
    }
    std::map<std::array<int, 3>, std::vector<std::pair<int, int>>> faces;
    for (int t = 0; t < nt; ++t)
        for (int f = 0; f < 4; ++f) {
            std::array<int, 3> k;
            int q = 0;
            for (int v = 0; v < 4; ++v)
                if (v != f) k[q++] = mesh->tet[4 * t + v];
            std::sort(k.begin(), k.end());
            faces[k].push_back({t, f});
        }
    bool natural = false;
    out->slip = false;
    for (auto& kv : faces) {
        auto& lst = kv.second;
        if (lst.size() > 2) {
            *err = "a face is shared by more than two macros";
            return false;
        }
        if (lst.size() == 2) {
            for (auto& tf : lst)
                if (out->macros[tf.first].bc[tf.second] != 0) {
                    *err = "an interior face is tagged as boundary";
                    return false;
                }
        } else {
            int t = lst[0].first, f = lst[0].second;
            int8_t b = out->macros[t].bc[f];
            if (b == 0) {
                *err = "a boundary face is tagged interior";
                return false;
            }
            if (b == 2) natural = true;
            if (b == 3) out->slip = true;
            // the face must lie in a plane of the bounding box
            bool onplane = false;
            for (int c = 0; c < 3 && !onplane; ++c)
                for (int val : {0, out->ext[c]}) {
                    bool all = true;
                    for (int vv : kv.first)
                        if (V[vv][c] != val) all = false;
                    if (all) onplane = true;
                }
            if (!onplane && !mesh->phys) {
                *err = "macro tetrahedra do not tile their bounding box (open face inside)";
                return false;
            }
        }
    }
    out->project = !natural;
    return true;
}

// ---------------------------------------------------------------------------
static std::vector<Tile> make_tiles(int n, int nm, bool interior, int order) {
    std::vector<Tile> tiles;
    for (int m = 0; m < nm; ++m) {
        int k0 = interior ? 1 : 0, k1 = interior ? n - 1 : n;
        for (int k = k0; k <= k1; ++k) {
            int mm = n - k;
            int jl = interior ? 1 : 0, jh = interior ? mm - 2 : mm;
            if (jh < jl) continue;
            int npairs = (jh - jl + 2) / 2;
            int W = 0;
            for (int p = 0; p < npairs; ++p) {
                int ja = jl + p, jb = jh - p;
                int w = (mm + 4 - ja) >> 2;
                if (jb > ja) w += (mm + 4 - jb) >> 2;
                W = std::max(W, w);
            }
            int lanes = npairs * W;
            for (int t0 = 0; t0 < lanes; t0 += 256)
                tiles.push_back({m, k, t0, W, (int32_t)tiles.size()});
        }
    }
    const int T = (int)tiles.size();
    if (order == 0 || T == 0) return tiles;
    std::vector<Tile> out;
    if (order == 2) {
        out.assign(tiles.rbegin(), tiles.rend());
        return out;
    }
    // XCD-aware: workgroup b runs on XCD b % 8; give every XCD a contiguous
    // range of tiles so that neighbouring slabs share that XCD's L2.
    const int T8 = (T + 7) / 8 * 8, chunk = T8 / 8;
    out.resize(T8);
    for (int b = 0; b < T8; ++b) {
        int t = (b % 8) * chunk + b / 8;
        out[b] = t < T ? tiles[t] : Tile{-1, 0, 0, 1, -1};
    }
    return out;
}

bool build_level(const MeshInfo& mi, int R, int block_order, HostLevel* out, std::string* err) {
    HostLevel& L = *out;
    L.R = R;
    L.n = 1 << R;
    L.nm = (int)mi.macros.size();
    const int n = L.n, nm = L.nm;
    L.slab_base.assign(n + 2, 0);
    for (int k = 0; k <= n; ++k) L.slab_base[k + 1] = L.slab_base[k] + R4(n - k + 1);
    L.mstride = ((int64_t)L.slab_base[n + 1] + 63) / 64 * 64;
    L.len = L.mstride * nm;
    for (int c = 0; c < 3; ++c) L.lat[c] = mi.ext[c] * n + 1;
    L.N = (int64_t)L.lat[0] * L.lat[1] * L.lat[2];
    // slot indices are 32-bit, and the stencil loads address a field with a
    // 32-bit byte offset (8-byte values)
    if (L.len >= (1LL << 29) || L.N >= (1LL << 31)) {
        *err = "problem too large for 32-bit slot offsets";
        return false;
    }
    L.slot_node.assign(L.len, -1);
    L.node_slot.assign(L.N, -1);
    L.node_sid.assign(L.N, 0);
    L.node_dir.assign(L.N, 0);
    L.node_slip.assign(L.N, 0);

    struct Ent {
        int64_t lat;
        int32_t macro, slot, i, j, k, pattern;
    };
    std::vector<Ent> ents;
    for (int m = 0; m < nm; ++m) {
        const MacroInfo& M = mi.macros[m];
        for (int k = 0; k <= n; ++k)
            for (int j = 0; j <= n - k; ++j)
                for (int i = 0; i <= n - k - j; ++i) {
                    int X[3] = {M.o[0] * n, M.o[1] * n, M.o[2] * n};
                    X[M.ax[0]] += i + j + k;
                    X[M.ax[1]] += j + k;
                    X[M.ax[2]] += k;
                    int64_t lat = X[0] + (int64_t)L.lat[0] * (X[1] + (int64_t)L.lat[1] * X[2]);
                    int64_t s = local_slot(L, m, i, j, k);
                    L.slot_node[s] = (int32_t)lat;
                    int pattern = (n - i - j - k == 0 ? 1 : 0) | (i == 0 ? 2 : 0) |
                                  (j == 0 ? 4 : 0) | (k == 0 ? 8 : 0);
                    if (pattern == 0) {
                        L.node_slot[lat] = (int32_t)s;
                        L.node_sid[lat] = -(m + 1);
                    } else {
                        ents.push_back({lat, m, (int32_t)s, i, j, k, pattern});
                    }
                }
    }
    std::sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) {
        return a.lat != b.lat ? a.lat < b.lat : a.macro < b.macro;
    });

    struct KeyInfo {
        int32_t id;
        int route[15];   // copy index that contains X + d_g, or -1
        bool dirichlet, slip;
    };
    std::map<Key, KeyInfo> keymap;
    L.keys.clear();

    struct Node {
        int64_t lat;
        int colour, flag, self, sid;
        int nb[14];
        std::vector<int32_t> copies;
    };
    std::vector<Node> nodes;
    for (size_t g0 = 0; g0 < ents.size();) {
        size_t g1 = g0;
        while (g1 < ents.size() && ents[g1].lat == ents[g0].lat) ++g1;
        Key key;
        for (size_t e = g0; e < g1; ++e) key.push_back({ents[e].macro, ents[e].pattern});
        auto it = keymap.find(key);
        if (it == keymap.end()) {
            KeyInfo ki;
            ki.id = (int32_t)L.keys.size();
            ki.dirichlet = ki.slip = false;
            for (auto& mp : key) {
                const MacroInfo& M = mi.macros[mp.first];
                for (int f = 0; f < 4; ++f) {
                    if ((mp.second >> f & 1) && M.bc[f] == 1) ki.dirichlet = true;
                    if ((mp.second >> f & 1) && M.bc[f] == 3) ki.slip = true;
                }
            }
            if (ki.dirichlet) ki.slip = false;   // no-slip wins where the faces meet
            for (int g = 0; g < 15; ++g) {
                ki.route[g] = -1;
                double d[3] = {(double)GDIR[g][0], (double)GDIR[g][1], (double)GDIR[g][2]};
                for (size_t c = 0; c < key.size() && ki.route[g] < 0; ++c) {
                    double dl[4];
                    dlambda(mi.macros[key[c].first], d, dl);
                    bool ok = true;
                    for (int z = 0; z < 4; ++z)
                        if ((key[c].second >> z & 1) && dl[z] < 0) ok = false;
                    if (ok) ki.route[g] = (int)c;
                }
            }
            it = keymap.emplace(key, ki).first;
            L.keys.push_back(key);
        }
        const KeyInfo& ki = it->second;
        Node nd;
        nd.lat = ents[g0].lat;
        int64_t lat = nd.lat;
        int X[3] = {(int)(lat % L.lat[0]), (int)((lat / L.lat[0]) % L.lat[1]),
                    (int)(lat / ((int64_t)L.lat[0] * L.lat[1]))};
        nd.colour = (X[0] + X[1] + X[2]) & 3;
        nd.flag = ki.dirichlet ? 1 : ki.slip ? 2 : 0;
        nd.self = ents[g0].slot;
        nd.sid = nm + ki.id;
        for (size_t e = g0; e < g1; ++e) nd.copies.push_back(ents[e].slot);
        for (int g = 1; g < 15; ++g) {
            int c = ki.route[g];
            if (c < 0) {
                nd.nb[g - 1] = nd.self;
                continue;
            }
            const Ent& E = ents[g0 + c];
            const MacroInfo& M = mi.macros[E.macro];
            int Y[3] = {X[0] + GDIR[g][0], X[1] + GDIR[g][1], X[2] + GDIR[g][2]};
            int i, j, k;
            if (!global_to_local(M, n, Y, &i, &j, &k)) {
                *err = "internal error: neighbour routing left the macro closure";
                return false;
            }
            nd.nb[g - 1] = (int32_t)local_slot(L, E.macro, i, j, k);
        }
        L.node_slot[lat] = nd.self;
        L.node_sid[lat] = nd.sid;
        L.node_dir[lat] = (int8_t)(nd.flag == 1);
        L.node_slip[lat] = (int8_t)(nd.flag == 2);
        nodes.push_back(std::move(nd));
        g0 = g1;
    }
    std::sort(nodes.begin(), nodes.end(), [](const Node& a, const Node& b) {
        if (a.colour != b.colour) return a.colour < b.colour;
        if (a.flag != b.flag) return a.flag < b.flag;
        if (a.sid != b.sid) return a.sid < b.sid;   // wave-uniform stencil records
        return a.self < b.self;
    });
    const int nif = (int)nodes.size();
    L.nif = nif;
    L.if_self.resize(nif);
    L.if_sid.resize(nif);
    L.if_flag.resize(nif);
    L.if_lat.resize(nif);
    L.if_nb.resize((size_t)14 * nif);
    L.if_cptr.assign(nif + 1, 0);
    L.if_copy.clear();
    for (int c = 0; c < 5; ++c) L.col_start[c] = nif;
    for (int c = 0; c < 4; ++c) L.vel_end[c] = -1;
    for (int t = 0; t < nif; ++t) {
        const Node& nd = nodes[t];
        L.if_self[t] = nd.self;
        L.if_sid[t] = nd.sid;
        L.if_flag[t] = nd.flag;
        L.if_lat[t] = nd.lat;
        for (int g = 0; g < 14; ++g) L.if_nb[(size_t)g * nif + t] = nd.nb[g];
        for (int32_t s : nd.copies) L.if_copy.push_back(s);
        L.if_cptr[t + 1] = (int32_t)L.if_copy.size();
        if (L.col_start[nd.colour] == nif) L.col_start[nd.colour] = t;
    }
    // colour ranges (colours with no vertex get empty ranges)
    for (int c = 3; c >= 0; --c)
        if (L.col_start[c] == nif || L.col_start[c] > L.col_start[c + 1])
            L.col_start[c] = L.col_start[c + 1];
    for (int c = 0; c < 4; ++c) {
        int e = L.col_start[c];
        while (e < L.col_start[c + 1] && L.if_flag[e] == 0) ++e;
        L.vel_end[c] = e;
        while (e < L.col_start[c + 1] && L.if_flag[e] == 1) ++e;
        L.slip_beg[c] = e;
    }
    // Compact mirror: interface vertices keep their list index; the volume
    // vertices they couple to follow.  Halo indices are handed out tap by tap
    // within each run of equal (colour, flag, stencil record), so the lanes of
    // a wave, which walk such a run in slot order, read one mirror run per tap.
    {
        std::vector<int32_t> comp(L.len, -1);
        for (int t = 0; t < nif; ++t)
            for (int q = L.if_cptr[t]; q < L.if_cptr[t + 1]; ++q) comp[L.if_copy[q]] = t;
        std::vector<int> colour_of(nif, 0);
        for (int c = 0; c < 4; ++c)
            for (int t = L.col_start[c]; t < L.col_start[c + 1]; ++t) colour_of[t] = c;
        L.if_tap.assign((size_t)14 * nif, 0);
        L.halo_slot.clear();
        int32_t next = nif;
        for (int g0 = 0; g0 < nif;) {
            int g1 = g0 + 1;
            while (g1 < nif && colour_of[g1] == colour_of[g0] && L.if_flag[g1] == L.if_flag[g0] &&
                   L.if_sid[g1] == L.if_sid[g0])
                ++g1;
            for (int g = 0; g < 14; ++g)
                for (int t = g0; t < g1; ++t) {
                    const int32_t sl = L.if_nb[(size_t)g * nif + t];
                    int32_t ci = comp[sl];
                    if (ci < 0) {
                        ci = next++;
                        comp[sl] = ci;
                        L.halo_slot.push_back(sl);
                    }
                    L.if_tap[(size_t)g * nif + t] = ci;
                }
            g0 = g1;
        }
        L.ncomp = next;
        L.comp_of_slot.swap(comp);
    }
    // hybrid ordering tables: the primitive of an interface vertex is its key
    // (all vertices of one macro vertex, edge or face share it); its class
    // follows from the number of vanishing barycentric coordinates
    {
        std::vector<int> cls(nif);
        for (int t = 0; t < nif; ++t) {
            const int pat = L.keys[L.if_sid[t] - nm][0].second;
            const int zeros = (pat & 1) + (pat >> 1 & 1) + (pat >> 2 & 1) + (pat >> 3 & 1);
            cls[t] = 3 - zeros;
        }
        L.hyb_list.clear();
        for (int kind = 0; kind < 2; ++kind)
            for (int k = 0; k < 3; ++k)
                for (int c = 0; c < 4; ++c) {
                    L.hyb_off[12 * kind + 4 * k + c] = (int32_t)L.hyb_list.size();
                    for (int t = L.col_start[c]; t < L.col_start[c + 1]; ++t)
                        if (cls[t] == k && (kind == 1 || L.if_flag[t] == 0)) L.hyb_list.push_back(t);
                }
        L.hyb_off[24] = (int32_t)L.hyb_list.size();
        L.hyb_off[25] = 0;
        L.hyb_mask.assign(std::max(nif, 1), 0);
        for (int t = 0; t < nif; ++t)
            for (int g = 0; g < 14; ++g) {
                const int32_t e = L.if_tap[(size_t)g * nif + t];
                if (e < nif && e != t && cls[e] == cls[t] && L.if_sid[e] != L.if_sid[t])
                    L.hyb_mask[t] |= 1 << g;
            }
    }
    L.nfree = 0;
    L.nnodes = 0;
    for (int64_t v = 0; v < L.N; ++v)
        if (L.node_slot[v] >= 0) {
            ++L.nnodes;
            if (!L.node_dir[v]) ++L.nfree;
        }
    // lattice points in no macro: a hole of a mesh with physical coordinates
    if (L.nnodes != L.N && !mi.general) {
        *err = "internal error: lattice node without a macro";
        return false;
    }
    L.vtiles = make_tiles(n, nm, true, block_order);
    L.ctiles = make_tiles(n, nm, false, block_order);
    return compute_stencils(mi, &L, err);
}

// An interior stencil of the Kuhn lattice is invariant under x -> -x of the
// offsets: in the local tap order the 14 neighbours come in opposite pairs
// (2q+1, 2q+2), and A, C and M are symmetric over a pair, B_k antisymmetric,
// and B^T_k(d) = B_k(-d).  Checked to round-off and then made exact, so that
// kernels may evaluate interior rows from pair sums and differences.
static bool pair_symmetries(double* r, std::string* err) {
    auto fail_sym = [&](const char* what) {
        *err = std::string("internal error: interior stencil not pair-symmetric (") + what + ")";
        return false;
    };
    for (int blk : {ST_A, ST_C, ST_M}) {
        double sc = 0.0;
        for (int g = 0; g < 15; ++g) sc = std::max(sc, std::fabs(r[blk + g]));
        for (int q = 0; q < 7; ++q) {
            double& a = r[blk + 2 * q + 1];
            double& b = r[blk + 2 * q + 2];
            if (std::fabs(a - b) > 1e-12 * sc) return fail_sym("A, C or M");
            a = b = 0.5 * (a + b);
        }
    }
    for (int f = 0; f < 3; ++f) {
        double* B = r + ST_B + 15 * f;
        double* BT = r + ST_BT + 15 * f;
        double sc = 0.0;
        for (int g = 0; g < 15; ++g) sc = std::max(sc, std::max(std::fabs(B[g]), std::fabs(BT[g])));
        if (B[0] != 0.0 || BT[0] != 0.0) return fail_sym("divergence centre");
        for (int q = 0; q < 7; ++q) {
            const int d = 2 * q + 1, e = 2 * q + 2;
            if (std::fabs(B[d] + B[e]) > 1e-12 * sc || std::fabs(BT[d] - B[e]) > 1e-12 * sc ||
                std::fabs(BT[e] - B[d]) > 1e-12 * sc)
                return fail_sym("B");
            const double v = 0.5 * (B[d] - B[e]);
            B[d] = v;
            B[e] = -v;
            BT[d] = -v;
            BT[e] = v;
        }
    }
    return true;
}

bool compute_stencils(const MeshInfo& mi, HostLevel* Lp, std::string* err) {
    HostLevel& L = *Lp;
    const int nm = L.nm, n = L.n;
    const double h = 1.0 / n;
    static const std::vector<Incident> inc = incident_tets();
    const size_t nst = nm + L.keys.size();
    L.st.assign(nst * ST_SIZE, 0.0);
    L.st_vol_global.assign((size_t)nm * ST_SIZE, 0.0);
    L.gst.assign((size_t)nm * 16 * GR_SIZE, 0.0);
    std::vector<double> g(ST_SIZE);
    // volume stencils: all 24 tetrahedra around an interior vertex lie in the macro
    for (int m = 0; m < nm; ++m) {
        const MacroInfo& M = mi.macros[m];
        std::fill(g.begin(), g.end(), 0.0);
        for (const Incident& t : inc) add_element(g.data(), t, M.F, h, M.nu, M.nu, M.nu, true);
        if (!mi.general && (!clean_axis_only(&g[ST_A], err) || !clean_axis_only(&g[ST_C], err)))
            return false;
        if (mi.lap_blocks) laplace_blocks(g.data());
        // at an interior vertex the B, B^T, G and G^T centre taps vanish
        // (the gradients of a basis function integrate to zero); clear the
        // round-off so the volume kernels may skip them
        for (int blk = ST_B; blk < ST_INVA; blk += 15) {
            double sc = 0.0;
            for (int q = 1; q < 15; ++q) sc = std::max(sc, std::fabs(g[blk + q]));
            if (std::fabs(g[blk]) > 1e-12 * sc) {
                *err = "internal error: non-zero centre tap of a divergence stencil";
                return false;
            }
            g[blk] = 0.0;
        }
        finish_record(g.data());
        std::copy(g.begin(), g.end(), L.st_vol_global.begin() + (size_t)m * ST_SIZE);
        double* loc = &L.st[(size_t)m * ST_SIZE];
        to_local(M, g.data(), loc, 15);   // A, C, M, B(3), BT(3), G(3), GT(3)
        for (int q = ST_INVA; q < ST_SIZE; ++q) loc[q] = g[q];
        to_local(M, g.data() + ST_A2, loc + ST_A2, 9);   // A_2 blocks
        if (!pair_symmetries(loc, err)) return false;
    }
    // interface stencils: every tetrahedron around the vertex belongs to the
    // macro whose closure contains its centroid strictly
    for (size_t kid = 0; kid < L.keys.size(); ++kid) {
        const Key& key = L.keys[kid];
        double* rec = &L.st[(nm + kid) * ST_SIZE];
        for (const Incident& t : inc) {
            double cen[3] = {0, 0, 0};
            for (int q = 0; q < 4; ++q)
                for (int c = 0; c < 3; ++c) cen[c] += 0.25 * t.off[q][c];
            for (auto& mp : key) {
                double dl[4];
                dlambda(mi.macros[mp.first], cen, dl);
                bool in = true;
                for (int z = 0; z < 4; ++z)
                    if ((mp.second >> z & 1) && dl[z] <= 0) in = false;
                if (in) {
                    const MacroInfo& M = mi.macros[mp.first];
                    add_element(rec, t, M.F, h, M.nu, M.nu, M.nu, true);
                    break;
                }
            }
        }
        if (!mi.general &&
            (!clean_axis_only(&rec[ST_A], err) || !clean_axis_only(&rec[ST_C], err)))
            return false;
        if (mi.lap_blocks) laplace_blocks(rec);
        finish_record(rec);
        // mass-conservative normal <grad phi_x, 1> = -(B^T 1)_x (Section 6.1)
        double nv[3], nn = 0.0;
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int g = 0; g < 15; ++g) acc += rec[ST_BT + 15 * k + g];
            nv[k] = -acc;
            nn += nv[k] * nv[k];
        }
        nn = std::sqrt(nn);
        double scale = 0.0;
        for (int g = 0; g < 15; ++g)
            for (int k = 0; k < 3; ++k) scale = std::max(scale, std::fabs(rec[ST_BT + 15 * k + g]));
        for (int k = 0; k < 3; ++k) rec[ST_NRM + k] = nn > 1e-12 * scale ? nv[k] / nn : 0.0;
    }
    // one-sided per-macro stencils at unit viscosity for the gradient
    for (int m = 0; m < nm; ++m) {
        const MacroInfo& M = mi.macros[m];
        for (int pat = 0; pat < 15; ++pat) {
            std::fill(g.begin(), g.end(), 0.0);
            for (const Incident& t : inc) {
                double cen[3] = {0, 0, 0};
                for (int q = 0; q < 4; ++q)
                    for (int c = 0; c < 3; ++c) cen[c] += 0.25 * t.off[q][c];
                double dl[4];
                dlambda(M, cen, dl);
                bool in = true;
                for (int z = 0; z < 4; ++z)
                    if ((pat >> z & 1) && dl[z] <= 0) in = false;
                if (in) add_element(g.data(), t, M.F, h, 1.0, 1.0, 1.0, false);
            }
            double* o = &L.gst[((size_t)m * 16 + pat) * GR_SIZE];
            to_local(M, &g[ST_A], o + GR_A, 1);
            to_local(M, &g[ST_C], o + GR_C, 1);
            to_local(M, &g[ST_G], o + GR_G, 3);
            to_local(M, &g[ST_A2], o + GR_A2, 9);
        }
    }
    return true;
}

void link_levels(HostLevel* coarse, const HostLevel& fine) {
    std::unordered_map<int64_t, int32_t> idx;
    idx.reserve(fine.nif * 2);
    for (int t = 0; t < fine.nif; ++t) idx[fine.if_lat[t]] = t;
    coarse->rif_fine.assign(coarse->nif, -1);
    for (int t = 0; t < coarse->nif; ++t) {
        int64_t lat = coarse->if_lat[t];
        int64_t X = lat % coarse->lat[0], Y = (lat / coarse->lat[0]) % coarse->lat[1],
                Z = lat / ((int64_t)coarse->lat[0] * coarse->lat[1]);
        int64_t lf = 2 * X + fine.lat[0] * (2 * Y + (int64_t)fine.lat[1] * 2 * Z);
        auto it = idx.find(lf);
        coarse->rif_fine[t] = it == idx.end() ? -1 : it->second;
    }
    const int nif = coarse->nif;
    coarse->rif_tap.assign((size_t)15 * std::max(nif, 1), -1);
    for (int t = 0; t < nif; ++t) {
        const int tf = coarse->rif_fine[t];
        if (tf < 0) continue;
        const int32_t self = fine.if_self[tf];
        coarse->rif_tap[t] = self;
        for (int g = 0; g < 14; ++g) {
            const int32_t nb = fine.if_nb[(size_t)g * fine.nif + tf];
            coarse->rif_tap[(size_t)(g + 1) * nif + t] = nb != self ? nb : -1;
        }
    }
}

// ---------------------------------------------------------------------------
// Inverse of a dense n x n matrix by Gauss-Jordan elimination with partial
// pivoting (row-major, in place); false if it is numerically singular.
static bool invert_dense(std::vector<double>& M, int n) {
    std::vector<int> perm(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    double scale = 0.0;
    for (double v : M) scale = std::max(scale, std::fabs(v));
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(M[(size_t)r * n + c]) > std::fabs(M[(size_t)piv * n + c])) piv = r;
        if (!(std::fabs(M[(size_t)piv * n + c]) > 1e-13 * scale)) return false;
        if (piv != c) {
            for (int q = 0; q < n; ++q) std::swap(M[(size_t)piv * n + q], M[(size_t)c * n + q]);
            std::swap(perm[piv], perm[c]);
        }
        double* rc = &M[(size_t)c * n];
        const double inv = 1.0 / rc[c];
        rc[c] = 1.0;
        for (int q = 0; q < n; ++q) rc[q] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double* rr = &M[(size_t)r * n];
            const double f = rr[c];
            if (f == 0.0) continue;
            rr[c] = 0.0;
            for (int q = 0; q < n; ++q) rr[q] -= f * rc[q];
        }
    }
    // the row swaps act on the columns of the inverse: undo them
    std::vector<double> out((size_t)n * n);
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) out[(size_t)r * n + perm[c]] = M[(size_t)r * n + c];
    M.swap(out);
    return true;
}

bool build_coarse(const MeshInfo& mi, const HostLevel& L, bool direct, bool schur, bool dform,
                  CoarseHost* out, std::string* err) {
    CoarseHost& C = *out;
    // vertices in lattice order (the lattice points of a hole are skipped)
    std::vector<int32_t> cidx(L.N, -1);
    C.node_lat.clear();
    for (int64_t v = 0; v < L.N; ++v)
        if (L.node_slot[v] >= 0) {
            cidx[v] = (int32_t)C.node_lat.size();
            C.node_lat.push_back((int32_t)v);
        }
    const int N = (int)C.node_lat.size();
    C.N = N;
    std::vector<int32_t> vidx(N, -1);
    C.vel_node.clear();
    C.nslip = 0;
    for (int v = 0; v < N; ++v)
        if (!L.node_dir[C.node_lat[v]]) {
            vidx[v] = (int32_t)C.vel_node.size();
            C.vel_node.push_back(v);
            if (L.node_slip[C.node_lat[v]]) ++C.nslip;
        }
    if (C.nslip > 0 && (!direct || schur || dform)) {
        *err = "free-slip boundaries need the direct coarse solver and the Laplace form";
        return false;
    }
    const int nfv = (int)C.vel_node.size();
    C.nfv = nfv;
    C.nd = 3 * nfv + N;
    if (C.nd > COARSE_DIRECT_MAX) {
        *err = "level-0 system too large (" + std::to_string(C.nd) + " unknowns, at most " +
               std::to_string(COARSE_DIRECT_MAX) + ")";
        return false;
    }
    auto rec_of = [&](int v) -> const double* {
        int sid = L.node_sid[C.node_lat[v]];
        if (sid < 0) return &L.st_vol_global[(size_t)(-sid - 1) * ST_SIZE];
        return &L.st[(size_t)sid * ST_SIZE];
    };
    // vertex next to v in direction g, or -1 (outside the box or in a hole,
    // where every tap of the record is zero)
    auto nbr = [&](int v, int g) -> int {
        const int lv = C.node_lat[v];
        int X = lv % L.lat[0], Y = (lv / L.lat[0]) % L.lat[1], Z = lv / (L.lat[0] * L.lat[1]);
        X += GDIR[g][0];
        Y += GDIR[g][1];
        Z += GDIR[g][2];
        if (X < 0 || Y < 0 || Z < 0 || X >= L.lat[0] || Y >= L.lat[1] || Z >= L.lat[2]) return -1;
        return cidx[X + L.lat[0] * (Y + L.lat[1] * Z)];
    };
    C.rowptr.assign(1, 0);
    C.col.clear();
    C.val.clear();
    std::vector<double> A((size_t)nfv * nfv, 0.0);
    auto push = [&](int c, double v) {
        if (v != 0.0) {
            C.col.push_back(c);
            C.val.push_back(v);
        }
    };
    for (int k = 0; k < 3; ++k)
        for (int iv = 0; iv < nfv; ++iv) {
            int v = C.vel_node[iv];
            const double* r = rec_of(v);
            for (int g = 0; g < 15; ++g) {
                int w = g == 0 ? v : nbr(v, g);
                if (w < 0) continue;
                if (vidx[w] >= 0) {
                    if (dform) {
                        // D form: the velocity rows couple all three components
                        for (int l = 0; l < 3; ++l)
                            push(l * nfv + vidx[w], r[ST_A2 + 15 * (3 * k + l) + g]);
                    } else {
                        push(k * nfv + vidx[w], r[ST_A + g]);
                    }
                    if (k == 0) A[(size_t)iv * nfv + vidx[w]] += r[ST_A + g];
                }
                push(3 * nfv + w, r[ST_BT + 15 * k + g]);
            }
            C.rowptr.push_back((int32_t)C.col.size());
        }
    for (int v = 0; v < N; ++v) {
        const double* r = rec_of(v);
        for (int g = 0; g < 15; ++g) {
            int w = g == 0 ? v : nbr(v, g);
            if (w < 0) continue;
            if (vidx[w] >= 0)
                for (int k = 0; k < 3; ++k) push(k * nfv + vidx[w], r[ST_B + 15 * k + g]);
            push(3 * nfv + w, -r[ST_C + g]);
        }
        C.rowptr.push_back((int32_t)C.col.size());
    }
    // dense inverse of the SPD free-free block of A by Cholesky (the MINRES
    // preconditioner and the velocity cycle's coarse solve; neither runs on
    // meshes with free-slip faces)
    C.ainv.clear();
    std::vector<double> Lc(mi.slip ? 0 : A.size());
    if (!mi.slip) Lc = A;
    for (int j = 0; j < (mi.slip ? 0 : nfv); ++j) {
        double d = Lc[(size_t)j * nfv + j];
        for (int q = 0; q < j; ++q) d -= Lc[(size_t)j * nfv + q] * Lc[(size_t)j * nfv + q];
        if (!(d > 0.0)) {
            *err = "coarse velocity block is not positive definite";
            return false;
        }
        d = std::sqrt(d);
        Lc[(size_t)j * nfv + j] = d;
        for (int i = j + 1; i < nfv; ++i) {
            double s = Lc[(size_t)i * nfv + j];
            for (int q = 0; q < j; ++q) s -= Lc[(size_t)i * nfv + q] * Lc[(size_t)j * nfv + q];
            Lc[(size_t)i * nfv + j] = s / d;
        }
    }
    if (!mi.slip) C.ainv.assign((size_t)nfv * nfv, 0.0);
    std::vector<double> y(nfv);
    for (int c = 0; c < (mi.slip ? 0 : nfv); ++c) {
        for (int i = 0; i < nfv; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int q = 0; q < i; ++q) s -= Lc[(size_t)i * nfv + q] * y[q];
            y[i] = s / Lc[(size_t)i * nfv + i];
        }
        for (int i = nfv - 1; i >= 0; --i) {
            double s = y[i];
            for (int q = i + 1; q < nfv; ++q) s -= Lc[(size_t)q * nfv + i] * C.ainv[(size_t)q * nfv + c];
            C.ainv[(size_t)i * nfv + c] = s / Lc[(size_t)i * nfv + i];
        }
    }
    // Exact Schur complement S = sum_k B_k A^-1 B_k^T + C of the level-0
    // system (dense); a rank-one term alpha m m^T on the constant pressure
    // makes it SPD when the pressure has a null space.  Its inverse is the
    // pressure block of the block-diagonal MINRES preconditioner.
    C.sinv.clear();
    if (schur) {
        std::vector<double> Bk((size_t)N * nfv), BA((size_t)N * nfv), S((size_t)N * N, 0.0);
        for (int k = 0; k < 3; ++k) {
            std::fill(Bk.begin(), Bk.end(), 0.0);
            for (int v = 0; v < N; ++v) {
                const int row = 3 * nfv + v;
                for (int e = C.rowptr[row]; e < C.rowptr[row + 1]; ++e) {
                    const int col = C.col[e];
                    if (col >= k * nfv && col < (k + 1) * nfv) Bk[(size_t)v * nfv + (col - k * nfv)] = C.val[e];
                }
            }
            for (int v = 0; v < N; ++v)
                for (int j = 0; j < nfv; ++j) {
                    double acc = 0.0;
                    for (int q = 0; q < nfv; ++q) acc += Bk[(size_t)v * nfv + q] * C.ainv[(size_t)q * nfv + j];
                    BA[(size_t)v * nfv + j] = acc;
                }
            for (int v = 0; v < N; ++v)
                for (int w = 0; w < N; ++w) {
                    double acc = 0.0;
                    for (int q = 0; q < nfv; ++q) acc += BA[(size_t)v * nfv + q] * Bk[(size_t)w * nfv + q];
                    S[(size_t)v * N + w] += acc;
                }
        }
        for (int v = 0; v < N; ++v) {
            const int row = 3 * nfv + v;
            for (int e = C.rowptr[row]; e < C.rowptr[row + 1]; ++e)
                if (C.col[e] >= 3 * nfv) S[(size_t)v * N + (C.col[e] - 3 * nfv)] -= C.val[e];
        }
        std::vector<double> mvec(N);
        double mm = 0.0, tr = 0.0;
        for (int v = 0; v < N; ++v) {
            mvec[v] = rec_of(v)[ST_MASS];
            mm += mvec[v] * mvec[v];
            tr += S[(size_t)v * N + v];
        }
        if (mi.project) {
            const double alpha = tr / mm;
            for (int v = 0; v < N; ++v)
                for (int w = 0; w < N; ++w) S[(size_t)v * N + w] += alpha * mvec[v] * mvec[w];
        }
        // symmetrise round-off, then invert by Cholesky
        for (int v = 0; v < N; ++v)
            for (int w = 0; w < v; ++w) {
                const double a = 0.5 * (S[(size_t)v * N + w] + S[(size_t)w * N + v]);
                S[(size_t)v * N + w] = S[(size_t)w * N + v] = a;
            }
        std::vector<double> Lf(S);
        for (int j = 0; j < N; ++j) {
            double d = Lf[(size_t)j * N + j];
            for (int q = 0; q < j; ++q) d -= Lf[(size_t)j * N + q] * Lf[(size_t)j * N + q];
            if (!(d > 0.0)) {
                *err = "coarse Schur complement is not positive definite";
                return false;
            }
            d = std::sqrt(d);
            Lf[(size_t)j * N + j] = d;
            for (int i = j + 1; i < N; ++i) {
                double sacc = Lf[(size_t)i * N + j];
                for (int q = 0; q < j; ++q) sacc -= Lf[(size_t)i * N + q] * Lf[(size_t)j * N + q];
                Lf[(size_t)i * N + j] = sacc / d;
            }
        }
        C.sinv.assign((size_t)N * N, 0.0);
        std::vector<double> yv(N);
        for (int c = 0; c < N; ++c) {
            for (int i = 0; i < N; ++i) {
                double sacc = (i == c) ? 1.0 : 0.0;
                for (int q = 0; q < i; ++q) sacc -= Lf[(size_t)i * N + q] * yv[q];
                yv[i] = sacc / Lf[(size_t)i * N + i];
            }
            for (int i = N - 1; i >= 0; --i) {
                double sacc = yv[i];
                for (int q = i + 1; q < N; ++q) sacc -= Lf[(size_t)q * N + i] * C.sinv[(size_t)q * N + c];
                C.sinv[(size_t)i * N + c] = sacc / Lf[(size_t)i * N + i];
            }
        }
    }
    // D form: inverse of the coupled free velocity block (velocity multigrid
    // of the Krylov solvers), from the velocity-velocity entries of the rows
    C.a2inv.clear();
    if (dform) {
        const int n3 = 3 * nfv;
        std::vector<double> K((size_t)n3 * n3, 0.0);
        for (int r = 0; r < n3; ++r)
            for (int e = C.rowptr[r]; e < C.rowptr[r + 1]; ++e)
                if (C.col[e] < n3) K[(size_t)r * n3 + C.col[e]] += C.val[e];
        if (!invert_dense(K, n3)) {
            *err = "coupled coarse velocity block is singular";
            return false;
        }
        C.a2inv.swap(K);
    }
    // direct solver: K_0 bordered by the constraint sum_i m_i p_i = 0 (only
    // when the pressure has a null space); the leading nd x nd block of its
    // inverse maps any right-hand side to the mean-zero solution of the
    // consistent part of it.  The device inverts it (set-up).
    C.kb.clear();
    C.nb = 0;
    if (direct) {
        const int nd = C.nd;
        const int nb = nd + (mi.project ? 1 : 0);
        C.nb = nb;
        C.kb.assign((size_t)nb * nb, 0.0);
        std::vector<double>& K = C.kb;
        for (int r = 0; r < nd; ++r)
            for (int e = C.rowptr[r]; e < C.rowptr[r + 1]; ++e) K[(size_t)r * nb + C.col[e]] += C.val[e];
        if (mi.project)
            for (int v = 0; v < N; ++v) {
                const double m = rec_of(v)[ST_MASS];
                K[(size_t)(3 * nfv + v) * nb + nd] = m;
                K[(size_t)nd * nb + 3 * nfv + v] = m;
            }
        // free-slip vertices: Q K Q + a (I - Q) on their three velocity rows
        // and columns, Q = I - n n^T, a the centre tap of A (a scale like the
        // rest of the row); the normal component then solves to zero for a
        // right-hand side without one, and the rest is the constrained system
        for (int iv = 0; iv < nfv; ++iv) {
            const int v = C.vel_node[iv];
            if (!L.node_slip[C.node_lat[v]]) continue;
            const double* nrm = rec_of(v) + ST_NRM;
            double Q[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Q[a][b] = (a == b ? 1.0 : 0.0) - nrm[a] * nrm[b];
            const size_t r[3] = {(size_t)iv, (size_t)(nfv + iv), (size_t)(2 * nfv + iv)};
            for (int q = 0; q < nb; ++q) {   // rows
                double o[3], w[3];
                for (int a = 0; a < 3; ++a) o[a] = K[r[a] * nb + q];
                for (int a = 0; a < 3; ++a) w[a] = Q[a][0] * o[0] + Q[a][1] * o[1] + Q[a][2] * o[2];
                for (int a = 0; a < 3; ++a) K[r[a] * nb + q] = w[a];
            }
            for (int q = 0; q < nb; ++q) {   // columns
                double o[3], w[3];
                for (int a = 0; a < 3; ++a) o[a] = K[(size_t)q * nb + r[a]];
                for (int a = 0; a < 3; ++a) w[a] = o[0] * Q[0][a] + o[1] * Q[1][a] + o[2] * Q[2][a];
                for (int a = 0; a < 3; ++a) K[(size_t)q * nb + r[a]] = w[a];
            }
            const double aii = rec_of(v)[ST_A];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) K[r[a] * nb + r[b]] += aii * nrm[a] * nrm[b];
        }
    }
    C.pdinv.resize(N);
    C.mass.resize(N);
    C.node_slot.resize(N);
    C.node_cptr.assign(1, 0);
    C.node_copy.clear();
    std::unordered_map<int64_t, int32_t> ifidx;
    for (int t = 0; t < L.nif; ++t) ifidx[L.if_lat[t]] = t;
    for (int v = 0; v < N; ++v) {
        const double* r = rec_of(v);
        C.pdinv[v] = 1.0 / r[ST_MASSNU];
        C.mass[v] = r[ST_MASS];
        C.node_slot[v] = L.node_slot[C.node_lat[v]];
        auto it = ifidx.find(C.node_lat[v]);
        if (it == ifidx.end()) {
            C.node_copy.push_back(C.node_slot[v]);
        } else {
            int t = it->second;
            for (int q = L.if_cptr[t]; q < L.if_cptr[t + 1]; ++q) C.node_copy.push_back(L.if_copy[q]);
        }
        C.node_cptr.push_back((int32_t)C.node_copy.size());
    }
    return true;
}

}  // namespace hhg
