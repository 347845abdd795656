// Device kernels of the Uzawa multigrid (gfx950).  Included once, by hhg.hip.
//
// Work decomposition.  Every level is processed by two kinds of workgroups in
// the same launch; the interface blocks come first (their count padded to a
// multiple of 8 so that volume tile b still runs on XCD b % 8), so that their
// scattered accesses overlap the volume tiles instead of forming the tail:
//  * volume tiles: 256 lanes over the rows of one slab k of one macro.  Rows
//    j and jh-j of the slab are folded into one row of constant width W so
//    that the triangular slab fills whole wavefronts; a lane owns one quad
//    (4 consecutive i of a row).  Every sub-row (i mod 4) is contiguous, so
//    a colour sweep (one node per quad) and every neighbour access of a wave
//    is a unit-stride load.
//  * interface blocks: 256 vertices of the interface list (vertices on macro
//    faces, edges and corners), addressed through their neighbour table; the
//    new value is written into every macro copy of the vertex, which is the
//    ghost exchange (Section 3.4) fused into the update.
#pragma once
#include <hip/hip_runtime.h>

#include "hhg_internal.hpp"

namespace hhg {

constexpr int TPB = 256;

__host__ __device__ __forceinline__ int R4d(int L) {
    int a = L >> 2, b = L & 3;
    return 4 * (a + 1) * (2 * a + b);
}
__host__ __device__ __forceinline__ int at(int base, int Q, int i) { return base + (i & 3) * Q + (i >> 2); }

// Slab k of a macro (m = n - k) holds rows j = 0..m of Q_j = ceil((m+1-j)/4)
// quads.  It is split by i mod 4 into four sub-arrays of equal length
// S = sum_j Q_j; inside a sub-array the even rows come first, then the odd
// rows, each row's Q_j entries contiguous.  Colour c = (i + 2j + 3k) mod 4
// then occupies the even-row block of sub-array (c+k) mod 4 and the odd-row
// block of sub-array (c+k+2) mod 4, and its neighbours (colours c -+ 1) fill
// sub-arrays (c+k-+1) mod 4 entirely: a colour sweep streams whole blocks.
// Vertex (i, j, k) sits at sb[k] + row_off(m, j) + (i & 3) S + (i >> 2).
__host__ __device__ __forceinline__ int sub_stride(int m) { return R4d(m + 1) >> 2; }
// sum of Q_j' over the rows j' < j of the parity of j
__host__ __device__ __forceinline__ int parity_prefix(int m, int j) {
    const int J = j >> 1, A = m + 4 - (j & 1);
    const int E = (J + 1) >> 1, O = J >> 1;
    return E * (A >> 2) - ((E * (E - 1)) >> 1) + O * ((A - 2) >> 2) - ((O * (O - 1)) >> 1);
}
__host__ __device__ __forceinline__ int row_off(int m, int j) {
    return (j & 1) ? parity_prefix(m, ((m >> 1) << 1) + 2) + parity_prefix(m, j) : parity_prefix(m, j);
}

// Row bases and sub-array strides around row (j, k) of a macro:
// 0:(j,k) 1:(j+1,k) 2:(j-1,k) 3:(j-1,k+1) 4:(j+1,k-1) 5:(j,k+1) 6:(j,k-1)
struct Rows {
    int b[7];
    int Q[7];
};

__host__ __device__ __forceinline__ void make_rows(const int* __restrict__ sb, int n, int mb, int j, int k,
                                          Rows& R) {
    const int mm = n - k;
    const int b0 = mb + sb[k], bp = mb + sb[k + 1], bm = mb + sb[k - 1];
    const int S0 = sub_stride(mm), Sp = sub_stride(mm - 1), Sm = sub_stride(mm + 1);
    R.b[0] = b0 + row_off(mm, j);
    R.b[1] = b0 + row_off(mm, j + 1);
    R.b[2] = b0 + row_off(mm, j - 1);
    R.b[3] = bp + row_off(mm - 1, j - 1);
    R.b[4] = bm + row_off(mm + 1, j + 1);
    R.b[5] = bp + row_off(mm - 1, j);
    R.b[6] = bm + row_off(mm + 1, j);
    R.Q[0] = R.Q[1] = R.Q[2] = S0;
    R.Q[3] = R.Q[5] = Sp;
    R.Q[4] = R.Q[6] = Sm;
}

// slot of macro-local vertex (i, j, k) in a macro whose array starts at mb
__host__ __device__ __forceinline__ int slot_of(const int* __restrict__ sb, int n, int mb, int i, int j,
                                       int k) {
    const int mm = n - k;
    return mb + sb[k] + row_off(mm, j) + (i & 3) * sub_stride(mm) + (i >> 2);
}

// slots of the centre and the 14 neighbours in macro-local offset order
__host__ __device__ __forceinline__ void nbr_slots(const Rows& R, int i, int s[15]) {
    s[0] = at(R.b[0], R.Q[0], i);
    s[1] = at(R.b[0], R.Q[0], i + 1);
    s[2] = at(R.b[0], R.Q[0], i - 1);
    s[3] = at(R.b[1], R.Q[1], i - 1);
    s[4] = at(R.b[2], R.Q[2], i + 1);
    s[5] = at(R.b[1], R.Q[1], i);
    s[6] = at(R.b[2], R.Q[2], i);
    s[7] = at(R.b[3], R.Q[3], i);
    s[8] = at(R.b[4], R.Q[4], i);
    s[9] = at(R.b[5], R.Q[5], i - 1);
    s[10] = at(R.b[6], R.Q[6], i + 1);
    s[11] = at(R.b[5], R.Q[5], i);
    s[12] = at(R.b[6], R.Q[6], i);
    s[13] = at(R.b[3], R.Q[3], i + 1);
    s[14] = at(R.b[4], R.Q[4], i - 1);
}


// the 7 taps of A and C (centre, +-e_a, +-e_b, +-e_c) in local order
__host__ __device__ __forceinline__ void axis_slots(const Rows& R, int i, int s[7]) {
    s[0] = at(R.b[0], R.Q[0], i);
    s[1] = at(R.b[0], R.Q[0], i + 1);
    s[2] = at(R.b[0], R.Q[0], i - 1);
    s[3] = at(R.b[1], R.Q[1], i - 1);
    s[4] = at(R.b[2], R.Q[2], i + 1);
    s[5] = at(R.b[3], R.Q[3], i);
    s[6] = at(R.b[4], R.Q[4], i);
}

// Lane -> (row j, quad q) of a folded slab; rows jl..jh are paired (jl+p, jh-p).
struct LanePos {
    int j, q;
    bool ok;
};
__host__ __device__ __forceinline__ LanePos decode_lane(const Tile& T, int n, int jl, int jh, int lane) {
    LanePos P{0, 0, false};
    const int mm = n - T.k;
    const int t = T.t0 + lane;
    const int p = (int)(((float)t + 0.5f) * (1.0f / (float)T.W));
    const int q = t - p * T.W;
    const int npairs = (jh - jl + 2) >> 1;
    if (p >= npairs) return P;
    const int ja = jl + p, jb = jh - p;
    const int Qa = (mm + 4 - ja) >> 2;
    if (q < Qa) {
        P.j = ja;
        P.q = q;
        P.ok = true;
    } else if (jb > ja) {
        const int q2 = q - Qa;
        if (q2 < ((mm + 4 - jb) >> 2)) {
            P.j = jb;
            P.q = q2;
            P.ok = true;
        }
    }
    return P;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// sum over a 256-thread block, result valid in thread 0
__device__ __forceinline__ double block_sum256(double v, double* sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}

// ---------------------------------------------------------------------------
// Colour sweeps (Section 3.5): one launch updates every vertex of colour c.
// Velocity: u_k = (ru_k - sum_{y != x} A_xy u_k(y)) / A_xx, ru = f - B^T p
// precomputed with the pressure frozen; three components at once.
// Pressure: p += omega (bp - (C p)_x) / C_xx with bp = B u - g.
// ---------------------------------------------------------------------------
// A volume vertex at distance one from its macro's boundary may be a
// neighbour of an interface vertex, and then has a mirror entry.
__host__ __device__ __forceinline__ bool near_boundary(int n, int i, int j, int k) {
    return i <= 1 || j <= 1 || k <= 1 || i + j + k >= n - 1;
}

// Point-block Gauss-Seidel update of the D form (a_2) at one vertex:
// u(x) = D_xx^-1 (t(x) - sum_{taps g != 0} sum_l A_2^{kl}_g u_l(g)), D_xx the
// 3x3 centre block of the record.  v[g] (g = 1..14) holds the slots of the
// 14 neighbours in the record's tap order, in fields of stride xs.
template <typename T>
__device__ __forceinline__ void dform_block(const T* __restrict__ st, const int* v,
                                            const T* __restrict__ u, size_t xs, T res[3]) {
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const T* ul = u + l * xs;
#pragma unroll
        for (int g = 1; g < 15; ++g) {
            const T val = ul[v[g]];
#pragma unroll
            for (int k = 0; k < 3; ++k) res[k] -= st[ST_A2 + 15 * (3 * k + l) + g] * val;
        }
    }
    const T* di = st + ST_DINV;
    const T r0 = res[0], r1 = res[1], r2 = res[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) res[k] = di[3 * k] * r0 + di[3 * k + 1] * r1 + di[3 * k + 2] * r2;
}

// One interface vertex t of a colour sweep: its neighbours come from the
// mirror (unit-stride runs), the new value goes to every macro copy of the
// vertex (the ghost exchange fused into the update) and to the mirror.
// (The D form's interface sweep runs in k_colour, four lanes per vertex.)
// GEN: general meshes, where a_1 and c_l couple all 14 neighbours.
template <typename T, bool VEL, bool GEN = false>
__device__ __forceinline__ void iface_colour(const LevelDev<T>& L, const T* __restrict__ st, int t,
                                             T* __restrict__ x, const T* __restrict__ rhs, T omega,
                                             int fa = 0, int fb = 3) {
    constexpr int NT = GEN ? 14 : 6;   // neighbour taps of A and C (global order)
    const size_t len = (size_t)L.len, cs = (size_t)L.cstride;
    const int nif = L.nif;
    const int self = L.if_self[t];
    T* cx = L.cx;
    const int c0 = L.if_cptr[t], c1 = L.if_cptr[t + 1];
    int nb[NT];
#pragma unroll
    for (int g = 0; g < NT; ++g) nb[g] = L.if_tap[g * nif + t];
    if (VEL) {
        // components fa .. fb-1 (the Laplace form updates each on its own)
        for (int f = fa; f < fb; ++f) {
            const T* u = cx + f * cs;
            T acc = T(0);
#pragma unroll
            for (int g = 0; g < NT; ++g) acc += st[ST_A + 1 + g] * u[nb[g]];
            const T v = (rhs[f * len + self] - acc) * st[ST_INVA];
            for (int q = c0; q < c1; ++q) x[f * len + L.if_copy[q]] = v;
            cx[f * cs + t] = v;
        }
    } else {
        const T* p = cx + 3 * cs;
        const T p0 = p[t];
        T cp = st[ST_C] * p0;
#pragma unroll
        for (int g = 0; g < NT; ++g) cp += st[ST_C + 1 + g] * p[nb[g]];
        const T v = p0 + omega * (rhs[3 * len + self] - cp) * st[ST_INVC];
        for (int q = c0; q < c1; ++q) x[3 * len + L.if_copy[q]] = v;
        cx[3 * cs + t] = v;
    }
}

// Free-slip vertices (Section 6.1): the velocity lives in the tangent plane
// of the record's mass-conservative normal; v <- (I - n n^T) v.
template <typename T>
__device__ __forceinline__ void tangential(const T* __restrict__ nrm, T v[3]) {
    const T d = nrm[0] * v[0] + nrm[1] * v[1] + nrm[2] * v[2];
    v[0] -= d * nrm[0];
    v[1] -= d * nrm[1];
    v[2] -= d * nrm[2];
}

// The free-slip interface vertex t of a velocity colour sweep: the point
// update of all three components (a_1: the centre block is a_xx I), then its
// projection onto the tangent plane; every copy and the mirror are written.
template <typename T, bool GEN>
__device__ __forceinline__ void slip_colour(const LevelDev<T>& L, int t, T* __restrict__ x,
                                            const T* __restrict__ rhs) {
    constexpr int NT = GEN ? 14 : 6;
    const size_t len = (size_t)L.len, cs = (size_t)L.cstride;
    const int nif = L.nif;
    const T* st = L.st + (size_t)L.if_sid[t] * ST_SIZE;
    const int self = L.if_self[t];
    int nb[NT];
#pragma unroll
    for (int g = 0; g < NT; ++g) nb[g] = L.if_tap[g * nif + t];
    T v[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const T* u = L.cx + f * cs;
        T acc = T(0);
#pragma unroll
        for (int g = 0; g < NT; ++g) acc += st[ST_A + 1 + g] * u[nb[g]];
        v[f] = (rhs[f * len + self] - acc) * st[ST_INVA];
    }
    tangential(st + ST_NRM, v);
    for (int q = L.if_cptr[t]; q < L.if_cptr[t + 1]; ++q)
#pragma unroll
        for (int f = 0; f < 3; ++f) x[f * len + L.if_copy[q]] = v[f];
#pragma unroll
    for (int f = 0; f < 3; ++f) L.cx[f * cs + t] = v[f];
}

// the free-slip vertices of colour c alone (the colour-0 sweep that the
// fused f - B^T p pass leaves to them)
template <typename T, bool GEN>
__global__ void k_slip_colour(LevelDev<T> L, int c, T* __restrict__ x, const T* __restrict__ rhs) {
    const int t = L.slip_beg[c] + (int)blockIdx.x * blockDim.x + (int)threadIdx.x;
    if (t < L.col_start[c + 1]) slip_colour<T, GEN>(L, t, x, rhs);
}

// x <- (I - n n^T) x on the velocity of every free-slip vertex, all copies
template <typename T>
__global__ void k_slip_project(LevelDev<T> L, T* __restrict__ x) {
    const int t = (int)blockIdx.x * blockDim.x + (int)threadIdx.x;
    if (t >= L.nif || !(L.if_flag[t] & 2)) return;
    const size_t len = (size_t)L.len;
    const int self = L.if_self[t];
    T v[3] = {x[self], x[len + self], x[2 * len + self]};
    tangential(L.st + (size_t)L.if_sid[t] * ST_SIZE + ST_NRM, v);
    for (int q = L.if_cptr[t]; q < L.if_cptr[t + 1]; ++q)
#pragma unroll
        for (int f = 0; f < 3; ++f) x[f * len + L.if_copy[q]] = v[f];
}

// Point update of volume vertex (i, j, k) of a Kuhn macro, whose a_1 and c_l
// couple only the six axis neighbours: the velocity Gauss-Seidel of the three
// components, or the relaxed pressure update; the mirror entry follows when
// the vertex has one.
template <typename T, bool VEL>
__device__ __forceinline__ void axis_update(const LevelDev<T>& L, const T* __restrict__ st,
                                            const Rows& R, int n, int i, int j, int k,
                                            T* __restrict__ x, const T* __restrict__ rhs, T omega) {
    const size_t len = (size_t)L.len, cs = (size_t)L.cstride;
    int s[7];
    axis_slots(R, i, s);
    const int cm = near_boundary(n, i, j, k) ? L.comp_of_slot[s[0]] : -1;
    if (VEL) {
        const T a1 = st[ST_A + 1], a2 = st[ST_A + 2], a3 = st[ST_A + 3], a4 = st[ST_A + 4],
                a7 = st[ST_A + 7], a8 = st[ST_A + 8], ia = st[ST_INVA];
        // all 21 values before the first store: one wait on memory per lane
        // (the vertex's neighbours are of other colours, never written here)
        T r[3], u[3][6];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const T* uf = x + f * len;
            r[f] = rhs[f * len + s[0]];
#pragma unroll
            for (int g = 0; g < 6; ++g) u[f][g] = uf[s[g + 1]];
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            T v = r[f] - (a1 * u[f][0] + a2 * u[f][1] + a3 * u[f][2] + a4 * u[f][3] + a7 * u[f][4] +
                          a8 * u[f][5]);
            v *= ia;
            x[f * len + s[0]] = v;
            if (cm >= 0) L.cx[f * cs + cm] = v;
        }
    } else {
        T* p = x + 3 * len;
        const T cp = st[ST_C + 0] * p[s[0]] + st[ST_C + 1] * p[s[1]] + st[ST_C + 2] * p[s[2]] +
                     st[ST_C + 3] * p[s[3]] + st[ST_C + 4] * p[s[4]] + st[ST_C + 7] * p[s[5]] +
                     st[ST_C + 8] * p[s[6]];
        const T v = p[s[0]] + omega * (rhs[3 * len + s[0]] - cp) * st[ST_INVC];
        p[s[0]] = v;
        if (cm >= 0) L.cx[3 * cs + cm] = v;
    }
}

// Colour sweeps keep the mirror of x current: a level's smoothing starts
// with a current mirror (refreshed, filled or written by the prolongation).
// DOP: point-block velocity sweeps (D form); GEN: sweeps over all 15 taps of
// a_1 or c_l (general meshes); SLIP: the level has free-slip vertices (their
// lanes follow the component lanes; without them the kernel keeps the
// register budget of the plain sweep).
template <typename T, bool VEL, bool DOP = false, bool GEN = false, bool SLIP = false>
__global__ void __launch_bounds__(TPB) k_colour(LevelDev<T> L, int c, T* __restrict__ x,
                                                const T* __restrict__ rhs, T omega, int ib) {
    static_assert(!(DOP && GEN), "one velocity form per launch");
    const size_t len = (size_t)L.len, cs = (size_t)L.cstride;
    if ((int)blockIdx.x >= ib) {
        const Tile tl = L.vtiles[blockIdx.x - ib];
        if (tl.macro < 0) return;
        const int n = L.n, k = tl.k, mm = n - k;
        const LanePos P = decode_lane(tl, n, 1, mm - 2, threadIdx.x);
        if (!P.ok) return;
        const int j = P.j;
        const int i = 4 * P.q + ((c + 2 * j + k) & 3);
        if (i < 1 || i > mm - 1 - j) return;
        Rows R;
        make_rows(L.slab_base, n, (int)(tl.macro * L.mstride), j, k, R);
        const T* st = L.st + (size_t)tl.macro * ST_SIZE;
        if (VEL && DOP) {
            int v[15];
            nbr_slots(R, i, v);
            const int cm = near_boundary(n, i, j, k) ? L.comp_of_slot[v[0]] : -1;
            T res[3];
#pragma unroll
            for (int f = 0; f < 3; ++f) res[f] = rhs[f * len + v[0]];
            dform_block<T>(st, v, x, len, res);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                x[f * len + v[0]] = res[f];
                if (cm >= 0) L.cx[f * cs + cm] = res[f];
            }
            return;
        }
        if (VEL && GEN) {
            int v[15];
            nbr_slots(R, i, v);
            const int cm = near_boundary(n, i, j, k) ? L.comp_of_slot[v[0]] : -1;
            const T ia = st[ST_INVA];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                // one component's 14 loads in flight at a time (all three
                // hoisted need 112 VGPRs and halve the waves per SIMD)
                __builtin_amdgcn_sched_barrier(0);
                T* u = x + f * len;
                T acc = rhs[f * len + v[0]];
#pragma unroll
                for (int g = 1; g < 15; ++g) acc -= st[ST_A + g] * u[v[g]];
                const T val = acc * ia;
                u[v[0]] = val;
                if (cm >= 0) L.cx[f * cs + cm] = val;
            }
            return;
        }
        if (!VEL && GEN) {
            int v[15];
            nbr_slots(R, i, v);
            const int cm = near_boundary(n, i, j, k) ? L.comp_of_slot[v[0]] : -1;
            T* p = x + 3 * len;
            T cp = T(0);
#pragma unroll
            for (int g = 0; g < 15; ++g) cp += st[ST_C + g] * p[v[g]];
            const T val = p[v[0]] + omega * (rhs[3 * len + v[0]] - cp) * st[ST_INVC];
            p[v[0]] = val;
            if (cm >= 0) L.cx[3 * cs + cm] = val;
            return;
        }
        axis_update<T, VEL>(L, st, R, n, i, j, k, x, rhs, omega);
        return;
    }
    const int t0 = L.col_start[c];
    const int tend = VEL ? L.vel_end[c] : L.col_start[c + 1];
    if (VEL && DOP) {
        // D form: four lanes per interface vertex (groups of four consecutive
        // lanes, never split across waves).  Lane k < 3 forms row k of the
        // block residual (the rows of dform_block, in its order), the lanes
        // exchange the three rows, and lane k applies row k of the inverse
        // centre block and writes component k.
        const int q = (int)blockIdx.x * TPB + (int)threadIdx.x, t = t0 + (q >> 2), k = q & 3;
        const bool act = t < tend && k < 3;
        const size_t len = (size_t)L.len, cs = (size_t)L.cstride;
        const int nif = L.nif;
        const int tt = t < tend ? t : t0;
        const T* st = L.st + (size_t)L.if_sid[tt] * ST_SIZE;
        T r = T(0);
        if (act) {
            int v[15];
#pragma unroll
            for (int g = 1; g < 15; ++g) v[g] = L.if_tap[(g - 1) * nif + tt];
            r = rhs[k * len + L.if_self[tt]];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const T* ul = L.cx + l * cs;
#pragma unroll
                for (int g = 1; g < 15; ++g) r -= st[ST_A2 + 15 * (3 * k + l) + g] * ul[v[g]];
            }
        }
        const int g0 = (int)threadIdx.x & ~3;
        const T r0 = __shfl(r, g0), r1 = __shfl(r, g0 + 1), r2 = __shfl(r, g0 + 2);
        if (act) {
            const T* di = st + ST_DINV;
            const T val = di[3 * k] * r0 + di[3 * k + 1] * r1 + di[3 * k + 2] * r2;
            for (int qq = L.if_cptr[tt]; qq < L.if_cptr[tt + 1]; ++qq) x[k * len + L.if_copy[qq]] = val;
            L.cx[k * cs + tt] = val;
        }
        return;
    }
    if (VEL && !DOP) {
        // a lane per interface vertex and velocity component: the scattered
        // loads of a colour's interface vertices spread over three times as
        // many workgroups (on small levels they are the launch's longest path);
        // then a lane per free-slip vertex (three components and the projection)
        const int q = (int)blockIdx.x * TPB + (int)threadIdx.x, nfc = tend - t0;
        if (q < 3 * nfc) {
            const int t = t0 + q / 3, f = q % 3;
            iface_colour<T, VEL, GEN>(L, L.st + (size_t)L.if_sid[t] * ST_SIZE, t, x, rhs, omega, f,
                                      f + 1);
            return;
        }
        if (SLIP) {
            const int ts = L.slip_beg[c] + (q - 3 * nfc);
            if (ts < L.col_start[c + 1]) slip_colour<T, GEN>(L, ts, x, rhs);
        }
        return;
    }
    const int t = t0 + (int)blockIdx.x * TPB + (int)threadIdx.x;
    if (t >= tend) return;
    iface_colour<T, VEL, GEN>(L, L.st + (size_t)L.if_sid[t] * ST_SIZE, t, x, rhs, omega);
}

// Volume blocks of a red-black launch: two per tile (the quad's two vertices
// of the parity), block v taking tile 8 (v / 16) + v % 8 and half (v / 8) % 2,
// so that both halves of a tile run on its XCD.
__host__ __device__ __forceinline__ int rb_tile(int v) { return (v >> 4) * 8 + (v & 7); }
__host__ __device__ __forceinline__ int rb_half(int v) { return (v >> 3) & 1; }
__host__ __device__ __forceinline__ int rb_blocks(int n_vtiles) { return 2 * ((n_vtiles + 7) / 8 * 8); }

// Red-black sweep of Kuhn meshes (ordering 2): a_1 and c_l couple only the six
// axis neighbours, whose colours differ from the vertex's by one, so the
// colours p and p + 2 never couple and one launch updates both (parity p:
// 0 red, 1 black).  Volume: two blocks per tile, each taking one of a quad's
// two vertices of the parity in every lane; interface: a lane per vertex and
// velocity component (pressure: per vertex) of either colour range.
template <typename T, bool VEL>
__global__ void __launch_bounds__(TPB) k_colour_rb(LevelDev<T> L, int p, T* __restrict__ x,
                                                   const T* __restrict__ rhs, T omega, int ib) {
    if ((int)blockIdx.x >= ib) {
        // two blocks per tile, one per vertex of the parity in every quad,
        // dealt to the tile's XCD like the full passes' sub-row blocks
        const int v = (int)blockIdx.x - ib;
        const int ti = rb_tile(v), e = rb_half(v);
        if (ti >= L.n_vtiles) return;
        const Tile tl = L.vtiles[ti];
        if (tl.macro < 0) return;
        const int n = L.n, k = tl.k, mm = n - k;
        const LanePos P = decode_lane(tl, n, 1, mm - 2, threadIdx.x);
        if (!P.ok) return;
        const int j = P.j;
        const int i = 4 * P.q + ((p + 2 * j + k + 2 * e) & 3);
        if (i < 1 || i > mm - 1 - j) return;
        Rows R;
        make_rows(L.slab_base, n, (int)(tl.macro * L.mstride), j, k, R);
        axis_update<T, VEL>(L, L.st + (size_t)tl.macro * ST_SIZE, R, n, i, j, k, x, rhs, omega);
        return;
    }
    const int n0 = (VEL ? L.vel_end[p] : L.col_start[p + 1]) - L.col_start[p];
    const int n2 = (VEL ? L.vel_end[p + 2] : L.col_start[p + 3]) - L.col_start[p + 2];
    const int q = (int)blockIdx.x * TPB + (int)threadIdx.x;
    const int v = VEL ? q / 3 : q, f = VEL ? q % 3 : 0;
    int t;
    if (v < n0)
        t = L.col_start[p] + v;
    else if (v < n0 + n2)
        t = L.col_start[p + 2] + (v - n0);
    else
        return;
    const T* st = L.st + (size_t)L.if_sid[t] * ST_SIZE;
    if (VEL)
        iface_colour<T, true>(L, st, t, x, rhs, omega, f, f + 1);
    else
        iface_colour<T, false>(L, st, t, x, rhs, omega);
}

// ---------------------------------------------------------------------------
// Hybrid ordering (Section 3.4): the interface vertices of one primitive class
// and colour, listed in `list`.  Taps flagged in mask[t] reach another
// primitive of the same class and read `snap` (the mirror's values when the
// class started: block Jacobi between primitives); every other tap reads the
// current mirror (Gauss-Seidel).  Velocity: a lane per vertex and component;
// pressure: a lane per vertex, relaxed by omega.  GEN: a_1 and c_l couple all
// 14 neighbours (general meshes), otherwise the 6 axis neighbours.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_hyb_snap(LevelDev<T> L, const int* __restrict__ list, int cnt, int f0, int f1,
                           T* __restrict__ snap) {
    const int q = (int)blockIdx.x * blockDim.x + (int)threadIdx.x;
    if (q >= cnt) return;
    const int t = list[q];
    for (int f = f0; f < f1; ++f) snap[(size_t)f * L.nif + t] = L.cx[(size_t)f * L.cstride + t];
}

template <typename T, bool VEL, bool GEN>
__global__ void __launch_bounds__(TPB) k_hyb_iface(LevelDev<T> L, const int* __restrict__ list,
                                                   int cnt, T* __restrict__ x,
                                                   const T* __restrict__ rhs, T omega,
                                                   const T* __restrict__ snap,
                                                   const int* __restrict__ mask) {
    constexpr int NT = GEN ? 14 : 6;
    const int q = (int)blockIdx.x * TPB + (int)threadIdx.x;
    const int i = VEL ? q / 3 : q, f = VEL ? q % 3 : 3;
    if (i >= cnt) return;
    const int t = list[i];
    const size_t len = (size_t)L.len, cs = (size_t)L.cstride;
    const int nif = L.nif;
    const T* st = L.st + (size_t)L.if_sid[t] * ST_SIZE;
    const int m = mask[t];
    const T* cur = L.cx + f * cs;
    const T* old = snap + (size_t)f * nif;
    const int blk = VEL ? ST_A : ST_C;
    T acc = T(0);
#pragma unroll
    for (int g = 0; g < NT; ++g) {
        const int e = L.if_tap[g * nif + t];
        acc += st[blk + 1 + g] * ((m >> g & 1) ? old[e] : cur[e]);
    }
    T v;
    if (VEL) {
        v = (rhs[f * len + L.if_self[t]] - acc) * st[ST_INVA];
    } else {
        const T p0 = cur[t];
        v = p0 + omega * (rhs[3 * len + L.if_self[t]] - (st[ST_C] * p0 + acc)) * st[ST_INVC];
    }
    for (int qq = L.if_cptr[t]; qq < L.if_cptr[t + 1]; ++qq) x[f * len + L.if_copy[qq]] = v;
    L.cx[f * cs + t] = v;
}

// ---------------------------------------------------------------------------
// Full passes over every vertex (volume interior + interface), one template
// for the operators that read all 15 taps:
//   MODE_APPLY   y = K x                         (Dirichlet velocity rows 0)
//   MODE_RES     r = b - K x, sum r^2 into per-block partials
//   MODE_RU      t_k = b_k - (B^T p)_k  (k = 0..2; Dirichlet rows 0)
//   MODE_BP      t_3 = (B u) - b_3
//   MODE_RHS     y = (M f on free rows, sum_k G_k f_k)    (in: f in fields 0..2)
//   MODE_GRADF   y_k = M lam_k + GT_k lam_p                (in: lambda)
//   MODE_ARES    t_k = b_k - (A u_k)  (k = 0..2; Dirichlet rows 0)  velocity multigrid
//   MODE_BTN     t_k = -(B^T p)_k     (k = 0..2; Dirichlet rows 0)  Schur complement
//   MODE_SCHUR   t_3 = (C p) - (B u)                               Schur complement
// ---------------------------------------------------------------------------
enum { MODE_APPLY = 0, MODE_RES = 1, MODE_RU = 2, MODE_BP = 3, MODE_RHS = 4, MODE_GRADF = 5,
       MODE_ARES = 6, MODE_BTN = 7, MODE_SCHUR = 8 };

// Load from a uniform field base at a 32-bit byte offset: the address is an
// SGPR base plus one 32-bit VGPR per tap, shared by all fields (slot offsets
// in bytes stay below 2^32; the host checks it).
template <typename T>
__device__ __forceinline__ T ldo(const T* __restrict__ base, uint32_t boff) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
}

// One row of a full pass.  s[] are the 15 taps of x (centre first) in a
// field of stride xs (a macro array, or the compact mirror for interface
// vertices); the vertex's own entries of b sit at slot bslot of fields of
// stride bs.
// Velocity residual of A alone at one vertex: tp[] the centre and the six
// axis taps, ca[] the record positions of their coefficients (A couples only
// the axis neighbours on Kuhn lattices).
template <typename T>
__device__ __forceinline__ void eval_ares(const T* __restrict__ st, const int* tp, const int* ca,
                                          bool dir, const T* __restrict__ x, size_t xs,
                                          const T* __restrict__ b, size_t bs, int bslot,
                                          T out[4]) {
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        T acc = T(0);
#pragma unroll
        for (int g = 0; g < 7; ++g) acc += st[ST_A + ca[g]] * x[f * xs + tp[g]];
        out[f] = dir ? T(0) : b[f * bs + bslot] - acc;
    }
}

// tt (residual rows, Laplace form): also b_k - (B^T p)_k, k = 0..2, summed
// over the taps in the order of the f - B^T p pass (bitwise its values).
template <typename T, int MODE, bool DOP = false>
__device__ __forceinline__ void eval_node(const T* __restrict__ st, const int* s, bool dir,
                                          const T* __restrict__ x, size_t xs,
                                          const T* __restrict__ b, size_t bs, int bslot,
                                          T out[4], int fa = 0, int fb = 3, T* tt = nullptr) {
    if (MODE == MODE_ARES && DOP) {
        // D form: every tap of all three components
        T ru[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int g = 0; g < 15; ++g) {
                const T uv = x[l * xs + s[g]];
#pragma unroll
                for (int k = 0; k < 3; ++k) ru[k] += st[ST_A2 + 15 * (3 * k + l) + g] * uv;
            }
#pragma unroll
        for (int k = 0; k < 3; ++k) out[k] = dir ? T(0) : b[k * bs + bslot] - ru[k];
        return;
    }
    if (MODE == MODE_ARES) {
        // interface rows: the axis taps are 1..6 of the global direction order
        const int ca[7] = {0, 1, 2, 3, 4, 5, 6};
        eval_ares<T>(st, s, ca, dir, x, xs, b, bs, bslot, out);
        return;
    }
    if (MODE == MODE_BTN) {
        const T* p = x + 3 * xs;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            T acc = T(0);
#pragma unroll
            for (int g = 0; g < 15; ++g) acc += st[ST_BT + 15 * f + g] * p[s[g]];
            out[f] = dir ? T(0) : -acc;
        }
        return;
    }
    if (MODE == MODE_SCHUR) {
        const T* p = x + 3 * xs;
        T acc = T(0);
#pragma unroll
        for (int g = 0; g < 15; ++g) acc += st[ST_C + g] * p[s[g]];
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int g = 0; g < 15; ++g) acc -= st[ST_B + 15 * f + g] * x[f * xs + s[g]];
        out[3] = acc;
        return;
    }
    if (MODE == MODE_RU) {
        // components fa .. fb-1
        const T* p = x + 3 * xs;
        for (int f = fa; f < fb; ++f) {
            T acc = T(0);
#pragma unroll
            for (int g = 0; g < 15; ++g) acc += st[ST_BT + 15 * f + g] * p[s[g]];
            out[f] = dir ? T(0) : b[f * bs + bslot] - acc;
        }
        return;
    }
    if (MODE == MODE_BP) {
        T acc = T(0);
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int g = 0; g < 15; ++g) acc += st[ST_B + 15 * f + g] * x[f * xs + s[g]];
        out[3] = acc - b[3 * bs + bslot];
        return;
    }
    if (MODE == MODE_RHS || MODE == MODE_GRADF) {
        const T* pl = x + 3 * xs;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            T m = T(0);
#pragma unroll
            for (int g = 0; g < 15; ++g) m += st[ST_M + g] * x[f * xs + s[g]];
            if (MODE == MODE_RHS) {
                out[f] = dir ? T(0) : m;
            } else {
                T gt = T(0);
#pragma unroll
                for (int g = 0; g < 15; ++g) gt += st[ST_GT + 15 * f + g] * pl[s[g]];
                out[f] = m + gt;
            }
        }
        if (MODE == MODE_RHS) {
            T acc = T(0);
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int g = 0; g < 15; ++g) acc += st[ST_G + 15 * f + g] * x[f * xs + s[g]];
            out[3] = acc;
        }
        return;
    }
    // MODE_APPLY / MODE_RES
    uint32_t o[15];
#pragma unroll
    for (int g = 0; g < 15; ++g) o[g] = (uint32_t)s[g] * (uint32_t)sizeof(T);
    const T* p = x + 3 * xs;
    T pv[15];
#pragma unroll
    for (int g = 0; g < 15; ++g) pv[g] = ldo(p, o[g]);
    if (DOP) {
        // D form: the velocity rows couple the three components
        T ku[3] = {T(0), T(0), T(0)}, bu = T(0);
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const T* u = x + l * xs;
#pragma unroll
            for (int g = 0; g < 15; ++g) {
                const T uv = ldo(u, o[g]);
#pragma unroll
                for (int k = 0; k < 3; ++k) ku[k] += st[ST_A2 + 15 * (3 * k + l) + g] * uv;
                bu += st[ST_B + 15 * l + g] * uv;
            }
        }
        T cp = T(0);
#pragma unroll
        for (int g = 0; g < 15; ++g) cp += st[ST_C + g] * pv[g];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            T btp = T(0);
#pragma unroll
            for (int g = 0; g < 15; ++g) btp += st[ST_BT + 15 * k + g] * pv[g];
            const T kk = ku[k] + btp;
            out[k] = dir ? T(0) : (MODE == MODE_RES ? b[k * bs + bslot] - kk : kk);
        }
        const T kp = bu - cp;
        out[3] = MODE == MODE_RES ? b[3 * bs + bslot] - kp : kp;
        return;
    }
    T bu = T(0);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const T* u = x + f * xs;
        T au = T(0), btp = T(0);
#pragma unroll
        for (int g = 0; g < 15; ++g) {
            const T uv = ldo(u, o[g]);
            au += st[ST_A + g] * uv;
            btp += st[ST_BT + 15 * f + g] * pv[g];
            bu += st[ST_B + 15 * f + g] * uv;
        }
        const T ku = au + btp;
        out[f] = dir ? T(0) : (MODE == MODE_RES ? b[f * bs + bslot] - ku : ku);
        if (MODE == MODE_RES && tt) tt[f] = dir ? T(0) : b[f * bs + bslot] - btp;
    }
    T cp = T(0);
#pragma unroll
    for (int g = 0; g < 15; ++g) cp += st[ST_C + g] * pv[g];
    const T kp = bu - cp;
    out[3] = MODE == MODE_RES ? b[3 * bs + bslot] - kp : kp;
}

// Interior rows of K x or of the residual from the pair symmetries of an
// interior stencil (A and C symmetric, B_k antisymmetric and B^T_k(d) =
// B_k(-d) over the opposite taps (2q+1, 2q+2); checked and made exact when the
// records are built): with pair sums for the three axis pairs (taps 1-2, 3-4,
// 7-8, where A and C live) and pair differences for all seven pairs, 29
// coefficients and half the products of the general row.
// tt: as in eval_node.
template <typename T, int MODE>
__device__ __forceinline__ void eval_vol_pairs(const T* __restrict__ st, const int* s,
                                               const T* __restrict__ x, const T* __restrict__ b,
                                               size_t len, T out[4], T* tt = nullptr) {
    uint32_t o[15];
#pragma unroll
    for (int g = 0; g < 15; ++g) o[g] = (uint32_t)s[g] * (uint32_t)sizeof(T);
    T ku[3], kp;
    {
        const T* p = x + 3 * len;
        T pv[15];
#pragma unroll
        for (int g = 0; g < 15; ++g) pv[g] = ldo(p, o[g]);
        const T p0 = pv[0];
        if (MODE == MODE_RES && tt) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                T acc = T(0);
#pragma unroll
                for (int g = 0; g < 15; ++g) acc += st[ST_BT + 15 * f + g] * pv[g];
                tt[f] = b[f * len + s[0]] - acc;
            }
        }
        T pd[7], ps[3];
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const T a = pv[2 * q + 1], c = pv[2 * q + 2];
            pd[q] = a - c;
            if (q == 0) ps[0] = a + c;
            if (q == 1) ps[1] = a + c;
            if (q == 3) ps[2] = a + c;
        }
        kp = -(st[ST_C] * p0 + st[ST_C + 1] * ps[0] + st[ST_C + 3] * ps[1] + st[ST_C + 7] * ps[2]);
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            T acc = T(0);
#pragma unroll
            for (int q = 0; q < 7; ++q) acc += st[ST_BT + 15 * f + 2 * q + 1] * pd[q];
            ku[f] = acc;
        }
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const T* u = x + f * len;
        const T u0 = ldo(u, o[0]);
        T bu = T(0), us[3];
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const T a = ldo(u, o[2 * q + 1]), c = ldo(u, o[2 * q + 2]);
            bu += st[ST_B + 15 * f + 2 * q + 1] * (a - c);
            if (q == 0) us[0] = a + c;
            if (q == 1) us[1] = a + c;
            if (q == 3) us[2] = a + c;
        }
        ku[f] += st[ST_A] * u0 + st[ST_A + 1] * us[0] + st[ST_A + 3] * us[1] + st[ST_A + 7] * us[2];
        kp += bu;
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) out[f] = MODE == MODE_RES ? b[f * len + s[0]] - ku[f] : ku[f];
    out[3] = MODE == MODE_RES ? b[3 * len + s[0]] - kp : kp;
}

template <int MODE>
__device__ __forceinline__ void mode_fields(int& f0, int& f1) {
    f0 = 0;
    f1 = 4;
    if (MODE == MODE_RU || MODE == MODE_GRADF || MODE == MODE_ARES || MODE == MODE_BTN) f1 = 3;
    if (MODE == MODE_BP || MODE == MODE_SCHUR) f0 = 3;
}

// Colour-c update fused into a full pass (velocity Gauss-Seidel into the
// B^T p pass, pressure relaxation into the B u pass): out[] holds the
// node's freshly computed right-hand side, tp the 7 axis taps (centre first)
// into xr (stride rs).  The update reads only colours c -+ 1 (and, for the
// pressure, the vertex itself) and writes colour c, which no other lane of
// the launch reads, so it runs alongside the full pass.  Axis coefficients
// sit at record positions 1, 2, 3, 4, 7, 8 in the local order of volume
// records and 1..6 in the global direction order of interface records.
// Volume vertices write their slot, interface vertices every copy; both
// write mirror entry cm when there is one.  GEN (general meshes): tp holds all
// 15 taps in the record's order and a_1, c_l couple every one of them.
template <typename T, int MODE, bool IFACE, bool GEN = false>
__device__ __forceinline__ void fused_update(const T* __restrict__ st, const int* tp, const T* xr,
                                             size_t rs, T* xw, size_t len, const T out[4], T omega,
                                             int ncopy, const int* copies, T* cx, size_t cs, int cm,
                                             int fa = 0, int fb = 3) {
    constexpr int q5 = IFACE ? 5 : 7, q6 = IFACE ? 6 : 8;
    if (GEN) {
        if (MODE == MODE_RU) {
            for (int f = fa; f < fb; ++f) {
                const T* u = xr + f * rs;
                T v = out[f];
#pragma unroll
                for (int g = 1; g < 15; ++g) v -= st[ST_A + g] * u[tp[g]];
                const T un = v * st[ST_INVA];
                if (IFACE)
                    for (int q = 0; q < ncopy; ++q) xw[f * len + copies[q]] = un;
                else
                    xw[f * len + tp[0]] = un;
                if (cm >= 0) cx[f * cs + cm] = un;
            }
        } else {
            const T* p = xr + 3 * rs;
            const T p0 = IFACE ? cx[3 * cs + cm] : xw[3 * len + tp[0]];
            T cp = st[ST_C] * p0;
#pragma unroll
            for (int g = 1; g < 15; ++g) cp += st[ST_C + g] * p[tp[g]];
            const T pn = p0 + omega * (out[3] - cp) * st[ST_INVC];
            if (IFACE)
                for (int q = 0; q < ncopy; ++q) xw[3 * len + copies[q]] = pn;
            else
                xw[3 * len + tp[0]] = pn;
            if (cm >= 0) cx[3 * cs + cm] = pn;
        }
        return;
    }
    if (MODE == MODE_RU) {
        // components fa .. fb-1
        for (int f = fa; f < fb; ++f) {
            const T* u = xr + f * rs;
            const T v = out[f] - (st[ST_A + 1] * u[tp[1]] + st[ST_A + 2] * u[tp[2]] +
                                  st[ST_A + 3] * u[tp[3]] + st[ST_A + 4] * u[tp[4]] +
                                  st[ST_A + q5] * u[tp[5]] + st[ST_A + q6] * u[tp[6]]);
            const T un = v * st[ST_INVA];
            if (IFACE)
                for (int q = 0; q < ncopy; ++q) xw[f * len + copies[q]] = un;
            else
                xw[f * len + tp[0]] = un;
            if (cm >= 0) cx[f * cs + cm] = un;
        }
    } else {
        // the vertex's own pressure is read where it is written (the mirror
        // entry of an interface vertex, the slot of a volume vertex through
        // xw): nothing read through a restrict pointer changes
        const T* p = xr + 3 * rs;
        const T p0 = IFACE ? cx[3 * cs + cm] : xw[3 * len + tp[0]];
        const T cp = st[ST_C] * p0 + st[ST_C + 1] * p[tp[1]] + st[ST_C + 2] * p[tp[2]] +
                     st[ST_C + 3] * p[tp[3]] + st[ST_C + 4] * p[tp[4]] + st[ST_C + q5] * p[tp[5]] +
                     st[ST_C + q6] * p[tp[6]];
        const T pn = p0 + omega * (out[3] - cp) * st[ST_INVC];
        if (IFACE)
            for (int q = 0; q < ncopy; ++q) xw[3 * len + copies[q]] = pn;
        else
            xw[3 * len + tp[0]] = pn;
        if (cm >= 0) cx[3 * cs + cm] = pn;
    }
}

// Volume blocks of a full pass: four per tile, one per sub-row r = i mod 4, so
// that a lane owns one vertex and every tap of a wave is a unit-stride run.
// Block v of the volume range takes tile 8 (v / 32) + v % 8 and sub-row
// (v / 8) % 4: the four blocks of a tile run on the tile's XCD (tiles are
// dealt to XCDs by index mod 8) and are dispatched close together.
__host__ __device__ __forceinline__ int full_tile(int v) { return (v >> 5) * 8 + (v & 7); }
__host__ __device__ __forceinline__ int full_sub(int v) { return (v >> 3) & 3; }
__host__ __device__ __forceinline__ int full_blocks(int n_vtiles) { return 4 * ((n_vtiles + 7) / 8 * 8); }
// The passes that read all four fields at every tap (K x, the residual, the
// right-hand side and the forcing gradient) keep one block per tile and four
// vertices per lane, evaluated one after another: one vertex per lane would
// need every tap of all fields in flight at once (over 256 VGPRs).
__host__ __device__ constexpr bool quad_lanes(int mode) {
    return mode == MODE_APPLY || mode == MODE_RES || mode == MODE_RHS || mode == MODE_GRADF;
}

// Quad windows: a lane that evaluates the 4 vertices i = 4q..4q+3 of a row
// loads every distinct tap value once.  Row rho of make_rows contributes the
// positions 4q + QW_LO[rho] .. +5 (row 0) or +4; tap g of vertex r is window
// QW_ROW[g] at r + QW_OFF[g] (taps in the local offset order of nbr_slots).
// Per field that is 36 loads for 4 vertices instead of 60.
__device__ constexpr int QW_ROW[15] = {0, 0, 0, 1, 2, 1, 2, 3, 4, 5, 6, 5, 6, 3, 4};
__device__ constexpr int QW_OFF[15] = {1, 2, 0, 0, 1, 1, 0, 0, 1, 0, 1, 1, 0, 1, 0};
__device__ constexpr int QW_LO[7] = {-1, -1, 0, 0, -1, -1, 0};

// window slots of the quad q (positions past a row's end fall on other slots
// of the same slab, which only vertices outside the row would use)
__device__ __forceinline__ void quad_window_slots(const Rows& R, int q, int w[7][6]) {
#pragma unroll
    for (int rho = 0; rho < 7; ++rho)
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const int i = 4 * q + QW_LO[rho] + e;
            w[rho][e] = R.b[rho] + (i & 3) * R.Q[rho] + (i >> 2);
        }
}

// Positions e and e + 4 of a window row are consecutive entries of one
// sub-array (slots w and w + 1): they are read as one pair, a 16-byte load
// for FP64 at 8-byte alignment (the global memory path accepts unaligned
// vector loads), which leaves 28 load instructions per field instead of 36.
template <typename T>
__device__ __forceinline__ void quad_window_load(const T* __restrict__ f, const int w[7][6], T v[7][6]) {
    typedef T tpair __attribute__((ext_vector_type(2), aligned(sizeof(T))));
#pragma unroll
    for (int rho = 0; rho < 7; ++rho) {
        const int cnt = rho == 0 ? 6 : 5;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t off = (uint32_t)w[rho][e] * (uint32_t)sizeof(T);
            if (e + 4 < cnt) {
                const tpair pr =
                    *reinterpret_cast<const tpair*>(reinterpret_cast<const char*>(f) + off);
                v[rho][e] = pr.x;
                v[rho][e + 4] = pr.y;
            } else {
                v[rho][e] = ldo(f, off);
            }
        }
    }
}

// RU (t_k = b_k - (B^T p)_k), BP (t_3 = B u - b_3), K x or the residual
// b - K x for the four vertices of a quad; out[r] receives the values of
// vertex 4q + r.
// TOUT (residual): tt[r] also receives b_k - (B^T p)_k, k = 0..2, from the
// pair form of the residual's own B^T p (the RU branch's value up to
// rounding); the A u_f parts are kept apart until the end for it.
template <typename T, int MODE, bool TOUT = false>
__device__ __forceinline__ void quad_eval(const T* __restrict__ st, const int w[7][6],
                                          const T* __restrict__ x, const T* __restrict__ b,
                                          size_t len, T out[4][4], T (*tt)[3] = nullptr) {
    T v[7][6];
    if (MODE == MODE_APPLY || MODE == MODE_RES) {
        // interior rows from the pair symmetries (as eval_vol_pairs), one
        // field's window at a time: the pressure's (B^T p into the velocity
        // rows, -C p into the pressure row), then each velocity component's
        // (A u_f into row f, B_f u_f into the pressure row).  Opposite taps
        // 2q+1, 2q+2 of vertex r sit at window (QW_ROW, r + QW_OFF).
        T ku[4][3], kp[4], ka[4][3];
        quad_window_load(x + 3 * len, w, v);
        if (TOUT)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int f = 0; f < 3; ++f) ka[r][f] = T(0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T pd[7], ps[3];
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                const T a = v[QW_ROW[2 * q + 1]][r + QW_OFF[2 * q + 1]];
                const T c = v[QW_ROW[2 * q + 2]][r + QW_OFF[2 * q + 2]];
                pd[q] = a - c;
                if (q == 0) ps[0] = a + c;
                if (q == 1) ps[1] = a + c;
                if (q == 3) ps[2] = a + c;
            }
            kp[r] = -(st[ST_C] * v[QW_ROW[0]][r + QW_OFF[0]] + st[ST_C + 1] * ps[0] +
                      st[ST_C + 3] * ps[1] + st[ST_C + 7] * ps[2]);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                T acc = T(0);
#pragma unroll
                for (int q = 0; q < 7; ++q) acc += st[ST_BT + 15 * f + 2 * q + 1] * pd[q];
                ku[r][f] = acc;
            }
        }
        // a loop the compiler keeps rolled: one velocity window in registers at
        // a time (unrolled, all four windows' loads were issued together)
#pragma unroll 1
        for (int f = 0; f < 3; ++f) {
            quad_window_load(x + f * len, w, v);
            const T* bf = st + ST_B + 15 * f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T bu = T(0), us[3];
#pragma unroll
                for (int q = 0; q < 7; ++q) {
                    const T a = v[QW_ROW[2 * q + 1]][r + QW_OFF[2 * q + 1]];
                    const T c = v[QW_ROW[2 * q + 2]][r + QW_OFF[2 * q + 2]];
                    bu += bf[2 * q + 1] * (a - c);
                    if (q == 0) us[0] = a + c;
                    if (q == 1) us[1] = a + c;
                    if (q == 3) us[2] = a + c;
                }
                const T au = st[ST_A] * v[QW_ROW[0]][r + QW_OFF[0]] + st[ST_A + 1] * us[0] +
                             st[ST_A + 3] * us[1] + st[ST_A + 7] * us[2];
#pragma unroll
                for (int g = 0; g < 3; ++g) {
                    if (TOUT)
                        ka[r][g] = g == f ? au : ka[r][g];
                    else
                        ku[r][g] += g == f ? au : T(0);
                }
                kp[r] += bu;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                if (TOUT) {
                    const T bv = b[f * len + w[0][r + 1]];
                    out[r][f] = bv - (ku[r][f] + ka[r][f]);
                    tt[r][f] = bv - ku[r][f];
                    continue;
                }
                out[r][f] = MODE == MODE_RES ? b[f * len + w[0][r + 1]] - ku[r][f] : ku[r][f];
            }
            out[r][3] = MODE == MODE_RES ? b[3 * len + w[0][r + 1]] - kp[r] : kp[r];
        }
    } else if (MODE == MODE_RU) {
        quad_window_load(x + 3 * len, w, v);
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T acc = T(0);
#pragma unroll
                for (int g = 0; g < 15; ++g) acc += st[ST_BT + 15 * f + g] * v[QW_ROW[g]][r + QW_OFF[g]];
                out[r][f] = b[f * len + w[0][r + 1]] - acc;
            }
    } else {
        T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            // one field's window at a time: without the scheduling barrier
            // the compiler hoists all three windows (over 256 VGPRs)
            __builtin_amdgcn_sched_barrier(0);
            quad_window_load(x + f * len, w, v);
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int g = 0; g < 15; ++g) acc[r] += st[ST_B + 15 * f + g] * v[QW_ROW[g]][r + QW_OFF[g]];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) out[r][3] = acc[r] - b[3 * len + w[0][r + 1]];
    }
}

// Interface vertex t of a fused pass updated along with it: fcol 0..3 names one
// colour, 4 + p the two colours p and p + 2 of the red-black order; velocity
// updates skip the velocity Dirichlet vertices (and the free-slip ones, which
// have their own launch).
template <typename T>
__device__ __forceinline__ bool fused_vertex(const LevelDev<T>& L, int t, int fcol, bool vel) {
    const int c0 = fcol & 3;
    if (t >= L.col_start[c0] && t < (vel ? L.vel_end[c0] : L.col_start[c0 + 1])) return true;
    if (fcol < 4) return false;
    return t >= L.col_start[c0 + 2] && t < (vel ? L.vel_end[c0 + 2] : L.col_start[c0 + 3]);
}

// Interface vertex t of a full pass with the stencil record st.  With MIRROR
// its taps of x come from the mirror; with FUSE (which needs the mirror) the
// colour-fc vertices (velocity: those without Dirichlet data) are updated too.
template <typename T, int MODE, bool FUSE, bool MIRROR, bool DOP = false, bool GEN = false>
__device__ __forceinline__ void iface_full(const LevelDev<T>& L, const T* __restrict__ st, int t,
                                           const T* __restrict__ x, const T* __restrict__ b, T* xw,
                                           int fcol, T omega, T out[4], int fa = 0, int fb = 3,
                                           T* tt = nullptr) {
    static_assert(!FUSE || MIRROR, "fused updates keep the mirror current");
    const size_t len = (size_t)L.len, cs = (size_t)L.cstride;
    const int nif = L.nif;
    const int self = L.if_self[t];
    int s[15];
    s[0] = MIRROR ? t : self;
    const int32_t* taps = MIRROR ? L.if_tap : L.if_nb;
#pragma unroll
    for (int g = 1; g < 15; ++g) s[g] = taps[(g - 1) * nif + t];
    const bool dir = (L.if_flag[t] & 1) != 0;
    eval_node<T, MODE, DOP>(st, s, dir, MIRROR ? L.cx : x, MIRROR ? cs : len, b, len, self, out, fa,
                            fb, tt);
    // velocity rows of a free-slip vertex: their tangential part
    if ((MODE == MODE_APPLY || MODE == MODE_RES || MODE == MODE_RHS) && (L.if_flag[t] & 2))
        tangential(st + ST_NRM, out);
    if (FUSE && fused_vertex(L, t, fcol, MODE == MODE_RU)) {
        const int c0 = L.if_cptr[t];
        fused_update<T, MODE, true, GEN>(st, s, L.cx, cs, xw, len, out, omega, L.if_cptr[t + 1] - c0,
                                    L.if_copy + c0, L.cx, cs, t, fa, fb);
    }
}

// The fused colour updates of a windowed quad on Kuhn meshes: the quad's
// vertex of colour fcol, or its two vertices of parity fcol - 4.  Every
// neighbour value of every update is loaded before the first store (the
// updated vertices never read each other: their axis neighbours are of the
// other colours), so the lane waits on memory once rather than once per
// vertex and component; the arithmetic is fused_update's.
template <typename T, int MODE>
__device__ __forceinline__ void quad_fused_axis(const LevelDev<T>& L, const T* __restrict__ st,
                                                const Rows& R, int n, int j, int k, int q, int fcol,
                                                const T out[4][4], const T* __restrict__ x, T* xw,
                                                T omega) {
    const size_t len = (size_t)L.len, cs = (size_t)L.cstride;
    const int mm = n - k;
    int tp[2][7], cm[2];
    bool ok[2];
    T o[2][4];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int rc = ((fcol & 3) + 2 * j + k + 2 * e) & 3, i = 4 * q + rc;
        ok[e] = (e == 0 || fcol >= 4) && i >= 1 && i <= mm - 1 - j;
        axis_slots(R, i, tp[e]);
        cm[e] = ok[e] && near_boundary(n, i, j, k) ? L.comp_of_slot[tp[e][0]] : -1;
#pragma unroll
        for (int f = 0; f < 4; ++f)
            o[e][f] = rc == 0 ? out[0][f] : rc == 1 ? out[1][f] : rc == 2 ? out[2][f] : out[3][f];
    }
    if (MODE == MODE_RU) {
        T u[2][3][6];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (!ok[e]) continue;
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int g = 0; g < 6; ++g) u[e][f][g] = x[f * len + tp[e][g + 1]];
        }
        const T a1 = st[ST_A + 1], a2 = st[ST_A + 2], a3 = st[ST_A + 3], a4 = st[ST_A + 4],
                a7 = st[ST_A + 7], a8 = st[ST_A + 8], ia = st[ST_INVA];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (!ok[e]) continue;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const T v = o[e][f] - (a1 * u[e][f][0] + a2 * u[e][f][1] + a3 * u[e][f][2] +
                                       a4 * u[e][f][3] + a7 * u[e][f][4] + a8 * u[e][f][5]);
                const T un = v * ia;
                xw[f * len + tp[e][0]] = un;
                if (cm[e] >= 0) L.cx[f * cs + cm[e]] = un;
            }
        }
    } else {
        // the vertex's own pressure is read where it is written (through xw)
        T p[2][7];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (!ok[e]) continue;
            p[e][0] = xw[3 * len + tp[e][0]];
#pragma unroll
            for (int g = 1; g < 7; ++g) p[e][g] = x[3 * len + tp[e][g]];
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (!ok[e]) continue;
            const T cp = st[ST_C] * p[e][0] + st[ST_C + 1] * p[e][1] + st[ST_C + 2] * p[e][2] +
                         st[ST_C + 3] * p[e][3] + st[ST_C + 4] * p[e][4] + st[ST_C + 7] * p[e][5] +
                         st[ST_C + 8] * p[e][6];
            const T pn = p[e][0] + omega * (o[e][3] - cp) * st[ST_INVC];
            xw[3 * len + tp[e][0]] = pn;
            if (cm[e] >= 0) L.cx[3 * cs + cm[e]] = pn;
        }
    }
}

// WIN (RU and BP only): one block per tile, a quad per lane, quad windows.
// PART 1 / 2: a launch of the volume blocks only (ib = 0) or of the interface
// blocks only (grid = ib); each then gets the registers of its own branch.
// DOP (K x and the residual only): the D form a_2, every row from eval_node.
// GEN (fused passes only): the fused colour update of a general mesh, whose
// a_1 and c_l couple all 14 neighbours.
// TOUT (residual, Laplace form): the residual only enters the partial sums of
// its norm; y receives t = b_k - (B^T p)_k (k = 0..2) instead, the values of
// the f - B^T p pass up to rounding, for a smoothing step that follows at once.
template <typename T, int MODE, bool FUSE, bool MIRROR, bool WIN = false, int PART = 0,
          bool DOP = false, bool GEN = false, bool TOUT = false>
__global__ void __launch_bounds__(TPB) k_full(LevelDev<T> L, const T* __restrict__ x,
                                              const T* __restrict__ b,
                                              T* __restrict__ y, double* __restrict__ partials,
                                              int ib, T* xw, int fcol, T omega) {
    static_assert(!TOUT || (MODE == MODE_RES && !DOP && !FUSE && !GEN),
                  "t output: the residual of the Laplace form");
    static_assert(!WIN || MODE == MODE_RU || MODE == MODE_BP ||
                      ((MODE == MODE_APPLY || MODE == MODE_RES) && PART == 1 && !DOP && !GEN),
                  "quad windows: RU, BP, and the volume launch of K x and the residual");
    static_assert(!DOP || ((MODE == MODE_APPLY || MODE == MODE_RES || MODE == MODE_ARES) && !FUSE),
                  "D form: K x and the residuals");
    // fcol + 8: the rows of the vertices the pass updates are not stored (a
    // B u - g pass whose relaxed colour is not swept again in the step)
    const bool own_rows = fcol < 8;
    if (fcol >= 8) fcol -= 8;
    if (PART == 1) ib = 0;
    // volume block or interface block (decided at compile time for PART 1, 2)
    const bool vol = PART == 1 ? true : PART == 2 ? false : (int)blockIdx.x >= ib;
    __shared__ double sh[4];
    const size_t len = (size_t)L.len;
    int f0, f1;
    mode_fields<MODE>(f0, f1);
    double ss = 0.0;
    int slot = -1;   // partial-sum slot of this block
    if (WIN && vol) {
        const Tile tl = L.vtiles[blockIdx.x - ib];
        // K x and the residual: the tile's four partial-sum slots (one per
        // sub-row in the one-vertex-per-lane launch), the sum in the first
        if (MODE == MODE_RES && tl.macro >= 0) {
            slot = 4 * tl.nat;
            if (threadIdx.x >= 1 && threadIdx.x < 4) partials[slot + threadIdx.x] = 0.0;
        }
        if (tl.macro >= 0) {
            const int n = L.n, k = tl.k, mm = n - k;
            const LanePos P = decode_lane(tl, n, 1, mm - 2, threadIdx.x);
            if (P.ok) {
                const int j = P.j;
                Rows R;
                make_rows(L.slab_base, n, (int)(tl.macro * L.mstride), j, k, R);
                const T* st = L.st + (size_t)tl.macro * ST_SIZE;
                int w[7][6];
                quad_window_slots(R, P.q, w);
                T out[4][4], tt[4][3];
                quad_eval<T, MODE, TOUT>(st, w, x, b, len, out, tt);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * P.q + r;
                    if (i < 1 || i > mm - 1 - j) continue;
                    if (TOUT) {
#pragma unroll
                        for (int f = 0; f < 3; ++f) y[f * len + w[0][r + 1]] = tt[r][f];
#pragma unroll
                        for (int f = 0; f < 4; ++f) ss += (double)out[r][f] * (double)out[r][f];
                        continue;
                    }
                    if (MODE == MODE_BP && FUSE && !own_rows) {
                        const int cr = (i + 2 * j + 3 * k) & 3;
                        if (fcol < 4 ? cr == fcol : (cr & 1) == fcol - 4) continue;
                    }
                    for (int f = f0; f < f1; ++f) {
                        y[f * len + w[0][r + 1]] = out[r][f];
                        if (MODE == MODE_RES) ss += (double)out[r][f] * (double)out[r][f];
                    }
                }
                // the quad's vertex of colour fcol, or its two vertices of
                // parity fcol - 4 (red-black order)
                if constexpr (FUSE && !GEN) {
                    quad_fused_axis<T, MODE>(L, st, R, n, j, k, P.q, fcol, out, x, xw, omega);
                } else
                for (int e = 0; e < (FUSE ? (fcol < 4 ? 1 : 2) : 0); ++e) {
                    const int rc = ((fcol & 3) + 2 * j + k + 2 * e) & 3, i = 4 * P.q + rc;
                    if (i >= 1 && i <= mm - 1 - j) {
                        T o[4];
#pragma unroll
                        for (int f = 0; f < 4; ++f)
                            o[f] = rc == 0 ? out[0][f] : rc == 1 ? out[1][f] : rc == 2 ? out[2][f] : out[3][f];
                        int s7[GEN ? 15 : 7];
                        if (GEN)
                            nbr_slots(R, i, s7);
                        else
                            axis_slots(R, i, s7);
                        const int cm = near_boundary(n, i, j, k) ? L.comp_of_slot[s7[0]] : -1;
                        fused_update<T, MODE, false, GEN>(st, s7, x, len, xw, len, o, omega, 0,
                                                          nullptr, L.cx, (size_t)L.cstride, cm);
                    }
                }
            }
        }
    } else if (quad_lanes(MODE) && PART == 0 && vol) {
        const Tile tl = L.vtiles[blockIdx.x - ib];
        slot = tl.nat;
        if (tl.macro >= 0) {
            const int n = L.n, k = tl.k, mm = n - k;
            const LanePos P = decode_lane(tl, n, 1, mm - 2, threadIdx.x);
            if (P.ok) {
                const int j = P.j;
                Rows R;
                make_rows(L.slab_base, n, (int)(tl.macro * L.mstride), j, k, R);
                const T* st = L.st + (size_t)tl.macro * ST_SIZE;
#pragma unroll 1
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * P.q + r;
                    if (i < 1 || i > mm - 1 - j) continue;
                    int s[15];
                    nbr_slots(R, i, s);
                    T out[4], tt[3];
                    if (DOP)
                        eval_node<T, MODE, true>(st, s, false, x, len, b, len, s[0], out);
                    else if (MODE == MODE_APPLY || MODE == MODE_RES)
                        eval_vol_pairs<T, MODE>(st, s, x, b, len, out, TOUT ? tt : nullptr);
                    else
                        eval_node<T, MODE>(st, s, false, x, len, b, len, s[0], out);
                    if (TOUT) {
#pragma unroll
                        for (int f = 0; f < 3; ++f) y[f * len + s[0]] = tt[f];
#pragma unroll
                        for (int f = 0; f < 4; ++f) ss += (double)out[f] * (double)out[f];
                        continue;
                    }
                    for (int f = f0; f < f1; ++f) {
                        y[f * len + s[0]] = out[f];
                        if (MODE == MODE_RES) ss += (double)out[f] * (double)out[f];
                    }
                }
            }
        }
    } else if (vol) {
        const int v = (int)blockIdx.x - ib;
        const int ti = full_tile(v), r = full_sub(v);
        if (ti < L.n_vtiles) {
            const Tile tl = L.vtiles[ti];
            if (tl.macro >= 0) {
                slot = 4 * tl.nat + r;
                const int n = L.n, k = tl.k, mm = n - k;
                const LanePos P = decode_lane(tl, n, 1, mm - 2, threadIdx.x);
                const int j = P.j, i = 4 * P.q + r;
                if (P.ok && i >= 1 && i <= mm - 1 - j) {
                    Rows R;
                    make_rows(L.slab_base, n, (int)(tl.macro * L.mstride), j, k, R);
                    const T* st = L.st + (size_t)tl.macro * ST_SIZE;
                    int s[15];
                    nbr_slots(R, i, s);
                    T out[4];
                    if (MODE == MODE_ARES && !DOP) {
                        // volume rows: axis taps 1, 2, 3, 4, 7, 8 of the local order
                        const int tp[7] = {s[0], s[1], s[2], s[3], s[4], s[7], s[8]};
                        const int ca[7] = {0, 1, 2, 3, 4, 7, 8};
                        eval_ares<T>(st, tp, ca, false, x, len, b, len, s[0], out);
                    } else if (DOP) {
                        eval_node<T, MODE, true>(st, s, false, x, len, b, len, s[0], out);
                    } else if (MODE == MODE_APPLY || MODE == MODE_RES) {
                        eval_vol_pairs<T, MODE>(st, s, x, b, len, out);
                    } else {
                        eval_node<T, MODE>(st, s, false, x, len, b, len, s[0], out);
                    }
                    const bool upd = FUSE && (fcol < 4 ? ((i + 2 * j + 3 * k) & 3) == fcol
                                                       : ((i + 2 * j + 3 * k) & 1) == fcol - 4);
                    if (!(MODE == MODE_BP && upd && !own_rows))
                        for (int f = f0; f < f1; ++f) {
                            y[f * len + s[0]] = out[f];
                            if (MODE == MODE_RES) ss += (double)out[f] * (double)out[f];
                        }
                    if (upd) {
                        const int tp[7] = {s[0], s[1], s[2], s[3], s[4], s[7], s[8]};
                        const int cm = near_boundary(n, i, j, k) ? L.comp_of_slot[s[0]] : -1;
                        fused_update<T, MODE, false, GEN>(st, GEN ? s : tp, x, len, xw, len, out,
                                                          omega, 0, nullptr, L.cx,
                                                          (size_t)L.cstride, cm);
                    }
                }
            }
        }
    } else if (MODE == MODE_RU && FUSE) {
        // a lane per interface vertex and velocity component (the components
        // of f - B^T p and of the colour-fcol update are independent): the
        // scattered loads of the interface vertices spread over three times
        // as many workgroups
        const int q = (int)blockIdx.x * TPB + (int)threadIdx.x, t = q / 3, f = q % 3;
        if (t < L.nif) {
            const T* st = L.st + (size_t)L.if_sid[t] * ST_SIZE;
            T out[4];
            iface_full<T, MODE, FUSE, MIRROR, DOP, GEN>(L, st, t, x, b, xw, fcol, omega, out, f,
                                                        f + 1);
            const int c0 = L.if_cptr[t], c1 = L.if_cptr[t + 1];
            for (int q2 = c0; q2 < c1; ++q2) y[f * len + L.if_copy[q2]] = out[f];
        }
    } else if (MODE == MODE_BP && FUSE && MIRROR && !WIN) {
        // small levels: four lanes per interface vertex (groups of four
        // consecutive lanes, never split across waves): lane k < 3 sums B_k u_k
        // over the taps, two lane exchanges add the three sums, and lane 3 forms
        // B u - b_3, writes it and relaxes the pressure of a colour-fcol vertex.
        // The scattered loads of the few interface vertices spread over four
        // times as many lanes and workgroups.  (With quad windows the launch
        // carries the windows' register budget, and one lane per vertex is
        // faster.)
        const int q = (int)blockIdx.x * TPB + (int)threadIdx.x, t = q >> 2, k = q & 3;
        const bool act = t < L.nif;
        const size_t cs = (size_t)L.cstride;
        const int tt = act ? t : 0;
        const T* st = L.st + (size_t)L.if_sid[tt] * ST_SIZE;
        int sl[15];
        sl[0] = tt;
#pragma unroll
        for (int g = 1; g < 15; ++g) sl[g] = L.if_tap[(g - 1) * L.nif + tt];
        T part = T(0);
        if (act && k < 3) {
            const T* u = L.cx + k * cs;
#pragma unroll
            for (int g = 0; g < 15; ++g) part += st[ST_B + 15 * k + g] * u[sl[g]];
        }
        part += __shfl_xor(part, 1);
        part += __shfl_xor(part, 2);
        if (act && k == 3) {
            T out[4];
            out[3] = part - b[3 * len + L.if_self[t]];
            const int c0 = L.if_cptr[t], c1 = L.if_cptr[t + 1];
            const bool upd = fused_vertex(L, t, fcol, false);
            if (own_rows || !upd)
                for (int qq = c0; qq < c1; ++qq) y[3 * len + L.if_copy[qq]] = out[3];
            if (upd)
                fused_update<T, MODE, true, GEN>(st, sl, L.cx, cs, xw, len, out, omega, c1 - c0,
                                            L.if_copy + c0, L.cx, cs, t);
        }
    } else {
        if ((int)blockIdx.x * TPB < L.nif)
            slot = (quad_lanes(MODE) && PART == 0 ? 1 : 4) * L.nv_nat + (int)blockIdx.x;
        const int t = (int)blockIdx.x * TPB + (int)threadIdx.x;
        if (t < L.nif) {
            const T* st = L.st + (size_t)L.if_sid[t] * ST_SIZE;
            T out[4], tt[3];
            iface_full<T, MODE, FUSE, MIRROR, DOP, GEN>(L, st, t, x, b, xw, fcol, omega, out, 0, 3,
                                                        TOUT ? tt : nullptr);
            const int c0 = L.if_cptr[t], c1 = L.if_cptr[t + 1];
            if (TOUT) {
#pragma unroll
                for (int f = 0; f < 3; ++f)
                    for (int q = c0; q < c1; ++q) y[f * len + L.if_copy[q]] = tt[f];
#pragma unroll
                for (int f = 0; f < 4; ++f) ss += (double)out[f] * (double)out[f];
            }
            const bool skip = MODE == MODE_BP && FUSE && !own_rows && fused_vertex(L, t, fcol, false);
            for (int f = f0; f < (TOUT ? f0 : f1); ++f) {
                if (!skip)
                    for (int q = c0; q < c1; ++q) y[f * len + L.if_copy[q]] = out[f];
                if (MODE == MODE_RES) ss += (double)out[f] * (double)out[f];
            }
        }
    }
    if (MODE == MODE_RES) {
        const double tot = block_sum256(ss, sh);
        if (threadIdx.x == 0 && slot >= 0) partials[slot] = tot;
    }
}

// ---------------------------------------------------------------------------
// Restriction r_c = P^T r_f (weights 1 at the coincident vertex, 1/2 at its 14
// neighbours); velocity Dirichlet rows of the coarse level are zero.
// ---------------------------------------------------------------------------
// NF = 3: velocity fields only (multigrid for the velocity block).
template <typename T, int NF = 4>
__global__ void __launch_bounds__(TPB) k_restrict(LevelDev<T> C, LevelDev<T> F,
                                                  const T* __restrict__ rf, T* __restrict__ bc,
                                                  int ib) {
    const size_t lc = (size_t)C.len, lf = (size_t)F.len;
    if ((int)blockIdx.x >= ib) {
        // one coarse vertex per lane, four blocks per tile (dealt to XCDs as
        // in the full passes).  Coarse levels with n >= 128: each block takes
        // a quarter of the tile's quads with the four vertices of a quad in
        // consecutive lanes, so that a wave reads every fine vertex of a row
        // segment (the taps of one coarse vertex sit two fine vertices apart),
        // whole cache lines rather than every second entry of one sub-array;
        // smaller ones (shorter rows, where that was slower): one block per
        // sub-row r = i mod 4
        const int v = (int)blockIdx.x - ib;
        const int ti = full_tile(v), h = full_sub(v);
        if (ti >= C.n_vtiles) return;
        const Tile tl = C.vtiles[ti];
        if (tl.macro < 0) return;
        const int n = C.n, k = tl.k, mm = n - k;
        const bool spread = n >= 128;
        const int r = spread ? (int)threadIdx.x & 3 : h;
        const LanePos P =
            decode_lane(tl, n, 1, mm - 2, spread ? 64 * h + ((int)threadIdx.x >> 2) : (int)threadIdx.x);
        const int j = P.j, i = 4 * P.q + r;
        if (!P.ok || i < 1 || i > mm - 1 - j) return;
        Rows RF;
        make_rows(F.slab_base, F.n, (int)(tl.macro * F.mstride), 2 * j, 2 * k, RF);
        int s[15];
        nbr_slots(RF, 2 * i, s);
        const int sc = slot_of(C.slab_base, n, (int)(tl.macro * C.mstride), i, j, k);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T* vf = rf + f * lf;
            T acc = T(0);
#pragma unroll
            for (int g = 1; g < 15; ++g) acc += vf[s[g]];
            bc[f * lc + sc] = vf[s[0]] + T(0.5) * acc;
        }
        return;
    }
    // interface vertices: one lane per vertex and field, so that the
    // scattered loads of the few interface vertices of a small level spread
    // over NF times as many workgroups (and CUs)
    const int tf = (int)blockIdx.x * TPB + (int)threadIdx.x;
    const int t = tf / NF, f = tf - t * NF;
    if (t >= C.nif) return;
    const int nif = C.nif;
    const int self = C.rif_tap[t];
    int nb[14];
#pragma unroll
    for (int g = 0; g < 14; ++g) nb[g] = C.rif_tap[(g + 1) * nif + t];
    const bool dir = (C.if_flag[t] & 1) != 0;
    const int c0 = C.if_cptr[t], c1 = C.if_cptr[t + 1];
    if (f < 3 && (C.if_flag[t] & 2)) {
        // free-slip vertex: lane 0 restricts the three velocity fields and
        // keeps their tangential part
        if (f > 0) return;
        T w[3];
#pragma unroll
        for (int ff = 0; ff < 3; ++ff) {
            const T* v = rf + ff * lf;
            T acc = T(0);
#pragma unroll
            for (int g = 0; g < 14; ++g)
                if (nb[g] >= 0) acc += v[nb[g]];
            w[ff] = v[self] + T(0.5) * acc;
        }
        tangential(C.st + (size_t)C.if_sid[t] * ST_SIZE + ST_NRM, w);
        for (int q = c0; q < c1; ++q)
#pragma unroll
            for (int ff = 0; ff < 3; ++ff) bc[ff * lc + C.if_copy[q]] = w[ff];
        return;
    }
    const T* v = rf + f * lf;
    T acc = T(0);
#pragma unroll
    for (int g = 0; g < 14; ++g)
        if (nb[g] >= 0) acc += v[nb[g]];
    T val = v[self] + T(0.5) * acc;
    if (f < 3 && dir) val = T(0);
    for (int q = c0; q < c1; ++q) bc[f * lc + C.if_copy[q]] = val;
}

// ---------------------------------------------------------------------------
// Prolongation x_f += P e_c over every closure vertex of every macro: a fine
// vertex with even local index copies the coarse value, any other vertex is
// the midpoint of a coarse edge along the local direction given by its parity
// pattern.  Copies stay identical because every copy averages the same two
// coarse values.
// ---------------------------------------------------------------------------

// local edge direction whose midpoints have the parity pattern pi | pj<<1 | pk<<2
__host__ __device__ __forceinline__ void parity_dir(int pat, int* di, int* dj, int* dk) {
    switch (pat) {
        case 1: *di = 1; *dj = 0; *dk = 0; break;     // (1,0,0)
        case 2: *di = 0; *dj = 1; *dk = 0; break;     // (0,1,0)
        case 4: *di = 0; *dj = 0; *dk = 1; break;     // (0,0,1)
        case 3: *di = -1; *dj = 1; *dk = 0; break;    // (-1,1,0)
        case 6: *di = 0; *dj = -1; *dk = 1; break;    // (0,-1,1)
        case 5: *di = -1; *dj = 0; *dk = 1; break;    // (-1,0,1)
        default: *di = 1; *dj = -1; *dk = 1; break;   // (1,-1,1)
    }
}

// SET (full multigrid): x_f = P e_c instead of x_f += P e_c, except on the
// velocity slots of Dirichlet vertices, which keep their values.
// NF = 3: velocity fields only.  SLIP = false: the level has no free-slip
// vertex (no flag lookup on the lanes next to a macro boundary).
template <typename T, bool SET = false, int NF = 4, bool SLIP = true>
__global__ void __launch_bounds__(TPB) k_prolong(LevelDev<T> F, LevelDev<T> C,
                                                 const T* __restrict__ ec, T* __restrict__ xf) {
    const size_t lc = (size_t)C.len, lf = (size_t)F.len;
    // one fine closure vertex per lane, blocks mapped as in the full passes
    const int v = (int)blockIdx.x;
    const int ti = full_tile(v), r = full_sub(v);
    if (ti >= F.n_ctiles) return;
    const Tile tl = F.ctiles[ti];
    if (tl.macro < 0) return;
    const int n = F.n, k = tl.k, mm = n - k;
    const LanePos P = decode_lane(tl, n, 0, mm, threadIdx.x);
    const int j = P.j, i = 4 * P.q + r;
    if (!P.ok || i > mm - j) return;
    const int mbf = (int)(tl.macro * F.mstride), mbc = (int)(tl.macro * C.mstride);
    const int sf = slot_of(F.slab_base, n, mbf, i, j, k);
    // the fine level's mirror follows x (every copy of an interface vertex
    // computes the same value, so concurrent writes of its entry agree)
    const int cm = near_boundary(n, i, j, k) ? F.comp_of_slot[sf] : -1;
    const size_t cs = (size_t)F.cstride;
    // velocity slots kept by SET: those of Dirichlet vertices (interface
    // vertices, so their mirror entry is their list index)
    const bool keep = SET && cm >= 0 && cm < F.nif && (F.if_flag[cm] & 1);
    // free-slip vertex: the interpolated velocity keeps its tangential part
    const bool slip = SLIP && NF >= 3 && cm >= 0 && cm < F.nif && (F.if_flag[cm] & 2);
    const int pi = i & 1, pj = j & 1, pk = k & 1;
    T e[NF];
    if ((pi | pj | pk) == 0) {
        const int sc = slot_of(C.slab_base, C.n, mbc, i >> 1, j >> 1, k >> 1);
#pragma unroll
        for (int f = 0; f < NF; ++f) e[f] = ec[f * lc + sc];
    } else {
        int di, dj, dk;
        parity_dir(pi | (pj << 1) | (pk << 2), &di, &dj, &dk);
        const int sa = slot_of(C.slab_base, C.n, mbc, (i - di) >> 1, (j - dj) >> 1, (k - dk) >> 1);
        const int sb2 = slot_of(C.slab_base, C.n, mbc, (i + di) >> 1, (j + dj) >> 1, (k + dk) >> 1);
#pragma unroll
        for (int f = 0; f < NF; ++f) e[f] = T(0.5) * (ec[f * lc + sa] + ec[f * lc + sb2]);
    }
    if (slip) tangential(F.st + (size_t)F.if_sid[cm] * ST_SIZE + ST_NRM, e);
    // every field of the fine vertex read before the first store, so that
    // the lane waits on memory once
    T xv[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) xv[f] = (!SET || (keep && f < 3)) ? xf[f * lf + sf] : T(0);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        T v = e[f];
        if (!SET)
            v += xv[f];
        else if (keep && f < 3)
            v = xv[f];
        xf[f * lf + sf] = v;
        if (cm >= 0) F.cx[f * cs + cm] = v;
    }
}

// Level-0 start of full multigrid: every slot but the velocity slots of
// Dirichlet vertices set to zero.
template <typename T>
__global__ void k_keep_dirichlet(LevelDev<T> L, T* __restrict__ x) {
    const size_t s = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (s >= (size_t)L.len) return;
    const int cm = L.comp_of_slot[s];
    const bool dir = cm >= 0 && cm < L.nif && (L.if_flag[cm] & 1);
    const size_t len = (size_t)L.len;
#pragma unroll
    for (int f = 0; f < 3; ++f)
        if (!dir) x[f * len + s] = T(0);
    x[3 * len + s] = T(0);
}

// ---------------------------------------------------------------------------
// Viscosity gradient: per macro e, sum over its closure vertices x of
//   lam_u(x) . (A_e u)(x) + nu_e^-2 lam_p(x) ((C_e p)(x) + (G_e f)(x))
// with the one-sided unit-viscosity stencils of e; the caller negates.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int slot_checked(const int* __restrict__ sb, int n, int mb, int i, int j,
                                            int k) {
    if (i < 0 || j < 0 || k < 0 || i + j + k > n) return -1;
    return slot_of(sb, n, mb, i, j, k);
}
__device__ constexpr int LOFFD[15][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {-1, 1, 0}, {1, -1, 0},
                                         {0, 1, 0},  {0, -1, 0}, {0, -1, 1}, {0, 1, -1}, {-1, 0, 1},
                                         {1, 0, -1}, {0, 0, 1},  {0, 0, -1}, {1, -1, 1}, {-1, 1, -1}};

// dform: the velocity part from the coupled one-sided blocks of a_2.
__global__ void __launch_bounds__(TPB) k_grad_nu(LevelDev<double> L, const double* __restrict__ x,
                                                 const double* __restrict__ lam,
                                                 const double* __restrict__ f, double* partials,
                                                 int dform) {
    __shared__ double sh[4];
    const size_t len = (size_t)L.len;
    double acc = 0.0;
    const Tile tl = L.ctiles[blockIdx.x];
    if (tl.macro >= 0) {
        const int n = L.n, k = tl.k, mm = n - k;
        const LanePos P = decode_lane(tl, n, 0, mm, threadIdx.x);
        if (P.ok) {
            const int j = P.j, m = tl.macro;
            const int mb = (int)(m * L.mstride);
            const double inu2 = 1.0 / (L.macro_nu[m] * L.macro_nu[m]);
#pragma unroll 1
            for (int r = 0; r < 4; ++r) {
                const int i = 4 * P.q + r;
                if (i > mm - j) continue;
                const int pat = (mm - j - i == 0 ? 1 : 0) | (i == 0 ? 2 : 0) | (j == 0 ? 4 : 0) |
                                (k == 0 ? 8 : 0);
                const double* gs = L.gst + ((size_t)m * 16 + pat) * GR_SIZE;
                int s[15];
#pragma unroll
                for (int g = 0; g < 15; ++g)
                    s[g] = slot_checked(L.slab_base, n, mb, i + LOFFD[g][0], j + LOFFD[g][1],
                                        k + LOFFD[g][2]);
                double v = 0.0;
                if (dform) {
                    for (int c = 0; c < 3; ++c) {
                        double au = 0.0;
                        for (int l = 0; l < 3; ++l)
#pragma unroll
                            for (int g = 0; g < 15; ++g)
                                if (s[g] >= 0)
                                    au += gs[GR_A2 + 15 * (3 * c + l) + g] * x[l * len + s[g]];
                        v += lam[c * len + s[0]] * au;
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        double au = 0.0;
#pragma unroll
                        for (int g = 0; g < 15; ++g)
                            if (s[g] >= 0) au += gs[GR_A + g] * x[c * len + s[g]];
                        v += lam[c * len + s[0]] * au;
                    }
                }
                double cp = 0.0;
#pragma unroll
                for (int g = 0; g < 15; ++g)
                    if (s[g] >= 0) {
                        cp += gs[GR_C + g] * x[3 * len + s[g]];
                        if (f)
                            for (int c = 0; c < 3; ++c)
                                cp += gs[GR_G + 15 * c + g] * f[c * len + s[g]];
                    }
                v += inu2 * lam[3 * len + s[0]] * cp;
                acc += v;
            }
        }
    }
    const double tot = block_sum256(acc, sh);
    if (threadIdx.x == 0 && tl.nat >= 0) partials[tl.nat] = tot;
}

// Per-macro reduction of the gradient partials (one block per macro).  In
// natural order the closure tiles of macro m are a contiguous range.
__global__ void k_grad_reduce(const int* __restrict__ macro_tile0, const double* __restrict__ partials,
                              double* __restrict__ out) {
    __shared__ double sh[4];
    const int m = blockIdx.x;
    double acc = 0.0;
    for (int b = macro_tile0[m] + threadIdx.x; b < macro_tile0[m + 1]; b += TPB) acc += partials[b];
    const double tot = block_sum256(acc, sh);
    if (threadIdx.x == 0) out[m] = -tot;
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
// Sum of n partial sums (square root with sqrt_out) by one block of RTPB
// threads: a residual on the finest level leaves tens of thousands of
// partials, and a single block reads them at the rate of the loads it keeps
// in flight (sixteen waves, eight running sums per lane: entries b + m RTPB,
// m = 0..7, of each stride of 8 RTPB); fixed order, so the sum is the same
// on every run.
constexpr int RTPB = 1024;
__global__ void __launch_bounds__(RTPB) k_reduce_sum(const double* __restrict__ partials, int n,
                                                     double* __restrict__ out, int sqrt_out) {
    __shared__ double sh[RTPB / 64];
    double a[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) a[m] = 0.0;
    for (int b = threadIdx.x; b < n; b += 8 * RTPB) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
            if (b + m * RTPB < n) a[m] += partials[b + m * RTPB];
    }
    double v = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < RTPB / 64; ++w) tot += sh[w];
        out[0] = sqrt_out ? sqrt(tot) : tot;
    }
}

template <typename T>
__global__ void k_fill(T* __restrict__ x, size_t n, T v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        x[i] = v;
}

template <typename T>
__global__ void k_add(T* __restrict__ x, const T* __restrict__ y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        x[i] += y[i];
}

// y = x / s (s = device scalar), FP64 -> T
template <typename T>
__global__ void k_scale_cast(const double* __restrict__ x, const double* __restrict__ s,
                             T* __restrict__ y, size_t n) {
    const double inv = s[0] > 0.0 ? 1.0 / s[0] : 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        y[i] = (T)(x[i] * inv);
}

// x += s * e (s = device scalar), T -> FP64
template <typename T>
__global__ void k_axpy_cast(double* __restrict__ x, const double* __restrict__ s,
                            const T* __restrict__ e, size_t n) {
    const double sc = s[0];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        x[i] += sc * (double)e[i];
}

// weighted pressure sum sum_i m_i p_i over unique vertices (block partials);
// UNIT: the plain sum sum_i p_i
template <typename T, bool UNIT = false>
__global__ void __launch_bounds__(TPB) k_mass_dot(LevelDev<T> L, const T* __restrict__ p,
                                                  double* __restrict__ partials, int ib) {
    __shared__ double sh[4];
    double acc = 0.0;
    int slot = -1;
    if ((int)blockIdx.x >= ib) {
        const Tile tl = L.vtiles[blockIdx.x - ib];
        slot = tl.nat;
        if (tl.macro >= 0) {
            const int n = L.n, k = tl.k, mm = n - k;
            const LanePos P = decode_lane(tl, n, 1, mm - 2, threadIdx.x);
            if (P.ok) {
                const int j = P.j;
                const int b0 = (int)(tl.macro * L.mstride) + L.slab_base[k] + row_off(mm, j);
                const int Q0 = sub_stride(mm);
                const double w = UNIT ? 1.0 : (double)L.st[(size_t)tl.macro * ST_SIZE + ST_MASS];
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * P.q + r;
                    if (i < 1 || i > mm - 1 - j) continue;
                    acc += w * (double)p[at(b0, Q0, i)];
                }
            }
        }
    } else {
        if ((int)blockIdx.x * TPB < L.nif) slot = L.nv_nat + (int)blockIdx.x;
        const int t = (int)blockIdx.x * TPB + (int)threadIdx.x;
        if (t < L.nif)
            acc = (UNIT ? 1.0 : (double)L.st[(size_t)L.if_sid[t] * ST_SIZE + ST_MASS]) *
                  (double)p[L.if_self[t]];
    }
    const double tot = block_sum256(acc, sh);
    if (threadIdx.x == 0 && slot >= 0) partials[slot] = tot;
}

// Right-hand side of the adjoint system K lambda = (dJ/du on free velocity
// rows, Pi^T dJ/dp) from g = (dJ/du, dJ/dp) in the internal layout, with
// Pi^T q = q - m (sum_i q_i) / (sum_i m_i) the transpose of the mean-zero
// projection (applied when `project`); *psum holds sum_i q_i.  Launched
// over the volume tiles and the interface list like k_mass_dot; writes
// every vertex slot (all copies of interface vertices), padding untouched.
__global__ void __launch_bounds__(TPB) k_adjoint_rhs(LevelDev<double> L, const double* __restrict__ g,
                                                     double* __restrict__ y,
                                                     const double* __restrict__ psum,
                                                     double inv_mass, int project, int ib) {
    const size_t len = (size_t)L.len;
    const double mean = project ? psum[0] * inv_mass : 0.0;
    if ((int)blockIdx.x >= ib) {
        const Tile tl = L.vtiles[blockIdx.x - ib];
        if (tl.macro < 0) return;
        const int n = L.n, k = tl.k, mm = n - k;
        const LanePos P = decode_lane(tl, n, 1, mm - 2, threadIdx.x);
        if (!P.ok) return;
        const int j = P.j;
        const int b0 = (int)(tl.macro * L.mstride) + L.slab_base[k] + row_off(mm, j);
        const int Q0 = sub_stride(mm);
        const double w = L.st[(size_t)tl.macro * ST_SIZE + ST_MASS];
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * P.q + r;
            if (i < 1 || i > mm - 1 - j) continue;
            const size_t sl = (size_t)at(b0, Q0, i);
#pragma unroll
            for (int f = 0; f < 3; ++f) y[f * len + sl] = g[f * len + sl];
            y[3 * len + sl] = g[3 * len + sl] - w * mean;
        }
        return;
    }
    const int t = (int)blockIdx.x * TPB + (int)threadIdx.x;
    if (t >= L.nif) return;
    const int self = L.if_self[t];
    const bool dir = (L.if_flag[t] & 1) != 0;
    const double w = L.st[(size_t)L.if_sid[t] * ST_SIZE + ST_MASS];
    double v[4];
#pragma unroll
    for (int f = 0; f < 3; ++f) v[f] = dir ? 0.0 : g[f * len + self];
    v[3] = g[3 * len + self] - w * mean;
    for (int q = L.if_cptr[t]; q < L.if_cptr[t + 1]; ++q) {
        const size_t sl = (size_t)L.if_copy[q];
#pragma unroll
        for (int f = 0; f < 4; ++f) y[f * len + sl] = v[f];
    }
}

// p -= mean, mean = (sum_i m_i p_i) / (sum_i m_i) from a device scalar
template <typename T>
__global__ void k_sub_mean(T* __restrict__ p, size_t n, const double* __restrict__ wsum,
                           double inv_mass) {
    const T mean = (T)(wsum[0] * inv_mass);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] -= mean;
}

// The mirror taken from x: interface vertices (primary slots) and halo.
template <typename T>
__global__ void k_mirror_gather(LevelDev<T> L, const T* __restrict__ x) {
    const int e = (int)blockIdx.x * TPB + (int)threadIdx.x;
    if (e >= L.ncomp) return;
    const int sl = e < L.nif ? L.if_self[e] : L.halo_slot[e - L.nif];
#pragma unroll
    for (int f = 0; f < 4; ++f) L.cx[f * (size_t)L.cstride + e] = x[f * (size_t)L.len + sl];
}

// x <- v on n values and y <- v on m values (an iterate and its mirror)
template <typename T>
__global__ void k_fill2(T* __restrict__ x, size_t n, T* __restrict__ y, size_t m, T v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n + m;
         i += (size_t)gridDim.x * blockDim.x) {
        if (i < n)
            x[i] = v;
        else
            y[i - n] = v;
    }
}

// p -= mean on an iterate's pressure (n values) and its mirror (m values)
template <typename T>
__global__ void k_sub_mean2(T* __restrict__ p, size_t n, T* __restrict__ q, size_t m,
                            const double* __restrict__ wsum, double inv_mass) {
    const T mean = (T)(wsum[0] * inv_mass);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n + m;
         i += (size_t)gridDim.x * blockDim.x) {
        if (i < n)
            p[i] -= mean;
        else
            q[i - n] -= mean;
    }
}

// layout conversion and ghost exchange
__global__ void k_scatter(const int* __restrict__ slot_node, size_t len, int nfields,
                          const double* __restrict__ nodal, size_t N, double* __restrict__ x) {
    for (size_t s = blockIdx.x * (size_t)blockDim.x + threadIdx.x; s < len;
         s += (size_t)gridDim.x * blockDim.x) {
        const int v = slot_node[s];
        for (int f = 0; f < nfields; ++f) x[f * len + s] = v >= 0 ? nodal[f * N + v] : 0.0;
    }
}
__global__ void k_gather(const int* __restrict__ node_slot, size_t N, int nfields,
                         const double* __restrict__ x, size_t len, double* __restrict__ nodal) {
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < N;
         v += (size_t)gridDim.x * blockDim.x) {
        const int s = node_slot[v];   // -1: a lattice point in no macro (hole)
        for (int f = 0; f < nfields; ++f) nodal[f * N + v] = s >= 0 ? x[f * len + s] : 0.0;
    }
}
template <typename T>
__global__ void k_exchange(LevelDev<T> L, int nfields, T* __restrict__ x) {
    const int t = blockIdx.x * TPB + threadIdx.x;
    if (t >= L.nif) return;
    const size_t len = (size_t)L.len;
    const int self = L.if_self[t];
    for (int f = 0; f < nfields; ++f) {
        const T v = x[f * len + self];
        for (int q = L.if_cptr[t]; q < L.if_cptr[t + 1]; ++q) x[f * len + L.if_copy[q]] = v;
    }
}

// ---------------------------------------------------------------------------
// Coarse grid (Section 3.7): block-diagonal preconditioned MINRES on the
// level-0 Stokes system in one workgroup.  The preconditioner is
// diag(A_0^-1 (dense inverse, per velocity component), lumped mass weighted
// by 1/nu); the recurrence is the standard preconditioned MINRES (Lanczos in
// the preconditioner inner product with Givens rotations).
// ---------------------------------------------------------------------------
struct CoarseDev {
    int nd, nfv, N, maxit, project;
    double tol, inv_mass;
    int nnz;
    const int* rowptr;
    const int* col;
    const double* val;
    const double* ainv;     // symmetric [nfv][nfv]
    const double* pdinv;    // [N]
    const double* sinv;     // [N][N] symmetric, used when schur != 0
    int schur;
    const double* mass;     // [N]
    const int* vel_node;    // [nfv]
    const int* node_vidx;   // [N] compact velocity index or -1
    const int* node_slot;   // [N]
    const int* node_cptr;   // [N+1]
    const int* node_copy;
    double* gscratch;       // 8 * nd doubles when the vectors do not fit in LDS
    double* zinv;           // [nb][nb] inverse of the bordered level-0 matrix up to
                            // the column permutation zperm (direct solver)
    const int* zperm;       // [nb]
    int nb;
    const double* a2inv;    // D form: [3 nfv][3 nfv] inverse of the coupled velocity block
    int coupled;            // 1: the velocity block couples the components (D form)
    // what lives in the dynamic LDS (in this order): vectors, CSR (val, then
    // col and row pointers), A^-1, S^-1
    int vec_lds, csr_lds, ainv_lds, sinv_lds;
};

constexpr int CTPB = 1024;

__device__ __forceinline__ double csum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int q = 0; q < nw; ++q) t += red[q];
    return t;
}

// Products of the coarse solve: every row is handled by a segment of SEG
// consecutive lanes that split its entries and combine them with shuffles,
// so that all 1024 threads work and the dependent load chains stay short.
constexpr int SEG = 8;

__device__ __forceinline__ double seg_sum(double v) {
#pragma unroll
    for (int o = SEG / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, SEG);
    return v;
}

// y_c = M x_c for nb right-hand sides of a dense symmetric M [n][n] stored
// row-major (row r is contiguous)
__device__ __forceinline__ void seg_gemv(const double* __restrict__ M, int n, int nb,
                                         const double* __restrict__ x, double* __restrict__ y) {
    const int sl = threadIdx.x % SEG, g = threadIdx.x / SEG, ng = blockDim.x / SEG;
    for (int rr = g; rr < n * nb; rr += ng) {
        const int c = rr / n, r = rr - c * n;
        const double* xc = x + c * n;
        double acc = 0.0;
        for (int q = sl; q < n; q += SEG) acc += M[(size_t)r * n + q] * xc[q];
        acc = seg_sum(acc);
        if (sl == 0) y[rr] = acc;
    }
}

__device__ void coarse_precond(const CoarseDev& cd, const double* ainv, const double* sinv,
                               const double* __restrict__ v, double* __restrict__ z) {
    const int nfv = cd.nfv;
    seg_gemv(ainv, nfv, 3, v, z);    // the three velocity components at once
    if (cd.schur) {
        seg_gemv(sinv, cd.N, 1, v + 3 * nfv, z + 3 * nfv);
    } else {
        for (int i = threadIdx.x; i < cd.N; i += blockDim.x) z[3 * nfv + i] = cd.pdinv[i] * v[3 * nfv + i];
    }
}

// q = K z s (CSR, z scaled by s on the fly); returns this thread's share of
// (z s) . q
__device__ __forceinline__ double coarse_matvec(const CoarseDev& cd, const int* rowptr, const int* col,
                                                const double* val, const double* __restrict__ z,
                                                double sc, double* __restrict__ q) {
    const int sl = threadIdx.x % SEG, g = threadIdx.x / SEG, ng = blockDim.x / SEG;
    double part = 0.0;
    for (int i = g; i < cd.nd; i += ng) {
        double acc = 0.0;
        for (int e = rowptr[i] + sl; e < rowptr[i + 1]; e += SEG) acc += val[e] * z[col[e]];
        acc = seg_sum(acc) * sc;
        if (sl == 0) {
            q[i] = acc;
            part += acc * z[i] * sc;
        }
    }
    return part;
}

template <typename T>
__global__ void __launch_bounds__(CTPB) k_coarse(CoarseDev cd, const T* __restrict__ b, size_t blen,
                                                 T* __restrict__ x, size_t xlen,
                                                 double* __restrict__ stats) {
    extern __shared__ double smem[];
    __shared__ double red[16];
    const int nd = cd.nd, nfv = cd.nfv, N = cd.N;
    // carve the dynamic LDS
    double* lds = smem;
    double* base = cd.vec_lds ? lds : cd.gscratch;
    if (cd.vec_lds) lds += 8 * nd;
    const double* val = cd.val;
    const int* col = cd.col;
    const int* rowptr = cd.rowptr;
    if (cd.csr_lds) {
        double* v_ = lds;
        int* c_ = reinterpret_cast<int*>(v_ + cd.nnz);
        int* r_ = c_ + cd.nnz;
        for (int e = threadIdx.x; e < cd.nnz; e += blockDim.x) {
            v_[e] = cd.val[e];
            c_[e] = cd.col[e];
        }
        for (int i = threadIdx.x; i <= nd; i += blockDim.x) r_[i] = cd.rowptr[i];
        val = v_;
        col = c_;
        rowptr = r_;
        lds += cd.nnz + (cd.nnz + nd + 2) / 2;
    }
    const double* ainv = cd.ainv;
    if (cd.ainv_lds) {
        for (int e = threadIdx.x; e < nfv * nfv; e += blockDim.x) lds[e] = cd.ainv[e];
        ainv = lds;
        lds += (size_t)nfv * nfv;
    }
    const double* sinv = cd.sinv;
    if (cd.sinv_lds) {
        for (int e = threadIdx.x; e < N * N; e += blockDim.x) lds[e] = cd.sinv[e];
        sinv = lds;
        lds += (size_t)N * N;
    }
    double* vo = base;
    double* v = vo + nd;
    double* z = v + nd;
    double* zn = z + nd;
    double* q = zn + nd;
    double* wo = q + nd;
    double* w = wo + nd;
    double* xs = w + nd;
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
        double bi;
        if (i < 3 * nfv) {
            const int c = i / nfv;
            bi = (double)b[c * blen + cd.node_slot[cd.vel_node[i - c * nfv]]];
        } else {
            bi = (double)b[3 * blen + cd.node_slot[i - 3 * nfv]];
        }
        v[i] = bi;
        vo[i] = 0.0;
        wo[i] = 0.0;
        w[i] = 0.0;
        xs[i] = 0.0;
    }
    __syncthreads();
    double part = 0.0;
    if (cd.project) {
        // K_0 is singular (constant pressure); make the right-hand side
        // consistent the way the mean-zero constraint does: b_p -= mu m with
        // mu = (sum_i b_p,i) / (sum_i m_i), the Lagrange multiplier of
        // sum_i m_i p_i = 0.  Rounding in the restricted residual would
        // otherwise leave a small inconsistent part that MINRES cannot remove.
        for (int i = threadIdx.x; i < N; i += blockDim.x) part += v[3 * nfv + i];
        const double mu = csum(part, red) * cd.inv_mass;
        for (int i = threadIdx.x; i < N; i += blockDim.x) v[3 * nfv + i] -= mu * cd.mass[i];
        __syncthreads();
        part = 0.0;
    }
    coarse_precond(cd, ainv, sinv, v, z);
    __syncthreads();
    for (int i = threadIdx.x; i < nd; i += blockDim.x) part += z[i] * v[i];
    double gamma = sqrt(fmax(csum(part, red), 0.0));
    const double gamma1 = gamma;
    double eta = gamma, gamma_old = 1.0;
    double c0 = 1.0, c1 = 1.0, s0 = 0.0, s1 = 0.0;
    int it = 0;
    double rel = 0.0;
    if (gamma1 > 0.0) {
        for (it = 1; it <= cd.maxit; ++it) {
            // z <- z / gamma is folded into the product; the scaled z is
            // stored for the direction update below
            const double ig = 1.0 / gamma;
            part = coarse_matvec(cd, rowptr, col, val, z, ig, q);
            const double delta = csum(part, red);
            for (int i = threadIdx.x; i < nd; i += blockDim.x) z[i] *= ig;
            const double a = delta / gamma, bq = gamma / gamma_old;
            for (int i = threadIdx.x; i < nd; i += blockDim.x) q[i] = q[i] - a * v[i] - bq * vo[i];
            __syncthreads();
            coarse_precond(cd, ainv, sinv, q, zn);
            __syncthreads();
            part = 0.0;
            for (int i = threadIdx.x; i < nd; i += blockDim.x) part += zn[i] * q[i];
            const double gnew = sqrt(fmax(csum(part, red), 0.0));
            const double al0 = c1 * delta - c0 * s1 * gamma;
            const double al1 = sqrt(al0 * al0 + gnew * gnew);
            const double al2 = s1 * delta + c0 * c1 * gamma;
            const double al3 = s0 * gamma;
            c0 = c1;
            s0 = s1;
            c1 = al0 / al1;
            s1 = gnew / al1;
            const double ce = c1 * eta;
            for (int i = threadIdx.x; i < nd; i += blockDim.x) {
                const double wn = (z[i] - al3 * wo[i] - al2 * w[i]) / al1;
                wo[i] = wn;   // becomes the new w after the swap below
                xs[i] += ce * wn;
            }
            __syncthreads();
            eta = -s1 * eta;
            // rotate buffers: (vo, v, q) <- (v, q, vo); (z, zn) swap; (wo, w) swap
            double* t0 = vo;
            vo = v;
            v = q;
            q = t0;
            double* t1 = z;
            z = zn;
            zn = t1;
            double* t2 = wo;
            wo = w;
            w = t2;
            gamma_old = gamma;
            gamma = gnew;
            rel = fabs(eta) / gamma1;
            if (rel <= cd.tol || gnew == 0.0) break;
        }
        if (it > cd.maxit) it = cd.maxit;
    }
    // zero-mean pressure
    if (cd.project) {
        part = 0.0;
        for (int i = threadIdx.x; i < N; i += blockDim.x) part += cd.mass[i] * xs[3 * nfv + i];
        const double mean = csum(part, red) * cd.inv_mass;
        for (int i = threadIdx.x; i < N; i += blockDim.x) xs[3 * nfv + i] -= mean;
        __syncthreads();
    }
    for (int vtx = threadIdx.x; vtx < N; vtx += blockDim.x) {
        const int iv = cd.node_vidx[vtx];
        T val4[4];
        for (int c = 0; c < 3; ++c) val4[c] = iv >= 0 ? (T)xs[c * nfv + iv] : T(0);
        val4[3] = (T)xs[3 * nfv + vtx];
        for (int e = cd.node_cptr[vtx]; e < cd.node_cptr[vtx + 1]; ++e) {
            const int sl = cd.node_copy[e];
            for (int c = 0; c < 4; ++c) x[c * xlen + sl] = val4[c];
        }
    }
    if (threadIdx.x == 0 && stats) {
        stats[0] = (double)it;
        stats[1] = rel;
    }
}

// ---------------------------------------------------------------------------
// Set-up of the direct level-0 solver: in-place Gauss-Jordan inversion of the
// bordered level-0 matrix M [nb][nb] with partial pivoting, one pivot column
// per three launches.  Step c swaps the pivot row into row c, scales it by
// the pivot and eliminates column c from every other row; the row swaps
// leave the inverse with its columns permuted (perm), which the solve undoes
// by reading the right-hand side through perm.
// ---------------------------------------------------------------------------
struct GJState {
    int piv, bad;
    double p;     // pivot value
    double acc;   // M[c][c] before the swap
    double tiny;  // pivots at or below this magnitude make the matrix singular
};

// pivot search over rows c..nb-1 of column c (one workgroup)
__global__ void __launch_bounds__(1024) k_gj_pivot(const double* __restrict__ M, int nb, int c,
                                                   int* __restrict__ perm, GJState* st) {
    __shared__ double sv[16];
    __shared__ int si[16];
    double best = -1.0;
    int bi = c;
    for (int r = c + (int)threadIdx.x; r < nb; r += blockDim.x) {
        const double v = fabs(M[(size_t)r * nb + c]);
        if (v > best) {
            best = v;
            bi = r;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov > best || (ov == best && oi < bi)) {
            best = ov;
            bi = oi;
        }
    }
    if ((threadIdx.x & 63) == 0) {
        sv[threadIdx.x >> 6] = best;
        si[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            if (sv[w] > best || (sv[w] == best && si[w] < bi)) {
                best = sv[w];
                bi = si[w];
            }
        st->piv = bi;
        st->acc = M[(size_t)c * nb + c];
        double p = M[(size_t)bi * nb + c];
        if (!(fabs(p) > st->tiny)) {
            st->bad = 1;
            p = 1.0;   // keeps the remaining steps finite; the result is discarded
        }
        st->p = p;
        const int t = perm[c];
        perm[c] = perm[bi];
        perm[bi] = t;
    }
}

// row swap and scaling of the pivot row; col receives column c of the other
// rows after the swap (the elimination factors)
__global__ void k_gj_swap(double* __restrict__ M, int nb, int c, const GJState* __restrict__ st,
                          double* __restrict__ col) {
    const int i = (int)blockIdx.x * blockDim.x + (int)threadIdx.x;
    if (i >= nb) return;
    const int piv = st->piv;
    const double p = st->p;
    const double a = M[(size_t)c * nb + i], bv = M[(size_t)piv * nb + i];
    M[(size_t)c * nb + i] = (i == c ? 1.0 : bv) / p;
    if (piv != c) M[(size_t)piv * nb + i] = a;
    // rows other than c and piv are not written by this launch
    col[i] = i == c ? 0.0 : i == piv ? st->acc : M[(size_t)i * nb + c];
}

// elimination of column c from every row r != c (rows with a zero factor are
// unchanged)
__global__ void k_gj_update(double* __restrict__ M, int nb, int c, const double* __restrict__ col) {
    const int r = (int)blockIdx.y;
    const int q = (int)blockIdx.x * blockDim.x + (int)threadIdx.x;
    if (r == c || q >= nb) return;
    const double f = col[r];
    if (f == 0.0) return;
    double* mr = M + (size_t)r * nb;
    mr[q] = (q == c ? 0.0 : mr[q]) - f * M[(size_t)c * nb + q];
}

// ---------------------------------------------------------------------------
// Direct level-0 solve x0 = Z b0 with Z the leading block of the inverse of
// the level-0 system bordered by the mean constraint: one wave per row of Z
// (rows are contiguous), the gathered b0 (and the border's zero) staged in
// LDS by every workgroup and read through the column permutation.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(TPB) k_coarse_direct(CoarseDev cd, const T* __restrict__ b,
                                                       size_t blen, T* __restrict__ x, size_t xlen,
                                                       double* __restrict__ stats) {
    extern __shared__ double bl[];
    const int nd = cd.nd, nfv = cd.nfv, N = cd.N, nb = cd.nb;
    for (int i = threadIdx.x; i < nb; i += TPB) {
        if (i < 3 * nfv) {
            const int c = i / nfv;
            bl[i] = (double)b[c * blen + cd.node_slot[cd.vel_node[i - c * nfv]]];
        } else if (i < nd) {
            bl[i] = (double)b[3 * blen + cd.node_slot[i - 3 * nfv]];
        } else {
            bl[i] = 0.0;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int row = (int)blockIdx.x * (TPB / 64) + ((int)threadIdx.x >> 6);
    if (row < nd) {
        const double* z = cd.zinv + (size_t)row * nb;
        const int* __restrict__ perm = cd.zperm;
        double acc = 0.0;
        for (int q = lane; q < nb; q += 64) acc += z[q] * bl[perm[q]];
        acc = wave_sum(acc);
        if (lane == 0) {
            int comp, vtx;
            if (row < 3 * nfv) {
                comp = row / nfv;
                vtx = cd.vel_node[row - comp * nfv];
            } else {
                comp = 3;
                vtx = row - 3 * nfv;
            }
            for (int e = cd.node_cptr[vtx]; e < cd.node_cptr[vtx + 1]; ++e)
                x[comp * xlen + cd.node_copy[e]] = (T)acc;
        }
    }
    // velocity of the Dirichlet vertices: no correction
    const int g = (int)blockIdx.x * TPB + (int)threadIdx.x;
    if (g < N && cd.node_vidx[g] < 0)
        for (int e = cd.node_cptr[g]; e < cd.node_cptr[g + 1]; ++e)
            for (int c = 0; c < 3; ++c) x[c * xlen + cd.node_copy[e]] = T(0);
    if (blockIdx.x == 0 && threadIdx.x == 0 && stats) {
        stats[0] = 1.0;
        stats[1] = 0.0;
    }
}

}  // namespace hhg
