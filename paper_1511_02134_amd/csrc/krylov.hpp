// Kernels of the global Krylov solvers (Section 3.1, Algorithm 1: the
// Schur-complement CG; Section 3.2: MINRES with the block-diagonal
// preconditioner of eq. precond_block_diag): the level-0 solve of the
// velocity multigrid and the vector updates of the finest level.
//
// Vectors hold 4 fields of `len` slots (u, v, w, p); every copy of an
// interface vertex carries the vertex's value and padding slots hold zeros,
// so elementwise updates run over all slots and keep both properties.  Inner
// products count every vertex once: the `owned` byte of a slot is 1 for the
// vertex's primary slot only.  Partial sums go to one entry per workgroup of
// a fixed grid, reduced in a fixed order (deterministic results).
#pragma once
#include "kernels.hpp"

namespace hhg {

constexpr int VGRID_MAX = 2048;   // workgroups of the reducing vector kernels

// Velocity block of the level-0 system: x_k = A_0^-1 b_k on the free
// vertices (every copy), zero on Dirichlet vertices, k = 0..2 (D form: the
// coupled block, x = A_2,0^-1 b over all three components at once).  One wave
// per row of the dense inverse; b gathered into LDS by every workgroup.
template <typename T>
__global__ void __launch_bounds__(TPB) k_coarse_avel(CoarseDev cd, const T* __restrict__ b,
                                                     size_t blen, T* __restrict__ x, size_t xlen) {
    extern __shared__ double bl[];
    const int nfv = cd.nfv, N = cd.N;
    for (int i = threadIdx.x; i < 3 * nfv; i += TPB) {
        const int c = i / nfv;
        bl[i] = (double)b[c * blen + cd.node_slot[cd.vel_node[i - c * nfv]]];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int row = (int)blockIdx.x * (TPB / 64) + ((int)threadIdx.x >> 6);
    if (row < 3 * nfv) {
        const int comp = row / nfv, r = row - comp * nfv;
        double acc = 0.0;
        if (cd.coupled) {
            const double* a = cd.a2inv + (size_t)row * 3 * nfv;
            for (int q = lane; q < 3 * nfv; q += 64) acc += a[q] * bl[q];
        } else {
            const double* a = cd.ainv + (size_t)r * nfv;
            const double* bb = bl + comp * nfv;
            for (int q = lane; q < nfv; q += 64) acc += a[q] * bb[q];
        }
        acc = wave_sum(acc);
        if (lane == 0) {
            const int vtx = cd.vel_node[r];
            for (int e = cd.node_cptr[vtx]; e < cd.node_cptr[vtx + 1]; ++e)
                x[comp * xlen + cd.node_copy[e]] = (T)acc;
        }
    }
    const int g = (int)blockIdx.x * TPB + (int)threadIdx.x;
    if (g < N && cd.node_vidx[g] < 0)
        for (int e = cd.node_cptr[g]; e < cd.node_cptr[g + 1]; ++e)
            for (int c = 0; c < 3; ++c) x[c * xlen + cd.node_copy[e]] = T(0);
}

// workgroup partial of a reduction into part[blockIdx.x]
__device__ __forceinline__ void put_partial(double v, double* __restrict__ part) {
    __shared__ double sh[4];
    const double tot = block_sum256(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// sum_{owned slots} sum_{f < nf} a[f][s] b[f][s]
__global__ void __launch_bounds__(TPB) k_vdot(const double* __restrict__ a,
                                              const double* __restrict__ b,
                                              const uint8_t* __restrict__ owned, size_t len,
                                              int nf, double* __restrict__ part) {
    double acc = 0.0;
    for (size_t s = blockIdx.x * (size_t)TPB + threadIdx.x; s < len; s += (size_t)gridDim.x * TPB) {
        if (!owned[s]) continue;
        for (int f = 0; f < nf; ++f) acc += a[f * len + s] * b[f * len + s];
    }
    put_partial(acc, part);
}

// Lanczos step of MINRES on unnormalised vectors V_j = beta_j v_j, Z_j =
// beta_j z_j with Q = K Z_j:  V_{j-1} <- Q / beta - (alpha / beta) V_j -
// (beta / beta_prev) V_{j-1}, alpha = <Q, Z_j> / beta^2 read from dq.
__global__ void __launch_bounds__(TPB) k_mr_lanczos(const double* __restrict__ Q,
                                                    const double* __restrict__ V,
                                                    double* __restrict__ Vold, size_t n4,
                                                    double beta, double cprev,
                                                    const double* __restrict__ dq) {
    const double ia = 1.0 / beta;
    const double cb = dq[0] * ia * ia * ia;
    for (size_t i = blockIdx.x * (size_t)TPB + threadIdx.x; i < n4; i += (size_t)gridDim.x * TPB)
        Vold[i] = Q[i] * ia - cb * V[i] - cprev * Vold[i];
}

// Pressure block of the preconditioner, Z_p = V_p / (lumped mass weighted by
// 1/nu), with the inner product <V, Z> over all four fields (the velocity of
// Z comes from the velocity multigrid).
__global__ void __launch_bounds__(TPB) k_mr_precp_dot(const double* __restrict__ V,
                                                      double* __restrict__ Z,
                                                      const double* __restrict__ pinv,
                                                      const uint8_t* __restrict__ owned,
                                                      size_t len, double* __restrict__ part) {
    double acc = 0.0;
    for (size_t s = blockIdx.x * (size_t)TPB + threadIdx.x; s < len; s += (size_t)gridDim.x * TPB) {
        const double vp = V[3 * len + s], zp = vp * pinv[s];
        Z[3 * len + s] = zp;
        if (!owned[s]) continue;
        acc += V[s] * Z[s] + V[len + s] * Z[len + s] + V[2 * len + s] * Z[2 * len + s] + vp * zp;
    }
    put_partial(acc, part);
}

// Search direction, solution and residual of MINRES:
//   W_j  = (Z_j / beta - eps W_{j-2} - delta W_{j-1}) / gamma   (into W2)
//   x   += tau W_j
//   KW_j = (Q / beta - eps KW_{j-2} - delta KW_{j-1}) / gamma   (into KW2)
//   r   -= tau KW_j,  partial sums of |r|^2 over owned slots
struct MrCoef {
    double zs;    // 1 / (beta gamma)
    double e;     // eps / gamma
    double d;     // delta / gamma
    double tau;
};

__global__ void __launch_bounds__(TPB) k_mr_update(const double* __restrict__ Z,
                                                   double* __restrict__ W2,
                                                   const double* __restrict__ W1,
                                                   double* __restrict__ X,
                                                   const double* __restrict__ Q,
                                                   double* __restrict__ KW2,
                                                   const double* __restrict__ KW1,
                                                   double* __restrict__ Rr,
                                                   const uint8_t* __restrict__ owned, size_t len,
                                                   MrCoef k, double* __restrict__ part) {
    double acc = 0.0;
    for (size_t s = blockIdx.x * (size_t)TPB + threadIdx.x; s < len; s += (size_t)gridDim.x * TPB) {
        const bool own = owned[s] != 0;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const size_t i = f * len + s;
            const double w = Z[i] * k.zs - k.e * W2[i] - k.d * W1[i];
            W2[i] = w;
            X[i] += k.tau * w;
            const double kw = Q[i] * k.zs - k.e * KW2[i] - k.d * KW1[i];
            KW2[i] = kw;
            const double r = Rr[i] - k.tau * kw;
            Rr[i] = r;
            if (own) acc += r * r;
        }
    }
    put_partial(acc, part);
}

// Start of the CG on the Schur complement from the pass y = C p - B u:
//   rho = B u - C p - g = -y - g,  z = rho / M,  d = z,  partial <rho, z>
__global__ void __launch_bounds__(TPB) k_cg_start(const double* __restrict__ y,
                                                  const double* __restrict__ g,
                                                  double* __restrict__ rho,
                                                  double* __restrict__ z,
                                                  double* __restrict__ d,
                                                  const double* __restrict__ pinv,
                                                  const uint8_t* __restrict__ owned, size_t len,
                                                  double* __restrict__ part) {
    double acc = 0.0;
    for (size_t s = blockIdx.x * (size_t)TPB + threadIdx.x; s < len; s += (size_t)gridDim.x * TPB) {
        const double r = -y[s] - g[s], zz = r * pinv[s];
        rho[s] = r;
        z[s] = zz;
        d[s] = zz;
        if (owned[s]) acc += r * zz;
    }
    put_partial(acc, part);
}

// CG step with y = S d:  a = rz / <d, y> (0 when <d, y> = 0),  p += a d,
// rho -= a y,  z = rho / M,  partial <rho, z>
__global__ void __launch_bounds__(TPB) k_cg_step(double* __restrict__ p,
                                                 const double* __restrict__ d,
                                                 double* __restrict__ rho,
                                                 const double* __restrict__ y,
                                                 double* __restrict__ z,
                                                 const double* __restrict__ pinv,
                                                 const uint8_t* __restrict__ owned, size_t len,
                                                 const double* __restrict__ rz,
                                                 const double* __restrict__ dy,
                                                 double* __restrict__ part) {
    const double a = dy[0] != 0.0 ? rz[0] / dy[0] : 0.0;
    double acc = 0.0;
    for (size_t s = blockIdx.x * (size_t)TPB + threadIdx.x; s < len; s += (size_t)gridDim.x * TPB) {
        p[s] += a * d[s];
        const double r = rho[s] - a * y[s], zz = r * pinv[s];
        rho[s] = r;
        z[s] = zz;
        if (owned[s]) acc += r * zz;
    }
    put_partial(acc, part);
}

// d = z + (rz_new / rz) d  (coefficient 0 when rz = 0)
__global__ void __launch_bounds__(TPB) k_cg_dir(double* __restrict__ d,
                                                const double* __restrict__ z, size_t len,
                                                const double* __restrict__ rz_new,
                                                const double* __restrict__ rz) {
    const double bta = rz[0] != 0.0 ? rz_new[0] / rz[0] : 0.0;
    for (size_t s = blockIdx.x * (size_t)TPB + threadIdx.x; s < len; s += (size_t)gridDim.x * TPB)
        d[s] = z[s] + bta * d[s];
}

__global__ void k_copy(double* __restrict__ y, const double* __restrict__ x, size_t n) {
    for (size_t i = blockIdx.x * (size_t)TPB + threadIdx.x; i < n; i += (size_t)gridDim.x * TPB)
        y[i] = x[i];
}

}  // namespace hhg
