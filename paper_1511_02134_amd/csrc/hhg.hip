// C ABI of the Uzawa multigrid Stokes solver: context, workspace layout,
// device upload and the multigrid driver (Sections 3.3 - 3.7).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hhg.h"
#include "hierarchy.hpp"
#include "kernels.hpp"
#include "krylov.hpp"

using namespace hhg;

// Static scratch of hhg_residual_noalloc: the per-block partial sums of the
// residual norm, for callers that cannot allocate.  Every GPU the library
// runs on holds its own copy until the process ends.  In host code the
// array's name is not a device address: the address of the current device's
// copy comes from hipGetSymbolAddress (scratch_address below).
constexpr size_t NOALLOC_SCRATCH_DOUBLES = size_t(1) << 20;   // 8 MiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {

// device address of `scratch` on device dev (which must be current), looked
// up once per device and kept
std::mutex g_scratch_mu;
double* g_scratch_addr[256] = {};

hipError_t scratch_address(int dev, double** out) {
    if (dev < 0 || dev >= 256) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

thread_local std::string g_error;

// leading interface blocks of a launch: ceil(count / TPB), padded to a multiple of 8
inline int iface_blocks(int count) { return ((count + TPB - 1) / TPB + 7) / 8 * 8; }

struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(char* b) : base(b) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) / 256 * 256;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

struct DevLevelArrays {
    int32_t *slab_base, *if_self, *if_nb, *if_sid, *if_cptr, *if_copy, *if_flag, *rif_tap;
    Tile *vtiles, *ctiles;
    double *st64, *gst64, *nu64;
    float *st32, *gst32, *nu32;
    int32_t *slot_node, *node_slot;
    int32_t* ctile_macro0;   // [nm+1] first natural closure tile of each macro
    int32_t *if_tap, *halo_slot, *comp_of_slot;
    double* cx64;            // mirror of the level's iterate (4 fields x cstride)
    float* cx32;
    // work vectors (4 fields each)
    double *x64, *b64, *r64, *t64;
    float *x32, *b32, *r32, *t32;
    // finest level: primary-slot flags (inner products count each vertex
    // once) and 1 / (lumped pressure mass weighted by 1/nu) on every copy
    uint8_t* owned;
    double* pinv;
    // hybrid ordering: grouped interface lists, cross-primitive tap masks and
    // the class's starting values of the interface vertices (4 fields x nif)
    int32_t *hyb_list, *hyb_mask;
    double* snap64;
    float* snap32;
};

constexpr int KV_N = 10;   // finest-level vectors of the Krylov solvers

struct TimerPair {
    hipEvent_t a, b;
    int n;          // launches between the two events
    int lev = -1;   // phase pairs: the level whose work they bracket
};

}  // namespace

struct hhg_ctx {
    MeshInfo mi;
    hhg_opts opts;
    int R = 0, L = 0;
    std::vector<HostLevel> H;
    CoarseHost CH;
    bool device = false;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<DevLevelArrays> A;
    std::vector<LevelDev<double>> D64;
    std::vector<LevelDev<float>> D32;
    CoarseDev cd{};
    size_t coarse_smem = 0;
    double* partials = nullptr;
    int npartials = 0;
    double* scal = nullptr;        // small device scalars
    double* kv[KV_N] = {};         // Krylov vectors (4 fields each; opts.krylov)
    double* kpart = nullptr;       // partial sums of the vector kernels
    double* kscal = nullptr;       // device scalars of the Krylov solvers
    double* gpart = nullptr;       // gradient partials
    double* gj_col = nullptr;      // set-up of the direct coarse solver: elimination factors
    GJState* gj_state = nullptr;   // and pivot state
    std::vector<double> inv_mass;  // 1 / sum_i m_i per level
    // operator evaluations per level (A, B, C, M) since the last reset; a
    // colour sweep counts a quarter of its operator (Section 4.2)
    std::vector<std::array<double, 4>> opc;
    // captured solver cycles (hhg_solve), re-used while x and b stay the same
    struct CycleGraph {
        const void* x;
        const void* b;
        hipGraphExec_t exec;
        std::vector<std::array<double, 4>> ops;   // operator counts of one replay
    };
    std::vector<CycleGraph> graphs;
    hipStream_t cap = nullptr;
    std::string err;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> evpool;
    size_t evused = 0;
    std::vector<TimerPair> tpairs[HHG_K_NCLASS];
    int tgroup_cls = -1;   // class whose launches a TimedGroup brackets together
    int tgroup_n = 0;
    double tbytes[HHG_K_NCLASS] = {0, 0, 0, 0};
    // algorithmic bytes per launch (finest level) of the timed classes
    double bytes_vel[4] = {0, 0, 0, 0}, bytes_pres[4] = {0, 0, 0, 0};
    double bytes_ru = 0, bytes_bp = 0, bytes_res = 0;
    // index 0..3: one fused colour; 4, 5: the two colours of a red-black parity
    double bytes_ru_fused[6] = {0, 0, 0, 0, 0, 0}, bytes_bp_fused[6] = {0, 0, 0, 0, 0, 0};
    int dev = -1;                  // device of the workspace
    double* scratch = nullptr;     // that device's copy of the static scratch
    // phase timing of hhg_solve (smoothing, transfers, coarse solve, residuals)
    bool phase_timing = false, phase_active = false;
    std::vector<TimerPair> ppairs[4];
};

namespace {

hhg_status fail(hhg_ctx* c, hhg_status s, const std::string& msg) {
    if (c) c->err = msg;
    g_error = msg;
    return s;
}

#define HIPCHECK(ctx, call)                                                         \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            return fail(ctx, HHG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool opts_ok(const hhg_opts* o, std::string* err) {
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 == 0 || o->nu1 > 64 || o->nu2 > 64) {
        *err = "smoothing steps must be in 0..64 with nu1 + nu2 > 0";
        return false;
    }
    if (o->cycle < 0 || o->cycle > 1 || o->p_sweep < 0 || o->p_sweep > 1 || o->precision < 0 ||
        o->precision > 1 || o->block_order < 0 || o->block_order > 2) {
        *err = "invalid option value";
        return false;
    }
    if (!(o->omega > 0.0 && o->omega < 2.0)) {
        *err = "omega must lie in (0, 2)";
        return false;
    }
    if (!(o->coarse_rtol > 0.0) || o->coarse_maxit < 1 || o->coarse_maxit > 100000 ||
        o->coarse_prec < 0 || o->coarse_prec > 1 || o->coarse_solver < 0 || o->coarse_solver > 1) {
        *err = "invalid coarse solver settings";
        return false;
    }
    if (o->krylov < 0 || o->krylov > 1 || o->graphs < 0 || o->graphs > 1) {
        *err = "krylov and graphs must be 0 or 1";
        return false;
    }
    if (o->op < 0 || o->op > 1) {
        *err = "op must be 0 (Laplace form) or 1 (D form)";
        return false;
    }
    if (o->op == 1 && o->coarse_solver != 0) {
        *err = "the D form needs the exact coarse solver (coarse_solver = 0)";
        return false;
    }
    if (o->ordering < 0 || o->ordering > 2) {
        *err = "ordering must be 0 (colours), 1 (hybrid primitive classes) or 2 (red-black)";
        return false;
    }
    if (o->ordering == 2 && (o->op != 0 || o->krylov != 0)) {
        *err = "the red-black ordering runs the Laplace form without the Krylov solvers";
        return false;
    }
    if (o->ordering == 1 && (o->op != 0 || o->krylov != 0)) {
        *err = "the hybrid ordering runs the Laplace form without the Krylov solvers";
        return false;
    }
    return true;
}

// The full passes over velocity rows run the point-block kernels, which read
// every tap of the coupled blocks: the D form, and general meshes (whose a_1
// stencils couple all 14 neighbours; their records hold the blocks
// delta_kl A).  The colour sweeps of general meshes with a_1 read the 15
// taps of A per component instead.
inline bool dpath(const hhg_ctx* c) { return c->opts.op == 1 || c->mi.general; }

// level-0 system of the context's options: the solution operator for the
// direct solver, the dense Schur complement only for MINRES preconditioned
// with it
bool build_coarse_for(hhg_ctx* c, std::string* err) {
    const bool direct = c->opts.coarse_solver == 0;
    const bool schur = c->opts.coarse_solver == 1 && c->opts.coarse_prec == 0;
    return build_coarse(c->mi, c->H[0], direct, schur, c->opts.op == 1, &c->CH, err);
}

// Builds the host hierarchy and computes the workspace layout (when ws is
// NULL only the size).
hhg_status build_host(hhg_ctx* c, const hhg_mesh* mesh, int R, const hhg_opts* opts) {
    std::string err;
    if (!mesh) return fail(c, HHG_EINVAL, "mesh is NULL");
    if (R < 2 || R > 10) return fail(c, HHG_EINVAL, "n_refine must lie in 2..10");
    hhg_opts o;
    hhg_default_opts(&o);
    if (opts) o = *opts;
    if (!opts_ok(&o, &err)) return fail(c, HHG_EINVAL, err);
    if (!validate_mesh(mesh, &c->mi, &err)) return fail(c, HHG_EINVAL, err);
    c->mi.lap_blocks = c->mi.general && o.op == 0;
    if (o.ordering == 2 && c->mi.general)
        return fail(c, HHG_EINVAL,
                    "the red-black ordering needs Kuhn macros (general stencils couple colours two apart)");
    if (c->mi.slip && (o.op != 0 || o.ordering != 0 || o.krylov != 0 || o.coarse_solver != 0))
        return fail(c, HHG_EINVAL,
                    "free-slip faces need the Laplace form, the colour ordering, the direct coarse "
                    "solver and no Krylov vectors");
    c->opts = o;
    c->R = R;
    c->L = R - 2;
    c->H.resize(c->L + 1);
    for (int l = 0; l <= c->L; ++l)
        if (!build_level(c->mi, l + 2, o.block_order, &c->H[l], &err))
            return fail(c, HHG_EINVAL, err);
    for (int l = 0; l < c->L; ++l) {
        link_levels(&c->H[l], c->H[l + 1]);
        for (int32_t t : c->H[l].rif_fine)
            if (t < 0) return fail(c, HHG_EINVAL, "internal error: coarse interface vertex missing");
    }
    if (!build_coarse_for(c, &err)) return fail(c, HHG_EINVAL, err);
    return HHG_OK;
}

// fields of the compact mirror are padded to 64 entries
inline int64_t mirror_stride(int32_t ncomp) { return ((int64_t)ncomp + 63) / 64 * 64; }
template <typename T>
T* mirror_of(DevLevelArrays& a);
template <>
double* mirror_of<double>(DevLevelArrays& a) { return a.cx64; }
template <>
float* mirror_of<float>(DevLevelArrays& a) { return a.cx32; }

size_t layout(hhg_ctx* c, char* ws) {
    Carver cv(ws);
    const int nl = c->L + 1;
    c->A.assign(nl, DevLevelArrays{});
    const bool mixed = c->opts.precision == 1;
    int maxblocks = 1;
    for (int l = 0; l < nl; ++l) {
        HostLevel& h = c->H[l];
        DevLevelArrays& a = c->A[l];
        a.slab_base = cv.take<int32_t>(h.slab_base.size());
        a.vtiles = cv.take<Tile>(std::max<size_t>(1, h.vtiles.size()));
        a.ctiles = cv.take<Tile>(std::max<size_t>(1, h.ctiles.size()));
        a.if_self = cv.take<int32_t>(std::max(1, h.nif));
        a.if_nb = cv.take<int32_t>(std::max<size_t>(1, h.if_nb.size()));
        a.if_sid = cv.take<int32_t>(std::max(1, h.nif));
        a.if_cptr = cv.take<int32_t>(h.if_cptr.size());
        a.if_copy = cv.take<int32_t>(std::max<size_t>(1, h.if_copy.size()));
        a.if_flag = cv.take<int32_t>(std::max(1, h.nif));
        a.rif_tap = l < c->L ? cv.take<int32_t>((size_t)15 * std::max(1, h.nif)) : nullptr;
        a.st64 = cv.take<double>(h.st.size());
        a.gst64 = cv.take<double>(h.gst.size());
        a.nu64 = cv.take<double>(h.nm);
        a.st32 = cv.take<float>(h.st.size());
        a.gst32 = cv.take<float>(h.gst.size());
        a.nu32 = cv.take<float>(h.nm);
        a.slot_node = cv.take<int32_t>(h.len);
        a.ctile_macro0 = cv.take<int32_t>(h.nm + 1);
        a.node_slot = cv.take<int32_t>(h.N);
        a.if_tap = cv.take<int32_t>(std::max<size_t>(1, h.if_tap.size()));
        a.halo_slot = cv.take<int32_t>(std::max<size_t>(1, h.halo_slot.size()));
        a.comp_of_slot = cv.take<int32_t>(h.len);
        const size_t c4 = 4 * (size_t)mirror_stride(h.ncomp);
        a.cx64 = cv.take<double>(c4);
        a.cx32 = mixed ? cv.take<float>(c4) : nullptr;
        const size_t v4 = 4 * (size_t)h.len;
        a.r64 = cv.take<double>(v4);
        a.t64 = cv.take<double>(v4);
        // corrections and right-hand sides of the coarser levels; on the finest
        // level the caller's x and b take their place
        a.x64 = l < c->L ? cv.take<double>(v4) : nullptr;
        a.b64 = l < c->L ? cv.take<double>(v4) : nullptr;
        a.x32 = a.b32 = a.r32 = a.t32 = nullptr;
        if (mixed) {
            a.x32 = cv.take<float>(v4);
            a.b32 = cv.take<float>(v4);
            a.r32 = cv.take<float>(v4);
            a.t32 = cv.take<float>(v4);
        }
        a.hyb_list = cv.take<int32_t>(std::max<size_t>(1, h.hyb_list.size()));
        a.hyb_mask = cv.take<int32_t>(std::max<size_t>(1, h.hyb_mask.size()));
        a.snap64 = c->opts.ordering == 1 ? cv.take<double>((size_t)4 * std::max(1, h.nif)) : nullptr;
        a.snap32 = c->opts.ordering == 1 && mixed ? cv.take<float>((size_t)4 * std::max(1, h.nif))
                                                  : nullptr;
        a.owned = nullptr;
        a.pinv = nullptr;
        if (l == c->L) {
            a.owned = cv.take<uint8_t>(h.len);
            a.pinv = cv.take<double>(h.len);
            for (int q = 0; q < KV_N; ++q)
                c->kv[q] = c->opts.krylov ? cv.take<double>(v4) : nullptr;
        }
        const int nb = full_blocks((int)h.vtiles.size()) + iface_blocks(h.nif);
        maxblocks = std::max(maxblocks, nb);
        maxblocks = std::max(maxblocks, (int)h.ctiles.size());
    }
    c->npartials = maxblocks;
    c->partials = cv.take<double>(maxblocks);
    c->gpart = cv.take<double>(maxblocks);
    c->scal = cv.take<double>(64);
    c->kpart = cv.take<double>(VGRID_MAX);
    c->kscal = cv.take<double>(16);
    // coarse system
    CoarseHost& C = c->CH;
    CoarseDev& d = c->cd;
    d.nd = C.nd;
    d.nfv = C.nfv;
    d.N = C.N;
    d.rowptr = cv.take<int32_t>(C.rowptr.size());
    d.col = cv.take<int32_t>(std::max<size_t>(1, C.col.size()));
    d.val = cv.take<double>(std::max<size_t>(1, C.val.size()));
    d.ainv = cv.take<double>(std::max<size_t>(1, C.ainv.size()));
    d.pdinv = cv.take<double>(C.N);
    d.sinv = cv.take<double>(std::max<size_t>(1, C.sinv.size()));
    d.mass = cv.take<double>(C.N);
    d.vel_node = cv.take<int32_t>(std::max(1, C.nfv));
    d.node_vidx = cv.take<int32_t>(C.N);
    d.node_slot = cv.take<int32_t>(C.N);
    d.node_cptr = cv.take<int32_t>(C.node_cptr.size());
    d.node_copy = cv.take<int32_t>(C.node_copy.size());
    d.gscratch = cv.take<double>((size_t)8 * C.nd);
    // direct solver: the bordered matrix, inverted in place at set-up, its
    // column permutation, the elimination factors and the pivot state
    d.nb = C.nb;
    d.zinv = cv.take<double>(std::max<size_t>(1, C.kb.size()));
    d.zperm = cv.take<int32_t>(std::max(1, C.nb));
    c->gj_col = cv.take<double>(std::max(1, C.nb));
    c->gj_state = cv.take<GJState>(1);
    d.a2inv = cv.take<double>(std::max<size_t>(1, C.a2inv.size()));
    d.coupled = C.a2inv.empty() ? 0 : 1;
    return cv.off + 256;
}

template <typename T>
void fill_view(hhg_ctx* c, int l, LevelDev<T>& v) {
    HostLevel& h = c->H[l];
    DevLevelArrays& a = c->A[l];
    v.n = h.n;
    v.nm = h.nm;
    v.mstride = h.mstride;
    v.len = h.len;
    v.slab_base = a.slab_base;
    v.vtiles = a.vtiles;
    v.n_vtiles = (int32_t)h.vtiles.size();
    v.nv_nat = 0;
    for (const Tile& t : h.vtiles) v.nv_nat += t.macro >= 0 ? 1 : 0;
    v.ctiles = a.ctiles;
    v.n_ctiles = (int32_t)h.ctiles.size();
    v.nif = h.nif;
    v.if_self = a.if_self;
    v.if_nb = a.if_nb;
    v.if_sid = a.if_sid;
    v.if_cptr = a.if_cptr;
    v.if_copy = a.if_copy;
    v.if_flag = a.if_flag;
    for (int q = 0; q < 5; ++q) v.col_start[q] = h.col_start[q];
    for (int q = 0; q < 4; ++q) v.vel_end[q] = h.vel_end[q];
    for (int q = 0; q < 4; ++q) v.slip_beg[q] = h.slip_beg[q];
    v.rif_tap = a.rif_tap;
    v.ncomp = h.ncomp;
    v.cstride = mirror_stride(h.ncomp);
    v.if_tap = a.if_tap;
    v.halo_slot = a.halo_slot;
    v.comp_of_slot = a.comp_of_slot;
    v.cx = mirror_of<T>(a);
}

template <typename T>
hhg_status upload(hhg_ctx* c, T* dst, const void* src, size_t count) {
    if (count == 0) return HHG_OK;
    HIPCHECK(c, hipMemcpy(dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    return HHG_OK;
}

// Direct level-0 solver: uploads the bordered matrix and inverts it in place
// on the device (Gauss-Jordan with partial pivoting, three launches per
// column); fails when a pivot vanishes relative to the largest entry.
hhg_status coarse_direct_setup(hhg_ctx* c) {
    CoarseHost& C = c->CH;
    const int nb = C.nb;
    if (nb == 0) return HHG_OK;
    hhg_status s;
    if ((s = upload<double>(c, c->cd.zinv, C.kb.data(), C.kb.size())) != HHG_OK) return s;
    std::vector<int32_t> perm(nb);
    for (int i = 0; i < nb; ++i) perm[i] = i;
    if ((s = upload<int32_t>(c, (int32_t*)c->cd.zperm, perm.data(), perm.size())) != HHG_OK) return s;
    double scale = 0.0;
    for (double v : C.kb) scale = std::max(scale, std::fabs(v));
    GJState st0{0, 0, 1.0, 0.0, 1e-13 * scale};
    if ((s = upload<GJState>(c, c->gj_state, &st0, 1)) != HHG_OK) return s;
    const hipStream_t st = nullptr;
    double* M = c->cd.zinv;
    const dim3 ugrid((nb + TPB - 1) / TPB, nb);
    for (int col = 0; col < nb; ++col) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, st, M, nb, col,
                           (int*)c->cd.zperm, c->gj_state);
        hipLaunchKernelGGL(k_gj_swap, dim3((nb + TPB - 1) / TPB), dim3(TPB), 0, st, M, nb, col,
                           c->gj_state, c->gj_col);
        hipLaunchKernelGGL(k_gj_update, ugrid, dim3(TPB), 0, st, M, nb, col, c->gj_col);
    }
    HIPCHECK(c, hipGetLastError());
    GJState st1;
    HIPCHECK(c, hipMemcpy(&st1, c->gj_state, sizeof(GJState), hipMemcpyDeviceToHost));
    if (st1.bad) return fail(c, HHG_EINVAL, "level-0 system is singular");
    std::vector<double>().swap(C.kb);   // the device holds the inverse
    return HHG_OK;
}

hhg_status upload_stencils(hhg_ctx* c) {
    for (int l = 0; l <= c->L; ++l) {
        HostLevel& h = c->H[l];
        DevLevelArrays& a = c->A[l];
        std::vector<double> nu(h.nm);
        for (int m = 0; m < h.nm; ++m) nu[m] = c->mi.macros[m].nu;
        std::vector<float> st32(h.st.begin(), h.st.end()), gst32(h.gst.begin(), h.gst.end()),
            nu32(nu.begin(), nu.end());
        hhg_status s;
        if ((s = upload<double>(c, a.st64, h.st.data(), h.st.size())) != HHG_OK) return s;
        if ((s = upload<double>(c, a.gst64, h.gst.data(), h.gst.size())) != HHG_OK) return s;
        if ((s = upload<double>(c, a.nu64, nu.data(), nu.size())) != HHG_OK) return s;
        if ((s = upload<float>(c, a.st32, st32.data(), st32.size())) != HHG_OK) return s;
        if ((s = upload<float>(c, a.gst32, gst32.data(), gst32.size())) != HHG_OK) return s;
        if ((s = upload<float>(c, a.nu32, nu32.data(), nu32.size())) != HHG_OK) return s;
        c->D64[l].st = a.st64;
        c->D64[l].gst = a.gst64;
        c->D64[l].macro_nu = a.nu64;
        c->D32[l].st = a.st32;
        c->D32[l].gst = a.gst32;
        c->D32[l].macro_nu = a.nu32;
        double msum = 0.0;
        for (int64_t v = 0; v < h.N; ++v) {
            if (h.node_slot[v] < 0) continue;   // hole
            int sid = h.node_sid[v];
            const double* rec = sid < 0 ? &h.st_vol_global[(size_t)(-sid - 1) * ST_SIZE]
                                        : &h.st[(size_t)sid * ST_SIZE];
            msum += rec[ST_MASS];
        }
        c->inv_mass[l] = 1.0 / msum;
    }
    CoarseHost& C = c->CH;
    hhg_status s;
    if ((s = upload<double>(c, (double*)c->cd.val, C.val.data(), C.val.size())) != HHG_OK) return s;
    if ((s = upload<double>(c, (double*)c->cd.ainv, C.ainv.data(), C.ainv.size())) != HHG_OK)
        return s;
    if ((s = upload<double>(c, (double*)c->cd.pdinv, C.pdinv.data(), C.pdinv.size())) != HHG_OK)
        return s;
    if ((s = upload<double>(c, (double*)c->cd.sinv, C.sinv.data(), C.sinv.size())) != HHG_OK)
        return s;
    if ((s = coarse_direct_setup(c)) != HHG_OK) return s;
    if (!C.a2inv.empty() &&
        (s = upload<double>(c, (double*)c->cd.a2inv, C.a2inv.data(), C.a2inv.size())) != HHG_OK)
        return s;
    if ((s = upload<double>(c, (double*)c->cd.mass, C.mass.data(), C.mass.size())) != HHG_OK)
        return s;
    c->cd.inv_mass = c->inv_mass[0];
    {
        // pressure preconditioner of the Krylov solvers on the finest level:
        // 1 / (lumped pressure mass weighted by 1/nu) on every copy; it
        // depends on the viscosity, so it is rebuilt with the stencils
        HostLevel& h = c->H[c->L];
        std::vector<double> pinv((size_t)h.len, 0.0);
        for (int64_t q = 0; q < h.len; ++q) {
            const int32_t nd = h.slot_node[q];
            if (nd < 0) continue;
            const int32_t sid = h.node_sid[nd];
            const double* rec = sid < 0 ? &h.st_vol_global[(size_t)(-sid - 1) * ST_SIZE]
                                        : &h.st[(size_t)sid * ST_SIZE];
            pinv[q] = 1.0 / rec[ST_MASSNU];
        }
        if ((s = upload<double>(c, c->A[c->L].pinv, pinv.data(), pinv.size())) != HHG_OK) return s;
    }
    return HHG_OK;
}

hhg_status upload_all(hhg_ctx* c) {
    const int nl = c->L + 1;
    c->D64.assign(nl, LevelDev<double>{});
    c->D32.assign(nl, LevelDev<float>{});
    c->inv_mass.assign(nl, 0.0);
    c->opc.assign(nl, std::array<double, 4>{0.0, 0.0, 0.0, 0.0});
    for (int l = 0; l < nl; ++l) {
        HostLevel& h = c->H[l];
        DevLevelArrays& a = c->A[l];
        hhg_status s;
#define UP(T, dst, vec) \
    if ((s = upload<T>(c, dst, vec.data(), vec.size())) != HHG_OK) return s;
        UP(int32_t, a.slab_base, h.slab_base);
        UP(Tile, a.vtiles, h.vtiles);
        UP(Tile, a.ctiles, h.ctiles);
        UP(int32_t, a.if_self, h.if_self);
        UP(int32_t, a.if_nb, h.if_nb);
        UP(int32_t, a.if_sid, h.if_sid);
        UP(int32_t, a.if_cptr, h.if_cptr);
        UP(int32_t, a.if_copy, h.if_copy);
        UP(int32_t, a.if_flag, h.if_flag);
        if (!h.rif_tap.empty()) UP(int32_t, a.rif_tap, h.rif_tap);
        UP(int32_t, a.slot_node, h.slot_node);
        UP(int32_t, a.node_slot, h.node_slot);
        UP(int32_t, a.if_tap, h.if_tap);
        UP(int32_t, a.halo_slot, h.halo_slot);
        UP(int32_t, a.comp_of_slot, h.comp_of_slot);
        UP(int32_t, a.hyb_list, h.hyb_list);
        UP(int32_t, a.hyb_mask, h.hyb_mask);
        {
            std::vector<int32_t> m0(h.nm + 1, 0);
            for (const Tile& t : h.ctiles)
                if (t.macro >= 0) m0[t.macro + 1]++;
            for (int m = 0; m < h.nm; ++m) m0[m + 1] += m0[m];
            UP(int32_t, a.ctile_macro0, m0);
        }
        fill_view(c, l, c->D64[l]);
        fill_view(c, l, c->D32[l]);
    }
    CoarseHost& C = c->CH;
    CoarseDev& d = c->cd;
    std::vector<int32_t> vidx(C.N, -1);
    for (int i = 0; i < C.nfv; ++i) vidx[C.vel_node[i]] = i;
    hhg_status s;
    UP(int32_t, (int32_t*)d.rowptr, C.rowptr);
    UP(int32_t, (int32_t*)d.col, C.col);
    UP(int32_t, (int32_t*)d.vel_node, C.vel_node);
    UP(int32_t, (int32_t*)d.node_vidx, vidx);
    UP(int32_t, (int32_t*)d.node_slot, C.node_slot);
    UP(int32_t, (int32_t*)d.node_cptr, C.node_cptr);
    UP(int32_t, (int32_t*)d.node_copy, C.node_copy);
#undef UP
    d.maxit = c->opts.coarse_maxit;
    d.tol = c->opts.coarse_rtol;
    d.project = c->mi.project ? 1 : 0;
    d.schur = c->opts.coarse_prec == 0 ? 1 : 0;
    // dynamic LDS of the coarse kernel: vectors, then the CSR matrix, A^-1
    // and S^-1, each only if it still fits into the device's per-workgroup LDS
    {
        int dev = 0, maxlds = 65536;
        if (hipGetDevice(&dev) == hipSuccess) {
            int v = 0;
            if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                    hipSuccess && v > 0)
                maxlds = v;
        }
        const size_t budget = (size_t)maxlds - 1024;   // static LDS of the kernel
        d.nnz = (int)C.val.size();
        size_t used = 0;
        const size_t vb = (size_t)8 * C.nd * sizeof(double);
        const size_t cb = ((size_t)d.nnz + ((size_t)d.nnz + C.nd + 2) / 2) * sizeof(double);
        const size_t ab = (size_t)C.nfv * C.nfv * sizeof(double);
        const size_t sbytes = (size_t)C.N * C.N * sizeof(double);
        d.vec_lds = used + vb <= budget;
        if (d.vec_lds) used += vb;
        d.csr_lds = used + cb <= budget;
        if (d.csr_lds) used += cb;
        d.ainv_lds = used + ab <= budget;
        if (d.ainv_lds) used += ab;
        d.sinv_lds = d.schur && used + sbytes <= budget;
        if (d.sinv_lds) used += sbytes;
        c->coarse_smem = used;
        if (used > 65536) {
            if (hipFuncSetAttribute((const void*)k_coarse<double>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)used) != hipSuccess ||
                hipFuncSetAttribute((const void*)k_coarse<float>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)used) != hipSuccess)
                return fail(c, HHG_EDEVICE, "cannot raise the LDS limit of the coarse kernel");
        }
        const size_t dl = (size_t)C.nb * sizeof(double);   // k_coarse_direct's staged b0
        if (dl > 65536 &&
            (hipFuncSetAttribute((const void*)k_coarse_direct<double>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)dl) != hipSuccess ||
             hipFuncSetAttribute((const void*)k_coarse_direct<float>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)dl) != hipSuccess))
            return fail(c, HHG_EDEVICE, "cannot raise the LDS limit of the direct coarse kernel");
    }
    if ((s = upload_stencils(c)) != HHG_OK) return s;
    {
        // primary-slot flags of the finest level (inner products count each
        // vertex once); the pressure preconditioner came with the stencils
        HostLevel& h = c->H[c->L];
        std::vector<uint8_t> own((size_t)h.len, 0);
        for (int64_t q = 0; q < h.len; ++q) {
            const int32_t nd = h.slot_node[q];
            if (nd >= 0 && h.node_slot[nd] == q) own[q] = 1;
        }
        DevLevelArrays& a = c->A[c->L];
        if ((s = upload<uint8_t>(c, a.owned, own.data(), own.size())) != HHG_OK) return s;
    }
    // algorithmic bytes of the timed kernel classes on the finest level
    HostLevel& h = c->H[c->L];
    double Nc[4] = {0, 0, 0, 0}, Nfc[4] = {0, 0, 0, 0}, Nf = 0;
    for (int64_t v = 0; v < h.N; ++v) {
        if (h.node_slot[v] < 0) continue;   // hole
        int X = (int)(v % h.lat[0]), Y = (int)((v / h.lat[0]) % h.lat[1]),
            Z = (int)(v / ((int64_t)h.lat[0] * h.lat[1]));
        int col = (X + Y + Z) & 3;
        Nc[col] += 1;
        if (!h.node_dir[v]) {
            Nfc[col] += 1;
            Nf += 1;
        }
    }
    const double Nall = (double)h.nnodes;
    const double vs = c->opts.precision == 1 ? 4.0 : 8.0;
    for (int col = 0; col < 4; ++col) {
        const double nbr = Nc[(col + 1) & 3] + Nc[(col + 3) & 3];
        // the D form's velocity sweep reads the neighbours of every other colour
        const double vnbr = dpath(c) ? Nall - Nc[col] : nbr;   // 15-tap rows read every other colour
        c->bytes_vel[col] = vs * 3.0 * (vnbr + 2.0 * Nfc[col]);
        c->bytes_pres[col] = vs * ((c->mi.general ? Nall - Nc[col] : nbr) + 3.0 * Nc[col]);
    }
    c->bytes_ru = vs * (Nall + 6.0 * Nf);
    c->bytes_bp = vs * (3.0 * Nall + 2.0 * Nall);
    for (int col = 0; col < 4; ++col) {
        const double nbr = Nc[(col + 1) & 3] + Nc[(col + 3) & 3];
        // + the colour's sweep: neighbours read, the colour written (its
        // right-hand side stays in registers)
        c->bytes_ru_fused[col] = c->bytes_ru + vs * 3.0 * (nbr + Nfc[col]);
        c->bytes_bp_fused[col] = c->bytes_bp + vs * (nbr + 2.0 * Nc[col]);
    }
    for (int p = 0; p < 2; ++p) {
        // parity p: the neighbours (colours p +- 1) read once, both colours written
        const double nbr = Nc[(p + 1) & 3] + Nc[(p + 3) & 3];
        c->bytes_ru_fused[4 + p] = c->bytes_ru + vs * 3.0 * (nbr + Nfc[p] + Nfc[p + 2]);
        c->bytes_bp_fused[4 + p] = c->bytes_bp + vs * (nbr + 2.0 * (Nc[p] + Nc[p + 2]));
    }
    c->bytes_res = vs * (4.0 * Nall + 2.0 * (3.0 * Nf + Nall));
    return HHG_OK;
}

// ------------------------------------------------------------------ timing
hipEvent_t next_event(hhg_ctx* c) {
    if (c->evused == c->evpool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->evpool.push_back(e);
    }
    return c->evpool[c->evused++];
}

struct Timed {
    hhg_ctx* c;
    int cls;
    hipStream_t s;
    TimerPair tp{nullptr, nullptr, 1};
    bool on;
    Timed(hhg_ctx* c_, int cls_, hipStream_t s_, bool finest, double bytes)
        : c(c_), cls(cls_), s(s_), on(c_->timing && finest) {
        if (!on) return;
        if (c->tgroup_cls == cls) {   // inside a group bracket: count only
            on = false;
            ++c->tgroup_n;
            c->tbytes[cls] += bytes;
            return;
        }
        tp.a = next_event(c);
        tp.b = next_event(c);
        if (!tp.a || !tp.b) {
            on = false;
            return;
        }
        (void)hipEventRecord(tp.a, s);
        c->tbytes[cls] += bytes;
    }
    ~Timed() {
        if (!on) return;
        (void)hipEventRecord(tp.b, s);
        c->tpairs[cls].push_back(tp);
    }
};

// One pair of events around consecutive launches of one class on the finest
// level (the velocity colour sweeps of a smoothing step), so that the event
// packets between the launches do not count into their duration.
struct TimedGroup {
    hhg_ctx* c;
    int cls;
    hipStream_t s;
    TimerPair tp{nullptr, nullptr, 0};
    bool on;
    TimedGroup(hhg_ctx* c_, int cls_, hipStream_t s_, bool finest)
        : c(c_), cls(cls_), s(s_), on(c_->timing && finest && c_->tgroup_cls < 0) {
        if (!on) return;
        tp.a = next_event(c);
        tp.b = next_event(c);
        if (!tp.a || !tp.b) {
            on = false;
            return;
        }
        (void)hipEventRecord(tp.a, s);
        c->tgroup_cls = cls;
        c->tgroup_n = 0;
    }
    ~TimedGroup() {
        if (!on) return;
        (void)hipEventRecord(tp.b, s);
        tp.n = c->tgroup_n;
        c->tgroup_cls = -1;
        if (tp.n > 0) c->tpairs[cls].push_back(tp);
    }
};

// Event pair around the launches of one phase of a cycle on one level
// (hhg_solve's phase and level timers; off unless requested).
enum { PH_SMOOTH = 0, PH_TRANSFER = 1, PH_COARSE = 2, PH_RESIDUAL = 3 };
struct PhaseTimed {
    hhg_ctx* c;
    int ph;
    hipStream_t s;
    TimerPair tp{nullptr, nullptr, 1};
    bool on;
    PhaseTimed(hhg_ctx* c_, int ph_, int lev, hipStream_t s_)
        : c(c_), ph(ph_), s(s_), on(c_->phase_timing && c_->phase_active) {
        if (!on) return;
        tp.lev = lev;
        tp.a = next_event(c);
        tp.b = next_event(c);
        if (!tp.a || !tp.b) {
            on = false;
            return;
        }
        (void)hipEventRecord(tp.a, s);
    }
    ~PhaseTimed() {
        if (!on) return;
        (void)hipEventRecord(tp.b, s);
        c->ppairs[ph].push_back(tp);
    }
};

inline int grid_for(size_t n) { return (int)std::min<size_t>((n + TPB - 1) / TPB, 8192); }

// ------------------------------------------------------------------ operator counts
inline void ops(hhg_ctx* c, int l, double a, double b, double cc, double m) {
    std::array<double, 4>& o = c->opc[l];
    o[0] += a;
    o[1] += b;
    o[2] += cc;
    o[3] += m;
}

void reset_ops(hhg_ctx* c) {
    c->opc.assign(c->L + 1, std::array<double, 4>{0.0, 0.0, 0.0, 0.0});
}

// weighted counts of eq. op_count: sum_l 8^(l-L) n_op,l
void put_ops(hhg_ctx* c, hhg_solve_info* I) {
    for (int q = 0; q < 4; ++q) {
        double t = 0.0;
        for (int l = 0; l <= c->L; ++l) t += std::ldexp(c->opc[l][q], 3 * (l - c->L));
        I->n_op[q] = t;
    }
}

// ------------------------------------------------------------------ captured cycles
void drop_graphs(hhg_ctx* c) {
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

// Executable graph of body(stream) for the pair (x, b): captured on the
// library's own stream the first time (the launches are recorded, not run)
// and kept; at most four pairs are kept.  Returns nullptr if capturing fails
// (the caller then launches on its stream).
template <typename F>
hhg_ctx::CycleGraph* cycle_graph(hhg_ctx* c, const void* x, const void* b, F&& body) {
    for (auto& g : c->graphs)
        if (g.x == x && g.b == b) return &g;
    if (!c->cap && hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
        c->cap = nullptr;
        return nullptr;
    }
    const std::vector<std::array<double, 4>> before = c->opc;
    if (hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    body(c->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap, &graph);
    std::vector<std::array<double, 4>> delta = c->opc;
    c->opc = before;
    if (e != hipSuccess || !graph) {
        (void)hipGetLastError();
        return nullptr;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    for (size_t l = 0; l < delta.size(); ++l)
        for (int q = 0; q < 4; ++q) delta[l][q] -= before[l][q];
    if (c->graphs.size() >= 4) {
        (void)hipGraphExecDestroy(c->graphs.front().exec);
        c->graphs.erase(c->graphs.begin());
    }
    c->graphs.push_back(hhg_ctx::CycleGraph{x, b, exec, delta});
    return &c->graphs.back();
}

// replay of a captured cycle on stream s, with its operator counts
hipError_t replay(hhg_ctx* c, hhg_ctx::CycleGraph* g, hipStream_t s) {
    for (size_t l = 0; l < g->ops.size(); ++l)
        for (int q = 0; q < 4; ++q) c->opc[l][q] += g->ops[l][q];
    return hipGraphLaunch(g->exec, s);
}

// ------------------------------------------------------------------ operators
template <typename T>
LevelDev<T>& view(hhg_ctx* c, int l);
template <>
LevelDev<double>& view<double>(hhg_ctx* c, int l) {
    return c->D64[l];
}
template <>
LevelDev<float>& view<float>(hhg_ctx* c, int l) {
    return c->D32[l];
}

template <typename T>
void vecs(hhg_ctx* c, int l, T** x, T** b, T** r, T** t);
template <>
void vecs<double>(hhg_ctx* c, int l, double** x, double** b, double** r, double** t) {
    DevLevelArrays& a = c->A[l];
    *x = a.x64;
    *b = a.b64;
    *r = a.r64;
    *t = a.t64;
}
template <>
void vecs<float>(hhg_ctx* c, int l, float** x, float** b, float** r, float** t) {
    DevLevelArrays& a = c->A[l];
    *x = a.x32;
    *b = a.b32;
    *r = a.r32;
    *t = a.t32;
}

// volume blocks of a full pass in the given mode
inline int full_vblocks(int mode, int n_vtiles) {
    return quad_lanes(mode) ? n_vtiles : full_blocks(n_vtiles);
}

// levels with at least this many intervals per macro edge launch the volume
// and the interface blocks of K x and the residual separately: the volume
// kernel is then not held to the interface lanes' register budget
constexpr int SPLIT_MIN_N = 64;

// K x or the residual (MODE_APPLY / MODE_RES); MIRROR: interface taps from
// the level's mirror of x
template <typename T, int MODE, bool MIRROR, bool DOP>
void launch_kx_op(LevelDev<T>& v, int ib, const T* x, const T* b, T* y, double* partials,
                  hipStream_t s) {
    if (v.n >= SPLIT_MIN_N) {
        if constexpr (DOP) {
            // volume launch: one vertex per lane (four blocks per tile)
            hipLaunchKernelGGL((k_full<T, MODE, false, MIRROR, false, 1, DOP>),
                               dim3(full_blocks(v.n_vtiles)), dim3(TPB), 0, s, v, x, b, y, partials,
                               0, (T*)nullptr, -1, T(0));
        } else {
            // volume launch: a quad per lane, quad windows (one block per tile)
            hipLaunchKernelGGL((k_full<T, MODE, false, MIRROR, true, 1, false>), dim3(v.n_vtiles),
                               dim3(TPB), 0, s, v, x, b, y, partials, 0, (T*)nullptr, -1, T(0));
        }
        if (ib > 0)
            hipLaunchKernelGGL((k_full<T, MODE, false, MIRROR, false, 2, DOP>), dim3(ib), dim3(TPB), 0,
                               s, v, x, b, y, partials, ib, (T*)nullptr, -1, T(0));
        return;
    }
    hipLaunchKernelGGL((k_full<T, MODE, false, MIRROR, false, 0, DOP>), dim3(ib + v.n_vtiles),
                       dim3(TPB), 0, s, v, x, b, y, partials, ib, (T*)nullptr, -1, T(0));
}

// the velocity form of the context: Laplace (a_1) or D (a_2); the residual's
// per-block partial sums go to `partials` (the workspace's by default)
template <typename T, int MODE, bool MIRROR>
void launch_kx(hhg_ctx* c, LevelDev<T>& v, int ib, const T* x, const T* b, T* y, hipStream_t s,
               double* partials = nullptr) {
    if (!partials) partials = c->partials;
    if (dpath(c))
        launch_kx_op<T, MODE, MIRROR, true>(v, ib, x, b, y, partials, s);
    else
        launch_kx_op<T, MODE, MIRROR, false>(v, ib, x, b, y, partials, s);
}

// number of per-block partial sums of a residual on level l (the entries
// k_reduce_sum adds up): the volume ones, then one per interface block
template <typename T>
inline int residual_partials(const LevelDev<T>& v) {
    return (v.n >= SPLIT_MIN_N ? 4 : 1) * v.nv_nat + (v.nif + TPB - 1) / TPB;
}

// levels with at least this many intervals per macro edge evaluate RU and BP
// by quad windows (fewer load instructions); smaller ones one vertex per lane
// (more lanes for a latency-bound launch)
constexpr int WIN_MIN_N = 32;

template <typename T, int MODE>
void full_pass(hhg_ctx* c, int l, const T* x, const T* b, T* y, hipStream_t s) {
    LevelDev<T>& v = view<T>(c, l);
    const int ib = iface_blocks(v.nif);
    const int grid = ib + full_vblocks(MODE, v.n_vtiles);
    const bool finest = l == c->L;
    double bytes = MODE == MODE_RU ? c->bytes_ru : MODE == MODE_BP ? c->bytes_bp : c->bytes_res;
    Timed tm(c, HHG_K_APPLY, s, finest && (MODE == MODE_RU || MODE == MODE_BP || MODE == MODE_RES),
             bytes);
    if (MODE == MODE_APPLY || MODE == MODE_RES) ops(c, l, 1, 2, 1, 0);
    if (MODE == MODE_RU || MODE == MODE_BP || MODE == MODE_BTN) ops(c, l, 0, 1, 0, 0);
    if (MODE == MODE_ARES) ops(c, l, 1, 0, 0, 0);
    if (MODE == MODE_SCHUR) ops(c, l, 0, 1, 1, 0);
    if constexpr (MODE == MODE_RU || MODE == MODE_BP) {
        if (v.n >= WIN_MIN_N) {
            // unfused f - B^T p or B u - g on large levels: quad windows
            hipLaunchKernelGGL((k_full<T, MODE, false, false, true>), dim3(ib + v.n_vtiles),
                               dim3(TPB), 0, s, v, x, b, y, c->partials, ib, (T*)nullptr, -1, T(0));
            return;
        }
    }
    if (MODE == MODE_APPLY || MODE == MODE_RES)
        launch_kx<T, (MODE == MODE_RES ? MODE_RES : MODE_APPLY), false>(c, v, ib, x, b, y, s);
    else if (MODE == MODE_ARES && dpath(c))
        hipLaunchKernelGGL((k_full<T, MODE_ARES, false, false, false, 0, true>), dim3(grid),
                           dim3(TPB), 0, s, v, x, b, y, c->partials, ib, (T*)nullptr, -1, T(0));
    else
        hipLaunchKernelGGL((k_full<T, MODE, false, false>), dim3(grid), dim3(TPB), 0, s, v, x, b, y,
                           c->partials, ib, (T*)nullptr, -1, T(0));
}

// residual of the level's smoothed iterate: interface taps from its mirror
template <typename T>
void residual_mirror(hhg_ctx* c, int l, const T* x, const T* b, T* r, hipStream_t s) {
    LevelDev<T>& v = view<T>(c, l);
    const int ib = iface_blocks(v.nif);
    const int grid = ib + full_vblocks(MODE_RES, v.n_vtiles);
    Timed tm(c, HHG_K_APPLY, s, l == c->L, c->bytes_res);
    (void)grid;
    ops(c, l, 1, 2, 1, 0);
    launch_kx<T, MODE_RES, true>(c, v, ib, x, b, r, s);
}

// ||b - K x||_2 into *out from the mirror of x (which must be current), with
// t = b_k - (B^T p)_k (k = 0..2) written in place of the residual: the right-
// hand side of the velocity sweeps of a Uzawa step that starts from this x
// (Laplace form on Kuhn macros)
template <typename T>
void residual_norm_t(hhg_ctx* c, int l, const T* x, const T* b, T* t, double* out, hipStream_t s) {
    LevelDev<T>& v = view<T>(c, l);
    const int ib = iface_blocks(v.nif);
    {
        Timed tm(c, HHG_K_APPLY, s, l == c->L, c->bytes_res);
        ops(c, l, 1, 2, 1, 0);
        if (v.n >= SPLIT_MIN_N) {
            hipLaunchKernelGGL((k_full<T, MODE_RES, false, true, true, 1, false, false, true>),
                               dim3(v.n_vtiles), dim3(TPB), 0, s, v, x, b, t, c->partials, 0,
                               (T*)nullptr, -1, T(0));
            if (ib > 0)
                hipLaunchKernelGGL((k_full<T, MODE_RES, false, true, false, 2, false, false, true>),
                                   dim3(ib), dim3(TPB), 0, s, v, x, b, t, c->partials, ib,
                                   (T*)nullptr, -1, T(0));
        } else {
            hipLaunchKernelGGL((k_full<T, MODE_RES, false, true, false, 0, false, false, true>),
                               dim3(ib + v.n_vtiles), dim3(TPB), 0, s, v, x, b, t, c->partials, ib,
                               (T*)nullptr, -1, T(0));
        }
    }
    hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(RTPB), 0, s, c->partials,
                       residual_partials(v), out, 1);
}

// mirror of x taken afresh (entry points that smooth a caller's vector)
template <typename T>
void mirror_refresh(hhg_ctx* c, int l, const T* x, hipStream_t s) {
    LevelDev<T>& v = view<T>(c, l);
    hipLaunchKernelGGL(k_mirror_gather<T>, dim3((v.ncomp + TPB - 1) / TPB), dim3(TPB), 0, s, v, x);
}

// x <- 0 together with its mirror
template <typename T>
void fill_iterate(hhg_ctx* c, int l, T* x, hipStream_t s) {
    LevelDev<T>& v = view<T>(c, l);
    const size_t n4 = 4 * (size_t)v.len, m4 = 4 * (size_t)v.cstride;
    hipLaunchKernelGGL(k_fill2<T>, dim3(grid_for(n4 + m4)), dim3(TPB), 0, s, x, n4, v.cx, m4, T(0));
}

// RU with the velocity sweep of colour col, or BP with the pressure sweep of
// colour col, in one launch (x is updated in place, t receives the pass)

template <typename T, int MODE>
void full_pass_fused(hhg_ctx* c, int l, T* x, const T* b, T* t, int colx, hipStream_t s) {
    LevelDev<T>& v = view<T>(c, l);
    // colx = col + 8: the updated vertices' rows of the pass are not stored
    const int col = colx >= 8 ? colx - 8 : colx;
    // f - B^T p takes a lane per interface vertex and velocity component, B u
    // - g four lanes per interface vertex on levels without quad windows
    const int ib = iface_blocks(MODE == MODE_RU ? 3 * v.nif : v.n < WIN_MIN_N ? 4 * v.nif : v.nif);
    const bool finest = l == c->L;
    const double bytes = MODE == MODE_RU ? c->bytes_ru_fused[col] : c->bytes_bp_fused[col];
    Timed tm(c, MODE == MODE_RU ? HHG_K_RU : HHG_K_APPLY, s, finest, bytes);
    const double share = col < 4 ? 0.25 : 0.5;   // one colour or a red-black parity
    if (MODE == MODE_RU) ops(c, l, share, 1, 0, 0);
    else ops(c, l, 0, 1, share, 0);
    if (c->mi.general) {
        // 15-tap fused updates
        if (v.n >= WIN_MIN_N)
            hipLaunchKernelGGL((k_full<T, MODE, true, true, true, 0, false, true>),
                               dim3(ib + v.n_vtiles), dim3(TPB), 0, s, v, (const T*)x, b, t,
                               c->partials, ib, x, colx, (T)c->opts.omega);
        else
            hipLaunchKernelGGL((k_full<T, MODE, true, true, false, 0, false, true>),
                               dim3(ib + full_blocks(v.n_vtiles)), dim3(TPB), 0, s, v, (const T*)x, b,
                               t, c->partials, ib, x, colx, (T)c->opts.omega);
    } else if (v.n >= WIN_MIN_N) {
        hipLaunchKernelGGL((k_full<T, MODE, true, true, true>), dim3(ib + v.n_vtiles), dim3(TPB), 0, s,
                           v, (const T*)x, b, t, c->partials, ib, x, colx, (T)c->opts.omega);
    } else {
        hipLaunchKernelGGL((k_full<T, MODE, true, true>), dim3(ib + full_blocks(v.n_vtiles)),
                           dim3(TPB), 0, s, v, (const T*)x, b, t, c->partials, ib, x, colx,
                           (T)c->opts.omega);
    }
}

template <typename T>
void colour_pass(hhg_ctx* c, int l, int col, bool vel, T* x, const T* rhs, hipStream_t s) {
    LevelDev<T>& v = view<T>(c, l);
    const int cnt = vel ? v.vel_end[col] - v.col_start[col] : v.col_start[col + 1] - v.col_start[col];
    // velocity sweeps: a lane per interface vertex and component (Laplace
    // form; then a lane per free-slip vertex), four lanes per interface vertex
    // (D form)
    const int nslip = v.col_start[col + 1] - v.slip_beg[col];
    const int ib = iface_blocks(!vel ? cnt : c->opts.op == 1 ? 4 * cnt : 3 * cnt + nslip);
    const int grid = ib + v.n_vtiles;
    const bool finest = l == c->L;
    ops(c, l, vel ? 0.25 : 0.0, 0, vel ? 0.0 : 0.25, 0);
    if (vel) {
        Timed tm(c, HHG_K_VEL, s, finest, c->bytes_vel[col]);
        if (c->opts.op == 1)
            hipLaunchKernelGGL((k_colour<T, true, true>), dim3(grid), dim3(TPB), 0, s, v, col, x, rhs,
                               T(0), ib);
        else if (c->mi.general && c->mi.slip)
            hipLaunchKernelGGL((k_colour<T, true, false, true, true>), dim3(grid), dim3(TPB), 0, s, v,
                               col, x, rhs, T(0), ib);
        else if (c->mi.general)
            hipLaunchKernelGGL((k_colour<T, true, false, true>), dim3(grid), dim3(TPB), 0, s, v, col,
                               x, rhs, T(0), ib);
        else if (c->mi.slip)
            hipLaunchKernelGGL((k_colour<T, true, false, false, true>), dim3(grid), dim3(TPB), 0, s, v,
                               col, x, rhs, T(0), ib);
        else
            hipLaunchKernelGGL((k_colour<T, true>), dim3(grid), dim3(TPB), 0, s, v, col, x, rhs, T(0),
                               ib);
    } else {
        Timed tm(c, HHG_K_PRES, s, finest, c->bytes_pres[col]);
        if (c->mi.general)
            hipLaunchKernelGGL((k_colour<T, false, false, true>), dim3(grid), dim3(TPB), 0, s, v, col,
                               x, rhs, (T)c->opts.omega, ib);
        else
            hipLaunchKernelGGL((k_colour<T, false>), dim3(grid), dim3(TPB), 0, s, v, col, x, rhs,
                               (T)c->opts.omega, ib);
    }
}

template <typename T>
T* snap_of(DevLevelArrays& a);
template <>
double* snap_of<double>(DevLevelArrays& a) { return a.snap64; }
template <>
float* snap_of<float>(DevLevelArrays& a) { return a.snap32; }

// One pass of the hybrid ordering (Section 3.4) on the velocity (vel) or the
// pressure: for each primitive class (macro vertices, edges, faces) the
// class's starting values are saved, then its colours run in the given
// order; the volume class follows as volume-only colour launches (volume
// primitives, the macro interiors, never couple to each other).
template <typename T>
void hybrid_pass(hhg_ctx* c, int l, bool vel, bool backward, T* x, const T* rhs, hipStream_t s) {
    LevelDev<T>& v = view<T>(c, l);
    DevLevelArrays& a = c->A[l];
    const HostLevel& h = c->H[l];
    T* snap = snap_of<T>(a);
    const int kind = vel ? 0 : 1;
    const T omega = vel ? T(0) : (T)c->opts.omega;
    for (int k = 0; k < 3; ++k) {
        // starting values of every vertex of the class (the pressure groups
        // list all of them: a masked tap may reach a velocity Dirichlet vertex)
        const int g0 = h.hyb_off[12 + 4 * k], g1 = h.hyb_off[12 + 4 * k + 4];
        if (g1 > g0)
            hipLaunchKernelGGL(k_hyb_snap<T>, dim3((g1 - g0 + TPB - 1) / TPB), dim3(TPB), 0, s, v,
                               a.hyb_list + g0, g1 - g0, vel ? 0 : 3, vel ? 3 : 4, snap);
        for (int q = 0; q < 4; ++q) {
            const int col = backward ? 3 - q : q;
            const int o0 = h.hyb_off[12 * kind + 4 * k + col], o1 = h.hyb_off[12 * kind + 4 * k + col + 1];
            const int cnt = o1 - o0;
            if (cnt == 0) continue;
            const int lanes = vel ? 3 * cnt : cnt;
            const dim3 grid((lanes + TPB - 1) / TPB);
            if (vel && c->mi.general)
                hipLaunchKernelGGL((k_hyb_iface<T, true, true>), grid, dim3(TPB), 0, s, v,
                                   a.hyb_list + o0, cnt, x, rhs, omega, (const T*)snap, a.hyb_mask);
            else if (vel)
                hipLaunchKernelGGL((k_hyb_iface<T, true, false>), grid, dim3(TPB), 0, s, v,
                                   a.hyb_list + o0, cnt, x, rhs, omega, (const T*)snap, a.hyb_mask);
            else if (c->mi.general)
                hipLaunchKernelGGL((k_hyb_iface<T, false, true>), grid, dim3(TPB), 0, s, v,
                                   a.hyb_list + o0, cnt, x, rhs, omega, (const T*)snap, a.hyb_mask);
            else
                hipLaunchKernelGGL((k_hyb_iface<T, false, false>), grid, dim3(TPB), 0, s, v,
                                   a.hyb_list + o0, cnt, x, rhs, omega, (const T*)snap, a.hyb_mask);
        }
    }
    // volume primitives: every block a volume tile (no interface blocks)
    const dim3 grid(v.n_vtiles);
    for (int q = 0; q < 4; ++q) {
        const int col = backward ? 3 - q : q;
        Timed tm(c, vel ? HHG_K_VEL : HHG_K_PRES, s, l == c->L,
                 vel ? c->bytes_vel[col] : c->bytes_pres[col]);
        if (vel && c->mi.general)
            hipLaunchKernelGGL((k_colour<T, true, false, true>), grid, dim3(TPB), 0, s, v, col, x, rhs,
                               omega, 0);
        else if (vel)
            hipLaunchKernelGGL((k_colour<T, true>), grid, dim3(TPB), 0, s, v, col, x, rhs, omega, 0);
        else if (c->mi.general)
            hipLaunchKernelGGL((k_colour<T, false, false, true>), grid, dim3(TPB), 0, s, v, col, x,
                               rhs, omega, 0);
        else
            hipLaunchKernelGGL((k_colour<T, false>), grid, dim3(TPB), 0, s, v, col, x, rhs, omega, 0);
    }
}

// one inexact Uzawa step in the hybrid ordering: f - B^T p, the forward and
// the backward hybrid velocity passes (SHGS), B u - g, the forward hybrid
// pressure pass (and the backward one with p_sweep = 1)
template <typename T>
void uzawa_step_hybrid(hhg_ctx* c, int l, T* x, const T* b, T* t, hipStream_t s) {
    // a full sweep of either operator counts as one evaluation of it
    full_pass<T, MODE_RU>(c, l, x, b, t, s);
    ops(c, l, 2.0, 0, 0, 0);
    hybrid_pass<T>(c, l, true, false, x, t, s);
    hybrid_pass<T>(c, l, true, true, x, t, s);
    full_pass<T, MODE_BP>(c, l, x, b, t, s);
    ops(c, l, 0, 0, c->opts.p_sweep == 1 ? 2.0 : 1.0, 0);
    hybrid_pass<T>(c, l, false, false, x, t, s);
    if (c->opts.p_sweep == 1) hybrid_pass<T>(c, l, false, true, x, t, s);
}

// One launch of the red-black order (ordering 2): parity p (0 red: colours 0
// and 2, 1 black: colours 1 and 3) of the velocity or the pressure.
template <typename T>
void colour_pass_rb(hhg_ctx* c, int l, int p, bool vel, T* x, const T* rhs, hipStream_t s) {
    LevelDev<T>& v = view<T>(c, l);
    int cnt = 0;
    for (int col : {p, p + 2})
        cnt += vel ? v.vel_end[col] - v.col_start[col] : v.col_start[col + 1] - v.col_start[col];
    const int ib = iface_blocks(vel ? 3 * cnt : cnt);
    const int grid = ib + rb_blocks(v.n_vtiles);
    const bool finest = l == c->L;
    ops(c, l, vel ? 0.5 : 0.0, 0, vel ? 0.0 : 0.5, 0);
    if (vel) {
        Timed tm(c, HHG_K_VEL, s, finest, c->bytes_vel[p] + c->bytes_vel[p + 2]);
        hipLaunchKernelGGL((k_colour_rb<T, true>), dim3(grid), dim3(TPB), 0, s, v, p, x, rhs, T(0),
                           ib);
    } else {
        Timed tm(c, HHG_K_PRES, s, finest, c->bytes_pres[p] + c->bytes_pres[p + 2]);
        hipLaunchKernelGGL((k_colour_rb<T, false>), dim3(grid), dim3(TPB), 0, s, v, p, x, rhs,
                           (T)c->opts.omega, ib);
    }
}

// one inexact Uzawa step in the red-black order: the symmetric velocity sweep
// red, black, red (a second black sweep right after the first would
// recompute identical values), its first red half inside the pass that forms
// f - B^T p; the pressure red (inside the pass that forms B u - g), black,
// and with p_sweep = 1 black, red again
// (vr: f - B^T p of this x is given, and the first red half is a sweep of
// its own)
template <typename T>
void uzawa_step_rb(hhg_ctx* c, int l, T* x, const T* b, T* t, hipStream_t s, const T* vr) {
    if (!vr) full_pass_fused<T, MODE_RU>(c, l, x, b, t, 4, s);
    {
        TimedGroup tg(c, HHG_K_VEL, s, l == c->L);
        const T* rhs = vr ? vr : t;
        if (vr) colour_pass_rb<T>(c, l, 0, true, x, rhs, s);
        colour_pass_rb<T>(c, l, 1, true, x, rhs, s);
        colour_pass_rb<T>(c, l, 0, true, x, rhs, s);
    }
    full_pass_fused<T, MODE_BP>(c, l, x, b, t, c->opts.p_sweep == 1 ? 4 : 4 + 8, s);
    colour_pass_rb<T>(c, l, 1, false, x, t, s);
    if (c->opts.p_sweep == 1) {
        colour_pass_rb<T>(c, l, 1, false, x, t, s);
        colour_pass_rb<T>(c, l, 0, false, x, t, s);
    }
}

// one inexact Uzawa step (eq. Uzawa_smooth) in place.  vr (colour and
// red-black orders): the velocity fields of vr hold f - B^T p of this x (b
// itself when x = 0, or what the residual before the step wrote), so the step
// skips the pass that forms it and starts with the velocity sweeps
template <typename T>
void uzawa_step(hhg_ctx* c, int l, T* x, const T* b, T* t, hipStream_t s,
                const T* vr = nullptr) {
    if (c->opts.ordering == 1) {
        uzawa_step_hybrid<T>(c, l, x, b, t, s);
        return;
    }
    if (c->opts.ordering == 2) {
        uzawa_step_rb<T>(c, l, x, b, t, s, vr);
        return;
    }
    // symmetric Gauss-Seidel on A: colours 0 1 2 3 2 1 0 (a second sweep of
    // colour 3 right after the first would recompute identical values); the
    // first sweep runs inside the pass that forms f - B^T p, except for the D
    // form, whose point-block sweeps run on their own
    static const int vorder[6] = {1, 2, 3, 2, 1, 0};
    if (vr) {
        // f - B^T p given
    } else if (c->opts.op == 1) {
        full_pass<T, MODE_RU>(c, l, x, b, t, s);
    } else {
        full_pass_fused<T, MODE_RU>(c, l, x, b, t, 0, s);
        if (c->mi.slip) {
            // the colour-0 free-slip vertices, which the fused pass leaves out
            LevelDev<T>& v = view<T>(c, l);
            const int ns = v.col_start[1] - v.slip_beg[0];
            if (ns > 0) {
                if (c->mi.general)
                    hipLaunchKernelGGL((k_slip_colour<T, true>), dim3((ns + TPB - 1) / TPB),
                                       dim3(TPB), 0, s, v, 0, x, (const T*)t);
                else
                    hipLaunchKernelGGL((k_slip_colour<T, false>), dim3((ns + TPB - 1) / TPB),
                                       dim3(TPB), 0, s, v, 0, x, (const T*)t);
            }
        }
    }
    {
        TimedGroup tg(c, HHG_K_VEL, s, l == c->L);
        const T* rhs = vr ? vr : t;
        if (c->opts.op == 1 || vr) colour_pass<T>(c, l, 0, true, x, rhs, s);
        for (int q = 0; q < 6; ++q) colour_pass<T>(c, l, vorder[q], true, x, rhs, s);
    }
    // forward pressure sweep; colour 0 inside the pass that forms B u - g
    full_pass_fused<T, MODE_BP>(c, l, x, b, t, c->opts.p_sweep == 1 ? 0 : 8, s);
    for (int col = 1; col < 4; ++col) colour_pass<T>(c, l, col, false, x, t, s);
    if (c->opts.p_sweep == 1)
        for (int col = 3; col >= 0; --col) colour_pass<T>(c, l, col, false, x, t, s);
}

template <typename T>
void fill(T* x, size_t n, T val, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(TPB), 0, s, x, n, val);
}

// r = b - K x and ||r||_2 into *out; with mirror the interface taps come
// from the level's mirror of x (which must then be current)
template <typename T>
void residual_norm(hhg_ctx* c, int l, const T* x, const T* b, T* r, double* out, hipStream_t s,
                   bool mirror = false) {
    LevelDev<T>& v = view<T>(c, l);
    const int ib = iface_blocks(v.nif);
    if (mirror) {
        residual_mirror<T>(c, l, x, b, r, s);
    } else {
        const int grid = ib + full_vblocks(MODE_RES, v.n_vtiles);
        Timed tm(c, HHG_K_APPLY, s, l == c->L, c->bytes_res);
        (void)grid;
        ops(c, l, 1, 2, 1, 0);
        launch_kx<T, MODE_RES, false>(c, v, ib, x, b, r, s);
    }
    hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(RTPB), 0, s, c->partials,
                       residual_partials(v), out, 1);
}

template <typename T, int NF = 4>
void restrict_to(hhg_ctx* c, int l, const T* rf, T* bc, hipStream_t s) {
    LevelDev<T>& C = view<T>(c, l - 1);
    LevelDev<T>& F = view<T>(c, l);
    const int ib = iface_blocks(NF * C.nif);   // a lane per interface vertex and field
    const int grid = ib + full_blocks(C.n_vtiles);
    hipLaunchKernelGGL((k_restrict<T, NF>), dim3(grid), dim3(TPB), 0, s, C, F, rf, bc, ib);
}

template <typename T, int NF = 4>
void prolong_add(hhg_ctx* c, int l, const T* ec, T* xf, hipStream_t s) {
    LevelDev<T>& C = view<T>(c, l - 1);
    LevelDev<T>& F = view<T>(c, l);
    if (c->mi.slip)
        hipLaunchKernelGGL((k_prolong<T, false, NF>), dim3(full_blocks(F.n_ctiles)), dim3(TPB), 0, s,
                           F, C, ec, xf);
    else
        hipLaunchKernelGGL((k_prolong<T, false, NF, false>), dim3(full_blocks(F.n_ctiles)), dim3(TPB),
                           0, s, F, C, ec, xf);
}

template <typename T>
void coarse_solve(hhg_ctx* c, const T* b, T* x, hipStream_t s) {
    const size_t len = (size_t)c->H[0].len;
    if (c->opts.coarse_solver == 0) {
        const int rows = (c->cd.nd + TPB / 64 - 1) / (TPB / 64);
        const int grid = std::max(rows, (c->cd.N + TPB - 1) / TPB);
        hipLaunchKernelGGL(k_coarse_direct<T>, dim3(grid), dim3(TPB), c->cd.nb * sizeof(double), s,
                           c->cd, b, len, x, len, c->scal + 8);
        return;
    }
    hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(CTPB), c->coarse_smem, s, c->cd, b, len, x, len,
                       c->scal + 8);
}

template <typename T>
void project(hhg_ctx* c, int l, T* x, hipStream_t s) {
    if (!c->mi.project) return;
    LevelDev<T>& v = view<T>(c, l);
    const int ib = iface_blocks(v.nif);
    const int grid = ib + v.n_vtiles;
    const size_t len = (size_t)v.len;
    hipLaunchKernelGGL(k_mass_dot<T>, dim3(grid), dim3(TPB), 0, s, v, x + 3 * len, c->partials, ib);
    hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(RTPB), 0, s, c->partials,
                       v.nv_nat + (v.nif + TPB - 1) / TPB, c->scal + 4, 0);
    const size_t cs = (size_t)v.cstride;
    hipLaunchKernelGGL(k_sub_mean2<T>, dim3(grid_for(len + cs)), dim3(TPB), 0, s, x + 3 * len, len,
                       v.cx + 3 * cs, cs, c->scal + 4, c->inv_mass[l]);
}

// V-cycle from level l whose top level is `top` (the variable cycle adds
// 2 (top - l) smoothing steps on level l); vr0: f - B^T p of x on entry, for
// the first Uzawa step (see uzawa_step), or null
template <typename T>
void vcycle(hhg_ctx* c, int l, int top, T* x, const T* b, hipStream_t s,
            const T* vr0 = nullptr) {
    T *xl, *bl, *rl, *tl;
    vecs<T>(c, l, &xl, &bl, &rl, &tl);
    if (l == 0) {
        // x += K_0^-1 (b - K_0 x)
        PhaseTimed pt(c, PH_COARSE, 0, s);
        full_pass<T, MODE_RES>(c, 0, x, b, rl, s);
        coarse_solve<T>(c, rl, tl, s);
        const size_t n4 = 4 * (size_t)c->H[0].len;
        hipLaunchKernelGGL(k_add<T>, dim3(grid_for(n4)), dim3(TPB), 0, s, x, (const T*)tl, n4);
        return;
    }
    // the mirror of x is current on entry (refreshed, filled, or written by
    // the previous cycle's sweeps and projection) and the sweeps keep it so
    const int extra = c->opts.cycle == 1 ? 2 * (top - l) : 0;
    {
        PhaseTimed pt(c, PH_SMOOTH, l, s);
        for (int q = 0; q < c->opts.nu1 + extra; ++q)
            uzawa_step<T>(c, l, x, b, tl, s, q == 0 ? vr0 : nullptr);
    }
    {
        PhaseTimed pt(c, PH_RESIDUAL, l, s);
        residual_mirror<T>(c, l, x, b, rl, s);
    }
    T *xc, *bc, *rc, *tc;
    vecs<T>(c, l - 1, &xc, &bc, &rc, &tc);
    {
        PhaseTimed pt(c, PH_TRANSFER, l, s);
        restrict_to<T>(c, l, rl, bc, s);
    }
    if (l - 1 == 0) {
        PhaseTimed pt(c, PH_COARSE, 0, s);
        coarse_solve<T>(c, bc, xc, s);
    } else {
        {
            PhaseTimed pt(c, PH_TRANSFER, l - 1, s);
            fill_iterate<T>(c, l - 1, xc, s);
        }
        // from x = 0: f - B^T p = b
        vcycle<T>(c, l - 1, top, xc, bc, s, bc);
    }
    {
        PhaseTimed pt(c, PH_TRANSFER, l, s);
        prolong_add<T>(c, l, xc, x, s);
    }
    PhaseTimed pt(c, PH_SMOOTH, l, s);
    for (int q = 0; q < c->opts.nu2 + extra; ++q) uzawa_step<T>(c, l, x, b, tl, s);
}

// ------------------------------------------------------- velocity multigrid
// Multigrid for the velocity block A alone (Sections 3.1, 3.2 and Table
// "settings", SCG and PMINRES columns): V(nu1, nu2) with forward colour
// Gauss-Seidel (colours 0..3) before and backward (3..0) after the coarse
// correction, the A-residual restricted by P^T (three fields), A_0 inverted
// exactly on level 0.  Works on fields 0..2 of x and b; field 3 of x is left
// alone.  The mirror of x is current on entry and kept so.
template <typename T>
void coarse_avel(hhg_ctx* c, const T* b, T* x, hipStream_t s) {
    const size_t len = (size_t)c->H[0].len;
    const int rows = (3 * c->cd.nfv + TPB / 64 - 1) / (TPB / 64);
    const int grid = std::max(std::max(rows, (c->cd.N + TPB - 1) / TPB), 1);
    hipLaunchKernelGGL(k_coarse_avel<T>, dim3(grid), dim3(TPB), 3 * c->cd.nfv * sizeof(double), s,
                       c->cd, b, len, x, len);
}

// velocity fields of x <- 0, with their mirror entries
template <typename T>
void fill_velocity(hhg_ctx* c, int l, T* x, hipStream_t s) {
    LevelDev<T>& v = view<T>(c, l);
    const size_t n3 = 3 * (size_t)v.len, m3 = 3 * (size_t)v.cstride;
    hipLaunchKernelGGL(k_fill2<T>, dim3(grid_for(n3 + m3)), dim3(TPB), 0, s, x, n3, v.cx, m3, T(0));
}

template <typename T>
void vel_cycle(hhg_ctx* c, int l, int nu1, int nu2, T* x, const T* b, hipStream_t s) {
    T *xl, *bl, *rl, *tl;
    vecs<T>(c, l, &xl, &bl, &rl, &tl);
    if (l == 0) {
        full_pass<T, MODE_ARES>(c, 0, x, b, rl, s);
        coarse_avel<T>(c, rl, tl, s);
        const size_t n3 = 3 * (size_t)c->H[0].len;
        hipLaunchKernelGGL(k_add<T>, dim3(grid_for(n3)), dim3(TPB), 0, s, x, (const T*)tl, n3);
        return;
    }
    for (int q = 0; q < nu1; ++q)
        for (int col = 0; col < 4; ++col) colour_pass<T>(c, l, col, true, x, b, s);
    full_pass<T, MODE_ARES>(c, l, x, b, rl, s);
    T *xc, *bc, *rc, *tc;
    vecs<T>(c, l - 1, &xc, &bc, &rc, &tc);
    restrict_to<T, 3>(c, l, rl, bc, s);
    if (l - 1 == 0) {
        coarse_avel<T>(c, bc, xc, s);
    } else {
        fill_velocity<T>(c, l - 1, xc, s);
        vel_cycle<T>(c, l - 1, nu1, nu2, xc, bc, s);
    }
    prolong_add<T, 3>(c, l, xc, x, s);
    for (int q = 0; q < nu2; ++q)
        for (int col = 3; col >= 0; --col) colour_pass<T>(c, l, col, true, x, b, s);
}

// ------------------------------------------------------- Krylov helpers
inline int vgrid(size_t n) {
    return (int)std::max<size_t>(1, std::min<size_t>((n + TPB - 1) / TPB, VGRID_MAX));
}

// reduce the partials of a vector kernel launched with vgrid(len) into *out
void vreduce(hhg_ctx* c, size_t len, double* out, bool sqrt_out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(RTPB), 0, s, c->kpart, vgrid(len), out,
                       sqrt_out ? 1 : 0);
}

// <a, b> over owned slots of the finest level, fields 0..nf-1 -> *out
void vdot(hhg_ctx* c, const double* a, const double* b, int nf, double* out, hipStream_t s) {
    const size_t len = (size_t)c->H[c->L].len;
    hipLaunchKernelGGL(k_vdot, dim3(vgrid(len)), dim3(TPB), 0, s, a, b, c->A[c->L].owned, len, nf,
                       c->kpart);
    vreduce(c, len, out, false, s);
}

// z = diag(Ahat, Shat)^-1 v on the finest level (eq. precond_block_diag):
// one velocity V(nu, nu) cycle from zero and the weighted lumped mass; *vz
// receives <v, z>
void block_prec(hhg_ctx* c, int nu, const double* v, double* z, double* vz, hipStream_t s) {
    const int L = c->L;
    const size_t len = (size_t)c->H[L].len;
    fill_velocity<double>(c, L, z, s);
    vel_cycle<double>(c, L, nu, nu, z, v, s);
    ops(c, L, 0, 0, 0, 1);
    hipLaunchKernelGGL(k_mr_precp_dot, dim3(vgrid(len)), dim3(TPB), 0, s, v, z, c->A[L].pinv,
                       c->A[L].owned, len, c->kpart);
    vreduce(c, len, vz, false, s);
}

hhg_status read_scalars(hhg_ctx* c, double* h, const double* d, int n, hipStream_t s) {
    HIPCHECK(c, hipMemcpyAsync(h, d, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(c, hipStreamSynchronize(s));
    return HHG_OK;
}

// residual history entry k (the info keeps the first 256)
void hist_put(hhg_solve_info* I, int k, double r) {
    if (k < 256) I->res_hist[k] = r;
    I->cycles = k;
    I->r_final = r;
    I->rel_res = I->r0 > 0.0 ? r / I->r0 : 0.0;
    if (k >= 1 && k < 256 && I->res_hist[k - 1] > 0.0)
        I->rho_max = std::max(I->rho_max, r / I->res_hist[k - 1]);
}

// elapsed time between two recorded events (0 when timing is unavailable)
double event_ms(hipEvent_t a, hipEvent_t b) {
    if (!a || !b) return 0.0;
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms;
}

}  // namespace

// ============================================================== ABI
extern "C" {

void hhg_default_opts(hhg_opts* o) {
    if (!o) return;
    o->nu1 = 3;
    o->nu2 = 3;
    o->cycle = 0;
    o->p_sweep = 0;
    o->omega = 0.3;
    o->precision = 0;
    o->coarse_rtol = 1e-14;
    o->coarse_maxit = 500;
    o->block_order = 1;
    o->coarse_prec = 1;
    o->coarse_solver = 0;
    o->krylov = 0;
    o->graphs = 0;
    o->op = 0;
    o->ordering = 0;
}

const char* hhg_global_error(void) { return g_error.c_str(); }
const char* hhg_last_error(const hhg_ctx* c) { return c ? c->err.c_str() : g_error.c_str(); }

hhg_status hhg_plan(const hhg_mesh* mesh, int32_t R, const hhg_opts* opts, size_t* bytes) {
    if (!bytes) return fail(nullptr, HHG_EINVAL, "workspace_bytes is NULL");
    std::unique_ptr<hhg_ctx> c(new hhg_ctx());
    hhg_status s = build_host(c.get(), mesh, R, opts);
    if (s != HHG_OK) return s;
    *bytes = layout(c.get(), nullptr);
    return HHG_OK;
}

hhg_status hhg_create(const hhg_mesh* mesh, int32_t R, const hhg_opts* opts, void* ws, size_t bytes,
                      hhg_ctx** out) {
    if (!out) return fail(nullptr, HHG_EINVAL, "ctx output pointer is NULL");
    *out = nullptr;
    std::unique_ptr<hhg_ctx> c(new hhg_ctx());
    hhg_status s = build_host(c.get(), mesh, R, opts);
    if (s != HHG_OK) return s;
    const size_t need = layout(c.get(), nullptr);
    if (ws) {
        if (bytes < need)
            return fail(nullptr, HHG_ENOMEM,
                        "workspace too small: need " + std::to_string(need) + " bytes");
        if (((uintptr_t)ws) % 256 != 0) return fail(nullptr, HHG_EINVAL, "workspace not 256-byte aligned");
        c->ws = (char*)ws;
        c->ws_bytes = bytes;
        layout(c.get(), c->ws);
        if ((s = upload_all(c.get())) != HHG_OK) {
            g_error = c->err;
            return s;
        }
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return fail(nullptr, HHG_EDEVICE, hipGetErrorString(e));
        if ((e = hipGetDevice(&c->dev)) != hipSuccess)
            return fail(nullptr, HHG_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
        if ((e = scratch_address(c->dev, &c->scratch)) != hipSuccess)
            return fail(nullptr, HHG_EDEVICE,
                        std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        c->device = true;
    }
    *out = c.release();
    return HHG_OK;
}

void hhg_destroy(hhg_ctx* c) {
    if (!c) return;
    for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
    drop_graphs(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
}

int32_t hhg_num_levels(const hhg_ctx* c) { return c ? c->L + 1 : 0; }
int64_t hhg_vec_len(const hhg_ctx* c, int32_t l) {
    return (c && l >= 0 && l <= c->L) ? c->H[l].len : -1;
}
int64_t hhg_num_nodes(const hhg_ctx* c, int32_t l) {
    return (c && l >= 0 && l <= c->L) ? c->H[l].N : -1;
}
int64_t hhg_num_dofs(const hhg_ctx* c, int32_t l) {
    return (c && l >= 0 && l <= c->L) ? 3 * c->H[l].nfree + c->H[l].nnodes : -1;
}
int64_t hhg_num_interface(const hhg_ctx* c, int32_t l) {
    return (c && l >= 0 && l <= c->L) ? c->H[l].nif : -1;
}

hhg_status hhg_node_info(const hhg_ctx* c, int32_t l, int32_t* ijk, int8_t* dir) {
    if (!c || l < 0 || l > c->L) return fail(nullptr, HHG_EINVAL, "bad context or level");
    const HostLevel& h = c->H[l];
    for (int64_t v = 0; v < h.N; ++v) {
        if (ijk) {
            ijk[3 * v + 0] = (int32_t)(v % h.lat[0]);
            ijk[3 * v + 1] = (int32_t)((v / h.lat[0]) % h.lat[1]);
            ijk[3 * v + 2] = (int32_t)(v / ((int64_t)h.lat[0] * h.lat[1]));
        }
        if (dir) dir[v] = h.node_dir[v] ? 1 : h.node_slip[v] ? 2 : 0;
    }
    return HHG_OK;
}

hhg_status hhg_primitive_classes(const hhg_ctx* c, int32_t l, int8_t* cls) {
    if (!c || l < 0 || l > c->L || !cls)
        return fail(nullptr, HHG_EINVAL, "bad context, level or array");
    const HostLevel& h = c->H[l];
    for (int64_t v = 0; v < h.N; ++v) cls[v] = h.node_slot[v] >= 0 ? 3 : -1;
    for (int t = 0; t < h.nif; ++t) {
        const int pat = h.keys[h.if_sid[t] - h.nm][0].second;
        const int zeros = (pat & 1) + (pat >> 1 & 1) + (pat >> 2 & 1) + (pat >> 3 & 1);
        cls[h.if_lat[t]] = (int8_t)(3 - zeros);
    }
    return HHG_OK;
}

hhg_status hhg_mass_weights(const hhg_ctx* c, int32_t l, double* m) {
    if (!c || l < 0 || l > c->L || !m) return fail(nullptr, HHG_EINVAL, "bad context, level or array");
    const HostLevel& h = c->H[l];
    for (int64_t v = 0; v < h.N; ++v) {
        if (h.node_slot[v] < 0) {   // hole
            m[v] = 0.0;
            continue;
        }
        const int sid = h.node_sid[v];
        const double* rec = sid < 0 ? &h.st_vol_global[(size_t)(-sid - 1) * ST_SIZE]
                                    : &h.st[(size_t)sid * ST_SIZE];
        m[v] = rec[ST_MASS];
    }
    return HHG_OK;
}

#define CHECK_DEV(c)                                                                     \
    do {                                                                                 \
        if (!(c)) return fail(nullptr, HHG_EINVAL, "context is NULL");                   \
        if (!(c)->device) return fail(c, HHG_EINVAL, "host-only context (no workspace)"); \
    } while (0)
#define CHECK_LEVEL(c, l) \
    if ((l) < 0 || (l) > (c)->L) return fail(c, HHG_EINVAL, "level out of range")
#define CHECK_PTR(c, p) \
    if (!(p)) return fail(c, HHG_EINVAL, #p " is NULL")
#define LAUNCH_CHECK(c)                                                              \
    do {                                                                             \
        hipError_t e_ = hipGetLastError();                                           \
        if (e_ != hipSuccess) return fail(c, HHG_EDEVICE, hipGetErrorString(e_));    \
    } while (0)

hhg_status hhg_scatter(hhg_ctx* c, int32_t l, const double* nodal, int32_t nf, void* x,
                       hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_LEVEL(c, l);
    CHECK_PTR(c, nodal);
    CHECK_PTR(c, x);
    if (nf < 1 || nf > 4) return fail(c, HHG_EINVAL, "nfields must be 1..4");
    const HostLevel& h = c->H[l];
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(h.len)), dim3(TPB), 0, (hipStream_t)stream,
                       c->A[l].slot_node, (size_t)h.len, nf, nodal, (size_t)h.N, (double*)x);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_gather(hhg_ctx* c, int32_t l, const void* x, int32_t nf, double* nodal,
                      hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_LEVEL(c, l);
    CHECK_PTR(c, nodal);
    CHECK_PTR(c, x);
    if (nf < 1 || nf > 4) return fail(c, HHG_EINVAL, "nfields must be 1..4");
    const HostLevel& h = c->H[l];
    hipLaunchKernelGGL(k_gather, dim3(grid_for(h.N)), dim3(TPB), 0, (hipStream_t)stream,
                       c->A[l].node_slot, (size_t)h.N, nf, (const double*)x, (size_t)h.len, nodal);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_exchange(hhg_ctx* c, int32_t l, void* x, int32_t nf, hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_LEVEL(c, l);
    CHECK_PTR(c, x);
    if (nf < 1 || nf > 4) return fail(c, HHG_EINVAL, "nfields must be 1..4");
    const HostLevel& h = c->H[l];
    if (h.nif > 0)
        hipLaunchKernelGGL(k_exchange<double>, dim3((h.nif + TPB - 1) / TPB), dim3(TPB), 0,
                           (hipStream_t)stream, c->D64[l], nf, (double*)x);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_rhs(hhg_ctx* c, const void* f, void* rhs, hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_PTR(c, f);
    CHECK_PTR(c, rhs);
    if (f == rhs) return fail(c, HHG_EINVAL, "f and rhs must not alias");
    full_pass<double, MODE_RHS>(c, c->L, (const double*)f, nullptr, (double*)rhs,
                                (hipStream_t)stream);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_rhs_level(hhg_ctx* c, int32_t l, const void* f, void* rhs, hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_LEVEL(c, l);
    CHECK_PTR(c, f);
    CHECK_PTR(c, rhs);
    if (f == rhs) return fail(c, HHG_EINVAL, "f and rhs must not alias");
    full_pass<double, MODE_RHS>(c, l, (const double*)f, nullptr, (double*)rhs, (hipStream_t)stream);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_apply(hhg_ctx* c, int32_t l, const void* x, void* y, hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_LEVEL(c, l);
    CHECK_PTR(c, x);
    CHECK_PTR(c, y);
    if (x == y) return fail(c, HHG_EINVAL, "x and y must not alias");
    full_pass<double, MODE_APPLY>(c, l, (const double*)x, nullptr, (double*)y, (hipStream_t)stream);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_residual(hhg_ctx* c, int32_t l, const void* x, const void* b, void* r,
                        double* h_norm, hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_LEVEL(c, l);
    CHECK_PTR(c, x);
    CHECK_PTR(c, b);
    CHECK_PTR(c, r);
    if (r == x || r == b) return fail(c, HHG_EINVAL, "r must not alias x or b");
    hipStream_t s = (hipStream_t)stream;
    residual_norm<double>(c, l, (const double*)x, (const double*)b, (double*)r, c->scal, s);
    LAUNCH_CHECK(c);
    if (h_norm) {
        HIPCHECK(c, hipMemcpyAsync(h_norm, c->scal, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(c, hipStreamSynchronize(s));
    }
    return HHG_OK;
}

hhg_status hhg_residual_noalloc(hhg_ctx* c, int32_t l, const void* x, const void* b, void* r,
                                double* d_norm, hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_LEVEL(c, l);
    CHECK_PTR(c, x);
    CHECK_PTR(c, b);
    CHECK_PTR(c, r);
    CHECK_PTR(c, d_norm);
    if (r == x || r == b) return fail(c, HHG_EINVAL, "r must not alias x or b");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->dev)
        return fail(c, HHG_EINVAL, "the context's device must be the current device");
    LevelDev<double>& v = view<double>(c, l);
    const int np = residual_partials(v);
    if ((size_t)np > NOALLOC_SCRATCH_DOUBLES)
        return fail(c, HHG_EINVAL,
                    "level too large for the static scratch: " + std::to_string(np) +
                        " partial sums, at most " + std::to_string(NOALLOC_SCRATCH_DOUBLES));
    hipStream_t s = (hipStream_t)stream;
    // every partial in [0, np) is written by its block before the sum reads
    // it, so the scratch needs no clearing between calls
    launch_kx<double, MODE_RES, false>(c, v, iface_blocks(v.nif), (const double*)x,
                                       (const double*)b, (double*)r, s, c->scratch);
    hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(RTPB), 0, s, (const double*)c->scratch, np, d_norm,
                       1);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_smooth(hhg_ctx* c, int32_t l, void* x, const void* b, int32_t steps,
                      hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_LEVEL(c, l);
    CHECK_PTR(c, x);
    CHECK_PTR(c, b);
    if (steps < 0 || steps > 1000) return fail(c, HHG_EINVAL, "steps must be 0..1000");
    mirror_refresh<double>(c, l, (const double*)x, (hipStream_t)stream);
    for (int q = 0; q < steps; ++q)
        uzawa_step<double>(c, l, (double*)x, (const double*)b, c->A[l].t64, (hipStream_t)stream);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_restrict(hhg_ctx* c, int32_t l, const void* rf, void* bc, hhg_stream stream) {
    CHECK_DEV(c);
    if (l < 1 || l > c->L) return fail(c, HHG_EINVAL, "level must be 1..L");
    CHECK_PTR(c, rf);
    CHECK_PTR(c, bc);
    restrict_to<double>(c, l, (const double*)rf, (double*)bc, (hipStream_t)stream);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_prolong_add(hhg_ctx* c, int32_t l, const void* ec, void* xf, hhg_stream stream) {
    CHECK_DEV(c);
    if (l < 1 || l > c->L) return fail(c, HHG_EINVAL, "level must be 1..L");
    CHECK_PTR(c, ec);
    CHECK_PTR(c, xf);
    prolong_add<double>(c, l, (const double*)ec, (double*)xf, (hipStream_t)stream);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_coarse_solve(hhg_ctx* c, const void* b0, void* x0, int32_t* iters, double* relres,
                            hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_PTR(c, b0);
    CHECK_PTR(c, x0);
    if (b0 == x0) return fail(c, HHG_EINVAL, "b0 and x0 must not alias");
    hipStream_t s = (hipStream_t)stream;
    coarse_solve<double>(c, (const double*)b0, (double*)x0, s);
    LAUNCH_CHECK(c);
    if (iters || relres) {
        double st[2];
        HIPCHECK(c, hipMemcpyAsync(st, c->scal + 8, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(c, hipStreamSynchronize(s));
        if (iters) *iters = (int32_t)st[0];
        if (relres) *relres = st[1];
    }
    return HHG_OK;
}

hhg_status hhg_project(hhg_ctx* c, int32_t l, void* x, hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_LEVEL(c, l);
    CHECK_PTR(c, x);
    project<double>(c, l, (double*)x, (hipStream_t)stream);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

}  // extern "C"

namespace {

// one solver iteration on the finest level; on entry of the mixed variant
// r64_L must hold b - K x and scal[0] its norm, of the FP64 one with t_ready
// t64_L f - B^T p
void cycle_fp64(hhg_ctx* c, double* x, const double* b, hipStream_t s, bool t_ready = false) {
    vcycle<double>(c, c->L, c->L, x, b, s, t_ready ? c->A[c->L].t64 : nullptr);
    project<double>(c, c->L, x, s);
}

void cycle_mixed(hhg_ctx* c, double* x, hipStream_t s) {
    const int L = c->L;
    DevLevelArrays& a = c->A[L];
    const size_t n4 = 4 * (size_t)c->H[L].len;
    hipLaunchKernelGGL(k_scale_cast<float>, dim3(grid_for(n4)), dim3(TPB), 0, s, a.r64, c->scal,
                       a.b32, n4);
    fill_iterate<float>(c, L, a.x32, s);
    // the correction starts from 0: f - B^T p = b
    vcycle<float>(c, L, L, a.x32, a.b32, s, a.b32);
    hipLaunchKernelGGL(k_axpy_cast<float>, dim3(grid_for(n4)), dim3(TPB), 0, s, x, c->scal, a.x32,
                       n4);
    project<double>(c, L, x, s);
}

}  // namespace

extern "C" {

hhg_status hhg_vcycle(hhg_ctx* c, void* x, const void* b, hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_PTR(c, x);
    CHECK_PTR(c, b);
    if (x == b) return fail(c, HHG_EINVAL, "x and b must not alias");
    hipStream_t s = (hipStream_t)stream;
    if (c->opts.precision == 1) {
        residual_norm<double>(c, c->L, (const double*)x, (const double*)b, c->A[c->L].r64, c->scal, s);
        cycle_mixed(c, (double*)x, s);
    } else {
        mirror_refresh<double>(c, c->L, (const double*)x, s);
        cycle_fp64(c, (double*)x, (const double*)b, s);
    }
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_fmg(hhg_ctx* c, void* const* xs, const void* const* bs, int32_t cycles,
                   hhg_stream stream) {
    CHECK_DEV(c);
    if (!xs || !bs) return fail(c, HHG_EINVAL, "level pointer arrays are NULL");
    if (c->opts.precision != 0) return fail(c, HHG_EINVAL, "full multigrid runs in FP64 only");
    if (cycles < 1 || cycles > 16) return fail(c, HHG_EINVAL, "cycles must be 1..16");
    for (int l = 0; l <= c->L; ++l) {
        CHECK_PTR(c, xs[l]);
        CHECK_PTR(c, bs[l]);
        if (xs[l] == bs[l]) return fail(c, HHG_EINVAL, "x and b of a level must not alias");
        for (int q = 0; q < l; ++q)
            if (xs[q] == xs[l]) return fail(c, HHG_EINVAL, "iterates of two levels alias");
    }
    hipStream_t s = (hipStream_t)stream;
    // level 0: x_0 = x_D + K_0^-1 (b_0 - K_0 x_D) from the Dirichlet values alone
    {
        LevelDev<double>& v = view<double>(c, 0);
        hipLaunchKernelGGL(k_keep_dirichlet<double>, dim3(grid_for((size_t)v.len)), dim3(TPB), 0, s, v,
                           (double*)xs[0]);
        vcycle<double>(c, 0, 0, (double*)xs[0], (const double*)bs[0], s);
        project<double>(c, 0, (double*)xs[0], s);
    }
    for (int l = 1; l <= c->L; ++l) {
        LevelDev<double>& F = view<double>(c, l);
        LevelDev<double>& C = view<double>(c, l - 1);
        // x_l = P x_(l-1) (Dirichlet velocity kept); writes the mirror of x_l too
        hipLaunchKernelGGL((k_prolong<double, true>), dim3(full_blocks(F.n_ctiles)), dim3(TPB), 0, s, F,
                           C, (const double*)xs[l - 1], (double*)xs[l]);
        for (int q = 0; q < cycles; ++q) {
            vcycle<double>(c, l, l, (double*)xs[l], (const double*)bs[l], s);
            project<double>(c, l, (double*)xs[l], s);
        }
    }
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_solve(hhg_ctx* c, void* xv, const void* bv, double rtol, int32_t max_cycles,
                     hhg_solve_info* info, hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_PTR(c, xv);
    CHECK_PTR(c, bv);
    if (xv == bv) return fail(c, HHG_EINVAL, "x and b must not alias");
    if (!(rtol > 0.0) || max_cycles < 0 || max_cycles > 255)
        return fail(c, HHG_EINVAL, "need rtol > 0 and 0 <= max_cycles <= 255");
    hipStream_t s = (hipStream_t)stream;
    double* x = (double*)xv;
    const double* b = (const double*)bv;
    hhg_solve_info loc;
    hhg_solve_info* I = info ? info : &loc;
    std::memset(I, 0, sizeof(*I));
    reset_ops(c);
    if (c->mi.slip) {
        // the iterate starts in the constrained space (u . n = 0 on free-slip vertices)
        LevelDev<double>& vf = view<double>(c, c->L);
        hipLaunchKernelGGL(k_slip_project<double>, dim3((vf.nif + TPB - 1) / TPB), dim3(TPB), 0, s,
                           vf, x);
    }
    hipEvent_t e0 = next_event(c), e1 = next_event(c);
    double* r = c->A[c->L].r64;
    // FP64 cycles smooth x itself: take its mirror once; the cycles and the
    // projection keep it current, so the stopping test may use it too.  On
    // Kuhn macros in the Laplace form (colour or red-black order) the
    // stopping test also leaves f - B^T p of x in t for the next cycle's
    // first Uzawa step.
    const bool fp64 = c->opts.precision != 1;
    const bool tfuse = fp64 && !dpath(c) && c->opts.ordering != 1;
    double* tL = c->A[c->L].t64;
    if (tfuse) {
        mirror_refresh<double>(c, c->L, x, s);
        residual_norm_t<double>(c, c->L, x, b, tL, c->scal, s);
    } else {
        residual_norm<double>(c, c->L, x, b, r, c->scal, s);
    }
    double nrm;
    HIPCHECK(c, hipMemcpyAsync(&nrm, c->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(c, hipStreamSynchronize(s));
    I->r0 = nrm;
    I->res_hist[0] = nrm;
    I->r_final = nrm;
    I->rel_res = nrm > 0 ? 1.0 : 0.0;
    if (!std::isfinite(nrm)) {
        I->status = HHG_ENAN;
        return fail(c, HHG_ENAN, "initial residual is not finite");
    }
    if (nrm == 0.0) {
        I->status = HHG_OK;
        return HHG_OK;
    }
    const double r0 = nrm;
    double prev = nrm;
    int stagn = 0;
    hhg_status st = HHG_ENOCONV;
    if (e0) (void)hipEventRecord(e0, s);
    if (fp64 && !tfuse) mirror_refresh<double>(c, c->L, x, s);
    int k = 0;
    // one cycle and its stopping-test residual: the same launches every cycle,
    // replayed from a captured graph unless graphs are off or timing is on
    auto body = [&](hipStream_t st) {
        if (!fp64)
            cycle_mixed(c, x, st);
        else
            cycle_fp64(c, x, b, st, tfuse);
        PhaseTimed pt(c, PH_RESIDUAL, c->L, st);
        if (tfuse)
            residual_norm_t<double>(c, c->L, x, b, tL, c->scal, st);
        else
            residual_norm<double>(c, c->L, x, b, r, c->scal, st, fp64);
    };
    for (auto& v : c->ppairs) v.clear();
    c->phase_active = c->phase_timing;
    hhg_ctx::CycleGraph* graph = (c->opts.graphs && !c->timing && !c->phase_timing)
                                     ? cycle_graph(c, x, b, body)
                                     : nullptr;
    for (k = 1; k <= max_cycles; ++k) {
        if (graph)
            HIPCHECK(c, replay(c, graph, s));
        else
            body(s);
        HIPCHECK(c, hipMemcpyAsync(&nrm, c->scal, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(c, hipStreamSynchronize(s));
        I->res_hist[k] = nrm;
        I->cycles = k;
        I->r_final = nrm;
        I->rel_res = nrm / r0;
        if (!std::isfinite(nrm)) {
            st = HHG_ENAN;
            break;
        }
        const double rho = nrm / prev;
        I->rho_max = std::max(I->rho_max, rho);
        prev = nrm;
        if (nrm <= rtol * r0) {
            st = HHG_OK;
            break;
        }
        if (nrm > 1e3 * r0) break;               // divergence
        stagn = rho > 0.99 ? stagn + 1 : 0;      // stagnation
        if (stagn >= 5) break;
    }
    c->phase_active = false;
    if (e1) (void)hipEventRecord(e1, s);
    if (e0 && e1) {
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        I->t_solve_ms = ms;
    }
    if (I->cycles > 0) I->rho_mean = std::pow(I->rel_res, 1.0 / I->cycles);
    put_ops(c, I);
    {
        double* dst[4] = {&I->t_smooth_ms, &I->t_transfer_ms, &I->t_coarse_ms, &I->t_residual_ms};
        for (int q = 0; q < HHG_MAX_LEVELS; ++q) I->t_level_ms[q] = 0.0;
        for (int ph = 0; ph < 4; ++ph) {
            double t = 0.0;
            for (const TimerPair& tp : c->ppairs[ph]) {
                const double ms = event_ms(tp.a, tp.b);
                t += ms;
                if (tp.lev >= 0 && tp.lev < HHG_MAX_LEVELS) I->t_level_ms[tp.lev] += ms;
            }
            *dst[ph] = t;
            c->ppairs[ph].clear();
        }
    }
    I->status = st;
    c->evused = c->timing ? c->evused : 0;
    LAUNCH_CHECK(c);
    if (st == HHG_ENAN) return fail(c, HHG_ENAN, "residual norm is not finite");
    if (st == HHG_ENOCONV) return fail(c, HHG_ENOCONV, "tolerance not reached");
    return HHG_OK;
}

hhg_status hhg_grad(hhg_ctx* c, const void* x, const void* lam, const void* f, double* dnu,
                    void* df, hhg_stream stream) {
    CHECK_DEV(c);
    if (c->mi.slip) return fail(c, HHG_EINVAL, "the gradient does not handle free-slip faces");
    CHECK_PTR(c, x);
    CHECK_PTR(c, lam);
    CHECK_PTR(c, dnu);
    hipStream_t s = (hipStream_t)stream;
    LevelDev<double>& v = c->D64[c->L];
    hipLaunchKernelGGL(k_grad_nu, dim3(v.n_ctiles), dim3(TPB), 0, s, v, (const double*)x,
                       (const double*)lam, (const double*)f, c->gpart, c->opts.op == 1 ? 1 : 0);
    hipLaunchKernelGGL(k_grad_reduce, dim3(v.nm), dim3(TPB), 0, s, c->A[c->L].ctile_macro0,
                       c->gpart, dnu);
    if (df) {
        if (df == lam) return fail(c, HHG_EINVAL, "dJ_df must not alias lambda");
        full_pass<double, MODE_GRADF>(c, c->L, (const double*)lam, nullptr, (double*)df, s);
    }
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_adjoint_rhs(hhg_ctx* c, const void* g, void* y, hhg_stream stream) {
    CHECK_DEV(c);
    if (c->mi.slip) return fail(c, HHG_EINVAL, "the adjoint does not handle free-slip faces");
    CHECK_PTR(c, g);
    CHECK_PTR(c, y);
    if (g == y) return fail(c, HHG_EINVAL, "g and rhs must not alias");
    hipStream_t s = (hipStream_t)stream;
    const int L = c->L;
    LevelDev<double>& v = view<double>(c, L);
    const int ib = iface_blocks(v.nif);
    const int grid = ib + v.n_vtiles;
    const size_t len = (size_t)v.len;
    if (c->mi.project) {
        hipLaunchKernelGGL((k_mass_dot<double, true>), dim3(grid), dim3(TPB), 0, s, v,
                           (const double*)g + 3 * len, c->partials, ib);
        hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(RTPB), 0, s, c->partials,
                           v.nv_nat + (v.nif + TPB - 1) / TPB, c->scal + 16, 0);
    }
    fill<double>((double*)y, 4 * len, 0.0, s);
    hipLaunchKernelGGL(k_adjoint_rhs, dim3(grid), dim3(TPB), 0, s, v, (const double*)g, (double*)y,
                       (const double*)(c->scal + 16), c->inv_mass[L], c->mi.project ? 1 : 0, ib);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_set_viscosity(hhg_ctx* c, const double* nu) {
    if (!c) return fail(nullptr, HHG_EINVAL, "context is NULL");
    CHECK_PTR(c, nu);
    for (size_t m = 0; m < c->mi.macros.size(); ++m)
        if (!std::isfinite(nu[m]) || nu[m] <= 0.0)
            return fail(c, HHG_EINVAL, "viscosity must be finite and positive");
    for (size_t m = 0; m < c->mi.macros.size(); ++m) c->mi.macros[m].nu = nu[m];
    std::string err;
    for (int l = 0; l <= c->L; ++l)
        if (!compute_stencils(c->mi, &c->H[l], &err)) return fail(c, HHG_EINVAL, err);
    if (!build_coarse_for(c, &err)) return fail(c, HHG_EINVAL, err);
    if (!c->device) return HHG_OK;
    drop_graphs(c);
    // kernels queued on any stream may still read the old tables: the
    // uploads below are not ordered after them
    HIPCHECK(c, hipDeviceSynchronize());
    hhg_status st = upload_stencils(c);
    if (st != HHG_OK) return st;
    HIPCHECK(c, hipDeviceSynchronize());
    return HHG_OK;
}

}  // extern "C"

namespace {

// lattice index of macro-local vertex (i, j, k) of macro m at level h
int64_t lattice_of(const hhg_ctx* c, const HostLevel& h, int m, int i, int j, int k) {
    const MacroInfo& M = c->mi.macros[m];
    int X[3] = {M.o[0] * h.n, M.o[1] * h.n, M.o[2] * h.n};
    X[M.ax[0]] += i + j + k;
    X[M.ax[1]] += j + k;
    X[M.ax[2]] += k;
    return X[0] + (int64_t)h.lat[0] * (X[1] + (int64_t)h.lat[1] * X[2]);
}

const int CK_LOFF[15][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {-1, 1, 0}, {1, -1, 0},
                            {0, 1, 0},  {0, -1, 0}, {0, -1, 1}, {0, 1, -1}, {-1, 0, 1},
                            {1, 0, -1}, {0, 0, 1},  {0, 0, -1}, {1, -1, 1}, {-1, 1, -1}};
const int CK_GDIR[15][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                            {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {0, 1, 1},
                            {0, -1, -1}, {1, 0, 1},  {-1, 0, -1}, {1, 1, 1},  {-1, -1, -1}};

#define CK(cond, msg)                                                                  \
    do {                                                                               \
        if (!(cond)) {                                                                 \
            *err = std::string("layout check, level ") + std::to_string(l) + ": " + msg; \
            return false;                                                              \
        }                                                                              \
    } while (0)

bool check_level(const hhg_ctx* c, int l, std::string* err) {
    const HostLevel& h = c->H[l];
    const int n = h.n;
    const int* sb = h.slab_base.data();
    auto slot_ok = [&](int s, int m) {
        return s >= (int64_t)m * h.mstride && s < (int64_t)(m + 1) * h.mstride && s < h.len;
    };
    // interior tiles: every interior vertex exactly once, all 15 taps exact
    std::vector<uint8_t> seen(h.len, 0);
    for (const Tile& t : h.vtiles) {
        if (t.macro < 0) continue;
        const int m = t.macro, k = t.k, mm = n - k;
        CK(k >= 1 && k <= n - 1, "interior tile outside slabs 1..n-1");
        for (int lane = 0; lane < TPB; ++lane) {
            LanePos P = decode_lane(t, n, 1, mm - 2, lane);
            if (!P.ok) continue;
            const int j = P.j;
            CK(j >= 1 && j <= mm - 2 && P.q < ((mm + 4 - j) >> 2), "lane decoded outside its slab");
            Rows R;
            make_rows(sb, n, (int)(m * h.mstride), j, k, R);
            for (int cc = 0; cc < 4; ++cc) {
                const int i = 4 * P.q + ((cc + 2 * j + k) & 3);
                if (i < 1 || i > mm - 1 - j) continue;
                int64_t lat = lattice_of(c, h, m, i, j, k);
                int X = (int)(lat % h.lat[0]), Y = (int)((lat / h.lat[0]) % h.lat[1]),
                    Z = (int)(lat / ((int64_t)h.lat[0] * h.lat[1]));
                CK(((X + Y + Z) & 3) == cc, "colour sweep picks a vertex of another colour");
            }
            for (int r = 0; r < 4; ++r) {
                const int i = 4 * P.q + r;
                if (i < 1 || i > mm - 1 - j) continue;
                int s[15], a[7];
                nbr_slots(R, i, s);
                axis_slots(R, i, a);
                const int ax[7] = {0, 1, 2, 3, 4, 7, 8};
                for (int q = 0; q < 7; ++q) CK(a[q] == s[ax[q]], "axis taps differ from full taps");
                for (int q = 0; q < 15; ++q) {
                    CK(slot_ok(s[q], m), "tap slot outside the macro");
                    CK(h.slot_node[s[q]] ==
                           lattice_of(c, h, m, i + CK_LOFF[q][0], j + CK_LOFF[q][1], k + CK_LOFF[q][2]),
                       "tap slot holds the wrong vertex");
                }
                CK(seen[s[0]] == 0, "interior vertex visited twice");
                seen[s[0]] = 1;
            }
        }
    }
    for (int m = 0; m < h.nm; ++m)
        for (int k = 1; k < n; ++k)
            for (int j = 1; j <= n - k - 2; ++j)
                for (int i = 1; i <= n - k - 1 - j; ++i)
                    CK(seen[local_slot(h, m, i, j, k)] == 1, "interior vertex not covered");
    // red-black volume blocks: each tile once per colour of the parity (the
    // lanes' colour picks are the colour sweeps' above), both halves of a tile
    // eight blocks apart, so on one XCD whatever the leading interface blocks
    {
        const int nvt = (int)h.vtiles.size();
        std::vector<int> half_block((size_t)nvt * 2, -1);
        for (int v = 0; v < rb_blocks(nvt); ++v) {
            const int ti = rb_tile(v), e = rb_half(v);
            if (ti >= nvt) continue;
            CK(half_block[(size_t)ti * 2 + e] < 0, "red-black tile half visited twice");
            half_block[(size_t)ti * 2 + e] = v;
        }
        for (int ti = 0; ti < nvt; ++ti) {
            const int v0 = half_block[(size_t)ti * 2], v1 = half_block[(size_t)ti * 2 + 1];
            CK(v0 >= 0 && v1 >= 0, "red-black tile half not covered");
            CK(((v0 ^ v1) & 7) == 0, "red-black halves of a tile on different XCDs");
        }
    }
    // compact mirror: taps name the same vertex as the slot taps; every copy
    // of an interface vertex and every halo slot maps to its entry; a slot
    // with an entry passes the kernels' near-boundary test
    {
        const int nif = h.nif;
        CK(h.ncomp == nif + (int)h.halo_slot.size(), "mirror size");
        CK((int64_t)h.comp_of_slot.size() == h.len, "mirror slot table size");
        auto slot_of_entry = [&](int e) { return e < nif ? h.if_self[e] : h.halo_slot[e - nif]; };
        for (int t = 0; t < nif; ++t)
            for (int g = 0; g < 14; ++g) {
                const int e = h.if_tap[(size_t)g * nif + t];
                CK(e >= 0 && e < h.ncomp, "mirror tap out of range");
                CK(h.slot_node[slot_of_entry(e)] == h.slot_node[h.if_nb[(size_t)g * nif + t]],
                   "mirror tap names another vertex");
            }
        for (int t = 0; t < nif; ++t)
            for (int q = h.if_cptr[t]; q < h.if_cptr[t + 1]; ++q)
                CK(h.comp_of_slot[h.if_copy[q]] == t, "interface copy without its mirror entry");
        for (size_t e = 0; e < h.halo_slot.size(); ++e)
            CK(h.comp_of_slot[h.halo_slot[e]] == nif + (int)e, "halo slot without its mirror entry");
        int64_t with_entry = 0;
        for (int m = 0; m < h.nm; ++m)
            for (int k = 0; k <= n; ++k)
                for (int j = 0; j <= n - k; ++j)
                    for (int i = 0; i <= n - k - j; ++i) {
                        const int64_t sl = local_slot(h, m, i, j, k);
                        if (h.comp_of_slot[sl] < 0) continue;
                        ++with_entry;
                        CK(near_boundary(n, i, j, k), "mirror entry away from the macro boundary");
                    }
        CK(with_entry == (int64_t)h.if_copy.size() + (int64_t)h.halo_slot.size(),
           "mirror entries on padding slots");
    }
    // hybrid ordering: every interface vertex in one pressure group and every
    // velocity-free one in one velocity group, of its own colour; masked taps
    // reach interface vertices of another primitive in the same group class
    {
        const int nif = h.nif;
        std::vector<int> colour(nif, -1), cls(nif, -1);
        for (int cc = 0; cc < 4; ++cc)
            for (int t = h.col_start[cc]; t < h.col_start[cc + 1]; ++t) colour[t] = cc;
        for (int kind = 0; kind < 2; ++kind) {
            std::vector<int> seen(nif, 0);
            for (int k = 0; k < 3; ++k)
                for (int cc = 0; cc < 4; ++cc)
                    for (int q = h.hyb_off[12 * kind + 4 * k + cc]; q < h.hyb_off[12 * kind + 4 * k + cc + 1];
                         ++q) {
                        const int t = h.hyb_list[q];
                        CK(t >= 0 && t < nif, "hybrid list entry out of range");
                        CK(colour[t] == cc, "hybrid group holds a vertex of another colour");
                        CK(kind == 1 || h.if_flag[t] == 0, "hybrid velocity group holds a Dirichlet vertex");
                        seen[t]++;
                        CK(cls[t] < 0 || cls[t] == k, "vertex in two primitive classes");
                        cls[t] = k;
                    }
            for (int t = 0; t < nif; ++t)
                CK(seen[t] == ((kind == 1 || h.if_flag[t] == 0) ? 1 : 0),
                   "hybrid groups do not partition the interface");
        }
        for (int t = 0; t < nif; ++t)
            for (int g = 0; g < 14; ++g)
                if (h.hyb_mask[t] >> g & 1) {
                    const int e = h.if_tap[(size_t)g * nif + t];
                    CK(e < nif && cls[e] == cls[t] && h.if_sid[e] != h.if_sid[t],
                       "hybrid mask flags a tap outside the vertex's class");
                }
    }
    // full-pass blocks: each real tile once per sub-row, on the tile's XCD,
    // partial slots 4 nat + r distinct and below the reduction count (the
    // prolongation maps its closure tiles the same way)
    for (const std::vector<Tile>* tv : {&h.vtiles, &h.ctiles}) {
        const std::vector<Tile>& tiles = *tv;
        const int lead = tv == &h.vtiles ? iface_blocks(h.nif) : 0;
        const int nvt = (int)tiles.size(), nfb = full_blocks(nvt);
        std::vector<uint8_t> hit((size_t)nvt * 4, 0);
        int nat_real = 0;
        for (const Tile& t : tiles) nat_real += t.macro >= 0 ? 1 : 0;
        std::vector<uint8_t> pslot((size_t)4 * nat_real, 0);
        for (int v = 0; v < nfb; ++v) {
            const int ti = full_tile(v), r = full_sub(v);
            if (ti >= nvt) continue;
            CK(((lead + v) & 7) == (ti & 7) || c->opts.block_order != 1,
               "full-pass block off its tile's XCD");
            CK(hit[(size_t)ti * 4 + r] == 0, "full-pass tile/sub-row visited twice");
            hit[(size_t)ti * 4 + r] = 1;
            const Tile& t = tiles[ti];
            if (t.macro < 0) continue;
            CK(t.nat >= 0 && t.nat < nat_real, "tile natural index out of range");
            CK(pslot[(size_t)4 * t.nat + r] == 0, "partial slot used twice");
            pslot[(size_t)4 * t.nat + r] = 1;
        }
        for (size_t q = 0; q < hit.size(); ++q) CK(hit[q] == 1, "full-pass tile/sub-row not covered");
    }
    // closure tiles: every closure vertex exactly once; grad taps; prolongation
    std::fill(seen.begin(), seen.end(), 0);
    for (const Tile& t : h.ctiles) {
        if (t.macro < 0) continue;
        const int m = t.macro, k = t.k, mm = n - k;
        for (int lane = 0; lane < TPB; ++lane) {
            LanePos P = decode_lane(t, n, 0, mm, lane);
            if (!P.ok) continue;
            const int j = P.j;
            for (int r = 0; r < 4; ++r) {
                const int i = 4 * P.q + r;
                if (i > mm - j) continue;
                const int sf = slot_of(sb, n, (int)(m * h.mstride), i, j, k);
                CK(sf == local_slot(h, m, i, j, k), "closure slot mismatch");
                CK(seen[sf] == 0, "closure vertex visited twice");
                seen[sf] = 1;
                for (int q = 0; q < 15; ++q) {
                    const int ii = i + CK_LOFF[q][0], jj = j + CK_LOFF[q][1], kk = k + CK_LOFF[q][2];
                    const int sq = slot_checked(sb, n, (int)(m * h.mstride), ii, jj, kk);
                    const bool inside = ii >= 0 && jj >= 0 && kk >= 0 && ii + jj + kk <= n;
                    CK((sq >= 0) == inside, "closure tap validity");
                    if (inside)
                        CK(slot_ok(sq, m) && h.slot_node[sq] == lattice_of(c, h, m, ii, jj, kk),
                           "closure tap holds the wrong vertex");
                }
                if (l == 0) continue;
                const HostLevel& hc = c->H[l - 1];
                const int mbc = (int)(m * hc.mstride);
                const int pi = i & 1, pj = j & 1, pk = k & 1;
                if ((pi | pj | pk) == 0) {
                    const int sc = slot_of(hc.slab_base.data(), hc.n, mbc, i >> 1, j >> 1, k >> 1);
                    CK(hc.slot_node[sc] == lattice_of(c, hc, m, i >> 1, j >> 1, k >> 1),
                       "prolongation source");
                } else {
                    int di, dj, dk;
                    parity_dir(pi | (pj << 1) | (pk << 2), &di, &dj, &dk);
                    for (int sg = -1; sg <= 1; sg += 2) {
                        const int I = i + sg * di, J = j + sg * dj, K = k + sg * dk;
                        CK((I % 2 == 0) && (J % 2 == 0) && (K % 2 == 0) && I >= 0 && J >= 0 &&
                               K >= 0 && I + J + K <= n,
                           "prolongation endpoint not a coarse closure vertex");
                        const int sc = slot_of(hc.slab_base.data(), hc.n, mbc, I >> 1, J >> 1, K >> 1);
                        CK(sc >= 0 && sc < hc.len &&
                               hc.slot_node[sc] == lattice_of(c, hc, m, I >> 1, J >> 1, K >> 1),
                           "prolongation endpoint slot");
                    }
                }
            }
        }
    }
    for (int64_t s = 0; s < h.len; ++s)
        CK((h.slot_node[s] >= 0) == (seen[s] == 1), "closure tiles and slot map disagree");
    // interface vertices
    for (int cc = 0; cc < 4; ++cc) {
        CK(h.col_start[cc] <= h.vel_end[cc] && h.vel_end[cc] <= h.slip_beg[cc] &&
               h.slip_beg[cc] <= h.col_start[cc + 1],
           "colour ranges");
        for (int t = h.col_start[cc]; t < h.col_start[cc + 1]; ++t) {
            int64_t lat = h.if_lat[t];
            int X = (int)(lat % h.lat[0]), Y = (int)((lat / h.lat[0]) % h.lat[1]),
                Z = (int)(lat / ((int64_t)h.lat[0] * h.lat[1]));
            CK(((X + Y + Z) & 3) == cc, "interface colour");
            CK(h.if_flag[t] == (t < h.vel_end[cc] ? 0 : t < h.slip_beg[cc] ? 1 : 2),
               "interface order: free, Dirichlet, free-slip");
            CK(h.slot_node[h.if_self[t]] == lat, "interface self slot");
            for (int q = h.if_cptr[t]; q < h.if_cptr[t + 1]; ++q)
                CK(h.if_copy[q] >= 0 && h.if_copy[q] < h.len && h.slot_node[h.if_copy[q]] == lat,
                   "interface copy slot");
            const double* rec = &h.st[(size_t)h.if_sid[t] * ST_SIZE];
            for (int g = 1; g < 15; ++g) {
                const int sn = h.if_nb[(size_t)(g - 1) * h.nif + t];
                CK(sn >= 0 && sn < h.len, "interface neighbour slot out of range");
                if (sn == h.if_self[t]) {
                    const int blocks[9] = {ST_A, ST_C, ST_M, ST_B, ST_B + 15, ST_B + 30,
                                           ST_BT, ST_BT + 15, ST_BT + 30};
                    for (int bq : blocks) CK(rec[bq + g] == 0.0, "absent neighbour with a coefficient");
                } else {
                    int64_t want = (X + CK_GDIR[g][0]) +
                                   (int64_t)h.lat[0] * ((Y + CK_GDIR[g][1]) +
                                                        (int64_t)h.lat[1] * (Z + CK_GDIR[g][2]));
                    CK(h.slot_node[sn] == want, "interface neighbour holds the wrong vertex");
                }
            }
            if (l < c->L) {
                const HostLevel& hf = c->H[l + 1];
                const int tf = h.rif_fine[t];
                CK(tf >= 0 && tf < hf.nif, "restriction map out of range");
                int64_t lf = 2 * X + (int64_t)hf.lat[0] * (2 * Y + (int64_t)hf.lat[1] * 2 * Z);
                CK(hf.if_lat[tf] == lf, "restriction map vertex");
            }
        }
    }
    CK(h.col_start[4] == h.nif, "colour ranges do not cover the interface list");
    // restriction of interior coarse vertices: fine taps around (2i, 2j, 2k)
    if (l < c->L) {
        const HostLevel& hf = c->H[l + 1];
        for (const Tile& t : h.vtiles) {
            if (t.macro < 0) continue;
            const int m = t.macro, k = t.k, mm = n - k;
            for (int lane = 0; lane < TPB; ++lane) {
                LanePos P = decode_lane(t, n, 1, mm - 2, lane);
                if (!P.ok) continue;
                Rows RF;
                make_rows(hf.slab_base.data(), hf.n, (int)(m * hf.mstride), 2 * P.j, 2 * k, RF);
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * P.q + r;
                    if (i < 1 || i > mm - 1 - P.j) continue;
                    int s[15];
                    nbr_slots(RF, 2 * i, s);
                    for (int q = 0; q < 15; ++q)
                        CK(s[q] >= 0 && s[q] < hf.len &&
                               hf.slot_node[s[q]] == lattice_of(c, hf, m, 2 * i + CK_LOFF[q][0],
                                                                2 * P.j + CK_LOFF[q][1],
                                                                2 * k + CK_LOFF[q][2]),
                           "restriction tap");
                }
            }
        }
    }
    // grids fit the reduction buffers
    CK(full_blocks((int)h.vtiles.size()) + (h.nif + TPB - 1) / TPB <= c->npartials, "partials too small");
    CK((int)h.ctiles.size() <= c->npartials, "gradient partials too small");
    return true;
}
#undef CK

}  // namespace

extern "C" hhg_status hhg_check_layout(const hhg_ctx* c) {
    if (!c) return fail(nullptr, HHG_EINVAL, "context is NULL");
    std::string err;
    for (int l = 0; l <= c->L; ++l)
        if (!check_level(c, l, &err)) return fail(const_cast<hhg_ctx*>(c), HHG_EINVAL, err);
    return HHG_OK;
}

extern "C" {

hhg_status hhg_set_phase_timing(hhg_ctx* c, int32_t on) {
    if (!c) return fail(nullptr, HHG_EINVAL, "context is NULL");
    if (on != 0 && on != 1) return fail(c, HHG_EINVAL, "on must be 0 or 1");
    c->phase_timing = on == 1;
    for (auto& v : c->ppairs) v.clear();
    return HHG_OK;
}

hhg_status hhg_set_timing(hhg_ctx* c, int32_t on) {
    CHECK_DEV(c);
    c->timing = on != 0;
    c->tgroup_cls = -1;
    for (int q = 0; q < HHG_K_NCLASS; ++q) {
        c->tpairs[q].clear();
        c->tbytes[q] = 0.0;
    }
    c->evused = 0;
    return HHG_OK;
}

hhg_status hhg_kernel_time(hhg_ctx* c, int32_t cls, int64_t* launches, double* ms, double* bytes) {
    CHECK_DEV(c);
    if (cls < 0 || cls >= HHG_K_NCLASS) return fail(c, HHG_EINVAL, "kernel class out of range");
    double tot = 0.0;
    int64_t n = 0;
    for (const TimerPair& p : c->tpairs[cls]) {
        HIPCHECK(c, hipEventSynchronize(p.b));
        float t = 0.f;
        HIPCHECK(c, hipEventElapsedTime(&t, p.a, p.b));
        tot += t;
        n += p.n;
    }
    if (launches) *launches = n;
    if (ms) *ms = tot;
    if (bytes) *bytes = c->tbytes[cls];
    return HHG_OK;
}


hhg_status hhg_vel_cycle(hhg_ctx* c, int32_t nu1, int32_t nu2, void* x, const void* b,
                         hhg_stream stream) {
    CHECK_DEV(c);
    if (c->mi.slip) return fail(c, HHG_EINVAL, "the velocity cycle does not handle free-slip faces");
    CHECK_PTR(c, x);
    CHECK_PTR(c, b);
    if (x == b) return fail(c, HHG_EINVAL, "x and b must not alias");
    if (nu1 < 0 || nu2 < 0 || nu1 + nu2 == 0 || nu1 > 64 || nu2 > 64)
        return fail(c, HHG_EINVAL, "smoothing steps must be in 0..64 with nu1 + nu2 > 0");
    hipStream_t s = (hipStream_t)stream;
    mirror_refresh<double>(c, c->L, (const double*)x, s);
    vel_cycle<double>(c, c->L, nu1, nu2, (double*)x, (const double*)b, s);
    LAUNCH_CHECK(c);
    return HHG_OK;
}

hhg_status hhg_pminres(hhg_ctx* c, void* xv, const void* bv, double rtol, int32_t maxit, int32_t nu,
                       hhg_solve_info* info, hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_PTR(c, xv);
    CHECK_PTR(c, bv);
    if (xv == bv) return fail(c, HHG_EINVAL, "x and b must not alias");
    if (!c->kv[0]) return fail(c, HHG_EINVAL, "Krylov vectors not reserved (create with krylov = 1)");
    if (!(rtol >= 0.0) || maxit < 0 || maxit > 100000 || nu < 1 || nu > 16)
        return fail(c, HHG_EINVAL, "need rtol >= 0, 0 <= maxit <= 100000, 1 <= nu <= 16");
    hipStream_t s = (hipStream_t)stream;
    double* x = (double*)xv;
    const double* b = (const double*)bv;
    hhg_solve_info loc;
    hhg_solve_info* I = info ? info : &loc;
    std::memset(I, 0, sizeof(*I));
    reset_ops(c);
    const int L = c->L;
    const size_t len = (size_t)c->H[L].len, n4 = 4 * len;
    double* R = c->kv[0];
    double* Vb[2] = {c->kv[1], c->kv[2]};
    double* Zb[2] = {c->kv[3], c->kv[4]};
    double* Q = c->kv[5];
    double* Wb[2] = {c->kv[6], c->kv[7]};
    double* KWb[2] = {c->kv[8], c->kv[9]};
    for (int q = 0; q < KV_N; ++q) fill<double>(c->kv[q], n4, 0.0, s);
    hipEvent_t e0 = next_event(c), e1 = next_event(c);
    if (e0) (void)hipEventRecord(e0, s);
    // r_0 = f~ - K x_0, V_1 = r_0, Z_1 = P^-1 r_0 (unnormalised Lanczos vectors)
    residual_norm<double>(c, L, x, b, R, c->kscal + 2, s);
    hipLaunchKernelGGL(k_copy, dim3(vgrid(n4)), dim3(TPB), 0, s, Vb[1], (const double*)R, n4);
    block_prec(c, nu, Vb[1], Zb[0], c->kscal + 1, s);
    double h[3];
    hhg_status rs = read_scalars(c, h, c->kscal, 3, s);
    if (rs != HHG_OK) return rs;
    const double r0 = h[2];
    I->r0 = r0;
    hist_put(I, 0, r0);
    if (!std::isfinite(r0) || !std::isfinite(h[1])) {
        I->status = HHG_ENAN;
        return fail(c, HHG_ENAN, "initial residual is not finite");
    }
    hhg_status st = HHG_ENOCONV;
    if (r0 == 0.0) st = HHG_OK;
    int cur = 1, zc = 0, wc = 0, it = 0;
    double beta = std::sqrt(std::max(h[1], 0.0)), beta_prev = 0.0;
    double c_old = 1.0, s_old = 0.0, cs = 1.0, sn = 0.0, eta = beta;
    bool pending = false;
    while (st == HHG_ENOCONV && beta > 0.0) {
        if (it >= maxit) break;
        // Lanczos: Q = K Z_j, alpha_j = <Q, Z_j> / beta_j^2, V_{j+1}, Z_{j+1} = P^-1 V_{j+1}
        full_pass<double, MODE_APPLY>(c, L, Zb[zc], nullptr, Q, s);
        vdot(c, Q, Zb[zc], 4, c->kscal + 0, s);
        hipLaunchKernelGGL(k_mr_lanczos, dim3(vgrid(n4)), dim3(TPB), 0, s, (const double*)Q,
                           (const double*)Vb[cur], Vb[cur ^ 1], n4, beta,
                           it == 0 ? 0.0 : beta / beta_prev, (const double*)c->kscal);
        block_prec(c, nu, Vb[cur ^ 1], Zb[zc ^ 1], c->kscal + 1, s);
        if ((rs = read_scalars(c, h, c->kscal, 3, s)) != HHG_OK) return rs;
        if (pending) {
            // residual of the previous update (Q, V and Z do not touch x or r)
            hist_put(I, it, h[2]);
            pending = false;
            if (!std::isfinite(h[2])) {
                st = HHG_ENAN;
                break;
            }
            if (h[2] <= rtol * r0) {
                st = HHG_OK;
                break;
            }
        }
        const double alpha = h[0] / (beta * beta);
        const double beta_new = std::sqrt(std::max(h[1], 0.0));
        // rotations G_{j-2}, G_{j-1} on column j of the tridiagonal matrix,
        // then G_j annihilating beta_{j+1}
        const double eps = s_old * beta, dhat = c_old * beta;
        const double delta = cs * dhat + sn * alpha, ghat = -sn * dhat + cs * alpha;
        const double gamma = std::hypot(ghat, beta_new);
        if (!std::isfinite(gamma)) {
            st = HHG_ENAN;
            break;
        }
        if (gamma == 0.0) break;
        const double c_new = ghat / gamma, s_new = beta_new / gamma;
        const double tau = c_new * eta;
        eta = -s_new * eta;
        MrCoef k{1.0 / (beta * gamma), eps / gamma, delta / gamma, tau};
        hipLaunchKernelGGL(k_mr_update, dim3(vgrid(len)), dim3(TPB), 0, s, (const double*)Zb[zc],
                           Wb[wc], (const double*)Wb[wc ^ 1], x, (const double*)Q, KWb[wc],
                           (const double*)KWb[wc ^ 1], R, (const uint8_t*)c->A[L].owned, len, k,
                           c->kpart);
        vreduce(c, len, c->kscal + 2, true, s);
        pending = true;
        ++it;
        wc ^= 1;
        cur ^= 1;
        zc ^= 1;
        c_old = cs;
        s_old = sn;
        cs = c_new;
        sn = s_new;
        beta_prev = beta;
        beta = beta_new;
    }
    if (pending) {
        if ((rs = read_scalars(c, h, c->kscal + 2, 1, s)) != HHG_OK) return rs;
        hist_put(I, it, h[0]);
        if (!std::isfinite(h[0]))
            st = HHG_ENAN;
        else if (h[0] <= rtol * r0)
            st = HHG_OK;
    }
    project<double>(c, L, x, s);
    if (e1) (void)hipEventRecord(e1, s);
    I->t_solve_ms = event_ms(e0, e1);
    if (I->cycles > 0 && I->rel_res > 0.0) I->rho_mean = std::pow(I->rel_res, 1.0 / I->cycles);
    put_ops(c, I);
    I->status = st;
    c->evused = c->timing ? c->evused : 0;
    LAUNCH_CHECK(c);
    if (st == HHG_ENAN) return fail(c, HHG_ENAN, "residual norm is not finite");
    if (st == HHG_ENOCONV) return fail(c, HHG_ENOCONV, "tolerance not reached");
    return HHG_OK;
}

hhg_status hhg_scg(hhg_ctx* c, void* xv, const void* bv, double rtol, int32_t max_outer,
                   int32_t n_A, int32_t n_S, int32_t n_I, int32_t nu, hhg_solve_info* info,
                   hhg_stream stream) {
    CHECK_DEV(c);
    CHECK_PTR(c, xv);
    CHECK_PTR(c, bv);
    if (xv == bv) return fail(c, HHG_EINVAL, "x and b must not alias");
    if (!c->kv[0]) return fail(c, HHG_EINVAL, "Krylov vectors not reserved (create with krylov = 1)");
    if (!(rtol >= 0.0) || max_outer < 0 || max_outer > 255 || n_A < 1 || n_A > 64 || n_S < 1 ||
        n_S > 64 || n_I < 1 || n_I > 64 || nu < 1 || nu > 16)
        return fail(c, HHG_EINVAL,
                    "need rtol >= 0, 0 <= max_outer <= 255, n_A, n_S, n_I in 1..64, nu in 1..16");
    hipStream_t s = (hipStream_t)stream;
    double* x = (double*)xv;
    const double* b = (const double*)bv;
    hhg_solve_info loc;
    hhg_solve_info* I = info ? info : &loc;
    std::memset(I, 0, sizeof(*I));
    reset_ops(c);
    const int L = c->L;
    const size_t len = (size_t)c->H[L].len, n4 = 4 * len;
    double* T = c->kv[0];              // velocity right-hand sides
    double* DW = c->kv[1];             // w = -Ahat^-1 B^T d (fields 0..2), d (field 3)
    double* Y = c->kv[2];              // field 3: C p - B u, then S d
    double* RHO = c->kv[3];            // Schur residual
    double* ZP = c->kv[3] + len;       // M^-1 rho
    double* D = DW + 3 * len;
    double* Rr = c->A[L].r64;
    const uint8_t* own = c->A[L].owned;
    const double* pinv = c->A[L].pinv;
    for (int q = 0; q < 4; ++q) fill<double>(c->kv[q], n4, 0.0, s);
    hipEvent_t e0 = next_event(c), e1 = next_event(c);
    if (e0) (void)hipEventRecord(e0, s);
    residual_norm<double>(c, L, x, b, Rr, c->kscal + 2, s);
    double h[1];
    hhg_status rs = read_scalars(c, h, c->kscal + 2, 1, s);
    if (rs != HHG_OK) return rs;
    const double r0 = h[0];
    I->r0 = r0;
    hist_put(I, 0, r0);
    if (!std::isfinite(r0)) {
        I->status = HHG_ENAN;
        return fail(c, HHG_ENAN, "initial residual is not finite");
    }
    hhg_status st = r0 == 0.0 ? HHG_OK : HHG_ENOCONV;
    double* rz = c->kscal + 4;         // ping-pong pair rz[0], rz[1]
    double* dy = c->kscal + 6;
    for (int k = 1; k <= max_outer && st == HHG_ENOCONV; ++k) {
        // n_A cycles for A u = f - B^T p from the previous u
        full_pass<double, MODE_RU>(c, L, x, b, T, s);
        mirror_refresh<double>(c, L, x, s);
        for (int q = 0; q < n_A; ++q) vel_cycle<double>(c, L, nu, nu, x, T, s);
        // CG on S p = B A^-1 f - g from p with rho = B u - C p - g
        full_pass<double, MODE_SCHUR>(c, L, x, nullptr, Y, s);
        ops(c, L, 0, 0, 0, 1);
        hipLaunchKernelGGL(k_cg_start, dim3(vgrid(len)), dim3(TPB), 0, s,
                           (const double*)(Y + 3 * len), b + 3 * len, RHO, ZP, D, pinv, own, len,
                           c->kpart);
        vreduce(c, len, rz, false, s);
        int cur = 0;
        for (int i = 0; i < n_S; ++i) {
            // S d = B A^-1 B^T d + C d with A^-1 ~ n_I cycles from zero
            full_pass<double, MODE_BTN>(c, L, DW, nullptr, T, s);
            fill_velocity<double>(c, L, DW, s);
            for (int q = 0; q < n_I; ++q) vel_cycle<double>(c, L, nu, nu, DW, T, s);
            full_pass<double, MODE_SCHUR>(c, L, DW, nullptr, Y, s);
            vdot(c, D, Y + 3 * len, 1, dy, s);
            ops(c, L, 0, 0, 0, 1);
            hipLaunchKernelGGL(k_cg_step, dim3(vgrid(len)), dim3(TPB), 0, s, x + 3 * len,
                               (const double*)D, RHO, (const double*)(Y + 3 * len), ZP, pinv, own,
                               len, (const double*)(rz + cur), (const double*)dy, c->kpart);
            vreduce(c, len, rz + (cur ^ 1), false, s);
            hipLaunchKernelGGL(k_cg_dir, dim3(vgrid(len)), dim3(TPB), 0, s, D, (const double*)ZP,
                               len, (const double*)(rz + (cur ^ 1)), (const double*)(rz + cur));
            cur ^= 1;
        }
        project<double>(c, L, x, s);
        residual_norm<double>(c, L, x, b, Rr, c->kscal + 2, s);
        if ((rs = read_scalars(c, h, c->kscal + 2, 1, s)) != HHG_OK) return rs;
        hist_put(I, k, h[0]);
        if (!std::isfinite(h[0]))
            st = HHG_ENAN;
        else if (h[0] <= rtol * r0)
            st = HHG_OK;
    }
    if (e1) (void)hipEventRecord(e1, s);
    I->t_solve_ms = event_ms(e0, e1);
    if (I->cycles > 0 && I->rel_res > 0.0) I->rho_mean = std::pow(I->rel_res, 1.0 / I->cycles);
    put_ops(c, I);
    I->status = st;
    c->evused = c->timing ? c->evused : 0;
    LAUNCH_CHECK(c);
    if (st == HHG_ENAN) return fail(c, HHG_ENAN, "residual norm is not finite");
    if (st == HHG_ENOCONV) return fail(c, HHG_ENOCONV, "tolerance not reached");
    return HHG_OK;
}

}  // extern "C"
