"""MI355X Uzawa-multigrid Stokes solver: Python binding of the C ABI (hhg.h).

Argument marshalling only: every step of the solver runs in the HIP kernels of
libhhg.so.  PyTorch provides device memory and the current stream.  Importing
this package fails if libhhg.so has not been built (there is no CPU fallback):

    python paper_1511_02134_amd/build.py
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch ships its own HIP runtime under the same soname as the system one;
# loading it first makes libhhg.so bind to that single runtime (two runtimes
# in one process do not see the device).
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhhg.so")

HHG_OK, HHG_EINVAL, HHG_ENOMEM, HHG_EDEVICE, HHG_ENOCONV, HHG_ENAN = range(6)
K_VEL, K_PRES, K_APPLY, K_RU = 0, 1, 2, 3
STATUS_NAMES = {0: "HHG_OK", 1: "HHG_EINVAL", 2: "HHG_ENOMEM", 3: "HHG_EDEVICE",
                4: "HHG_ENOCONV", 5: "HHG_ENAN"}


class HHGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Mesh(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int32), ("xyz", ctypes.POINTER(ctypes.c_double)),
                ("nt", ctypes.c_int32), ("tet", ctypes.POINTER(ctypes.c_int32)),
                ("nu", ctypes.POINTER(ctypes.c_double)),
                ("face_bc", ctypes.POINTER(ctypes.c_int8)),
                ("phys", ctypes.POINTER(ctypes.c_double))]


class Opts(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32), ("cycle", ctypes.c_int32),
                ("p_sweep", ctypes.c_int32), ("omega", ctypes.c_double),
                ("precision", ctypes.c_int32), ("coarse_rtol", ctypes.c_double),
                ("coarse_maxit", ctypes.c_int32), ("block_order", ctypes.c_int32),
                ("coarse_prec", ctypes.c_int32), ("coarse_solver", ctypes.c_int32),
                ("krylov", ctypes.c_int32), ("graphs", ctypes.c_int32), ("op", ctypes.c_int32),
                ("ordering", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("status", ctypes.c_int32), ("r0", ctypes.c_double),
                ("r_final", ctypes.c_double), ("rel_res", ctypes.c_double),
                ("rho_mean", ctypes.c_double), ("rho_max", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("res_hist", ctypes.c_double * 256),
                ("n_op", ctypes.c_double * 4), ("t_smooth_ms", ctypes.c_double),
                ("t_transfer_ms", ctypes.c_double), ("t_coarse_ms", ctypes.c_double),
                ("t_residual_ms", ctypes.c_double), ("t_level_ms", ctypes.c_double * 16)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with "
                          "`python paper_1511_02134_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    S = ctypes.c_int
    sig = {
        "hhg_default_opts": (None, [ctypes.POINTER(Opts)]),
        "hhg_plan": (S, [ctypes.POINTER(Mesh), I32, ctypes.POINTER(Opts),
                         ctypes.POINTER(ctypes.c_size_t)]),
        "hhg_create": (S, [ctypes.POINTER(Mesh), I32, ctypes.POINTER(Opts), P, ctypes.c_size_t,
                           ctypes.POINTER(P)]),
        "hhg_destroy": (None, [P]),
        "hhg_last_error": (ctypes.c_char_p, [P]),
        "hhg_global_error": (ctypes.c_char_p, []),
        "hhg_num_levels": (I32, [P]),
        "hhg_vec_len": (I64, [P, I32]),
        "hhg_num_nodes": (I64, [P, I32]),
        "hhg_num_dofs": (I64, [P, I32]),
        "hhg_num_interface": (I64, [P, I32]),
        "hhg_node_info": (S, [P, I32, P, P]),
        "hhg_check_layout": (S, [P]),
        "hhg_mass_weights": (S, [P, I32, P]),
        "hhg_primitive_classes": (S, [P, I32, P]),
        "hhg_scatter": (S, [P, I32, P, I32, P, P]),
        "hhg_gather": (S, [P, I32, P, I32, P, P]),
        "hhg_exchange": (S, [P, I32, P, I32, P]),
        "hhg_rhs": (S, [P, P, P, P]),
        "hhg_rhs_level": (S, [P, I32, P, P, P]),
        "hhg_fmg": (S, [P, P, P, I32, P]),
        "hhg_apply": (S, [P, I32, P, P, P]),
        "hhg_residual": (S, [P, I32, P, P, P, ctypes.POINTER(D), P]),
        "hhg_residual_noalloc": (S, [P, I32, P, P, P, P, P]),
        "hhg_smooth": (S, [P, I32, P, P, I32, P]),
        "hhg_restrict": (S, [P, I32, P, P, P]),
        "hhg_prolong_add": (S, [P, I32, P, P, P]),
        "hhg_coarse_solve": (S, [P, P, P, ctypes.POINTER(I32), ctypes.POINTER(D), P]),
        "hhg_project": (S, [P, I32, P, P]),
        "hhg_vcycle": (S, [P, P, P, P]),
        "hhg_solve": (S, [P, P, P, D, I32, ctypes.POINTER(SolveInfo), P]),
        "hhg_vel_cycle": (S, [P, I32, I32, P, P, P]),
        "hhg_pminres": (S, [P, P, P, D, I32, I32, ctypes.POINTER(SolveInfo), P]),
        "hhg_scg": (S, [P, P, P, D, I32, I32, I32, I32, I32, ctypes.POINTER(SolveInfo), P]),
        "hhg_grad": (S, [P, P, P, P, P, P, P]),
        "hhg_adjoint_rhs": (S, [P, P, P, P]),
        "hhg_set_phase_timing": (S, [P, I32]),
        "hhg_set_viscosity": (S, [P, P]),
        "hhg_set_timing": (S, [P, I32]),
        "hhg_kernel_time": (S, [P, I32, ctypes.POINTER(I64), ctypes.POINTER(D),
                                ctypes.POINTER(D)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()

# exported symbols declared in include/hhg.h (checked by the CPU tests)
ABI_FUNCTIONS = ("hhg_default_opts", "hhg_plan", "hhg_create", "hhg_destroy", "hhg_last_error",
                 "hhg_global_error", "hhg_num_levels", "hhg_vec_len", "hhg_num_nodes",
                 "hhg_num_dofs", "hhg_num_interface", "hhg_node_info", "hhg_mass_weights",
                 "hhg_primitive_classes", "hhg_check_layout", "hhg_scatter",
                 "hhg_gather", "hhg_exchange", "hhg_rhs", "hhg_rhs_level", "hhg_fmg",
                 "hhg_apply", "hhg_residual", "hhg_residual_noalloc",
                 "hhg_smooth", "hhg_restrict", "hhg_prolong_add", "hhg_coarse_solve",
                 "hhg_project", "hhg_vcycle", "hhg_solve", "hhg_vel_cycle", "hhg_pminres",
                 "hhg_scg", "hhg_grad", "hhg_adjoint_rhs", "hhg_set_viscosity",
                 "hhg_set_timing", "hhg_set_phase_timing", "hhg_kernel_time")


def default_opts(**kw) -> Opts:
    o = Opts()
    lib.hhg_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class _MeshArrays:
    """Keeps the host arrays of a Mesh struct alive."""

    def __init__(self, xyz, tet, nu, face_bc, phys=None):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tet = np.ascontiguousarray(tet, dtype=np.int32)
        self.nu = None if nu is None else np.ascontiguousarray(nu, dtype=np.float64)
        self.face_bc = np.ascontiguousarray(face_bc, dtype=np.int8)
        self.phys = None if phys is None else np.ascontiguousarray(phys, dtype=np.float64)
        m = Mesh()
        m.nv = self.xyz.shape[0]
        m.xyz = self.xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        m.nt = self.tet.shape[0]
        m.tet = self.tet.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        m.nu = (self.nu.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                if self.nu is not None else ctypes.POINTER(ctypes.c_double)())
        m.face_bc = self.face_bc.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
        m.phys = (self.phys.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                  if self.phys is not None else ctypes.POINTER(ctypes.c_double)())
        self.struct = m


def _check(status, ctx=None):
    if status != HHG_OK:
        msg = (lib.hhg_last_error(ctx) if ctx else lib.hhg_global_error()) or b""
        raise HHGError(status, msg.decode())


def plan(xyz, tet, nu, face_bc, R, phys=None, **opts) -> int:
    """Workspace bytes for the mesh (host only, validates the inputs)."""
    m = _MeshArrays(xyz, tet, nu, face_bc, phys)
    o = default_opts(**opts)
    nbytes = ctypes.c_size_t(0)
    _check(lib.hhg_plan(ctypes.byref(m.struct), R, ctypes.byref(o), ctypes.byref(nbytes)))
    return nbytes.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Solver:
    """Hierarchy, stencils and work space of one macro mesh refined R times."""

    def __init__(self, xyz, tet, nu, face_bc, R, device="cuda", host_only=False, phys=None,
                 **opts):
        self._mesh = _MeshArrays(xyz, tet, nu, face_bc, phys)
        self.opts = default_opts(**opts)
        self.R = R
        self.nt = self._mesh.tet.shape[0]
        self.ctx = ctypes.c_void_p()
        self.ws = None
        if host_only:
            _check(lib.hhg_create(ctypes.byref(self._mesh.struct), R, ctypes.byref(self.opts),
                                  None, 0, ctypes.byref(self.ctx)))
        else:
            import torch
            nbytes = ctypes.c_size_t(0)
            _check(lib.hhg_plan(ctypes.byref(self._mesh.struct), R, ctypes.byref(self.opts),
                                ctypes.byref(nbytes)))
            self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
            _check(lib.hhg_create(ctypes.byref(self._mesh.struct), R, ctypes.byref(self.opts),
                                  _ptr(self.ws), nbytes.value, ctypes.byref(self.ctx)))
        self.levels = lib.hhg_num_levels(self.ctx)
        self.L = self.levels - 1
        self.device = device

    def __del__(self):
        try:
            if getattr(self, "ctx", None) and lib is not None:
                lib.hhg_destroy(self.ctx)
                self.ctx = None
        except Exception:   # interpreter shutdown
            pass

    # -- sizes -------------------------------------------------------------
    def vec_len(self, level=None):
        return lib.hhg_vec_len(self.ctx, self.L if level is None else level)

    def num_nodes(self, level=None):
        return lib.hhg_num_nodes(self.ctx, self.L if level is None else level)

    def num_dofs(self, level=None):
        return lib.hhg_num_dofs(self.ctx, self.L if level is None else level)

    def num_interface(self, level=None):
        return lib.hhg_num_interface(self.ctx, self.L if level is None else level)

    def node_flags(self, level=None):
        """Lattice coordinates [N,3] and boundary flags [N] (1 Dirichlet, 2
        free-slip, 0 otherwise)."""
        level = self.L if level is None else level
        N = self.num_nodes(level)
        ijk = np.zeros((N, 3), dtype=np.int32)
        d = np.zeros(N, dtype=np.int8)
        _check(lib.hhg_node_info(self.ctx, level, ijk.ctypes.data_as(ctypes.c_void_p),
                                 d.ctypes.data_as(ctypes.c_void_p)), self.ctx)
        return ijk, d

    def node_info(self, level=None):
        """Lattice coordinates [N,3] and the velocity Dirichlet mask [N]."""
        ijk, d = self.node_flags(level)
        return ijk, d == 1

    def mass_weights(self, level=None):
        level = self.L if level is None else level
        m = np.zeros(self.num_nodes(level))
        _check(lib.hhg_mass_weights(self.ctx, level, m.ctypes.data_as(ctypes.c_void_p)), self.ctx)
        return m

    def primitive_classes(self, level=None):
        """HHG primitive class of every lattice point (0 macro vertex, 1 edge,
        2 face, 3 volume, -1 hole)."""
        level = self.L if level is None else level
        cls = np.zeros(self.num_nodes(level), dtype=np.int8)
        _check(lib.hhg_primitive_classes(self.ctx, level, cls.ctypes.data_as(ctypes.c_void_p)),
               self.ctx)
        return cls

    def check_layout(self):
        """Host-side verification of every index the kernels compute."""
        _check(lib.hhg_check_layout(self.ctx), self.ctx)

    # -- vectors -------------------------------------------------------------
    def vector(self, level=None, nfields=4):
        import torch
        return torch.zeros(nfields, self.vec_len(level), dtype=torch.float64, device=self.device)

    def scatter(self, nodal, level=None):
        level = self.L if level is None else level
        nodal = nodal.contiguous()
        nf = nodal.shape[0]
        x = self.vector(level, nf)
        _check(lib.hhg_scatter(self.ctx, level, _ptr(nodal), nf, _ptr(x), _stream()), self.ctx)
        return x

    def gather(self, x, level=None):
        import torch
        level = self.L if level is None else level
        nf = x.shape[0]
        out = torch.empty(nf, self.num_nodes(level), dtype=torch.float64, device=self.device)
        _check(lib.hhg_gather(self.ctx, level, _ptr(x), nf, _ptr(out), _stream()), self.ctx)
        return out

    def exchange(self, x, level=None):
        level = self.L if level is None else level
        _check(lib.hhg_exchange(self.ctx, level, _ptr(x), x.shape[0], _stream()), self.ctx)

    # -- operators -------------------------------------------------------------
    def rhs(self, f_internal):
        b = self.vector()
        _check(lib.hhg_rhs(self.ctx, _ptr(f_internal), _ptr(b), _stream()), self.ctx)
        return b

    def rhs_level(self, f_internal, level):
        """Right-hand side on `level` from the forcing at that level's vertices."""
        b = self.vector(level)
        _check(lib.hhg_rhs_level(self.ctx, level, _ptr(f_internal), _ptr(b), _stream()), self.ctx)
        return b

    def fmg(self, xs, bs, cycles=1):
        """Full multigrid over per-level iterates xs[l] (holding the level's
        Dirichlet values) and right-hand sides bs[l]; xs[-1] is the result."""
        n = self.L + 1
        if len(xs) != n or len(bs) != n:
            raise ValueError(f"need {n} iterates and right-hand sides")
        px = (ctypes.c_void_p * n)(*[_ptr(x) for x in xs])
        pb = (ctypes.c_void_p * n)(*[_ptr(b) for b in bs])
        _check(lib.hhg_fmg(self.ctx, px, pb, cycles, _stream()), self.ctx)

    def apply(self, x, level=None, out=None):
        level = self.L if level is None else level
        y = self.vector(level) if out is None else out
        _check(lib.hhg_apply(self.ctx, level, _ptr(x), _ptr(y), _stream()), self.ctx)
        return y

    def residual(self, x, b, level=None, norm=True):
        level = self.L if level is None else level
        r = self.vector(level)
        nrm = ctypes.c_double(0.0)
        _check(lib.hhg_residual(self.ctx, level, _ptr(x), _ptr(b), _ptr(r),
                                ctypes.byref(nrm) if norm else None, _stream()), self.ctx)
        return r, nrm.value

    def residual_noalloc(self, x, b, r, norm, level=None):
        """r = b - K x and ||r||_2 into the device scalar `norm` (a float64
        tensor of one element); allocates nothing (static library scratch)."""
        level = self.L if level is None else level
        _check(lib.hhg_residual_noalloc(self.ctx, level, _ptr(x), _ptr(b), _ptr(r), _ptr(norm),
                                        _stream()), self.ctx)

    def smooth(self, x, b, steps=1, level=None):
        level = self.L if level is None else level
        _check(lib.hhg_smooth(self.ctx, level, _ptr(x), _ptr(b), steps, _stream()), self.ctx)

    def restrict(self, r, level=None):
        level = self.L if level is None else level
        bc = self.vector(level - 1)
        _check(lib.hhg_restrict(self.ctx, level, _ptr(r), _ptr(bc), _stream()), self.ctx)
        return bc

    def prolong_add(self, e, x, level=None):
        level = self.L if level is None else level
        _check(lib.hhg_prolong_add(self.ctx, level, _ptr(e), _ptr(x), _stream()), self.ctx)

    def coarse_solve(self, b0):
        x0 = self.vector(0)
        it = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        _check(lib.hhg_coarse_solve(self.ctx, _ptr(b0), _ptr(x0), ctypes.byref(it),
                                    ctypes.byref(rel), _stream()), self.ctx)
        return x0, it.value, rel.value

    def project(self, x, level=None):
        level = self.L if level is None else level
        _check(lib.hhg_project(self.ctx, level, _ptr(x), _stream()), self.ctx)

    def vcycle(self, x, b):
        _check(lib.hhg_vcycle(self.ctx, _ptr(x), _ptr(b), _stream()), self.ctx)

    def _info(self, st, info, raise_on_noconv):
        if st not in (HHG_OK, HHG_ENOCONV) or (st == HHG_ENOCONV and raise_on_noconv):
            _check(st, self.ctx)
        k = info.cycles
        return {"status": st, "cycles": k, "r0": info.r0, "r_final": info.r_final,
                "rel_res": info.rel_res, "rho_mean": info.rho_mean, "rho_max": info.rho_max,
                "t_solve_ms": info.t_solve_ms, "res_hist": list(info.res_hist[:min(k, 255) + 1]),
                "n_op": dict(zip("ABCM", list(info.n_op))),
                "t_phase_ms": {"smooth": info.t_smooth_ms, "transfer": info.t_transfer_ms,
                               "coarse": info.t_coarse_ms, "residual": info.t_residual_ms},
                "t_level_ms": list(info.t_level_ms[:self.L + 1])}

    def solve(self, x, b, rtol=1e-8, max_cycles=100, raise_on_noconv=False):
        info = SolveInfo()
        st = lib.hhg_solve(self.ctx, _ptr(x), _ptr(b), rtol, max_cycles, ctypes.byref(info),
                           _stream())
        return self._info(st, info, raise_on_noconv)

    def vel_cycle(self, x, b, nu1=1, nu2=1):
        """One velocity V(nu1, nu2) cycle for A u = b on fields 0..2 of x."""
        _check(lib.hhg_vel_cycle(self.ctx, nu1, nu2, _ptr(x), _ptr(b), _stream()), self.ctx)

    def pminres(self, x, b, rtol=1e-8, maxit=1000, nu=1, raise_on_noconv=False):
        """Block-diagonal preconditioned MINRES (needs krylov=1 at creation);
        rtol=0 runs exactly maxit iterations."""
        info = SolveInfo()
        st = lib.hhg_pminres(self.ctx, _ptr(x), _ptr(b), rtol, maxit, nu, ctypes.byref(info),
                             _stream())
        return self._info(st, info, raise_on_noconv)

    def scg(self, x, b, rtol=1e-8, max_outer=200, n_A=3, n_S=3, n_I=1, nu=3,
            raise_on_noconv=False):
        """Schur-complement CG, Algorithm 1 (needs krylov=1 at creation);
        rtol=0 runs exactly max_outer outer iterations."""
        info = SolveInfo()
        st = lib.hhg_scg(self.ctx, _ptr(x), _ptr(b), rtol, max_outer, n_A, n_S, n_I, nu,
                         ctypes.byref(info), _stream())
        return self._info(st, info, raise_on_noconv)

    def grad(self, x, lam, f=None, want_df=True):
        import torch
        dnu = torch.zeros(self.nt, dtype=torch.float64, device=self.device)
        df = self.vector(nfields=3) if want_df else None
        _check(lib.hhg_grad(self.ctx, _ptr(x), _ptr(lam), _ptr(f), _ptr(dnu), _ptr(df),
                            _stream()), self.ctx)
        return dnu, df

    def adjoint_rhs(self, g):
        """(dJ/du with Dirichlet rows zeroed, Pi^T dJ/dp) from g (4 fields,
        internal layout of the finest level)."""
        y = self.vector()
        _check(lib.hhg_adjoint_rhs(self.ctx, _ptr(g), _ptr(y), _stream()), self.ctx)
        return y

    def set_viscosity(self, nu):
        nu = np.ascontiguousarray(nu, dtype=np.float64)
        self._nu_keep = nu
        _check(lib.hhg_set_viscosity(self.ctx, nu.ctypes.data_as(ctypes.c_void_p)), self.ctx)

    def set_timing(self, on=True):
        _check(lib.hhg_set_timing(self.ctx, int(on)), self.ctx)

    def set_phase_timing(self, on=True):
        _check(lib.hhg_set_phase_timing(self.ctx, int(on)), self.ctx)

    def kernel_time(self, cls):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        by = ctypes.c_double(0.0)
        _check(lib.hhg_kernel_time(self.ctx, cls, ctypes.byref(n), ctypes.byref(ms),
                                   ctypes.byref(by)), self.ctx)
        return n.value, ms.value, by.value


def solver_for(workload, R=None, device="cuda", **opts):
    """Solver for a workloads.Workload (the shared input generator)."""
    xyz, tet, nu, tags = workload.mesh()
    if "precision" not in opts:
        opts["precision"] = 1 if workload.precision == "mixed" else 0
    return Solver(xyz, tet, nu, tags, workload.R if R is None else R, device=device,
                  phys=workload.physical(), **opts)
