"""GPU: mixed-precision iterative refinement and the adjoint gradients
(hhg_grad behind torch.autograd) against the oracle and finite differences."""
import numpy as np
import pytest

import workloads as W
from oracle import UMG, build_hierarchy
from oracle.adjoint import adjoint_rhs, grad_forcing, grad_viscosity, loss
from oracle.umg import direct_solve

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("cid,R", [(1, 4), (1, 5), (5, 4), (4, 4)])
def test_mixed_precision_solve_reaches_fp64_tolerance(cid, R):
    """FP32 cycles inside FP64 refinement: ||f~ - K x|| <= 1e-8 ||f~ - K x0||
    with K the oracle's FP64 operator; the error against the oracle's FP64
    solution (h-norm of the paper's TME section, h = 2^-R) is reported."""
    import paper_1511_02134_amd as P
    cfg = W.WORKLOADS[cid].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    _announce(f"mixed config {cid} R={R}")
    s = P.Solver(xyz, tet, nu, tags, R, precision=1)
    umg = UMG(build_hierarchy(xyz, tet, nu, tags, R))
    lv = umg.H.finest
    bo = umg.rhs(cfg.forcing_field())
    x0 = np.zeros((4, lv.N))
    x0[:3] = cfg.dirichlet_field()
    x0[:3, lv.free] = 0.0
    xd = s.scatter(_dev(x0))
    info = s.solve(xd, s.scatter(_dev(bo)), rtol=1e-8, max_cycles=60)
    assert info["status"] == 0, info
    xm = s.gather(xd).cpu().numpy()
    r0 = umg.norm(umg.L, umg.residual(umg.L, x0, bo))
    assert umg.norm(umg.L, umg.residual(umg.L, xm, bo)) <= 1e-8 * r0
    xo, hist = umg.solve(x0.copy(), bo, rtol=1e-8)
    h = 1.0 / lv.n
    hn = lambda y: np.sqrt(np.sum(y[:3] ** 2) + h * h * np.sum(y[3] ** 2))
    err = hn(xm - xo) / hn(xo)
    print(f"mixed cycles {info['cycles']} vs fp64 {len(hist) - 1}, h-norm rel. error {err:.2e}")
    assert err < 1e-6
    assert info["cycles"] <= len(hist) - 1 + 3


def _problem(cid, R, rtol, precision=0, op="laplace"):
    import paper_1511_02134_amd as P
    from paper_1511_02134_amd.autograd import StokesProblem
    cfg = W.WORKLOADS[cid].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    s = P.Solver(xyz, tet, nu, tags, R, precision=precision, op=1 if op == "D" else 0)
    return cfg, nu, StokesProblem(s, cfg.dirichlet_field(), rtol=rtol, max_cycles=100)


@pytest.mark.parametrize("cid,R,op", [(4, 3, "laplace"), (5, 3, "laplace"), (4, 4, "laplace"),
                                     (4, 3, "D"), (5, 3, "D")])
def test_adjoint_gradient_matches_oracle(cid, R, op):
    from paper_1511_02134_amd.autograd import StokesSolve
    _announce(f"adjoint config {cid} R={R} form={op}")
    cfg, nu, prob = _problem(cid, R, rtol=1e-12, op=op)
    f = cfg.forcing_field() + W.nodal_noise(cfg.points().shape[0], 11, 0.3)
    nu_obs = cfg.observation_viscosity()
    ft = _dev(f)
    with torch.no_grad():
        u_obs, _ = StokesSolve.apply(ft, _dev(nu_obs), prob)
    ft.requires_grad_(True)
    nut = _dev(nu).requires_grad_(True)
    u, p = StokesSolve.apply(ft, nut, prob)
    J = 0.5 * ((u - u_obs) ** 2).sum()
    J.backward()
    # oracle: direct solves on the same inputs
    xyz, tet, _, tags = cfg.mesh()
    Ho = build_hierarchy(xyz, tet, nu, tags, R, R0=R, op=op)
    lv = Ho.finest
    b = np.zeros((4, lv.N))
    for k in range(3):
        b[k] = lv.M @ f[k]
        b[k][lv.dirichlet] = 0.0
    b[3] = sum(lv.Gf[k] @ f[k] for k in range(3))
    x0 = np.zeros((4, lv.N))
    x0[:3] = cfg.dirichlet_field()
    x0[:3, lv.free] = 0.0
    x = direct_solve(lv, b, Ho.project, xbc=x0)
    Hobs = build_hierarchy(xyz, tet, nu_obs, tags, R, R0=R, op=op)
    bo = b.copy()
    lvo = Hobs.finest
    for k in range(3):
        bo[k] = lvo.M @ f[k]
        bo[k][lvo.dirichlet] = 0.0
    bo[3] = sum(lvo.Gf[k] @ f[k] for k in range(3))
    uo = direct_solve(lvo, bo, Hobs.project, xbc=x0)[:3]
    lam = direct_solve(lv, adjoint_rhs(lv, x[:3], uo), Ho.project)
    gf = grad_forcing(lv, lam)
    gnu = grad_viscosity(lv, x, lam, f, nu, op)
    assert J.item() == pytest.approx(loss(x[:3], uo), rel=1e-8)
    gf_gpu = ft.grad.cpu().numpy()
    gnu_gpu = nut.grad.cpu().numpy()
    assert np.abs(gf_gpu - gf).max() <= 1e-8 * np.abs(gf).max()
    assert np.abs(gnu_gpu - gnu).max() <= 1e-8 * np.abs(gnu).max()


@pytest.mark.parametrize("cid,R,precision,op", [(4, 4, 0, "laplace"), (5, 4, 1, "laplace"),
                                                (4, 6, 0, "laplace"), (5, 7, 1, "laplace"),
                                                (4, 4, 0, "D")])
def test_adjoint_gradient_matches_finite_differences(cid, R, precision, op):
    """Central differences with eps = 1e-6 per macro viscosity, forward solves
    driven to rtol 1e-13 (1e-12 with FP32 cycles); gradients within 1e-6.
    The last two cases are the full box (R = 6, FP64) and the full channel
    (R = 7, FP32 cycles in FP64 refinement) in the solver's default launch
    configuration."""
    from paper_1511_02134_amd.autograd import StokesSolve
    _announce(f"finite differences config {cid} R={R} precision={precision} form={op}")
    rtol = 1e-13 if precision == 0 else 1e-12
    cfg, nu, prob = _problem(cid, R, rtol=rtol, precision=precision, op=op)
    f = _dev(cfg.forcing_field() + W.nodal_noise(cfg.points().shape[0], 12, 0.3))
    with torch.no_grad():
        u_obs, _ = StokesSolve.apply(f, _dev(cfg.observation_viscosity()), prob)

    def J(nu_np):
        with torch.no_grad():
            u, _ = StokesSolve.apply(f, _dev(nu_np), prob)
        return 0.5 * ((u - u_obs) ** 2).sum().item()

    nut = _dev(nu).requires_grad_(True)
    fg = f.clone().requires_grad_(True)
    u, p = StokesSolve.apply(fg, nut, prob)
    (0.5 * ((u - u_obs) ** 2).sum()).backward()
    g = nut.grad.cpu().numpy()
    rng = np.random.default_rng(0)
    eps = 1e-6
    for e in rng.choice(nu.shape[0], size=4, replace=False):
        dn = np.zeros_like(nu)
        dn[e] = eps
        fd = (J(nu + dn) - J(nu - dn)) / (2 * eps)
        assert abs(g[e] - fd) <= 1e-6 * np.abs(g).max(), (e, g[e], fd)
    # J is quadratic in f: central differences along random directions
    d = _dev(rng.normal(size=(3, cfg.points().shape[0])))
    eps = 1.0
    def Jf(ff):
        with torch.no_grad():
            uu, _ = StokesSolve.apply(ff, _dev(nu), prob)
        return 0.5 * ((uu - u_obs) ** 2).sum().item()
    fd = (Jf(f + eps * d) - Jf(f - eps * d)) / (2 * eps)
    assert (fg.grad * d).sum().item() == pytest.approx(fd, rel=1e-6)


@pytest.mark.parametrize("cid", [4, 5])
def test_backward_after_another_forward(cid):
    """The observation is solved after the forward solve whose gradient is
    taken (so the problem holds another viscosity when backward runs), and
    the loss observes the pressure too: J = 1/2 ||u - u_obs||^2 +
    1/2 ||p - p_obs||^2.  The gradients equal the oracle's direct-solve
    gradients, whose adjoint right-hand side carries Pi^T (p - p_obs) when
    the pressure has a null space (box) and p - p_obs when it has none
    (channel)."""
    from oracle.adjoint import adjoint_rhs_general
    from paper_1511_02134_amd.autograd import StokesSolve
    R = 3
    _announce(f"backward after another forward, config {cid} R={R}")
    cfg, nu, prob = _problem(cid, R, rtol=1e-12)
    f = cfg.forcing_field() + W.nodal_noise(cfg.points().shape[0], 13, 0.3)
    nu_obs = cfg.observation_viscosity()
    ft = _dev(f).requires_grad_(True)
    nut = _dev(nu).requires_grad_(True)
    u, p = StokesSolve.apply(ft, nut, prob)
    with torch.no_grad():
        u_obs, p_obs = StokesSolve.apply(_dev(f), _dev(nu_obs), prob)
    J = 0.5 * ((u - u_obs) ** 2).sum() + 0.5 * ((p - p_obs) ** 2).sum()
    J.backward()
    xyz, tet, _, tags = cfg.mesh()
    x0 = np.zeros((4, cfg.points().shape[0]))
    x0[:3] = cfg.dirichlet_field()

    def solve(nu_):
        H = build_hierarchy(xyz, tet, nu_, tags, R, R0=R)
        lv = H.finest
        b = np.zeros((4, lv.N))
        for k in range(3):
            b[k] = lv.M @ f[k]
            b[k][lv.dirichlet] = 0.0
        b[3] = sum(lv.Gf[k] @ f[k] for k in range(3))
        xb = x0.copy()
        xb[:3, lv.free] = 0.0
        return H, direct_solve(lv, b, H.project, xbc=xb)

    H, x = solve(nu)
    _, xo = solve(nu_obs)
    lv = H.finest
    lam = direct_solve(lv, adjoint_rhs_general(lv, x[:3] - xo[:3], x[3] - xo[3], H.project),
                       H.project)
    gf = grad_forcing(lv, lam)
    gnu = grad_viscosity(lv, x, lam, f, nu)
    e_f = np.abs(ft.grad.cpu().numpy() - gf).max() / np.abs(gf).max()
    e_nu = np.abs(nut.grad.cpu().numpy() - gnu).max() / np.abs(gnu).max()
    _announce(f"dJ/df rel. difference {e_f:.2e}, dJ/dnu {e_nu:.2e}")
    assert e_f <= 1e-8
    assert e_nu <= 1e-8
