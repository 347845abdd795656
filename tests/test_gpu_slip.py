"""GPU parity of free-slip boundaries (face tag 3, Section 6.1): u . n = 0 at
the vertices of free-slip faces with the mass-conservative normals
n_i = -(B^T 1)_i / |.| held in the interface stencil records.  Compared with
the oracle (pinned against component-wise Dirichlet conditions on flat slip
planes) on the unit cube with free-slip planes z = 0, 1 and on the spherical
shell with free-slip on the inner sphere or on both (15-tap stencils): K x, the right-hand
side and the residual, the transfers, Uzawa steps, the level-0 solve
(Q K Q + a (I - Q) inverted on the device against the oracle's tangential
basis), cycles and solves; discrete mass conservation and the vanishing
normal velocity at full size."""
import numpy as np
import pytest

import workloads as W
from oracle import UMG, build_hierarchy
from oracle.fem import FACE_SLIP, project_slip

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _cube_mesh(R):
    cfg = W.WORKLOADS[1].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    tags = tags.copy()
    for t in range(tet.shape[0]):
        for f in range(4):
            z = xyz[np.delete(tet[t], f), 2]
            if tags[t, f] != 0 and (np.all(z == 0) or np.all(z == 1)):
                tags[t, f] = FACE_SLIP
    return cfg, (xyz, tet, nu, tags), None


def _shell_mesh(R, slip="inner"):
    cfg = W.WORKLOADS[9].with_slip(slip).with_R(R)
    return cfg, cfg.mesh(), cfg.physical()


class Case:
    def __init__(self, kind, R, **opts):
        import paper_1511_02134_amd as P
        if kind == "cube":
            self.cfg, self.mesh, self.phys = _cube_mesh(R)
        else:
            self.cfg, self.mesh, self.phys = _shell_mesh(R, "both" if kind == "shell-both" else "inner")
        xyz, tet, nu, tags = self.mesh
        _announce(f"free-slip {kind} R={R} opts={opts}")
        self.s = P.Solver(xyz, tet, nu, tags, R, phys=self.phys, **opts)
        H = build_hierarchy(xyz, tet, nu, tags, R, phys=self.phys)
        self.umg = UMG(H, nu1=self.s.opts.nu1, nu2=self.s.opts.nu2,
                       variable=bool(self.s.opts.cycle))

    def put(self, x, l=None):
        l = self.umg.L if l is None else l
        lv = self.umg.H.levels[l]
        out = np.zeros((x.shape[0], self.s.num_nodes(l)))
        out[:, lv.lat] = x
        return self.s.scatter(_dev(out), l)

    def get(self, xd, l=None):
        l = self.umg.L if l is None else l
        return _host(self.s.gather(xd, l))[:, self.umg.H.levels[l].lat]


def _state(lv, seed):
    """Random state in the constrained space (Dirichlet velocity 0, normal
    velocity 0 at slip vertices)."""
    x = np.random.default_rng(seed).normal(size=(4, lv.N))
    x[:3, lv.dirichlet] = 0.0
    return project_slip(lv, x)


@pytest.fixture(scope="module", params=["cube", "shell", "shell-both"])
def case(request):
    return Case(request.param, 4)


def test_slip_operators_match_oracle(case):
    """K x (on an unconstrained x as well: the rows are projected), the
    right-hand side, the residual and its norm, and the transfers."""
    cs = case
    umg = cs.umg
    for l, lv in enumerate(umg.H.levels):
        x = np.random.default_rng(20 + l).normal(size=(4, lv.N))
        y = cs.get(cs.s.apply(cs.put(x, l), l), l)
        err = _relerr(y, umg.apply(l, x))
        _announce(f"K x level {l}: {err:.2e}")
        assert err < 1e-13, l
    lv = umg.H.finest
    f = np.random.default_rng(4).normal(size=(3, lv.N))
    bo = umg.rhs(f)
    assert _relerr(cs.get(cs.s.rhs(cs.put(f))), bo) < 1e-13
    x = _state(lv, 5)
    r, nrm = cs.s.residual(cs.put(x), cs.put(bo))
    ro = umg.residual(umg.L, x, bo)
    assert _relerr(cs.get(r), ro) < 1e-13
    assert nrm == pytest.approx(umg.norm(umg.L, ro), rel=1e-13)
    for l in range(1, umg.L + 1):
        lf, lc = umg.H.levels[l], umg.H.levels[l - 1]
        rr = np.random.default_rng(30 + l).normal(size=(4, lf.N))
        rr[:3, lf.dirichlet] = 0.0
        bc = cs.get(cs.s.restrict(cs.put(rr, l), l), l - 1)
        assert _relerr(bc, umg.restrict(l, rr)) < 1e-14
        e = _state(lc, 40 + l)
        xx = _state(lf, 50 + l)
        xd = cs.put(xx, l)
        cs.s.prolong_add(cs.put(e, l - 1), xd, l)
        assert _relerr(cs.get(xd, l), xx + umg.prolong(l, e)) < 1e-14


def test_slip_smoother_and_coarse_solve_match_oracle(case):
    cs = case
    umg = cs.umg
    for l in (0, 1, umg.L):
        lv = umg.H.levels[l]
        x = _state(lv, 60 + l)
        b = np.random.default_rng(70 + l).normal(size=(4, lv.N))
        b[:3, lv.dirichlet] = 0.0
        project_slip(lv, b)
        xd, bd = cs.put(x, l), cs.put(b, l)
        cs.s.smooth(xd, bd, 2, l)
        xo = x.copy()
        for _ in range(2):
            umg.uzawa(l, xo, b)
        err = _relerr(cs.get(xd, l), xo)
        _announce(f"Uzawa steps level {l}: {err:.2e}")
        assert err < 1e-12, l
    lv = umg.H.levels[0]
    b = umg.apply(0, _state(lv, 80))
    xg, it, rel = cs.s.coarse_solve(cs.put(b, 0))
    err = _relerr(cs.get(xg, 0), umg.coarse_solve(b))
    _announce(f"level-0 solve: {err:.2e}")
    assert it == 1 and err < 1e-10


def test_slip_cycles_and_solve_match_oracle(case):
    cs = case
    umg = cs.umg
    lv = umg.H.finest
    f = np.random.default_rng(9).normal(size=(3, lv.N))
    bo = umg.rhs(f)
    x0 = np.zeros((4, lv.N))
    xd, bd = cs.put(x0), cs.put(bo)
    xo = x0.copy()
    r0 = umg.norm(umg.L, umg.residual(umg.L, x0, bo))
    for k in range(3):
        cs.s.vcycle(xd, bd)
        xo = umg.cycle(xo, bo)
        d = cs.get(xd) - xo
        d[:3, lv.dirichlet] = 0.0
        rel = umg.norm(umg.L, umg.apply(umg.L, d)) / r0
        _announce(f"cycle {k}: ||K (x_gpu - x_oracle)|| / ||r0|| = {rel:.2e}")
        assert rel <= 1e-10, k
    xd = cs.put(x0)
    info = cs.s.solve(xd, bd, rtol=1e-8, max_cycles=80)
    xo, hist = umg.solve(x0.copy(), bo, rtol=1e-8, max_cycles=80)
    _announce(f"solve: {info['cycles']} cycles (oracle {len(hist) - 1}), rho {info['rho_mean']:.3f}")
    assert info["status"] == 0 and abs(info["cycles"] - (len(hist) - 1)) <= 1
    xg = cs.get(xd)
    un = np.sum(lv.normal[lv.slip] * xg[:3, lv.slip].T, axis=1)
    assert np.abs(un).max() <= 1e-12 * np.abs(xg[:3]).max()


def test_slip_solve_projects_the_start():
    """hhg_solve first removes the normal velocity of the start vector: a
    start with a normal part at the slip vertices gives the iterates of its
    projection (to rounding: the projection of a projected vector moves its
    last bits)."""
    cs = Case("cube", 4)
    lv = cs.umg.H.finest
    bo = cs.umg.rhs(np.random.default_rng(10).normal(size=(3, lv.N)))
    xa = np.random.default_rng(11).normal(size=(4, lv.N))
    xa[:3, lv.dirichlet] = 0.0
    xb = project_slip(lv, xa.copy())
    outs = []
    for x in (xa, xb):
        xd = cs.put(x)
        cs.s.solve(xd, cs.put(bo), rtol=1e-6, max_cycles=3)
        outs.append(_host(xd))
    assert _relerr(outs[0], outs[1]) < 1e-12


def test_slip_mixed_precision_meets_tolerance():
    cs = Case("shell", 4, precision=1)
    umg = cs.umg
    lv = umg.H.finest
    bo = umg.rhs(np.random.default_rng(12).normal(size=(3, lv.N)))
    xd = cs.put(np.zeros((4, lv.N)))
    info = cs.s.solve(xd, cs.put(bo), rtol=1e-8, max_cycles=80)
    x = cs.get(xd)
    rel = umg.norm(umg.L, umg.residual(umg.L, x, bo)) / umg.norm(umg.L, bo)
    _announce(f"mixed: {info['cycles']} cycles, oracle-operator residual {rel:.2e}")
    assert info["status"] == 0 and rel <= 1.05e-8


def test_slip_shell_full_size_conserves_mass():
    """The shell with a free-slip inner sphere at 5 refinements (workload 9): the solve reaches
    1e-8; the net outflow 1^T B u of the solution, summed from the pressure
    rows of K [u, 0], vanishes relative to the magnitude of B u."""
    import paper_1511_02134_amd as P
    cfg = W.WORKLOADS[9]
    xyz, tet, nu, tags = cfg.mesh()
    s = P.Solver(xyz, tet, nu, tags, cfg.R, phys=cfg.physical(), cycle=1)
    _announce(f"free-slip shell R={cfg.R}: {s.num_dofs()} unknowns")
    f = _dev(cfg.forcing_field())
    b = s.rhs(s.scatter(f))
    xd = s.scatter(_dev(np.zeros((4, s.num_nodes()))))
    info = s.solve(xd, b, rtol=1e-8, max_cycles=100)
    _announce(f"solve: {info['cycles']} cycles, rho {info['rho_mean']:.3f}, {info['t_solve_ms']:.1f} ms")
    assert info["status"] == 0 and info["rel_res"] <= 1e-8
    xn = _host(s.gather(xd))
    xn[3] = 0.0
    bu = _host(s.gather(s.apply(s.scatter(_dev(xn)))))[3]
    present = s.mass_weights() > 0
    assert abs(bu[present].sum()) <= 1e-12 * np.abs(bu[present]).sum()
