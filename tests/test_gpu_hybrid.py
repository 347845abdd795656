"""GPU parity of the hybrid ordering (opts.ordering = 1, Section 3.4): the
Uzawa smoother sweeps the primitive classes (macro vertices, edges, faces,
volumes) in order, decouples the primitives of a class (block Jacobi through
saved starting values) and runs the colours inside each primitive.  Compared
with the oracle's hybrid smoother (ordering="hybrid", pinned to the textbook
block Gauss-Seidel operator) on Kuhn meshes and on the spherical shell
(15-tap stencils), in FP64, and in FP32 cycles against the oracle's FP64
operator."""
import numpy as np
import pytest

import workloads as W
from oracle import UMG, build_hierarchy

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


class Case:
    def __init__(self, cid, R, **opts):
        import paper_1511_02134_amd as P
        self.cfg = W.WORKLOADS[cid].with_R(R)
        xyz, tet, nu, tags = self.cfg.mesh()
        phys = self.cfg.physical()
        _announce(f"hybrid ordering: config {cid} R={R} opts={opts}")
        self.s = P.Solver(xyz, tet, nu, tags, R, phys=phys, ordering=1, **opts)
        H = build_hierarchy(xyz, tet, nu, tags, R, phys=phys)
        self.umg = UMG(H, nu1=self.s.opts.nu1, nu2=self.s.opts.nu2, ordering="hybrid",
                       variable=bool(self.s.opts.cycle),
                       p_sweep="symmetric" if self.s.opts.p_sweep else "forward")

    def put(self, x, l=None):
        l = self.umg.L if l is None else l
        lv = self.umg.H.levels[l]
        out = np.zeros((x.shape[0], self.s.num_nodes(l)))
        out[:, lv.lat] = x
        return self.s.scatter(_dev(out), l)

    def get(self, xd, l=None):
        l = self.umg.L if l is None else l
        return _host(self.s.gather(xd, l))[:, self.umg.H.levels[l].lat]


def _rand_state(lv, seed, dirichlet=None):
    x = np.random.default_rng(seed).normal(size=(4, lv.N))
    x[:3, lv.dirichlet] = 0.0 if dirichlet is None else dirichlet[:, lv.dirichlet]
    return x


@pytest.mark.parametrize("cid,R,opts", [(1, 4, {}), (4, 4, {}), (5, 4, {"p_sweep": 1}),
                                        (8, 3, {})])
def test_hybrid_uzawa_steps_match_oracle(cid, R, opts):
    cs = Case(cid, R, **opts)
    umg = cs.umg
    for l in (0, 1, umg.L):
        lv = umg.H.levels[l]
        x = _rand_state(lv, 60 + l, np.random.default_rng(7).normal(size=(3, lv.N)))
        b = _rand_state(lv, 70 + l)
        xd, bd = cs.put(x, l), cs.put(b, l)
        cs.s.smooth(xd, bd, 2, l)
        xo = x.copy()
        for _ in range(2):
            umg.uzawa(l, xo, b)
        err = _relerr(cs.get(xd, l), xo)
        _announce(f"hybrid Uzawa steps level {l}: max rel. difference {err:.2e}")
        assert err < 1e-12, l


@pytest.mark.parametrize("cid,R,opts", [(4, 4, {}), (5, 4, {"cycle": 1}), (7, 4, {"cycle": 1})])
def test_hybrid_cycles_match_oracle(cid, R, opts):
    cs = Case(cid, R, **opts)
    umg = cs.umg
    lv = umg.H.finest
    if cid == 7:
        x0 = _rand_state(lv, 90)
        bo = np.zeros((4, lv.N))
    else:
        bo = umg.rhs(cs.cfg.forcing_field()[:, lv.lat])
        x0 = np.zeros((4, lv.N))
        x0[:3] = cs.cfg.dirichlet_field()[:, lv.lat]
        x0[:3, lv.free] = 0.0
    xd, bd = cs.put(x0), cs.put(bo)
    xo = x0.copy()
    r0 = umg.norm(umg.L, umg.residual(umg.L, x0, bo))
    for k in range(3):
        cs.s.vcycle(xd, bd)
        xo = umg.cycle(xo, bo)
        d = cs.get(xd) - xo
        d[:3, lv.dirichlet] = 0.0
        rel = umg.norm(umg.L, umg.apply(umg.L, d)) / r0
        _announce(f"hybrid cycle {k}: ||K (x_gpu - x_oracle)|| / ||r0|| = {rel:.2e}")
        assert rel <= 1e-10, k


def test_hybrid_solve_matches_oracle():
    """A full solve: the oracle's cycle count and residual history."""
    cs = Case(4, 4)
    umg = cs.umg
    lv = umg.H.finest
    bo = umg.rhs(cs.cfg.forcing_field()[:, lv.lat])
    x0 = np.zeros((4, lv.N))
    xd = cs.put(x0)
    info = cs.s.solve(xd, cs.put(bo), rtol=1e-8, max_cycles=60)
    xo, hist = umg.solve(x0.copy(), bo, rtol=1e-8, max_cycles=60)
    _announce(f"hybrid solve: {info['cycles']} cycles (oracle {len(hist) - 1}), "
              f"rho_mean {info['rho_mean']:.3f}")
    assert info["status"] == 0 and info["cycles"] == len(hist) - 1
    assert np.abs(np.array(info["res_hist"]) - np.array(hist)).max() <= 1e-12 * hist[0]


def test_hybrid_mixed_precision_meets_tolerance():
    """FP32 cycles in FP64 refinement with the hybrid smoother reach 1e-8 in
    the oracle's FP64 operator."""
    cs = Case(4, 5, precision=1)
    umg = cs.umg
    lv = umg.H.finest
    bo = umg.rhs(cs.cfg.forcing_field()[:, lv.lat])
    xd = cs.put(np.zeros((4, lv.N)))
    info = cs.s.solve(xd, cs.put(bo), rtol=1e-8, max_cycles=80)
    r = umg.residual(umg.L, cs.get(xd), bo)
    rel = umg.norm(umg.L, r) / umg.norm(umg.L, bo)
    _announce(f"hybrid mixed: {info['cycles']} cycles, oracle-operator residual {rel:.2e}")
    assert info["status"] == 0 and rel <= 1.05e-8
