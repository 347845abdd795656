"""GPU parity of the red-black order (opts.ordering = 2) on Kuhn meshes: the
velocity sweep red, black, red with the first red half fused into the pass
that forms f - B^T p, the pressure sweep red (fused into B u - g), black;
one launch per parity (two workgroups per tile of the volume part, one
per colour of the parity; one vertex per lane).  Compared with the
oracle's red-black smoother (pinned to the textbook SGS / SOR operators in
that order) on the cube, the box and the channel, on levels with and without
quad windows, in FP64 and in FP32 cycles."""
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


def _setup(cid, R, **opts):
    import paper_1511_02134_amd as P
    cfg = W.WORKLOADS[cid].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    _announce(f"red-black: config {cid} R={R} opts={opts}")
    s = P.Solver(xyz, tet, nu, tags, R, ordering=2, **opts)
    umg = UMG(build_hierarchy(xyz, tet, nu, tags, R), nu1=s.opts.nu1, nu2=s.opts.nu2,
              variable=bool(s.opts.cycle), ordering="redblack",
              p_sweep="symmetric" if s.opts.p_sweep else "forward")
    return cfg, s, umg


def _rand_state(lv, seed, dirichlet=None):
    x = np.random.default_rng(seed).normal(size=(4, lv.N))
    x[:3, lv.dirichlet] = 0.0 if dirichlet is None else dirichlet[:, lv.dirichlet]
    return x


@pytest.mark.parametrize("cid,R,opts", [(1, 4, {}), (4, 4, {}), (5, 4, {"p_sweep": 1}),
                                        (1, 6, {})])
def test_redblack_uzawa_steps_match_oracle(cid, R, opts):
    cfg, s, umg = _setup(cid, R, **opts)
    for l in sorted({0, 1, umg.L - 1, umg.L}):
        lv = umg.H.levels[l]
        x = _rand_state(lv, 60 + l, cfg.dirichlet_field() if l == umg.L else None)
        b = _rand_state(lv, 70 + l)
        xd, bd = s.scatter(_dev(x), l), s.scatter(_dev(b), l)
        s.smooth(xd, bd, 2, l)
        xo = x.copy()
        for _ in range(2):
            umg.uzawa(l, xo, b)
        err = _relerr(_host(s.gather(xd, l)), xo)
        _announce(f"red-black Uzawa steps level {l}: {err:.2e}")
        assert err < 1e-12, l


@pytest.mark.parametrize("cid,R,opts", [(1, 5, {"cycle": 1}), (4, 4, {}), (5, 4, {"cycle": 1})])
def test_redblack_cycles_and_solve_match_oracle(cid, R, opts):
    cfg, s, umg = _setup(cid, R, **opts)
    lv = umg.H.finest
    bo = umg.rhs(cfg.forcing_field())
    x0 = np.zeros((4, lv.N))
    x0[:3] = cfg.dirichlet_field()
    x0[:3, lv.free] = 0.0
    xd, bd = s.scatter(_dev(x0)), s.scatter(_dev(bo))
    xo = x0.copy()
    r0 = umg.norm(umg.L, umg.residual(umg.L, x0, bo))
    for k in range(3):
        s.vcycle(xd, bd)
        xo = umg.cycle(xo, bo)
        d = _host(s.gather(xd)) - xo
        d[:3, lv.dirichlet] = 0.0
        rel = umg.norm(umg.L, umg.apply(umg.L, d)) / r0
        _announce(f"red-black cycle {k}: {rel:.2e}")
        assert rel <= 1e-10, k
    xd = s.scatter(_dev(x0))
    info = s.solve(xd, bd, rtol=1e-8, max_cycles=60)
    xo, hist = umg.solve(x0.copy(), bo, rtol=1e-8, max_cycles=60)
    _announce(f"red-black solve: {info['cycles']} cycles (oracle {len(hist) - 1}), "
              f"rho {info['rho_mean']:.3f}")
    assert info["status"] == 0 and info["cycles"] == len(hist) - 1
    assert np.abs(np.array(info["res_hist"]) - np.array(hist)).max() <= 1e-12 * hist[0]


def test_redblack_mixed_precision_meets_tolerance():
    cfg, s, umg = _setup(1, 5, precision=1, cycle=1)
    lv = umg.H.finest
    bo = umg.rhs(cfg.forcing_field())
    xd = s.scatter(_dev(np.zeros((4, lv.N))))
    info = s.solve(xd, s.scatter(_dev(bo)), rtol=1e-8, max_cycles=60)
    r = umg.residual(umg.L, _host(s.gather(xd)), bo)
    rel = umg.norm(umg.L, r) / umg.norm(umg.L, bo)
    _announce(f"red-black mixed: {info['cycles']} cycles, oracle-operator residual {rel:.2e}")
    assert info["status"] == 0 and rel <= 1.05e-8
