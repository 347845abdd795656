"""GPU parity of the D form a_2 = 2 <nu D(u), D(v)> (Section 2.1): K x, the
residual, the point-block Uzawa smoothing step, V-cycle iterates and full
solves through the C ABI against the oracle (FP64), mixed precision against
the oracle's FP64 operator, and the entry points the D form does not
support."""
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
    _announce(f"D form: config {cid} R={R} opts={opts}")
    s = P.Solver(xyz, tet, nu, tags, R, op=1, **opts)
    H = build_hierarchy(xyz, tet, nu, tags, R, op="D")
    return cfg, s, UMG(H, nu1=s.opts.nu1, nu2=s.opts.nu2, variable=bool(s.opts.cycle))


def _rand_state(lv, seed, cfg=None):
    x = np.random.default_rng(seed).normal(size=(4, lv.N))
    x[:3, lv.dirichlet] = 0.0 if cfg is None else cfg.dirichlet_field()[:, lv.dirichlet]
    return x


CASES = [(1, 3), (1, 4), (4, 4), (5, 4), (4, 5)]


@pytest.mark.parametrize("cid,R", CASES)
def test_apply_and_residual_match_oracle(cid, R):
    cfg, s, umg = _setup(cid, R)
    for l, lv in enumerate(umg.H.levels):
        x = _rand_state(lv, 20 + l)
        x[:3, lv.dirichlet] = np.random.default_rng(3).normal(size=(3, lv.N))[:, lv.dirichlet]
        y = _host(s.gather(s.apply(s.scatter(_dev(x), l), l), l))
        yo = umg.apply(l, x)
        assert _relerr(y, yo) < 1e-13, (l, _relerr(y, yo))
    lv = umg.H.finest
    b = umg.rhs(cfg.forcing_field())
    x = _rand_state(lv, 5, cfg)
    r, nrm = s.residual(s.scatter(_dev(x)), s.scatter(_dev(b)))
    ro = umg.residual(umg.L, x, b)
    assert _relerr(_host(s.gather(r)), ro) < 1e-13
    assert abs(nrm - umg.norm(umg.L, ro)) <= 1e-12 * umg.norm(umg.L, ro)


@pytest.mark.parametrize("cid,R", CASES[:4])
def test_smoothing_step_matches_oracle(cid, R):
    """One inexact Uzawa step with the point-block velocity sweep, on every
    level."""
    cfg, s, umg = _setup(cid, R)
    for l, lv in enumerate(umg.H.levels):
        if l == 0:
            continue
        x = _rand_state(lv, 30 + l)
        b = np.random.default_rng(40 + l).normal(size=(4, lv.N))
        b[:3, lv.dirichlet] = 0.0
        xd = s.scatter(_dev(x), l)
        s.smooth(xd, s.scatter(_dev(b), l), 1, l)
        xo = umg.uzawa(l, x.copy(), b)
        err = _relerr(_host(s.gather(xd, l)), xo)
        _announce(f"level {l}: smoothing step max rel. difference {err:.2e}")
        assert err < 1e-12


@pytest.mark.parametrize("cid,R", CASES[:4])
def test_cycles_and_solve_match_oracle(cid, R):
    """V(3,3) iterates cycle by cycle, then the full solve: the same cycle
    count and residual history."""
    cfg, s, umg = _setup(cid, R)
    lv = umg.H.finest
    b = umg.rhs(cfg.forcing_field())
    x0 = np.zeros((4, lv.N))
    x0[:3, lv.dirichlet] = cfg.dirichlet_field()[:, lv.dirichlet]
    xd = s.scatter(_dev(x0))
    bd = s.scatter(_dev(b))
    xo = x0.copy()
    for k in range(3):
        s.vcycle(xd, bd)
        xo = umg.cycle(xo, b)
        err = _relerr(_host(s.gather(xd)), xo)
        _announce(f"cycle {k + 1}: max rel. difference {err:.2e}")
        assert err < 1e-10
    xd = s.scatter(_dev(x0))
    info = s.solve(xd, bd, rtol=1e-8, max_cycles=100)
    xs, hist = umg.solve(x0.copy(), b, rtol=1e-8)
    _announce(f"solve: {info['cycles']} cycles (oracle {len(hist) - 1}), "
              f"rel. residual {info['rel_res']:.2e}")
    assert info["status"] == 0
    assert info["cycles"] == len(hist) - 1
    h = np.array(info["res_hist"])
    assert np.abs(h - np.array(hist)).max() <= 1e-10 * hist[0]
    assert _relerr(_host(s.gather(xd)), xs) < 1e-9


def test_mixed_precision_solve_meets_tolerance_in_fp64_operator():
    """FP32 cycles inside FP64 refinement for the D form: the final residual,
    evaluated with the oracle's FP64 operator, meets 1e-8."""
    cfg, s, umg = _setup(5, 4, precision=1)
    lv = umg.H.finest
    b = umg.rhs(cfg.forcing_field())
    x0 = np.zeros((4, lv.N))
    x0[:3, lv.dirichlet] = cfg.dirichlet_field()[:, lv.dirichlet]
    xd = s.scatter(_dev(x0))
    info = s.solve(xd, s.scatter(_dev(b)), rtol=1e-8, max_cycles=100)
    assert info["status"] == 0
    x = _host(s.gather(xd))
    r0 = umg.norm(umg.L, umg.residual(umg.L, x0, b))
    r = umg.norm(umg.L, umg.residual(umg.L, x, b))
    _announce(f"mixed: {info['cycles']} cycles, oracle-evaluated rel. residual {r / r0:.2e}")
    assert r <= 1.0e-8 * r0 * (1 + 1e-6)


def test_d_form_rejects_unsupported_options():
    import paper_1511_02134_amd as P
    cfg = W.WORKLOADS[1].with_R(3)
    xyz, tet, nu, tags = cfg.mesh()
    with pytest.raises(P.HHGError):
        P.Solver(xyz, tet, nu, tags, 3, op=1, coarse_solver=1)
    with pytest.raises(P.HHGError):
        P.Solver(xyz, tet, nu, tags, 3, op=2)


@pytest.mark.parametrize("cid,R,nu1,nu2", [(1, 2, 1, 1), (1, 4, 1, 1), (4, 4, 3, 3),
                                          (5, 4, 2, 0), (5, 3, 0, 2)])
def test_velocity_cycle_matches_oracle(cid, R, nu1, nu2):
    """D-form velocity V(nu1, nu2): point-block sweeps, coupled A-residual,
    coupled level-0 inverse."""
    from oracle.krylov import VelocityMG
    cfg, s, umg = _setup(cid, R, krylov=1)
    H = umg.H
    lv = H.finest
    rng = np.random.default_rng(200 + R)
    x = rng.normal(size=(4, lv.N))
    b = rng.normal(size=(4, lv.N))
    xd = s.scatter(_dev(x))
    s.vel_cycle(xd, s.scatter(_dev(b)), nu1, nu2)
    xg = _host(s.gather(xd))
    xo = VelocityMG(H, nu1, nu2).cycle(len(H.levels) - 1, x[:3].copy(), b[:3])
    err = _relerr(xg[:3], xo)
    _announce(f"D velocity cycle V({nu1},{nu2}): max rel. difference {err:.2e}")
    assert err < 1e-12
    assert np.array_equal(xg[3], x[3])


@pytest.mark.parametrize("cid,R", [(1, 3), (4, 4), (5, 4)])
def test_krylov_iterates_match_oracle(cid, R):
    """PMINRES (12 iterations) and SCG (2 outer iterations) for the D form,
    iterates and residual histories against the oracle."""
    from oracle.krylov import StokesKrylov
    cfg, s, umg = _setup(cid, R, krylov=1)
    H = umg.H
    lv = H.finest
    f = cfg.forcing_field() + W.nodal_noise(lv.N, 7, 1.0)
    b = umg.rhs(f)
    x0 = np.random.default_rng(8).normal(size=(4, lv.N))
    x0[:3, lv.dirichlet] = cfg.dirichlet_field()[:, lv.dirichlet]
    bd = s.scatter(_dev(b))
    xo, ho = StokesKrylov(H, 1, 1).pminres(x0, b, iters=12)
    xd = s.scatter(_dev(x0))
    info = s.pminres(xd, bd, rtol=0.0, maxit=12)
    err = _relerr(_host(s.gather(xd)), xo)
    herr = np.abs(np.array(info["res_hist"]) - np.array(ho)).max() / ho[0]
    _announce(f"D PMINRES 12 iterations: {err:.2e}, history {herr:.2e}")
    assert err < 1e-9 and herr < 1e-11
    xo, ho = StokesKrylov(H, 3, 3).scg(x0, b, outer=2)
    xd = s.scatter(_dev(x0))
    info = s.scg(xd, bd, rtol=0.0, max_outer=2)
    err = _relerr(_host(s.gather(xd)), xo)
    herr = np.abs(np.array(info["res_hist"]) - np.array(ho)).max() / ho[0]
    _announce(f"D SCG 2 outer iterations: {err:.2e}, history {herr:.2e}")
    assert err < 1e-10 and herr < 1e-11
