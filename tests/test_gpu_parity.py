"""GPU parity: every step of the hot path through the C ABI against the oracle
on the same seeded inputs (FP64).  Sizes span several volume tiles, all three
kinds of interface primitives and ragged fold tails."""
import numpy as np
import pytest

import workloads as W
from oracle import UMG, build_hierarchy

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _setup(cid, R, **opts):
    import paper_1511_02134_amd as P
    cfg = W.WORKLOADS[cid].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    _announce(f"config {cid} R={R} opts={opts}")
    s = P.Solver(xyz, tet, nu, tags, R, **opts)
    H = build_hierarchy(xyz, tet, nu, tags, R)
    return cfg, s, UMG(H, nu1=s.opts.nu1, nu2=s.opts.nu2,
                       variable=bool(s.opts.cycle), p_sweep="symmetric" if s.opts.p_sweep else "forward")


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rand_state(lv, seed, dirichlet_values=None):
    x = np.random.default_rng(seed).normal(size=(4, lv.N))
    if dirichlet_values is None:
        x[:3, lv.dirichlet] = 0.0
    else:
        x[:3, lv.dirichlet] = dirichlet_values[:, lv.dirichlet]
    return x


def _relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = [(1, 4), (4, 4), (5, 4), (1, 5)]


@pytest.mark.parametrize("cid,R", CASES)
def test_scatter_gather_exchange(cid, R):
    cfg, s, umg = _setup(cid, R)
    for l, lv in enumerate(umg.H.levels):
        x = _rand_state(lv, 10 + l)
        xi = s.scatter(_dev(x), l)
        assert np.array_equal(_host(s.gather(xi, l)), x)
        # the exchange of a consistent vector changes nothing
        y = xi.clone()
        s.exchange(y, l)
        assert torch.equal(y, xi)
        # slot -> node (scatter of node ids) and node -> primary slot (gather
        # of slot ids), both through the ABI
        N, ln = lv.N, s.vec_len(l)
        ids = _host(s.scatter(_dev(np.arange(1, N + 1, dtype=np.float64)[None, :]), l))[0]
        node_of = ids.astype(np.int64) - 1                       # -1 on padding
        prim = _host(s.gather(_dev(np.arange(ln, dtype=np.float64)[None, :]), l))[0].astype(np.int64)
        assert np.array_equal(node_of[prim], np.arange(N))
        copies = np.nonzero((node_of >= 0) & (np.arange(ln) != prim[np.maximum(node_of, 0)]))[0]
        if l >= 1:
            assert copies.size > 0
        # overwrite every non-primary copy with other values; the exchange
        # restores all of them from the primary, and gather is unchanged
        bad = xi.clone()
        noise = torch.tensor(np.random.default_rng(90 + l).normal(size=(4, copies.size)),
                             dtype=torch.float64, device="cuda")
        bad[:, torch.tensor(copies, device="cuda")] += 1.0 + noise
        assert np.array_equal(_host(s.gather(bad, l)), x)
        assert not torch.equal(bad, xi) or copies.size == 0
        s.exchange(bad, l)
        assert torch.equal(bad, xi)


@pytest.mark.parametrize("cid,R", CASES)
def test_apply_matches_oracle(cid, R):
    cfg, s, umg = _setup(cid, R)
    for l, lv in enumerate(umg.H.levels):
        x = _rand_state(lv, 20 + l, None)
        if l == umg.L:
            x[:3, lv.dirichlet] = np.random.default_rng(3).normal(size=(3, lv.N))[:, lv.dirichlet]
        y = _host(s.gather(s.apply(s.scatter(_dev(x), l), l), l))
        yo = umg.apply(l, x)
        assert _relerr(y, yo) < 1e-13, (l, _relerr(y, yo))


@pytest.mark.parametrize("cid,R", CASES)
def test_rhs_and_residual_match_oracle(cid, R):
    cfg, s, umg = _setup(cid, R)
    lv = umg.H.finest
    f = cfg.forcing_field() + W.nodal_noise(lv.N, 4, 1.0)
    b = _host(s.gather(s.rhs(s.scatter(_dev(f))), umg.L))
    bo = umg.rhs(f)
    assert _relerr(b, bo) < 1e-13
    x = _rand_state(lv, 5, cfg.dirichlet_field())
    r, nrm = s.residual(s.scatter(_dev(x)), s.scatter(_dev(bo)))
    ro = umg.residual(umg.L, x, bo)
    assert _relerr(_host(s.gather(r)), ro) < 1e-13
    assert nrm == pytest.approx(umg.norm(umg.L, ro), rel=1e-13)


@pytest.mark.parametrize("cid,R", CASES)
def test_transfers_match_oracle(cid, R):
    cfg, s, umg = _setup(cid, R)
    for l in range(1, umg.L + 1):
        lf, lc = umg.H.levels[l], umg.H.levels[l - 1]
        r = _rand_state(lf, 30 + l)
        bc = _host(s.gather(s.restrict(s.scatter(_dev(r), l), l), l - 1))
        assert _relerr(bc, umg.restrict(l, r)) < 1e-14
        e = _rand_state(lc, 40 + l)
        x = _rand_state(lf, 50 + l)
        xd = s.scatter(_dev(x), l)
        s.prolong_add(s.scatter(_dev(e), l - 1), xd, l)
        assert _relerr(_host(s.gather(xd, l)), x + umg.prolong(l, e)) < 1e-14


@pytest.mark.parametrize("cid,R", CASES)
def test_uzawa_step_matches_oracle(cid, R):
    cfg, s, umg = _setup(cid, R)
    for l in (1, umg.L):
        lv = umg.H.levels[l]
        x = _rand_state(lv, 60 + l, cfg.dirichlet_field() if l == umg.L else None)
        b = _rand_state(lv, 70 + l)
        xd, bd = s.scatter(_dev(x), l), s.scatter(_dev(b), l)
        s.smooth(xd, bd, 2, l)
        xo = x.copy()
        for _ in range(2):
            umg.uzawa(l, xo, b)
        assert _relerr(_host(s.gather(xd, l)), xo) < 1e-12, l


@pytest.mark.parametrize("cid", [1, 4])
def test_large_level_passes_match_oracle(cid):
    """64 intervals per macro edge, where K x and the residual run as separate
    volume and interface launches and the B^T p and B u passes (with their
    colour-0 sweeps) read quad windows: K x, the residual and Uzawa steps
    against the oracle on the whole level, and two steps on the next coarser
    level (32 intervals)."""
    cfg, s, umg = _setup(cid, 6)
    lv = umg.H.finest
    x = _rand_state(lv, 81, None)
    x[:3, lv.dirichlet] = np.random.default_rng(82).normal(size=(3, lv.N))[:, lv.dirichlet]
    y = _host(s.gather(s.apply(s.scatter(_dev(x), umg.L), umg.L), umg.L))
    err = _relerr(y, umg.apply(umg.L, x))
    _announce(f"K x: max rel. difference {err:.2e}")
    assert err < 1e-13
    b = _rand_state(lv, 83)
    x = _rand_state(lv, 84, cfg.dirichlet_field())
    r, nrm = s.residual(s.scatter(_dev(x)), s.scatter(_dev(b)))
    ro = umg.residual(umg.L, x, b)
    err = _relerr(_host(s.gather(r)), ro)
    _announce(f"residual: max rel. difference {err:.2e}")
    assert err < 1e-13
    assert nrm == pytest.approx(umg.norm(umg.L, ro), rel=1e-13)
    for l in (umg.L, umg.L - 1):
        lv = umg.H.levels[l]
        x = _rand_state(lv, 90 + l, cfg.dirichlet_field() if l == umg.L else None)
        b = _rand_state(lv, 95 + l)
        xd, bd = s.scatter(_dev(x), l), s.scatter(_dev(b), l)
        s.smooth(xd, bd, 2, l)
        xo = x.copy()
        for _ in range(2):
            umg.uzawa(l, xo, b)
        err = _relerr(_host(s.gather(xd, l)), xo)
        _announce(f"Uzawa steps, level {l}: max rel. difference {err:.2e}")
        assert err < 1e-12, l


@pytest.mark.parametrize("cid,solver,prec", [(1, 0, 1), (4, 0, 1), (5, 0, 1),
                                             (1, 1, 0), (4, 1, 0), (5, 1, 0), (1, 1, 1), (5, 1, 1)])
def test_coarse_solve_matches_dense(cid, solver, prec):
    """Direct solver (bordered inverse) and MINRES with both pressure
    preconditioners (exact Schur complement, lumped mass) against the
    oracle's bordered dense solve; an inconsistent right-hand side checks that
    its component along the constant pressure is removed."""
    cfg, s, umg = _setup(cid, 3, coarse_prec=prec, coarse_solver=solver)
    lv = umg.H.levels[0]
    x = _rand_state(lv, 80)
    b = umg.apply(0, x)                  # compatible right-hand side
    for bb in (b, b + np.concatenate([np.zeros((3, lv.N)), np.full((1, lv.N), 0.1)])):
        xg, it, rel = s.coarse_solve(s.scatter(_dev(bb), 0))
        xo = umg.coarse_solve(bb)
        if solver == 1:
            assert it < 500 and rel < 1e-13
            print(f"coarse PMINRES: {it} iterations, preconditioned residual {rel:.1e}")
        else:
            assert it == 1 and rel == 0.0
        assert _relerr(_host(s.gather(xg, 0)), xo) < 1e-11


@pytest.mark.parametrize("cid,R", CASES)
def test_cycles_match_oracle_iterate_by_iterate(cid, R):
    cfg, s, umg = _setup(cid, R)
    lv = umg.H.finest
    f = cfg.forcing_field()
    bo = umg.rhs(f)
    x0 = np.zeros((4, lv.N))
    x0[:3] = cfg.dirichlet_field()
    x0[:3, lv.free] = 0.0
    xd, bd = s.scatter(_dev(x0)), s.scatter(_dev(bo))
    xo = x0.copy()
    r0 = umg.norm(umg.L, umg.residual(umg.L, x0, bo))
    for k in range(4):
        s.vcycle(xd, bd)
        xo = umg.cycle(xo, bo)
        xg = _host(s.gather(xd))
        # ||K (x_gpu - x_orc)|| / ||r_0|| with the oracle operator
        d = xg - xo
        d[:3, lv.dirichlet] = 0.0
        assert umg.norm(umg.L, umg.apply(umg.L, d)) <= 1e-10 * r0, k
        assert _relerr(xg, xo) < 1e-10, k


@pytest.mark.parametrize("cid,R,opts", [(1, 4, {"cycle": 1}), (5, 4, {"p_sweep": 1}),
                                         (4, 4, {"cycle": 1, "p_sweep": 1, "nu1": 2, "nu2": 1})])
def test_cycle_switches_match_oracle(cid, R, opts):
    """The variable V-cycle (+2 smoothing steps per coarser level), the
    symmetric pressure sweep and other smoothing counts: iterates agree with
    the oracle's cycle of the same settings."""
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
        xg = _host(s.gather(xd))
        d = xg - xo
        d[:3, lv.dirichlet] = 0.0
        assert umg.norm(umg.L, umg.apply(umg.L, d)) <= 1e-10 * r0, k
        assert _relerr(xg, xo) < 1e-10, k


@pytest.mark.parametrize("cid,R", CASES)
def test_solve_matches_oracle(cid, R):
    cfg, s, umg = _setup(cid, R)
    lv = umg.H.finest
    bo = umg.rhs(cfg.forcing_field())
    x0 = np.zeros((4, lv.N))
    x0[:3] = cfg.dirichlet_field()
    x0[:3, lv.free] = 0.0
    xd = s.scatter(_dev(x0))
    info = s.solve(xd, s.scatter(_dev(bo)), rtol=1e-8, max_cycles=60)
    xo, hist = umg.solve(x0.copy(), bo, rtol=1e-8, max_cycles=60)
    assert info["status"] == 0
    assert info["cycles"] == len(hist) - 1
    assert info["rho_mean"] <= 0.3
    # residual histories agree to rounding relative to the initial residual
    assert np.abs(np.array(info["res_hist"]) - np.array(hist)).max() <= 1e-12 * hist[0]
    xg = _host(s.gather(xd))
    d = xg - xo
    d[:3, lv.dirichlet] = 0.0
    assert umg.norm(umg.L, umg.apply(umg.L, d)) <= 1e-10 * hist[0]


def test_schedule_permutation_is_bitwise_identical():
    """Reversed workgroup -> tile order: same bits (no race inside a colour)."""
    out = []
    for order in (1, 2):
        cfg, s, umg = _setup(4, 4, block_order=order)
        lv = umg.H.finest
        bo = umg.rhs(cfg.forcing_field())
        xd = s.scatter(_dev(np.zeros((4, lv.N))))
        bd = s.scatter(_dev(bo))
        for _ in range(2):
            s.vcycle(xd, bd)
        out.append(_host(s.gather(xd)))
    assert np.array_equal(out[0], out[1])
