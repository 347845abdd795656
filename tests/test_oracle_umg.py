"""Pins of the oracle's Uzawa multigrid: preconditioner algebra, fixed points,
direct solutions, convergence rates, discretisation order and the paper's
serial iteration counts."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import UMG, build_hierarchy

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _umg(cfg_id, R, **kw):
    cfg = W.WORKLOADS[cfg_id].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    return cfg, UMG(build_hierarchy(xyz, tet, nu, tags, R), **kw)


@pytest.fixture(scope="module")
def box_r3():
    return _umg(4, 3)


def _colour_perm(lv, idx):
    """Indices idx ordered by colour 0..3 (stable)."""
    return idx[np.argsort(lv.colour[idx], kind="stable")]


def test_sgs_is_symmetric_gauss_seidel(box_r3):
    """Ahat^{-1} r equals the textbook SGS preconditioner (D+L) D^{-1} (D+U) in
    the colour ordering, built densely."""
    _, umg = box_r3
    l = 1
    lv = umg.H.levels[l]
    fr = _colour_perm(lv, np.nonzero(lv.free)[0])
    A = lv.A[fr][:, fr].toarray()
    D = np.diag(np.diag(A))
    Lo, Up = np.tril(A, -1), np.triu(A, 1)
    Ahat = (D + Lo) @ np.linalg.solve(D, D + Up)
    r = np.random.default_rng(0).normal(size=lv.N)
    r[lv.dirichlet] = 0.0
    d = umg.sgs(l, r)
    assert np.all(d[lv.dirichlet] == 0.0)
    assert np.allclose(d[fr], np.linalg.solve(Ahat, r[fr]), rtol=1e-11, atol=1e-13 * abs(d).max())


def test_sor_is_forward_relaxed_gauss_seidel(box_r3):
    """Shat^{-1} s with Shat = D_C / omega + L_C (colour ordering)."""
    _, umg = box_r3
    l = 1
    lv = umg.H.levels[l]
    p = _colour_perm(lv, np.arange(lv.N))
    C = lv.C[p][:, p].toarray()
    Shat = np.diag(np.diag(C)) / umg.omega + np.tril(C, -1)
    s = np.random.default_rng(1).normal(size=lv.N)
    assert np.allclose(umg.sor(l, s)[p], sla.solve_triangular(Shat, s[p], lower=True),
                       rtol=1e-11)


def test_symmetric_sor_is_textbook_ssor(box_r3):
    """With p_sweep = 'symmetric', Shat^{-1} s is one forward SOR sweep (colours
    0..3) followed by one backward sweep (colours 3..0) from zero.  Its
    operator is the textbook SSOR preconditioner in product form,
    Shat = omega/(2-omega) (D/omega + L) D^{-1} (D/omega + U), with L and U the
    strictly lower and upper parts of C in the colour ordering: a closed form
    that shares nothing with the sweep loop.  A wrong backward order, a
    missing repeat of colour 3 or a relaxation on the wrong side breaks the
    equality; the symmetry of Shat is checked as well."""
    cfg, _ = box_r3
    xyz, tet, nu, tags = cfg.mesh()
    umg = UMG(build_hierarchy(xyz, tet, nu, tags, 3), p_sweep="symmetric")
    l = 1
    lv = umg.H.levels[l]
    p = _colour_perm(lv, np.arange(lv.N))
    C = lv.C[p][:, p].toarray()
    w = umg.omega
    D = np.diag(np.diag(C))
    Lo, Up = np.tril(C, -1), np.triu(C, 1)
    Shat = w / (2.0 - w) * (D / w + Lo) @ np.linalg.solve(D, D / w + Up)
    assert np.allclose(Shat, Shat.T, rtol=0, atol=1e-13 * np.abs(Shat).max())
    s = np.random.default_rng(11).normal(size=lv.N)
    d = umg.sor(l, s)
    ref = np.linalg.solve(Shat, s[p])
    assert np.allclose(d[p], ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())
    # forward half alone differs (the backward half is not a no-op)
    fwd = UMG(umg.H, p_sweep="forward").sor(l, s)
    assert np.abs(fwd - d).max() > 1e-3 * np.abs(d).max()


def test_exact_solution_is_fixed_point(box_r3):
    """The discrete solution is a fixed point of the Uzawa step and of the
    V-cycle (consistency of eq. Uzawa_smooth and the coarse correction)."""
    cfg, umg = box_r3
    b = umg.rhs(cfg.forcing_field())
    xs = umg.direct_solve(b)
    L = umg.L
    assert umg.norm(L, umg.residual(L, xs, b)) < 1e-12 * umg.norm(L, b)
    x1 = umg.uzawa(L, xs.copy(), b)
    assert np.abs(x1 - xs).max() < 1e-10 * np.abs(xs).max()
    x2 = umg.cycle(xs.copy(), b)
    assert np.abs(x2 - xs).max() < 1e-10 * np.abs(xs).max()


def test_coarse_solve_is_exact_and_mean_free(box_r3):
    _, umg = box_r3
    lv = umg.H.levels[0]
    rng = np.random.default_rng(5)
    x = rng.normal(size=(4, lv.N))
    x[:3, lv.dirichlet] = 0.0
    b = umg.apply(0, x)                      # compatible right-hand side
    e = umg.coarse_solve(b)
    assert umg.norm(0, umg.residual(0, e, b)) < 1e-12 * umg.norm(0, b)
    assert abs(lv.mass @ e[3]) < 1e-13 * np.abs(e[3]).max()
    xm = x.copy()
    xm[3] -= (lv.mass @ x[3]) / lv.mass.sum()
    assert np.abs(e - xm).max() < 1e-11 * np.abs(xm).max()


@pytest.mark.parametrize("cfg_id,R", [(1, 4), (4, 4), (5, 4), (4, 3), (5, 3)])
def test_vcycle_convergence_factor(cfg_id, R):
    """V(3,3) Uzawa multigrid from x0 = 0 (Dirichlet values set): mean
    convergence factor per cycle at most 0.3; at R = 3 the solution also
    agrees with the sparse direct solution."""
    cfg, umg = _umg(cfg_id, R)
    lv = umg.H.finest
    b = umg.rhs(cfg.forcing_field())
    x0 = np.zeros((4, lv.N))
    x0[:3] = cfg.dirichlet_field()
    x0[:3, lv.free] = 0.0
    x, hist = umg.solve(x0.copy(), b, rtol=1e-8)
    K = len(hist) - 1
    rho_mean = (hist[-1] / hist[0]) ** (1.0 / K)
    assert rho_mean <= 0.3, hist
    assert hist[-1] <= 1e-8 * hist[0]
    if R > 3:
        return
    xd = umg.direct_solve(b, xbc=x0)
    err = np.sqrt(np.sum((x - xd) ** 2))
    assert err <= 1e-6 * np.sqrt(np.sum(xd ** 2))


def test_manufactured_velocity_converges_second_order():
    errs = []
    for R in (3, 4, 5):
        cfg, umg = _umg(1, R)
        b = umg.rhs(cfg.forcing_field())
        x, _ = umg.solve(np.zeros((4, umg.H.finest.N)), b, rtol=1e-11)
        ue = W.manufactured_velocity(cfg.points())
        errs.append(np.sqrt(np.mean((x[:3] - ue) ** 2)))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert ratios[-1] > 3.5, (errs, ratios)


def test_paper_style_iteration_count():
    """Section 3.6 / Table T:itertime1: f = 0, u0 ~ U[0,1], p0 ~ U[0, 1/h_min],
    Vvar(3,3), eps = 1e-8: 9 cycles at L=2 (R=4).  The global 4-colour ordering
    differs from the paper's hybrid Gauss-Seidel, so a band of +-2 is allowed."""
    gold = json.load(open(os.path.join(GOLD, "paper_serial_table.json")))
    cfg, umg = _umg(1, 4, variable=True)
    lv = umg.H.finest
    hmin = (1.0 / (6 * lv.n ** 3)) ** (1.0 / 3.0)
    x0 = W.random_initial_guess(lv.N, 1.0 / hmin, seed=0)
    x0[:3, lv.dirichlet] = 0.0
    b = np.zeros_like(x0)
    _, hist = umg.solve(x0, b, rtol=1e-8)
    it = len(hist) - 1
    assert abs(it - gold["umg_iterations"]["2"]) <= 2, hist


def test_primitive_classes_of_the_unit_cube():
    """fem.primitives against the combinatorics of the 6-tetrahedron Kuhn cube
    (8 corners, 19 edges, 18 faces, 6 volumes; edge, face and volume
    primitives hold n-1, (n-1)(n-2)/2 and (n-1)(n-2)(n-3)/6 nodes at 2^R = n)
    and against closed-form rules for nodes inside the cube: the main
    diagonal X = Y = Z is an edge, the planes X = Y, Y = Z, X = Z are faces,
    and points with distinct coordinates lie in a volume."""
    from oracle.fem import primitives
    cfg = W.WORKLOADS[1].with_R(4)
    xyz, tet, nu, tags = cfg.mesh()
    H = build_hierarchy(xyz, tet, nu, tags, 4)
    for lv in H.levels:
        n = lv.n
        cls, prim = primitives(lv, H.macro_int, H.tet)
        counts = [len(np.unique(prim[cls == k])) for k in range(4)]
        assert counts == [8, 19, 18, 6]
        sizes = [1, n - 1, (n - 1) * (n - 2) // 2, (n - 1) * (n - 2) * (n - 3) // 6]
        for k in range(4):
            assert np.all(np.bincount(prim[cls == k])[np.unique(prim[cls == k])] == sizes[k])
        X, Y, Z = lv.X.T
        inner = (X > 0) & (Y > 0) & (Z > 0) & (X < n) & (Y < n) & (Z < n)
        diag = inner & (X == Y) & (Y == Z)
        plane = inner & ~diag & ((X == Y) | (Y == Z) | (X == Z))
        free = inner & (X != Y) & (Y != Z) & (X != Z)
        assert np.all(cls[diag] == 1) and np.all(cls[plane] == 2) and np.all(cls[free] == 3)


def test_hybrid_sweeps_are_textbook_block_gauss_seidel(box_r3):
    """ordering='hybrid' (Section 3.4): the forward sweep from zero is
    W_f^{-1} r with W_f = D + (the entries of A towards earlier classes, and
    towards earlier colours inside the node's own primitive); entries towards
    other primitives of the same class are left out (block Jacobi).  The
    backward sweep keeps the class order and reverses the colours inside a
    primitive (W_b).  Velocity: d = d1 + W_b^{-1}(r - A d1), d1 = W_f^{-1} r;
    pressure: (D/omega + L_f) d = s.  Both closed forms are built densely
    from the partition; the velocity operator is not symmetric (the paper's
    'pseudo-symmetric' SHGS), and it differs from the colour ordering."""
    from oracle.fem import primitives
    cfg, _ = box_r3
    xyz, tet, nu, tags = cfg.mesh()
    H = build_hierarchy(xyz, tet, nu, tags, 3)
    umg = UMG(H, ordering="hybrid")
    l = 1
    lv = H.levels[l]
    cls, prim = primitives(lv, H.macro_int, H.tet)
    col = lv.colour
    earlier_cls = cls[None, :] < cls[:, None]
    same_prim = (cls[None, :] == cls[:, None]) & (prim[None, :] == prim[:, None])
    low_f = earlier_cls | (same_prim & (col[None, :] < col[:, None]))
    low_b = earlier_cls | (same_prim & (col[None, :] > col[:, None]))
    fr = np.nonzero(lv.free)[0]
    A = lv.A.toarray()[np.ix_(fr, fr)]
    D = np.diag(np.diag(A))
    Wf = D + np.where(low_f[np.ix_(fr, fr)], A, 0.0)
    Wb = D + np.where(low_b[np.ix_(fr, fr)], A, 0.0)
    r = np.zeros(lv.N)
    r[fr] = np.random.default_rng(12).normal(size=fr.shape[0])
    d = umg.sgs(l, r)
    d1 = np.linalg.solve(Wf, r[fr])
    ref = d1 + np.linalg.solve(Wb, r[fr] - A @ d1)
    assert np.allclose(d[fr], ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())
    assert np.all(d[lv.dirichlet] == 0.0)
    # the smoother's operator S with d = S r is not symmetric
    S = np.linalg.inv(Wf) + np.linalg.solve(Wb, np.eye(fr.shape[0]) - A @ np.linalg.inv(Wf))
    assert np.abs(S - S.T).max() > 1e-6 * np.abs(S).max()
    # ... and the colour ordering gives another result
    dc = UMG(H).sgs(l, r)
    assert np.abs(dc - d).max() > 1e-6 * np.abs(d).max()
    # pressure: forward hybrid SOR
    C = lv.C.toarray()
    w = umg.omega
    s = np.random.default_rng(13).normal(size=lv.N)
    dp = umg.sor(l, s)
    Wp = np.diag(np.diag(C)) / w + np.where(low_f, C, 0.0)
    refp = np.linalg.solve(Wp, s)
    assert np.allclose(dp, refp, rtol=1e-11, atol=1e-13 * np.abs(refp).max())


def test_redblack_sweeps_are_textbook(box_r3):
    """ordering='redblack': on Kuhn meshes the parities of X+Y+Z are
    independent sets of A and C (checked), and the velocity smoother is the
    textbook symmetric Gauss-Seidel (D+L)^-1 ... (D+U)^-1 in the red-black
    order, the pressure smoother forward SOR (D/omega + L) in that order; the
    iterates differ from the 4-colour order's.  On the shell (15-point
    stencils) the red-black order is rejected."""
    cfg, _ = box_r3
    xyz, tet, nu, tags = cfg.mesh()
    H = build_hierarchy(xyz, tet, nu, tags, 3)
    umg = UMG(H, ordering="redblack")
    l = 1
    lv = H.levels[l]
    par = lv.colour % 2
    fr = np.nonzero(lv.free)[0]
    idx = fr[np.argsort(par[fr], kind="stable")]
    A = lv.A.toarray()[np.ix_(idx, idx)]
    D = np.diag(np.diag(A))
    Lo, Up = np.tril(A, -1), np.triu(A, 1)
    r = np.zeros(lv.N)
    r[fr] = np.random.default_rng(31).normal(size=fr.shape[0])
    d = umg.sgs(l, r)
    d1 = np.linalg.solve(D + Lo, r[idx])
    ref = d1 + np.linalg.solve(D + Up, r[idx] - A @ d1)
    assert np.allclose(d[idx], ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())
    assert np.abs(UMG(H).sgs(l, r) - d).max() > 1e-6 * np.abs(d).max()
    ip = np.argsort(par, kind="stable")
    C = lv.C.toarray()[np.ix_(ip, ip)]
    s = np.random.default_rng(32).normal(size=lv.N)
    dp = umg.sor(l, s)
    refp = np.linalg.solve(np.diag(np.diag(C)) / umg.omega + np.tril(C, -1), s[ip])
    assert np.allclose(dp[ip], refp, rtol=1e-11, atol=1e-13 * np.abs(refp).max())
    # symmetric pressure sweep: then (D/omega + U) on the remaining residual
    us = UMG(H, ordering="redblack", p_sweep="symmetric")
    dps = us.sor(l, s)
    Dw = np.diag(np.diag(C)) / us.omega
    refs = refp + np.linalg.solve(Dw + np.triu(C, 1), s[ip] - C @ refp)
    assert np.allclose(dps[ip], refs, rtol=1e-11, atol=1e-13 * np.abs(refs).max())
    # the red-black multigrid contracts like the 4-colour one
    lf = H.finest
    b = umg.rhs(cfg.forcing_field())
    x0 = np.zeros((4, lf.N))
    x0[:3] = cfg.dirichlet_field()
    x0[:3, lf.free] = 0.0
    _, h_rb = umg.solve(x0.copy(), b, rtol=1e-8, max_cycles=40)
    _, h_c = UMG(H).solve(x0.copy(), b, rtol=1e-8, max_cycles=40)
    rho = (h_rb[-1] / h_rb[0]) ** (1.0 / (len(h_rb) - 1))
    assert rho <= 0.3 and abs(len(h_rb) - len(h_c)) <= 1
    sh = W.WORKLOADS[8].with_R(3)
    sxyz, stet, snu, stags = sh.mesh()
    with pytest.raises(ValueError):
        UMG(build_hierarchy(sxyz, stet, snu, stags, 3, phys=sh.physical()), ordering="redblack")
