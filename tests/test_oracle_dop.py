"""Pins of the oracle's D form a_2(u, v) = 2 <nu D(u), D(v)> (Section 2.1):
rigid motions in the kernel of A_2 on every row, the identity
a_2 = a_1 + <div u, div v> on H^1_0 at constant viscosity, symmetry, the
textbook point-block Gauss-Seidel, O(h^2) convergence and the multigrid
rate."""
import numpy as np
import pytest

import workloads as W
from oracle import UMG, build_hierarchy
from oracle.umg import direct_solve


def _H(cid, R, op="D"):
    cfg = W.WORKLOADS[cid].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    return cfg, build_hierarchy(xyz, tet, nu, tags, R, op=op)


@pytest.fixture(scope="module")
def channel_r3():
    return _H(5, 3)


def _rigid(X, w, c):
    """u(x) = w x x + c at the points X [N,3]; [3, N]."""
    return (np.cross(np.asarray(w)[None, :], X) + np.asarray(c)[None, :]).T


def test_rigid_motions_are_in_the_kernel_of_a2(channel_r3):
    """D(u) = 0 for u = w x x + c, so a_2(u, v) = 0 for every v: every row of
    A_2 u vanishes, the natural-boundary and interface rows included, with
    variable viscosity.  A_1 does not annihilate a rotation on boundary rows
    (the check tells the two forms apart)."""
    _, H = channel_r3
    lv = H.finest
    X = lv.X / lv.n
    for w, c in (((0.3, -1.2, 0.7), (0, 0, 0)), ((0, 0, 0), (1.0, -2.0, 0.5)),
                 ((1.0, 0.5, -0.25), (0.1, 0.2, 0.3))):
        u = _rigid(X, w, c)
        y = (lv.A2 @ u.ravel()).reshape(3, -1)
        scale = np.abs(lv.A2).sum(axis=1).max() * np.abs(u).max()
        assert np.abs(y).max() <= 1e-13 * scale
    u = _rigid(X, (0.3, -1.2, 0.7), (0, 0, 0))
    y1 = np.stack([lv.A @ u[k] for k in range(3)])
    assert np.abs(y1).max() > 1e-3 * np.abs(lv.A).sum(axis=1).max()


def test_a2_is_a1_plus_divdiv_on_the_free_block():
    """For u, v in H^1_0 and constant viscosity, 2 <D u, D v> = <grad u, grad v>
    + <div u, div v>; on the free block A_2 = diag(A_1) + Dv with the div-div
    matrix Dv^{kl}[a, b] = sum_T |T| d_k phi_a d_l phi_b, assembled here from
    the element gradients.  Off the free block the two differ (the test that
    they are not the same matrix)."""
    _, H = _H(1, 3)
    lv = H.finest
    N, fr = lv.N, np.nonzero(lv.free)[0]
    import scipy.sparse as sp
    Dv = [[None] * 3 for _ in range(3)]
    rows = np.repeat(lv.tets[:, :, None], 4, axis=2).ravel()
    cols = np.repeat(lv.tets[:, None, :], 4, axis=1).ravel()
    for k in range(3):
        for l in range(3):
            v = (lv.vol[:, None, None] * lv.G[:, :, None, k] * lv.G[:, None, :, l]).ravel()
            Dv[k][l] = sp.coo_matrix((v, (rows, cols)), shape=(N, N)).tocsr()
    for k in range(3):
        for l in range(3):
            ref = Dv[k][l] + (lv.A if k == l else 0)
            got = lv.A2[k * N:(k + 1) * N, l * N:(l + 1) * N]
            d = (got - ref)[fr][:, fr]
            assert abs(d).max() <= 1e-13 * abs(lv.A).max(), (k, l)
    assert abs(lv.A2[0:N, N:2 * N] - Dv[0][1]).max() > 1e-3 * abs(lv.A).max()


def test_a2_symmetric_and_positive_definite_on_the_free_block():
    _, H = _H(4, 2)
    lv = H.finest
    A2 = lv.A2.toarray()
    assert np.allclose(A2, A2.T, rtol=0, atol=1e-14 * np.abs(A2).max())
    fr = np.nonzero(lv.free)[0]
    f3 = np.concatenate([fr, fr + lv.N, fr + 2 * lv.N])
    assert np.linalg.eigvalsh(A2[np.ix_(f3, f3)]).min() > 0


def test_point_block_gauss_seidel_is_textbook():
    """The velocity sweep of the D form equals the symmetric block
    Gauss-Seidel (D_B + L_B) D_B^-1 (D_B + U_B) in the colour ordering, with
    3x3 vertex blocks D_B, built densely."""
    _, H = _H(4, 3)
    umg = UMG(H)
    l = 1
    lv = H.levels[l]
    N = lv.N
    fr = np.nonzero(lv.free)[0]
    fr = fr[np.argsort(lv.colour[fr], kind="stable")]
    f3 = np.concatenate([fr + k * N for k in range(3)])
    A = lv.A2[f3][:, f3].toarray()
    nv = fr.shape[0]
    vert = np.tile(np.arange(nv), 3)              # vertex position in colour order
    col = lv.colour[fr][vert]
    same = vert[:, None] == vert[None, :]
    lower = col[:, None] > col[None, :]
    DB = np.where(same, A, 0.0)
    LB = np.where(lower & ~same, A, 0.0)
    UB = np.where(lower.T & ~same, A, 0.0)
    Ahat = (DB + LB) @ np.linalg.solve(DB, DB + UB)
    r = np.random.default_rng(0).normal(size=(3, N))
    r[:, lv.dirichlet] = 0.0
    d = umg.sgs(l, r)
    assert np.all(d[:, lv.dirichlet] == 0.0)
    ref = np.linalg.solve(Ahat, r.ravel()[f3])
    assert np.allclose(d.ravel()[f3], ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_d_form_converges_at_second_order_and_agrees_with_laplace_form():
    """Manufactured divergence-free solution at nu = 1: -div(2 D(u)) = -Lap u,
    so both forms approximate the same u; the D-form error decays like h^2
    and its difference to the Laplace-form solution is of the order of the
    discretisation error."""
    errs, diffs = [], []
    for R in (3, 4, 5):
        cfg, H = _H(1, R)
        umg = UMG(H)
        b = umg.rhs(cfg.forcing_field())
        x, hist = umg.solve(np.zeros((4, H.finest.N)), b, rtol=1e-11)
        ue = W.manufactured_velocity(cfg.points())
        errs.append(np.sqrt(np.mean((x[:3] - ue) ** 2)))
        _, HL = _H(1, R, "laplace")
        uL = UMG(HL)
        xL, _ = uL.solve(np.zeros((4, HL.finest.N)), uL.rhs(cfg.forcing_field()), rtol=1e-11)
        diffs.append(np.sqrt(np.mean((x[:3] - xL[:3]) ** 2)))
    assert errs[1] / errs[2] > 3.5, errs
    assert all(d < 2.0 * e for d, e in zip(diffs, errs)), (diffs, errs)


def test_d_form_multigrid_rate_and_direct_solution():
    """V(3,3) contracts by at most 0.3 per cycle, nearly independently of the
    level, and converges to the direct solution (box, variable viscosity)."""
    rates = []
    for R in (4, 5):
        cfg, H = _H(1, R)
        umg = UMG(H)
        b = umg.rhs(cfg.forcing_field())
        _, hist = umg.solve(np.zeros((4, H.finest.N)), b, rtol=1e-8)
        rates.append((hist[-1] / hist[0]) ** (1.0 / (len(hist) - 1)))
    assert max(rates) <= 0.3, rates
    assert abs(rates[0] - rates[1]) < 0.08, rates
    cfg, H = _H(4, 3)
    umg = UMG(H)
    b = umg.rhs(cfg.forcing_field())
    x, hist = umg.solve(np.zeros((4, H.finest.N)), b, rtol=1e-12)
    xd = direct_solve(H.finest, b, H.project)
    assert np.abs(x - xd).max() <= 1e-9 * np.abs(xd).max()


def test_d_form_velocity_multigrid_two_grid_operator_and_symmetry():
    """Velocity multigrid of the Krylov solvers for the D form: on two levels
    V(1,1) has the error propagation (I - (D_B+U_B)^-1 A)(I - P A_c^-1 P^T A)
    (I - (D_B+L_B)^-1 A) with the 3x3 vertex blocks D_B and the Galerkin
    A_c = P^T A_2 P (equal to the rediscretised coupled block); V(1,1) from
    zero is symmetric, V(1,0) and V(0,1) adjoint."""
    from oracle.krylov import VelocityMG
    import scipy.sparse as sp
    _, H = _H(4, 3)
    f, c = H.levels[1], H.levels[0]
    ff = np.nonzero(f.free)[0]
    ff = ff[np.argsort(f.colour[ff], kind="stable")]
    fc = np.nonzero(c.free)[0]
    F3 = np.concatenate([ff + k * f.N for k in range(3)])
    C3 = np.concatenate([fc + k * c.N for k in range(3)])
    A = f.A2[F3][:, F3].toarray()
    P = sp.block_diag([H.P[1]] * 3).tocsr()[F3][:, C3].toarray()
    Ac = P.T @ A @ P
    assert np.allclose(Ac, c.A2[C3][:, C3].toarray(), rtol=1e-12, atol=1e-12 * np.abs(Ac).max())
    nv = ff.shape[0]
    vert = np.tile(np.arange(nv), 3)
    col = f.colour[ff][vert]
    same = vert[:, None] == vert[None, :]
    lower = col[:, None] > col[None, :]
    DB = np.where(same, A, 0.0)
    LB = np.where(lower & ~same, A, 0.0)
    UB = np.where(lower.T & ~same, A, 0.0)
    I = np.eye(A.shape[0])
    E = ((I - np.linalg.solve(DB + UB, A)) @ (I - P @ np.linalg.solve(Ac, P.T @ A))
         @ (I - np.linalg.solve(DB + LB, A)))
    rng = np.random.default_rng(1)
    us = rng.normal(size=(3, f.N))
    us[:, f.dirichlet] = 0.0
    b = (f.A2 @ us.ravel()).reshape(3, -1)
    b[:, f.dirichlet] = 0.0
    u0 = rng.normal(size=(3, f.N))
    u0[:, f.dirichlet] = 0.0
    mg = VelocityMG(H, 1, 1)
    u1 = mg.cycle(1, u0.copy(), b)
    e_ref = E @ (us - u0).ravel()[F3]
    assert np.allclose((us - u1).ravel()[F3], e_ref, rtol=1e-10, atol=1e-12 * np.abs(us).max())
    _, H4 = _H(4, 4)
    lv = H4.finest
    b1, b2 = rng.normal(size=(3, lv.N)), rng.normal(size=(3, lv.N))
    b1[:, lv.dirichlet] = 0.0
    b2[:, lv.dirichlet] = 0.0
    m11 = VelocityMG(H4, 1, 1)
    s1, s2 = np.sum(m11.inv(b1) * b2), np.sum(b1 * m11.inv(b2))
    assert abs(s1 - s2) <= 1e-12 * abs(s1)
    s1 = np.sum(VelocityMG(H4, 1, 0).inv(b1) * b2)
    s2 = np.sum(b1 * VelocityMG(H4, 0, 1).inv(b2))
    assert abs(s1 - s2) <= 1e-12 * abs(s1)


def test_d_form_krylov_solvers_reach_direct_solution_and_paper_trend():
    """PMINRES and SCG for the D form converge to the direct solution (box,
    variable viscosity); on the unit cube in the setting of Table
    T:itertime_D_ser both need fewer iterations than for the Laplace form,
    as the paper reports (PMINRES 68/65 against 73/70 at L = 4, 5)."""
    from oracle.krylov import StokesKrylov
    cfg, H = _H(4, 3)
    lv = H.finest
    b = UMG(H).rhs(W.fourier_forcing(W.lattice_points(cfg.a, 3), 41))
    xd = direct_solve(lv, b, H.project)
    x, hist = StokesKrylov(H, 1, 1).pminres(np.zeros((4, lv.N)), b, rtol=1e-12)
    assert np.abs(x - xd).max() <= 1e-8 * np.abs(xd).max()
    x, hist = StokesKrylov(H, 3, 3).scg(np.zeros((4, lv.N)), b, rtol=1e-12)
    assert np.abs(x - xd).max() <= 1e-8 * np.abs(xd).max()
    its = {}
    for op in ("laplace", "D"):
        _, Hc = _H(1, 4, op)
        lc = Hc.finest
        hmin = (1.0 / (6 * lc.n ** 3)) ** (1.0 / 3.0)
        x0 = W.random_initial_guess(lc.N, 1.0 / hmin, seed=0)
        x0[:3, lc.dirichlet] = 0.0
        z = np.zeros_like(x0)
        its[op] = (len(StokesKrylov(Hc, 1, 1).pminres(x0, z)[1]) - 1,
                   len(StokesKrylov(Hc, 3, 3).scg(x0, z)[1]) - 1)
    assert its["D"][0] < its["laplace"][0] and its["D"][1] < its["laplace"][1], its
    assert 50 <= its["D"][0] <= 80, its
