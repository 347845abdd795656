"""Pins of the oracle's velocity multigrid, block-diagonal PMINRES and
Schur-complement CG (Sections 3.1, 3.2, 3.5): textbook two-grid algebra,
adjointness of the sweep orders, exactness on the coarse grid, library
MINRES and CG, brute-force minimal residuals, direct solutions and the
mesh-independent iteration counts of Table T:itertime1."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import build_hierarchy
from oracle.krylov import StokesKrylov, VelocityMG, lumped_mass_nu, minres
from oracle.umg import direct_solve


def _H(cfg_id, R):
    cfg = W.WORKLOADS[cfg_id].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    return cfg, build_hierarchy(xyz, tet, nu, tags, R)


@pytest.fixture(scope="module")
def box_r3():
    return _H(4, 3)        # two unit cubes, variable viscosity, two levels


@pytest.fixture(scope="module")
def box_r4():
    return _H(4, 4)


def _rand_vel(lv, seed):
    v = np.random.default_rng(seed).normal(size=(3, lv.N))
    v[:, lv.dirichlet] = 0.0
    return v


def test_lumped_mass_nu_row_sums():
    """For nu = 1 the weighted lumped mass is the row sum of the consistent
    mass matrix (int phi_i); it scales like 1/nu."""
    _, H = _H(1, 3)
    lv = H.finest
    assert np.allclose(lumped_mass_nu(lv, H.nu), np.asarray(lv.M.sum(axis=1)).ravel(), rtol=1e-14)
    assert np.allclose(lumped_mass_nu(lv, 4.0 * H.nu), lv.mass / 4.0, rtol=1e-14)
    assert np.isclose(lv.mass.sum(), 1.0, rtol=1e-13)       # |unit cube|


def test_velocity_mg_two_grid_error_operator(box_r3):
    """On two levels, V(1,1) with (FHGS, BHGS) has the textbook error
    propagation (I - (D+U)^-1 A)(I - P A_c^-1 P^T A)(I - (D+L)^-1 A) on the
    free velocity unknowns in the colour ordering, with the Galerkin coarse
    matrix P^T A P (equal to the rediscretised one for nested P1 spaces and
    macro-wise constant viscosity)."""
    _, H = box_r3
    mg = VelocityMG(H, 1, 1)
    f, c = H.levels[1], H.levels[0]
    ff = np.nonzero(f.free)[0]
    ff = ff[np.argsort(f.colour[ff], kind="stable")]
    fc = np.nonzero(c.free)[0]
    A = f.A[ff][:, ff].toarray()
    P = H.P[1][ff][:, fc].toarray()
    Ac = P.T @ A @ P
    assert np.allclose(Ac, c.A[fc][:, fc].toarray(), rtol=1e-12, atol=1e-12 * np.abs(Ac).max())
    D = np.diag(np.diag(A))
    I = np.eye(len(ff))
    E = ((I - np.linalg.solve(D + np.triu(A, 1), A))
         @ (I - P @ np.linalg.solve(Ac, P.T @ A))
         @ (I - np.linalg.solve(D + np.tril(A, -1), A)))
    u_star = _rand_vel(f, 1)
    b = np.stack([f.A @ u_star[k] for k in range(3)])
    b[:, f.dirichlet] = 0.0
    u0 = _rand_vel(f, 2)
    u1 = mg.cycle(1, u0.copy(), b)
    for k in range(3):
        e_ref = E @ (u_star[k][ff] - u0[k][ff])
        assert np.allclose(u_star[k][ff] - u1[k][ff], e_ref, rtol=1e-10,
                           atol=1e-12 * np.abs(u_star).max())
    assert np.all(u1[:, f.dirichlet] == 0.0)


def test_velocity_mg_symmetric_and_sweep_orders_adjoint(box_r4):
    """V(1,1) from zero is a symmetric operator; V(1,0) (forward sweep) and
    V(0,1) (backward sweep) are adjoint to each other."""
    _, H = box_r4
    lv = H.finest
    b1, b2 = _rand_vel(lv, 3), _rand_vel(lv, 4)
    m11 = VelocityMG(H, 1, 1)
    s1, s2 = np.sum(m11.inv(b1) * b2), np.sum(b1 * m11.inv(b2))
    assert abs(s1 - s2) <= 1e-12 * abs(s1)
    m10, m01 = VelocityMG(H, 1, 0), VelocityMG(H, 0, 1)
    s1, s2 = np.sum(m10.inv(b1) * b2), np.sum(b1 * m01.inv(b2))
    assert abs(s1 - s2) <= 1e-12 * abs(s1)
    # the forward sweep alone is not symmetric (the test can tell orders apart)
    s3 = np.sum(b1 * m10.inv(b2))
    assert abs(s1 - s3) > 1e-6 * abs(s1)


def test_velocity_mg_is_exact_on_level0():
    _, H = _H(1, 2)
    lv = H.finest
    b = _rand_vel(lv, 5)
    fr = np.nonzero(lv.free)[0]
    u = VelocityMG(H, 1, 1).inv(b)
    for k in range(3):
        assert np.allclose(u[k][fr], np.linalg.solve(lv.A[fr][:, fr].toarray(), b[k][fr]),
                           rtol=1e-12)


@pytest.mark.parametrize("nu1,nu2,bound", [(1, 1, 0.5), (3, 3, 0.2)])
def test_velocity_mg_contraction_is_mesh_independent(nu1, nu2, bound):
    """A-norm contraction of the cycle on a random error, at R=4 and R=5 of
    the unit cube: below a textbook Poisson bound and nearly level
    independent."""
    rates = []
    for R in (4, 5):
        _, H = _H(1, R)
        lv = H.finest
        mg = VelocityMG(H, nu1, nu2)
        e = _rand_vel(lv, 6)
        b = np.zeros_like(e)

        def anorm(v):
            return np.sqrt(sum(v[k] @ (lv.A @ v[k]) for k in range(3)))
        u = e.copy()
        for _ in range(3):
            u = mg.cycle(mg.L, u, b)
        u0 = anorm(u)
        u = mg.cycle(mg.L, u, b)
        u = mg.cycle(mg.L, u, b)
        rates.append(np.sqrt(anorm(u) / u0))
    assert max(rates) < bound, rates
    assert abs(rates[0] - rates[1]) < 0.05, rates


def _indefinite(seed, n=40):
    rng = np.random.default_rng(seed)
    Q = rng.normal(size=(n, n))
    K = Q + Q.T
    Pd = rng.uniform(0.5, 2.0, size=n)
    return K, Pd, rng.normal(size=n), rng.normal(size=n)


@pytest.mark.parametrize("k", [1, 3, 8])
def test_minres_matches_library_minres(k):
    """On a symmetric indefinite matrix with an SPD diagonal preconditioner
    the iterates equal scipy's preconditioned MINRES after k steps."""
    K, Pd, b, x0 = _indefinite(0)
    n = K.shape[0]
    M = spla.LinearOperator((n, n), matvec=lambda v: v / Pd)
    xs, _ = spla.minres(K, b, x0=x0, M=M, maxiter=k, rtol=1e-300)
    xo, h = minres(lambda v: K @ v, lambda v: v / Pd, np.linalg.norm, x0, b, iters=k)
    assert len(h) == k + 1
    assert np.allclose(xo, xs, rtol=1e-12, atol=1e-12 * np.abs(xs).max())


def test_minres_minimises_preconditioned_residual_over_krylov_space():
    """Brute force: x_k minimises ||b - K x||_{P^-1} over x_0 + K_k(P^-1 K,
    P^-1 r_0), found by least squares over an explicit Krylov basis; the
    recurred residual norms are the true ones."""
    K, Pd, b, x0 = _indefinite(1)
    r0 = b - K @ x0
    for k in (1, 2, 4, 7):
        xo, h = minres(lambda v: K @ v, lambda v: v / Pd, np.linalg.norm, x0, b, iters=k)
        V = [r0 / Pd]
        for _ in range(k - 1):
            V.append((K @ V[-1]) / Pd)
        V = np.linalg.qr(np.array(V).T)[0]
        W = (K @ V) / np.sqrt(Pd)[:, None]
        c = np.linalg.lstsq(W, r0 / np.sqrt(Pd), rcond=None)[0]
        assert np.allclose(xo, x0 + V @ c, rtol=1e-9, atol=1e-9 * np.abs(xo).max())
        assert np.isclose(h[-1], np.linalg.norm(b - K @ xo), rtol=1e-9)


def test_pminres_stokes_reaches_direct_solution(box_r3):
    """PMINRES on the Stokes system (variable viscosity, pressure up to a
    constant) converges to the direct solution; the recurred residual is the
    true one."""
    cfg, H = box_r3
    ks = StokesKrylov(H, 1, 1)
    lv = H.finest
    from oracle import UMG
    b = UMG(H).rhs(W.fourier_forcing(W.lattice_points(cfg.a, 3), 41))
    x0 = np.zeros((4, lv.N))
    x, hist = ks.pminres(x0, b, rtol=1e-12)
    assert hist[-1] <= 1e-12 * hist[0]
    assert np.isclose(ks.norm(b - ks.apply(x)), hist[-1], rtol=1e-4, atol=1e-14 * hist[0])
    xd = direct_solve(lv, b, H.project)
    assert np.abs(x - xd).max() <= 1e-8 * np.abs(xd).max()


class _ExactMG(VelocityMG):
    """Velocity 'multigrid' replaced by exact solves (for the SCG pin)."""

    def __init__(self, H):
        super().__init__(H, 1, 1)
        lv = H.finest
        self._fr = np.nonzero(lv.free)[0]
        self._Af = lv.A[self._fr][:, self._fr].toarray()

    def cycle(self, l, u, b):
        u = u.copy()
        for k in range(3):
            u[k][self._fr] = np.linalg.solve(self._Af, b[k][self._fr])
        return u


def test_scg_with_exact_velocity_solves_is_pcg_on_schur_complement():
    """With exact inner solves, one outer iteration of Algorithm 1 gives
    u = A^-1 (f - B^T p_0) and then n_S steps of preconditioned CG on the
    assembled S = B A^-1 B^T + C (scipy's CG, lumped mass preconditioner)
    from p_0.  Channel workload: an outflow face, so S is nonsingular."""
    cfg, H = _H(5, 3)
    lv = H.finest
    ks = StokesKrylov(H, 3, 3)
    ks.mg = _ExactMG(H)
    from oracle import UMG
    b = UMG(H).rhs(W.fourier_forcing(W.lattice_points(cfg.a, 3), 7))
    rng = np.random.default_rng(8)
    x0 = np.zeros((4, lv.N))
    x0[3] = rng.normal(size=lv.N)
    fr = np.nonzero(lv.free)[0]
    Af = lv.A[fr][:, fr].toarray()
    Bf = [lv.B[k][:, fr].toarray() for k in range(3)]
    S = sum(Bk @ np.linalg.solve(Af, Bk.T) for Bk in Bf) + lv.C.toarray()
    h = sum(Bk @ np.linalg.solve(Af, b[k][fr]) for k, Bk in enumerate(Bf)) - b[3]
    for n_S in (1, 3, 6):
        x, _ = ks.scg(x0, b, n_A=1, n_S=n_S, n_I=1, outer=1)
        n = lv.N
        M = spla.LinearOperator((n, n), matvec=lambda v: v / ks.mnu)
        p_ref, _ = spla.cg(S, h, x0=x0[3], M=M, maxiter=n_S, rtol=1e-300)
        assert np.allclose(x[3], p_ref, rtol=1e-9, atol=1e-9 * np.abs(p_ref).max())
        u_ref = [np.linalg.solve(Af, b[k][fr] - Bf[k].T @ x0[3]) for k in range(3)]
        for k in range(3):
            assert np.allclose(x[k][fr], u_ref[k], rtol=1e-10, atol=1e-12)


def test_scg_stokes_reaches_direct_solution(box_r3):
    cfg, H = box_r3
    ks = StokesKrylov(H, 3, 3)
    lv = H.finest
    from oracle import UMG
    b = UMG(H).rhs(W.fourier_forcing(W.lattice_points(cfg.a, 3), 41))
    x, hist = ks.scg(np.zeros((4, lv.N)), b, rtol=1e-12)
    assert hist[-1] <= 1e-12 * hist[0]
    xd = direct_solve(lv, b, H.project)
    assert np.abs(x - xd).max() <= 1e-8 * np.abs(xd).max()


def test_iteration_counts_are_mesh_independent():
    """Table T:itertime1 setting (f = 0, u0 ~ U[0,1], p0 ~ U[0, 1/h_min],
    eps = 1e-8): iteration numbers of PMINRES (paper: 73 and 70 at L = 4, 5)
    and SCG stay nearly constant under refinement (R = 4, 5 here, the
    paper's L = 2, 3)."""
    its = {"pminres": [], "scg": []}
    for R in (4, 5):
        _, H = _H(1, R)
        lv = H.finest
        hmin = (1.0 / (6 * lv.n ** 3)) ** (1.0 / 3.0)
        x0 = W.random_initial_guess(lv.N, 1.0 / hmin, seed=0)
        x0[:3, lv.dirichlet] = 0.0
        b = np.zeros_like(x0)
        _, h = StokesKrylov(H, 1, 1).pminres(x0, b)
        its["pminres"].append(len(h) - 1)
        _, h = StokesKrylov(H, 3, 3).scg(x0, b)
        its["scg"].append(len(h) - 1)
    assert all(60 <= n <= 85 for n in its["pminres"]), its
    assert abs(its["pminres"][0] - its["pminres"][1]) <= 6, its
    assert all(8 <= n <= 20 for n in its["scg"]), its
    assert abs(its["scg"][0] - its["scg"][1]) <= 2, its
