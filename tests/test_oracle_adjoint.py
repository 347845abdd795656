"""Pins of the oracle's adjoint gradients against central finite differences of
its own forward map (direct solves), which share nothing with the gradient
formulas."""
import numpy as np
import pytest

import workloads as W
from oracle import build_hierarchy
from oracle.adjoint import adjoint_rhs, grad_forcing, grad_viscosity, loss
from oracle.umg import direct_solve


def _forward(cfg, nu, f, R, op="laplace"):
    """Finest level only (R0 = R) and a sparse direct solve."""
    xyz, tet, _, tags = cfg.mesh()
    H = build_hierarchy(xyz, tet, nu, tags, R, R0=R, op=op)
    lv = H.finest
    x0 = np.zeros((4, lv.N))
    x0[:3] = cfg.dirichlet_field()
    x0[:3, lv.free] = 0.0
    b = np.zeros((4, lv.N))
    for k in range(3):
        b[k] = lv.M @ f[k]
        b[k][lv.dirichlet] = 0.0
    b[3] = sum(lv.Gf[k] @ f[k] for k in range(3))
    return H, direct_solve(lv, b, H.project, xbc=x0)


@pytest.mark.parametrize("cfg_id,op", [(4, "laplace"), (5, "laplace"), (4, "D"), (5, "D")])
def test_gradients_match_finite_differences(cfg_id, op):
    R = 3
    cfg = W.WORKLOADS[cfg_id].with_R(R)
    _, tet, nu, _ = cfg.mesh()
    f = cfg.forcing_field() + W.nodal_noise(cfg.points().shape[0], 11, 0.3)
    H, x = _forward(cfg, nu, f, R, op)
    lv = H.finest
    _, xo = _forward(cfg, cfg.observation_viscosity(), f, R, op)
    u_obs = xo[:3]
    lam = direct_solve(lv, adjoint_rhs(lv, x[:3], u_obs), H.project)
    gf = grad_forcing(lv, lam)
    gnu = grad_viscosity(lv, x, lam, f, nu, op)

    def J(nu_, f_):
        _, xx = _forward(cfg, nu_, f_, R, op)
        return loss(xx[:3], u_obs)

    rng = np.random.default_rng(9)
    for _ in range(2):
        d = rng.normal(size=f.shape)
        eps = 1.0                              # J is quadratic in f: central FD is exact
        fd = (J(nu, f + eps * d) - J(nu, f - eps * d)) / (2 * eps)
        assert np.sum(gf * d) == pytest.approx(fd, rel=1e-8, abs=1e-14)
    eps = 1e-6
    macros = rng.choice(nu.shape[0], size=4, replace=False)
    fd = np.zeros(4)
    for i, e in enumerate(macros):
        dn = np.zeros_like(nu)
        dn[e] = eps
        fd[i] = (J(nu + dn, f) - J(nu - dn, f)) / (2 * eps)
    assert np.abs(gnu[macros] - fd).max() <= 1e-6 * np.abs(gnu).max()


def test_projection_transpose_identity():
    """Pi^T is the transpose of the mean-zero projection: <Pi p, q> = <p, Pi^T q>
    for random p, q, and Pi^T q has zero sum (it is orthogonal to the
    constants, the null space of the pressure)."""
    from oracle.adjoint import project_transpose
    cfg = W.WORKLOADS[1].with_R(3)
    xyz, tet, nu, tags = cfg.mesh()
    lv = build_hierarchy(xyz, tet, nu, tags, 3).finest
    rng = np.random.default_rng(3)
    p, q = rng.normal(size=lv.N), rng.normal(size=lv.N)
    proj = p - (lv.mass @ p) / lv.mass.sum()
    assert np.dot(proj, q) == pytest.approx(np.dot(p, project_transpose(lv, q)), rel=1e-13)
    assert abs(project_transpose(lv, q).sum()) < 1e-13 * np.abs(q).sum()


def test_pressure_loss_gradient_matches_finite_differences():
    """A loss that observes the pressure as well, J = 1/2 ||u - u_obs||^2 +
    1/2 ||p - p_obs||^2 with p the mean-zero discrete pressure: the adjoint
    right-hand side (u - u_obs on free rows, Pi^T (p - p_obs)) gives dJ/df
    equal to central differences of J through direct solves (exact up to
    rounding, J being quadratic in f).  Without Pi^T the pressure part of
    the right-hand side is incompatible with the null space and the
    gradient is wrong, which the test also checks."""
    from oracle.adjoint import adjoint_rhs_general
    R = 3
    cfg = W.WORKLOADS[4].with_R(R)
    _, tet, nu, _ = cfg.mesh()
    f = cfg.forcing_field() + W.nodal_noise(cfg.points().shape[0], 12, 0.3)
    H, x = _forward(cfg, nu, f, R)
    lv = H.finest
    assert H.project
    rng = np.random.default_rng(21)
    u_obs = x[:3] + rng.normal(size=x[:3].shape)
    p_obs = rng.normal(size=lv.N)

    def J(f_):
        _, xx = _forward(cfg, nu, f_, R)
        return loss(xx[:3], u_obs) + 0.5 * float(np.sum((xx[3] - p_obs) ** 2))

    gu, gp = x[:3] - u_obs, x[3] - p_obs
    lam = direct_solve(lv, adjoint_rhs_general(lv, gu, gp, True), H.project)
    gf = grad_forcing(lv, lam)
    bad = adjoint_rhs_general(lv, gu, gp, False)
    lam_bad = direct_solve(lv, bad, H.project)
    gf_bad = grad_forcing(lv, lam_bad)
    for _ in range(2):
        d = rng.normal(size=f.shape)
        fd = (J(f + d) - J(f - d)) / 2.0
        assert np.sum(gf * d) == pytest.approx(fd, rel=1e-8)
        assert abs(np.sum(gf_bad * d) - fd) > 1e-6 * abs(fd)
