"""Discrete adjoint gradients of J = 1/2 ||u - u_obs||_2^2 (oracle).

Not part of the paper.  K of eq. (linear-system) is symmetric, so with
K x = f~(f) and J depending on the nodal velocity u only, the adjoint state
lambda solves K lambda = (u - u_obs on free velocity rows, 0 on pressure rows)
and
  * dJ/df_k = M lambda_{u,k} + G_k^T lambda_p  (f~ = R f is linear in the nodal
    forcing: M f_k on velocity rows, g_l = sum_k G_k f_k on pressure rows);
  * dJ/dnu_e = lambda^T (d f~/dnu_e - dK/dnu_e x).  a_1 is linear in nu_e and
    the PSPG terms carry delta h_T^2 / nu_T, so with A_e, C_e, g_e the parts
    of macro e at unit viscosity:
      dJ/dnu_e = -lambda_u^T A_e u - nu_e^-2 lambda_p^T (C_e p + g_e)
               = -sum_{T in e} |T| sum_k grad(lambda_k) . grad(u_k)
                 - nu_e^-2 sum_{T in e} delta h_T^2 int_T (grad p - f_h) . grad(lambda_p)
    where u includes its Dirichlet values and lambda vanishes on Dirichlet
    nodes.
The pressure constant of lambda does not enter either gradient (G_k^T 1 = 0).
For the D form a_2 = 2 <nu D(u), D(v)>, also linear in nu_e, the velocity
part becomes -sum_{T in e} |T| 2 D(lambda_u) : D(u)
= -sum_{T in e} |T| (sum_k grad(lambda_k) . grad(u_k) + sum_{k,l} d_l lambda_k d_k u_l).
"""
from __future__ import annotations

import numpy as np


def loss(u, u_obs):
    return 0.5 * float(np.sum((u - u_obs) ** 2))


def adjoint_rhs(lv, u, u_obs):
    b = np.zeros((4, lv.N))
    b[:3] = u - u_obs
    b[:3, lv.dirichlet] = 0.0
    return b


def project_transpose(lv, q):
    """Pi^T q for the mean-zero projection Pi p = p - 1 (m . p) / sum(m) of the
    pressure (Section 2.1: the pressure lives in L^2_0; m_i = int phi_i):
    Pi^T q = q - m (1 . q) / sum(m)."""
    return q - lv.mass * (q.sum() / lv.mass.sum())


def adjoint_rhs_general(lv, gu, gp, project):
    """Right-hand side of K lambda = dJ/dx for a loss J(u, Pi p) with
    gradients gu [3,N] (velocity) and gp [N] (pressure): gu on the free
    velocity rows (Dirichlet rows are not unknowns), Pi^T gp on the pressure
    rows (the identity when `project` is False, i.e. without a null space)."""
    b = np.zeros((4, lv.N))
    b[:3] = gu
    b[:3, lv.dirichlet] = 0.0
    b[3] = project_transpose(lv, gp) if project else gp
    return b


def grad_forcing(lv, lam):
    lu = lam[:3].copy()
    lu[:, lv.dirichlet] = 0.0
    return np.stack([lv.M @ lu[k] + lv.Gf[k].T @ lam[3] for k in range(3)])


def grad_viscosity(lv, x, lam, f_nodal, nu, op="laplace"):
    """x = (u, p) with Dirichlet values, lam = adjoint state, f_nodal [3,N];
    op selects the velocity form (a_1 or a_2)."""
    from .fem import DELTA
    lu = lam[:3].copy()
    lu[:, lv.dirichlet] = 0.0
    T = lv.tets
    acc = np.zeros(T.shape[0])
    gus = [np.einsum("ta,tai->ti", x[k][T], lv.G) for k in range(3)]
    gls = [np.einsum("ta,tai->ti", lu[k][T], lv.G) for k in range(3)]
    for k in range(3):
        acc += lv.vol * np.einsum("ti,ti->t", gus[k], gls[k])
    if op == "D":
        for k in range(3):
            for l in range(3):
                acc += lv.vol * gls[k][:, l] * gus[l][:, k]
    glp = np.einsum("ta,tai->ti", lam[3][T], lv.G)
    gp = np.einsum("ta,tai->ti", x[3][T], lv.G)
    fbar = np.stack([f_nodal[k][T].mean(axis=1) for k in range(3)], axis=1)   # int_T f_h / |T|
    nu_t = nu[lv.tet_macro]
    pspg = DELTA * lv.vol ** (2.0 / 3.0) * lv.vol * np.einsum("ti,ti->t", gp - fbar, glp)
    acc += pspg / nu_t ** 2
    return -np.bincount(lv.tet_macro, weights=acc, minlength=nu.shape[0])
