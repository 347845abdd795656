"""Velocity multigrid, block-diagonal preconditioned MINRES and the
Schur-complement CG (oracle; test infrastructure only: used by the tests, the
smoke check and the CPU baseline, never by the product path).

Section 3.1 (Algorithm 1), Section 3.2 (eq. precond_block_diag) and Section
3.5 with Table "settings" (the SCG and PMINRES columns):

  * Ahat^{-1} is a multigrid cycle for the velocity block A alone (the three
    components are decoupled copies of the scalar A): forward colour
    Gauss-Seidel (colours 0,1,2,3) in the pre-smoothing steps, backward
    (3,2,1,0) in the post-smoothing steps, "(FHGS, BHGS)".  V(1,1) for
    PMINRES, V(3,3) for SCG.  The residual is restricted by the transpose of
    P1 interpolation with velocity Dirichlet rows zeroed, the coarse
    correction starts from zero.
  * Shat^{-1} is the inverse of the lumped pressure mass matrix, weighted by
    1/nu: diagonal entries sum_{T around x} |T| / (4 nu_T) (the Schur
    complement B A^-1 B^T scales like 1/nu; for nu = 1 this is the plain
    lumped mass matrix of the paper).
  * PMINRES: MINRES on K x = f~ preconditioned by diag(Ahat, Shat), Lanczos
    in the Shat/Ahat inner product with Givens rotations.  The Euclidean
    residual of the stopping test (Section 3.6) is carried by the recurrence
    r_j = r_{j-1} - tau_j K w_j, where K w_j follows the recurrence of the
    search directions w_j.
  * SCG (Algorithm 1): per outer iteration, n_A cycles for A u = f - B^T p
    from the previous u, then n_S steps of CG on S p = B A^-1 f - g with
    S = B A^-1 B^T + C, the lumped mass as preconditioner, started from the
    previous p with the residual B u - C p - g; inside CG every A^-1 is n_I
    cycles from zero.

Readings (listed in the design notes):
  * coarse grid: the paper runs CG on level 0; here A_0 is inverted exactly,
    so that Ahat^{-1} is a fixed symmetric positive definite operator (MINRES
    and CG on S need a fixed symmetric preconditioner).
  * Algorithm 1 writes the initial Schur residual with "+ g"; in the sign
    convention of eq. linear-system (second row B u - C p = g) the residual
    of S p = B A^-1 f - g at p is B A^-1 (f - B^T p) - C p - g, so the
    oracle takes B u - C p - g.
  * the stopping test of SCG is evaluated after every outer iteration; the
    pressure is projected to zero mean there (when it is only defined up to
    a constant), as after every UMG cycle; PMINRES projects once at the end.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .fem import Hierarchy


def lumped_mass_nu(lv, nu_macro):
    """Diagonal of the 1/nu-weighted lumped pressure mass: sum over the
    elements T around each vertex of |T| / (4 nu_T)."""
    w = lv.vol / (4.0 * np.asarray(nu_macro, dtype=np.float64)[lv.tet_macro])
    m = np.zeros(lv.N)
    for a in range(4):
        np.add.at(m, lv.tets[:, a], w)
    return m


class VelocityMG:
    """Multigrid for the velocity block, cycle V(nu1, nu2) with (FHGS, BHGS)
    smoothing.  Laplace form: the scalar A applied to each component.  D form
    (a_2): the coupled block A_2, point-block Gauss-Seidel sweeps (the 3x3
    block of each vertex solved exactly, as in the Uzawa smoother) and the
    coupled level-0 block inverted exactly."""

    def __init__(self, H: Hierarchy, nu1=1, nu2=1):
        self.H = H
        self.nu1, self.nu2 = nu1, nu2
        self.L = len(H.levels) - 1
        self.dform = H.op == "D"
        self._gs = []
        for lv in H.levels:
            dA = lv.A.diagonal()
            g = []
            for c in range(4):
                iv = np.nonzero(lv.free & (lv.colour == c))[0]
                if self.dform:
                    r3 = np.concatenate([iv, iv + lv.N, iv + 2 * lv.N])
                    blk = np.empty((iv.shape[0], 3, 3))
                    for k in range(3):
                        for m in range(3):
                            blk[:, k, m] = lv.A2[iv + k * lv.N, iv + m * lv.N].A.ravel()
                    g.append((r3, lv.A2[r3], np.linalg.inv(blk)))
                else:
                    g.append((iv, lv.A[iv], dA[iv]))
            self._gs.append(g)
        lv0 = H.levels[0]
        self._fr0 = np.nonzero(lv0.free)[0]
        if self.dform:
            f3 = np.concatenate([self._fr0 + k * lv0.N for k in range(3)])
            self._f30 = f3
            self._chol0 = sla.cho_factor(lv0.A2[f3][:, f3].toarray())
        else:
            self._chol0 = sla.cho_factor(lv0.A[self._fr0][:, self._fr0].toarray())

    def sweep(self, l, u, b, order):
        """Gauss-Seidel on A u = b over the colours in `order` (in place; the
        nodes of one colour are mutually uncoupled)."""
        if self.dform:
            uf, bf = u.reshape(-1), b.reshape(-1)
            for c in order:
                r3, rows, dinv = self._gs[l][c]
                res = (bf[r3] - rows @ uf).reshape(3, -1)
                uf[r3] += np.einsum("ikm,mi->ki", dinv, res).ravel()
            return u
        for c in order:
            idx, rows, diag = self._gs[l][c]
            for k in range(3):
                u[k][idx] += (b[k][idx] - rows @ u[k]) / diag
        return u

    def residual(self, l, u, b):
        lv = self.H.levels[l]
        if self.dform:
            r = b[:3] - (lv.A2 @ u.reshape(-1)).reshape(3, -1)
        else:
            r = np.stack([b[k] - lv.A @ u[k] for k in range(3)])
        r[:, lv.dirichlet] = 0.0
        return r

    def coarse(self, b):
        lv = self.H.levels[0]
        u = np.zeros((3, lv.N))
        if self.dform:
            u.reshape(-1)[self._f30] = sla.cho_solve(self._chol0, b[:3].reshape(-1)[self._f30])
            return u
        for k in range(3):
            u[k][self._fr0] = sla.cho_solve(self._chol0, b[k][self._fr0])
        return u

    def cycle(self, l, u, b):
        """One V(nu1, nu2) cycle on level l from u (in place, returned); the
        Dirichlet entries of u are left as they are."""
        if l == 0:
            return u + self.coarse(self.residual(0, u, b))
        for _ in range(self.nu1):
            self.sweep(l, u, b, (0, 1, 2, 3))
        P = self.H.P[l]
        r = self.residual(l, u, b)
        bc = np.stack([P.T @ r[k] for k in range(3)])
        bc[:, self.H.levels[l - 1].dirichlet] = 0.0
        ec = self.cycle(l - 1, np.zeros_like(bc), bc)
        u += np.stack([P @ ec[k] for k in range(3)])
        for _ in range(self.nu2):
            self.sweep(l, u, b, (3, 2, 1, 0))
        return u

    def inv(self, b, cycles=1):
        """Ahat^{-1} b: `cycles` cycles on the finest level from zero (velocity
        Dirichlet entries of b are ignored and those of the result are 0)."""
        u = np.zeros((3, self.H.levels[self.L].N))
        for _ in range(cycles):
            u = self.cycle(self.L, u, b)
        return u


class StokesKrylov:
    """Global Krylov solvers for K x = f~ on the finest level."""

    def __init__(self, H: Hierarchy, nu1=1, nu2=1):
        self.H = H
        self.L = len(H.levels) - 1
        self.lv = H.levels[self.L]
        self.mg = VelocityMG(H, nu1, nu2)
        self.mnu = lumped_mass_nu(self.lv, H.nu)

    # -- operators ------------------------------------------------------------
    def apply(self, x):
        from .umg import apply_level
        return apply_level(self.lv, x)

    def norm(self, r):
        return float(np.sqrt(np.sum(r[:3, self.lv.free] ** 2) + np.sum(r[3] ** 2)))

    def precond(self, v):
        """diag(Ahat, Shat)^{-1} v (eq. precond_block_diag)."""
        z = np.zeros_like(v)
        z[:3] = self.mg.inv(v[:3])
        z[3] = v[3] / self.mnu
        return z

    def project(self, x):
        if self.H.project:
            x[3] -= np.dot(self.lv.mass, x[3]) / self.lv.mass.sum()
        return x

    # -- PMINRES (Section 3.2) --------------------------------------------------
    def pminres(self, x, b, rtol=1e-8, maxit=500, iters=None):
        """Preconditioned MINRES from x (which carries the Dirichlet velocity
        values).  Stops when ||f~ - K x||_2 <= rtol ||f~ - K x_0||_2, or after
        `iters` iterations when that is given.  Returns (x, history of the
        Euclidean residual norms, from the recurrence)."""
        return minres(self.apply, self.precond, self.norm, x, b, rtol, maxit, iters,
                      finish=self.project)

    # -- SCG (Algorithm 1) ------------------------------------------------------
    def scg(self, x, b, rtol=1e-8, max_outer=200, n_A=3, n_S=3, n_I=1, outer=None):
        """Schur-complement CG from x.  The multigrid of the velocity block is
        the one given at construction (V(3,3) in Table "settings").  Stops
        when the Euclidean residual of K x = f~ falls to rtol times its initial
        value, or after `outer` outer iterations when that is given.  Returns
        (x, residual history per outer iteration)."""
        lv = self.lv
        x = x.copy()
        r0 = self.norm(b - self.apply(x))
        hist = [r0]
        if r0 == 0.0:
            return x, hist
        k_max = max_outer if outer is None else outer
        for _ in range(k_max):
            u, p = x[:3], x[3]
            # velocity: n_A cycles for A u = f - B^T p from the previous u
            t = np.stack([b[k] - lv.B[k].T @ p for k in range(3)])
            t[:, lv.dirichlet] = 0.0
            for _ in range(n_A):
                u = self.mg.cycle(self.L, u, t)
            # pressure: n_S steps of CG on S p = B A^-1 f - g
            rho = sum(lv.B[k] @ u[k] for k in range(3)) - lv.C @ p - b[3]
            z = rho / self.mnu
            d = z.copy()
            rz = float(np.dot(rho, z))
            for _ in range(n_S):
                if rz == 0.0:
                    break
                bt = np.stack([-(lv.B[k].T @ d) for k in range(3)])
                bt[:, lv.dirichlet] = 0.0
                w = self.mg.inv(bt, n_I)                 # w = -Ahat^{-1} B^T d
                y = lv.C @ d - sum(lv.B[k] @ w[k] for k in range(3))
                a = rz / float(np.dot(d, y))
                p = p + a * d
                rho = rho - a * y
                z = rho / self.mnu
                rz_new = float(np.dot(rho, z))
                d = z + (rz_new / rz) * d
                rz = rz_new
            x = np.concatenate([u, p[None, :]])
            x = self.project(x)
            r = self.norm(b - self.apply(x))
            hist.append(r)
            if outer is None and r <= rtol * r0:
                break
        return x, hist


def minres(apply, prec, norm, x, b, rtol=1e-8, maxit=500, iters=None, finish=None,
           dot=None):
    """Preconditioned MINRES (Lanczos process in the inner product of the
    preconditioner, QR factorisation of the tridiagonal matrix by Givens
    rotations).  apply(v) = K v, prec(v) = P^{-1} v (symmetric positive
    definite), norm the Euclidean norm of the stopping test.  Runs until the
    recurred residual meets rtol, or exactly `iters` iterations.  Returns
    (x, residual norms)."""
    dot = dot or (lambda a, c: float(np.sum(a * c)))
    x = x.copy()
    r = b - apply(x)
    r0 = norm(r)
    hist = [r0]
    if r0 == 0.0:
        return (finish(x) if finish else x), hist
    z = prec(r)
    beta = np.sqrt(dot(r, z))
    v_old = np.zeros_like(r)
    v = r / beta
    z = z / beta
    w_old2 = np.zeros_like(r)
    w_old = np.zeros_like(r)
    kw_old2 = np.zeros_like(r)
    kw_old = np.zeros_like(r)
    c_old, s_old, c, s = 1.0, 0.0, 1.0, 0.0
    eta = beta
    n_it = maxit if iters is None else iters
    for _ in range(n_it):
        q = apply(z)
        alpha = dot(q, z)
        v_new = q - alpha * v - beta * v_old
        z_new = prec(v_new)
        beta_new = np.sqrt(max(dot(v_new, z_new), 0.0))
        # rotations G_{j-2}, G_{j-1} applied to column j of the tridiagonal
        # matrix (beta above the diagonal, alpha on it), then G_j to zero
        # beta_new below it
        eps = s_old * beta
        dhat = c_old * beta
        delta = c * dhat + s * alpha
        ghat = -s * dhat + c * alpha
        gamma = np.hypot(ghat, beta_new)
        if gamma == 0.0:
            break
        c_new, s_new = ghat / gamma, beta_new / gamma
        tau = c_new * eta
        eta = -s_new * eta
        w = (z - eps * w_old2 - delta * w_old) / gamma
        kw = (q - eps * kw_old2 - delta * kw_old) / gamma
        x = x + tau * w
        r = r - tau * kw
        hist.append(norm(r))
        w_old2, w_old = w_old, w
        kw_old2, kw_old = kw_old, kw
        c_old, s_old, c, s = c, s, c_new, s_new
        if beta_new == 0.0:
            break
        v_old, v = v, v_new / beta_new
        z = z_new / beta_new
        beta = beta_new
        if iters is None and hist[-1] <= rtol * r0:
            break
    if finish:
        x = finish(x)
    return x, hist
