"""All-at-once Uzawa multigrid (UMG) on the assembled global matrices (oracle).

Section 3.3, eq. (Uzawa_smooth): one smoothing step is the inexact Uzawa
iteration
    u_{k+1} = u_k + Ahat^{-1} (f - A u_k - B^T p_k)
    p_{k+1} = p_k + Shat^{-1} (B u_{k+1} - C p_k - g)
with, per Section 3.5 and Table "settings" (UMG column), Ahat a symmetric
Gauss-Seidel sweep on A (forward then backward) and Shat a forward
Gauss-Seidel sweep on C with under-relaxation omega = 0.3.

Readings taken (listed again in the design notes):
  * ordering: the paper's hybrid Gauss-Seidel runs "row-wise red-black" inside
    each primitive and block-Jacobi across primitives of one class.  Here both
    sweeps use one global 4-colour ordering, colour (X+Y+Z) mod 4 of the
    integer lattice coordinates, forward = colours 0,1,2,3 and backward =
    3,2,1,0.  Nodes of one colour are never coupled by A or C (tests check
    this), so a colour is updated simultaneously.
  * "FHGS on C with under-relaxation omega" is point SOR: Shat = D_C/omega + L_C.
  * the V-cycle (Section 3.5, "V(n_pre, n_post)") restricts the residual with
    the transpose of P1 interpolation, zeroes velocity Dirichlet rows, starts
    the coarse correction from zero and uses rediscretised coarse operators
    (c_l is level dependent).  The variable cycle adds 2 pre- and 2
    post-smoothing steps per coarser level (Section 3.5).
  * coarse solve (Section 3.7 uses a loose PMINRES): here the level-0 system
    is solved exactly by a dense factorisation, bordered by the constraint
    sum_i m_i p_i = 0 when the pressure is only defined up to a constant.
  * after each cycle the finest pressure is projected to zero mean,
    p <- p - (sum m_i p_i)/(sum m_i) with m_i = int phi_i (Section 2.1, L^2_0);
    the projection is skipped when a natural (outflow) face removes the
    null space.
  * stopping criterion (Section 3.6): ||K x_k - f~||_2 <= eps ||K x_0 - f~||_2,
    Euclidean over free velocity rows and all pressure rows.
  * ordering="hybrid": the hybrid Gauss-Seidel of HHG (Section 3.4).  The
    nodes are grouped by primitive (macro vertex, edge, face, volume: the
    sub-simplex whose relative interior holds the node) and updated class by
    class, vertices -> edges -> faces -> volumes.  Primitives of one class are
    decoupled (block Jacobi): a node reads the nodes of other primitives of
    its own class as they were when the class started.  Inside a primitive
    the Gauss-Seidel order is the 4-colouring (colours 0..3 forward); the
    backward sweep reverses only the order inside the primitives (colours
    3..0), not the class order, so forward + backward (SHGS) is not
    symmetric.  The paper uses a row-wise red-black order inside a
    primitive; the 4-colouring is the order the device can run in parallel.
  * ordering="redblack": on Kuhn meshes a_1 and c_l couple only the six axis
    neighbours, whose colours differ by one, so the parities of X+Y+Z (red:
    colours 0 and 2, black: 1 and 3) are independent sets too.  The sweeps
    then run red, black (forward) and black, red (backward) -- the paper's
    red-black colouring applied to the whole lattice.
  * free-slip nodes (Section 6.1, fem.project_slip): the velocity lives in
    the tangent plane.  The velocity rows of K x, of the right-hand side and
    of a restricted residual are projected there, and so is a prolongated
    correction; the velocity sweep updates the three components of a colour
    together and projects the new values of its slip nodes (for the Laplace
    form the 3x3 centre block is a multiple of the identity, so this is the
    exact constrained point update).  The level-0 system is solved in the
    tangential basis (fem.tangential_basis).
  * D form (a_2, Section 2.1): the velocity block couples the three
    components, so the velocity sweep is a point-block Gauss-Seidel: at each
    vertex of the colour the 3x3 diagonal block is solved exactly.  The
    same 4-colouring applies (the coupling stays within the 15-point
    neighbourhood), and with the order 0 1 2 3 2 1 0 the repeated sweep of
    colour 3 is again skipped.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .fem import Hierarchy, project_slip, tangential_basis


class UMG:
    def __init__(self, H: Hierarchy, nu1=3, nu2=3, omega=0.3, variable=False,
                 p_sweep="forward", ordering="colour"):
        if ordering not in ("colour", "hybrid", "redblack"):
            raise ValueError(ordering)
        self.ordering = ordering
        self.H = H
        self.nu1, self.nu2, self.omega = nu1, nu2, omega
        self.variable = variable
        self.p_sweep = p_sweep
        self.L = len(H.levels) - 1
        self.dform = H.op == "D"
        self._gs = []
        for lv in H.levels:
            dA, dC = lv.A.diagonal(), lv.C.diagonal()
            g = {"v": [], "p": []}
            for c in range(4):
                iv = np.nonzero(lv.free & (lv.colour == c))[0]
                ip = np.nonzero(lv.colour == c)[0]
                if self.dform:
                    r3 = np.concatenate([iv, iv + lv.N, iv + 2 * lv.N])
                    blk = np.empty((iv.shape[0], 3, 3))
                    for k in range(3):
                        for l in range(3):
                            blk[:, k, l] = lv.A2[iv + k * lv.N, iv + l * lv.N].A.ravel()
                    g["v"].append((iv, r3, lv.A2[r3], np.linalg.inv(blk)))
                else:
                    g["v"].append((iv, lv.A[iv], dA[iv]))
                g["p"].append((ip, lv.C[ip], dC[ip]))
            self._gs.append(g)
        ncol = 4
        if ordering == "redblack":
            if self.dform:
                raise ValueError("red-black ordering: Laplace form only")
            ncol = 2
            for l, lv in enumerate(H.levels):
                par = lv.colour % 2
                for Mx in (lv.A, lv.C):
                    m = Mx.tocoo()
                    off = (m.row != m.col) & (m.data != 0)
                    if np.any(off & (par[m.row] == par[m.col])):
                        raise ValueError("red-black ordering: a parity couples to itself")
                dA, dC = lv.A.diagonal(), lv.C.diagonal()
                g = {"v": [], "p": []}
                for c in range(2):
                    iv = np.nonzero(lv.free & (par == c))[0]
                    ip = np.nonzero(par == c)[0]
                    g["v"].append((iv, lv.A[iv], dA[iv]))
                    g["p"].append((ip, lv.C[ip], dC[ip]))
                self._gs[l] = g
        fwd = list(range(ncol))
        self._vorder = fwd + fwd[::-1]
        self._porder = fwd + (fwd[::-1] if p_sweep == "symmetric" else [])
        self.slip = any(lv.slip is not None and lv.slip.any() for lv in H.levels)
        if self.slip and (self.dform or ordering == "hybrid"):
            raise ValueError("free-slip nodes: Laplace form with the colour ordering only")
        if ordering == "hybrid":
            if self.dform:
                raise ValueError("hybrid ordering: Laplace form only")
            self._hyb = [self._hybrid_groups(lv) for lv in H.levels]
        self._coarse = self._factor_coarse(H.levels[0])

    def _hybrid_groups(self, lv):
        """Per (class, colour): the rows updated together, their rows of A or
        C, the diagonal, and the entries towards nodes of other primitives of
        the same class (read from the class's starting values)."""
        from .fem import primitives
        cls, prim = primitives(lv, self.H.macro_int, self.H.tet)
        out = {"v": {}, "p": {}}
        for key, M, rowmask in (("v", lv.A, lv.free), ("p", lv.C, np.ones(lv.N, dtype=bool))):
            diag = M.diagonal()
            for k in range(4):
                for c in range(4):
                    idx = np.nonzero(rowmask & (cls == k) & (lv.colour == c))[0]
                    rows = M[idx].tocoo()
                    jac = (cls[rows.col] == k) & (prim[rows.col] != prim[idx[rows.row]])
                    J = sp.csr_matrix((rows.data[jac], (rows.row[jac], rows.col[jac])),
                                      shape=(idx.shape[0], lv.N))
                    out[key][(k, c)] = (idx, M[idx], J, diag[idx])
        return out

    def _hybrid_pass(self, l, kind, r, d, colours, omega=1.0):
        """One hybrid pass (classes 0..3, the given colour order inside each)
        on M d = r in place, kind "v" (A) or "p" (C, relaxed by omega)."""
        g = self._hyb[l][kind]
        for k in range(4):
            snap = d.copy()
            for c in colours:
                idx, rows, J, diag = g[(k, c)]
                if idx.shape[0] == 0:
                    continue
                s = rows @ d - J @ (d - snap)
                d[idx] += omega * (r[idx] - s) / diag
        return d

    # -- operators -------------------------------------------------------
    def rhs(self, f_nodal, l=None):
        """f~ = (M I_h f on free velocity rows, g_l(I_h f))."""
        lv = self.H.levels[self.L if l is None else l]
        b = np.zeros((4, lv.N))
        for k in range(3):
            b[k] = lv.M @ f_nodal[k]
            b[k][lv.dirichlet] = 0.0
        b[3] = sum(lv.Gf[k] @ f_nodal[k] for k in range(3))
        return project_slip(lv, b)

    def apply(self, l, x):
        """y = K x on free velocity rows and all pressure rows; x carries the
        Dirichlet values in its Dirichlet velocity entries."""
        return apply_level(self.H.levels[l], x)

    def residual(self, l, x, b):
        return b - self.apply(l, x)

    def norm(self, l, r):
        lv = self.H.levels[l]
        return float(np.sqrt(np.sum(r[:3, lv.free] ** 2) + np.sum(r[3] ** 2)))

    # -- smoother (eq. Uzawa_smooth) ---------------------------------------
    def sgs(self, l, r):
        """Ahat^{-1} r: one symmetric Gauss-Seidel sweep on A d = r from d = 0
        (Laplace form: per component; D form: r and the result are [3, N]
        and every vertex solves its 3x3 diagonal block)."""
        d = np.zeros_like(r)
        order = self._vorder
        if r.ndim == 2 and not self.dform:
            # the three components of a colour together, the new values of its
            # free-slip nodes projected onto their tangent planes
            lv = self.H.levels[l]
            for c in order:
                idx, rows, diag = self._gs[l]["v"][c]
                d[:, idx] += (r[:, idx] - (rows @ d.T).T) / diag
                sl = idx[lv.slip[idx]]
                if sl.shape[0]:
                    n = lv.normal[sl]
                    ds = d[:, sl]
                    d[:, sl] = ds - n.T * np.sum(n.T * ds, axis=0)
            return d
        if self.ordering == "hybrid":
            self._hybrid_pass(l, "v", r, d, range(4))
            return self._hybrid_pass(l, "v", r, d, range(3, -1, -1))
        if self.dform:
            N = r.shape[-1]
            rf, df = r.ravel(), d.ravel()
            for c in order:
                iv, r3, rows, dinv = self._gs[l]["v"][c]
                res = (rf[r3] - rows @ df).reshape(3, -1)
                df[r3] += np.einsum("ikl,li->ki", dinv, res).ravel()
            return df.reshape(3, N)
        for c in order:
            idx, rows, diag = self._gs[l]["v"][c]
            d[idx] += (r[idx] - rows @ d) / diag
        return d

    def sor(self, l, s):
        """Shat^{-1} s with Shat = D/omega + L (forward), or its symmetric
        version (forward then backward) when p_sweep == 'symmetric'."""
        d = np.zeros_like(s)
        if self.ordering == "hybrid":
            self._hybrid_pass(l, "p", s, d, range(4), self.omega)
            if self.p_sweep == "symmetric":
                self._hybrid_pass(l, "p", s, d, range(3, -1, -1), self.omega)
            return d
        for c in self._porder:
            idx, rows, diag = self._gs[l]["p"][c]
            d[idx] += self.omega * (s[idx] - rows @ d) / diag
        return d

    def uzawa(self, l, x, b):
        lv = self.H.levels[l]
        u, p = x[:3], x[3]
        if self.dform:
            au = (lv.A2 @ u.ravel()).reshape(3, -1)
            ru = np.stack([b[k] - au[k] - lv.B[k].T @ p for k in range(3)])
            ru[:, lv.dirichlet] = 0.0
            u += self.sgs(l, ru)
        elif self.slip:
            ru = np.stack([b[k] - lv.A @ u[k] - lv.B[k].T @ p for k in range(3)])
            ru[:, lv.dirichlet] = 0.0
            u += self.sgs(l, ru)
        else:
            for k in range(3):
                ru = b[k] - lv.A @ u[k] - lv.B[k].T @ p
                ru[lv.dirichlet] = 0.0
                u[k] += self.sgs(l, ru)
        s = sum(lv.B[k] @ u[k] for k in range(3)) - lv.C @ p - b[3]
        x[3] = p + self.sor(l, s)
        return x

    # -- grid transfer -------------------------------------------------------
    def restrict(self, l, r):
        """Residual of level l -> right-hand side of level l-1: P^T r, velocity
        Dirichlet rows of the coarse level set to zero."""
        P = self.H.P[l]
        c = self.H.levels[l - 1]
        rc = np.stack([P.T @ r[k] for k in range(4)])
        rc[:3, c.dirichlet] = 0.0
        return project_slip(c, rc)

    def prolong(self, l, e):
        P = self.H.P[l]
        return project_slip(self.H.levels[l], np.stack([P @ e[k] for k in range(4)]))

    # -- coarse grid -------------------------------------------------------
    def _coarse_system(self, lv):
        """Dense level-0 matrix over the free velocity unknowns and all
        pressures; with free-slip nodes, the velocity in the tangential
        basis T (K_T = diag(T, I)^T K diag(T, I))."""
        fr, K = self._coarse_cartesian(lv)
        if self.slip:
            T = tangential_basis(lv).toarray()
            nv = 3 * fr.shape[0]
            Z = np.zeros((T.shape[1] + lv.N, nv + lv.N))
            Z[:T.shape[1], :nv] = T.T
            Z[T.shape[1]:, nv:] = np.eye(lv.N)
            self._coarse_T = T
            K = Z @ K @ Z.T
        return fr, K

    def _coarse_cartesian(self, lv):
        fr = np.nonzero(lv.free)[0]
        nf, N = fr.shape[0], lv.N
        A = lv.A[fr][:, fr].toarray()
        K = np.zeros((3 * nf + N, 3 * nf + N))
        for k in range(3):
            Bk = lv.B[k][:, fr].toarray()
            K[k * nf:(k + 1) * nf, k * nf:(k + 1) * nf] = A
            if lv.E is not None:
                for l in range(3):
                    K[k * nf:(k + 1) * nf, l * nf:(l + 1) * nf] += lv.E[k][l][fr][:, fr].toarray()
            K[3 * nf:, k * nf:(k + 1) * nf] = Bk
            K[k * nf:(k + 1) * nf, 3 * nf:] = Bk.T
        K[3 * nf:, 3 * nf:] = -lv.C.toarray()
        return fr, K

    def _factor_coarse(self, lv):
        fr, K = self._coarse_system(lv)
        if self.H.project:
            n = K.shape[0]
            Kb = np.zeros((n + 1, n + 1))
            Kb[:n, :n] = K
            Kb[n, n - lv.N:n] = lv.mass
            Kb[n - lv.N:n, n] = lv.mass
            K = Kb
        return fr, sla.lu_factor(K)

    def coarse_solve(self, b):
        """Exact solution of the level-0 system (mean-zero pressure if needed)."""
        lv = self.H.levels[0]
        fr, lu = self._coarse
        nf = fr.shape[0]
        rv = np.concatenate([b[0][fr], b[1][fr], b[2][fr]])
        if self.slip:
            rv = self._coarse_T.T @ rv
        rhs = np.concatenate([rv, b[3]])
        if self.H.project:
            rhs = np.append(rhs, 0.0)
        sol = sla.lu_solve(lu, rhs)
        nv = rv.shape[0]
        sv = sol[:nv] if not self.slip else self._coarse_T @ sol[:nv]
        x = np.zeros((4, lv.N))
        for k in range(3):
            x[k][fr] = sv[k * nf:(k + 1) * nf]
        x[3] = sol[nv:nv + lv.N]
        return x

    # -- cycle -----------------------------------------------------------------
    def steps(self, l, top=None):
        """Smoothing steps on level l of a cycle whose top level is `top`: the
        variable V-cycle adds two per level below the top (Section 3.5)."""
        top = self.L if top is None else top
        extra = 2 * (top - l) if self.variable else 0
        return self.nu1 + extra, self.nu2 + extra

    def vcycle(self, l, x, b, top=None):
        if l == 0:
            return x + self.coarse_solve(self.residual(0, x, b))
        pre, post = self.steps(l, top)
        for _ in range(pre):
            self.uzawa(l, x, b)
        bc = self.restrict(l, self.residual(l, x, b))
        ec = self.vcycle(l - 1, np.zeros_like(bc), bc, top)
        x += self.prolong(l, ec)
        for _ in range(post):
            self.uzawa(l, x, b)
        return x

    def fmg(self, bs, xbc, cycles=1):
        """Full multigrid (Section 5, Figure "FMG"): bs[l] the right-hand side
        and xbc[l] the Dirichlet velocity values of level l.  Level 0 is solved
        exactly; every finer level starts from the interpolated solution of the
        level below (its Dirichlet values restored) and runs `cycles` V-cycles
        with itself as the top level, each followed by the projection.
        Returns the solutions of all levels."""
        lv = self.H.levels[0]
        x = np.zeros((4, lv.N))
        x[:3, lv.dirichlet] = xbc[0][:3, lv.dirichlet]
        x = self.project(x + self.coarse_solve(self.residual(0, x, bs[0])), 0)
        xs = [x]
        for l in range(1, self.L + 1):
            lv = self.H.levels[l]
            x = self.prolong(l, x)
            x[:3, lv.dirichlet] = xbc[l][:3, lv.dirichlet]
            for _ in range(cycles):
                x = self.project(self.vcycle(l, x, bs[l], top=l), l)
            xs.append(x)
        return xs

    def project(self, x, l=None):
        lv = self.H.levels[self.L if l is None else l]
        if self.H.project:
            x[3] -= np.dot(lv.mass, x[3]) / lv.mass.sum()
        return x

    def cycle(self, x, b):
        """One solver iteration: a V-cycle on the finest level, then the
        mean-zero projection of the pressure."""
        x = self.vcycle(self.L, x, b)
        return self.project(x)

    def solve(self, x, b, rtol=1e-8, max_cycles=100, callback=None):
        L = self.L
        r0 = self.norm(L, self.residual(L, x, b))
        hist = [r0]
        if r0 == 0.0:
            return x, hist
        for _ in range(max_cycles):
            x = self.cycle(x, b)
            r = self.norm(L, self.residual(L, x, b))
            hist.append(r)
            if callback is not None:
                callback(x, r)
            if r <= rtol * r0:
                break
        return x, hist

    # -- direct reference ------------------------------------------------------
    def direct_solve(self, b, l=None, xbc=None):
        l = self.L if l is None else l
        return direct_solve(self.H.levels[l], b, self.H.project, xbc)


def apply_level(lv, x):
    """y = K x on one level (same as UMG.apply, usable without a hierarchy)."""
    y = np.zeros_like(x)
    au = (lv.A2 @ x[:3].ravel()).reshape(3, -1) if lv.A2 is not None else None
    for k in range(3):
        y[k] = (au[k] if au is not None else lv.A @ x[k]) + lv.B[k].T @ x[3]
        y[k][lv.dirichlet] = 0.0
    y[3] = sum(lv.B[k] @ x[k] for k in range(3)) - lv.C @ x[3]
    return project_slip(lv, y)


def direct_solve(lv, b, project, xbc=None):
    """Sparse direct solution of K x = b - K x_D on one level; used as a
    reference at small sizes.  xbc carries Dirichlet velocity values.  When the
    pressure is only defined up to a constant, the pressure of node 0 is fixed
    to zero (the remaining system is regular for a compatible right-hand side)
    and the result is projected to zero mean."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    fr = np.nonzero(lv.free)[0]
    nf, N = fr.shape[0], lv.N
    xd = np.zeros((4, N)) if xbc is None else xbc.copy()
    xd[:3, fr] = 0.0
    xd[3] = 0.0
    r = b - apply_level(lv, xd)
    A = lv.A[fr][:, fr]
    blocks = [[None] * 4 for _ in range(4)]
    for k in range(3):
        blocks[k][k] = A
        if lv.E is not None:
            for l in range(3):
                Ekl = lv.E[k][l][fr][:, fr]
                blocks[k][l] = Ekl if blocks[k][l] is None else blocks[k][l] + Ekl
        Bk = lv.B[k][:, fr]
        blocks[3][k] = Bk
        blocks[k][3] = Bk.T
    blocks[3][3] = -lv.C
    K = sp.bmat(blocks, format="csr")
    rhs = np.concatenate([r[0][fr], r[1][fr], r[2][fr], r[3]])
    slip = lv.slip is not None and lv.slip.any()
    if slip:
        # free-slip nodes: the velocity in the tangential basis
        T = tangential_basis(lv)
        Z = sp.block_diag([T, sp.identity(N)], format="csr")
        K = Z.T @ K @ Z
        rhs = Z.T @ rhs
    K = K.tolil()
    nv = K.shape[0] - N
    if project:
        i0 = nv
        K[i0, :] = 0.0
        K[:, i0] = 0.0
        K[i0, i0] = 1.0
        rhs[i0] = 0.0
    sol = spla.spsolve(K.tocsc(), rhs)
    sv = T @ sol[:nv] if slip else sol[:nv]
    x = xd.copy()
    for k in range(3):
        x[k][fr] = sv[k * nf:(k + 1) * nf]
    x[3] = sol[nv:nv + N]
    if project:
        x[3] -= np.dot(lv.mass, x[3]) / lv.mass.sum()
    return x
