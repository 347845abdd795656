"""Rows of the discrete Stokes system at chosen vertices (test infrastructure).

For problems too large to assemble, single rows of f~ and K x are formed from
the element matrices of the tetrahedra around the vertex, with the bilinear
forms of Section 2.1 exactly as in the global assembly (fem.assemble_level):

  a_1:  nu_T |T| grad phi_a . grad phi_b                    (per component)
  a_2:  a_1 + nu_T |T| d_l phi_a d_k phi_b (row component k, column l; D form)
  b:    b(phi_v e_k, phi_q) = -(|T|/4) d_k phi_v
  c_l:  delta h_T^2 / nu_T |T| grad phi_a . grad phi_b,  h_T = |T|^(1/3)
  f~:   M I_h f on free velocity rows (M_T = |T|/20 (1 + delta_ab)),
        g_l(phi_a) = -sum_k delta h_T^2 / nu_T (|T|/4) d_k phi_a sum_{b in T} f_k(b)

The uniformly refined Kuhn macro mesh is the Kuhn triangulation of the
lattice: every lattice cube [c, c+1] is split into the 6 tetrahedra
{c, c+e_s0, c+e_s0+e_s1, c+(1,1,1)}.  The tetrahedra around a vertex are
therefore those of the 8 cubes that have it as a corner and contain it.  The
viscosity of a tetrahedron is that of the macro containing its centroid.
"""
from __future__ import annotations

import itertools

import numpy as np

from .fem import DELTA, _dirichlet_nodes, macro_maps, p1_geometry

_E = np.eye(3, dtype=np.int64)
_KUHN = [np.array([np.zeros(3, np.int64), _E[s[0]], _E[s[0]] + _E[s[1]], np.ones(3, np.int64)])
         for s in itertools.permutations(range(3))]


def _patch(X, ext):
    """Lattice tetrahedra [m,4,3] around vertex X (integer coordinates) in the
    lattice 0 <= X <= ext, and the local index of X in each."""
    tets, loc = [], []
    for d in itertools.product((0, 1), repeat=3):
        c = X - np.array(d)
        if np.any(c < 0) or np.any(c + 1 > ext):
            continue
        for K in _KUHN:
            V = c[None, :] + K
            hit = np.nonzero(np.all(V == X[None, :], axis=1))[0]
            if hit.size:
                tets.append(V)
                loc.append(int(hit[0]))
    return np.array(tets), np.array(loc)


def _macro_of(points, xyz, tet, holes=False):
    """Index of the macro tetrahedron containing each point (strictly inside);
    with holes, -1 for points in no macro."""
    P = xyz[tet]                                   # [nt,4,3]
    J = P[:, 1:, :] - P[:, :1, :]
    Jinv = np.linalg.inv(np.transpose(J, (0, 2, 1)))   # maps x - x0 to (l1, l2, l3)
    out = np.full(points.shape[0], -1, dtype=np.int64)
    for t in range(tet.shape[0]):
        lam = (points - P[t, 0]) @ Jinv[t].T
        lam = np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)
        inside = np.all(lam > 1e-12, axis=1) & (out < 0)
        out[inside] = t
    if np.any(out < 0) and not holes:
        raise ValueError("a lattice tetrahedron lies in no macro")
    return out


def stokes_rows(xyz, tet, nu, face_bc, R, verts, x, f, op="laplace", phys=None):
    """Rows of f~ and of K x at the vertices verts [m,3] (integer lattice
    coordinates at 2^R per unit length).

    phys: physical coordinates of the macro vertices (general geometry, as in
    fem.build_hierarchy); the lattice tetrahedra around a vertex then keep
    only those inside a macro and are carried to physical space by their
    macro's affine map.

    x [4,N] (velocity with its Dirichlet values, pressure) and f [3,N] are
    nodal fields in lattice order (index X + nx (Y + ny Z)).  Returns
    (b [4,m], Kx [4,m], dirichlet [m], scale [4,m]); velocity rows of
    Dirichlet vertices are zero in b and Kx, as in the assembled system.
    scale is the sum of the magnitudes of all products entering the row of
    b and of K x (|M||f| + |K||x| elementwise): the size that rounding
    errors of any summation order are relative to."""
    n = 1 << R
    macro_int = np.rint(xyz).astype(np.int64)
    ext = macro_int.max(axis=0) * n
    nx, ny = ext[0] + 1, ext[1] + 1
    nu = np.asarray(nu, dtype=np.float64)
    verts = np.asarray(verts, dtype=np.int64)
    dirich = _dirichlet_nodes(verts, n, macro_int, tet, face_bc)
    maps = None if phys is None else macro_maps(macro_int, tet, phys)
    b = np.zeros((4, verts.shape[0]))
    kx = np.zeros((4, verts.shape[0]))
    scale = np.zeros((4, verts.shape[0]))
    for m, X in enumerate(verts):
        T, a = _patch(X, ext)
        cen = T.mean(axis=1).astype(np.float64) / n
        mac = _macro_of(cen, macro_int.astype(np.float64), tet, holes=maps is not None)
        keep = mac >= 0
        T, a, mac = T[keep], a[keep], mac[keep]
        if maps is None:
            vol, G = p1_geometry(T.astype(np.float64) / n)
        else:
            L0, O, F = maps
            Pt = O[mac][:, None, :] + np.einsum("tqd,tde->tqe",
                                                T.astype(np.float64) / n - L0[mac][:, None, :],
                                                F[mac])
            vol, G = p1_geometry(Pt)
        nuT = nu[mac]
        hT2 = vol ** (2.0 / 3.0)
        idx = T[..., 0] + nx * (T[..., 1] + ny * T[..., 2])      # [m,4] node indices
        Ga = G[np.arange(T.shape[0]), a]                          # [m,3] grad phi of the vertex
        GG = np.einsum("tk,tbk->tb", Ga, G)                       # grad phi_a . grad phi_b
        u = x[:3][:, idx]                                         # [3,m,4]
        p = x[3][idx]                                             # [m,4]
        fk = f[:, idx]                                            # [3,m,4]
        Mrow = (vol / 20.0)[:, None] * (1.0 + (np.arange(4)[None, :] == a[:, None]))
        for k in range(3):
            au = (nuT * vol)[:, None] * GG * u[k]
            if op == "D":
                au = au + sum((nuT * vol)[:, None] * Ga[:, l, None] * G[:, :, k] * u[l]
                              for l in range(3))
            btp = -(vol / 4.0)[:, None] * Ga[:, k, None] * p
            mf = Mrow * fk[k]
            kx[k, m] = 0.0 if dirich[m] else np.sum(au) + np.sum(btp)
            b[k, m] = 0.0 if dirich[m] else np.sum(mf)
            scale[k, m] = np.abs(au).sum() + np.abs(btp).sum() + np.abs(mf).sum()
        bu = [-(vol / 4.0)[:, None] * G[:, :, k] * u[k] for k in range(3)]
        cp = (DELTA * hT2 * vol / nuT)[:, None] * GG * p
        gf = [-(DELTA * hT2 * vol / (4.0 * nuT))[:, None] * Ga[:, k, None] * fk[k] for k in range(3)]
        kx[3, m] = sum(np.sum(t) for t in bu) - np.sum(cp)
        b[3, m] = sum(np.sum(t) for t in gf)
        scale[3, m] = sum(np.abs(t).sum() for t in bu + gf) + np.abs(cp).sum()
    return b, kx, dirich, scale
