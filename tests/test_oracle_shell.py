"""Pins of the oracle on a general (non-Kuhn) macro mesh: the spherical shell
0.55 < |x| < 1 of Section 4.4, built as the hollow cube [0,3]^3 minus its
central cell (156 Kuhn macros in lattice coordinates) with its vertices put
on the two spheres by the equiangular cubed-sphere map, so that every macro
is an arbitrary affine tetrahedron.

Each check compares with something the oracle does not compute: the volume of
the polyhedral shell from its boundary triangles (divergence theorem),
integrals of linear fields over the macro tetrahedra from their physical
vertices (exact P1 quadrature), identities of nested P1 spaces, and the
algebraic structure of the forms.  The host hierarchy of the library is
checked against the oracle's independently refined mesh.
"""
import numpy as np
import pytest

import workloads as W
from oracle import build_hierarchy
from oracle.fem import DELTA

R_IN, R_OUT = 0.55, 1.0


@pytest.fixture(scope="module")
def shell():
    cfg = W.WORKLOADS[8]
    xyz, tet, nu, tags = cfg.mesh()
    phys = cfg.physical()
    H = build_hierarchy(xyz, tet, nu, tags, 3, phys=phys)
    return xyz, tet, tags, phys, H


def _macro_volumes(phys, tet):
    """Unsigned volumes and centroids of the macro tetrahedra."""
    P = phys[tet]
    E = P[:, 1:] - P[:, :1]
    return np.abs(np.linalg.det(E)) / 6.0, P.mean(axis=1)


def _boundary_volume(phys, tet, tags):
    """Volume enclosed by the tagged boundary triangles, (1/6) sum det(a, b, c)
    over outward oriented triangles; each triangle is oriented away from the
    vertex of its macro opposite to it."""
    vol = 0.0
    for t in range(tet.shape[0]):
        for f in range(4):
            if tags[t, f] == 0:
                continue
            a, b, c = (phys[v] for v in np.delete(tet[t], f))
            opp = phys[tet[t, f]]
            if np.dot(np.cross(b - a, c - a), opp - a) > 0:
                b, c = c, b
            vol += np.linalg.det(np.stack([a, b, c])) / 6.0
    return vol


def test_shell_mesh(shell):
    """156 conforming macros, every vertex on one of the two spheres, each
    macro keeping the orientation of its lattice tetrahedron, the 12 inner
    and 108 outer boundary triangles tagged Dirichlet, and macro volumes that
    add up to the boundary volume."""
    xyz, tet, tags, phys, _ = shell
    assert tet.shape[0] == 156
    r = np.linalg.norm(phys, axis=1)
    assert np.all(np.isclose(r, R_IN) | np.isclose(r, R_OUT))
    sp = np.linalg.det(phys[tet][:, 1:] - phys[tet][:, :1])
    sl = np.linalg.det(xyz[tet][:, 1:] - xyz[tet][:, :1])
    assert np.all(sp * sl > 0) and np.all(np.abs(sl) == 1.0)
    vols, _ = _macro_volumes(phys, tet)
    ntri = np.count_nonzero(tags)
    assert ntri == 12 + 108
    inner = 0
    for t, f in zip(*np.nonzero(tags)):
        face = np.delete(tet[t], f)
        rr = np.linalg.norm(phys[face], axis=1)
        assert np.allclose(rr, rr[0])
        inner += np.isclose(rr[0], R_IN)
    assert inner == 12
    # the inner boundary is the inscribed cube of the inner sphere
    side = 2.0 * R_IN / np.sqrt(3.0)
    vb = _boundary_volume(phys, tet, tags)
    assert vols.sum() == pytest.approx(vb, rel=1e-13)
    outer_tags = tags.copy()
    for t, f in zip(*np.nonzero(tags)):
        if np.isclose(np.linalg.norm(phys[np.delete(tet[t], f)[0]]), R_IN):
            outer_tags[t, f] = 0
    assert vb == pytest.approx(_boundary_volume(phys, tet, outer_tags) - side ** 3, rel=1e-13)
    # the polyhedral shell lies inside the true one
    assert 0 < vb < 4.0 / 3.0 * np.pi * (R_OUT ** 3 - R_IN ** 3)


def test_refined_vertices_are_affine_images(shell):
    """Every refined vertex sits at the barycentric combination of its macro's
    physical vertices; workloads.refined_points (written independently of the
    oracle's refinement) gives the same coordinates in lattice order."""
    xyz, tet, tags, phys, H = shell
    lv = H.finest
    pts = W.refined_points(xyz, tet, phys, lv.R)
    assert np.array_equal(np.nonzero(~np.isnan(pts[:, 0]))[0], lv.lat)
    assert np.abs(pts[lv.lat] - lv.Xphys).max() < 1e-14
    r = np.linalg.norm(lv.Xphys, axis=1)
    assert r.min() >= R_IN * np.sqrt(1.0 / 3.0) - 1e-12 and r.max() <= R_OUT + 1e-12


def test_linear_field_integrals(shell):
    """The refined forms integrate linear fields exactly over the polyhedral
    shell: every identity is summed over the 156 macro tetrahedra from their
    physical vertices (nu = 1, h_T^2 = (|T_macro| / 8^R)^(2/3) since uniform
    refinement splits a tetrahedron into 8 of equal volume)."""
    xyz, tet, tags, phys, H = shell
    lv = H.finest
    X = lv.Xphys
    rng = np.random.default_rng(11)
    b, c = rng.normal(size=3), rng.normal()
    d, e = rng.normal(size=3), rng.normal()
    v, w = X @ b + c, X @ d + e
    vols, cen = _macro_volumes(phys, tet)
    # a_1: |b|^2 |Omega|
    assert v @ (lv.A @ v) == pytest.approx(np.dot(b, b) * vols.sum(), rel=1e-12)
    # mass: exact P1 x P1 quadrature on each macro, |T|/20 (sum f_i g_i + sum f_i sum g_j)
    fv = phys[tet] @ b + c
    gv = phys[tet] @ d + e
    exact = np.sum(vols / 20.0 * (np.sum(fv * gv, axis=1) + fv.sum(axis=1) * gv.sum(axis=1)))
    assert v @ (lv.M @ w) == pytest.approx(exact, rel=1e-12)
    # c_l: delta sum_T h_T^2 |b|^2 |T|
    hT2 = (vols / 8.0 ** lv.R) ** (2.0 / 3.0)
    assert v @ (lv.C @ v) == pytest.approx(DELTA * np.dot(b, b) * np.sum(hT2 * vols), rel=1e-12)
    # b(u, q) = -int div(u) q for u = D x and q = w
    D = rng.normal(size=(3, 3))
    U = X @ D.T
    qBu = sum(w @ (lv.B[k] @ U[:, k]) for k in range(3))
    assert qBu == pytest.approx(-np.trace(D) * np.sum(vols * (cen @ d + e)), rel=1e-12)
    # g_l(q) = -delta sum_T h_T^2 int_T f . grad q for f = D x + f0
    f0 = rng.normal(size=3)
    F = U + f0
    gq = sum(w @ (lv.Gf[k] @ F[:, k]) for k in range(3))
    exact = -DELTA * np.sum(hT2 * vols * ((cen @ D.T + f0) @ d))
    assert gq == pytest.approx(exact, rel=1e-12)


def test_operator_structure(shell):
    """Symmetric A, C, M; constants in the kernels of A, C and B; B^T 1 = 0 at
    interior vertices; the four colours (X+Y+Z) mod 4 still separate every
    coupling; and A is a genuine 15-point stencil (non-axis couplings)."""
    *_, H = shell
    for lv in H.levels:
        for Mx in (lv.A, lv.C, lv.M):
            assert abs(Mx - Mx.T).max() < 1e-15 * abs(Mx).max()
        one = np.ones(lv.N)
        assert np.abs(lv.A @ one).max() < 1e-13 * abs(lv.A).max()
        assert np.abs(lv.C @ one).max() < 1e-13 * abs(lv.C).max()
        for k in range(3):
            assert np.abs((lv.B[k].T @ one)[lv.free]).max() < 1e-14
            assert np.abs(lv.B[k] @ one).max() < 1e-14
        for Mx in [lv.A, lv.C] + lv.B:
            m = Mx.tocoo()
            off = (m.row != m.col) & (np.abs(m.data) > 0)
            assert not np.any(off & (lv.colour[m.row] == lv.colour[m.col]))
        Acoo = lv.A.tocoo()
        dX = np.abs(lv.X[Acoo.row] - lv.X[Acoo.col]).sum(axis=1)
        nz = np.abs(Acoo.data) > 1e-12 * abs(lv.A).max()
        assert np.any(dX[nz] > 1)
        assert np.all(dX[nz] <= 3)


def test_galerkin_identities(shell):
    """Nested P1 spaces on affinely refined macros: P^T K_f P = K_c for A, B
    and M, and 4 P^T C_f P = C_c (h_T^2 shrinks by 4 per refinement)."""
    *_, H = shell
    for l in range(1, len(H.levels)):
        P, f, c = H.P[l], H.levels[l], H.levels[l - 1]

        def close(X, Y):
            return abs(X - Y).max() <= 1e-13 * abs(Y).max()
        assert close(P.T @ f.A @ P, c.A)
        assert close(P.T @ f.M @ P, c.M)
        assert close(4 * (P.T @ f.C @ P), c.C)
        for k in range(3):
            assert close(P.T @ f.B[k] @ P, c.B[k])
        # P reproduces linear functions of the physical coordinates
        for b in np.eye(3):
            assert np.allclose(P @ (c.Xphys @ b + 0.3), f.Xphys @ b + 0.3)
