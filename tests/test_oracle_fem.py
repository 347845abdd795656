"""Pins of the oracle's mesh hierarchy and finite element matrices.

Every check compares against something the oracle does not compute itself:
closed-form integrals of linear functions, closed-form interior stencils of
the Kuhn lattice, numbers printed in the paper, and exact algebraic identities
between levels.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import build_hierarchy
from oracle.fem import DELTA, refine

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def cube3():
    xyz, tet, nu, tags = W.WORKLOADS[1].mesh()
    return build_hierarchy(xyz, tet, nu, tags, 3)


@pytest.fixture(scope="module")
def box3():
    cfg = W.WORKLOADS[4]
    xyz, tet, nu, tags = cfg.mesh()
    return build_hierarchy(xyz, tet, nu, tags, 3), nu


def _lin(X, n, b, c):
    return (X / n) @ b + c


def test_refinement_gives_kuhn_lattice():
    """Uniform refinement of the Kuhn macro mesh yields only Kuhn simplices of
    the finer lattice: vertices sorted by coordinate sum differ by three
    distinct unit steps (Section 2.1: uniform shape regularity)."""
    xyz, tet, _, _ = W.WORKLOADS[4].mesh()
    P = np.rint(xyz).astype(np.int64)[tet]
    for r in range(1, 4):
        P = refine(P)
        assert P.shape[0] == tet.shape[0] * 8 ** r
        order = np.argsort(P.sum(axis=2), axis=1)
        S = np.take_along_axis(P, order[:, :, None], axis=1)
        steps = np.diff(S, axis=1)                       # [nt,3,3]
        assert np.all(np.abs(steps).sum(axis=2) == 1)
        assert np.all(steps.sum(axis=1) == 1)            # the three steps are e_x, e_y, e_z
        vol = np.abs(np.linalg.det(steps.astype(float)))
        assert np.all(vol == 1.0)


def test_dofs_match_paper():
    gold = json.load(open(os.path.join(GOLD, "paper_serial_table.json")))
    xyz, tet, nu, tags = W.WORKLOADS[1].mesh()
    H = build_hierarchy(xyz, tet, nu, tags, 5)
    lv0 = H.levels[0]
    assert 3 * int(lv0.free.sum()) == gold["coarse_dofs"]["velocity_only"]
    assert lv0.ndofs() == gold["coarse_dofs"]["stokes"]
    for lv in H.levels[2:]:
        L = lv.R - 2
        mant, ex = gold["dofs_printed"][str(L)]
        d = lv.ndofs()
        # the table keeps two digits, sometimes rounded and sometimes cut off
        assert abs(d / 10 ** (ex - 1) - mant * 10) < 1.0, (L, d)


def test_interior_stencils_closed_form(cube3):
    """Interior rows on the Kuhn lattice: A = H(6; -1 on +-e_i; 0 on the other 8),
    C = (1/12) 6^(-2/3) H^3 x the same pattern, M = H^3/120 (48; 6 on +-e_i and
    +-(1,1,1); 4 on +-(e_i+e_j)), B_k = H^2/24 x (-6 at +e_k, +6 at -e_k, and
    +-2 at the other 12 neighbours with the signs below)."""
    lv = cube3.finest
    n, Hh = lv.n, 1.0 / lv.n
    X0 = np.array([n // 2] * 3)

    def idx(X):
        return np.searchsorted(lv.lat, X[0] + lv.shape[0] * (X[1] + lv.shape[1] * X[2]))

    i0 = idx(X0)
    axis = [np.eye(3, dtype=int)[k] for k in range(3)]
    diag2 = [np.array(v) for v in ((1, 1, 0), (0, 1, 1), (1, 0, 1))]
    d3 = np.array((1, 1, 1))
    nbrs = axis + diag2 + [d3]

    def entry(Mx, d):
        return Mx[i0, idx(X0 + d)]

    for Mx, s in ((lv.A, Hh), (lv.C, DELTA * 6 ** (-2 / 3) * Hh ** 3)):
        assert Mx[i0, i0] == pytest.approx(6 * s, rel=1e-13)
        for d in axis:
            assert entry(Mx, d) == pytest.approx(-s, rel=1e-13)
            assert entry(Mx, -d) == pytest.approx(-s, rel=1e-13)
        for d in diag2 + [d3]:
            assert abs(entry(Mx, d)) < 1e-14 * s and abs(entry(Mx, -d)) < 1e-14 * s
        row = Mx[i0].toarray().ravel()
        assert np.count_nonzero(np.abs(row) > 1e-14 * s) == 7
    s = Hh ** 3 / 120
    assert lv.M[i0, i0] == pytest.approx(48 * s, rel=1e-13)
    for d, w in [(v, 6) for v in axis + [d3]] + [(v, 4) for v in diag2]:
        assert entry(lv.M, d) == pytest.approx(w * s, rel=1e-13)
        assert entry(lv.M, -d) == pytest.approx(w * s, rel=1e-13)
    s = Hh ** 2 / 24
    for k in range(3):
        Bk = lv.B[k]
        assert abs(Bk[i0, i0]) < 1e-15
        for d in nbrs:
            if np.array_equal(d, axis[k]):
                w = -6
            elif d.sum() == 1:
                w = 2                       # other axis directions
            elif d.sum() == 3:
                w = -2
            else:                           # face diagonals: -2 if they contain e_k
                w = -2 if d[k] == 1 else 2
            assert entry(Bk, d) == pytest.approx(w * s, rel=1e-12), (k, d)
            assert entry(Bk, -d) == pytest.approx(-w * s, rel=1e-12), (k, d)


def test_linear_function_integrals(box3):
    """Assembled forms reproduce exact integrals of P1-exact (linear) fields on
    [0,2]x[0,1]^2 with per-macro viscosity (eq. varform, c_l and g_l)."""
    H, nu = box3
    lv = H.finest
    rng = np.random.default_rng(7)
    vol_box, cen = 2.0, np.array([1.0, 0.5, 0.5])
    Lx = np.array([2.0, 1.0, 1.0])
    b, c = rng.normal(size=3), rng.normal()
    d, e = rng.normal(size=3), rng.normal()
    v = _lin(lv.X, lv.n, b, c)
    w = _lin(lv.X, lv.n, d, e)
    # a_1: sum_e nu_e |b|^2 |Omega_e|, every Kuhn macro has volume 1/6
    assert v @ (lv.A @ v) == pytest.approx(np.dot(b, b) * nu.sum() / 6.0, rel=1e-12)
    # mass: int (b.x+c)(d.x+e)
    Exx = np.outer(Lx, Lx) / 4.0
    np.fill_diagonal(Exx, Lx ** 2 / 3.0)
    exact = vol_box * (b @ Exx @ d + c * (d @ cen) + e * (b @ cen) + c * e)
    assert v @ (lv.M @ w) == pytest.approx(exact, rel=1e-12)
    # c_l with h_T = |T|^(1/3) constant on a level and weight 1/nu_e per macro:
    # delta h^2 |b|^2 sum_e |Omega_e| / nu_e
    h2 = (1.0 / (6 * lv.n ** 3)) ** (2.0 / 3.0)
    inv_nu = np.sum(1.0 / nu) / 6.0
    assert v @ (lv.C @ v) == pytest.approx(DELTA * h2 * np.dot(b, b) * inv_nu, rel=1e-12)
    # b(u, q) = -int div(u) q for u = D x (div = tr D) and q = w
    D = rng.normal(size=(3, 3))
    U = (lv.X / lv.n) @ D.T                            # u_k(x) = (D x)_k
    qBu = sum(w @ (lv.B[k] @ U[:, k]) for k in range(3))
    assert qBu == pytest.approx(-np.trace(D) * vol_box * (d @ cen + e), rel=1e-12)
    # g_l(q) = -sum_e delta h^2 / nu_e int_{Omega_e} f . grad q for f = D x + f0
    # and q = w (grad q = d); every Kuhn macro of the cube [c, c+1]^3 has
    # volume 1/6, its centroid is known exactly from its vertices
    f0 = rng.normal(size=3)
    F = U + f0
    gq = sum(w @ (lv.Gf[k] @ F[:, k]) for k in range(3))
    xyz, tet, _, _ = W.WORKLOADS[4].mesh()
    exact = 0.0
    for t in range(tet.shape[0]):
        ce = xyz[tet[t]].mean(axis=0)
        exact += -DELTA * h2 / nu[t] * (1.0 / 6.0) * d @ (D @ ce + f0)
    assert gq == pytest.approx(exact, rel=1e-12)


def test_operator_structure(box3):
    H, _ = box3
    for lv in H.levels:
        for Mx in (lv.A, lv.C, lv.M):
            assert abs(Mx - Mx.T).max() < 1e-15 * abs(Mx).max()
        one = np.ones(lv.N)
        assert np.abs(lv.A @ one).max() < 1e-13 * abs(lv.A).max()     # zero row sums
        assert np.abs(lv.C @ one).max() < 1e-13 * abs(lv.C).max()
        interior = lv.free
        for k in range(3):
            assert np.abs((lv.B[k].T @ one)[interior]).max() < 1e-14   # B^T 1 = 0 inside
            assert np.abs(lv.B[k] @ one).max() < 1e-14                 # div(const) = 0
        # A is 7-point on the lattice (only axis neighbours couple)
        Acoo = lv.A.tocoo()
        dX = np.abs(lv.X[Acoo.row] - lv.X[Acoo.col]).sum(axis=1)
        nz = np.abs(Acoo.data) > 1e-14 * abs(lv.A).max()
        assert np.all(dX[nz] <= 1)


def test_colouring_separates_couplings(box3):
    """Colour (X+Y+Z) mod 4: no two nodes of one colour are coupled by A, C or
    B (15-point stencil offsets have coordinate sums +-1, +-2, +-3)."""
    H, _ = box3
    for lv in H.levels:
        for Mx in [lv.A, lv.C] + lv.B:
            m = Mx.tocoo()
            off = m.row != m.col
            nz = np.abs(m.data) > 0
            same = lv.colour[m.row] == lv.colour[m.col]
            assert not np.any(off & nz & same)


def test_galerkin_identities(box3):
    """Nested P1 spaces: P^T A_f P = A_c, P^T B_f P = B_c, P^T M_f P = M_c, and
    P^T C_f P = C_c / 4 because h_T^2 shrinks by 4 per refinement."""
    H, _ = box3
    for l in range(1, len(H.levels)):
        P, f, c = H.P[l], H.levels[l], H.levels[l - 1]
        def close(X, Y):
            return abs(X - Y).max() <= 1e-13 * abs(Y).max()
        assert close(P.T @ f.A @ P, c.A)
        assert close(P.T @ f.M @ P, c.M)
        assert close(4 * (P.T @ f.C @ P), c.C)
        for k in range(3):
            assert close(P.T @ f.B[k] @ P, c.B[k])
        # interpolation weights: 1 at coincident nodes, 1/2 at edge midpoints,
        # so an interior coarse node gathers 1 + 14/2 = 8
        colsum = np.asarray(P.sum(axis=0)).ravel()
        assert np.allclose(colsum[c.free], 8.0)
        # P reproduces constants and linear functions
        for b in np.eye(3):
            assert np.allclose(P @ _lin(c.X, c.n, b, 0.3), _lin(f.X, f.n, b, 0.3))


def test_prolongation_keeps_dirichlet_zero():
    cfg = W.WORKLOADS[5].with_R(3)
    xyz, tet, nu, tags = cfg.mesh()
    H = build_hierarchy(xyz, tet, nu, tags, 3)
    rng = np.random.default_rng(3)
    for l in range(1, len(H.levels)):
        c, f = H.levels[l - 1], H.levels[l]
        e = rng.normal(size=c.N)
        e[c.dirichlet] = 0.0
        assert np.all((H.P[l] @ e)[f.dirichlet] == 0.0)
    # the natural outflow face at x = 4 keeps its interior nodes free
    f = H.finest
    out = (f.X[:, 0] == 4 * f.n)
    inner = out & (f.X[:, 1] > 0) & (f.X[:, 1] < f.n) & (f.X[:, 2] > 0) & (f.X[:, 2] < f.n)
    assert not np.any(f.dirichlet[inner]) and np.all(f.dirichlet[out & ~inner])
    assert not H.project
