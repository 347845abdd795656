"""Pins of the oracle's free-slip boundaries (Section 6.1): u . n = 0 at the
nodes of free-slip faces with the mass-conservative normals
n_i = <grad phi_i, 1> / |.| = -(B^T 1)_i / |.|, the tangential stress left to
the weak form.

Checked against: exact face normals on flat faces (the unit cube's planes and
the shell's flat boundary triangles); discrete mass conservation 1^T B u = 0
for every constrained u; on axis-aligned slip planes, the constrained system
and its smoother against the same problem posed with component-wise
Dirichlet conditions (u_z = 0), assembled independently of the projection
and of the tangential basis; and the multigrid solve against the direct one.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import UMG, build_hierarchy
from oracle.fem import FACE_SLIP, project_slip


def _cube_slip_z(R):
    """Unit cube, free-slip on z = 0 and z = 1, no-slip elsewhere."""
    cfg = W.WORKLOADS[1].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    tags = tags.copy()
    for t in range(tet.shape[0]):
        for f in range(4):
            face = np.delete(tet[t], f)
            z = xyz[face, 2]
            if tags[t, f] != 0 and (np.all(z == 0) or np.all(z == 1)):
                tags[t, f] = FACE_SLIP
    return cfg, xyz, tet, nu, tags


@pytest.fixture(scope="module")
def cube():
    cfg, xyz, tet, nu, tags = _cube_slip_z(3)
    return cfg, build_hierarchy(xyz, tet, nu, tags, 3)


@pytest.fixture(scope="module", params=["inner", "both"])
def shell(request):
    """The shell with free-slip on the inner sphere (workload 9) or on both."""
    cfg = W.WORKLOADS[9].with_slip(request.param).with_R(3)
    xyz, tet, nu, tags = cfg.mesh()
    return cfg, build_hierarchy(xyz, tet, nu, tags, 3, phys=cfg.physical())


def test_normals_on_flat_faces(cube, shell):
    """The slip nodes of the cube's planes z = 0, 1 (edges stay no-slip) have
    the outward normals -e_z, +e_z; a shell slip node inside a boundary
    triangle has that triangle's outward unit normal."""
    _, H = cube
    for lv in H.levels:
        n = lv.n
        X = lv.X
        inner = (X[:, 0] > 0) & (X[:, 0] < n) & (X[:, 1] > 0) & (X[:, 1] < n)
        bottom, top = inner & (X[:, 2] == 0), inner & (X[:, 2] == n)
        assert np.array_equal(lv.slip, bottom | top)
        assert np.allclose(lv.normal[bottom], [0, 0, -1], atol=1e-14)
        assert np.allclose(lv.normal[top], [0, 0, 1], atol=1e-14)
    cfg, Hs = shell
    xyz, tet, _, tags = cfg.mesh()
    phys = cfg.physical()
    lv = Hs.finest
    n = lv.n
    checked = 0
    for t, f in zip(*np.nonzero(tags == FACE_SLIP)):
        face = np.delete(tet[t], f)
        a, b, c = (xyz[v] * n for v in face)
        pa, pb, pc = (phys[v] for v in face)
        nrm = np.cross(pb - pa, pc - pa)
        nrm /= np.linalg.norm(nrm)
        if np.dot(nrm, phys[tet[t, f]] - pa) > 0:
            nrm = -nrm
        # lattice nodes strictly inside the triangle (all three barycentrics > 0)
        M = np.stack([b - a, c - a], axis=1)
        sol, *_ = np.linalg.lstsq(M, (lv.X - a).T, rcond=None)
        on = np.all(np.abs(M @ sol - (lv.X - a).T) < 1e-9, axis=0)
        s1, s2 = sol
        strict = on & (s1 > 1e-9) & (s2 > 1e-9) & (s1 + s2 < 1 - 1e-9)
        assert np.all(lv.slip[strict])
        assert np.allclose(lv.normal[strict], nrm, atol=1e-12)
        checked += strict.sum()
    assert checked >= 200


def test_mass_conservation(shell):
    """With the mass-conservative normals every constrained velocity (zero at
    the no-slip vertices, tangential at the free-slip ones) has zero net
    outflow, 1^T B u = 0 (up to rounding), while one that is only zero at the
    no-slip vertices does not."""
    _, H = shell
    for lv in H.levels:
        u = np.random.default_rng(3).normal(size=(4, lv.N))
        u[:3, lv.dirichlet] = 0.0
        one = np.ones(lv.N)
        out = sum(one @ (lv.B[k] @ u[k]) for k in range(3))
        scale = sum(np.abs(lv.B[k]) @ np.abs(u[k]) for k in range(3)).sum()
        assert abs(out) > 1e-6 * scale
        project_slip(lv, u)
        out = sum(one @ (lv.B[k] @ u[k]) for k in range(3))
        assert abs(out) < 1e-14 * scale


def _componentwise_system(lv, project):
    """The cube's system with u_z = 0 imposed as a Dirichlet condition at its
    slip nodes and u_x, u_y free there: built from A, B, C directly."""
    fr = [np.nonzero(lv.free)[0]] * 2 + [np.nonzero(lv.free & ~lv.slip)[0]]
    blocks = [[None] * 4 for _ in range(4)]
    for k in range(3):
        blocks[k][k] = lv.A[fr[k]][:, fr[k]]
        Bk = lv.B[k][:, fr[k]]
        blocks[3][k] = Bk
        blocks[k][3] = Bk.T
    blocks[3][3] = -lv.C
    return fr, sp.bmat(blocks, format="lil")


def test_flat_slip_solve_is_componentwise_dirichlet(cube):
    """On the planes z = 0, 1 the constrained problem is the one with
    u_z = 0 and u_x, u_y free there: the oracle's direct solve (tangential
    basis) equals a direct solve of that component-wise system, and its
    multigrid solve converges to it."""
    cfg, H = cube
    lv = H.finest
    umg = UMG(H)
    f = cfg.forcing_field() + W.nodal_noise(lv.N, 8, 1.0)
    b = umg.rhs(f)
    x = umg.direct_solve(b)
    fr, K = _componentwise_system(lv, H.project)
    rhs = np.concatenate([b[0][fr[0]], b[1][fr[1]], b[2][fr[2]], b[3]])
    i0 = K.shape[0] - lv.N
    K[i0, :] = 0.0
    K[:, i0] = 0.0
    K[i0, i0] = 1.0
    rhs[i0] = 0.0
    sol = spla.spsolve(K.tocsc(), rhs)
    ref = np.zeros((4, lv.N))
    o = 0
    for k in range(3):
        ref[k][fr[k]] = sol[o:o + fr[k].shape[0]]
        o += fr[k].shape[0]
    ref[3] = sol[o:]
    ref[3] -= np.dot(lv.mass, ref[3]) / lv.mass.sum()
    assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max()
    xm, hist = umg.solve(np.zeros((4, lv.N)), b, rtol=1e-10, max_cycles=60)
    assert (hist[-1] / hist[0]) ** (1.0 / (len(hist) - 1)) <= 0.3
    assert np.abs(xm - ref).max() <= 1e-7 * np.abs(ref).max()


def test_flat_slip_smoother_is_componentwise_sgs(cube):
    """On the planes z = 0, 1 the velocity sweep with slip nodes is the
    textbook symmetric Gauss-Seidel of each component over its own free set
    (u_z fixed at the slip nodes), built densely in the colour order."""
    _, H = cube
    umg = UMG(H)
    l = 1
    lv = H.levels[l]
    r = np.random.default_rng(21).normal(size=(3, lv.N))
    r[:, lv.dirichlet] = 0.0
    project_slip(lv, r)
    d = umg.sgs(l, r)
    A = lv.A.toarray()
    for k in range(3):
        free = lv.free & ~lv.slip if k == 2 else lv.free
        idx = np.nonzero(free)[0]
        idx = idx[np.argsort(lv.colour[idx], kind="stable")]
        Ak = A[np.ix_(idx, idx)]
        Dk = np.diag(np.diag(Ak))
        Lk, Uk = np.tril(Ak, -1), np.triu(Ak, 1)
        # forward (colours 0..3) then backward (3..0): (D+U)^-1 [r - L (D+L)^-1 r] + ...
        d1 = np.linalg.solve(Dk + Lk, r[k][idx])
        ref = d1 + np.linalg.solve(Dk + Uk, r[k][idx] - Ak @ d1)
        assert np.allclose(d[k][idx], ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())
        assert np.all(d[k][lv.dirichlet] == 0.0)
        assert np.abs(d[k][~free]).max() <= 1e-14 * np.abs(ref).max()


def test_shell_slip_multigrid(shell):
    """Free-slip on one or both spheres: the variable V(3,3) contracts by <= 0.45
    per cycle to a 1e-10 residual; the normal velocity vanishes at every slip
    node and the net outflow 1^T B u is zero; on level 0 the multigrid's
    dense solve in the tangential basis equals the sparse direct solve."""
    cfg, H = shell
    lv = H.finest
    umg = UMG(H, variable=True)
    b = umg.rhs(cfg.forcing_field()[:, lv.lat])
    x, hist = umg.solve(np.zeros((4, lv.N)), b, rtol=1e-10, max_cycles=80)
    rho = (hist[-1] / hist[0]) ** (1.0 / (len(hist) - 1))
    assert rho <= 0.45 and hist[-1] <= 1e-10 * hist[0]
    un = np.sum(lv.normal[lv.slip] * x[:3, lv.slip].T, axis=1)
    assert np.abs(un).max() <= 1e-12 * np.abs(x[:3]).max()
    one = np.ones(lv.N)
    out = sum(one @ (lv.B[k] @ x[k]) for k in range(3))
    assert abs(out) <= 1e-13 * sum(np.abs(lv.B[k]) @ np.abs(x[k]) for k in range(3)).sum()
    l0 = H.levels[0]
    b0 = umg.rhs(np.random.default_rng(5).normal(size=(3, l0.N)), 0)
    x0 = umg.coarse_solve(b0)
    xd = umg.direct_solve(b0, 0)
    assert np.abs(x0 - xd).max() <= 1e-9 * np.abs(xd).max()
