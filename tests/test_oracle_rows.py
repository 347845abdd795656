"""The single-row evaluator of the oracle agrees with its global assembly
(every vertex class: interior, macro faces, edges, corners, Dirichlet and
outflow boundaries, viscosity jumps)."""
import numpy as np
import pytest

import workloads as W
from oracle import UMG, build_hierarchy
from oracle.rows import stokes_rows


@pytest.mark.parametrize("cid,op", [(1, "laplace"), (4, "laplace"), (5, "laplace"), (4, "D"),
                                   (5, "D")])
def test_rows_match_assembled_system(cid, op):
    R = 3
    cfg = W.WORKLOADS[cid].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    umg = UMG(build_hierarchy(xyz, tet, nu, tags, R, op=op))
    lv = umg.H.finest
    rng = np.random.default_rng(7)
    x = rng.normal(size=(4, lv.N))
    f = rng.normal(size=(3, lv.N))
    b_ref = umg.rhs(f)
    kx_ref = umg.apply(umg.L, x)
    verts = lv.X
    b, kx, dirich, scale = stokes_rows(xyz, tet, nu, tags, R, verts, x, f, op=op)
    # the magnitude sums bound the rows themselves (triangle inequality)
    assert np.all(scale >= np.abs(kx)) and np.all(scale >= np.abs(b))
    assert np.array_equal(dirich, lv.dirichlet)
    scale = np.abs(kx_ref).max()
    assert np.abs(kx - kx_ref).max() <= 1e-12 * scale
    assert np.abs(b - b_ref).max() <= 1e-12 * np.abs(b_ref).max()


def test_rows_match_assembled_system_on_the_shell():
    """General macro geometry with a hole: rows from the lattice patch around
    each vertex, restricted to the tetrahedra inside a macro and mapped
    affinely, equal the rows of the globally assembled shell system (fields
    in lattice order; the lattice points of the hole carry garbage that no
    row may read)."""
    R = 3
    cfg = W.WORKLOADS[8].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    phys = cfg.physical()
    umg = UMG(build_hierarchy(xyz, tet, nu, tags, R, phys=phys))
    lv = umg.H.finest
    rng = np.random.default_rng(8)
    x = rng.normal(size=(4, lv.N))
    f = rng.normal(size=(3, lv.N))
    Nlat = int(np.prod(lv.shape))
    xl = np.full((4, Nlat), 1e30)
    fl = np.full((3, Nlat), 1e30)
    xl[:, lv.lat] = x
    fl[:, lv.lat] = f
    b_ref = umg.rhs(f)
    kx_ref = umg.apply(umg.L, x)
    sel = rng.choice(lv.N, size=1500, replace=False)
    b, kx, dirich, scale = stokes_rows(xyz, tet, nu, tags, R, lv.X[sel], xl, fl, phys=phys)
    assert np.array_equal(dirich, lv.dirichlet[sel])
    assert np.abs(kx - kx_ref[:, sel]).max() <= 1e-12 * np.abs(kx_ref).max()
    assert np.abs(b - b_ref[:, sel]).max() <= 1e-12 * np.abs(b_ref).max()
