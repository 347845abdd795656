"""Checks of the shared input generator (not of the solver)."""
import numpy as np

import workloads as W


def test_manufactured_pair_solves_stokes():
    """f = -Lap(u) + grad(p) for the manufactured pair, checked with central
    differences of u; u is divergence free and vanishes on the cube boundary."""
    rng = np.random.default_rng(0)
    x = rng.uniform(0.1, 0.9, size=(50, 3))
    h = 1e-3
    lap = np.zeros((3, 50))
    div = np.zeros(50)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        up, um, u0 = (W.manufactured_velocity(x + e), W.manufactured_velocity(x - e),
                      W.manufactured_velocity(x))
        lap += (up - 2 * u0 + um) / h ** 2
        div += (up[a] - um[a]) / (2 * h)
    f = W.manufactured_forcing(x)
    assert np.allclose(f, -lap + 1.0, rtol=1e-4, atol=1e-3)
    assert np.abs(div).max() < 1e-5
    pts = W.lattice_points(1, 3)
    bnd = np.any((pts == 0.0) | (pts == 1.0), axis=1)
    assert np.abs(W.manufactured_velocity(pts[bnd])).max() < 1e-12


def test_box_mesh_is_conforming_kuhn():
    for a in (1, 2, 4):
        xyz, tet = W.box_mesh(a)
        assert tet.shape == (6 * a, 4)
        steps = np.diff(xyz[tet], axis=1)
        assert np.all(np.abs(steps).sum(axis=2) == 1) and np.all(steps.sum(axis=1) == 1)
        tags = W.face_tags(xyz, tet, a, natural_x=float(a) if a == 4 else None)
        # boundary triangles: 2 per unit square of the box surface
        assert np.count_nonzero(tags) == 2 * (4 * a + 2)
