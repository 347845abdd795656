"""Host-side checks of the C ABI (no GPU): exported symbols, argument and mesh
validation, and the hierarchy the library builds compared with the oracle's
mesh (counts, Dirichlet sets, lattice order)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
import paper_1511_02134_amd as P
from oracle import build_hierarchy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_function():
    header = open(os.path.join(ROOT, "include", "hhg.h")).read()
    declared = set(re.findall(r"\b(hhg_[a-z_]+)\s*\(", header))
    assert declared == set(P.ABI_FUNCTIONS)
    lib = ctypes.CDLL(P.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def _mesh(cid=1):
    return W.WORKLOADS[cid].mesh()


def _expect_einval(xyz, tet, nu, tags, R=3, **opts):
    with pytest.raises(P.HHGError) as e:
        P.plan(xyz, tet, nu, tags, R, **opts)
    assert e.value.status == P.HHG_EINVAL
    return str(e.value)


def test_plan_rejects_malformed_meshes():
    xyz, tet, nu, tags = _mesh()
    assert P.plan(xyz, tet, nu, tags, 3) > 0
    bad = tet.copy()
    bad[0, [1, 2]] = bad[0, [2, 1]]                       # breaks the Kuhn path
    assert "Kuhn" in _expect_einval(xyz, bad, nu, tags)
    bad = tet.copy()
    bad[0] = bad[0][::-1]                                 # reversed (negative steps)
    _expect_einval(xyz, bad, nu, tags)
    bad = tet.copy()
    bad[0, 0] = 99                                        # vertex id out of range
    _expect_einval(xyz, bad, nu, tags)
    _expect_einval(xyz, tet[1:], nu[1:], tags[1:])        # does not tile the box
    t2 = tags.copy()
    t2[t2 == 1] = 0                                       # boundary face tagged interior
    _expect_einval(xyz, tet, nu, t2)
    t3 = tags.copy()
    inner = np.argwhere(tags == 0)[0]
    t3[tuple(inner)] = 1                                  # interior face tagged boundary
    _expect_einval(xyz, tet, nu, t3)
    t4 = tags.copy()
    t4[0, 0] = 7
    _expect_einval(xyz, tet, nu, t4)
    n2 = nu.copy()
    n2[2] = -1.0
    _expect_einval(xyz, tet, n2, tags)
    n2[2] = np.nan
    _expect_einval(xyz, tet, n2, tags)
    x2 = xyz.copy()
    x2[0, 0] = 0.5                                        # not on the integer lattice
    _expect_einval(x2, tet, nu, tags)


def test_plan_rejects_bad_arguments():
    xyz, tet, nu, tags = _mesh()
    for R in (1, 11, -3):
        _expect_einval(xyz, tet, nu, tags, R=R)
    _expect_einval(xyz, tet, nu, tags, omega=0.0)
    _expect_einval(xyz, tet, nu, tags, nu1=0, nu2=0)
    _expect_einval(xyz, tet, nu, tags, precision=3)
    _expect_einval(xyz, tet, nu, tags, coarse_maxit=0)
    _expect_einval(xyz, tet, nu, tags, coarse_solver=2)
    _expect_einval(xyz, tet, nu, tags, coarse_prec=2)
    _expect_einval(xyz, tet, nu, tags, op=2)
    _expect_einval(xyz, tet, nu, tags, op=-1)
    assert "exact coarse" in _expect_einval(xyz, tet, nu, tags, op=1, coarse_solver=1)
    _expect_einval(xyz, tet, nu, tags, ordering=3)
    assert "red-black" in _expect_einval(xyz, tet, nu, tags, ordering=2, op=1)
    assert "red-black" in _expect_einval(xyz, tet, nu, tags, ordering=2, krylov=1)
    sh = W.WORKLOADS[8].with_R(3)
    sxyz, stet, snu, stags = sh.mesh()
    assert "red-black" in _expect_einval(sxyz, stet, snu, stags, ordering=2, phys=sh.physical())
    assert "hybrid" in _expect_einval(xyz, tet, nu, tags, ordering=1, op=1)
    assert "hybrid" in _expect_einval(xyz, tet, nu, tags, ordering=1, krylov=1)
    assert P.plan(xyz, tet, nu, tags, 3, ordering=1) > P.plan(xyz, tet, nu, tags, 3)
    _expect_einval(xyz, tet, nu, tags, krylov=2)
    _expect_einval(xyz, tet, nu, tags, graphs=-1)


def test_krylov_vectors_are_reserved_on_request():
    """krylov = 1 reserves ten finest-level vectors of 4 fields (FP64) and
    nothing else; the D form and graphs change no workspace size."""
    xyz, tet, nu, tags = _mesh()
    base = P.plan(xyz, tet, nu, tags, 4)
    kry = P.plan(xyz, tet, nu, tags, 4, krylov=1)
    s = P.Solver(xyz, tet, nu, tags, 4, host_only=True)
    need = 10 * 4 * s.vec_len() * 8
    assert need <= kry - base <= need + 10 * 256
    assert P.plan(xyz, tet, nu, tags, 4, op=1) >= base
    assert P.plan(xyz, tet, nu, tags, 4, graphs=1) == base


def test_host_context_rejects_device_calls():
    xyz, tet, nu, tags = _mesh()
    s = P.Solver(xyz, tet, nu, tags, 3, host_only=True)
    st = P.lib.hhg_apply(s.ctx, 0, ctypes.c_void_p(16), ctypes.c_void_p(32), None)
    assert st == P.HHG_EINVAL
    assert b"host-only" in P.lib.hhg_last_error(s.ctx)
    st = P.lib.hhg_solve(s.ctx, ctypes.c_void_p(16), ctypes.c_void_p(32), 1e-8, 5, None, None)
    assert st == P.HHG_EINVAL
    st = P.lib.hhg_pminres(s.ctx, ctypes.c_void_p(16), ctypes.c_void_p(32), 1e-8, 5, 1, None, None)
    assert st == P.HHG_EINVAL
    st = P.lib.hhg_scg(s.ctx, ctypes.c_void_p(16), ctypes.c_void_p(32), 1e-8, 5, 3, 3, 1, 3, None,
                       None)
    assert st == P.HHG_EINVAL
    st = P.lib.hhg_vel_cycle(s.ctx, 1, 1, ctypes.c_void_p(16), ctypes.c_void_p(32), None)
    assert st == P.HHG_EINVAL


@pytest.mark.parametrize("cid", [1, 4, 5])
def test_hierarchy_matches_oracle_mesh(cid):
    """Vertex counts, DoFs and velocity Dirichlet sets of every level agree
    with the oracle's independently refined mesh."""
    R = 4
    cfg = W.WORKLOADS[cid].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    s = P.Solver(xyz, tet, nu, tags, R, host_only=True)
    H = build_hierarchy(xyz, tet, nu, tags, R)
    assert s.levels == len(H.levels)
    for l, lv in enumerate(H.levels):
        assert s.num_nodes(l) == lv.N
        assert s.num_dofs(l) == lv.ndofs()
        ijk, d = s.node_info(l)
        assert np.array_equal(ijk, lv.X)
        assert np.array_equal(d, lv.dirichlet)
        # interface vertices = vertices on macro faces: at least the box surface
        assert s.num_interface(l) >= np.count_nonzero(
            np.any((lv.X == 0) | (lv.X == np.array(lv.shape) - 1), axis=1))
        assert np.allclose(s.mass_weights(l), lv.mass, rtol=1e-13, atol=0)
        # duplicated copies make the layout a little longer than the lattice
        assert s.vec_len(l) >= lv.N


@pytest.mark.parametrize("cid,R,order", [(1, 5, 1), (4, 4, 1), (5, 4, 1), (4, 4, 0), (4, 4, 2),
                                         (5, 2, 1), (4, 3, 2), (8, 4, 1)])
def test_kernel_index_arithmetic_on_host(cid, R, order):
    """The device index code (compiled for the host) reaches exactly the
    intended vertices on every level: no access outside a macro, every vertex
    once per sweep, colour sweeps touch only their colour; the hybrid
    ordering's groups partition the interface by class and colour."""
    cfg = W.WORKLOADS[cid].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    P.Solver(xyz, tet, nu, tags, R, host_only=True, block_order=order,
             phys=cfg.physical()).check_layout()


@pytest.mark.parametrize("cid", [1, 4, 8])
def test_hybrid_groups_match_oracle_primitives(cid):
    """The library's primitive classes (from its interface keys) agree with
    the oracle's (from barycentric coordinates): every interface vertex of
    the velocity and pressure groups sits in the class the oracle gives it,
    and every macro vertex, edge and face vertex of the oracle is listed."""
    from oracle.fem import primitives
    R = 3
    cfg = W.WORKLOADS[cid].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    s = P.Solver(xyz, tet, nu, tags, R, host_only=True, ordering=1, phys=cfg.physical())
    H = build_hierarchy(xyz, tet, nu, tags, R, phys=cfg.physical())
    for l, lv in enumerate(H.levels):
        cls, _ = primitives(lv, H.macro_int, H.tet)
        lib_cls = s.primitive_classes(l)       # lattice order, -1 at hole points
        assert np.array_equal(lib_cls[lv.lat], cls)
        assert np.all(np.delete(lib_cls, lv.lat) == -1)


def _shell(R=3):
    cfg = W.WORKLOADS[8].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    return cfg, xyz, tet, nu, tags, cfg.physical()


def test_shell_hierarchy_matches_oracle_mesh():
    """General macro geometry with a hole (the spherical shell): the library's
    vertices are the oracle's (lattice points of the removed cell are not
    vertices: mass weight 0, no Dirichlet flag), with equal DoF counts,
    Dirichlet sets and lumped masses of the physical elements on every level."""
    R = 4
    cfg, xyz, tet, nu, tags, phys = _shell(R)
    s = P.Solver(xyz, tet, nu, tags, R, host_only=True, phys=phys, coarse_solver=1)
    H = build_hierarchy(xyz, tet, nu, tags, R, phys=phys)
    for l, lv in enumerate(H.levels):
        m = s.mass_weights(l)
        ijk, d = s.node_info(l)
        present = np.nonzero(m > 0)[0]
        assert np.array_equal(present, lv.lat)
        assert s.num_nodes(l) == np.prod(lv.shape) > lv.N
        assert s.num_dofs(l) == lv.ndofs()
        assert np.array_equal(ijk[lv.lat], lv.X)
        assert np.array_equal(d[lv.lat], lv.dirichlet)
        assert not np.any(d[m == 0])
        assert np.allclose(m[lv.lat], lv.mass, rtol=1e-13, atol=0)
    s.check_layout()


def test_plan_rejects_bad_physical_coordinates():
    """Physical coordinates must be finite and keep every macro's orientation;
    a mesh with a hole needs them (without them the macros must tile their
    bounding box); the shell's level-0 system fits the MINRES coarse solver."""
    cfg, xyz, tet, nu, tags, phys = _shell()
    assert P.plan(xyz, tet, nu, tags, 3, phys=phys, coarse_solver=1) > 0
    assert "tile" in _expect_einval(xyz, tet, nu, tags)
    bad = phys.copy()
    bad[5, 1] = np.inf
    assert "finite" in _expect_einval(xyz, tet, nu, tags, phys=bad, coarse_solver=1)
    bad = phys.copy()
    bad[tet[0, 1]] = 2.0 * phys[tet[0, 0]] - phys[tet[0, 1]]   # turns macro 0 inside out
    assert "inverted" in _expect_einval(xyz, tet, nu, tags, phys=bad, coarse_solver=1)
    bxyz, btet, bnu, btags = _mesh()
    flat = bxyz.copy()
    flat[:, 2] = 0.0                                      # every macro degenerate
    _expect_einval(bxyz, btet, bnu, btags, phys=flat)


@pytest.mark.parametrize("cid", [8, 9])
def test_slip_flags_match_oracle(cid):
    """Free-slip faces (tag 3): the library's free-slip and Dirichlet vertices
    are the oracle's on every level; the interface lists keep free, Dirichlet
    and free-slip vertices in that order inside each colour (layout check);
    options that do not handle free-slip faces are rejected."""
    R = 4
    cfg = W.WORKLOADS[cid].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    phys = cfg.physical()
    s = P.Solver(xyz, tet, nu, tags, R, host_only=True, phys=phys)
    s.check_layout()
    H = build_hierarchy(xyz, tet, nu, tags, R, phys=phys)
    for l, lv in enumerate(H.levels):
        _, flags = s.node_flags(l)
        assert np.array_equal(flags[lv.lat] == 1, lv.dirichlet)
        assert np.array_equal(flags[lv.lat] == 2, lv.slip)
        assert s.num_dofs(l) == lv.ndofs()
    if cid == 9:
        for bad in ({"op": 1}, {"ordering": 1}, {"coarse_solver": 1}, {"krylov": 1}):
            assert "free-slip" in _expect_einval(xyz, tet, nu, tags, R=3, phys=phys, **bad)
