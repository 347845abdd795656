"""Full-size checks in the benchmark's launch configuration (default options,
XCD-aware tile order), on the target workloads themselves: unit cube at 7
refinements in FP64 (Laplace and D form), at 8 refinements in mixed precision
and in FP64 (with the 4-colour and with the red-black order, the benchmark's),
and the channel at 7 refinements in mixed precision.

The oracle cannot assemble these systems, so it evaluates rows one by one
(oracle.rows, pinned against its global assembly) at sampled vertices: every
class of vertex (macro interiors, macro faces, edges and corners, Dirichlet
walls, the outflow, interfaces between unit cubes) is sampled.  The GPU's
right-hand side and final residual f~ - K x must agree with the oracle's rows
at those vertices, and the GPU's residual norm must meet the 1e-8 target.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.rows import stokes_rows

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"\n[case] {msg}", flush=True)


def _sample(cfg, seed, per_set=40):
    """Lattice vertices: uniform random ones plus random ones on the planes of
    the Kuhn split (x' = y, y = z, x' = z, x' = y = z with x' the coordinate
    inside a unit cube), the cube interfaces x' = 0, the walls and the
    corners of the box."""
    n = 2 ** cfg.R
    ext = np.array([cfg.a * n, n, n])
    rng = np.random.default_rng(seed)
    pts = [rng.integers(0, ext + 1, size=(4 * per_set, 3))]

    def rand(k):
        return rng.integers(0, ext + 1, size=(per_set, 3))

    for rule in ("xy", "yz", "xz", "xyz", "cube", "wall0", "wall1", "x0", "xend"):
        P = rand(per_set)
        cx = P[:, 0] // n * n          # origin of the unit cube in x
        xl = P[:, 0] - cx
        if rule == "xy":
            P[:, 1] = np.minimum(xl, n)
        elif rule == "yz":
            P[:, 2] = P[:, 1]
        elif rule == "xz":
            P[:, 2] = np.minimum(xl, n)
        elif rule == "xyz":
            P[:, 1] = xl
            P[:, 2] = xl
        elif rule == "cube":
            P[:, 0] = cx
        elif rule == "wall0":
            P[:, 1] = 0
        elif rule == "wall1":
            P[:, 2] = n
        elif rule == "x0":
            P[:, 0] = 0
        elif rule == "xend":
            P[:, 0] = ext[0]
        pts.append(P)
    corners = np.array([[x, y, z] for x in (0, ext[0]) for y in (0, n) for z in (0, n)])
    pts.append(corners)
    P = np.unique(np.concatenate(pts), axis=0)
    return P[np.all((P >= 0) & (P <= ext), axis=1)]


# (workload, velocity form, precision, cycle): the unit cube at 7 refinements
# in V(3,3) (Laplace and D form); the unit cube at 8 refinements in mixed
# precision and in FP64 (the benchmark's workload) and the channel in mixed
# precision, all three in the variable V(3,3) cycle, where the plain V(3,3)
# cycle contracts by more than 0.3 per cycle at these sizes
FULL = [(2, "laplace", "fp64", 0, 0), (3, "laplace", "mixed", 1, 0), (3, "laplace", "fp64", 1, 0),
        (3, "laplace", "fp64", 1, 2), (3, "laplace", "mixed", 1, 2), (5, "laplace", "mixed", 1, 0),
        (2, "D", "fp64", 0, 0)]


@pytest.mark.parametrize("cid,op,prec,cycle,ordering", FULL)
def test_full_size_solve_residual_rows(cid, op, prec, cycle, ordering):
    import paper_1511_02134_amd as P
    cfg = W.WORKLOADS[cid]
    xyz, tet, nu, tags = cfg.mesh()
    precision = 1 if prec == "mixed" else 0
    _announce(f"{cfg.name}: R={cfg.R}, precision={prec}, form={op}, "
              f"cycle={'Vvar' if cycle else 'V'}, ordering={ordering}")
    s = P.Solver(xyz, tet, nu, tags, cfg.R, precision=precision, op=1 if op == "D" else 0,
                 cycle=cycle, ordering=ordering)
    dev = torch.device("cuda")
    f = cfg.forcing_field()
    x0 = np.zeros((4, s.num_nodes()))
    _, dmask = s.node_info()
    x0[:3] = np.where(dmask[None, :], cfg.dirichlet_field(), 0.0)
    b = s.rhs(s.scatter(torch.tensor(f, device=dev)))
    x = s.scatter(torch.tensor(x0, device=dev))
    info = s.solve(x, b, rtol=1e-8, max_cycles=100)
    print(f"{info['cycles']} cycles, rel. residual {info['rel_res']:.2e}, "
          f"mean contraction {info['rho_mean']:.3f}, {info['t_solve_ms']:.1f} ms", flush=True)
    assert info["status"] == P.HHG_OK
    assert info["rel_res"] <= 1e-8
    if cycle == 1:
        assert info["rho_mean"] <= 0.3
    r, rnorm = s.residual(x, b)
    assert rnorm <= 1e-8 * info["r0"] * (1 + 1e-12)

    xg = s.gather(x).cpu().numpy()
    bg = s.gather(b).cpu().numpy()
    rg = s.gather(r).cpu().numpy()
    verts = _sample(cfg, seed=100 + cid)
    nx, ny = cfg.a * 2 ** cfg.R + 1, 2 ** cfg.R + 1
    idx = verts[:, 0] + nx * (verts[:, 1] + ny * verts[:, 2])
    b_o, kx_o, dirich, scale = stokes_rows(xyz, tet, nu, tags, cfg.R, verts, xg, f, op=op)
    assert np.array_equal(dirich, dmask[idx])
    # rows of f~ and of the final residual f~ - K x, each against the sum of
    # the magnitudes of its products (FP64 rounding of ~100 products in any
    # order stays far below 1e-13 of it; a wrong coefficient or tap does not)
    scale = np.maximum(scale, np.finfo(float).tiny)
    eb = np.abs(bg[:, idx] - b_o) / scale
    er = np.abs(rg[:, idx] - (b_o - kx_o)) / scale
    print(f"{len(verts)} sampled vertices: max difference in f~ {eb.max():.2e}, "
          f"in f~ - K x {er.max():.2e} (relative to the row's magnitude sum)", flush=True)
    assert eb.max() <= 1e-13
    assert er.max() <= 1e-13
