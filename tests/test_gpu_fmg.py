"""Full multigrid through the C ABI (hhg_rhs_level, hhg_fmg) against the
oracle's full multigrid (Section 5): every level's solution, for one and two
variable V(2,2) cycles per level, on the analytic solution of the efficiency
study (non-homogeneous Dirichlet data) and on the box with per-macro
viscosity, in the Laplace and the D form."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import UMG, build_hierarchy

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("cid,R,cycles,op", [(6, 4, 1, "laplace"), (6, 4, 2, "laplace"),
                                             (4, 4, 1, "laplace"), (6, 3, 2, "laplace"),
                                             (6, 4, 1, "D"), (4, 4, 2, "D")])
def test_fmg_matches_oracle(cid, R, cycles, op):
    import paper_1511_02134_amd as P
    cfg = W.WORKLOADS[cid].with_R(R)
    print(f"\n[case] fmg {cfg.name} R={R} cycles={cycles} form={op}", flush=True)
    xyz, tet, nu, tags = cfg.mesh()
    s = P.Solver(xyz, tet, nu, tags, R, nu1=2, nu2=2, cycle=1, op=1 if op == "D" else 0)
    umg = UMG(build_hierarchy(xyz, tet, nu, tags, R, op=op), nu1=2, nu2=2, variable=True)
    xs, bs, bs_o, xbc = [], [], [], []
    for l in range(s.L + 1):
        c = cfg.with_R(2 + l)
        f = c.forcing_field()
        _, dmask = s.node_info(l)
        x0 = np.zeros((4, s.num_nodes(l)))
        x0[:3] = np.where(dmask[None, :], c.dirichlet_field(), 0.0)
        xs.append(s.scatter(_dev(x0), l))
        bs.append(s.rhs_level(s.scatter(_dev(f), l), l))
        bs_o.append(umg.rhs(f, l))
        xbc.append(x0)
    s.fmg(xs, bs, cycles)
    xo = umg.fmg(bs_o, xbc, cycles)
    for l in range(s.L + 1):
        xg = s.gather(xs[l], l).cpu().numpy()
        err = np.abs(xg - xo[l]).max() / np.abs(xo[l]).max()
        print(f"level {l}: max rel. difference {err:.2e}", flush=True)
        assert err < 1e-10, l


@pytest.mark.parametrize("cid,opts", [(8, {}), (9, {}), (8, {"ordering": 1})])
def test_fmg_on_the_shell_matches_oracle(cid, opts):
    """Full multigrid on the spherical shell (general macro geometry, a hole
    in the lattice): no-slip with the analytic data of the efficiency study,
    free-slip on the inner sphere (the prolongated solution keeps its tangential
    part), and the hybrid ordering; every level against the oracle."""
    import paper_1511_02134_amd as P
    R = 4
    cfg = W.WORKLOADS[cid].with_R(R)
    print(f"\n[case] fmg {cfg.name} R={R} opts={opts}", flush=True)
    xyz, tet, nu, tags = cfg.mesh()
    phys = cfg.physical()
    s = P.Solver(xyz, tet, nu, tags, R, nu1=2, nu2=2, cycle=1, phys=phys, **opts)
    H = build_hierarchy(xyz, tet, nu, tags, R, phys=phys)
    umg = UMG(H, nu1=2, nu2=2, variable=True,
              ordering="hybrid" if opts.get("ordering") else "colour")
    xs, bs, bs_o, xbc = [], [], [], []
    for l in range(s.L + 1):
        lv = H.levels[l]
        c = cfg.with_R(2 + l)
        f = c.forcing_field()
        _, dmask = s.node_info(l)
        x0 = np.zeros((4, s.num_nodes(l)))
        x0[:3] = np.where(dmask[None, :], c.dirichlet_field(), 0.0)
        xs.append(s.scatter(_dev(x0), l))
        bs.append(s.rhs_level(s.scatter(_dev(f), l), l))
        bs_o.append(umg.rhs(f[:, lv.lat], l))
        xbc.append(x0[:, lv.lat])
    s.fmg(xs, bs, 1)
    xo = umg.fmg(bs_o, xbc, 1)
    for l in range(s.L + 1):
        xg = s.gather(xs[l], l).cpu().numpy()[:, H.levels[l].lat]
        err = np.abs(xg - xo[l]).max() / np.abs(xo[l]).max()
        print(f"level {l}: max rel. difference {err:.2e}", flush=True)
        assert err < 1e-10, l
