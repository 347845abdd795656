"""The FP64 solve hands f - B^T p from the residual of its stopping test to the
first Uzawa step of the next cycle (Laplace form on Kuhn macros, colour and
red-black orders), which then starts with the velocity sweeps instead of the
pass that forms f - B^T p.  hhg_vcycle forms it in the step itself on its top
level, so k cycles of hhg_solve equal k calls of hhg_vcycle up to rounding.
Checked on levels whose residual takes the quad-window launch (6
refinements) and on smaller ones (4 and 5), in both orders and in the plain
and the variable cycle; the residual histories of the solve are the norms of
b - K x of those iterates."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _relerr(a, b):
    return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))


@pytest.mark.parametrize("cid,R,ordering,cycle", [(1, 4, 0, 0), (1, 4, 2, 0), (4, 5, 0, 0),
                                                  (3, 6, 2, 1), (3, 6, 0, 1)])
def test_solve_cycles_equal_vcycles(cid, R, ordering, cycle):
    import paper_1511_02134_amd as P
    cfg = W.WORKLOADS[cid].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    _announce(f"hand-over: config {cid} R={R} ordering={ordering} cycle={cycle}")
    s = P.Solver(xyz, tet, nu, tags, R, ordering=ordering, cycle=cycle)
    dev = torch.device("cuda")
    _, dmask = s.node_info()
    x0n = torch.zeros(4, s.num_nodes(), dtype=torch.float64, device=dev)
    x0n[:3] = torch.where(torch.tensor(dmask, device=dev)[None, :],
                          torch.tensor(cfg.dirichlet_field(), device=dev), 0.0)
    b = s.rhs(s.scatter(torch.tensor(cfg.forcing_field(), device=dev)))
    x0 = s.scatter(x0n)
    cycles = 3
    xa = x0.clone()
    info = s.solve(xa, b, rtol=1e-300, max_cycles=cycles)
    assert info["cycles"] == cycles
    xb = x0.clone()
    for k in range(cycles):
        s.vcycle(xb, b)
        _, nrm = s.residual(xb, b)
        # the stopping test's norm of the same iterate, up to rounding
        assert nrm == pytest.approx(info["res_hist"][k + 1], rel=1e-10), k
    torch.cuda.synchronize()
    ga, gb = s.gather(xa), s.gather(xb)
    err = _relerr(ga, gb)
    _announce(f"{cycles} solve cycles against {cycles} V-cycles: max rel. difference {err:.2e}")
    assert err <= 1e-11
