"""Kernel-class timing of the finest level: switching it on changes no result,
and it counts every velocity and pressure colour sweep of the smoothing steps
(Section 4: V(3,3), six Uzawa steps per cycle on the finest level), the
velocity sweeps of a step being timed as one group, and the fused f - B^T p
pass of every step but the first of each cycle, whose f - B^T p comes from the
stopping test's residual (Laplace form; the D form runs it unfused, with the
other full passes)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.mark.parametrize("cid,R,op", [(1, 4, 0), (5, 4, 0), (1, 4, 1)])
def test_timing_counts_sweeps_and_changes_nothing(cid, R, op):
    import paper_1511_02134_amd as P
    cfg = W.WORKLOADS[cid].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    _announce(f"timing: config {cid} R={R} op={op}")
    s = P.Solver(xyz, tet, nu, tags, R, op=op)
    dev = torch.device("cuda")
    _, dmask = s.node_info()
    x0n = torch.zeros(4, s.num_nodes(), dtype=torch.float64, device=dev)
    x0n[:3] = torch.where(torch.tensor(dmask, device=dev)[None, :],
                          torch.tensor(cfg.dirichlet_field(), device=dev), 0.0)
    b = s.rhs(s.scatter(torch.tensor(cfg.forcing_field(), device=dev)))
    x0 = s.scatter(x0n)
    xa = x0.clone()
    ia = s.solve(xa, b, rtol=1e-8, max_cycles=100)
    s.set_timing(True)
    xt = x0.clone()
    it = s.solve(xt, b, rtol=1e-8, max_cycles=100)
    nvel, ms_vel, bytes_vel = s.kernel_time(P.K_VEL)
    npres, ms_pres, bytes_pres = s.kernel_time(P.K_PRES)
    nru, ms_ru, bytes_ru = s.kernel_time(P.K_RU)
    s.set_timing(False)
    torch.cuda.synchronize()
    assert it["res_hist"] == ia["res_hist"]
    assert torch.equal(xt, xa)
    steps = it["cycles"] * (s.opts.nu1 + s.opts.nu2)
    per_step = 7 if op == 1 else 6
    _announce(f"{it['cycles']} cycles: {nvel} velocity sweeps in {ms_vel:.3f} ms, "
              f"{npres} pressure sweeps in {ms_pres:.3f} ms")
    # Laplace form: the first Uzawa step of every cycle takes f - B^T p from
    # the stopping test's residual and sweeps colour 0 on its own
    first = it["cycles"] if op == 0 else 0
    assert nvel == steps * per_step + first
    assert npres == steps * 3
    assert ms_vel > 0.0 and ms_pres > 0.0
    assert bytes_vel > 0.0 and bytes_pres > 0.0
    assert nru == (0 if op == 1 else steps - first)
    assert (ms_ru > 0.0 and bytes_ru > 0.0) if op == 0 else (ms_ru == 0.0)
    # timing switched off and on again starts from zero
    s.set_timing(True)
    n0, ms0, by0 = s.kernel_time(P.K_VEL)
    s.set_timing(False)
    assert (n0, ms0, by0) == (0, 0.0, 0.0)
    assert np.isfinite(ms_vel / nvel)
