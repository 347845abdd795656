"""GPU: hhg_residual_noalloc, the residual entry point that allocates nothing
(its partial sums live in a static device array of the library), against
hhg_residual on two calls in a row, the second on a smaller level; and under
HIP graph capture, replayed several times with eager work in between."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _inputs(s, level, seed):
    rng = np.random.default_rng(seed)
    N = s.num_nodes(level)
    return s.scatter(_dev(rng.normal(size=(4, N))), level), s.scatter(_dev(rng.normal(size=(4, N))), level)


@pytest.mark.parametrize("R", [5, 6])
def test_noalloc_residual_equals_residual(R):
    """Levels L (at R = 6 the split volume/interface launches) and then L - 1
    (smaller): r and ||r|| bitwise equal to hhg_residual's; the device's
    free memory is unchanged across the calls."""
    import paper_1511_02134_amd as P
    cfg = W.WORKLOADS[1].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    _announce(f"no-alloc residual, unit cube R={R}")
    s = P.Solver(xyz, tet, nu, tags, R)
    levels = (s.L, s.L - 1)
    cases = []
    for level in levels:
        x, b = _inputs(s, level, 10 * R + level)
        r_ref, n_ref = s.residual(x, b, level)
        cases.append((level, x, b, r_ref, n_ref, torch.full_like(r_ref, np.nan),
                      torch.zeros(1, dtype=torch.float64, device="cuda")))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for level, x, b, _, _, r, norm in cases:
        s.residual_noalloc(x, b, r, norm, level)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    for level, x, b, r_ref, n_ref, r, norm in cases:
        _announce(f"level {level}: norm {norm.item():.17e} vs {n_ref:.17e}")
        # every vertex slot (all copies) written and equal; the padding slots
        # of the layout are not part of the vector and stay untouched
        N = s.num_nodes(level)
        ids = s.scatter(_dev(np.arange(1, N + 1, dtype=np.float64)[None, :]), level)[0]
        vert = ids > 0
        assert torch.equal(r[:, vert], r_ref[:, vert])
        assert bool(torch.isnan(r[:, ~vert]).all())
        assert norm.item() == n_ref


def test_noalloc_residual_under_graph_capture():
    """Captured in a graph (which must not allocate while capturing) and
    replayed five times on changing inputs, with eager calls of hhg_residual
    between the replays: every replay equals the eager result."""
    import paper_1511_02134_amd as P
    R = 5
    cfg = W.WORKLOADS[4].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    _announce("no-alloc residual under graph capture, box R=5")
    s = P.Solver(xyz, tet, nu, tags, R)
    x, b = _inputs(s, s.L, 3)
    r = torch.zeros_like(x)
    norm = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.residual_noalloc(x, b, r, norm)          # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.residual_noalloc(x, b, r, norm)
    rng = np.random.default_rng(8)
    for k in range(5):
        N = s.num_nodes()
        x.copy_(s.scatter(_dev(rng.normal(size=(4, N)))))
        b.copy_(s.scatter(_dev(rng.normal(size=(4, N)))))
        g.replay()
        torch.cuda.synchronize()
        r_ref, n_ref = s.residual(x, b)
        assert torch.equal(r, r_ref), k
        assert norm.item() == n_ref, k


def test_noalloc_residual_rejects_bad_arguments():
    import paper_1511_02134_amd as P
    cfg = W.WORKLOADS[1].with_R(3)
    xyz, tet, nu, tags = cfg.mesh()
    s = P.Solver(xyz, tet, nu, tags, 3)
    x, b = _inputs(s, s.L, 1)
    norm = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(P.HHGError) as e:
        s.residual_noalloc(x, b, x, norm)
    assert e.value.status == P.HHG_EINVAL
    with pytest.raises(P.HHGError) as e:
        s.residual_noalloc(x, b, torch.zeros_like(x), norm, level=s.L + 1)
    assert e.value.status == P.HHG_EINVAL
