"""Benchmark: Stokes DoFs solved per second on one MI355X.

One step = one complete solve of the unit-cube Stokes problem refined 8 times
(257^3 lattice, 66,718,718 DoFs, FP64, manufactured forcing, variable V(3,3)
Uzawa multigrid with the red-black smoother order to a 1e-8 relative residual
from x0 = 0): right-hand side
assembly, every cycle and the per-cycle residual check.  Inputs are resident
in HBM before the timed region.  The same problem in mixed precision (FP32
cycles inside FP64 refinement) is timed beside it.

Printed as one JSON line with, besides the contract fields:
  tme_factor      solve time / time of one K apply on the finest level (the
                  paper's work unit, Section 5), both measured here;
  phases_ms       smoothing, transfers, coarse solves and residuals of one
                  solve (hipEvent pairs around every phase), levels_ms the
                  same by level;
  roofline        the dominant kernel of the finest level, the velocity sweep
                  or the fused f - B^T p pass, whichever has the larger total
                  time in the timed solves (the other as roofline_<name>),
                  against the 8 TB/s HBM peak: algorithmic bytes per launch /
                  its mean launch time (hipEvents on its stream; one pair
                  around the back-to-back velocity sweeps of each smoothing
                  step, one around every fused pass);
  mixed_precision the FP32-in-FP64 solve of the same problem;
  cpu_baseline    the FP64 oracle (numpy/scipy) solving the same problem at a
                  bounded size on the host, setup excluded.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 3]
    python bench.py --tme R        (full multigrid efficiency study)
    python bench.py --compare R    (UMG / PMINRES / SCG comparison)
    python bench.py --shell R      (spherical shell, general macro geometry)
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Stokes DoFs solved/s to 1e-8 rel. residual; TME factor; smoother HBM GB/s"
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_velocity_sweep_unitcube_R8_fp64.md")
SHELL_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_velocity_sweep_shell_R7_fp64.md")
RB_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles",
                                  "traffic_velocity_sweep_redblack_unitcube_R8_fp64.md")
RU_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_fused_ru_redblack_unitcube_R8_fp64.md")


def sources_digest() -> str:
    """SHA-256 over the native sources: a traffic figure measured for other
    sources describes another kernel."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1511_02134_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp", ".cpp", ".h")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(path=TRAFFIC_PROFILE):
    """HBM bytes per launch of the finest velocity sweep from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when it was taken for
    other sources (or is absent)."""
    try:
        with open(path) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    vals = {}
    for ln in lines:
        ln = ln.strip().lstrip("-").strip()
        if ":" in ln and ln.split(":", 1)[0].strip() in ("sources_sha256", "traffic_bytes_per_launch"):
            k, v = ln.split(":", 1)
            vals[k.strip()] = v.strip().split()[0].strip("`")
    if vals.get("sources_sha256") != sources_digest() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(workload_id: int, R: int, cycle: int, ordering: str = "colour",
                 timeout: float = 600.0):
    """Times the oracle's solve (setup excluded) in a child process."""
    code = f"""
import json, time, sys
sys.path.insert(0, {ROOT!r})
import numpy as np
import workloads as W
from oracle import build_hierarchy, UMG
cfg = W.WORKLOADS[{workload_id}].with_R({R})
xyz, tet, nu, tags = cfg.mesh()
H = build_hierarchy(xyz, tet, nu, tags, {R})
umg = UMG(H, variable={bool(cycle)}, ordering={ordering!r})
lv = H.finest
f = cfg.forcing_field()
t0 = time.perf_counter()
b = umg.rhs(f)
x0 = np.zeros((4, lv.N)); x0[:3] = cfg.dirichlet_field(); x0[:3, lv.free] = 0.0
x, hist = umg.solve(x0, b, rtol=1e-8, max_cycles=100)
t = time.perf_counter() - t0
print(json.dumps({{"seconds": t, "dofs": lv.ndofs(), "cycles": len(hist) - 1}}))
"""
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=timeout)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-2000:])
    return json.loads(out.stdout.strip().splitlines()[-1])


def run_ops(workload_id: int, R: int = 0, ordering: int = 0):
    """A short sequence of finest-level operations for counter collection
    (rocprofv3 --pmc): K x, the residual, restriction and prolongation three
    times each, two smoothing steps, then three device copies of 512 MiB whose
    counter readings calibrate FETCH_SIZE and WRITE_SIZE.  R: refinements
    (default: the workload's own)."""
    import torch
    import workloads as W
    import paper_1511_02134_amd as P

    cfg = W.WORKLOADS[workload_id]
    if R:
        cfg = cfg.with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    s = P.Solver(xyz, tet, nu, tags, cfg.R, precision=0, phys=cfg.physical(), ordering=ordering)
    L, N = s.L, s.num_nodes()
    rng = np.random.default_rng(0)
    x = s.scatter(torch.tensor(rng.normal(size=(4, N)), device="cuda"))
    b = s.scatter(torch.tensor(rng.normal(size=(4, N)), device="cuda"))
    y = torch.empty_like(x)
    for _ in range(3):
        s.apply(x, L, out=y)
        r, _ = s.residual(x, b, L, norm=False)
        xc = s.restrict(r, L)
        s.prolong_add(xc, x, L)
    s.smooth(x, b, 2, L)
    a = torch.empty(64 << 20, dtype=torch.float64, device="cuda").normal_()
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    print(f"operations done: workload {cfg.name}, {s.num_dofs()} DoFs", flush=True)


def run_tme(R: int, steps: int, warmup: int):
    """Full multigrid with one (FMG) and two (2FMG) variable V(2,2) cycles per
    level on the analytic solution of the efficiency study (Section 5):
    solve time, its cost in work units (one finest K apply) and the ratio
    gamma of total to discretisation error (Table "gamma_l"); the discrete
    solution is an FP64 solve to 1e-12 from the FMG result."""
    import torch
    import workloads as W
    import paper_1511_02134_amd as P

    cfg = W.WORKLOADS[6].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    s = P.Solver(xyz, tet, nu, tags, R, nu1=2, nu2=2, cycle=1)
    dev = torch.device("cuda")
    xs0, bs = [], []
    for l in range(s.L + 1):
        c = cfg.with_R(2 + l)
        _, dmask = s.node_info(l)
        x0 = torch.zeros(4, s.num_nodes(l), dtype=torch.float64, device=dev)
        x0[:3] = torch.where(torch.tensor(dmask, device=dev)[None, :],
                             torch.tensor(c.dirichlet_field(), device=dev), 0.0)
        xs0.append(s.scatter(x0, l))
        bs.append(s.rhs_level(s.scatter(torch.tensor(c.forcing_field(), device=dev), l), l))
    xs = [torch.empty_like(x) for x in xs0]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = {}
    _, dmask = s.node_info(s.L)
    ex = torch.tensor(cfg.exact_solution(), device=dev)
    mass = torch.tensor(s.mass_weights(), device=dev)
    h = 2.0 ** -R

    def hnorm(d):
        d = d.clone()
        d[3] -= (mass * d[3]).sum() / mass.sum()
        return float(torch.sqrt((d[:3] ** 2).sum() + h * h * (d[3] ** 2).sum()))

    yk = torch.empty_like(xs0[-1])
    times = []
    for _ in range(25):
        ev[0].record()
        s.apply(xs0[-1], None, out=yk)
        ev[1].record()
        torch.cuda.synchronize()
        times.append(ev[0].elapsed_time(ev[1]))
    t_apply = float(np.median(times[5:]))
    xdisc = None
    for cycles in (1, 2):
        t = []
        for k in range(warmup + steps):
            for a, b0 in zip(xs, xs0):
                a.copy_(b0)
            torch.cuda.synchronize()
            ev[0].record()
            s.fmg(xs, bs, cycles)
            ev[1].record()
            torch.cuda.synchronize()
            if k >= warmup:
                t.append(ev[0].elapsed_time(ev[1]))
        xf = s.gather(xs[-1])
        if xdisc is None:
            xd = xs[-1].clone()
            info = s.solve(xd, bs[-1], rtol=1e-12, max_cycles=100)
            xdisc = s.gather(xd)
        disc = hnorm(ex - xdisc)
        ms = float(np.median(t))
        out["FMG" if cycles == 1 else "2FMG"] = {
            "ms": ms, "work_units": ms / t_apply,
            "gamma": hnorm(ex - xf) / disc,
            "algebraic_error_h": hnorm(xf - xdisc) / hnorm(xdisc)}
    line = {"metric": "FMG Vvar(2,2) time in work units (TME factor) and error ratio gamma",
            "workload": cfg.name, "refinements": R, "dofs": s.num_dofs(),
            "t_apply_ms": t_apply, "model_E_TME": 9.07, "data": "synthetic (analytic solution)",
            **out}
    print(json.dumps(line), flush=True)


def run_compare(R: int, steps: int, warmup: int, dform: bool = False):
    """The solver comparison of Section 4 (Table T:itertime1, Figure opcount):
    unit cube, f = 0, nu = 1, random start u0 ~ U[0,1], p0 ~ U[0, 1/h_min]
    (Section 3.6), relative residual 1e-8; UMG with the variable V(3,3)
    cycle, block-diagonal PMINRES with a velocity V(1,1) cycle, and SCG with
    V(3,3), n_A = n_S = 3, n_I = 1 (Table "settings").  Prints iterations,
    time to solution (median of the timed solves, hipEvents) and the
    measured operator evaluations per block (eq. op_count)."""
    import torch
    import workloads as W
    import paper_1511_02134_amd as P

    cfg = W.WORKLOADS[1].with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    s = P.Solver(xyz, tet, nu, tags, R, cycle=1, krylov=1, op=1 if dform else 0)
    dev = torch.device("cuda")
    n = 2 ** R
    hmin = (1.0 / (6.0 * n ** 3)) ** (1.0 / 3.0)
    x0n = W.random_initial_guess(s.num_nodes(), 1.0 / hmin, seed=0)
    _, dmask = s.node_info()
    x0n[:3, dmask] = 0.0
    x0 = s.scatter(torch.tensor(x0n, device=dev))
    b = s.vector()
    x = torch.empty_like(x0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    print(f"[bench] comparison set up: R={R}, {s.num_dofs()} DoFs", file=sys.stderr, flush=True)
    runs = {"UMG": lambda: s.solve(x, b, rtol=1e-8, max_cycles=100),
            "PMINRES": lambda: s.pminres(x, b, rtol=1e-8, maxit=2000, nu=1),
            "SCG": lambda: s.scg(x, b, rtol=1e-8, max_outer=255, n_A=3, n_S=3, n_I=1, nu=3)}
    out = {}
    for name, fn in runs.items():
        t = []
        for k in range(warmup + steps):
            x.copy_(x0)
            torch.cuda.synchronize()
            ev[0].record()
            info = fn()
            ev[1].record()
            torch.cuda.synchronize()
            if k >= warmup:
                t.append(ev[0].elapsed_time(ev[1]))
        print(f"[bench] {name} done", file=sys.stderr, flush=True)
        out[name] = {"iterations": info["cycles"], "status": info["status"],
                     "rel_res": info["rel_res"], "ms": float(np.median(t)),
                     "n_op": {k: round(v, 2) for k, v in info["n_op"].items()}}
    line = {"metric": "time to solution and operator evaluations of UMG, PMINRES and SCG",
            "workload": f"unit cube, {R} refinements, f = 0, random start (seed 0)",
            "form": "D (a_2)" if dform else "Laplace (a_1)",
            "refinements": R, "paper_level": R - 2, "dofs": s.num_dofs(), "rtol": 1e-8,
            "dtype": "f64", "data": "synthetic", **out}
    print(json.dumps(line), flush=True)


def run_shell(R: int, steps: int, warmup: int, ordering: int = 0, slip: str | None = None):
    """The spherical shell 0.55 < |x| < 1 (Section 4.4) as 156 affinely mapped
    macros: f = 0, homogeneous Dirichlet data on both spheres (or, with slip,
    free-slip on the inner sphere or on both: Section 6.1), the paper's seeded
    random start (u in U[0,1], p in U[0, 1/h_min]), variable V(3,3) to a 1e-8
    relative residual and the direct
    coarse solver.  Reports DoFs solved per second, the phase
    split of one solve and the mean time and algorithmic HBM rate of the
    finest velocity colour sweep (15-tap stencils)."""
    import torch
    import workloads as W
    import paper_1511_02134_amd as P

    cfg = (W.WORKLOADS[9].with_slip(slip) if slip else W.WORKLOADS[7]).with_R(R)
    xyz, tet, nu, tags = cfg.mesh()
    t0 = time.perf_counter()
    s = P.Solver(xyz, tet, nu, tags, R, phys=cfg.physical(), cycle=1, ordering=ordering)
    t_setup = time.perf_counter() - t0
    dev = torch.device("cuda")
    dofs, N = s.num_dofs(), s.num_nodes()
    nvert = int(np.count_nonzero(s.mass_weights() > 0))
    x0n = W.random_initial_guess(N, 1.0 / cfg.h_min(), seed=0)
    _, dmask = s.node_info()
    x0n[:3, dmask.astype(bool)] = 0.0
    x0 = s.scatter(torch.tensor(x0n, device=dev))
    f_int = s.scatter(torch.zeros(3, N, dtype=torch.float64, device=dev))
    x = torch.empty_like(x0)
    print(f"[bench] shell set up: R={R}, {dofs} DoFs", file=sys.stderr, flush=True)
    ms, info, step = timed_solves(s, f_int, x0, x, steps, warmup)
    s.set_phase_timing(True)
    pinfo = step()
    s.set_phase_timing(False)
    s.set_timing(True)
    for _ in range(min(steps, 3)):
        step()
    torch.cuda.synchronize()
    nvel, ms_vel, _ = s.kernel_time(P.K_VEL)
    npres, ms_pres, _ = s.kernel_time(P.K_PRES)
    napp, ms_app, _ = s.kernel_time(P.K_APPLY)
    s.set_timing(False)
    vel_us = 1000.0 * ms_vel / max(nvel, 1)
    alg_bytes = 10.0 * 8.0 * nvert / 4.0
    achieved = alg_bytes / (vel_us * 1e-6) / 1e9
    traffic = measured_traffic(SHELL_TRAFFIC_PROFILE) if R == 7 and not slip and not ordering else None
    line = {"metric": "Stokes DoFs solved/s to 1e-8 rel. residual (spherical shell)",
            "value": dofs / (ms * 1e-3), "unit": "DoF/s", "ms_per_step": ms,
            "steps": steps, "warmup": warmup, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"shell{'-slip-' + slip if slip else ''}-R{R}-fp64",
                       "boundary": ({"inner": "free-slip on the inner sphere, no-slip on the outer",
                                     "both": "free-slip on both spheres"}[slip] + " (mass-"
                                    "conservative normals)") if slip else "no-slip",
                       "mesh": "spherical shell 0.55<|x|<1, "
                       "156 affinely mapped macros (hollow cube [0,3]^3 minus its centre cell)",
                       "refinements": R, "dofs": dofs, "vertices": nvert,
                       "cycle": "Vvar(3,3)",
                       "ordering": "hybrid" if ordering == 1 else "colour",
                       "coarse": "exact (inverse of the bordered level-0 system, 5788 unknowns)",
                       "cycles": info["cycles"], "rho_mean": info["rho_mean"],
                       "status": info["status"]},
            "phases_ms": {k: round(v, 3) for k, v in pinfo["t_phase_ms"].items()},
            "levels_ms": {f"R{l + 2}": round(v, 3) for l, v in enumerate(pinfo["t_level_ms"])},
            "setup_s": t_setup,
            "velocity_sweep": {"kernel": "k_colour<double,velocity,15 taps> (finest level)",
                               "avg_us": vel_us, "bytes_per_launch": alg_bytes,
                               "achieved_GBs": achieved, "frac_of_hbm_peak": achieved / HBM_PEAK_GBS,
                               "traffic": traffic,
                               "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + "
                                               "WRITE_SIZE, copy-calibrated)"},
            "kernel_classes": {"velocity_sweep": {"launches": nvel, "ms": ms_vel},
                               "pressure_sweep": {"launches": npres, "ms": ms_pres},
                               "full_passes": {"launches": napp, "ms": ms_app}}}
    print(json.dumps(line), flush=True)


def host_cpu():
    """(nproc, CPU model name) of the host."""
    model = "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return os.cpu_count() or 0, model


def timed_solves(s, f_int, x0, x, steps, warmup):
    """`warmup` then `steps` complete solves (right-hand side, every cycle,
    the per-cycle stopping test); returns (ms per solve, info of the last)."""
    import torch

    def step():
        b = s.rhs(f_int)
        x.copy_(x0)
        return s.solve(x, b, rtol=1e-8, max_cycles=100)

    info = None
    for _ in range(warmup):
        info = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = step()
    torch.cuda.synchronize()
    return 1000.0 * (time.perf_counter() - t0) / steps, info, step


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--R", type=int, default=0,
                    help="refinements of the workload's mesh (default: the workload's own)")
    ap.add_argument("--precision", choices=("fp64", "mixed", "workload"), default="fp64",
                    help="precision of the timed solve (default FP64, the paper's; 'workload': "
                         "the workload's own)")
    ap.add_argument("--cycle", choices=("V", "Vvar", "workload"), default="workload",
                    help="V(3,3) or the variable V(3,3) (default: Vvar on the unit cube at 8 "
                         "refinements and the channel, V otherwise)")
    ap.add_argument("--op", choices=("laplace", "D"), default="laplace",
                    help="velocity form: Laplace (a_1, default) or D (a_2 = 2<nu D(u), D(v)>)")
    ap.add_argument("--ordering", choices=("auto", "colour", "hybrid", "redblack"), default="auto",
                    help="Gauss-Seidel order of the smoother: the global 4-colouring, the hybrid "
                         "primitive-class order of HHG (Section 3.4), or red-black (Kuhn meshes: "
                         "the parities of X+Y+Z).  Default: red-black where the stencils allow it "
                         "(Kuhn macros, Laplace form), the 4-colouring otherwise")
    ap.add_argument("--graphs", type=int, choices=(0, 1), default=1,
                    help="1 (default): replay each cycle of the solves from a captured HIP graph "
                         "(opts.graphs; the timed runs of the kernel-class and phase timers launch "
                         "on the stream); 0: launch every kernel on the stream")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision solve reported beside the FP64 one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-R", type=int, default=6,
                    help="refinements of the oracle's bounded sample")
    ap.add_argument("--ops", action="store_true",
                    help="run the operation sequence used for counter collection and exit")
    ap.add_argument("--tme", type=int, default=0, metavar="R",
                    help="full multigrid efficiency study at R refinements (prints its own line)")
    ap.add_argument("--compare", type=int, default=0, metavar="R",
                    help="UMG / PMINRES / SCG comparison at R refinements (prints its own line)")
    ap.add_argument("--shell", type=int, default=0, metavar="R",
                    help="spherical shell 0.55 < |x| < 1 at R refinements: the paper's setting "
                         "(f = 0, random start) on general macro geometry (prints its own line)")
    ap.add_argument("--slip", nargs="?", const="inner", choices=("inner", "both"), default=None,
                    help="with --shell: free-slip on the inner sphere (no-slip on the outer), or "
                         "on both spheres")
    args = ap.parse_args()
    if args.ordering == "auto":
        # red-black needs 7-point a_1 and c_l: Kuhn macros (no physical
        # coordinates: not the shell) and the Laplace form
        args.ordering = "colour" if args.shell or args.op == "D" else "redblack"
        if args.ops and args.workload in (7, 8, 9):
            args.ordering = "colour"
    ordering = {"colour": 0, "hybrid": 1, "redblack": 2}[args.ordering]
    if args.ops:
        run_ops(args.workload, args.R, ordering)
        return
    if args.tme:
        run_tme(args.tme, max(args.steps, 3), args.warmup)
        return
    if args.compare:
        run_compare(args.compare, min(max(args.steps, 1), 3), min(args.warmup, 1),
                    args.op == "D")
        return
    if args.shell:
        run_shell(args.shell, args.steps, args.warmup, ordering, args.slip)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the solver has no multi-GPU path "
              f"(requested --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    import paper_1511_02134_amd as P

    cfg = W.WORKLOADS[args.workload]
    if args.R:
        cfg = cfg.with_R(args.R)
    xyz, tet, nu, tags = cfg.mesh()
    if args.precision == "workload":
        precision = 1 if cfg.precision == "mixed" else 0
    else:
        precision = 1 if args.precision == "mixed" else 0
    if args.cycle == "workload":
        cycle = 1 if args.workload in (3, 5) else 0
    else:
        cycle = 1 if args.cycle == "Vvar" else 0
    dform = args.op == "D"
    s = P.Solver(xyz, tet, nu, tags, cfg.R, precision=precision, op=1 if dform else 0,
                 cycle=cycle, ordering=ordering, graphs=args.graphs)
    dofs = s.num_dofs()
    nvert = s.num_nodes()
    name = cfg.name.rsplit("-", 1)[0] + ("-fp64" if precision == 0 else "-mixed")
    print(f"[bench] solver ready: {name}, R={cfg.R}, {dofs} DoFs", file=sys.stderr, flush=True)
    dev = torch.device("cuda")
    f = torch.tensor(cfg.forcing_field(), dtype=torch.float64, device=dev)
    x0n = torch.zeros(4, nvert, dtype=torch.float64, device=dev)
    x0n[:3] = torch.tensor(cfg.dirichlet_field(), device=dev)
    _, dmask = s.node_info()
    x0n[:3, ~torch.tensor(dmask, device=dev)] = 0.0
    f_int = s.scatter(f)
    x0 = s.scatter(x0n)
    x = torch.empty_like(x0)
    torch.cuda.synchronize()
    print("[bench] inputs on the device", file=sys.stderr, flush=True)

    ms_per_step, info, step = timed_solves(s, f_int, x0, x, args.steps, args.warmup)
    if info["status"] != 0:
        print(f"solve did not converge: {info}", file=sys.stderr)
        sys.exit(1)
    print(f"[bench] timed solves done: {ms_per_step:.2f} ms, {info['cycles']} cycles",
          file=sys.stderr, flush=True)

    # work unit: one K apply on the finest level in the solve's precision of
    # the finest sweeps (FP64 here)
    y = torch.empty_like(x)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = []
    for _ in range(25):
        ev[0].record()
        s.apply(x, None, out=y)
        ev[1].record()
        torch.cuda.synchronize()
        times.append(ev[0].elapsed_time(ev[1]))
    t_apply = float(np.median(times[5:]))

    # phase split of one solve (hipEvent pairs around every phase)
    s.set_phase_timing(True)
    pinfo = step()
    s.set_phase_timing(False)
    torch.cuda.synchronize()

    # roofline of the dominant kernel: the finest-level velocity sweeps and the
    # fused f - B^T p passes of the same steps, timed by hipEvents on the
    # solver's stream (one pair around the consecutive velocity sweeps of each
    # smoothing step, one around every fused pass); the one with the larger
    # total is the roofline entry, the other is reported beside it
    s.set_timing(True)
    for _ in range(min(args.steps, 3)):
        step()
    torch.cuda.synchronize()
    nvel, ms_vel, bytes_vel = s.kernel_time(P.K_VEL)
    npres, ms_pres, bytes_pres = s.kernel_time(P.K_PRES)
    napp, ms_app, bytes_app = s.kernel_time(P.K_APPLY)
    nru, ms_ru, bytes_ru = s.kernel_time(P.K_RU)
    s.set_timing(False)
    vel_avg_ms = ms_vel / max(nvel, 1)
    if nvel == 0:
        raise RuntimeError("no finest-level velocity sweep was timed")
    vs = 8.0 if precision == 0 else 4.0
    # algorithmic bytes of one colour launch: one direction of the velocity
    # Gauss-Seidel reads u (3 values), f (3) and p and writes u (3) per finest
    # vertex, 10 values; its four colour launches share them (the red-black
    # order's two parity launches)
    per_launch = 0.5 if ordering == 2 else 0.25
    alg_bytes = 10.0 * vs * nvert * per_launch
    achieved = alg_bytes / (vel_avg_ms * 1e-3) / 1e9
    traffic = (measured_traffic(RB_TRAFFIC_PROFILE if ordering == 2 else TRAFFIC_PROFILE)
               if args.workload == 3 and not args.R and precision == 0 and not dform
               and ordering in (0, 2) else None)

    # practical ceiling: device copies moving the same bytes (half read, half
    # written), timed like the sweeps: groups of six back-to-back launches,
    # each group bracketed by one pair of hipEvents
    src = torch.empty(int(alg_bytes // 16), dtype=torch.float64, device=dev).normal_()
    dst = torch.empty_like(src)
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(40)]
    for _ in range(5):
        dst.copy_(src)
    for a, b_ in pairs:
        a.record()
        for _ in range(6):
            dst.copy_(src)
        b_.record()
    torch.cuda.synchronize()
    ctime = float(np.mean([a.elapsed_time(b_) for a, b_ in pairs])) / 6
    copy_gbs = 2 * src.numel() * 8 / (ctime * 1e-3) / 1e9
    del src, dst

    prec_name = "double" if precision == 0 else "float"
    entries = {"velocity_sweep": {
        "bound": "hbm",
        "kernel": (f"{'k_colour_rb' if ordering == 2 else 'k_colour'}<{prec_name},velocity"
                   f"{',D' if dform else ''}> (finest level)"),
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "bytes_model": ("10 values per finest vertex per sweep direction (read u, f, p; "
                        "write u), " + ("half per red-black parity launch" if ordering == 2
                                        else "a quarter per colour launch")),
        "bytes_per_launch": alg_bytes,
        "launches": nvel,
        "avg_us": 1000.0 * vel_avg_ms,
        "copy_probe": {"GB/s": copy_gbs, "bytes": 2 * int(alg_bytes // 16) * 8,
                       "frac_of_copy": achieved / copy_gbs},
    }}
    if nru > 0:
        # f - B^T p with the fused update: read f (3 values), p, the other
        # colours' velocity and write t (3) and the updated colour's velocity,
        # per finest vertex: 10 values with a red-black parity, 9.25 with colour 0
        ru_bytes = (10.0 if ordering == 2 else 9.25) * vs * nvert
        ru_avg_ms = ms_ru / nru
        ru_achieved = ru_bytes / (ru_avg_ms * 1e-3) / 1e9
        ru_traffic = (measured_traffic(RU_TRAFFIC_PROFILE)
                      if args.workload == 3 and not args.R and precision == 0 and not dform
                      and ordering == 2 else None)
        entries["fused_ru"] = {
            "bound": "hbm",
            "kernel": f"k_full<{prec_name},f - B^T p,fused,windows> (finest level)",
            "achieved": ru_achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": ru_achieved / HBM_PEAK_GBS,
            "traffic": ru_traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated)",
            "bytes_model": ("read f (3 values), p and the other colours' velocity, write t (3) "
                            "and the updated colour's velocity, per finest vertex: "
                            + ("10 values (red parity)" if ordering == 2 else
                               "9.25 values (colour 0)")),
            "bytes_per_launch": ru_bytes,
            "launches": nru,
            "avg_us": 1000.0 * ru_avg_ms,
            "copy_probe": {"GB/s": copy_gbs, "frac_of_copy": ru_achieved / copy_gbs},
        }
    dominant = "fused_ru" if nru > 0 and ms_ru > ms_vel else "velocity_sweep"

    line = {
        "metric": METRIC,
        "value": dofs / (ms_per_step * 1e-3),
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f32-in-f64",
        "data": "synthetic",
        "config": {
            "workload": name,
            "mesh": f"box [0,{cfg.a}]x[0,1]^2, {tet.shape[0]} Kuhn macro tetrahedra",
            "refinements": cfg.R,
            "dofs": dofs,
            "vertices": nvert,
            "cycle": "Vvar(3,3)" if cycle else "V(3,3)",
            "form": "D (a_2)" if dform else "Laplace (a_1)",
            "ordering": args.ordering,
            "graphs": args.graphs,
            "rtol": 1e-8,
            "cycles": info["cycles"],
            "coarse": ("exact (inverse of the bordered level-0 system)" if s.opts.coarse_solver == 0
                       else "block-diagonal PMINRES"),
            "rho_mean": info["rho_mean"],
        },
        "tme_factor": ms_per_step / t_apply,
        "t_apply_ms": t_apply,
        "phases_ms": {k: round(v, 3) for k, v in pinfo["t_phase_ms"].items()},
        "levels_ms": {f"R{l + 2}": round(v, 3) for l, v in enumerate(pinfo["t_level_ms"])},
        "roofline": dict(entries[dominant], name=dominant),
        **{f"roofline_{k}": v for k, v in entries.items() if k != dominant},
        "kernel_classes": {
            "velocity_sweep": {"launches": nvel, "ms": ms_vel},
            "fused_ru": {"launches": nru, "ms": ms_ru},
            "pressure_sweep": {"launches": npres, "ms": ms_pres},
            "full_passes": {"launches": napp, "ms": ms_app},
        },
    }
    if precision == 0 and not args.no_mixed:
        sm = P.Solver(xyz, tet, nu, tags, cfg.R, precision=1, op=1 if dform else 0, cycle=cycle,
                      ordering=ordering, graphs=args.graphs)
        xm = torch.empty_like(x0)
        ms_m, info_m, _ = timed_solves(sm, f_int, x0, xm, args.steps, args.warmup)
        line["mixed_precision"] = {
            "value": dofs / (ms_m * 1e-3), "unit": "DoF/s", "ms_per_step": ms_m,
            "cycles": info_m["cycles"], "rho_mean": info_m["rho_mean"],
            "status": info_m["status"], "dtype": "f32 cycles in f64 iterative refinement"}
        print("[bench] mixed-precision solves done", file=sys.stderr, flush=True)
        del sm, xm
    if not args.no_cpu_baseline:
        cb = cpu_baseline(args.workload, args.cpu_R, cycle, args.ordering)
        nproc, model = host_cpu()
        line["cpu_baseline"] = {
            "value": cb["dofs"] / cb["seconds"],
            "unit": "DoF/s",
            "cores": 1,
            "kind": "oracle",
            "host": {"nproc": nproc, "cpu_model": model},
            "sample": (f"oracle (numpy/scipy FP64; its sparse products run on one thread of "
                       f"the {nproc} host cores) full solve of the same problem at "
                       f"{args.cpu_R} refinements instead of {cfg.R} ({cb['dofs']} DoFs, "
                       f"{'Vvar' if cycle else 'V'}(3,3), {args.ordering} ordering, "
                       f"{cb['cycles']} cycles, "
                       f"{cb['seconds']:.1f} s; setup excluded): the oracle's assembly of the "
                       f"full size does not fit a benchmark run"),
        }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
