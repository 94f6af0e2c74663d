"""Benchmark: steady solves/s of the Newton multigrid path on one MI355X.

Workload (default): the 1D shallow-water flow over a hump, N = 12800 cells, 8 grid levels,
subcritical (q = 4.42, h_out = 2), simplified Jacobian J3 (NMGM-3), FP64 throughout, solved
from the flat-surface initial guess to res < 1e-10.  A "step" is one batch of B such problems
(hump scale s ~ U(0.8, 1.2), one seed per problem) solved to convergence: every Newton step of
every instance runs the whole hot path (residual, Jacobian, coarse operators, nu3 V-cycles,
update).  value = B * steps / timed wall time.  Inputs are resident in HBM before the timed
region starts.

Also reported: Newton-MG DOF/s, the single-instance solve rate and latency, the full Jacobian
J5 side by side, the FP32-multigrid form, the uneven batch of 512 instances, the 2D jump over
a wedge (1024 x 512 cells, FP64 and FP32 multigrid) solved end to end, the
continuous-batching server (Poisson arrivals at 200 req/s, and saturated) with p50/p99
latency, the roofline of the dominant kernel (HIP events on the launch stream) and the CPU
oracle on a bounded sample of the same workload, run on the host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6
# ridge point of the FP64 roofline: a kernel doing fewer FP64 operations per algorithmic HBM
# byte than this is bound by HBM, more by the FP64 vector units
RIDGE_FLOP_PER_BYTE = FP64_VECTOR_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)

# Algorithmic FP64 operations of one local residual evaluation of eq. (10) (each add, mul, div
# and sqrt counts one): ten WENO3 reconstructions (22 each), two HLL fluxes (46 each), the
# two-point Gauss source (36) and the final differences (3).
FLOPS_LOCAL_RESIDUAL = 10 * 22 + 2 * 46 + 36 + 3
# FP64 operations the J3 Jacobian kernel performs per interior cell, as its source states them
# (the compiler shares more: a Q-perturbed flux reuses both sides' depths and celerities).  Each
# lane evaluates one face: 16 WENO3 reconstructions (the unperturbed four, then one or two per
# perturbation of the four cells k-1..k+2, two components), 9 HLL fluxes and the reciprocal of the
# face width; the tile's 17 extra face items (four reconstructions and a flux each) are shared by
# its 256 cells.  The row then forms the unperturbed source (36) and, per H column, a perturbed
# source, the two flux differences (3) and the two difference quotients (4); per Q column the
# differences and quotients; and the alpha ||R_j||_1 term.  Boundary cells (four per instance)
# re-evaluate everything.
FLOPS_FACE = 16 * 22 + 9 * 46 + 1
FLOPS_FACE_EXTRAS = 17 * (4 * 22 + 46 + 1) / 256
FLOPS_JACOBIAN_J3 = FLOPS_FACE + FLOPS_FACE_EXTRAS + 36 + 3 * (36 + 3 + 4) + 3 * (3 + 4) + 2
# residual kernel: read U 16 and the geometry 56, write R 16 and rn 8 per cell
BYTES_RESIDUAL = 16 + 56 + 16 + 8
# Algorithmic HBM bytes per cell and launch (FP64, J3):
#   Jacobian: read U 16, R 16, rn 8, geometry 7*8 = 56; write J 96, rhs 16 and the coarse
#   operators (J 96 per coarse cell) of the eight levels built inside its tile (sum over
#   l = 1..8 of 2^-l coarse cells per fine cell)
BYTES_JACOBIAN_J3 = 16 + 16 + 8 + 56 + 96 + 16 + 96 * (1.0 - 2.0 ** -8)
# the Jacobian launch that also evaluates the residual (the plan's default order): R and rn are
# not read, and the unperturbed fluxes of the row's two faces and the source give R (3) and its
# norm (1)
BYTES_JACOBIAN_J3_FUSED = BYTES_JACOBIAN_J3 - 16 - 8
FLOPS_JACOBIAN_J3_FUSED = FLOPS_JACOBIAN_J3 + 3 + 1
# HBM traffic of the Jacobian kernel measured with rocprofv3 counters (profiles/), valid while
# the kernel source is the one it was measured on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "jacobian_j3_fp64_hump12800_batch256_traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2505_10857_amd", "csrc", "swe1d.hip")
#   finest pre-smoothing of the first V-cycle of a Newton step (dU starts at zero): read J 96
#   and rhs 16; write dU 16 and the restricted rhs 8 per fine cell (the later cycles' finest
#   pre-smoothing runs in the launch of the previous post-smoothing)
BYTES_SMOOTH_PRE_J3 = 96 + 16 + 16 + 8
#   finest fused post- + pre-smoothing: read J 96, rhs 16, dU 16 and the coarse correction 8;
#   write dU 16 and the restricted rhs 8 per fine cell
BYTES_SMOOTH_FUSED_J3 = 96 + 16 + 16 + 8 + 16 + 8


def log(msg):
    """Progress on stderr (stdout carries the one JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # the GPU needs a few hundred milliseconds of load to reach its steady clock; 30 batch
    # solves (~0.5 s) of warmup keep the clock ramp out of the timed region
    ap.add_argument("--warmup", type=int, default=30)
    # 256 instances: one bottom-of-cycle workgroup per compute unit
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--n", type=int, default=12800)
    ap.add_argument("--levels", type=int, default=8)
    ap.add_argument("--variant", default="sub")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-instances", type=int, default=2, help="oracle instances per host thread")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy first (counter calibration under rocprofv3)")
    ap.add_argument("--vcycle2d-only", action="store_true",
                    help="time only the 2D V-cycle form (1024 x 512 wedge configuration) and print it")
    ap.add_argument("--served-only", action="store_true", help="run only the served forms")
    ap.add_argument("--nmgm21-only", action="store_true",
                    help="run only the NMGM-21 against NMGM-9 form (Table 5 assembly times, wedge solves)")
    ap.add_argument("--wedge2d-only", action="store_true",
                    help="run only the end-to-end 2D wedge form and print it")
    ap.add_argument("--table2-only", action="store_true",
                    help="run only the Table 2 form (E1, NMGM-3 / NMGM-5 / lexicographic Newton-SOR)")
    ap.add_argument("--served-requests", type=int, default=400)
    ap.add_argument("--served-budget-gib", type=int, default=16)
    return ap.parse_args()


def roofline_entry(kernel, bytes_per_launch, flops_per_launch, ms):
    """Roofline of one kernel from its algorithmic bytes and FP64 operations per launch and its
    launch time: bound by HBM when its arithmetic intensity is below the FP64 ridge, else by
    the FP64 vector units; the other resource's use is reported beside it."""
    gbs = bytes_per_launch / (ms * 1e-3) / 1e9
    tflops = flops_per_launch / (ms * 1e-3) / 1e12
    ai = flops_per_launch / bytes_per_launch
    e = {"kernel": kernel, "flop_per_byte": ai, "ridge_flop_per_byte": RIDGE_FLOP_PER_BYTE,
         "algorithmic_bytes_per_launch": bytes_per_launch, "algorithmic_flops_per_launch": flops_per_launch}
    if ai < RIDGE_FLOP_PER_BYTE:
        e.update(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS,
                 fp64_tflops=tflops, fp64_frac=tflops / FP64_VECTOR_TFLOPS)
    else:
        e.update(bound="fp64", achieved=tflops, peak=FP64_VECTOR_TFLOPS, unit="TFLOP/s",
                 frac=tflops / FP64_VECTOR_TFLOPS, hbm_gbs=gbs, hbm_frac=gbs / HBM_PEAK_GBS)
    return e


def measured_traffic(batch, n, fused=False):
    """HBM bytes per launch of the Jacobian kernel from the committed counter summary, or None
    if there is none for this workload and launch form or the kernel source changed since it
    was taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if kv.get("source_sha256") != sha or kv.get("cells") != str(batch * n):
        return None
    if kv.get("fused_residual", "0") != ("1" if fused else "0"):
        return None
    return float(kv["bytes_per_launch"])


def calibration_copy():
    """One device-to-device copy of 256 MiB (the reference dispatch for scaling the FETCH_SIZE
    and WRITE_SIZE counters to bytes)."""
    import torch
    src = torch.ones(32 << 20, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def config2(i, variant, n, levels):
    from swe_workloads import config2 as c2
    return c2(i, variant, n=n, levels=levels)


def make_batch(B, n, levels, variant):
    from swe_workloads import config2
    return [config2(i, variant, n=n, levels=levels) for i in range(B)]


def timed_solves(solver, U0s, steps, warmup, use_graph, profile_kernel=None):
    """Solve the batch warmup + steps times from fresh copies of the initial states (all
    copies made before timing).  Returns (elapsed s, per-solve stats list, kernel ms, launches)."""
    import torch
    sets = [[u.clone() for u in U0s] for _ in range(warmup + steps)]
    torch.cuda.synchronize()
    for w in range(warmup):
        solver.solve(sets[w], use_graph=use_graph)
    if profile_kernel is not None:
        solver.profile(profile_kernel)
        solver.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(steps):
        stats.append(solver.solve(sets[warmup + k], use_graph=use_graph))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kms, kcnt = (0.0, 0)
    if profile_kernel is not None:
        kms, kcnt = solver.profile_read()
        solver.profile(0)
    return el, stats, kms, kcnt, sets[-1]


def smooth2d_runs(C, nu):
    """Launch schedule of nu 2D smoothing iterations: the colour sequence of two symmetric
    multicolour steps per iteration with consecutive equal colours merged, as (colour, passes)."""
    seq = [c for _ in range(nu) for half in range(4)
           for c in (range(C) if half % 2 == 0 else range(C - 1, -1, -1))]
    runs = []
    for c in seq:
        if runs and runs[-1][0] == c:
            runs[-1][1] += 1
        else:
            runs.append([c, 1])
    return runs


def vcycle2d_bytes(nx, ny, levels, nu1, nu2, vsz):
    """Algorithmic bytes of the smoothing in one 2D V-cycle: every launch reads, for each cell of
    its colour, the off-diagonal blocks of the cell's row ((nb - 1) x 9), D^{-1} (9), the
    right-hand side (3) and dU (3), and writes dU (3); neighbour corrections are counted once, as
    the dU writes of their own colour.  Restriction, prolongation and the coarsest solve are not
    counted (a lower bound on the bytes moved)."""
    import numpy as np
    total = 0
    for l in range(levels - 1):
        n_x, n_y = nx >> l, ny >> l
        nb, C = (9, 3) if l == 0 else (5, 2)
        ii, jj = np.meshgrid(np.arange(n_x), np.arange(n_y))
        per_colour = np.bincount(((ii + jj) % C).ravel(), minlength=C)
        for nu in (nu1, nu2):
            for c, _ in smooth2d_runs(C, nu):
                total += int(per_colour[c]) * (9 * nb + 9) * vsz
    return total


def vcycle2d_form():
    import numpy as np
    import torch
    from paper_2505_10857_amd import NMG_FP32_MG, NMG_FP64, Solver2D
    from swe_workloads import synthetic_operator_2d, wedge_problem
    prob = wedge_problem(1024, 512)
    Jo, rhs_o = synthetic_operator_2d(1024, 512, seed=1)
    J = torch.tensor(np.ascontiguousarray(Jo.transpose(2, 3, 4, 0, 1)), dtype=torch.float64, device="cuda:0")
    out = {"workload": "one V-cycle, 1024 x 512 cells, 8 levels, nu1 = nu2 = 20, omega = 0.05, "
                       "seeded J9-shaped operator (the wedge's launch configuration)"}
    for name, prec, dt in (("fp64", NMG_FP64, torch.float64), ("fp32mg", NMG_FP32_MG, torch.float32)):
        s = Solver2D(prob, device="cuda:0", precision=prec)
        rhs = torch.tensor(np.ascontiguousarray(rhs_o.transpose(2, 0, 1)), dtype=dt, device="cuda:0")
        dU = torch.zeros((3, 512, 1024), dtype=dt, device="cuda:0")
        s.vcycle(J, rhs, dU, setup=True)
        s.vcycle(None, rhs, dU, setup=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            s.vcycle(None, rhs, dU, setup=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        vsz = 8 if prec == NMG_FP64 else 4
        b = vcycle2d_bytes(1024, 512, prob.levels, prob.params.nu1, prob.params.nu2, vsz)
        out[name] = {"ms_per_vcycle": ms, "algorithmic_bytes": b, "effective_gbs": b / (ms * 1e-3) / 1e9,
                     "frac_of_hbm_peak": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


def served(args, rate):
    """The request loop of paper_2505_10857_amd.serve on a seeded Poisson stream (FP32 multigrid,
    FP64 residual / update / test); the two smallest results are checked against the oracle."""
    import numpy as np
    import oracle
    from paper_2505_10857_amd import NMG_FP32_MG
    from paper_2505_10857_amd.serve import GpuEngine, Server, stream
    reqs = stream(args.served_requests, rate=rate, seed=0)
    eng = GpuEngine("cuda:0", precision=NMG_FP32_MG)
    # warm-up stream (first allocations, module loads), not reported
    Server(eng, hbm_budget=args.served_budget_gib << 30, steps_per_tick=2).run(stream(16, rate=rate, seed=99))
    server = Server(eng, hbm_budget=args.served_budget_gib << 30, steps_per_tick=2, keep_states=True)
    rep = server.run(reqs)
    out = rep.summary()
    out.update(rate_req_s=rate if rate < 1e6 else "all at t=0", requests=len(reqs),
               n_range=[min(r.prob.n for r in reqs), max(r.prob.n for r in reqs)],
               hbm_budget_gib=args.served_budget_gib)
    errs = []
    for r in sorted(rep.results, key=lambda r: r.n)[:2]:
        Uo, _, _, _ = oracle.Oracle1D(reqs[r.rid].prob).newton_solve()
        errs.append(float(np.abs(r.state.cpu().numpy() - Uo).max()))
    out["max_abs_err_vs_fp64_oracle_two_smallest"] = max(errs) if errs else None
    eng.close()
    return out


def served_mixed(args, rate=200.0, count=2000, frac_2d=0.005):
    """1D and 2D requests on one seeded Poisson stream (2D: the wedge on 64 x 32 to 512 x 256,
    solved by the server's worker threads on streams of their own beside the 1D batch; FP32
    multigrid), with a 2D share the device sustains; the solo 2D service times are reported
    beside it."""
    import numpy as np
    import torch
    from paper_2505_10857_amd import NMG_FP32_MG
    from paper_2505_10857_amd.serve import GpuEngine, Server, stream_mixed
    from paper_2505_10857_amd.solver import Solver2D
    from swe_workloads import SERVED_2D_GRIDS, wedge_problem
    svc = {}
    for nx, ny in SERVED_2D_GRIDS:
        s = Solver2D(wedge_problem(nx, ny, seed=1), device="cuda:0", precision=NMG_FP32_MG, check_every=8)
        U = s.state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, _ = s.newton_solve(U)
        torch.cuda.synchronize()
        svc[f"{nx}x{ny}"] = {"seconds": time.perf_counter() - t0, "newton_steps": st.iters}
    mean_svc = float(np.mean([v["seconds"] for v in svc.values()]))
    reqs = stream_mixed(count, rate=rate, frac_2d=frac_2d, seed=0)
    eng = GpuEngine("cuda:0", precision=NMG_FP32_MG)
    from paper_2505_10857_amd.serve import stream
    Server(eng, hbm_budget=args.served_budget_gib << 30, steps_per_tick=2).run(stream(16, rate=rate, seed=99))
    rep = Server(eng, hbm_budget=args.served_budget_gib << 30, steps_per_tick=2).run(reqs)
    eng.close()
    out = rep.summary()
    out.update(rate_req_s=rate, requests=len(reqs), frac_2d=frac_2d,
               requests_2d=sum(hasattr(r.prob, "ny") for r in reqs), workers_2d=eng.workers_2d,
               solo_2d_service_fp32mg=svc, mean_2d_service_s=mean_svc,
               one_lane_2d_req_s=1.0 / mean_svc)
    return out


def served_overload(args, rate=200.0, frac_2d=0.3, arrive_s=5.0, stop_s=10.0, workers_2d=3, lanes_2d_busy=None):
    """The 70 % 1D / 30 % 2D Poisson stream at 200 req/s (FP32 multigrid, HBM budget 80 % of the
    free device memory), which asks for far more 2D solves than the device completes: arrivals
    for arrive_s seconds, the server stopped at stop_s; the 1D latencies, the 2D completion rate
    (the 2D lane saturated) and the requests left waiting are reported."""
    import torch
    from paper_2505_10857_amd import NMG_FP32_MG
    from paper_2505_10857_amd.serve import GpuEngine, Server, stream, stream_mixed
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    count = int(rate * arrive_s)
    reqs = stream_mixed(count, rate=rate, frac_2d=frac_2d, seed=5)
    eng = GpuEngine("cuda:0", precision=NMG_FP32_MG, workers_2d=workers_2d)
    Server(eng, hbm_budget=budget, steps_per_tick=2).run(stream(16, rate=rate, seed=99))
    Server(eng, hbm_budget=budget, steps_per_tick=2).run(stream_mixed(6, rate=rate, frac_2d=0.5, seed=98))
    rep = Server(eng, hbm_budget=budget, steps_per_tick=2, lanes_2d_busy=lanes_2d_busy).run(reqs, stop_after=stop_s)
    eng.close()
    out = rep.summary()
    n2 = sum(hasattr(r.prob, "ny") for r in reqs)
    out.update(rate_req_s=rate, frac_2d=frac_2d, arrivals_s=arrive_s, stopped_at_s=stop_s,
               requests=count, requests_1d=count - n2, requests_2d=n2, workers_2d=eng.workers_2d,
               lanes_2d_while_1d_busy=lanes_2d_busy,
               hbm_budget_gib=budget / 2**30,
               completed_2d_per_s=out.get("completed_2d", 0) / stop_s)
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args):
    """The oracle as it stands on a bounded sample of the workload, its instances spread over
    the host's cores (one instance per thread at a time; the oracle's C code runs without the
    interpreter lock), median of three runs."""
    import statistics
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    probs = make_batch(args.cpu_instances * threads, args.n, args.levels, args.variant)
    oracle.lib()

    def one(p):
        return oracle.Oracle1D(p).newton_solve()[1]

    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=threads) as ex:
            its = sum(ex.map(one, probs))
        runs.append((time.perf_counter() - t0, its))
    el, its = sorted(runs)[1]
    return {"value": len(probs) / el, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(probs)} instances of the benchmark workload (seeds 0..{len(probs) - 1}), FP64 C "
                      f"oracle, {threads} threads across instances, {its} Newton steps in {el:.1f} s "
                      f"(median of 3 runs: {', '.join(f'{r[0]:.2f}' for r in runs)} s)",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "dof_per_s": 2 * args.n * its / el,
            "runs_s": [r[0] for r in runs]}


def wedge2d_form():
    """The 2D jump over a wedge (section 5.2.2 rescaled), 1024 x 512 cells, 8 levels, solved
    from the uniform inflow state to res < 1e-10 in FP64 and with FP32 multigrid; per-kernel
    launch times; and the error against the oracle's converged state on the 64 x 32 wedge."""
    import numpy as np
    import torch
    import oracle.swe2d
    from paper_2505_10857_amd import NMG_FP32_MG, NMG_FP64, Solver2D
    from paper_2505_10857_amd import _abi as A
    from swe_workloads import wedge_problem
    prob = wedge_problem(1024, 512)
    cells = prob.nx * prob.ny
    out = {"workload": "2D SWE jump over a wedge on [0,40]x[0,30], 1024 x 512 cells, 8 levels, J9, LLF, "
                       "nu = 20, nu3 = 3, omega = 0.05, eps = 1e-6, from the uniform inflow state to res < 1e-10"}
    states = {}
    # the launch schedule of each precision, picked by the autotuner on the operator at the
    # inflow state (outside the timed solves; every schedule gives the same results)
    s64 = Solver2D(prob, device="cuda:0")
    U = s64.state()
    R, rn, _ = s64.residual(U)
    J = s64.jacobian(U, R, rn)
    tuned = {}
    for name, prec, dt in (("fp64", NMG_FP64, torch.float64), ("fp32mg", NMG_FP32_MG, torch.float32)):
        st_ = Solver2D(prob, device="cuda:0", precision=prec)
        best, times = st_.autotune(J, R.to(dt).contiguous(), cycles=2)
        tuned[name] = {"schedule": best, "ms_per_vcycle": {str(k): v for k, v in times.items()}}
        del st_
    del J, s64
    out["autotuned_schedule"] = tuned
    for name, prec in (("fp64", NMG_FP64), ("fp32mg", NMG_FP32_MG)):
        s = Solver2D(prob, device="cuda:0", precision=prec, check_every=8, n_max=2000,
                     schedule=tuned[name]["schedule"])
        U = s.state()
        R, rn, _ = s.residual(U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, hist = s.newton_solve(U, max_hist=2000)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        states[name] = U
        e = {"solves_per_s": 1.0 / el, "seconds_per_solve": el, "newton_steps": st.iters,
             "status": st.status, "res": st.res, "ms_per_newton_step": 1e3 * el / max(st.iters, 1),
             "dof_per_s": 3 * cells * st.iters / el}
        if name == "fp64":
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(5):
                s.residual(U)
            ev[1].record()
            for _ in range(5):
                s.jacobian(U, R, rn)
            ev[2].record()
            torch.cuda.synchronize()
            e["residual_ms"] = ev[0].elapsed_time(ev[1]) / 5
            e["jacobian_j9_ms"] = ev[1].elapsed_time(ev[2]) / 5
        out[name] = e
    out["fp32mg"]["max_abs_diff_vs_fp64_gpu"] = float((states["fp32mg"] - states["fp64"]).abs().max())
    small = wedge_problem(64, 32)
    Uo, ito, reso, _ = oracle.swe2d.Oracle2D(small).newton_solve()
    small_sw = wedge_problem(32, 16)
    Uo_m, _, _, _ = oracle.swe2d.Oracle2D(small_sw).newton_solve()
    Uo_sw, _, _, _ = oracle.swe2d.Oracle2D(small_sw).newton_solve(smoother=1)
    errs = {}
    for name, prec in (("fp64", NMG_FP64), ("fp32mg", NMG_FP32_MG)):
        s = Solver2D(small, device="cuda:0", precision=prec, check_every=8)
        U = s.state()
        st, _ = s.newton_solve(U)
        errs[name] = {"max_abs_err_vs_oracle": float(np.abs(U.cpu().numpy() - Uo).max()),
                      "newton_steps": st.iters, "oracle_newton_steps": ito}
    out["oracle_check_wedge64x32"] = errs
    # the surface reconstruction on the same grid: its residual and J9 launches on the wedge, and
    # still water over a mound and a ripple on 1024 x 512 (max |R|: the paper's scheme against
    # the surface variant)
    import dataclasses
    from swe_workloads import lake_at_rest_2d
    ss = Solver2D(dataclasses.replace(prob, recon=1), device="cuda:0")
    U = ss.state()
    R, rn, _ = ss.residual(U)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(5):
        ss.residual(U)
    ev[1].record()
    for _ in range(5):
        ss.jacobian(U, R, rn)
    ev[2].record()
    torch.cuda.synchronize()
    lake = lake_at_rest_2d(1024, 512, levels=8)
    still = {}
    for name, recon in (("paper", 0), ("surface", 1)):
        sl = Solver2D(dataclasses.replace(lake, recon=recon), device="cuda:0")
        still[name] = float(sl.residual(sl.state(lake.initial_guess()))[0].abs().max())
    # the paper's smoother (directional sweeps D1-D4, one workgroup per level, hyperplane after
    # hyperplane) against the multicolour one on the 32 x 16 wedge: Newton steps, time per solve
    smoothers = {}
    for name, lin in (("multicolour", A.NMG_LINEAR_MG), ("sweeps_d1_d4", A.NMG_LINEAR_MG_SWEEPS)):
        s = Solver2D(small_sw, device="cuda:0", check_every=8, linear=lin)
        U = s.state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, _ = s.newton_solve(U)
        torch.cuda.synchronize()
        smoothers[name] = {"newton_steps": st.iters, "status": st.status, "seconds_per_solve": time.perf_counter() - t0,
                           "max_abs_err_vs_oracle": float(np.abs(U.cpu().numpy() - (Uo_m if lin == A.NMG_LINEAR_MG else Uo_sw)).max())}
    out["smoothers_wedge32x16"] = smoothers
    out["surface_reconstruction"] = {"residual_ms": ev[0].elapsed_time(ev[1]) / 5,
                                     "jacobian_j9_ms": ev[1].elapsed_time(ev[2]) / 5,
                                     "lake_at_rest_1024x512_max_abs_residual": still}
    return out


def table2_form():
    """Section 5.1.1's Table 2 setting on the GPU: E1 (smooth subcritical flow over the bump of
    eq. 26) on 96, 192, 384 and 768 cells, each grid started from the Appendix A interpolation of
    the steady state on half as many cells, solved to res < 1e-11 by NMGM-3, NMGM-5 (4 levels,
    nu1 = nu2 = nu3 = 2, omega = 1, multicolour block SOR) and Newton-SOR with the lexicographic
    symmetric sweep (at most 10 steps per Newton step, stopped at an l1 change below 1e-7):
    Newton steps and milliseconds per solve, beside the printed counts (FP64)."""
    import dataclasses
    import torch
    from paper_2505_10857_amd import NMG_FP64, Solver1D
    from paper_2505_10857_amd.solver import interp_coarse_to_fine
    from swe_workloads import e1_problem
    printed = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "e1_table2.txt")):
        if line.strip() and not line.startswith("#"):
            v = line.split()
            printed[int(v[0])] = {"newton_sor": int(v[1]), "nmgm5": int(v[2]), "nmgm3": int(v[3])}
    solvers = {"nmgm3": (3, {}), "nmgm5": (5, {}),
               "newton_sor_lex": (3, dict(linear=2, sor_max=10, sor_tol=1e-7))}
    out = {}
    for n in (96, 192, 384, 768):
        sc = Solver1D(e1_problem(n // 2), device="cuda:0", precision=NMG_FP64, check_every=1)
        Uc = sc.state()
        stc, _ = sc.newton_solve(Uc)
        U0 = interp_coarse_to_fine(Uc)
        row = {"coarse_steps": stc.iters, "printed_newton_steps": printed.get(n)}
        for name, (jac, over) in solvers.items():
            prob = e1_problem(n)
            prob = dataclasses.replace(prob, params=dataclasses.replace(prob.params, **over))
            s = Solver1D(prob, device="cuda:0", jac=jac, precision=NMG_FP64, check_every=1)
            U = U0.clone()
            s.newton_solve(U.clone())                      # warm-up (allocations, module loads)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, _ = s.newton_solve(U)
            torch.cuda.synchronize()
            row[name] = {"newton_steps": st.iters, "status": st.status, "res": st.res,
                         "ms_per_solve": (time.perf_counter() - t0) * 1e3}
        out[str(n)] = row
    return out


def nmgm21_form():
    """NMGM-21 against NMGM-9 (section 4.1, Table 5's comparison): the time of one Jacobian
    assembly, full J21 against simplified J9, on the parabolic bump at Table 5's three grids and on
    the 1024 x 512 wedge (mean over 20 launches after 3 warm-up launches, HIP events on the
    launching stream, FP64 blocks, residual and norms given); and the 1024 x 512 wedge solved to
    res < 1e-10 by both (Newton steps, seconds, the largest state difference)."""
    import torch
    from paper_2505_10857_amd import NMG_FP64, Solver2D
    from swe_workloads import parabolic_bump_2d, wedge_problem
    out = {"assembly_ms": {}}
    for name, prob in (("bump16x8", parabolic_bump_2d(16, 8)), ("bump32x16", parabolic_bump_2d(32, 16)),
                       ("bump64x32", parabolic_bump_2d(64, 32)), ("wedge1024x512", wedge_problem(1024, 512))):
        row = {}
        for jac in (9, 21):
            s = Solver2D(prob, device="cuda:0", jac=jac)
            U = s.state()
            R, rn, _ = s.residual(U)
            for _ in range(3):
                s.jacobian(U, R, rn)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(20):
                s.jacobian(U, R, rn)
            ev[1].record()
            torch.cuda.synchronize()
            row[f"J{jac}"] = ev[0].elapsed_time(ev[1]) / 20
        row["ratio_J21_over_J9"] = row["J21"] / row["J9"]
        out["assembly_ms"][name] = row
    prob = wedge_problem(1024, 512)
    states = {}
    for jac in (9, 21):
        log(f"form nmgm21_vs_nmgm9: wedge 1024 x 512 solve with J{jac}")
        s = Solver2D(prob, device="cuda:0", precision=NMG_FP64, check_every=8, n_max=2000, jac=jac)
        U = s.state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, _ = s.newton_solve(U)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        states[jac] = U
        out[f"wedge1024x512_nmgm{jac}"] = {"seconds_per_solve": el, "newton_steps": st.iters, "status": st.status,
                                           "res": st.res, "ms_per_newton_step": 1e3 * el / max(st.iters, 1)}
    out["wedge1024x512_max_abs_diff_nmgm21_vs_nmgm9"] = float((states[21] - states[9]).abs().max())
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this build runs on "
              f"one MI355X; independent instances would shard across GPUs without communication).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2505_10857_amd import NMG_FP32_MG, NMG_FP64, BatchSolver1D
    from paper_2505_10857_amd import _abi as A

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        calibration_copy()
    if args.vcycle2d_only:
        print(json.dumps({"mg2d_vcycle_wedge1024x512": vcycle2d_form()}))
        return
    if args.wedge2d_only:
        print(json.dumps({"wedge2d_1024x512": wedge2d_form()}))
        return
    if args.served_only:
        print(json.dumps({"served_200rps": served(args, 200.0), "served_mixed_1d_2d": served_mixed(args),
                          "served_overload_70_30": served_overload(args)}))
        return
    if args.nmgm21_only:
        print(json.dumps({"nmgm21_vs_nmgm9": nmgm21_form()}))
        return
    if args.table2_only:
        print(json.dumps({"table2_e1": table2_form()}))
        return
    use_graph = not args.no_graph
    probs = make_batch(args.batch, args.n, args.levels, args.variant)
    solver = BatchSolver1D(probs, device="cuda:0", jac=3, precision=NMG_FP64)
    U0s = solver.states()
    # the plan's schedule is picked by the autotuner on this workload (outside the timed region)
    log("autotuning the plan options")
    tune_best, tune_times = solver.autotune([u.clone() for u in U0s], trial_steps=3, use_graph=use_graph)
    log(f"timed region: {args.warmup} warmup + {args.steps} batch solves")

    # ---- main timed region -------------------------------------------------------------------
    el, stats, _, _, Ulast = timed_solves(solver, U0s, args.steps, args.warmup, use_graph)
    newton = [s[0] for s in stats[-1]]
    ok = all(s[1] == 0 and s[2] < 1e-10 for st in stats for s in st)
    nsolves = args.batch * args.steps
    value = nsolves / el
    dofs = sum(2 * args.n * s[0] for st in stats for s in st) / el
    out = {
        "metric": "steady solves/s at FP64 res < 1e-10 (NMGM-3)",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"1D SWE flow over a hump on [0,25], N={args.n}, {args.levels} levels, "
                               f"{args.variant}critical, J3, FP64, batch of {args.batch} seeded instances "
                               f"per step solved to res<1e-10",
                   "n": args.n, "levels": args.levels, "batch": args.batch, "variant": args.variant,
                   "hip_graph": use_graph,
                   "autotuned": {"bottom_cells": tune_best["bottom_cells"],
                                 "smooth_tile": tune_best["smooth_tile"],
                                 "split_finest": tune_best["split_finest"],
                                 "split_residual": tune_best["split_residual"],
                                 "ms_per_newton_step": {f"bottom{b}_split{sp}_tile{t}_res{r}": ms
                                                        for (b, sp, t, r), ms in tune_times.items()}}},
        "dof_per_s": dofs,
        "newton_steps_per_solve": [min(newton), max(newton)],
        "converged": ok,
    }

    log(f"headline {value:.1f} solves/s; kernel timings")
    # ---- roofline of the dominant kernel: HIP events around its launches on the launch stream --
    el2, stj, jms, jcnt, _ = timed_solves(solver, U0s, 2, 0, False, A.NMG_K_JACOBIAN)
    _, stp, pms, pcnt, _ = timed_solves(solver, U0s, 2, 0, False, A.NMG_K_SMOOTH_PRE)
    fused = solver.options()["fused_finest"]
    if fused:
        _, stf, fms, fcnt, _ = timed_solves(solver, U0s, 2, 0, False, A.NMG_K_SMOOTH_FUSED)
    cells = args.batch * args.n
    # instances drop out of every launch once converged, so the work of the timed launches is
    # counted per active instance: the Jacobian runs once per Newton step of an instance, the
    # finest pre-smoothing once per V-cycle (nu3 = 2 per step); "full launches" = that work in
    # units of one launch over the whole batch
    fused_res = tune_best["split_residual"] == 0
    # fused order: one Jacobian launch per Newton step plus the one that begins the solve
    jac_full = sum(s[0] + (1 if fused_res else 0) for st in stj for s in st) / args.batch
    # finest pre-smoothing launches per Newton step: one per V-cycle, or only the first one
    # when the plan runs each later one together with the previous post-smoothing
    pre_per_step = 1 if fused else 2
    pre_full = pre_per_step * sum(s[0] for st in stp for s in st) / args.batch
    pre_bytes = BYTES_SMOOTH_PRE_J3 + (0 if fused else 8)   # unfused: dU read in the 2nd cycle
    jac_ms = jms / jac_full       # time of one launch over the whole batch
    pre_ms = pms / pre_full
    if fused_res:
        jac_flops, jac_bytes = cells * FLOPS_JACOBIAN_J3_FUSED, cells * BYTES_JACOBIAN_J3_FUSED
        jac_name = ("k_jacobian_batch<double,3,false,true> (residual eq. 10 + FD Jacobian J3 eq. 12-13 "
                    "+ coarse operators eq. 17, one launch)")
    else:
        jac_flops, jac_bytes = cells * FLOPS_JACOBIAN_J3, cells * BYTES_JACOBIAN_J3
        jac_name = "k_jacobian_batch<double,3,false,false> (FD Jacobian J3, eq. 12-13, with the coarse operators of eq. 17)"
    out["roofline"] = roofline_entry(jac_name, jac_bytes, jac_flops, jac_ms)
    out["roofline"].update({
        "traffic": measured_traffic(args.batch, args.n, fused_res),
        "avg_launch_ms": jms / max(jcnt, 1), "launches_timed": jcnt, "full_launch_ms": jac_ms,
        "full_launch_equivalents": jac_full, "share_of_solve_time": jms / (el2 * 1e3),
    })
    if not fused_res:
        _, str_, rms, rcnt, _ = timed_solves(solver, U0s, 2, 0, False, A.NMG_K_RESIDUAL)
        # the residual runs once at the start of a solve and once per Newton step of every
        # active instance
        res_full = sum(s[0] + 1 for st in str_ for s in st) / args.batch
        res_ms = rms / res_full
        out["residual_roofline"] = roofline_entry("k_residual_batch (eq. 10 and ||R_j||_1)", cells * BYTES_RESIDUAL,
                                                  cells * FLOPS_LOCAL_RESIDUAL, res_ms)
        out["residual_roofline"].update({"avg_launch_ms": rms / max(rcnt, 1), "launches_timed": rcnt,
                                         "full_launch_ms": res_ms})
    out["smoother_roofline"] = {
        "kernel": "k_smooth<double,3> mode 0, finest level (pre-smoothing + restriction)",
        "bound": "hbm", "avg_launch_ms": pms / max(pcnt, 1), "launches_timed": pcnt, "full_launch_ms": pre_ms,
        "full_launch_equivalents": pre_full,
        "achieved": cells * pre_bytes / (pre_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": cells * pre_bytes / (pre_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "note": "working set below the 256 MB Infinity Cache: effective GB/s",
    }
    if fused:
        # one launch per Newton step (nu3 = 2): post-smoothing of the first V-cycle and
        # pre-smoothing of the second on the finest level
        f_full = sum(s[0] for st in stf for s in st) / args.batch
        f_ms = fms / f_full
        out["smoother_fused_roofline"] = {
            "kernel": "k_smooth<double,3> mode 2, finest level (prolongation + post- and pre-smoothing + restriction)",
            "bound": "hbm", "avg_launch_ms": fms / max(fcnt, 1), "launches_timed": fcnt, "full_launch_ms": f_ms,
            "full_launch_equivalents": f_full,
            "achieved": cells * BYTES_SMOOTH_FUSED_J3 / (f_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": cells * BYTES_SMOOTH_FUSED_J3 / (f_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        }

    # ---- extra forms --------------------------------------------------------------------------
    if not args.no_extras:
        forms = {}
        # single instance, one solve at a time
        single = BatchSolver1D(probs[:1], device="cuda:0", jac=3, precision=NMG_FP64)
        u1 = single.states()
        e1, st1, _, _, _ = timed_solves(single, u1, 20, 10, use_graph)
        log("form fp64_single_instance")
        forms["fp64_single_instance"] = {"solves_per_s": 20 / e1, "latency_ms": 1e3 * e1 / 20,
                                         "newton_steps": st1[-1][0][0]}
        # full Jacobian J5, batched
        s5 = BatchSolver1D(probs, device="cuda:0", jac=5, precision=NMG_FP64)
        e5, st5, _, _, _ = timed_solves(s5, s5.states(), args.steps, 5, use_graph)
        log("form fp64_batch_J5")
        forms["fp64_batch_J5"] = {"solves_per_s": args.batch * args.steps / e5,
                                  "newton_steps": [min(s[0] for s in st5[-1]), max(s[0] for s in st5[-1])]}
        forms["fp64_batch_J3"] = {"solves_per_s": value, "newton_steps": out["newton_steps_per_solve"]}
        # FP32 multigrid, FP64 residual / update / test
        s32 = BatchSolver1D(probs, device="cuda:0", jac=3, precision=NMG_FP32_MG)
        e32, st32, _, _, U32 = timed_solves(s32, s32.states(), args.steps, 5, use_graph)
        err = max(float((a - b).abs().max()) for a, b in zip(U32, Ulast))
        log("form fp32mg_batch_J3")
        # both forms iterated on to the round-off floor (res < 1e-13), where the 1e-9 bar of the
        # FP32-multigrid form is defined (at the res < 1e-10 stop the two stop at different
        # iterates)
        import dataclasses
        fl = {}
        for nm, prc in (("fp64", NMG_FP64), ("fp32mg", NMG_FP32_MG)):
            fprobs = [dataclasses.replace(p, params=dataclasses.replace(p.params, tol=1e-13, n_max=5000))
                      for p in probs]
            sf = BatchSolver1D(fprobs, device="cuda:0", jac=3, precision=prc)
            Uf = sf.states()
            stf = sf.solve(Uf, use_graph=use_graph)
            fl[nm] = (Uf, stf)
            del sf
        err_floor = max(float((a - b).abs().max()) for a, b in zip(fl["fp32mg"][0], fl["fp64"][0]))
        forms["fp32mg_batch_J3"] = {"solves_per_s": args.batch * args.steps / e32,
                                    "newton_steps": [min(s[0] for s in st32[-1]), max(s[0] for s in st32[-1])],
                                    "max_abs_diff_vs_fp64_gpu": err,
                                    "max_abs_diff_vs_fp64_gpu_at_roundoff_floor": err_floor,
                                    "roundoff_floor_res": max(s[2] for s in fl["fp32mg"][1]),
                                    "converged": all(s[1] == 0 and s[2] < 1e-10 for st in st32 for s in st)}
        # the well-balanced surface reconstruction (WENO3 on H + zbar) on the same batch
        import dataclasses
        sprobs = [dataclasses.replace(p, recon=1) for p in probs]
        ssurf = BatchSolver1D(sprobs, device="cuda:0", jac=3, precision=NMG_FP64)
        esf, stsf, _, _, Usf = timed_solves(ssurf, ssurf.states(), args.steps, 5, use_graph)
        log("form fp64_batch_J3_surface")
        forms["fp64_batch_J3_surface"] = {
            "solves_per_s": args.batch * args.steps / esf,
            "newton_steps": [min(s[0] for s in stsf[-1]), max(s[0] for s in stsf[-1])],
            "converged": all(s[1] == 0 and s[2] < 1e-10 for st in stsf for s in st),
            "max_abs_diff_vs_conserved_reconstruction": max(float((a - b).abs().max()) for a, b in zip(Usf, Ulast))}
        del ssurf
        # Newton-SOR (the paper's reference solver: <= 10 multicolour block-SOR steps per Newton
        # step) against NMGM-3 on 256 config-1 instances (N = 200)
        from swe_workloads import config1
        c1 = [config1(i) for i in range(args.batch)]
        cmp1 = {}
        for name, lin in (("nmgm3", A.NMG_LINEAR_MG), ("newton_sor", A.NMG_LINEAR_SOR)):
            pp = [dataclasses.replace(p, params=dataclasses.replace(p.params, linear=lin)) for p in c1]
            sb = BatchSolver1D(pp, device="cuda:0", jac=3, precision=NMG_FP64)
            eb, stb, _, _, _ = timed_solves(sb, sb.states(), 1, 1, use_graph)
            last = stb[-1]
            cmp1[name] = {"solves_per_s": args.batch / eb,
                          "newton_steps": [min(x[0] for x in last), max(x[0] for x in last)],
                          "converged": sum(1 for x in last if x[1] == 0 and x[2] < 1e-10)}
            del sb
        log("form fp64_cfg1_nmgm3_vs_newton_sor")
        forms["fp64_cfg1_nmgm3_vs_newton_sor"] = cmp1
        log("form table2_e1")
        forms["table2_e1"] = table2_form()
        # transcritical hump (q = 1.53, h_out = 0.66): out of reach of plain Newton from the flat
        # surface; nested iteration (Algorithm 3) over the 8 grids 100 .. 12800, batched per grid
        from paper_2505_10857_amd.solver import NestedBatch
        tprobs = [config2(i, "trans", n=args.n, levels=args.levels) for i in range(args.batch)]
        nb_ = NestedBatch(tprobs, device="cuda:0", precision=NMG_FP64)
        sets = [nb_.states() for _ in range(3)]
        torch.cuda.synchronize()
        nb_.solve(sets[0], use_graph)                 # warmup (captures the graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = [nb_.solve(sets[k], use_graph) for k in (1, 2)]
        torch.cuda.synchronize()
        et = time.perf_counter() - t0
        fin = rep[-1][-1]
        log("form fp64_batch_trans_nested")
        forms["fp64_batch_trans_nested"] = {
            "solves_per_s": 2 * args.batch / et, "batch": args.batch,
            "newton_steps_finest": [min(x[0] for x in fin), max(x[0] for x in fin)],
            "newton_steps_per_grid_instance0": [r[0][0] for r in rep[-1]],
            "converged": all(x[1] == 0 and x[2] < 1e-10 for x in fin)}
        del nb_, sets
        # the same with the full Jacobian J5 on every multigrid grid (the coarsest, solved
        # directly, keeps J3): full against simplified Jacobian on the transcritical variant
        nb5 = NestedBatch(tprobs, device="cuda:0", precision=NMG_FP64, jac=5)
        sets = [nb5.states() for _ in range(3)]
        torch.cuda.synchronize()
        nb5.solve(sets[0], use_graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep5 = [nb5.solve(sets[k], use_graph) for k in (1, 2)]
        torch.cuda.synchronize()
        et5 = time.perf_counter() - t0
        fin5 = rep5[-1][-1]
        forms["fp64_batch_trans_nested_J5"] = {
            "solves_per_s": 2 * args.batch / et5, "batch": args.batch,
            "newton_steps_finest": [min(x[0] for x in fin5), max(x[0] for x in fin5)],
            "newton_steps_per_grid_instance0": [r[0][0] for r in rep5[-1]],
            "converged": all(x[1] == 0 and x[2] < 1e-10 for x in fin5)}
        del nb5, sets
        # uneven batch: 512 instances, N log-uniform in [256, 16384], FP32 multigrid, one plan
        from swe_workloads import config4_instance
        uprobs = [config4_instance(i) for i in range(512)]
        su = BatchSolver1D(uprobs, device="cuda:0", jac=3, precision=NMG_FP32_MG)
        eu, stu, _, _, _ = timed_solves(su, su.states(), 3, 2, use_graph)
        ucells = sum(p.n for p in uprobs)
        log("form fp32mg_uneven512")
        forms["fp32mg_uneven512"] = {
            "solves_per_s": 512 * 3 / eu, "cells_per_batch": ucells,
            "dof_per_s": sum(2 * p.n * st[0] for sts in stu for p, st in zip(uprobs, sts)) / eu,
            "newton_steps": [min(st[0] for st in stu[-1]), max(st[0] for st in stu[-1])],
            "converged": all(st[1] == 0 and st[2] < 1e-10 for sts in stu for st in sts)}
        # 2D multigrid at the wedge's size and launch configuration (1024 x 512, 8 levels,
        # nu = 20, omega = 0.05) on a seeded J9-shaped operator
        log("form mg2d_vcycle_wedge1024x512")
        forms["mg2d_vcycle_wedge1024x512"] = vcycle2d_form()
        # the same wedge solved end to end (Newton with the 2D residual, J9 and V-cycles)
        log("form wedge2d_1024x512")
        forms["wedge2d_1024x512"] = wedge2d_form()
        log("form nmgm21_vs_nmgm9")
        forms["nmgm21_vs_nmgm9"] = nmgm21_form()
        # continuous-batching server: Poisson arrivals at 200 req/s, N in [512, 32768]
        log("form served_200rps")
        forms["served_200rps"] = served(args, 200.0)
        log("form served_saturated")
        forms["served_saturated"] = served(args, 1e7)
        log("form served_mixed_1d_2d")
        forms["served_mixed_1d_2d"] = served_mixed(args)
        log("form served_overload_70_30")
        forms["served_overload_70_30"] = served_overload(args)
        out["forms"] = forms

    # ---- CPU oracle ----------------------------------------------------------------------------
    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
