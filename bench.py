"""Benchmark: forward solve + VJP pairs per second on one MI355X.

Workload: 256^3 cells (257^3 vertices), log D and log mua Gaussian random
fields (power spectrum k^-3, std 1, means log 1 and log 0.05, D contrast
<= 1e4), source = 16 Gaussian blobs + N(0, 0.01^2) noise, cotangent N(0, 1);
float32 V(2,2)-cycles inside float64 iterative refinement, forward and
pull-back each to 1e-10 relative residual.  One step = coefficient set-up
(exp, validation, hierarchy) + forward solve + pull-back with all three
gradients, on inputs already resident in device memory.  The forward and
adjoint solves of a step run concurrently (dmgs_forward_vjp) unless
--sequential.

Prints one JSON line.  `value` comes from the first timed region.  A second
timed region runs the same steps with the two solves one after the other;
the dominant kernel's roofline figure comes from HIP events around its
launches there (on its launch stream), where no other stream's kernels
stretch its duration.  The CPU baseline is the FP64 oracle timed on a
bounded sample of the same workload on the host cores.
"""
import argparse
import math
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def host_cpu():
    """The host's CPU model, its logical CPU count and the ones this process
    may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return model, os.cpu_count() or avail, avail


def cpu_baseline(c, smoother="rbgs", reps=3):
    """Time the oracle on whole fwd+VJP pairs of the benchmark's own workload:
    hierarchy set-up, forward solve to the benchmark's tolerance, pull-back
    to the same tolerance with the three gradients; the median of `reps`
    pairs (each pair is timed whole, so one-off costs count once per pair)."""
    from oracle import ref
    times, cyc = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        H = ref.Hierarchy(c["D"], c["mua"], smoother=smoother)
        rho, fi = H.forward(c["q"], rtol=1e-10)
        _, ai = H.vjp(rho, c["rhobar"], rtol=1e-10)
        times.append(time.perf_counter() - t0)
        cyc = (fi["cycles"], ai["cycles"])
        del H, rho
    times.sort()
    pair_s = times[len(times) // 2]
    model, nlog, avail = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", avail))
    return {"value": 1.0 / pair_s, "unit": "fwd+VJP pairs/s", "cores": min(threads, avail), "kind": "oracle",
            "cpu_model": model, "nproc": avail, "logical_cpus": nlog,
            "sample": "median of %d whole fwd+VJP pairs at N=%d (set-up, forward to 1e-10 in %d V-cycles, pull-back "
                      "to 1e-10 in %d V-cycles with gradients; FP64, C/OpenMP): %s s"
                      % (reps, c["N"], cyc[0], cyc[1], ", ".join("%.2f" % t for t in times))}


def sweep_cpu_baseline(nd, logD, logmu, q, w):
    """The oracle beside one line of the benchmark sweep, on a bounded
    sample: hierarchy set-up plus 2 fixed float64 V-cycles of the solve and 2
    of the pull-back (with gradients), scaled to the sweep's 15 cycles."""
    import numpy as np
    from oracle import ref, ref2d
    D, mu = np.exp(logD), np.exp(logmu)
    t0 = time.perf_counter()
    H = ref.Hierarchy(D, mu) if nd == 3 else ref2d.Hierarchy2D(D, mu)
    t1 = time.perf_counter()
    rho, _ = H.forward(q, fixed_cycles=2)
    t2 = time.perf_counter()
    H.forward(q, fixed_cycles=4)
    t3 = time.perf_counter()
    H.vjp(rho, w, fixed_cycles=2)
    t4 = time.perf_counter()
    H.vjp(rho, w, fixed_cycles=4)
    t5 = time.perf_counter()
    # per-cycle costs from the differences (4 - 2 cycles), so the calls'
    # one-off work (iterate set-up, gradients) is counted once
    setup, f2, f4, a2, a4 = t1 - t0, t2 - t1, t3 - t2, t4 - t3, t5 - t4
    fc, ac = max(f4 - f2, 0.0) / 2, max(a4 - a2, 0.0) / 2
    _, _, avail = host_cpu()
    cores = min(int(os.environ.get("OMP_NUM_THREADS", avail)), avail) if nd == 3 else 1
    return {"solve_ms": 1e3 * (setup + f2 + 13 * fc), "vjp_ms": 1e3 * (setup + a2 + 13 * ac),
            "cores": cores, "kind": "oracle",
            "sample": "set-up %.2fs; 2 and 4 forward cycles %.2fs / %.2fs; 2 and 4 pull-back cycles with gradients "
                      "%.2fs / %.2fs; per-cycle cost from the difference, extended to 15 cycles (FP64, %s)"
                      % (setup, f2, f4, a2, a4, "C/OpenMP" if nd == 3 else "numpy")}


def serving_leg(nreq):
    """The serving stream: nreq requests, grid sizes uniform over {64, 96, 128,
    192}^3, 50/50 forward+JVP / forward+VJP, each with its own seeded fields.
    First all at t = 0 (saturation throughput), then Poisson arrivals at 0.8 x
    that rate for p50/p99 latency."""
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.serving import Request, Server, TickServer, summarize
    budget = 96 << 30

    def reqs(rate):
        return [Request(id=d["id"], N=d["N"], mode=d["mode"], seed=d["seed"], arrival=d["arrival"])
                for d in synth.serving_stream(nreq=nreq, rate=rate)]

    def measure(srv, other_rate=None):
        srv.run(reqs(None)[:16], realtime=False)      # warm-up: plans for every size
        burst = summarize(srv.run(reqs(None), realtime=False))
        rate = 0.8 * burst["requests_per_s"]
        pois = summarize(srv.run(reqs(rate), realtime=True))
        out = {"saturation_requests_per_s": burst["requests_per_s"], "saturation_solves_per_s": burst["solves_per_s"],
               "poisson_rate_per_s": rate, "p50_ms": pois["p50_ms"], "p99_ms": pois["p99_ms"],
               "requests_per_s": pois["requests_per_s"], "solves_per_s": pois["solves_per_s"],
               "errors": pois["errors"] + burst["errors"]}
        if other_rate:   # latency at the other server's arrival rate
            same = summarize(srv.run(reqs(other_rate), realtime=True))
            out["at_thread_rate"] = {"poisson_rate_per_s": other_rate, "p50_ms": same["p50_ms"],
                                     "p99_ms": same["p99_ms"], "errors": same["errors"]}
        out["peak_accounted_GB"] = srv.adm.peak / 1e9
        srv.close()
        return out

    out = {"requests": nreq, "sizes": [64, 96, 128, 192], "modes": "50/50 fwd+JVP / fwd+VJP", "budget_GB": budget / 1e9,
           "max_slots": 8, "server": "one HIP stream per admitted request (threads)"}
    out.update(measure(Server(budget_bytes=budget, max_slots=8, keep_results=False)))
    # the same streams through grouped ticks (dmgs_batch_*)
    tick = TickServer(budget_bytes=budget, max_slots=8, keep_results=False)
    g = measure(tick, out["poisson_rate_per_s"])
    g["grouped_launches"], g["recorded_launches"] = tick.batch_stats["launches"], tick.batch_stats["recorded"]
    g["server"] = ("grouped ticks (dmgs_batch_*): a batch per grid size, each ticked on its own stream; a tick runs "
                   "one refinement step of every request of the batch and synchronises once")
    out["grouped_ticks"] = g
    return out


def config5_leg(reps=3):
    """512^3 (134M cells) forward + VJP through the torch.autograd.Function:
    GRF log-normal coefficients (clipped to a D contrast <= 1e4) and a
    16-blob source drawn on the device, float32 V-cycles inside float64
    refinement to 1e-10.  One untimed pair, then `reps` timed pairs (each
    the differentiable forward solve and torch.autograd.grad of <w, rho>
    with respect to q, log D and log mua); peak device memory = torch's peak
    allocation + the plan's bytes."""
    import torch
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.autograd import Solver
    N = 512
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(5000)
    logD = synth.grf_torch(N, g, dev).clamp_(-math.log(100.0), math.log(100.0))
    logmua = math.log(0.05) + synth.grf_torch(N, g, dev)
    q = synth.blob_source_torch(N, g, dev)
    w = synth.zero_boundary_torch(torch.randn(q.shape, generator=g, device=dev, dtype=torch.float64))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    S = Solver(N, precision="fp32-in-fp64")
    qv, lD, lm = (t.requires_grad_(True) for t in (q, logD, logmua))

    def pair():
        rho = S(qv, lD, lm)
        grads = torch.autograd.grad((rho * w).sum(), (qv, lD, lm))
        return rho, grads
    pair()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rho, grads = pair()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
        del rho, grads
    times.sort()
    ms = times[len(times) // 2]
    fi = S.plan._last_forward[1]
    rho = S(qv, lD, lm)
    (qb, _, _), vi = S.plan.vjp(rho.detach(), w, coef_grads=False)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() + S.plan.bytes
    nv = (N + 1) ** 3
    levels = sum(((N >> k) + 1) ** 3 for k in range(S.plan.levels)) / nv
    vc = fi["vcycles"] + vi["vcycles"]
    model = 26.25 * 4 * nv * levels * vc
    out = {"workload": "512^3 cells, GRF log-normal D (contrast <= 1e4) and mua, 16-blob source, fp32-in-fp64, "
                       "rtol 1e-10, forward + VJP through torch.autograd.Function",
           "ms_per_pair": ms, "ms_reps": times, "pairs_per_s": 1e3 / ms,
           "peak_device_GB": peak / 1e9, "torch_peak_GB": torch.cuda.max_memory_allocated() / 1e9,
           "plan_GB": S.plan.bytes / 1e9, "vcycles_fwd": fi["vcycles"], "vcycles_adj": vi["vcycles"],
           "rel_residual_fwd": fi["rel_residual"], "rel_residual_adj": vi["rel_residual"],
           "vcycle_model_GBps": model / (ms * 1e-3) / 1e9,
           "vcycle_model_frac": model / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
           "note": "model GB/s = the one-pass V-cycle byte model (26.25 words per fine vertex, all levels) times "
                   "the pair's V-cycles over the whole pair's time (refinement, set-up and gradient passes "
                   "included, so a lower bound)"}
    S.close()
    return out


def kernel_source_hash():
    """sha256 over the name and contents of the sources that define the
    dominant kernel's device code (the three-dimensional streaming passes:
    csrc/grid.hpp, kernels_stream.hpp, kernels_sweep2.hpp, in that order)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2608_00760_amd", "csrc")
    h = hashlib.sha256()
    for f in [os.path.join(csrc, n) for n in ("grid.hpp", "kernels_stream.hpp", "kernels_sweep2.hpp")]:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the kernel sources changed since the counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", "level0_sweep_256_traffic.md")
    try:
        with open(path) as fh:
            m = re.search(r"```json\n(.*?)```", fh.read(), re.S)
        rec = json.loads(m.group(1))
    except (OSError, AttributeError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec["traffic_bytes_per_launch"]


def run_steps(P, t, bufs, steps, sequential=False):
    """steps x (coefficient set-up, forward solve, VJP with gradients).  By
    default the forward and adjoint solves run concurrently
    (dmgs_forward_vjp); sequential: dmgs_forward, then dmgs_vjp."""
    info_f = info_a = None
    for _ in range(steps):
        P.set_log_coefficients(t["logD"], t["logmua"])
        if sequential:
            _, info_f = P.forward(t["q"], out=bufs[0])
            _, info_a = P.vjp(bufs[0], t["rhobar"], out=bufs[1:])
        else:
            _, info_f, info_a = P.forward_vjp(t["q"], t["rhobar"], out=bufs)
    return info_f, info_a


def paper_sweep(args):
    """The paper's timing benchmark shape (Sec. 3.3) on this solver: fixed 15
    V-cycles per solve, Solve / JVP / VJP timed separately over grid sizes,
    with peak device memory.  Coefficients are seeded log-normal fields drawn
    on the device (the timing of a fixed cycle count does not depend on their
    values).  One JSON line per size and precision."""
    import torch
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options, Plan
    dev = torch.device("cuda:0")
    nd = args.sweep_ndim
    sizes = [int(x) for x in (args.sweep_sizes or
                              ("768,1024,1536,2048,3072,4096,6144,8192" if nd == 2 else
                               "96,128,192,256,384,512,768")).split(",")]
    for N in sizes:
        for prec in (("fp64",) if nd == 2 else ("fp64", "fp32-in-fp64")):
            torch.cuda.empty_cache()
            torch.cuda.reset_peak_memory_stats()
            g = torch.Generator(device=dev)
            g.manual_seed(7000 + N)
            shape = (N + 1,) * nd
            rnd = lambda: torch.randn(shape, generator=g, device=dev, dtype=torch.float64)
            logD, logmu = 0.5 * rnd(), -3.0 + 0.5 * rnd()
            q, w, dq, dd, dm = rnd(), rnd(), rnd(), rnd(), rnd()
            for t in (q, w, dq, dm):   # boundary entries are ignored; keep them 0
                synth.zero_boundary_torch(t)
            # 15 V-cycles: float64 cycles, or 15 refinement steps of one float32 cycle
            P = Plan(Options(N, precision=prec, fixed_cycles=15, ir_inner_cycles=1, ir_adaptive=False, ndim=nd))
            P.set_log_coefficients(logD, logmu)
            rho, qbar, drho = torch.empty_like(q), torch.empty_like(q), torch.empty_like(q)
            gD, gmu = torch.empty_like(q), torch.empty_like(q)
            ops = {"solve": lambda: P.forward(q, out=rho),
                   "jvp": lambda: P.jvp(rho, dq, dd, dm, out=drho),
                   "vjp": lambda: P.vjp(rho, w, out=(qbar, gD, gmu))}
            res = {}
            for name, f in ops.items():
                f()
                torch.cuda.synchronize()
                ts = []
                for _ in range(args.sweep_reps):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    f()
                    e1.record()
                    e1.synchronize()
                    ts.append(e0.elapsed_time(e1))
                ts.sort()
                res[name + "_ms_median"] = ts[len(ts) // 2]
                res[name + "_ms_min"] = ts[0]
            torch.cuda.synchronize()
            peak = torch.cuda.max_memory_allocated() + P.bytes
            # one more solve with every finest-level launch timed: the
            # smoothing kernel's achieved bandwidth against the HBM peak
            P.timing(True, stride=1)
            ops["solve"]()
            torch.cuda.synchronize()
            per_class = P.timing_read()
            sm = per_class["smooth"]
            P.timing(False)
            # the unrolled adjoint (exact derivative of the 15-cycle map in
            # log D and log mua, through every step) for float64 3D plans
            unrolled = None
            if nd == 3 and prec == "fp64" and N <= args.sweep_unrolled_max:
                # the first call allocates the plan's work buffers for it (the
                # recorded states of every cycle, or checkpoints): measured
                # as the device memory it takes
                free0 = torch.cuda.mem_get_info()[0]
                P.vjp_unrolled(q, w)
                torch.cuda.synchronize()
                work = free0 - torch.cuda.mem_get_info()[0]
                tu = []
                for _ in range(3):
                    t0u = time.perf_counter()
                    P.vjp_unrolled(q, w)
                    tu.append((time.perf_counter() - t0u) * 1e3)
                tu.sort()
                unrolled = {"ms_median": tu[1], "work_GB": work / 1e9,
                            "vs_vjp": tu[1] / res["vjp_ms_median"]}
            cpu = None
            if args.sweep_cpu_baseline and prec == "fp64" and N <= (256 if nd == 3 else 1024):
                cpu = sweep_cpu_baseline(nd, *(t.cpu().numpy() for t in (logD, logmu, q, w)))
            gbps = sm["bytes"] / (sm["ms"] * 1e-3) / 1e9 if sm["ms"] > 0 else None
            print(json.dumps({"sweep": "fixed 15 V-cycles", "ndim": nd, "N": N, "points": (N + 1) ** nd,
                              "log2_points": round(math.log2((N + 1) ** nd), 2), "precision": prec,
                              "reps": args.sweep_reps, **res, "peak_device_GB": peak / 1e9,
                              "smooth_kernel": {"launches": sm["launches"],
                                                "avg_us": 1e3 * sm["ms"] / max(sm["launches"], 1),
                                                "GBps": gbps, "frac": gbps / HBM_PEAK_GBPS if gbps else None},
                              "finest_level_ms_per_solve": {k: v["ms"] for k, v in per_class.items() if v["launches"]},
                              "vjp_unrolled": unrolled, "cpu_baseline": cpu}),
                  flush=True)
            P.close()
            del logD, logmu, q, w, dq, dd, dm, rho, qbar, drho, gD, gmu


def graph_replay(args):
    """The fixed-cycle forward solve (15 V-cycles, NULL info: no host waits)
    launched eagerly and replayed from a captured HIP graph, on the same
    stream; median of --sweep-reps calls each, one JSON line per case."""
    import ctypes as C
    import torch
    from paper_2608_00760_amd import _abi, synth
    from paper_2608_00760_amd.solver import Options, Plan
    lib = _abi.lib()
    dev = torch.device("cuda:0")
    cases = [(3, 96, "fp64"), (3, 96, "fp32-in-fp64"), (3, 128, "fp64"), (2, 768, "fp64"), (2, 1024, "fp64")]
    for nd, N, prec in cases:
        g = torch.Generator(device=dev)
        g.manual_seed(4000 + N)
        shape = (N + 1,) * nd
        logD = synth.grf_torch(N, g, dev, ndim=nd).clamp_(-math.log(100.0), math.log(100.0))
        logmua = math.log(0.05) + synth.grf_torch(N, g, dev, ndim=nd)
        q = synth.zero_boundary_torch(torch.randn(shape, generator=g, device=dev, dtype=torch.float64))
        rho_e, rho_g = torch.empty_like(q), torch.empty_like(q)
        P = Plan(Options(N, precision=prec, fixed_cycles=15, ir_inner_cycles=1, ir_adaptive=False, ndim=nd))
        P.set_log_coefficients(logD, logmua)
        s = torch.cuda.Stream()

        def call(out):
            st = lib.dmgs_forward(P._h, C.c_void_p(q.data_ptr()), C.c_void_p(out.data_ptr()), None,
                                  C.c_void_p(s.cuda_stream))
            if st != 0:
                raise RuntimeError("dmgs_forward: %s" % lib.dmgs_last_error().decode())

        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            call(rho_e)
            s.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=s):
                call(rho_g)
            graph.replay()
            s.synchronize()
            bitwise = bool(torch.equal(rho_e, rho_g))
            times = {"eager": [], "graph": []}
            for _ in range(args.sweep_reps):
                for kind in ("eager", "graph"):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record(s)
                    call(rho_e) if kind == "eager" else graph.replay()
                    b.record(s)
                    s.synchronize()
                    times[kind].append(a.elapsed_time(b))
        med = {k: sorted(v)[len(v) // 2] for k, v in times.items()}
        print(json.dumps({"graph_replay": "fixed 15 V-cycles, forward", "ndim": nd, "N": N, "precision": prec,
                          "reps": args.sweep_reps, "eager_ms_median": med["eager"], "graph_ms_median": med["graph"],
                          "replay_bitwise_equal": bitwise}), flush=True)
        del graph
        P.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--precision", default="fp32-in-fp64", choices=["fp32-in-fp64", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--inner", type=int, default=8, help="float32 V-cycles per refinement step (the most, when adaptive)")
    ap.add_argument("--no-adaptive", action="store_true", help="run --inner V-cycles in every refinement step")
    ap.add_argument("--smoother", default="rbgs", choices=["rbgs", "wjacobi"],
                    help="red-black Gauss-Seidel (the method's) or weighted Jacobi (the alternative)")
    ap.add_argument("--paper-sweep", action="store_true",
                    help="only the fixed-15-cycle Solve/JVP/VJP timing sweep over --sweep-sizes (one JSON line each)")
    ap.add_argument("--sweep-sizes", default=None,
                    help="comma-separated N (default 96..768 in 3D, 768..8192 in 2D)")
    ap.add_argument("--sweep-ndim", type=int, default=3, choices=[2, 3],
                    help="the sweep's grids: 3D (7-point) or 2D (5-point, the paper's comparison setting)")
    ap.add_argument("--sweep-reps", type=int, default=20)
    ap.add_argument("--sweep-cpu-baseline", action="store_true",
                    help="time the oracle beside the float64 sweep lines (3D N <= 256, 2D N <= 1024)")
    ap.add_argument("--sweep-unrolled-max", type=int, default=512,
                    help="largest N at which the sweep also times the unrolled adjoint (float64 3D)")
    ap.add_argument("--sequential", action="store_true",
                    help="run the forward solve and the VJP one after the other (default: concurrently)")
    ap.add_argument("--serving-requests", type=int, default=512, help="requests in the serving stream (0: skip)")
    ap.add_argument("--no-512", action="store_true", help="skip the 512^3 autograd forward + VJP record")
    ap.add_argument("--graph-replay", action="store_true",
                    help="only time the fixed-cycle forward launched eagerly against its captured HIP graph")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the library's plain streaming copy (256 MiB, 3 times): HBM counter calibration")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU path (requested --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2608_00760_amd import synth
    from paper_2608_00760_amd.solver import Options, Plan, stream_copy

    if args.paper_sweep:
        paper_sweep(args)
        return

    if args.graph_replay:
        graph_replay(args)
        return

    if args.copy_calibration:
        nbytes = 256 << 20
        src = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            ms = stream_copy(src, dst)
            print(json.dumps({"copy_bytes": nbytes, "ms": ms, "GBps_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}))
        return

    N = args.size
    log("generating inputs N=%d" % N)
    c = synth.grf_case(N, {128: 2000, 256: 3000, 512: 5000}.get(N, 3000))
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(c[k]).to(dev) for k in ("logD", "logmua", "q", "rhobar")}
    shape = t["q"].shape
    bufs = [torch.empty(shape, dtype=torch.float64, device=dev) for _ in range(4)]

    P = Plan(Options(N, precision=args.precision, rtol=1e-10, max_cycles=100, ir_inner_cycles=args.inner,
                     smoother=args.smoother,
                     ir_adaptive=not args.no_adaptive))
    log("plan: %d levels, %.2f GB" % (P.levels, P.bytes / 1e9))
    run_steps(P, t, bufs, args.warmup, args.sequential)
    torch.cuda.synchronize()
    # Timed region 1 (the value): steps with the forward and adjoint solves
    # concurrent (unless --sequential).
    t0 = time.perf_counter()
    info_f, info_a = run_steps(P, t, bufs, args.steps, args.sequential)
    torch.cuda.synchronize()
    elapsed_value = time.perf_counter() - t0
    # Timed region 2 (per-kernel figures): the same steps with the solves one
    # after the other, so that a kernel's event-timed duration is not
    # stretched by the other stream's kernels; one finest-level launch in 8
    # of each class is bracketed by events (every launch would cost about 6 %
    # of the step).
    run_steps(P, t, bufs, 1, True)
    torch.cuda.synchronize()
    P.timing(True, stride=8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(P, t, bufs, args.steps, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stats = P.timing_read()
    P.timing(False)
    ms_per_step = elapsed_value / args.steps * 1e3
    log("step %.3f ms, fwd cycles %d (%.2e), adj cycles %d (%.2e)" % (
        ms_per_step, info_f["cycles"], info_f["rel_residual"], info_a["cycles"], info_a["rel_residual"]))
    dom = max(stats, key=lambda k: stats[k]["ms"])
    d = stats[dom]
    avg_ms = d["ms"] / max(d["launches"], 1)
    bytes_per_launch = d["bytes"] / max(d["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    # Algorithmic bytes of a launch on the one-pass-per-sweep unit (5 words
    # per red-black sweep per vertex: read u, q, D, mua or w, write u); a
    # level-0 pass of the V(2,2) red-black cycle applies two sweeps.  The
    # fused pass itself needs fewer (u, q, D, w read once for both sweeps):
    # that figure is reported beside it.
    unit = None
    if dom == "smooth" and args.smoother == "rbgs":
        word_b = 4 if args.precision == "fp32-in-fp64" else 8
        unit = 2 * 5 * word_b * (N + 1) ** 3
    fused = {"bytes_per_launch": bytes_per_launch, "achieved": achieved, "frac": achieved / HBM_PEAK_GBPS,
             "what": "the bytes the fused two-sweep pass needs: u, q, D, w read and u written once for both sweeps "
                     "(4 words from a zero iterate), plus the defect it writes or the coarse correction it reads"}
    kernels = {k: {"launches": v["launches"], "avg_us": 1e3 * v["ms"] / max(v["launches"], 1),
                   "GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None,
                   "share": v["ms"] / (elapsed * 1e3)} for k, v in stats.items() if v["launches"]}

    fp64 = None
    if args.precision != "fp64" and not args.no_fp64_compare:
        P64 = Plan(Options(N, precision="fp64", rtol=1e-10, max_cycles=100, smoother=args.smoother))
        run_steps(P64, t, bufs, 1, args.sequential)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        k64 = max(2, args.steps // 3)
        f64, a64 = run_steps(P64, t, bufs, k64, args.sequential)
        torch.cuda.synchronize()
        fp64 = {"ms_per_step": (time.perf_counter() - s0) / k64 * 1e3, "cycles_fwd": f64["cycles"],
                "cycles_adj": a64["cycles"]}
        P64.close()
        log("fp64 solver: %.3f ms/step" % fp64["ms_per_step"])

    # likelihood gradient of one source (Sec. 2.5.4, Eq. (likelihood)): forward solve, the
    # fused epilogue, the pull-back and the gradients; data from the noise
    # model with a 3-vertex edge mask
    rho_l, _ = P.forward(t["q"])
    Le = rho_l * torch.exp(t["logmua"])
    w_l = P.noise_weights(Le, 3)
    gl = torch.Generator(device=dev)
    gl.manual_seed(3005)
    sig = torch.maximum(0.05 * Le, 0.01 * Le.max())
    d_l = Le + sig * torch.randn(Le.shape, generator=gl, device=dev, dtype=torch.float64)
    P.likelihood_grad(t["q"], d_l, w_l)
    torch.cuda.synchronize()
    nl = max(3, args.steps // 2)
    s0 = time.perf_counter()
    for _ in range(nl):
        (_, val_l, _), lf, la = P.likelihood_grad(t["q"], d_l, w_l)
    torch.cuda.synchronize()
    likelihood = {"ms_per_eval": (time.perf_counter() - s0) / nl * 1e3, "evals": nl, "chi2": val_l["chi2"],
                  "nvox": val_l["nvox"], "vcycles_fwd": lf["vcycles"], "vcycles_adj": la["vcycles"],
                  "what": "forward solve + epilogue (L_e = mua rho, H, chi2, dH/drho) + pull-back + gradients"}
    log("likelihood gradient: %.3f ms per evaluation, chi2 %.4f" % (likelihood["ms_per_eval"], val_l["chi2"]))
    del rho_l, Le, w_l, d_l, sig

    serving = None
    if args.serving_requests > 0:
        log("serving stream: %d requests" % args.serving_requests)
        serving = serving_leg(args.serving_requests)
        log("serving: p50 %.2f ms p99 %.2f ms, %.1f requests/s (saturation %.1f)" % (
            serving["p50_ms"], serving["p99_ms"], serving["requests_per_s"], serving["saturation_requests_per_s"]))
        g = serving["grouped_ticks"]
        log("serving, grouped ticks: p50 %.2f ms p99 %.2f ms, %.1f requests/s (saturation %.1f); at the thread "
            "server's rate p50 %.2f ms p99 %.2f ms; %d grouped launches for %d" % (
                g["p50_ms"], g["p99_ms"], g["requests_per_s"], g["saturation_requests_per_s"],
                g["at_thread_rate"]["p50_ms"], g["at_thread_rate"]["p99_ms"], g["grouped_launches"],
                g["recorded_launches"]))

    big = None
    if not args.no_512 and not args.sequential:
        log("512^3 forward + VJP through the autograd Function")
        big = config5_leg()
        log("512^3: %.1f ms per pair, peak %.1f GB, %d + %d V-cycles" % (
            big["ms_per_pair"], big["peak_device_GB"], big["vcycles_fwd"], big["vcycles_adj"]))

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on whole fwd+VJP pairs")
        cpu = cpu_baseline(c, args.smoother)
        log("oracle: %.4f pairs/s (%s)" % (cpu["value"], cpu["sample"]))

    # V-cycle time against the one-pass-per-operator byte model: 4 sweeps of 5
    # words, defect and restriction 4 + 1/8, prolongation and correction
    # 2 + 1/8 words per fine vertex, times the size of all levels over the
    # finest; the refinement residual, set-up and gradient passes are taken out
    nv = (N + 1) ** 3
    word = 4 if args.precision == "fp32-in-fp64" else 8
    levels = sum(((N >> k) + 1) ** 3 for k in range(P.levels)) / nv
    model_bytes = 26.25 * word * nv * levels
    vc = info_f["vcycles"] + info_a["vcycles"]
    # the refinement residual, set-up and gradient kernels of a step (timed
    # in the sequential region, where both solves run on the plan's stream)
    other_ms = sum(stats[k]["ms"] for k in ("residual", "update", "coef", "grad") if k in stats) / args.steps

    def vcycle_figure(step_ms, where):
        us = (step_ms - other_ms) / vc * 1e3
        return {"vcycles_per_step": vc, "measured_in": where, "us": us, "model_bytes": model_bytes,
                "model_GBps": model_bytes / (us * 1e-6) / 1e9,
                "frac": model_bytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBPS}
    # per V-cycle of the steps behind `value` (with concurrent solves, the
    # effective time per V-cycle of the two overlapping solves), and of the
    # sequential steps
    vcycle = vcycle_figure(ms_per_step, "first timed region (the value's steps)")
    vcycle_seq = vcycle_figure(elapsed / args.steps * 1e3, "sequential timed region")
    out = {
        "metric": "fwd+VJP solves/s at 256^3 (1e-10 rel. residual); GB/s vs HBM peak",
        "value": args.steps / elapsed_value,
        "unit": "fwd+VJP pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-in-f64" if args.precision == "fp32-in-fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": "diffusion-absorption multigrid solve + adjoint, %d^3 cells, GRF log-normal D (contrast "
                               "<=1e4) and mua, 16-blob source, V(2,2) %s, rtol 1e-10, set-up+forward+VJP per step"
                               % (N, "RB-GS" if args.smoother == "rbgs" else "weighted Jacobi (6/7)"),
                   "N": N, "precision": args.precision, "rtol": 1e-10, "smoother": args.smoother,
                   "ir_inner_cycles": args.inner,
                   "ir_adaptive": not args.no_adaptive,
                   "fwd_vjp_solves": "sequential" if args.sequential else "concurrent (two streams)",
                   "steps_fwd": info_f["cycles"], "steps_adj": info_a["cycles"],
                   "vcycles_fwd": info_f["vcycles"], "vcycles_adj": info_a["vcycles"],
                   "rel_residual_fwd": info_f["rel_residual"], "rel_residual_adj": info_a["rel_residual"]},
        "sequential_solves": {"value": args.steps / elapsed, "ms_per_step": elapsed / args.steps * 1e3},
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": (unit if unit else bytes_per_launch) / (avg_ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": (unit if unit else bytes_per_launch) / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                     "traffic": measured_traffic(dom) if N == 256 and args.precision == "fp32-in-fp64" else None,
                     "measured_in": "sequential timed region", "avg_launch_us": avg_ms * 1e3,
                     "algorithmic_bytes_per_launch": unit if unit else bytes_per_launch,
                     "bytes_unit": ("5 words per red-black sweep per vertex, two sweeps per level-0 launch" if unit
                                    else "the pass's own bytes"),
                     "fused_pass": fused},
        "kernels": kernels,
        "vcycle": vcycle,
        "vcycle_sequential": vcycle_seq,
        "fp64_solver": fp64,
        "latency_p50_p99": serving,
        "likelihood_grad": likelihood,
        "autograd_512": big,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
