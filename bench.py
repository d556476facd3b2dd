"""Benchmark: interior-point Newton steps per second on one MI355X.

Default workload: the stiff random mass-action network with 100 species, 250 reactions (200 rate
constants estimated, 50 known), 20 observed species at 200 times, N = 10,000 Radau finite
elements with K = 3 (4,000,200 variables), one instance, FP64.  A step is one full ipm_step
(evaluation and derivatives, assembly, factorization with inertia retries, solve, line search,
update) replayed from a captured HIP graph with every input resident in HBM; value = Newton
iterations completed per second over the timed region (an inertia-correction retry is a step
that completes no iteration).  The same steps then run with FP32 block factors + FP64 refinement
(the mixed-precision form) and eagerly with the library's per-phase HIP events, which give the
per-kernel times for the roofline line and the per-step latency percentiles.  The CPU oracle's
Newton step is timed on a bounded sample for context.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 (vector and matrix), 256 CU x 2.4 GHz x 128 flop/clk
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    "net100_n10000": "stiff random mass-action network, 100 species, 250 reactions (200 estimated), "
                     "200 params, 20 observables at 200 times, N=10000 Radau elements K=3 "
                     "(4,000,200 variables), one instance",
    "net20_n1000": "random mass-action network, 20 species, 40 reactions, 40 params, N=1000 Radau "
                   "elements K=3 (80,040 variables), one instance",
}


def make_instance(name, N=None):
    from paper_2607_12201_amd import workloads
    if name == "net100_n10000":
        if N is None:
            return workloads.stiff_network(0)
        # the same network (seed, reactions, rates, initial state) on a shorter mesh
        return workloads.random_network(0, n_s=100, n_r=250, N=N, n_obs=20, n_times=N, klo=1e-3, khi=1e4,
                                        n_fixed=50, stiff=True)
    return workloads.random_network(0, N=N or 1000, n_times=50 if (N or 1000) % 50 == 0 else (N or 1000))


def element_flops(ns, np_, K, tiled):
    """Algorithmic flops (2 per multiply-add) of one element's factorization, split by kernel.
    panel: left-looking partial Cholesky of the mI = K ns interior columns of the R-row element
    matrix (R = mI + 2 ns + np), sum over columns c of (R - c) c multiply-adds; schur: the
    trailing Schur complement of the remaining R - mI rows and columns with the mI eliminated
    columns, without its np x np parameter block (formed separately for the border)."""
    mI = K * ns
    R = mI + 2 * ns + np_
    panel = 2.0 * sum((R - c) * c for c in range(mI))
    t = R - mI
    schur = 2.0 * mI * (t * (t + 1) / 2 - (np_ * (np_ + 1) / 2 if tiled else 0))
    return panel, schur


def assembly_bytes(ns, np_, K):
    """Algorithmic bytes of one element's assembly: the lower triangle of its R x R matrix written
    once in FP64 (the theta block to its FP64 side array)."""
    R = (K + 2) * ns + np_
    return 8.0 * R * (R + 1) / 2


def kernel_source_fingerprint():
    """sha256 of csrc/k_big.hip, the source of the tiled path's kernels."""
    with open(os.path.join(ROOT, "paper_2607_12201_amd", "csrc", "k_big.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter summary
    (profiles/<kernel>_<workload>_traffic.md: a 'traffic_bytes_per_launch:' line, FETCH_SIZE and
    WRITE_SIZE each scaled by the same counter's reading for a copy of known size).  None without
    one, or when its 'source_sha256:' line no longer matches the kernels' source file (the
    counters were taken on other code)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    val, sha = None, None
    try:
        with open(path) as f:
            for line in f:
                if line.startswith("traffic_bytes_per_launch:"):
                    val = float(line.split(":", 1)[1])
                elif line.startswith("source_sha256:"):
                    sha = line.split(":", 1)[1].strip()
    except OSError:
        return None
    if sha is None or sha != kernel_source_fingerprint():
        return None
    return val


def cpu_baseline(name, K, seconds=20.0):
    """The oracle's Newton iteration (natural-order block Cholesky path) timed on the host on a
    bounded sample: the same network on a mesh short enough for ~seconds of CPU work, the rate
    scaled to the full mesh by the element ratio (the oracle's cost per iteration is linear in
    the number of elements)."""
    from oracle import ipm, problem
    from paper_2607_12201_amd import workloads

    N_full = 10000 if name == "net100_n10000" else 1000
    N_s = 10 if name == "net100_n10000" else 1000
    inst = make_instance(name, N_s)
    m = problem.Model(inst, K)
    opt = ipm.Options()
    st = ipm.init_state(m, workloads.initial_point(inst, K), opt)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds and st.status == ipm.RUNNING:
        ipm.iterate(m, st, opt, solver="block")
        n += 1
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    return dict(value=n / dt * N_s / N_full, unit="Newton steps/s", cores=int(cores), kind="oracle",
                sample=f"first {n} oracle IPM iterations (natural-order block Cholesky) on the same "
                       f"network with N={N_s} elements in {dt:.1f} s, rate scaled by {N_s}/{N_full}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32-factor + FP64-refinement leg")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--workload", default="net100_n10000",
                    choices=["net100_n10000", "net20_n1000", "multistart", "serving"],
                    help="net100_n10000: one 100-species N=10000 instance (the headline line); "
                         "net20_n1000: one 20-species N=1000 instance; multistart: 256 uneven A<->B "
                         "instances batched; serving: Poisson arrivals through the continuous-batching "
                         "loop against the sequential per-instance FP64 path")
    ap.add_argument("--requests", type=int, default=60)
    ap.add_argument("--load", type=float, default=0.8,
                    help="arrival rate as a fraction of the per-instance path's saturation rate")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the timed region, copy a buffer of this size once (a plain "
                         "copy kernel of known traffic for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(instances are independent and shard across GPUs one process per GPU)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "multistart":
        return bench_multistart(args)
    if args.workload == "serving":
        return bench_serving(args)
    return bench_single(args)


def _timed_leg(P, x0, opts, precision, steps, warmup, side, calib_mib=0):
    """Graph-replayed timed region, then the same steps eagerly with per-phase events and a
    per-step wall clock.  Returns the measurements."""
    import torch
    with torch.cuda.stream(side):
        ws, state = P.workspace(precision), P.state()
        graph = P.graph_create(state, ws, opts, steps=1)
        P.ipm_init(x0, state, ws, opts)
        for _ in range(warmup):
            P.graph_launch(graph)
        side.synchronize()
        if calib_mib:
            n = calib_mib * 2 ** 20 // 8
            src = torch.ones(n, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            dst.copy_(src)
            side.synchronize()
            del src, dst
        P.ipm_init(x0, state, ws, opts)          # timed region starts from the same point
        side.synchronize()
        it0 = int(P.info(state)[0]["iter"])
        t0 = time.perf_counter()
        for _ in range(steps):
            P.graph_launch(graph)
        side.synchronize()
        dt = time.perf_counter() - t0
        info = P.info(state)[0]
        P.graph_destroy(graph)
        # eager pass: the library's per-phase HIP events are recorded on this stream around
        # each phase (a graph replay records none); the host clock per synchronized step gives
        # the latency distribution
        P.ipm_init(x0, state, ws, opts)
        side.synchronize()
        P.timing(True)
        lat = []
        for _ in range(steps):
            t1 = time.perf_counter()
            P.ipm_step(state, ws, opts)
            side.synchronize()
            lat.append(time.perf_counter() - t1)
        ph_ms, ph_n = P.timing_read()
        P.timing(False)
        info2 = P.info(state)[0]
        del ws, state
    return dict(dt=dt, newton=int(info["iter"]) - it0, info=info, ph_ms=ph_ms, ph_n=ph_n,
                lat_ms=1e3 * np.array(lat), ir_fallbacks=int(info2["ir_fallbacks"]),
                iter_eager=int(info2["iter"]))


def bench_single(args):
    import torch
    from paper_2607_12201_amd import colloc, workloads

    K = 3
    name = args.workload
    inst = make_instance(name)
    x0 = workloads.initial_point(inst, K)
    P = colloc.Problem(inst, K)
    # element blocks above 160 rows take the tiled matrix-core path (one fixed tiling)
    tiled = (K + 2) * P.ns + P.np_ > 160 or os.environ.get("COLLOC_FACTOR_PATH") == "tiled"
    tiles = None
    if not tiled:
        from paper_2607_12201_amd import autotune
        tiles = autotune.tune(P)           # thread grids per kernel (device-timed, cached per shape)
    side = torch.cuda.Stream()
    x0d = torch.tensor(x0, dtype=torch.float64, device="cuda")
    r64 = _timed_leg(P, x0d, colloc.default_opts(), colloc.FP64, args.steps, args.warmup, side,
                     args.calib_copy_mib)
    rmx = None
    if not args.no_mixed:
        torch.cuda.empty_cache()
        rmx = _timed_leg(P, x0d, colloc.default_opts(precision=colloc.FP32_IR), colloc.FP32_IR, args.steps,
                         args.warmup, side)
    value = r64["newton"] / r64["dt"]
    E = P.n_elem
    ph = {k: r64["ph_ms"][k] / max(1, r64["ph_n"][k]) for k in r64["ph_ms"]}
    kernels = {}
    if tiled:
        f_panel, f_schur = element_flops(P.ns, P.np_, K, True)
        # per-step launches of the element level: assembly (one launch), the interior-column
        # factorization (a diagonal and a strip launch per 32-column panel), the trailing update
        # (one launch); the dominant single launch carries the roofline line
        cand = {"assembly": ("k_big_asm", "element matrix assembly, one launch per step", "hbm",
                             assembly_bytes(P.ns, P.np_, K) * E),
                "schur": ("k_pchol_trail", "element Schur complement (trailing update), one launch per step",
                          "mfma", f_schur * E),
                "level0": ("k_pchol_diag + k_pchol_strip", "element interior-column factorization, "
                           "two launches per 32-column panel", "mfma", f_panel * E)}
        for key, (kn, desc, bound_k, work_k) in cand.items():
            ms_k = ph.get(key, 0.0)
            if ms_k <= 0:
                continue
            if bound_k == "hbm":
                a_k, p_k, u_k = work_k / (ms_k * 1e-3) / 1e9, PEAK_HBM_GBS, "GB/s"
            else:
                a_k, p_k, u_k = work_k / (ms_k * 1e-3) / 1e12, PEAK_FP64_TFLOPS, "TFLOP/s"
            kernels[kn] = {"what": desc, "bound": bound_k, "ms": ms_k, "achieved": a_k, "unit": u_k,
                           "frac": a_k / p_k}
        key = "assembly" if ph.get("assembly", 0.0) >= ph.get("schur", 0.0) else "schur"
        kname, kdesc, bound, work = cand[key]
    else:
        f_panel, f_schur = element_flops(P.ns, P.np_, K, False)
        key, kname, kdesc, bound, work = ("level0", "k_level0r", "fused assembly + element condensation",
                                          "mfma", (f_panel + f_schur) * E)
    ms = ph[key]
    if bound == "hbm":
        achieved, peak, unit = work / (ms * 1e-3) / 1e9, PEAK_HBM_GBS, "GB/s"
    else:
        achieved, peak, unit = work / (ms * 1e-3) / 1e12, PEAK_FP64_TFLOPS, "TFLOP/s"
    traffic = measured_traffic(kname, name)
    cfg = {"workload": WORKLOADS[name], "factor_path": "tiled" if tiled else "register",
           "newton_steps": r64["newton"], "ipm_step_calls": args.steps, "graph_replay": True,
           "final_status": int(r64["info"]["status"]), "iter_end": int(r64["info"]["iter"]),
           "phase_ms_per_call": ph,
           "step_latency_ms": {"p50": float(np.percentile(r64["lat_ms"], 50)),
                               "p99": float(np.percentile(r64["lat_ms"], 99))}}
    if tiles:
        cfg["tiles"] = {k: tiles[k] for k in colloc.Problem.TILE_KERNELS}
    if rmx is not None:
        cfg["fp32_ir"] = {"newton_steps_per_s": rmx["newton"] / rmx["dt"], "newton_steps": rmx["newton"],
                          "ms_per_step": 1e3 * rmx["dt"] / args.steps,
                          "ir_fallbacks": rmx["ir_fallbacks"], "iter_eager": rmx["iter_eager"],
                          "phase_ms_per_call": {k: rmx["ph_ms"][k] / max(1, rmx["ph_n"][k]) for k in rmx["ph_ms"]},
                          "step_latency_ms": {"p50": float(np.percentile(rmx["lat_ms"], 50)),
                                              "p99": float(np.percentile(rmx["lat_ms"], 99))}}
    line = {
        "metric": "IPM Newton steps/s (AD+KKT factor+solve) FP64 vs mixed-batched; p50/p99 latency",
        "value": value,
        "unit": "Newton steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r64["dt"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": {"bound": bound, "kernel": f"{kname} ({kdesc})", "achieved": achieved, "peak": peak,
                     "unit": unit, "frac": achieved / peak, "traffic": traffic, "avg_launch_ms": ms,
                     ("algorithmic_flops_per_launch" if bound != "hbm" else "algorithmic_bytes_per_launch"): work,
                     "other_kernels": kernels},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(name, K, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def _run_steps(P, state, ws, opts, steps, graph=None):
    for _ in range(steps):
        if graph is not None:
            P.graph_launch(graph)
        else:
            P.ipm_step(state, ws, opts)


def bench_multistart(args):
    """Batched multi-start: 256 A<->B instances, N uniform in [200, 2000] (multiples of 10),
    K = 3, random starting parameters; one replayed HIP graph per interior-point step, FP32
    block factors with FP64 refinement, thread grids from the autotuner.  value = Newton
    iterations completed per second summed over the instances.  Beside it: the plain FP64
    per-instance path (one handle per instance, eager steps) timed on a sample of instances."""
    import torch
    from paper_2607_12201_amd import autotune, colloc, workloads

    K = 3
    insts = workloads.multistart_batch(256, 200, 2000)
    P = colloc.Problem(insts, K)
    opts = colloc.default_opts(precision=colloc.FP32_IR)
    tiles = autotune.tune(P, precision=colloc.FP32_IR)
    x0 = torch.tensor(np.concatenate([workloads.initial_point(i, K) for i in insts]),
                      dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        ws, state = P.workspace(colloc.FP32_IR), P.state()
        P.ipm_init(x0, state, ws, opts)
        g = P.graph_create(state, ws, opts, steps=1)
        _run_steps(P, state, ws, opts, args.warmup, g)
        P.ipm_init(x0, state, ws, opts)
        side.synchronize()
        it0 = P.info(state)["iter"].astype(np.int64).sum()
        t0 = time.perf_counter()
        _run_steps(P, state, ws, opts, args.steps, g)
        side.synchronize()
        dt = time.perf_counter() - t0
        info = P.info(state)
        P.graph_destroy(g)
    newton = int(info["iter"].astype(np.int64).sum() - it0)
    # the same batch with FP64 factors (batching alone, no mixed precision)
    o64b = colloc.default_opts()
    autotune.tune(P, precision=colloc.FP64)
    with torch.cuda.stream(side):
        ws64, st64 = P.workspace(colloc.FP64), P.state()
        P.ipm_init(x0, st64, ws64, o64b)
        g64 = P.graph_create(st64, ws64, o64b, steps=1)
        _run_steps(P, st64, ws64, o64b, args.warmup, g64)
        P.ipm_init(x0, st64, ws64, o64b)
        side.synchronize()
        i64 = P.info(st64)["iter"].astype(np.int64).sum()
        t0 = time.perf_counter()
        _run_steps(P, st64, ws64, o64b, args.steps, g64)
        side.synchronize()
        dt64 = time.perf_counter() - t0
        newton64 = int(P.info(st64)["iter"].astype(np.int64).sum() - i64)
        P.graph_destroy(g64)
    # plain FP64 per-instance path on a sample of the same instances
    sample = insts[:: max(1, len(insts) // 8)][:8]
    o64 = colloc.default_opts()
    tot_it, tot_t = 0, 0.0
    for inst in sample:
        P1 = colloc.Problem(inst, K)
        ws1, st1 = P1.workspace(), P1.state()
        P1.ipm_init(torch.tensor(workloads.initial_point(inst, K), dtype=torch.float64, device="cuda"),
                    st1, ws1, o64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _run_steps(P1, st1, ws1, o64, args.steps)
        torch.cuda.synchronize()
        tot_t += time.perf_counter() - t1
        tot_it += int(P1.info(st1)[0]["iter"])
    line = {
        "metric": "IPM Newton steps/s (AD+KKT factor+solve), batched mixed precision",
        "value": newton / dt,
        "unit": "Newton steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 factors + f64 refinement",
        "data": "synthetic",
        "config": {"workload": "256 A<->B multi-start instances, N uniform in [200, 2000], K=3, "
                               "FP32 block factors + FP64 refinement, graph-replayed steps",
                   "total_elements": int(P.n_elem), "newton_steps": newton,
                   "solved": int(np.sum(info["status"] == colloc.SOLVED)),
                   "ir_fallbacks": int(info["ir_fallbacks"].sum()), "tiles": {
                       k: tiles[k] for k in colloc.Problem.TILE_KERNELS},
                   "batched_fp64_newton_steps_per_s": newton64 / dt64,
                   "per_instance_fp64_newton_steps_per_s": tot_it / tot_t,
                   "per_instance_sample": len(sample)},
    }
    print(json.dumps(line), flush=True)


def bench_serving(args):
    """Serving: requests with n_s uniform in 5..20 species (n_r = n_p = 2 n_s), N log-uniform in
    [100, 2000] (multiples of 50), arriving as a Poisson process at `load` times the saturation
    rate of the plain FP64 per-instance path (one request at a time, first come first served).
    The batched path admits requests under an HBM budget and batches them per shape class, with
    FP64 factors (the line's value) and with FP32 factors + FP64 refinement (a second leg).
    Latency = arrival to result.  Both paths run every request
    of the same trace; the per-instance latencies follow from its measured service times."""
    import torch
    from paper_2607_12201_amd import colloc, serving, workloads

    _, insts = workloads.serving_trace(args.requests, 1.0, seed=11, ns_lo=5, ns_hi=20, N_lo=100,
                                       N_hi=2000)
    o64 = colloc.default_opts()
    service, ok64, ref = [], 0, []
    serving.solve_alone(insts[0], o64)       # warm-up (code load)
    for inst in insts:
        st, it, x, obj, dt = serving.solve_alone(inst, o64)
        service.append(dt)
        ref.append((st, x))
        ok64 += st in (colloc.SOLVED, colloc.ACCEPTABLE)
    service = np.array(service)
    rate = args.load / service.mean()
    rng = np.random.default_rng(12)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, len(insts)))
    lat64 = serving.fifo_latencies(arrivals, service)
    makespan64 = float(np.max(arrivals + lat64) - arrivals[0])
    budget = 8 * 2 ** 30

    def good(r):
        """A solve counts when it succeeded and its parameters equal the per-instance FP64
        result within 1e-6 (relative, floor 1)."""
        st, x = ref[r.rid]
        if r.status not in (colloc.SOLVED, colloc.ACCEPTABLE) or st not in (colloc.SOLVED, colloc.ACCEPTABLE):
            return False
        npar = int(r.inst["n_p"])
        th, th0 = r.x[-npar:], x[-npar:]
        return bool(np.max(np.abs(th - th0) / np.maximum(1.0, np.abs(th0))) < 1e-6)

    def leg(opts):
        reqs = [serving.Request(q, float(a), inst) for q, (a, inst) in enumerate(zip(arrivals, insts))]
        res = serving.serve(reqs, opts, budget, steps_per_round=4)
        lat = res.latencies()
        span = max(r.t_done for r in reqs) - float(arrivals[0])
        ngood = sum(good(r) for r in reqs)
        return res, {"solves_per_s": ngood / span, "good_solves": int(ngood), "finished": len(reqs),
                     "status": res.status_counts(), "p50_s": float(np.percentile(lat, 50)),
                     "p99_s": float(np.percentile(lat, 99)), "peak_bytes": int(res.peak_bytes),
                     "peak_allocator_bytes": int(res.peak_allocator_bytes)}

    torch.cuda.synchronize()
    res64, b64 = leg(o64)                    # same trace, FP64 factors (the batching effect alone)
    res, bmx = leg(colloc.default_opts(precision=colloc.FP32_IR))
    st64 = {}
    for st, _ in ref:
        st64[colloc.STATUS_NAMES[st]] = st64.get(colloc.STATUS_NAMES[st], 0) + 1
    line = {
        "metric": "solves/s and p50/p99 latency, continuous batching vs per-instance FP64",
        "value": b64["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": int(res64.steps),
        "warmup": 1,
        "ms_per_step": 1e3 * res64.wall / max(1, res64.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{len(insts)} Poisson requests, n_s 5-20, N 100-2000, K=3, "
                               f"load {args.load} of the per-instance FP64 saturation rate; a solve "
                               f"counts when SOLVED/ACCEPTABLE with parameters equal to the "
                               f"per-instance FP64 result within 1e-6",
                   "hbm_budget_bytes": budget, "batched_fp32_ir": bmx, "batched_fp64": b64,
                   "per_instance_fp64": {"solves_per_s": ok64 / makespan64, "good_solves": int(ok64),
                                         "status": st64,
                                         "p50_s": float(np.percentile(lat64, 50)),
                                         "p99_s": float(np.percentile(lat64, 99)),
                                         "mean_service_s": float(service.mean())}},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
