"""Benchmark: interior-point Newton steps per second on one MI355X.

Workload: random mass-action network, 20 species, 40 reactions, 40 log-rate parameters,
N = 1000 Radau finite elements with K = 3 (80,040 variables), FP64, one instance.  A step is
one full ipm_step (evaluation + derivatives, assembly, factorization with inertia retries,
solve, line search, update) with all inputs resident in HBM.  value = Newton steps completed
per second over the timed region.  The level-0 factorization kernel (fused assembly and
static condensation of every element) is timed with HIP events on the library's stream for
the roofline line; the CPU oracle's Newton step is timed on a bounded sample for context.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 (vector and matrix), 256 CU x 2.4 GHz x 128 flop/clk
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the element kernel at this workload, per thread grid, from FETCH_SIZE and
# WRITE_SIZE counter passes scaled by a 256 MiB calibration copy (profiles/level0_*_traffic.md).
# An entry holds only for the kernel source it was taken on (fingerprint of the shared headers
# and the translation unit that instantiates that grid).
L0_COMMON = ["level0_impl.h", "regchol.h", "elem.h", "common.h", "kernels.h"]
L0_TRAFFIC = {20: {"tu": "k_level0_u.hip", "sha": "0cefb2fdc47464c9", "bytes": 113392642.0}}


def level0_traffic(tile):
    import hashlib
    ent = L0_TRAFFIC.get(tile)
    if ent is None:
        return None
    h = hashlib.sha256()
    for n in L0_COMMON + [ent["tu"]]:
        with open(os.path.join(ROOT, "paper_2607_12201_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return ent["bytes"] if h.hexdigest()[:16] == ent["sha"] else None


def level0_flops(ns, np_, K):
    """Algorithmic flops of one element's dense condensed block factorization:
    b^3/3 + b^2 p + b p^2 with b = (K+1) n_s (Cholesky of the element block, border solve,
    border Schur update)."""
    b = (K + 1) * ns
    return b ** 3 / 3.0 + b * b * np_ + b * np_ * np_


def level0_bytes(ns, np_, K):
    """Algorithmic bytes of one element's factor in FP64: S_e = b(b+1)/2 + n_s^2 + b p doubles
    written once."""
    b = (K + 1) * ns
    return 8.0 * (b * (b + 1) / 2 + ns * ns + b * np_)


def cpu_baseline(inst, K, seconds=20.0):
    """The oracle's Newton iteration (natural-order block Cholesky path) on the same workload,
    timed on the host for a bounded number of iterations."""
    from oracle import ipm, problem
    from paper_2607_12201_amd import workloads

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
    return dict(value=n / dt, unit="Newton steps/s", cores=int(cores), kind="oracle",
                sample=f"first {n} oracle IPM iterations (natural-order block Cholesky) on the "
                       f"same 20-species N=1000 instance, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--workload", default="net20_n1000", choices=["net20_n1000", "multistart", "serving"],
                    help="net20_n1000: one 20-species instance, FP64 (the headline line); "
                         "multistart: 256 uneven A<->B instances batched, FP32 factors + FP64 "
                         "refinement, graph-replayed steps, autotuned thread grids; serving: "
                         "Poisson arrivals of uneven requests through the continuous-batching "
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

    import torch
    from paper_2607_12201_amd import colloc, workloads

    K = 3
    inst = workloads.random_network(0)
    x0 = workloads.initial_point(inst, K)
    P = colloc.Problem(inst, K)
    opts = colloc.default_opts()
    from paper_2607_12201_amd import autotune
    tiles = autotune.tune(P)           # thread grids per kernel (device-timed, cached per shape)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        ws, state = P.workspace(), P.state()
        x0d = torch.tensor(x0, dtype=torch.float64, device="cuda")
        # one interior-point step captured as a HIP graph, replayed once per step
        graph = P.graph_create(state, ws, opts, steps=1)
        P.ipm_init(x0d, state, ws, opts)
        for _ in range(args.warmup):
            P.graph_launch(graph)
        side.synchronize()
        if args.calib_copy_mib:
            n = args.calib_copy_mib * 2 ** 20 // 8
            src = torch.ones(n, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            dst.copy_(src)
            side.synchronize()
            del src, dst
        P.ipm_init(x0d, state, ws, opts)          # timed region starts from the same point
        side.synchronize()
        it0 = int(P.info(state)[0]["iter"])
        t0 = time.perf_counter()
        for _ in range(args.steps):
            P.graph_launch(graph)
        side.synchronize()
        dt = time.perf_counter() - t0
        info = P.info(state)[0]
        # the same steps again, eager, with the library's per-phase HIP events (the events are
        # recorded on this stream around each phase; a graph replay records none)
        P.ipm_init(x0d, state, ws, opts)
        P.timing(True)
        for _ in range(args.steps):
            P.ipm_step(state, ws, opts)
        side.synchronize()
        ph_ms, ph_n = P.timing_read()
        P.timing(False)
        P.graph_destroy(graph)
    newton = int(info["iter"]) - it0
    value = newton / dt
    ms_per_step = 1e3 * dt / args.steps
    E = P.n_elem
    l0_ms = ph_ms["level0"] / max(1, ph_n["level0"])
    flops = level0_flops(P.ns, P.np_, K) * E
    achieved = flops / (l0_ms * 1e-3) / 1e12
    line = {
        "metric": "IPM Newton steps/s (AD+KKT factor+solve)",
        "value": value,
        "unit": "Newton steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "random mass-action network, 20 species, 40 reactions, 40 params, "
                               "N=1000 Radau elements K=3, FP64 plain IPM, one instance",
                   "newton_steps": newton, "ipm_step_calls": args.steps, "graph_replay": True,
                   "final_status": int(info["status"]), "iter_end": int(info["iter"]),
                   "tiles": {k: tiles[k] for k in colloc.Problem.TILE_KERNELS},
                   "phase_ms_per_call": {k: ph_ms[k] / max(1, ph_n[k]) for k in ph_ms}},
        "roofline": {"bound": "alu", "kernel": "k_level0 (fused assembly + element condensation)",
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": level0_traffic(tiles["level0"]),
                     "avg_launch_ms": l0_ms,
                     "algorithmic_flops_per_launch": flops,
                     "algorithmic_bytes_per_launch": level0_bytes(P.ns, P.np_, K) * E},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(inst, K, args.cpu_seconds)
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
    The batched path admits requests under an HBM budget and batches them per shape class with
    FP32 factors + FP64 refinement.  Latency = arrival to result.  Both paths run every request
    of the same trace; the per-instance latencies follow from its measured service times."""
    import torch
    from paper_2607_12201_amd import colloc, serving, workloads

    _, insts = workloads.serving_trace(args.requests, 1.0, seed=11, ns_lo=5, ns_hi=20, N_lo=100,
                                       N_hi=2000)
    o64 = colloc.default_opts()
    service, ok64 = [], 0
    serving.solve_alone(insts[0], o64)       # warm-up (code load)
    for inst in insts:
        st, it, x, obj, dt = serving.solve_alone(inst, o64)
        service.append(dt)
        ok64 += st in (colloc.SOLVED, colloc.ACCEPTABLE)
    service = np.array(service)
    rate = args.load / service.mean()
    rng = np.random.default_rng(12)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, len(insts)))
    lat64 = serving.fifo_latencies(arrivals, service)
    makespan64 = float(np.max(arrivals + lat64) - arrivals[0])
    reqs = [serving.Request(q, float(a), inst) for q, (a, inst) in enumerate(zip(arrivals, insts))]
    budget = 8 * 2 ** 30
    torch.cuda.synchronize()
    # same trace through the batching loop with FP64 factors (the batching effect alone)
    reqs64 = [serving.Request(q, float(a), inst) for q, (a, inst) in enumerate(zip(arrivals, insts))]
    res64 = serving.serve(reqs64, o64, budget, steps_per_round=4)
    lat_b64 = res64.latencies()
    opts = colloc.default_opts(precision=colloc.FP32_IR)
    res = serving.serve(reqs, opts, budget, steps_per_round=4)
    summ = res.summary()
    lat = res.latencies()
    line = {
        "metric": "solves/s and p50/p99 latency, continuous batching vs per-instance FP64",
        "value": summ["requests"] / (max(r.t_done for r in reqs) - float(arrivals[0])),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": int(res.steps),
        "warmup": 1,
        "ms_per_step": 1e3 * res.wall / max(1, res.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 factors + f64 refinement",
        "data": "synthetic",
        "config": {"workload": f"{len(insts)} Poisson requests, n_s 5-20, N 100-2000, K=3, "
                               f"load {args.load} of the per-instance FP64 saturation rate",
                   "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                   "solved": summ["solved"], "peak_bytes": summ["peak_bytes"],
                   "hbm_budget_bytes": budget,
                   "batched_fp64": {"solves_per_s": len(insts) / (max(r.t_done for r in reqs64) -
                                                                  float(arrivals[0])),
                                    "p50_s": float(np.percentile(lat_b64, 50)),
                                    "p99_s": float(np.percentile(lat_b64, 99))},
                   "per_instance_fp64": {"solves_per_s": len(insts) / makespan64,
                                         "p50_s": float(np.percentile(lat64, 50)),
                                         "p99_s": float(np.percentile(lat64, 99)),
                                         "mean_service_s": float(service.mean()), "solved": int(ok64)}},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
