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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the timed region, copy a buffer of this size once (a plain "
                         "copy kernel of known traffic for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(instances shard trivially across GPUs; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_12201_amd import colloc, workloads

    K = 3
    inst = workloads.random_network(0)
    x0 = workloads.initial_point(inst, K)
    P = colloc.Problem(inst, K)
    opts = colloc.default_opts()
    ws, state = P.workspace(), P.state()
    x0d = torch.tensor(x0, dtype=torch.float64, device="cuda")
    P.ipm_init(x0d, state, ws, opts)
    for _ in range(args.warmup):
        P.ipm_step(state, ws, opts)
    torch.cuda.synchronize()
    if args.calib_copy_mib:
        n = args.calib_copy_mib * 2 ** 20 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    P.ipm_init(x0d, state, ws, opts)          # timed region starts from the same point
    torch.cuda.synchronize()
    it0 = int(P.info(state)[0]["iter"])
    P.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P.ipm_step(state, ws, opts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ph_ms, ph_n = P.timing_read()
    P.timing(False)
    info = P.info(state)[0]
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
                   "newton_steps": newton, "ipm_step_calls": args.steps,
                   "final_status": int(info["status"]), "iter_end": int(info["iter"]),
                   "phase_ms_per_call": {k: ph_ms[k] / max(1, ph_n[k]) for k in ph_ms}},
        "roofline": {"bound": "alu", "kernel": "k_level0 (fused assembly + element condensation)",
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "avg_launch_ms": l0_ms,
                     "algorithmic_flops_per_launch": flops,
                     "algorithmic_bytes_per_launch": level0_bytes(P.ns, P.np_, K) * E},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(inst, K, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
