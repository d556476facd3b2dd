"""Thread-grid autotuner for the register-resident elimination kernels.

The element (level-0), separator-chain and border kernels each run on a TS x TS thread grid
that holds the kernel's matrix in registers (TS in 8, 16, 20, 24, as instantiated for the shape).
The grid changes which thread computes an entry, not the arithmetic, so every choice gives the
same result; only the time differs.  `tune` times each usable grid per kernel on the device, in
the interior-point step the kernels serve (HIP events recorded by the library around each phase
of ipm_step, per launch), on the handle's own instances; it keeps the fastest and caches the
choice in a JSON file keyed by device architecture, shape class (n_s, n_r, n_p, K) and factor
precision.  The choice
depends only on the shape class, never on the batch mix.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import colloc, workloads

DEFAULT_CACHE = os.environ.get(
    "COLLOC_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "colloc_tiles_v2.json"))
PHASE_OF = {"level0": "level0", "chain": "cr", "border": "border"}


def shape_key(P, precision, arch):
    return f"{arch}:ns{P.ns}:nr{P.nr}:np{P.np_}:K{P.K}:prec{int(precision)}"


def _arch(torch):
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _ipm_setup(P, precision, torch):
    """An interior-point state on the handle's own instances, with options that keep every
    instance iterating (no convergence stop) so each timed step runs the factorization."""
    insts = P.instances if isinstance(P.instances, (list, tuple)) else [P.instances]
    x0 = torch.tensor(np.concatenate([workloads.initial_point(i, P.K) for i in insts]),
                      dtype=torch.float64, device=P.device)
    opts = colloc.default_opts(precision=precision, tol=1e-300, acceptable_iter=1 << 30)
    ws, st = P.workspace(precision), P.state()
    return x0, opts, ws, st


def tune(P, precision=colloc.FP64, reps=4, cache_path=DEFAULT_CACHE, force=False, verbose=False):
    """Choose and apply the fastest thread grid per kernel for the handle P.  Returns
    {"level0": ts, "chain": ts, "border": ts, "ms": {...}} (ts = 0: built-in rule)."""
    import torch

    key = shape_key(P, precision, _arch(torch))
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        for k in colloc.Problem.TILE_KERNELS:
            P.tile_set(k, cache[key][k])
        return cache[key]
    x0, opts, ws, st = _ipm_setup(P, precision, torch)

    def measure(which, ts):
        P.tile_set(which, ts)
        P.ipm_init(x0, st, ws, opts)
        for _ in range(2):               # first iterations, code load
            P.ipm_step(st, ws, opts)
        torch.cuda.synchronize()
        P.timing(True)
        for _ in range(reps):
            P.ipm_step(st, ws, opts)
        torch.cuda.synchronize()
        ms, n = P.timing_read()
        P.timing(False)
        ph = PHASE_OF[which]
        return ms[ph] / max(1, n[ph])

    # bring the device to its working clocks before anything is compared
    P.ipm_init(x0, st, ws, opts)
    for _ in range(3 * reps):
        P.ipm_step(st, ws, opts)
    torch.cuda.synchronize()
    result = {"ms": {}}
    for which in colloc.Problem.TILE_KERNELS:
        cands = P.tile_options(which)
        best_of = {ts: float("inf") for ts in cands}
        for rnd in range(3):             # interleaved rounds, best time per candidate
            for ts in (cands if rnd % 2 == 0 else cands[::-1]):
                best_of[ts] = min(best_of[ts], measure(which, ts))
        best = min(cands, key=lambda t: best_of[t])
        for ts in cands:
            result["ms"][f"{which}:{ts}"] = best_of[ts]
            if verbose:
                print(f"autotune {key} {which} ts={ts}: {best_of[ts]:.4f} ms per phase", flush=True)
        P.tile_set(which, best)
        result[which] = best
    if cache_path:
        cache = _load(cache_path)
        cache[key] = result
        _save(cache_path, cache)
    return result
