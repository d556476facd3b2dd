"""Thread-grid autotuner for the register-resident elimination kernels.

The element (level-0), separator-chain and border kernels each run on a TS x TS thread grid
that holds the kernel's matrix in registers (TS in 8, 16, 24, as instantiated for the shape).
The grid changes which thread computes an entry, not the arithmetic, so every choice gives the
same result; only the time differs.  `tune` times each usable grid per kernel on the device
(HIP events recorded by the library around each phase of kkt_factor) on an assembled system
built from the handle's own instances, keeps the fastest, and caches the choice in a JSON file
keyed by device architecture, shape class (n_s, n_r, n_p, K) and factor precision.  The choice
depends only on the shape class, never on the batch mix.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import colloc, workloads

DEFAULT_CACHE = os.environ.get(
    "COLLOC_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "colloc_tiles.json"))
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


def _assembled_system(P, precision, torch):
    """kkt_assemble on the handle's starting point with moderate barrier terms (positive
    definite for every instance), as the factor input the candidates are timed on."""
    insts = P.instances if isinstance(P.instances, (list, tuple)) else [P.instances]
    x = np.concatenate([workloads.initial_point(i, P.K) for i in insts])
    dev = P.device
    T = lambda a: torch.tensor(np.asarray(a, float), dtype=torch.float64, device=dev)
    rng = np.random.default_rng(0)
    m, n, ni = P.m_total, P.n_total, P.n_inst
    y = 0.01 * rng.standard_normal(m)
    ws = P.workspace(precision)
    _, jac, hess = P.derivs(T(x), T(y))
    P.assemble(ws, jac, hess, T(np.ones(ni * P.np_)), T(np.ones(m)), T(np.ones(ni)), T(np.zeros(n)),
               T(np.zeros(m)), T(np.zeros(m)), precision=precision)
    return ws


def tune(P, precision=colloc.FP64, reps=5, cache_path=DEFAULT_CACHE, force=False, verbose=False):
    """Choose and apply the fastest thread grid per kernel for the handle P.  Returns
    {"level0": ts, "chain": ts, "border": ts, "ms": {...}} (ts = 0: built-in rule)."""
    import torch

    key = shape_key(P, precision, _arch(torch))
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        for k in colloc.Problem.TILE_KERNELS:
            P.tile_set(k, cache[key][k])
        return cache[key]
    ws = _assembled_system(P, precision, torch)
    result = {"ms": {}}
    for which in colloc.Problem.TILE_KERNELS:
        best, best_ms = 0, float("inf")
        for ts in P.tile_options(which):
            P.tile_set(which, ts)
            P.factor(ws, precision)          # warm-up (code load)
            torch.cuda.synchronize()
            P.timing(True)
            for _ in range(reps):
                P.factor(ws, precision)
            torch.cuda.synchronize()
            ms, _ = P.timing_read()
            P.timing(False)
            t = ms[PHASE_OF[which]] / reps
            result["ms"][f"{which}:{ts}"] = t
            if verbose:
                print(f"autotune {key} {which} ts={ts}: {t:.4f} ms", flush=True)
            if t < best_ms:
                best, best_ms = ts, t
        P.tile_set(which, best)
        result[which] = best
    if cache_path:
        cache = _load(cache_path)
        cache[key] = result
        _save(cache_path, cache)
    return result
