"""Continuous-batching serving loop for parameter-estimation requests.

Requests (one estimation instance each) arrive over time.  Each is admitted when the device
memory it needs fits the HBM budget, joins the running batch of its shape class (n_s, n_r,
n_p, K) at the next interior-point step boundary, and leaves it when its status is final.
Every shape class runs its batch on its own HIP stream, so the steps of different classes
overlap on the device, and inside a class the instances share every launch.  The interior-point
state stays device-resident: an instance moves from one batch to the next by copying its
segments of the state buffer (see colloc_state_layout in include/colloc.h) on the device.

Because no per-instance arithmetic depends on the other members of a batch (fixed reduction
orders, thread grids chosen per shape class), a request's result is the same alone and in the
mix, bit for bit; `solve_alone` runs one request by itself for that comparison and for the
sequential per-instance baseline.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import colloc, workloads

# state fields that carry an instance's iterate between steps, with their per-instance extent
_VEC_N = ("x",)                          # n_q = N_q b + n_p, at x_off
_VEC_M = ("s", "y", "vL", "vU")          # m_q = N_q b, at g_off
_VEC_P = ("zL", "zU")                    # n_p, at q n_p
_VEC_F = ("fth", "fph")                  # COLLOC_FILTER_CAP, at q CAP
FILTER_CAP = 128


@dataclass
class Request:
    rid: int
    arrival: float
    inst: dict
    K: int = 3
    shape: tuple = ()
    bytes: int = 0
    t_admit: float = -1.0
    t_done: float = -1.0
    status: int = colloc.RUNNING
    iters: int = 0
    x: np.ndarray | None = None
    obj: float = float("nan")

    @property
    def latency(self):
        return self.t_done - self.arrival


def shape_class(inst, K):
    return (int(inst["n_s"]), int(inst["n_r"]), int(inst["n_p"]), K)


def request_bytes(inst, K, precision):
    """Device bytes of the request alone (tables, state, workspace), from a host-only handle."""
    P = colloc.Problem(inst, K, upload=False)
    try:
        return P.device_bytes(precision)
    finally:
        P.close()


def _seg(P, name, q):
    """(byte offset, count of doubles) of instance q's segment of a state field."""
    base = P.state_layout[name]
    if name in _VEC_N:
        return base + 8 * int(P.x_off[q]), int(P.Ns[q]) * P.b + P.np_
    if name in _VEC_M:
        return base + 8 * int(P.g_off[q]), int(P.Ns[q]) * P.b
    if name in _VEC_P:
        return base + 8 * q * P.np_, P.np_
    return base + 8 * q * FILTER_CAP, FILTER_CAP


def copy_instance(Ps, ss, qs, Pd, sd, qd):
    """Move instance qs of (Ps, state ss) into slot qd of (Pd, state sd), on the device."""
    for name in _VEC_N + _VEC_M + _VEC_P + _VEC_F:
        o1, n = _seg(Ps, name, qs)
        o2, n2 = _seg(Pd, name, qd)
        assert n == n2
        sd[o2:o2 + 8 * n].copy_(ss[o1:o1 + 8 * n])
    isz = colloc.INFO_DTYPE.itemsize
    o1 = Ps.state_layout["info"] + isz * qs
    o2 = Pd.state_layout["info"] + isz * qd
    sd[o2:o2 + isz].copy_(ss[o1:o1 + isz])


class ClassBatch:
    """The running batch of one shape class on its own stream."""

    def __init__(self, shape, opts, torch, tiles=None):
        self.shape = shape
        self.opts = opts
        self.torch = torch
        self.stream = torch.cuda.Stream()
        self.members: list[Request] = []
        self.incoming: list[Request] = []
        self.P = self.ws = self.state = None
        self.tiles = tiles

    def busy(self):
        return bool(self.members or self.incoming)

    def device_bytes(self):
        return self.P.device_bytes(self.opts.precision) if self.P is not None else 0

    def _at_boundary(self):
        """Every member is between iterations (no inertia retry pending)."""
        if self.P is None:
            return True
        info = self.P.info(self.state)
        return bool(np.all((info["status"] != colloc.RUNNING) | (info["phase"] == 0)))

    def rebuild(self, now):
        """Apply membership changes at a step boundary: finished members leave, admitted
        requests join with a fresh ipm_init, continuing members keep their state."""
        torch = self.torch
        keep = [r for r in self.members if r.status == colloc.RUNNING]
        if len(keep) == len(self.members) and not self.incoming:
            return
        # a pending inertia retry reuses the workspace of its evaluation: the batch changes only
        # when every continuing member is between iterations
        if keep and not self._at_boundary():
            return
        new = list(self.incoming)
        self.incoming = []
        members = keep + new
        with torch.cuda.stream(self.stream):
            if not members:
                self.P = self.ws = self.state = None
                self.members = []
                return
            K = self.shape[3]
            P = colloc.Problem([r.inst for r in members], K)
            if self.tiles:
                for k, ts in self.tiles.items():
                    P.tile_set(k, ts)
            ws, st = P.workspace(self.opts.precision), P.state()
            if new:
                Pn = colloc.Problem([r.inst for r in new], K)
                wsn, stn = Pn.workspace(self.opts.precision), Pn.state()
                x0 = torch.tensor(np.concatenate([workloads.initial_point(r.inst, K) for r in new]),
                                  dtype=torch.float64, device="cuda")
                Pn.ipm_init(x0, stn, wsn, self.opts)
                for j in range(len(new)):
                    copy_instance(Pn, stn, j, P, st, len(keep) + j)
            for q, r in enumerate(keep):
                copy_instance(self.P, self.state, self.members.index(r), P, st, q)
            self.P, self.ws, self.state, self.members = P, ws, st, members

    def step(self, n):
        if self.P is None:
            return
        with self.torch.cuda.stream(self.stream):
            for _ in range(n):
                self.P.ipm_step(self.state, self.ws, self.opts)

    def poll(self, now):
        """Record finished members (their results are read back here)."""
        if self.P is None:
            return []
        with self.torch.cuda.stream(self.stream):
            info = self.P.info(self.state)
            done = []
            x = None
            for q, r in enumerate(self.members):
                if r.status == colloc.RUNNING and info[q]["status"] != colloc.RUNNING:
                    if x is None:
                        x = self.P.state_vec(self.state, "x").cpu().numpy()
                    r.status = int(info[q]["status"])
                    r.iters = int(info[q]["iter"])
                    r.obj = float(info[q]["obj"])
                    r.x = x[self.P.x_off[q]:self.P.x_off[q] + int(self.P.Ns[q]) * self.P.b + self.P.np_].copy()
                    r.t_done = now
                    done.append(r)
        return done


@dataclass
class ServeResult:
    requests: list
    wall: float
    peak_bytes: int
    steps: int = 0
    log: list = field(default_factory=list)

    def latencies(self):
        return np.array([r.latency for r in self.requests])

    def summary(self):
        lat = self.latencies()
        return {"requests": len(self.requests), "solves_per_s": len(self.requests) / self.wall,
                "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "wall_s": self.wall, "peak_bytes": int(self.peak_bytes),
                "solved": int(sum(r.status in (colloc.SOLVED, colloc.ACCEPTABLE) for r in self.requests))}


def serve(requests, opts, budget_bytes, steps_per_round=4, max_steps=3000, tiles_for=None,
          clock=time.perf_counter):
    """Run the requests through the continuous-batching loop in real time (arrival times in
    seconds from the start).  Returns a ServeResult with per-request latency and results."""
    import torch

    for r in requests:
        r.shape = shape_class(r.inst, r.K)
        r.bytes = request_bytes(r.inst, r.K, opts.precision)
        if r.bytes > budget_bytes:
            raise ValueError(f"request {r.rid} needs {r.bytes} bytes, above the budget")
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    classes: dict[tuple, ClassBatch] = {}
    reserved = 0          # bytes of admitted, unfinished requests
    peak = 0
    t0 = clock()
    rounds = 0
    while pending or any(c.busy() for c in classes.values()):
        now = clock() - t0
        while pending and pending[0].arrival <= now and reserved + pending[0].bytes <= budget_bytes:
            r = pending.popleft()
            r.t_admit = now
            reserved += r.bytes
            cb = classes.get(r.shape)
            if cb is None:
                tiles = tiles_for(r) if tiles_for else None
                cb = classes[r.shape] = ClassBatch(r.shape, opts, torch, tiles)
            cb.incoming.append(r)
        if not any(c.busy() for c in classes.values()):
            if pending:
                time.sleep(max(0.0, min(0.01, pending[0].arrival - now)))
            continue
        for cb in classes.values():
            cb.rebuild(now)
        peak = max(peak, sum(c.device_bytes() for c in classes.values()))
        for cb in classes.values():
            cb.step(steps_per_round)
        rounds += 1
        now = clock() - t0
        for cb in classes.values():
            for r in cb.poll(now):
                reserved -= r.bytes
        if rounds * steps_per_round > max_steps * 4:
            raise RuntimeError("serving loop did not drain")
    torch.cuda.synchronize()
    return ServeResult(list(requests), clock() - t0, peak, rounds * steps_per_round)


def solve_alone(inst, opts, K=3, max_steps=3000, tiles=None):
    """One request by itself (its own handle); returns (status, iters, x, obj, seconds)."""
    import torch

    P = colloc.Problem(inst, K)
    if tiles:
        for k, ts in tiles.items():
            P.tile_set(k, ts)
    ws, st = P.workspace(opts.precision), P.state()
    x0 = torch.tensor(workloads.initial_point(inst, K), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.ipm_init(x0, st, ws, opts)
    for k in range(max_steps):
        P.ipm_step(st, ws, opts)
        if k % 4 == 3 and P.info(st)[0]["status"] != colloc.RUNNING:
            break
    info = P.info(st)[0]
    dt = time.perf_counter() - t0
    return int(info["status"]), int(info["iter"]), P.state_vec(st, "x").cpu().numpy(), float(info["obj"]), dt


def fifo_latencies(arrivals, service):
    """Latencies of a single-server FIFO queue with the given service times."""
    t, out = 0.0, []
    for a, s in zip(arrivals, service):
        t = max(t, a) + s
        out.append(t - a)
    return np.array(out)
