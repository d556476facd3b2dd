"""Continuous-batching serving loop for parameter-estimation requests.

Requests (one estimation instance each) arrive over time and queue for the running batch of
their shape class (n_s, n_r, n_p, K).  At the next interior-point step boundary a batch is
rebuilt: finished members leave, and queued requests join as far as the HBM budget allows.  The
budget covers the true footprint of every batch (tables, state and workspace sized by the
batch's longest mesh) and the rebuild itself, during which the old and the new batch are both
alive; a request's memory is released only when the batch that held it is freed.
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
    return batch_bytes([inst], K, precision)


def admit_bytes(insts, K, precision):
    """Device bytes a batch of these instances needs while it is built: the batch, plus the
    rebuild's own temporaries (the starting points and 64 KiB for host-visible copies)."""
    return batch_bytes(insts, K, precision) + 65536 + alloc_bytes(8 * sum(
        int(i["N"]) * (K + 1) * int(i["n_s"]) + int(i["n_p"]) for i in insts))


# The torch caching allocator rounds a request up to 512 bytes, and hands a request above 1 MiB a
# cached block whole when less than 1 MiB of it would remain (it splits a large block only when
# more than 1 MiB is left over), so such a buffer can hold up to 1 MiB more than it asked for.
LARGE_BLOCK = 1 << 20


def alloc_bytes(n):
    """Device bytes one torch allocation of n bytes can hold at most."""
    n = (int(n) + 511) // 512 * 512
    return n + (LARGE_BLOCK if n > LARGE_BLOCK else 0)


def held_bytes(P, precision):
    """Device bytes a batch handle holds at most: its tables, state and workspace, each one
    allocator block."""
    return (alloc_bytes(P.table_bytes + 256) + alloc_bytes(P.lib.colloc_state_bytes(P.h)) +
            alloc_bytes(P.lib.colloc_workspace_bytes(P.h, precision)))


def batch_bytes(insts, K, precision):
    """Device bytes of a batch of these instances (its padding included), host-only."""
    P = colloc.Problem(list(insts), K, upload=False)
    try:
        return held_bytes(P, precision)
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
        return held_bytes(self.P, self.opts.precision) if self.P is not None else 0

    def _at_boundary(self):
        """Every member is between iterations (no inertia retry pending)."""
        if self.P is None:
            return True
        info = self.P.info(self.state)
        return bool(np.all((info["status"] != colloc.RUNNING) | (info["phase"] == 0)))

    def rebuild(self, now, room):
        """Apply membership changes at a step boundary: finished members leave, queued requests
        join with a fresh ipm_init (as many as fit), continuing members keep their state.
        room: device bytes this class may hold while rebuilding (its current batch included).
        Returns the bytes held at the peak of the rebuild (old and new batch alive)."""
        torch = self.torch
        keep = [r for r in self.members if r.status == colloc.RUNNING]
        old = self.device_bytes()
        if len(keep) == len(self.members) and not self.incoming:
            return old
        # a pending inertia retry reuses the workspace of its evaluation: the batch changes only
        # when every continuing member is between iterations
        if keep and not self._at_boundary():
            return old
        K, prec = self.shape[3], self.opts.precision

        def need(rs):
            return admit_bytes([r.inst for r in rs], K, prec)

        n_new = len(self.incoming)
        while n_new > 0 and old + need(keep + self.incoming[:n_new]) > room:
            n_new -= 1
        if n_new == 0 and len(keep) == len(self.members):
            return old                     # nothing leaves and nothing fits yet
        if n_new == 0 and keep and old + need(keep) > room:
            return old                     # shrinking would overrun the budget now: finished
                                           # members stay (masked) until it fits or all finish
        new, self.incoming = self.incoming[:n_new], self.incoming[n_new:]
        members = keep + new
        for r in new:
            r.t_admit = now
        with torch.cuda.stream(self.stream):
            if not members:
                self.P = self.ws = self.state = None
                self.members = []
                return old
            P = colloc.Problem([r.inst for r in members], K)
            if self.tiles:
                for k, ts in self.tiles.items():
                    P.tile_set(k, ts)
            ws, st = P.workspace(prec), P.state()
            # every slot starts from its initial point; continuing members then take their state
            x0 = torch.tensor(np.concatenate([workloads.initial_point(r.inst, K) for r in members]),
                              dtype=torch.float64, device="cuda")
            P.ipm_init(x0, st, ws, self.opts)
            for q, r in enumerate(keep):
                copy_instance(self.P, self.state, self.members.index(r), P, st, q)
            peak = old + need(members)
            self.stream.synchronize()          # init and copies done before x0 and the old batch go
            del x0
            if self.P is not None:
                self.P.close()
            self.P, self.ws, self.state, self.members = P, ws, st, members
        # the old batch's and the starting points' blocks go back to the device: a cached block
        # reused whole for a smaller buffer would hold more memory than the batch sizes account for
        torch.cuda.empty_cache()
        return peak

    def step(self, n):
        if self.P is None:
            return
        with self.torch.cuda.stream(self.stream):
            for _ in range(n):
                self.P.ipm_step(self.state, self.ws, self.opts)

    def poll(self, clock):
        """Record finished members (their results are read back here; the completion time is
        taken after the stream has synchronized)."""
        if self.P is None:
            return []
        with self.torch.cuda.stream(self.stream):
            info = self.P.info(self.state)
            now = clock()
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
    peak_bytes: int               # largest sum of the live batches' device bytes (rebuilds included)
    steps: int = 0
    peak_allocator_bytes: int = 0  # the torch allocator's peak over the run (state + workspaces)
    log: list = field(default_factory=list)

    def latencies(self):
        return np.array([r.latency for r in self.requests])

    def status_counts(self):
        out = {}
        for r in self.requests:
            out[colloc.STATUS_NAMES.get(r.status, str(r.status))] = out.get(
                colloc.STATUS_NAMES.get(r.status, str(r.status)), 0) + 1
        return out

    def summary(self):
        lat = self.latencies()
        return {"requests": len(self.requests), "finished_per_s": len(self.requests) / self.wall,
                "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "wall_s": self.wall, "peak_bytes": int(self.peak_bytes),
                "peak_allocator_bytes": int(self.peak_allocator_bytes),
                "solved": int(sum(r.status in (colloc.SOLVED, colloc.ACCEPTABLE) for r in self.requests)),
                "status": self.status_counts()}


def serve(requests, opts, budget_bytes, steps_per_round=4, max_steps=3000, tiles_for=None,
          clock=time.perf_counter):
    """Run the requests through the continuous-batching loop in real time (arrival times in
    seconds from the start).  Every batch, and every rebuild with its old and new batch alive at
    once, stays within budget_bytes of device memory.  Returns a ServeResult with per-request
    latency and results."""
    import torch

    for r in requests:
        r.shape = shape_class(r.inst, r.K)
        r.bytes = admit_bytes([r.inst], r.K, opts.precision)
        if r.bytes > budget_bytes:
            raise ValueError(f"request {r.rid} needs {r.bytes} bytes, above the budget")
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    classes: dict[tuple, ClassBatch] = {}
    peak = 0
    import gc
    gc.collect()                  # earlier handles freed before the baseline is taken
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    base_alloc = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    t0 = clock()
    rounds = 0
    while pending or any(c.busy() for c in classes.values()):
        now = clock() - t0
        while pending and pending[0].arrival <= now:   # arrivals queue at their class
            r = pending.popleft()
            cb = classes.get(r.shape)
            if cb is None:
                tiles = tiles_for(r) if tiles_for else None
                cb = classes[r.shape] = ClassBatch(r.shape, opts, torch, tiles)
            cb.incoming.append(r)
        if not any(c.members for c in classes.values()) and not any(c.incoming for c in classes.values()):
            if pending:
                time.sleep(max(0.0, min(0.01, pending[0].arrival - now)))
            continue
        for cb in classes.values():
            # room for this class's rebuild: the budget less what the other classes hold, by the
            # library's sizes and by the allocator's count, whichever is larger
            others = sum(c.device_bytes() for c in classes.values() if c is not cb)
            live = torch.cuda.memory_allocated() - base_alloc - cb.device_bytes()
            held = cb.rebuild(now, budget_bytes - max(others, live))
            peak = max(peak, others + held)
        for cb in classes.values():
            cb.step(steps_per_round)
        rounds += 1
        for cb in classes.values():
            cb.poll(lambda: clock() - t0)
        if rounds * steps_per_round > max_steps * 4:
            raise RuntimeError("serving loop did not drain")
    torch.cuda.synchronize()
    alloc_peak = torch.cuda.max_memory_allocated() - base_alloc
    return ServeResult(list(requests), clock() - t0, peak, rounds * steps_per_round, alloc_peak)


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
