"""Served form of the hot path: a request loop with continuous batching.

Requests (one encrypted query each, a database and a group) arrive over
time.  Rotation keys, every database and the queries stay resident in HBM.
The loop drives several *lanes*; a lane is a library context (own stream,
own device scratch) sharing the keys and databases, with its own slot
buffers.  Whenever a lane is idle and requests are waiting, it takes as
many as fit its slots and its scratch budget and launches the whole path
for them at once on its stream (the BSGS product of each request against
its own database and group -- from baby steps held over Q_l U P when the
databases are extended -- then the Chebyshev threshold).  Work already on
the device keeps running: a batch launched on another lane overlaps it, so
a request that arrives while others are on the GPU is admitted as soon as a
lane frees up, not when every batch in flight is done.  Completion is seen
by polling an event per batch; the host never waits for the whole device.

Admission follows the memory term of the stream-pool rule of §5.1.2 (Eq.
stream-pool): the slots in flight, S = min(units / 4, 0.2 F / (40 C), 32)
with F the free HBM and C one top-level ciphertext, are divided among the
lanes, and each lane's device scratch is capped (fr_ctx_set_scratch_limit)
at its share of the free HBM; a batch is sized from the measured scratch
per request so that it fits, and a batch that still meets FR_ENOMEM is
split and run again.

`plain` runs the same trace one request at a time through the one-query
calls, the reference the loop is compared against.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float           # seconds from the start of the trace
    kind: str                # "verify" or "identify"
    query: object            # fr.Ct at the top level
    db: object               # fr.Db
    group: int = 0
    admitted: float = -1.0
    done: float = -1.0
    lane: int = -1
    result: Optional[object] = None   # fr.Ct (kept only when asked)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def slot_count(ctx, compute_units: int = 256, cap: int = 64) -> int:
    """Number of query slots in flight from the free HBM (the stream-pool rule)."""
    import torch
    from . import fr
    free, _ = torch.cuda.mem_get_info(ctx.device)
    ct_bytes = 2.0 * (ctx.L + 1) * ctx.N * 8
    return min(cap, fr.stream_pool_size(compute_units, float(free), ct_bytes))


def _clone(ctx, ct):
    """Device copy of a ciphertext (its words are packed for its level)."""
    out = ctx.new_ct(ct.level)
    n = 2 * (ct.level + 1) * ctx.N
    out.buf[:n].copy_(ct.buf[:n])
    out.desc.level, out.desc.scale = ct.desc.level, ct.desc.scale
    return out


class Lane:
    """A context on its own stream with `slots` query buffers."""

    def __init__(self, fr, params, n1: int, slots: int, scratch_limit: int):
        import torch
        self.stream = torch.cuda.Stream()  # default priority
        with torch.cuda.stream(self.stream):
            self.ctx = fr.Context(**params)
            self.ctx.set_stream(self.stream)
            c = self.ctx
            self.rows = [[c.new_ct(c.L) for _ in range(n1 - 1)] for _ in range(slots)]
            self.scores = [c.new_ct(c.L - 1) for _ in range(slots)]
            self.chebs = [c.new_ct(c.L - 1) for _ in range(slots)]
        self.slots = slots
        self.limit = scratch_limit
        self.ctx.set_scratch_limit(scratch_limit)
        self.event = None
        self.batch: List[Request] = []
        self.max_batch = 0
        self.per_request = 0  # measured scratch bytes per request (peak over the largest batch)

    @property
    def busy(self) -> bool:
        return bool(self.batch)

    def room(self) -> int:
        """Requests a batch on this lane may take: its slots, and what its
        scratch budget holds at the measured scratch per request."""
        if self.per_request <= 0:
            return self.slots
        return max(1, min(self.slots, self.limit // self.per_request))


@dataclass
class Server:
    ctx: object              # the context that created the keys and databases
    keys: object
    coeffs: np.ndarray
    d1: int
    n1: int
    slots: int               # query slots in flight over all lanes
    lanes: int = 2
    keep_results: bool = False
    hbm_budget: Optional[int] = None  # device scratch over all lanes (default: 0.8 of the free HBM)
    poll_s: float = 50e-6
    batches: List[int] = field(default_factory=list)

    def __post_init__(self):
        import torch
        from . import fr
        c = self.ctx
        params = dict(log_n=c.N.bit_length() - 1, q0_bits=c.q[0].bit_length(), n_mid=c.L,
                      mid_bits=c.q[1].bit_length() if c.L else 30, n_special=c.nP,
                      special_bits=c.p[0].bit_length(), dnum=c.dnum)
        per_lane = max(1, self.slots // self.lanes)
        if self.hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(c.device)
            self.hbm_budget = int(0.8 * free)
        share = max(16 << 20, self.hbm_budget // self.lanes)
        self._lanes = [Lane(fr, params, self.n1, per_lane, share) for _ in range(self.lanes)]
        assert all(ln.ctx.moduli == c.moduli for ln in self._lanes)
        self.overlapped = 0   # batches launched while another lane's batch was on the device
        self.split = 0        # batches split after FR_ENOMEM

    # -- one batch on one lane ------------------------------------------------
    def _enqueue(self, lane: Lane, reqs: List[Request]):
        """The whole path for reqs on the lane's stream (no wait)."""
        import torch
        c, b = lane.ctx, len(reqs)
        with torch.cuda.stream(lane.stream):
            if all(r.db.extended for r in reqs):
                c.bsgs_matvec_hoisted_batch(self.keys, [r.query for r in reqs], [r.db for r in reqs],
                                            [r.group for r in reqs], outs=lane.scores[:b])
            else:
                rows = lane.rows[:b]
                c.rotate_hoisted_batch(self.keys, [r.query for r in reqs], range(1, self.n1), outs=rows)
                babies = [[r.query] + rows[i] for i, r in enumerate(reqs)]
                c.bsgs_diag_matvec_batch(self.keys, babies, [r.db for r in reqs], [r.group for r in reqs],
                                         outs=lane.scores[:b])
            c.chebyshev_eval_batch(self.keys, lane.scores[:b], self.coeffs, self.d1, outs=lane.chebs[:b])
            if self.keep_results:
                for i, r in enumerate(reqs):
                    r.result = _clone(c, lane.chebs[i])
            ev = torch.cuda.Event()
            ev.record(lane.stream)
        return ev

    def _launch(self, lane: Lane, reqs: List[Request]) -> List[Request]:
        """Launch as many of reqs as the lane's scratch takes (halving after
        FR_ENOMEM); returns the requests left over."""
        from . import fr
        take = reqs
        while True:
            try:
                ev = self._enqueue(lane, take)
                break
            except fr.FrError as e:
                if e.code != fr.FR_ENOMEM or len(take) == 1:
                    raise
                self.split += 1
                take = take[: len(take) // 2]
        lane.event, lane.batch = ev, take
        lane.max_batch = max(lane.max_batch, len(take))
        if lane.max_batch >= 2:
            lane.per_request = -(-lane.ctx.scratch_info()[1] // lane.max_batch)
        return reqs[len(take):]

    def run(self, trace: List[Request]) -> dict:
        """Serve the trace in real time; returns latency and throughput figures."""
        import torch
        trace = sorted(trace, key=lambda r: r.arrival)
        self.overlapped = self.split = 0  # counted per run
        waiting: List[Request] = []
        nxt, finished = 0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while finished < len(trace):
            now = time.perf_counter() - t0
            while nxt < len(trace) and trace[nxt].arrival <= now:
                waiting.append(trace[nxt])
                nxt += 1
            # retire the batches the device has finished
            for ln in self._lanes:
                if ln.busy and ln.event.query():
                    t = time.perf_counter() - t0
                    for r in ln.batch:
                        r.done = t
                    finished += len(ln.batch)
                    ln.batch, ln.event = [], None
            # admit waiting requests into idle lanes
            for li, ln in enumerate(self._lanes):
                if not waiting:
                    break
                if ln.busy:
                    continue
                take = waiting[: ln.room()]
                others_busy = any(o.busy for o in self._lanes if o is not ln)
                t = time.perf_counter() - t0
                back = self._launch(ln, take)
                waiting = back + waiting[len(take):]
                for r in ln.batch:
                    r.admitted, r.lane = t, li
                self.batches.append(len(ln.batch))
                self.overlapped += int(others_busy)
            if finished < len(trace):
                idle_all = not any(ln.busy for ln in self._lanes)
                if idle_all and not waiting and nxt < len(trace):
                    time.sleep(max(0.0, trace[nxt].arrival - (time.perf_counter() - t0)))
                else:
                    time.sleep(self.poll_s)
        res = summarize(trace, time.perf_counter() - t0, self.batches)
        res.update({"lanes": self.lanes, "slots": self.slots, "overlapped_batches": self.overlapped,
                    "split_batches": self.split, "scratch_budget_bytes": self.hbm_budget,
                    "per_request_scratch_bytes": [ln.per_request for ln in self._lanes]})
        return res


def plain(ctx, keys, coeffs, d1, n1, trace: List[Request], keep_results: bool = False) -> dict:
    """The same trace served one request at a time with the one-query calls."""
    import torch
    trace = sorted(trace, key=lambda r: r.arrival)
    rows = [ctx.new_ct(ctx.L) for _ in range(n1 - 1)]
    score, cheb = ctx.new_ct(ctx.L - 1), ctx.new_ct(ctx.L - 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in trace:
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        r.admitted = time.perf_counter() - t0
        if r.db.extended:
            ctx.bsgs_matvec_hoisted(keys, r.query, r.db, r.group, out=score)
        else:
            ctx.rotate_hoisted(keys, r.query, range(1, n1), outs=rows)
            ctx.bsgs_diag_matvec(keys, [r.query] + rows, r.db, r.group, out=score)
        ctx.chebyshev_eval(keys, score, coeffs, d1, out=cheb)
        if keep_results:
            r.result = _clone(ctx, cheb)
        torch.cuda.synchronize()
        r.done = time.perf_counter() - t0
    return summarize(trace, time.perf_counter() - t0, [1] * len(trace))


def summarize(trace: List[Request], wall: float, batches: List[int]) -> dict:
    lat = np.array([r.latency for r in trace]) * 1e3
    span = max(r.done for r in trace) - min(r.arrival for r in trace)
    return {"requests": len(trace), "wall_s": wall, "throughput_rps": len(trace) / span,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
            "batches": len(batches), "mean_batch": float(np.mean(batches)) if batches else 0.0}


def poisson_trace(rate: float, seconds: float, seed_rng) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate over [0, seconds)."""
    t, out = 0.0, []
    while True:
        t += seed_rng.exponential(1.0 / rate)
        if t >= seconds:
            return np.array(out)
        out.append(t)
