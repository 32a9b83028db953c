"""Served form of the hot path: a request loop over the batched C-ABI calls.

Requests (one encrypted query each, a database and a group) arrive over
time.  The loop keeps the rotation keys and every database resident, holds
a fixed pool of query slots whose size follows the paper's stream-pool rule
(Eq. stream-pool of §5.1.2: S = min(units / 4, 0.2 F / (40 C), 32) with F the
free HBM and C the size of one ciphertext), and runs continuous batching:
whenever the device finishes a batch, every request that has arrived since
is admitted into the free slots and the next batch runs the whole path for
all of them at once (the BSGS matvec with each request's own database and
group, from hoisted baby steps held over Q_l U P when every database of the
batch is extended, the Chebyshev threshold).  Requests that arrive
while a batch is in flight are admitted as soon as the slots free up.

`plain` runs the same trace one request at a time through the one-query
calls, the reference the batched loop is compared against.
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
    result: Optional[object] = None   # fr.Ct (kept only when asked)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def slot_count(ctx, compute_units: int = 256, cap: int = 64) -> int:
    """Number of query slots from the free HBM (the stream-pool rule)."""
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


@dataclass
class Server:
    ctx: object
    keys: object
    coeffs: np.ndarray
    d1: int
    n1: int
    slots: int
    keep_results: bool = False
    batches: List[int] = field(default_factory=list)

    def __post_init__(self):
        c = self.ctx
        self._rows = [[c.new_ct(c.L) for _ in range(self.n1 - 1)] for _ in range(self.slots)]
        self._scores = [c.new_ct(c.L - 1) for _ in range(self.slots)]
        self._chebs = [c.new_ct(c.L - 1) for _ in range(self.slots)]

    def _run_batch(self, reqs: List[Request]):
        c, b = self.ctx, len(reqs)
        if all(r.db.extended for r in reqs):
            c.bsgs_matvec_hoisted_batch(self.keys, [r.query for r in reqs], [r.db for r in reqs],
                                        [r.group for r in reqs], outs=self._scores[:b])
        else:
            rows = self._rows[:b]
            c.rotate_hoisted_batch(self.keys, [r.query for r in reqs], range(1, self.n1), outs=rows)
            babies = [[r.query] + rows[i] for i, r in enumerate(reqs)]
            c.bsgs_diag_matvec_batch(self.keys, babies, [r.db for r in reqs], [r.group for r in reqs],
                                     outs=self._scores[:b])
        c.chebyshev_eval_batch(self.keys, self._scores[:b], self.coeffs, self.d1, outs=self._chebs[:b])
        if self.keep_results:
            for i, r in enumerate(reqs):
                r.result = _clone(c, self._chebs[i])

    def run(self, trace: List[Request]) -> dict:
        """Serve the trace in real time; returns latency and throughput figures."""
        import torch
        trace = sorted(trace, key=lambda r: r.arrival)
        waiting: List[Request] = []
        nxt = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while nxt < len(trace) or waiting:
            now = time.perf_counter() - t0
            while nxt < len(trace) and trace[nxt].arrival <= now:
                waiting.append(trace[nxt])
                nxt += 1
            if not waiting:
                time.sleep(max(0.0, trace[nxt].arrival - now))
                continue
            take, waiting = waiting[: self.slots], waiting[self.slots:]
            for r in take:
                r.admitted = now
            self._run_batch(take)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            for r in take:
                r.done = t
            self.batches.append(len(take))
        return summarize(trace, time.perf_counter() - t0, self.batches)


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
