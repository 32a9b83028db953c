"""Autotuner of the library's launch choices, by measurement on the device.

What it picks (every candidate gives the same output words; only the kernel
variant and the work per launch change, so a choice is a speed decision):

* the NTT pass variant per launch size: for each of the four passes at
  N = 2^16 (forward columns / rows, inverse rows / columns), the largest
  launch, in limb polynomials, that takes the 4-words-per-thread passes
  (rounds of 2 stages, more threads) instead of the radix-16 register
  passes (16 words per thread, rounds of 4 stages) -- the radix and the
  limbs per block of a launch;
* the ModUp merge bound (inputs x digits up to which one conversion launch
  and one transform cover every digit);
* the order of the Chebyshev evaluation's launch groups (as recorded, or
  critical-first with level adjustments deferred to their consumers);
* whether the hoisted product forms its baby steps inside the MAC, and
  whether the giant steps' key inner products stage their keys in LDS;
* the batched forms' queries per chunk (products and Chebyshev passes);
* the Chebyshev baby-step degree d1 (a call parameter: fewer relinearised
  products against more levels and scalar work).

The search is coordinate descent over the knobs with the others held, each
candidate timed as the median of HIP-event durations of the caller's step on
the context's stream.  `tune` returns the choices and every trial so that a
run records what it measured.
"""
from __future__ import annotations

import json
import time
from typing import Callable, Dict, Iterable, List, Optional

import numpy as np

NTT_CANDIDATES = (0, 16, 32, 48, 64, 96, 128, 192, 256)
DEFAULT_SPACE = {
    "ntt_fwd_cols4": NTT_CANDIDATES,
    "ntt_fwd_rows4": NTT_CANDIDATES,
    "ntt_inv_rows4": NTT_CANDIDATES,
    "ntt_inv_cols4": NTT_CANDIDATES,
    "modup_merge": (3, 6, 12, 24, 48),
    "cheb_sched": (0, 1),
    "ksmac": (0, 1, 2),
    "ks_lds": (0, 1),
}
BATCH_SPACE = {"matvec_chunk": (2, 4, 8, 16), "cheb_chunk": (2, 4, 8, 16)}


def time_step(fn: Callable[[], None], reps: int = 5, warmup: int = 1) -> float:
    """Median duration (ms) of fn() between HIP events on torch's current
    stream (the library's stream)."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def tune(ctx, step: Callable[[], None], space: Optional[Dict[str, Iterable[int]]] = None, reps: int = 5,
         rounds: int = 1, log: Optional[Callable[[str], None]] = None) -> dict:
    """Coordinate descent over the knobs of `space` (default: the NTT pass
    variants and the ModUp merge bound) on the timing of `step`; leaves the
    context set to the best choices found and returns them with the trials."""
    space = dict(DEFAULT_SPACE if space is None else space)
    trials: List[dict] = []
    start = ctx.tune_state()
    base = time_step(step, reps)
    trials.append({"knobs": dict(start), "ms": base})
    best_ms = base
    t0 = time.perf_counter()
    for _ in range(rounds):
        for knob, cands in space.items():
            keep = ctx.get_tune(knob)
            best_v, best_t = keep, None
            for v in cands:
                ctx.set_tune(knob, v)
                t = time_step(step, reps)
                trials.append({"knobs": {knob: v}, "ms": t})
                if best_t is None or t < best_t:
                    best_v, best_t = v, t
            # keep the incumbent unless a candidate is measurably faster
            ctx.set_tune(knob, best_v if best_t is not None and best_t < best_ms * 0.995 else keep)
            if ctx.get_tune(knob) != keep:
                best_ms = best_t
            if log:
                log(f"autotune {knob}: {ctx.get_tune(knob)} ({best_ms:.3f} ms)")
    final = time_step(step, reps)
    return {"choices": ctx.tune_state(), "start": start, "start_ms": base, "final_ms": final,
            "search_s": time.perf_counter() - t0, "trials": trials}


def tune_d1(fr, step_for_d1: Callable[[int], None], degree: int, in_level: int,
            candidates: Iterable[int] = (4, 5, 6, 7, 8, 9, 10, 12, 16), reps: int = 5) -> dict:
    """The Chebyshev baby-step degree with the shortest measured step among
    those whose evaluation fits the levels left."""
    res = {}
    for d1 in candidates:
        if fr.cheb_out_level(in_level, degree, d1) < 0:
            continue
        res[d1] = time_step(lambda: step_for_d1(d1), reps)
    best = min(res, key=res.get)
    return {"d1": best, "ms": {str(k): v for k, v in res.items()},
            "products": {str(k): fr.cheb_mult_count(degree, k) for k in res}}


def save(record: dict, path: str):
    with open(path, "w") as f:
        json.dump(record, f, indent=1)
