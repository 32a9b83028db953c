#!/usr/bin/env python
"""Throughput of the encrypted identification hot path on one MI355X.

Workload (one "step" = one encrypted query, server side): 2^15 templates x
512-d, RNS-CKKS N = 2^16, Q = 60 + 14 x 40 bits, P = 5 x 60 bits, dnum = 3,
scale 2^40.  The paper's packing puts B = N/2 / 512 = 64 blocks of 512 x 512 in
each plaintext, so the whole database is one group of 512 pre-rotated
diagonals resident in HBM.  A step is
  31 hoisted baby-step rotations of the query (n1 = 32), formed inside
  the fused plaintext-diagonal multiply-accumulate of the 16 inner sums,
  16 rescales and the giant-step rotate-sum (n2 = 16),
  the degree-63 Chebyshev threshold at 0.3 on the score ciphertext.
Inputs (query ciphertext, keys, diagonals) are resident in HBM before the
timed region; the result ciphertext stays on the device for `value`.  The
host-side service time (the same step plus the download of the result
ciphertext, one query at a time) is reported beside it.

Prints one JSON line: scores/s (= 2^15 x steps / wall time), p50/p99 step
latency, the roofline figure of the dominant kernel class measured with HIP
events on the library's stream around every launch of that class over a
second pass of the same steps (the events themselves add time between
launches, so `value` comes from the uninstrumented pass), and the CPU oracle
timed on a bounded sample (one full query) on the host cores.
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

METRIC = "encrypted template scores/sec + p50/p99 query latency @2^15×512-d, 1 GPU"
HBM_PEAK_GBS = 8000.0
# INT32 VALU peak from the unit counts: 256 CUs x 128 lanes (the FP32 vector
# rate's lane count, 157.3 TFLOP/s / 2 per FMA) x 2.4 GHz
INT32_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
# algorithmic 32-bit integer operations per radix-2 butterfly on 64-bit
# residues: 10 multiplies for the 64x64-bit Shoup product and 20 adds,
# subtracts, compares and selects for the lazy reductions and both outputs
OPS_PER_BUTTERFLY = 30

# dominant kernel class (largest share of the step's kernel time in the trace)
ROOFLINE_KERNEL = {"class": "ntt", "bound": "alu"}
# HBM bytes per NTT launch (one forward or inverse transform of a batch of
# limbs, both passes), from the FETCH_SIZE / WRITE_SIZE counter runs recorded
# in profiles/ntt_query_2p15_counters.txt; None when the kernels have changed
# since those counters were taken
NTT_TRAFFIC_BYTES_PER_LAUNCH = 120250077


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def setup(args):
    import torch
    from paper_2604_00546_amd import fr, synth
    ctx = fr.Context(**fr.paper_params(), device=0)
    K, ell, n1 = 2 ** 15, 512, 32
    B = ctx.N // 2 // ell
    wl = synth.make_workload(3, K, ell, planted_frac=0.01)
    rots = fr.bsgs_rotation_set(ell, n1)
    t = time.time()
    keys = ctx.keygen(synth.int_seed(3, synth.SUB_KEYS), rots)
    db = ctx.db_load(wl.templates, ell, B, n1, ctx.L, 2.0 ** 40)
    if args.route == "hoisted":
        db.extend()
    qv = synth.replicate_query(wl.query, ctx.N // 2)
    q = ctx.encrypt(keys, ctx.encode(qv, ctx.L, 2.0 ** 40), synth.int_seed(3, synth.SUB_ENC))
    torch.cuda.synchronize()
    log(f"setup: keys ({len(rots)} rotations + relinearisation), {ell} diagonals, query: {time.time() - t:.1f} s")
    coeffs = fr.cheb_step_coeffs(63, 0.3)
    baby = [q] + [ctx.new_ct(ctx.L) for _ in range(n1 - 1)]
    score = ctx.new_ct(ctx.L - 1)
    cheb = ctx.new_ct(ctx.L - 1)
    return dict(fr=fr, ctx=ctx, wl=wl, keys=keys, db=db, q=q, baby=baby, score=score, cheb=cheb, coeffs=coeffs,
                n1=n1, ell=ell, B=B, K=K, route=args.route)


def matvec(s):
    """The score ciphertext of the query: the baby steps' ModDown hoisted
    past the inner sums, or hoisted rotations followed by the product."""
    ctx = s["ctx"]
    if s["route"] == "hoisted":
        ctx.bsgs_matvec_hoisted(s["keys"], s["q"], s["db"], 0, out=s["score"])
    else:
        ctx.rotate_hoisted(s["keys"], s["q"], range(1, s["n1"]), outs=s["baby"][1:])
        ctx.bsgs_diag_matvec(s["keys"], s["baby"], s["db"], 0, out=s["score"])


def step(s, d1):
    matvec(s)
    s["ctx"].chebyshev_eval(s["keys"], s["score"], s["coeffs"], d1, out=s["cheb"])


def batched(s, nq, steps, warmup, d1):
    """The same hot path for nq queries at once (rotation keys, giant-step
    keys and diagonals read once per batch): throughput and batch latency."""
    import torch
    fr, ctx, wl = s["fr"], s["ctx"], s["wl"]
    from paper_2604_00546_amd import synth
    Q = np.vstack([wl.query[None, :], synth.query_batch(3, nq - 1, s["ell"])])
    qs = [s["q"]] + [ctx.encrypt(s["keys"], ctx.encode(synth.replicate_query(Q[q], ctx.N // 2), ctx.L, 2.0 ** 40),
                                 synth.int_seed(3, synth.SUB_ENC, q)) for q in range(1, nq)]
    rows = [[ctx.new_ct(ctx.L) for _ in range(s["n1"] - 1)] for _ in range(nq)]
    babies = [[qs[q]] + rows[q] for q in range(nq)]
    scores = [ctx.new_ct(ctx.L - 1) for _ in range(nq)]
    chebs = [ctx.new_ct(ctx.L - 1) for _ in range(nq)]

    def bstep():
        if s["route"] == "hoisted":
            ctx.bsgs_matvec_hoisted_batch(s["keys"], qs, s["db"], 0, outs=scores)
        else:
            ctx.rotate_hoisted_batch(s["keys"], qs, range(1, s["n1"]), outs=rows)
            ctx.bsgs_diag_matvec_batch(s["keys"], babies, s["db"], 0, outs=scores)
        ctx.chebyshev_eval_batch(s["keys"], scores, s["coeffs"], d1, outs=chebs)

    for _ in range(warmup):
        bstep()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        bstep()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    # query 0 is the plain run's query: its result must be the plain run's words
    same = bool(np.array_equal(ctx.ct_export(chebs[0]), ctx.ct_export(s["cheb"])))
    return {"queries_per_batch": nq, "steps": steps, "value": s["K"] * nq * steps / wall, "unit": "scores/s",
            "ms_per_batch": wall * 1e3 / steps, "ms_per_query": wall * 1e3 / steps / nq,
            "batch_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "query0_equals_plain": same}


def mixed_batches(s, nbatch, d1):
    """Batches of 1..64 queries (sizes drawn from the batch stream), each query
    against its own database of 2^10..2^15 templates (sizes drawn per query),
    run batched and as a plain one-query loop on the same queries."""
    import torch
    from paper_2604_00546_amd import synth
    fr, ctx = s["fr"], s["ctx"]
    ell, n1 = s["ell"], s["n1"]
    r = synth.rng(4, synth.SUB_BATCH)
    sizes = r.integers(1, 65, size=nbatch)
    dbsz = [r.integers(10, 16, size=int(b)) for b in sizes]
    dbs = {}
    for e in range(10, 16):  # one resident database per size (prefixes of one template set)
        dbs[e] = ctx.db_load(s["wl"].templates[: 1 << e], ell, s["B"], n1, ctx.L, 2.0 ** 40)
        if s["route"] == "hoisted":
            dbs[e].extend()
    nmax = int(sizes.max())
    Q = synth.query_batch(4, nmax, ell)
    qs = [ctx.encrypt(s["keys"], ctx.encode(synth.replicate_query(Q[q], ctx.N // 2), ctx.L, 2.0 ** 40),
                      synth.int_seed(4, synth.SUB_ENC, q)) for q in range(nmax)]
    rows = [[ctx.new_ct(ctx.L) for _ in range(n1 - 1)] for _ in range(nmax)]
    babies = [[qs[q]] + rows[q] for q in range(nmax)]
    scores = [ctx.new_ct(ctx.L - 1) for _ in range(nmax)]
    chebs = [ctx.new_ct(ctx.L - 1) for _ in range(nmax)]
    torch.cuda.synchronize()

    hoisted = s["route"] == "hoisted"

    def run_batched(b, sz):
        if hoisted:
            ctx.bsgs_matvec_hoisted_batch(s["keys"], qs[:b], [dbs[int(e)] for e in sz], [0] * b, outs=scores[:b])
        else:
            ctx.rotate_hoisted_batch(s["keys"], qs[:b], range(1, n1), outs=rows[:b])
            ctx.bsgs_diag_matvec_batch(s["keys"], babies[:b], [dbs[int(e)] for e in sz], [0] * b,
                                       outs=scores[:b])
        ctx.chebyshev_eval_batch(s["keys"], scores[:b], s["coeffs"], d1, outs=chebs[:b])

    def run_plain(b, sz):
        for q in range(b):
            if hoisted:
                ctx.bsgs_matvec_hoisted(s["keys"], qs[q], dbs[int(sz[q])], 0, out=scores[q])
            else:
                ctx.rotate_hoisted(s["keys"], qs[q], range(1, n1), outs=rows[q])
                ctx.bsgs_diag_matvec(s["keys"], babies[q], dbs[int(sz[q])], 0, out=scores[q])
            ctx.chebyshev_eval(s["keys"], scores[q], s["coeffs"], d1, out=chebs[q])

    out = {}
    for name, fn in (("batched", run_batched), ("plain_loop", run_plain)):
        fn(int(sizes[0]), dbsz[0])  # warm the arena
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for b, sz in zip(sizes, dbsz):
            t1 = time.perf_counter()
            fn(int(b), sz)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t1) * 1e3)
        wall = time.perf_counter() - t0
        nq = int(sizes.sum())
        scored = int(sum((1 << int(e)) for sz in dbsz for e in sz))
        out[name] = {"queries": nq, "wall_s": wall, "queries_per_s": nq / wall, "scores_per_s": scored / wall,
                     "batch_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}}
    out["batches"] = int(nbatch)
    out["batch_sizes"] = [int(b) for b in sizes]
    out["speedup"] = out["plain_loop"]["wall_s"] / out["batched"]["wall_s"]
    return out


def served(s, seconds, d1, rates=(10.0, 50.0, 200.0), pool=64):
    """Poisson arrivals at each rate for `seconds`: half verification (one
    512-template block), half identification (2^10..2^15 templates), served
    with continuous batching and as a plain one-at-a-time loop on the same
    trace.  Requests reuse a pool of encrypted queries."""
    from paper_2604_00546_amd import serve, synth
    ctx, ell, n1 = s["ctx"], s["ell"], s["n1"]
    dbs = {e: ctx.db_load(s["wl"].templates[: 1 << e], ell, s["B"], n1, ctx.L, 2.0 ** 40) for e in range(9, 16)}
    if s["route"] == "hoisted":
        for d in dbs.values():
            d.extend()
    Q = synth.query_batch(5, pool, ell)
    qs = [ctx.encrypt(s["keys"], ctx.encode(synth.replicate_query(Q[q], ctx.N // 2), ctx.L, 2.0 ** 40),
                      synth.int_seed(5, synth.SUB_ENC, q)) for q in range(pool)]
    slots = serve.slot_count(ctx)
    srv = serve.Server(ctx, s["keys"], s["coeffs"], d1, n1, slots=slots)
    out = {"slots": slots, "seconds": seconds, "query_pool": pool}
    for rate in rates:
        arr = serve.poisson_trace(rate, seconds, synth.rng(5, synth.SUB_ARRIVAL, int(rate)))
        kr = synth.rng(5, synth.SUB_KIND, int(rate))
        kinds = kr.integers(0, 2, size=len(arr))
        sizes = kr.integers(10, 16, size=len(arr))

        def trace():
            return [serve.Request(i, float(t), "verify" if kinds[i] else "identify", qs[i % pool],
                                  dbs[9] if kinds[i] else dbs[int(sizes[i])]) for i, t in enumerate(arr)]
        srv.batches = []
        b = srv.run(trace())
        log(f"served {rate:g}/s: continuous batching done ({b['requests']} requests), plain loop ...")
        p = serve.plain(ctx, s["keys"], s["coeffs"], d1, n1, trace())
        out[f"{rate:g}/s"] = {"batched": b, "plain": p}
        log(f"served {rate:g}/s: batched p50 {b['latency_ms']['p50']:.1f} ms p99 {b['latency_ms']['p99']:.1f} ms; "
            f"plain p50 {p['latency_ms']['p50']:.1f} ms p99 {p['latency_ms']['p99']:.1f} ms")
    return out


def layout_b1(s, K, d1, steps=2):
    """The same identification with one 512 x 512 block per plaintext (B = 1):
    K / 512 groups of 512 diagonals, every group scored from the one set of
    baby steps (the group matvecs run batched), then the Chebyshev threshold
    on every score ciphertext.  Returns per-query time and scores/s."""
    import torch
    ctx, ell, n1 = s["ctx"], s["ell"], s["n1"]
    db = ctx.db_load(s["wl"].templates[:K], ell, 1, n1, ctx.L, 2.0 ** 40)
    G = db.G
    babies = [s["baby"]] * G
    scores = [ctx.new_ct(ctx.L - 1) for _ in range(G)]
    chebs = [ctx.new_ct(ctx.L - 1) for _ in range(G)]

    def run():
        ctx.rotate_hoisted(s["keys"], s["q"], range(1, n1), outs=s["baby"][1:])
        ctx.bsgs_diag_matvec_batch(s["keys"], babies, db, list(range(G)), outs=scores)
        ctx.chebyshev_eval_batch(s["keys"], scores, s["coeffs"], d1, outs=chebs)

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # check: the scores of group 0 and of the last group
    exact = s["wl"].exact_scores()[:K]
    err = 0.0
    for g in (0, G - 1):
        dec = ctx.decrypt_decode(s["keys"], scores[g])[:ell]
        err = max(err, float(np.max(np.abs(dec - exact[g * ell:(g + 1) * ell]))))
    return {"templates": K, "groups": G, "ms_per_query": dt * 1e3, "scores_per_s": K / dt,
            "diagonal_bytes": G * ell * ctx.N * sum(5 if q < (1 << 40) else 8 for q in ctx.q[: ctx.L + 1]),
            "score_max_abs_err": err}


def rotq_vs_bsgs(s, K, d1, steps=2):
    """Alg. bsgs-precomp's route against BSGS for K templates (G groups at
    B = 64): the full table of ell query rotations (every baby step rotated
    by every giant amount, batched), then per group a pure diagonal MAC over
    plain diagonals; BSGS: the giant-step key switches per group.  Both end
    with the Chebyshev threshold on every score ciphertext."""
    import torch
    from paper_2604_00546_amd import synth
    ctx, ell, n1, B = s["ctx"], s["ell"], s["n1"], s["B"]
    wl = synth.make_workload(3, K, ell, planted_frac=0.01)  # the same query as the bench's workload
    T = wl.templates
    db_bsgs = ctx.db_load(T, ell, B, n1, ctx.L, 2.0 ** 40)
    db_plain = ctx.db_load(T, ell, B, ell, ctx.L, 2.0 ** 40)
    G = db_bsgs.G
    giant = [n1 * j for j in range(1, ell // n1)]
    rows = [[ctx.new_ct(ctx.L) for _ in giant] for _ in range(n1)]
    table = [s["baby"][i] if j == 0 else rows[i][j - 1] for j in range(ell // n1) for i in range(n1)]
    scores = [ctx.new_ct(ctx.L - 1) for _ in range(G)]
    chebs = [ctx.new_ct(ctx.L - 1) for _ in range(G)]

    def bsgs():
        ctx.rotate_hoisted(s["keys"], s["q"], range(1, n1), outs=s["baby"][1:])
        ctx.bsgs_diag_matvec_batch(s["keys"], [s["baby"]] * G, db_bsgs, list(range(G)), outs=scores)
        ctx.chebyshev_eval_batch(s["keys"], scores, s["coeffs"], d1, outs=chebs)

    def rotq():
        ctx.rotate_hoisted(s["keys"], s["q"], range(1, n1), outs=s["baby"][1:])
        ctx.rotate_hoisted_batch(s["keys"], s["baby"], giant, outs=rows)
        ctx.bsgs_diag_matvec_batch(s["keys"], [table] * G, db_plain, list(range(G)), outs=scores)
        ctx.chebyshev_eval_batch(s["keys"], scores, s["coeffs"], d1, outs=chebs)

    out = {"templates": K, "groups": G}
    for name, fn in (("bsgs", bsgs), ("rotq_table", rotq)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        dec = ctx.decrypt_decode(s["keys"], scores[G - 1])
        exact = wl.exact_scores()[(G - 1) * B * ell: K]
        out[name] = {"ms_per_query": dt * 1e3, "scores_per_s": K / dt,
                     "score_max_abs_err": float(np.max(np.abs(dec[: len(exact)] - exact)))}
    return out


def encrypted_db(s, d1, steps=2):
    """The paper's setting: the 512 diagonals of the 2^15-template database
    encrypted.  Three routes to the group's score, each followed by the
    Chebyshev threshold:
      rotation table: Rescale(Relin(sum_d rot_d(q) (x) Enc(diag_d))) over the
        full table of query rotations, one relinearisation per group;
      BSGS-TBS: the server pre-rotates the encrypted diagonals by -j n1 with
        temporary negative giant-step keys (offline, then the keys are
        freed); online, one relinearisation per giant step and the giant
        rotate-sum (§5.3.1-§5.3.2);
      BSGS-TBE: the enroller pre-rotates the plaintext slots before
        encryption (§5.3.3); the same online product."""
    import torch
    from paper_2604_00546_amd import synth
    fr, ctx, ell, n1, keys = s["fr"], s["ctx"], s["ell"], s["n1"], s["keys"]
    n2 = ell // n1
    t = time.time()
    plain = ctx.db_load(s["wl"].templates, ell, s["B"], ell, ctx.L, 2.0 ** 40)
    enc = [ctx.encrypt(keys, ctx.pt_import(plain.export(0, d), ctx.L, 2.0 ** 40),
                       synth.int_seed(3, synth.SUB_ENC, 1000 + d)) for d in range(ell)]
    del plain
    torch.cuda.synchronize()
    setup_s = time.time() - t
    giant = [n1 * j for j in range(1, n2)]
    rows = [[ctx.new_ct(ctx.L) for _ in giant] for _ in range(n1)]
    table = [s["baby"][i] if j == 0 else rows[i][j - 1] for j in range(n2) for i in range(n1)]
    score, cheb = ctx.new_ct(ctx.L - 1), ctx.new_ct(ctx.L - 1)
    exact = s["wl"].exact_scores()

    def timed(run):
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        err = float(np.max(np.abs(ctx.decrypt_decode(keys, score) - exact)))
        return {"ms_per_query": dt * 1e3, "scores_per_s": s["K"] / dt, "score_max_abs_err": err}

    def table_route():
        ctx.rotate_hoisted(keys, s["q"], range(1, n1), outs=s["baby"][1:])
        ctx.rotate_hoisted_batch(keys, s["baby"], giant, outs=rows)
        ctx.tensor_sum_relin_rescale(keys, table, enc, out=score)
        ctx.chebyshev_eval(keys, score, s["coeffs"], d1, out=cheb)

    out = {"encrypted_diagonals": ell, "setup_s": setup_s, "rotation_table": timed(table_route)}
    del rows, table
    # BSGS-TBS: homomorphic pre-rotation with temporary negative giant-step keys
    t = time.time()
    tmp = ctx.keygen(synth.int_seed(3, synth.SUB_KEYS), [-g for g in giant])
    torch.cuda.synchronize()
    keygen_s = time.time() - t
    t = time.time()
    tbs = list(enc[:n1])
    for j in range(1, n2):
        tbs += [row[0] for row in ctx.rotate_hoisted_batch(tmp, enc[j * n1:(j + 1) * n1], [-n1 * j])]
    torch.cuda.synchronize()
    prerot_s = time.time() - t
    del tmp, enc
    torch.cuda.synchronize()

    def bsgs_route(diag):
        def run():
            ctx.rotate_hoisted(keys, s["q"], range(1, n1), outs=s["baby"][1:])
            ctx.bsgs_encrypted_matvec(keys, s["baby"], diag, out=score)
            ctx.chebyshev_eval(keys, score, s["coeffs"], d1, out=cheb)
        return run

    out["bsgs_tbs"] = dict(timed(bsgs_route(tbs)), temp_keys=len(giant), temp_keygen_s=keygen_s,
                           prerotation_s=prerot_s)
    del tbs
    # BSGS-TBE: the enroller encrypts the pre-rotated plaintext diagonals
    t = time.time()
    pre = ctx.db_load(s["wl"].templates, ell, s["B"], n1, ctx.L, 2.0 ** 40)
    tbe = [ctx.encrypt(keys, ctx.pt_import(pre.export(0, d), ctx.L, 2.0 ** 40),
                       synth.int_seed(3, synth.SUB_ENC, 2000 + d)) for d in range(ell)]
    del pre
    torch.cuda.synchronize()
    out["bsgs_tbe"] = dict(timed(bsgs_route(tbe)), enroll_s=time.time() - t)
    return out


def diagonal_method(s, d1, steps=2):
    """HyDia-style diagonal method (n1 = ell, n2 = 1): 511 hoisted rotations
    of the query and one MAC over the 512 plain diagonals, for the bench's
    2^15-template database; needs 511 rotation keys (about 29 GB)."""
    import torch
    ctx, ell = s["ctx"], s["ell"]
    fr = s["fr"]
    from paper_2604_00546_amd import synth
    t = time.time()
    keys = ctx.keygen(synth.int_seed(3, synth.SUB_KEYS), list(range(1, ell)))
    db = ctx.db_load(s["wl"].templates, ell, s["B"], ell, ctx.L, 2.0 ** 40)
    torch.cuda.synchronize()
    setup_s = time.time() - t
    baby = [s["q"]] + [ctx.new_ct(ctx.L) for _ in range(ell - 1)]
    score, cheb = ctx.new_ct(ctx.L - 1), ctx.new_ct(ctx.L - 1)

    def run():
        ctx.rotate_hoisted(keys, s["q"], range(1, ell), outs=baby[1:])
        ctx.bsgs_diag_matvec(keys, baby, db, 0, out=score)
        ctx.chebyshev_eval(keys, score, s["coeffs"], d1, out=cheb)

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    dec = ctx.decrypt_decode(keys, score)
    err = float(np.max(np.abs(dec - s["wl"].exact_scores())))
    del keys
    return {"rotation_keys": ell - 1, "setup_s": setup_s, "ms_per_query": dt * 1e3, "scores_per_s": s["K"] / dt,
            "score_max_abs_err": err}


def service_time(s, d1, n):
    """Host-side service time of one query at a time (start of the GPU work
    until the score ciphertext is on the host): the step, then the download
    of the Chebyshev output's words into pinned host memory, waited for."""
    import torch
    cheb = s["cheb"]
    words = 2 * (cheb.level + 1) * s["ctx"].N
    host = torch.empty(words, dtype=torch.int64, pin_memory=True)
    stream = torch.cuda.current_stream()
    lat = []
    for _ in range(n):
        t0 = time.perf_counter()
        step(s, d1)
        host.copy_(cheb.buf[:words], non_blocking=True)
        stream.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    lat = np.array(lat)
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)), "mean": float(lat.mean()),
            "queries": n, "bytes_downloaded": words * 8}


def hook_roofline(s, d1, cls, name, steps=3):
    """HBM roofline of one kernel class from the library's timing hook (HIP
    events around every launch of the class on its stream; algorithmic
    bytes of each launch) over `steps` extra steps."""
    ctx = s["ctx"]
    ctx.prof_begin(cls)
    for _ in range(steps):
        step(s, d1)
    n, ms, b = ctx.prof_end()
    if not n:
        return None
    avg = ms / n
    gbs = b / n / (avg * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": None, "launches_per_step": n / steps, "avg_launch_ms": avg,
            "bytes_per_launch": b / n}


def graph_form(s, d1, steps):
    """The same step recorded once as a HIP graph (fr_graph_begin/end) and
    replayed: before each replay one of two encrypted queries is copied into
    the recorded input buffer, and the replay's result must equal the eager
    step's words for that query."""
    import torch
    from paper_2604_00546_amd import synth
    ctx, keys = s["ctx"], s["keys"]
    q2 = ctx.encrypt(keys, ctx.encode(synth.replicate_query(synth.query_batch(3, 1, s["ell"])[0], ctx.N // 2),
                                      ctx.L, 2.0 ** 40), synth.int_seed(3, synth.SUB_ENC, 77))
    queries = [s["q"], q2]
    # eager reference words of both queries
    ref = []
    for q in queries:
        matvec_of(s, q, s["score"])
        ctx.chebyshev_eval(keys, s["score"], s["coeffs"], d1, out=s["cheb"])
        ref.append(ctx.ct_export(s["cheb"]))
    inp = ctx.new_ct(ctx.L)
    inp.buf.copy_(queries[0].buf)
    inp.desc.level, inp.desc.scale = queries[0].level, queries[0].scale

    def body():
        matvec_of(s, inp, s["score"])
        ctx.chebyshev_eval(keys, s["score"], s["coeffs"], d1, out=s["cheb"])

    body()  # the arena at its full size before the recording
    graph = ctx.capture(body)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        graph.launch()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        inp.buf.copy_(queries[i % 2].buf)
        graph.launch()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    last = (steps - 1) % 2
    same = bool(np.array_equal(ctx.ct_export(s["cheb"]), ref[last]))
    # host-side service time with the graph: copy in, replay, download, wait
    words = 2 * (s["cheb"].level + 1) * ctx.N
    host = torch.empty(words, dtype=torch.int64, pin_memory=True)
    svc = []
    for i in range(steps):
        t1 = time.perf_counter()
        inp.buf.copy_(queries[i % 2].buf)
        graph.launch()
        host.copy_(s["cheb"].buf[:words], non_blocking=True)
        stream.synchronize()
        svc.append((time.perf_counter() - t1) * 1e3)
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    svc = np.array(svc)
    step(s, d1)  # the bench query's own result back in score / cheb for the checks
    torch.cuda.synchronize()
    return {"steps": steps, "ms_per_step": wall * 1e3 / steps, "value": s["K"] * steps / wall, "unit": "scores/s",
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "service_ms": {"p50": float(np.percentile(svc, 50)), "p99": float(np.percentile(svc, 99)),
                           "mean": float(svc.mean())},
            "replays_equal_eager": same}


def matvec_of(s, q, out):
    ctx = s["ctx"]
    if s["route"] == "hoisted":
        ctx.bsgs_matvec_hoisted(s["keys"], q, s["db"], 0, out=out)
    else:
        baby = [q] + s["baby"][1:]
        ctx.rotate_hoisted(s["keys"], q, range(1, s["n1"]), outs=s["baby"][1:])
        ctx.bsgs_diag_matvec(s["keys"], baby, s["db"], 0, out=out)


def autotune_step(s, args):
    """Launch choices and the Chebyshev baby-step degree picked by the
    project's autotuner on this workload's step (same words for every
    choice)."""
    from paper_2604_00546_amd import autotune
    fr, ctx = s["fr"], s["ctx"]
    rec = autotune.tune(ctx, lambda: step(s, args.d1), log=log)
    d = autotune.tune_d1(fr, lambda d1: step(s, d1), len(s["coeffs"]) - 1, ctx.L - 1)
    rec["d1"] = d
    rec["trials"] = len(rec["trials"])
    return rec


def fewest_products_d1(fr, degree):
    """Baby-step degree with the fewest relinearised products (ties: smaller)."""
    counts = {d1: fr.cheb_mult_count(degree, d1) for d1 in range(2, degree + 2)}
    return min(counts, key=lambda d1: (counts[d1], d1))


def check(s):
    ctx, wl = s["ctx"], s["wl"]
    exact = wl.exact_scores()
    dec = ctx.decrypt_decode(s["keys"], s["score"])
    err_s = float(np.max(np.abs(dec - exact)))
    y = ctx.decrypt_decode(s["keys"], s["cheb"])
    want = np.polynomial.chebyshev.chebval(exact, s["coeffs"])
    err_c = float(np.max(np.abs(y - want)))
    found = np.nonzero(y >= 0.5)[0]
    return {"score_max_abs_err": err_s, "score_tol": 2.0 ** -20, "cheb_max_abs_err": err_c, "cheb_tol": 2.0 ** -12,
            "identified": int(len(found)), "planted": int(len(wl.planted)),
            "identification_exact": bool(np.array_equal(found, wl.planted))}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _last10(ts):
    """Mean and population std of the last 10 of 11 trials (the paper's
    benchmarking methodology, §6.2), in ms."""
    t = np.array(ts[1:]) * 1e3
    return {"trials": len(ts), "mean_ms": float(t.mean()), "std_ms": float(t.std())}


def oracle_small_pipeline(trials=11):
    """The oracle's whole plain pipeline on the small workload (N = 2^12, 64
    templates x 128-d, n1 = 8, n2 = 16, B = 16, no Chebyshev): encode,
    encrypt, 7 hoisted rotations, BSGS matvec, decrypt, decode; `trials`
    runs after key generation and diagonal encoding."""
    from oracle import oracle as O
    from paper_2604_00546_amd import synth
    o = O.Context(**O.small_params())
    rots = list(range(1, 8)) + [8 * j for j in range(1, 16)]
    keys = o.keygen(synth.int_seed(1, synth.SUB_KEYS), rots)
    wl = synth.make_workload(1, 64, 128)
    db = o.db_build(wl.templates, wl.K, 128, 16, 8, o.L, 2.0 ** 40)
    qv = synth.replicate_query(wl.query, o.N // 2)
    ts = []
    for t in range(trials):
        t0 = time.perf_counter()
        q = o.encrypt(keys, o.encode(qv, o.L, 2.0 ** 40), synth.int_seed(1, synth.SUB_ENC, t))
        baby = [q] + o.rotate_hoisted(keys, q, range(1, 8))
        o.decrypt_decode(keys, o.bsgs_matvec(keys, baby, db, 0))
        ts.append(time.perf_counter() - t0)
    return _last10(ts)


def cpu_baseline(s, d1, trials=3, one_thread_query=False):
    """The CPU oracle, as it stands, timed on the host cores: one full query
    of the same 2^15 x 512 workload (`trials` runs, all threads), and the
    small workload's whole pipeline (11 trials) on all threads and on one."""
    from oracle import oracle as O
    from paper_2604_00546_amd import synth
    fr = s["fr"]
    threads = O.get_threads()
    o = O.Context(**O.paper_params())
    rots = fr.bsgs_rotation_set(s["ell"], s["n1"])
    keys = o.keygen(synth.int_seed(3, synth.SUB_KEYS), rots)
    wl = s["wl"]
    db = o.db_build(wl.templates, wl.K, s["ell"], s["B"], s["n1"], o.L, 2.0 ** 40)
    if s["route"] == "hoisted":
        db.extend()
    q = o.encrypt(keys, o.encode(synth.replicate_query(wl.query, o.N // 2), o.L, 2.0 ** 40), 5)

    def query():
        t0 = time.perf_counter()
        if s["route"] == "hoisted":
            S = o.bsgs_matvec_hoisted(keys, q, db, 0)
        else:
            baby = [q] + o.rotate_hoisted(keys, q, range(1, s["n1"]))
            S = o.bsgs_matvec(keys, baby, db, 0)
        o.chebyshev(keys, S, s["coeffs"], d1)
        return time.perf_counter() - t0

    ts = [query() for _ in range(trials)]
    dt = float(np.mean(ts))
    out = {"value": s["K"] / dt, "unit": "scores/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "sample": f"one full query (31 hoisted rotations, BSGS matvec over 512 diagonals, degree-63 "
                     f"Chebyshev; route {s['route']}) of the same 2^15 x 512 workload, mean of {trials} runs "
                     f"({dt:.2f} s wall, std {float(np.std(ts)):.2f} s) on {threads} OpenMP threads; key "
                     f"generation and diagonal encoding (with the special-prime limbs) excluded as setup",
           "query_s": [float(t) for t in ts]}
    log(f"oracle query: {dt:.2f} s on {threads} threads; small pipeline, 11 trials ...")
    out["small_pipeline"] = {"workload": "N=2^12, 64 templates x 128-d, n1=8 n2=16 B=16, encode to decode",
                             f"{threads}_threads": oracle_small_pipeline()}
    O.set_threads(1)
    try:
        out["small_pipeline"]["1_thread"] = oracle_small_pipeline()
        if one_thread_query:
            log("oracle query on one thread ...")
            t1 = query()
            out["one_thread_query_s"] = t1
            out["one_thread_scores_per_s"] = s["K"] / t1
    finally:
        O.set_threads(threads)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--d1", type=int, default=None,
                    help="Chebyshev baby-step degree (default: the one with the fewest relinearised products)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-one-thread-query", action="store_true",
                    help="also time the oracle's full 2^15 query on one thread (minutes)")
    ap.add_argument("--mix", type=int, default=0,
                    help="also run this many batches of 1..64 queries against databases of 2^10..2^15 "
                         "templates, batched and as a plain loop")
    ap.add_argument("--serve", type=float, default=0.0,
                    help="also serve Poisson traces at 10, 50 and 200 requests/s for this many seconds each, "
                         "with continuous batching and as a plain loop")
    ap.add_argument("--b1", type=int, default=0,
                    help="also run the identification with one block per plaintext (B = 1) for this many "
                         "templates (a multiple of 512)")
    ap.add_argument("--rotq", type=int, default=0,
                    help="also compare the full rotation-table route with BSGS for this many templates")
    ap.add_argument("--dg", action="store_true", help="also time the diagonal method (511 rotation keys)")
    ap.add_argument("--edb", action="store_true", help="also time the encrypted-database route")
    ap.add_argument("--batch", type=int, default=16,
                    help="queries per batch for the batched-form figure (0: skip it)")
    ap.add_argument("--route", choices=("hoisted", "single"), default="hoisted",
                    help="hoisted: baby steps held over Q_l U P, inner sums' first polynomials summed before one "
                         "ModDown, one ModDown per second polynomial (fr_bsgs_matvec_hoisted); "
                         "single: hoisted rotations, each with its ModDown, then the product")
    ap.add_argument("--breakdown", action="store_true", help="extra pass timing every kernel class")
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default launch choices and "
                    "the fewest-products Chebyshev degree")
    ap.add_argument("--graph", action="store_true",
                    help="also time the HIP-graph replay form (capture is switched off in the library: "
                         "fr_graph_begin returns FR_EINVAL)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the steps, one device-to-device copy of this many MiB (the known-size "
                         "reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding by matrix "
              f"groups is a design note, not built", file=sys.stderr)
        sys.exit(2)
    import torch
    s = setup(args)
    if args.d1 is None:
        args.d1 = fewest_products_d1(s["fr"], len(s["coeffs"]) - 1)
    ctx = s["ctx"]
    for _ in range(args.warmup):
        step(s, args.d1)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")
    tuned = None
    if not args.no_autotune:
        tuned = autotune_step(s, args)
        args.d1 = tuned["d1"]["d1"]
        log(f"autotuned: {tuned['choices']}, d1 = {args.d1}")
        for _ in range(args.warmup):
            step(s, args.d1)
        torch.cuda.synchronize()
    if args.calib_copy_mib:
        # known-size device copy just before the timed steps: the reference
        # for the HBM byte counters and the marker that opens the timed
        # region in a kernel trace
        src = torch.ones(args.calib_copy_mib << 17, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calib_copy_mib} MiB done")
        del src, dst

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        step(s, args.d1)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    log(f"timed {args.steps} steps: {wall * 1e3 / args.steps:.2f} ms/step")
    # the roofline of the dominant kernel class: the same steps again, with a
    # pair of HIP events around every launch of that class on the stream it
    # runs on (the events add a little time between launches, so `value`
    # comes from the uninstrumented steps above)
    ctx.prof_begin(ROOFLINE_KERNEL["class"])
    t1 = time.perf_counter()
    for i in range(args.steps):
        step(s, args.d1)
    n_launch, k_ms, k_bytes = ctx.prof_end()
    hooked_ms = (time.perf_counter() - t1) * 1e3 / args.steps

    out = {
        "metric": METRIC,
        "value": s["K"] * args.steps / wall,
        "unit": "scores/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "identification of one encrypted query against 2^15 templates x 512-d "
                               "(1% planted at cosine 0.6-0.9), B=64 blocks per plaintext (one group of 512 "
                               "pre-rotated diagonals), n1=32 n2=16, degree-63 Chebyshev step at 0.3 "
                               f"(d1={args.d1}); RNS-CKKS N=2^16, Q=60+14x40 bits, P=5x60 bits, dnum=3, "
                               "scale 2^40", "templates": s["K"], "dim": s["ell"], "ring_dim": ctx.N,
                   "form": "plain, one query at a time",
                   "route": (("baby steps held over Q_l U P" +
                              (" and formed inside the MAC" if ctx.get_tune("ksmac") else "") +
                              "; inner sums' first polynomials rotated and summed before one ModDown, one ModDown "
                              "per second polynomial") if args.route == "hoisted"
                             else "hoisted rotations with one ModDown each, then the product")},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
    }
    if n_launch:
        avg_ms = k_ms / n_launch
        if ROOFLINE_KERNEL["bound"] == "alu":
            # the hook counts 16 B per coefficient per transform; a transform
            # of one limb is (N/2) log2 N butterflies
            logn = int(np.log2(ctx.N))
            bfly = k_bytes / n_launch / 16.0 / 2.0 * logn
            achieved = bfly * OPS_PER_BUTTERFLY / (avg_ms * 1e-3) / 1e12
            out["roofline"] = {"bound": "alu", "kernel": "ntt", "achieved": achieved, "peak": INT32_PEAK_TOPS,
                               "unit": "TOPS (int32)", "frac": achieved / INT32_PEAK_TOPS,
                               "traffic": NTT_TRAFFIC_BYTES_PER_LAUNCH, "launches": n_launch,
                               "avg_launch_ms": avg_ms, "butterflies_per_launch": bfly,
                               "ops_per_butterfly": OPS_PER_BUTTERFLY,
                               "hbm_view_GBps": k_bytes / n_launch / (avg_ms * 1e-3) / 1e9,
                               "timed_steps": args.steps, "ms_per_step_with_events": hooked_ms}
        else:
            achieved = k_bytes / n_launch / (avg_ms * 1e-3) / 1e9
            out["roofline"] = {"bound": ROOFLINE_KERNEL["bound"], "kernel": ROOFLINE_KERNEL["class"],
                               "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                               "launches": n_launch, "avg_launch_ms": avg_ms,
                               "bytes_per_launch": k_bytes / n_launch,
                               "timed_steps": args.steps, "ms_per_step_with_events": hooked_ms}
    out["service_ms"] = service_time(s, args.d1, args.steps)
    if tuned is not None:
        out["autotune"] = tuned
    if args.graph:
        log("graph form ...")
        out["graph"] = graph_form(s, args.d1, args.steps)
    fused = args.route == "hoisted" and ctx.get_tune("ksmac") > 0
    out["roofline_ks"] = hook_roofline(
        s, args.d1, "ks_inner",
        ("key-switch inner product (k_ks_inner, k_ks_inner_lds, k_ks_inner_sum_lds)" if ctx.get_tune("ks_lds")
         else "key-switch inner product (k_ks_inner, k_ks_inner_sum)") +
        ("; the baby steps' key inner products run inside the MAC" if fused else ""))
    out["roofline_mac"] = hook_roofline(
        s, args.d1, "mac", "plaintext-diagonal MAC with the baby steps' key inner products (k_bsgs_ksmac)" if fused
        else "plaintext-diagonal MAC (k_bsgs_mac3)")
    if args.breakdown:
        ev3 = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev3[0].record(stream)
        matvec(s)
        ev3[1].record(stream)
        ctx.chebyshev_eval(s["keys"], s["score"], s["coeffs"], args.d1, out=s["cheb"])
        ev3[2].record(stream)
        torch.cuda.synchronize()
        out["phase_ms"] = {"matvec": ev3[0].elapsed_time(ev3[1]), "chebyshev": ev3[1].elapsed_time(ev3[2])}
        bd = {}
        for cls in ctx.KERNEL_CLASSES:
            ctx.prof_begin(cls)
            step(s, args.d1)
            n, ms, b = ctx.prof_end()
            bd[cls] = {"launches": n, "ms_per_step": ms, "GB/s": (b / (ms * 1e-3) / 1e9) if ms else None}
        out["kernel_breakdown"] = bd
    out["checks"] = check(s)
    if args.batch:
        log(f"batched form: {args.batch} queries per batch ...")
        out["batched"] = batched(s, args.batch, max(2, min(args.steps, 5)), 1, args.d1)
    if args.serve:
        log(f"served form: {args.serve:g} s per arrival rate ...")
        out["served"] = served(s, args.serve, args.d1)
    if args.rotq:
        log(f"rotation-table route vs BSGS: {args.rotq} templates ...")
        out["rotq_vs_bsgs"] = rotq_vs_bsgs(s, args.rotq, args.d1)
    if args.edb:
        log("encrypted database ...")
        out["encrypted_db"] = encrypted_db(s, args.d1)
    if args.dg:
        log("diagonal method ...")
        out["diagonal_method"] = diagonal_method(s, args.d1)
    if args.b1:
        log(f"B = 1 layout: {args.b1} templates ...")
        out["layout_b1"] = layout_b1(s, args.b1, args.d1)
    if args.mix:
        log(f"mixed batches: {args.mix} ...")
        out["mixed_batches"] = mixed_batches(s, args.mix, args.d1)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on one query ...")
        out["cpu_baseline"] = cpu_baseline(s, args.d1, one_thread_query=args.cpu_one_thread_query)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
