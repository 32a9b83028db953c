"""The served form: a request loop with continuous batching over the batched
calls.  Every request's result is bit-identical to the same request run
alone through the one-query calls, whatever batch it landed in, and the
plain one-at-a-time loop gives the same words.

Ring N = 2^12 with the paper-scale modulus chain, 128-d templates, two
databases (64 and 40 templates), n1 = 8, n2 = 16; eleven requests, half
verification and half identification, arriving in two bursts into a pool
of 4 slots (ragged batches).
"""
import numpy as np
import pytest

from paper_2604_00546_amd import synth

pytestmark = pytest.mark.gpu

ELL, N1, NR = 128, 8, 11
ROTS = list(range(1, N1)) + [N1 * j for j in range(1, ELL // N1)]


@pytest.fixture(scope="module")
def S():
    from paper_2604_00546_amd import fr, serve
    g = fr.Context(**fr.deep_small_params())
    keys = g.keygen(synth.int_seed(5, synth.SUB_KEYS), ROTS)
    wl = synth.make_workload(5, 64, ELL)
    db_id = g.db_load(wl.templates, ELL, 16, N1, g.L, 2.0 ** 40)
    db_ver = g.db_load(wl.templates[:40], ELL, 16, N1, g.L, 2.0 ** 40)
    Q = synth.query_batch(5, NR, ELL)
    kinds = synth.rng(5, synth.SUB_KIND).integers(0, 2, size=NR)
    reqs = []
    for i in range(NR):
        ct = g.encrypt(keys, g.encode(synth.replicate_query(Q[i], g.N // 2), g.L, 2.0 ** 40),
                       synth.int_seed(5, synth.SUB_ENC, i))
        verify = bool(kinds[i])
        reqs.append(serve.Request(i, 0.0 if i < 7 else 0.05, "verify" if verify else "identify", ct,
                                  db_ver if verify else db_id, 0))
    coeffs = fr.cheb_step_coeffs(63, 0.3)
    return dict(fr=fr, serve=serve, g=g, keys=keys, wl=wl, Q=Q, reqs=reqs, coeffs=coeffs)


def _alone(S, r):
    g, keys = S["g"], S["keys"]
    baby = [r.query] + g.rotate_hoisted(keys, r.query, range(1, N1))
    return g.chebyshev_eval(keys, g.bsgs_diag_matvec(keys, baby, r.db, r.group), S["coeffs"], 8)


def test_served_results_equal_alone(S):
    g, serve = S["g"], S["serve"]
    srv = serve.Server(g, S["keys"], S["coeffs"], 8, N1, slots=4, keep_results=True)
    stats = srv.run(S["reqs"])
    assert stats["requests"] == NR
    assert max(srv.batches) <= 4 and sum(srv.batches) == NR and len(srv.batches) >= 3
    # the first burst fills both lanes: a batch was launched while another ran
    assert stats["overlapped_batches"] >= 1 and {r.lane for r in S["reqs"]} == {0, 1}
    for r in S["reqs"]:
        assert r.done >= r.admitted >= r.arrival
        a = _alone(S, r)
        assert (r.result.level, r.result.scale) == (a.level, a.scale)
        assert np.array_equal(g.ct_export(r.result), g.ct_export(a)), f"request {r.rid}"
    # the plain loop over the same trace
    plain_res = {}
    for r in S["reqs"]:
        plain_res[r.rid] = r.result
    serve.plain(g, S["keys"], S["coeffs"], 8, N1, S["reqs"], keep_results=True)
    for r in S["reqs"]:
        assert np.array_equal(g.ct_export(r.result), g.ct_export(plain_res[r.rid]))


def test_served_thresholds(S):
    g, wl = S["g"], S["wl"]
    r = S["reqs"][0]
    y = g.decrypt_decode(S["keys"], _alone(S, r))
    K = 40 if r.kind == "verify" else 64
    exact = wl.templates[:K].astype(np.float64) @ S["Q"][0].astype(np.float64)
    want = np.polynomial.chebyshev.chebval(exact, S["coeffs"])
    assert np.max(np.abs(y[:K] - want)) <= 2 ** -12


def test_served_hoisted_equal_alone(S):
    """With extended databases the loop runs the hoisted product: every
    request's result equals the same request through the one-query hoisted
    call, and the plain loop gives the same words."""
    g, serve, keys = S["g"], S["serve"], S["keys"]
    dbs = {}
    reqs = []
    for r in S["reqs"]:
        if id(r.db) not in dbs:
            dbs[id(r.db)] = g.db_import(np.stack([[r.db.export(0, d) for d in range(ELL)]]), 1, ELL, 16, N1, g.L,
                                        2.0 ** 40).extend()
        reqs.append(serve.Request(r.rid, r.arrival, r.kind, r.query, dbs[id(r.db)], 0))
    srv = serve.Server(g, keys, S["coeffs"], 8, N1, slots=4, keep_results=True)
    srv.run(reqs)
    assert sum(srv.batches) == NR and len(srv.batches) >= 3
    first = {}
    for r in reqs:
        a = g.chebyshev_eval(keys, g.bsgs_matvec_hoisted(keys, r.query, r.db, 0), S["coeffs"], 8)
        assert (r.result.level, r.result.scale) == (a.level, a.scale)
        assert np.array_equal(g.ct_export(r.result), g.ct_export(a)), f"request {r.rid}"
        first[r.rid] = r.result
    serve.plain(g, keys, S["coeffs"], 8, N1, reqs, keep_results=True)
    for r in reqs:
        assert np.array_equal(g.ct_export(r.result), g.ct_export(first[r.rid]))


def test_slot_count_rule(S):
    n = S["serve"].slot_count(S["g"])
    assert 2 <= n <= 64


def test_admission_by_scratch_budget(S):
    """Lanes whose scratch budget holds one request but not two: batches
    that meet FR_ENOMEM are split, and every result still equals the same
    request run alone."""
    g, serve, keys = S["g"], S["serve"], S["keys"]
    from paper_2604_00546_amd import fr
    probe = fr.Context(**fr.deep_small_params())
    r0 = S["reqs"][0]
    probe.chebyshev_eval(keys, probe.bsgs_matvec_hoisted(keys, r0.query, _extended(S, r0.db), 0), S["coeffs"], 8)
    one = probe.scratch_info()[1]
    reqs = [serve.Request(r.rid, 0.0, r.kind, r.query, _extended(S, r.db), 0) for r in S["reqs"][:6]]
    srv = serve.Server(g, keys, S["coeffs"], 8, N1, slots=6, lanes=2, keep_results=True,
                       hbm_budget=int(2 * 1.4 * one))
    stats = srv.run(reqs)
    assert stats["split_batches"] >= 1 and max(srv.batches) <= 2
    for r in reqs:
        a = g.chebyshev_eval(keys, g.bsgs_matvec_hoisted(keys, r.query, r.db, 0), S["coeffs"], 8)
        assert np.array_equal(g.ct_export(r.result), g.ct_export(a)), f"request {r.rid}"


_EXT = {}


def _extended(S, db):
    """An extended copy of db (the hoisted product's databases)."""
    g = S["g"]
    if id(db) not in _EXT:
        _EXT[id(db)] = g.db_import(np.stack([[db.export(0, d) for d in range(ELL)]]), 1, ELL, 16, N1, g.L,
                                   2.0 ** 40).extend()
    return _EXT[id(db)]
