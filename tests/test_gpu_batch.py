"""GPU parity of the batched forms (several queries sharing keys and
diagonals): every query's result is bit-identical to the result of the same
query run alone, and to the oracle.

Ring N = 2^12 with the paper-scale modulus chain (60 + 14 x 40 bits, P = 5 x
60 bits, dnum = 3), 64 templates x 128-d, B = 16 blocks per plaintext,
n1 = 8, n2 = 16.  Ten queries: more than one chunk of eight, with a ragged
second chunk.
"""
import numpy as np
import pytest

from paper_2604_00546_amd import synth

pytestmark = pytest.mark.gpu

ELL, N1, NQ = 128, 8, 10
ROTS = list(range(1, N1)) + [N1 * j for j in range(1, ELL // N1)]


def _oparams(p):
    return dict(logN=p["log_n"], q0_bits=p["q0_bits"], n_mid=p["n_mid"], mid_bits=p["mid_bits"],
                n_special=p["n_special"], special_bits=p["special_bits"], dnum=p["dnum"])


def _same_ct(g, a, b):
    assert (a.level, a.scale) == (b.level, b.scale)
    x, y = g.ct_export(a), g.ct_export(b)
    bad = np.argwhere(x != y)
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:3].tolist()}"


def _same_oracle(g, gct, oct_):
    assert (gct.level, gct.scale) == (oct_.level, oct_.scale)
    bad = np.argwhere(g.ct_export(gct) != oct_.coeffs())
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:3].tolist()}"


@pytest.fixture(scope="module")
def B(oracle_mod):
    from paper_2604_00546_amd import fr
    p = fr.deep_small_params()
    g, o = fr.Context(**p), oracle_mod.Context(**_oparams(p))
    seed = synth.int_seed(4, synth.SUB_KEYS)
    kg, ko = g.keygen(seed, ROTS), o.keygen(seed, ROTS)
    wl = synth.make_workload(4, 64, ELL)
    odb = o.db_build(wl.templates, wl.K, ELL, 16, N1, o.L, 2.0 ** 40)
    gdb = g.db_import(odb.export_all(), odb.G, ELL, 16, N1, g.L, 2.0 ** 40)
    Q = synth.query_batch(4, NQ, ELL)
    gq, oq = [], []
    for q in range(NQ):
        opt = o.encode(synth.replicate_query(Q[q], g.N // 2), o.L, 2.0 ** 40)
        es = synth.int_seed(4, synth.SUB_ENC, q)
        gq.append(g.encrypt(kg, g.pt_import(opt.coeffs(), g.L, 2.0 ** 40), es))
        oq.append(o.encrypt(ko, opt, es))
    return dict(fr=fr, g=g, o=o, kg=kg, ko=ko, wl=wl, odb=odb, gdb=gdb, Q=Q, gq=gq, oq=oq)


@pytest.fixture(scope="module")
def babies(B):
    g = B["g"]
    rows = g.rotate_hoisted_batch(B["kg"], B["gq"], range(1, N1))
    return [[B["gq"][q]] + rows[q] for q in range(NQ)]


def test_rotate_batch_equals_alone_and_oracle(B, babies):
    g, o = B["g"], B["o"]
    for q in (0, 7, 8, 9):
        alone = g.rotate_hoisted(B["kg"], B["gq"][q], range(1, N1))
        for r in range(N1 - 1):
            _same_ct(g, babies[q][1 + r], alone[r])
    ob = o.rotate_hoisted(B["ko"], B["oq"][9], [1, 5, 7])
    for r, ot in zip([1, 5, 7], ob):
        _same_oracle(g, babies[9][r], ot)


def test_rotate_batch_identity_and_single(B):
    g = B["g"]
    rows = g.rotate_hoisted_batch(B["kg"], B["gq"][:1], [0, 3])
    _same_ct(g, rows[0][0], B["gq"][0])
    _same_ct(g, rows[0][1], g.rotate_hoisted(B["kg"], B["gq"][0], [3])[0])


@pytest.fixture(scope="module")
def scores(B, babies):
    return B["g"].bsgs_diag_matvec_batch(B["kg"], babies, B["gdb"], 0)


@pytest.fixture(scope="module")
def oracle_scores(B):
    """Oracle score ciphertexts of queries 0 and 9, from the oracle's own inputs."""
    o = B["o"]
    out = {}
    for q in (0, 9):
        ob = [B["oq"][q]] + o.rotate_hoisted(B["ko"], B["oq"][q], range(1, N1))
        out[q] = o.bsgs_matvec(B["ko"], ob, B["odb"], 0)
    return out


def test_matvec_batch_equals_alone_and_oracle(B, babies, scores, oracle_scores):
    g, wl = B["g"], B["wl"]
    for q in range(NQ):
        _same_ct(g, scores[q], g.bsgs_diag_matvec(B["kg"], babies[q], B["gdb"], 0))
    for q in (0, 9):
        _same_oracle(g, scores[q], oracle_scores[q])
    for q in range(NQ):
        exact = wl.templates.astype(np.float64) @ B["Q"][q].astype(np.float64)
        dec = g.decrypt_decode(B["kg"], scores[q])
        assert np.max(np.abs(dec[: wl.K] - exact)) <= 2 ** -20


def test_matvec_batch_mixed_databases(B, babies, scores):
    """Queries scored against two databases of different sizes in one batch
    (interleaved, so the batch reorders them by group): each result is the
    one-query result against its own database."""
    g, o = B["g"], B["o"]
    wl2 = synth.make_workload(4, 40, ELL, extra=1)
    odb2 = o.db_build(wl2.templates, wl2.K, ELL, 16, N1, o.L, 2.0 ** 40)
    gdb2 = g.db_import(odb2.export_all(), odb2.G, ELL, 16, N1, g.L, 2.0 ** 40)
    dbs = [B["gdb"] if q % 2 == 0 else gdb2 for q in range(NQ)]
    mixed = g.bsgs_diag_matvec_batch(B["kg"], babies, dbs, [0] * NQ)
    for q in range(NQ):
        if q % 2 == 0:
            _same_ct(g, mixed[q], scores[q])
        else:
            _same_ct(g, mixed[q], g.bsgs_diag_matvec(B["kg"], babies[q], gdb2, 0))
    ob = [B["oq"][9]] + o.rotate_hoisted(B["ko"], B["oq"][9], range(1, N1))
    _same_oracle(g, mixed[9], o.bsgs_matvec(B["ko"], ob, odb2, 0))


def test_matvec_batch_single_query(B, babies, scores):
    g = B["g"]
    one = g.bsgs_diag_matvec_batch(B["kg"], babies[3:4], B["gdb"], 0)
    _same_ct(g, one[0], scores[3])


@pytest.mark.parametrize("d1", [2, 8])
def test_chebyshev_batch_equals_alone_and_oracle(B, scores, oracle_scores, d1):
    g, o = B["g"], B["o"]
    c = B["fr"].cheb_step_coeffs(63, 0.3)
    ys = g.chebyshev_eval_batch(B["kg"], scores, c, d1)
    for q in range(NQ):
        _same_ct(g, ys[q], g.chebyshev_eval(B["kg"], scores[q], c, d1))
    _same_oracle(g, ys[9], o.chebyshev(B["ko"], oracle_scores[9], c, d1))
    wl = B["wl"]
    for q in (0, 9):
        exact = wl.templates.astype(np.float64) @ B["Q"][q].astype(np.float64)
        y = g.decrypt_decode(B["kg"], ys[q])[: wl.K]
        assert np.max(np.abs(y - np.polynomial.chebyshev.chebval(exact, c))) <= 2 ** -12


def test_batch_rejects_mixed_levels(B, scores):
    g = B["g"]
    low = g.rescale(scores[0])
    with pytest.raises(B["fr"].FrError):
        g.chebyshev_eval_batch(B["kg"], [scores[1], low], B["fr"].cheb_step_coeffs(63, 0.3), 8)


def test_rotq_table_route(B, babies):
    """The full rotation table of Alg. bsgs-precomp: every baby step rotated
    by every giant amount (one batched hoisted call), then each group is a
    pure diagonal MAC over ell rotations and plain (not pre-rotated)
    diagonals.  Bit-exact against the oracle's same composition, scores
    within 2^-20."""
    g, o, wl = B["g"], B["o"], B["wl"]
    giant = [N1 * j for j in range(1, ELL // N1)]
    rows = g.rotate_hoisted_batch(B["kg"], babies[0], giant)   # rows[i][j-1] = Rot_{j n1}(baby_i)
    table = [babies[0][i] if j == 0 else rows[i][j - 1] for j in range(ELL // N1) for i in range(N1)]
    odm = o.db_build(wl.templates, wl.K, ELL, 16, ELL, o.L, 2.0 ** 40)
    gdm = g.db_import(odm.export_all(), odm.G, ELL, 16, ELL, g.L, 2.0 ** 40)
    gs = g.bsgs_diag_matvec(B["kg"], table, gdm, 0)
    ob = [B["oq"][0]] + o.rotate_hoisted(B["ko"], B["oq"][0], range(1, N1))
    orows = [o.rotate_hoisted(B["ko"], ob[i], giant) for i in range(N1)]
    otable = [ob[i] if j == 0 else orows[i][j - 1] for j in range(ELL // N1) for i in range(N1)]
    _same_oracle(g, gs, o.bsgs_matvec(B["ko"], otable, odm, 0))
    exact = wl.templates.astype(np.float64) @ B["Q"][0].astype(np.float64)
    assert np.max(np.abs(g.decrypt_decode(B["kg"], gs)[: wl.K] - exact)) <= 2 ** -20


def test_encrypted_database_route(B, babies):
    """Encrypted diagonals (the paper's setting): the group score is
    Rescale(Relin(sum_d rot_d(q) (x) Enc(diag_d))) with one relinearisation
    per group, over the full rotation table.  Bit-exact against the oracle,
    scores within 2^-20."""
    g, o, wl = B["g"], B["o"], B["wl"]
    giant = [N1 * j for j in range(1, ELL // N1)]
    rows = g.rotate_hoisted_batch(B["kg"], babies[0], giant)
    table = [babies[0][i] if j == 0 else rows[i][j - 1] for j in range(ELL // N1) for i in range(N1)]
    odm = o.db_build(wl.templates, wl.K, ELL, 16, ELL, o.L, 2.0 ** 40)
    gdiag, odiag = [], []
    for d in range(ELL):
        coeffs = odm.export(0, d)
        es = synth.int_seed(4, synth.SUB_ENC, 1000 + d)
        gdiag.append(g.encrypt(B["kg"], g.pt_import(coeffs, g.L, 2.0 ** 40), es))
        odiag.append(o.encrypt(B["ko"], o.pt_import(coeffs, o.L, 2.0 ** 40), es))
    gs = g.tensor_sum_relin_rescale(B["kg"], table, gdiag)
    ob = [B["oq"][0]] + o.rotate_hoisted(B["ko"], B["oq"][0], range(1, N1))
    orows = [o.rotate_hoisted(B["ko"], ob[i], giant) for i in range(N1)]
    otable = [ob[i] if j == 0 else orows[i][j - 1] for j in range(ELL // N1) for i in range(N1)]
    _same_oracle(g, gs, o.tensor_sum_relin_rescale(B["ko"], otable, odiag))
    exact = wl.templates.astype(np.float64) @ B["Q"][0].astype(np.float64)
    assert np.max(np.abs(g.decrypt_decode(B["kg"], gs)[: wl.K] - exact)) <= 2 ** -20
