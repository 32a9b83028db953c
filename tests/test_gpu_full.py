"""GPU tests at the paper-scale parameters (N = 2^16, Q = 60 + 14 x 40 bits,
P = 5 x 60 bits, dnum = 3), in the launch configuration bench.py times.

* The whole hot path of one query -- 31 hoisted baby-step rotations, the
  BSGS matrix-vector product over one group of 512 diagonals, the degree-63
  Chebyshev threshold -- is compared bit-exactly with the oracle on the
  2^12-template database (same keys, seeds and integer plaintexts).
* The 2^15-template identification workload with the device's own diagonal
  encoder: every decrypted score within 2^-20 of the FP64 inner product,
  every Chebyshev output within 2^-12 of the FP64 polynomial, and the set of
  identified templates equal to the planted set.
"""
import numpy as np
import pytest

from paper_2604_00546_amd import synth

pytestmark = pytest.mark.gpu

ELL, N1 = 512, 32


def _oparams(p):
    return dict(logN=p["log_n"], q0_bits=p["q0_bits"], n_mid=p["n_mid"], mid_bits=p["mid_bits"],
                n_special=p["n_special"], special_bits=p["special_bits"], dnum=p["dnum"])


@pytest.fixture(scope="module")
def F():
    from paper_2604_00546_amd import fr
    return fr


@pytest.fixture(scope="module")
def gctx(F):
    return F.Context(**F.paper_params())


def _same(g, gct, oct_):
    a, b = g.ct_export(gct), oct_.coeffs()
    assert (gct.level, gct.scale) == (oct_.level, oct_.scale)
    bad = np.argwhere(a != b)
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:3].tolist()}"


@pytest.fixture(scope="module")
def config2(F, gctx, oracle_mod):
    """Oracle side of the 2^12 x 512 query, and the GPU fed the same inputs."""
    g = gctx
    o = oracle_mod.Context(**_oparams(F.paper_params()))
    assert g.moduli == o.moduli
    rots = F.bsgs_rotation_set(ELL, N1)
    seed = synth.int_seed(2, synth.SUB_KEYS)
    kg, ko = g.keygen(seed, rots), o.keygen(seed, rots)
    wl = synth.make_workload(2, 2 ** 12, ELL)
    B = g.N // 2 // ELL
    odb = o.db_build(wl.templates, wl.K, ELL, B, N1, o.L, 2.0 ** 40)
    gdb = g.db_import(odb.export_all(), odb.G, ELL, B, N1, g.L, 2.0 ** 40)
    opt = o.encode(synth.replicate_query(wl.query, g.N // 2), o.L, 2.0 ** 40)
    es = synth.int_seed(2, synth.SUB_ENC)
    gq = g.encrypt(kg, g.pt_import(opt.coeffs(), g.L, 2.0 ** 40), es)
    oq = o.encrypt(ko, opt, es)
    return dict(o=o, kg=kg, ko=ko, wl=wl, odb=odb, gdb=gdb, gq=gq, oq=oq, B=B)


@pytest.mark.timeout(900)
def test_full_hot_path_bitexact(F, gctx, config2):
    g, c = gctx, config2
    o, kg, ko = c["o"], c["kg"], c["ko"]
    _same(g, c["gq"], c["oq"])
    gb = [c["gq"]] + g.rotate_hoisted(kg, c["gq"], range(1, N1))
    ob = [c["oq"]] + o.rotate_hoisted(ko, c["oq"], range(1, N1))
    for i in (1, 2, 17, 31):
        _same(g, gb[i], ob[i])
    gs = g.bsgs_diag_matvec(kg, gb, c["gdb"], 0)
    os_ = o.bsgs_matvec(ko, ob, c["odb"], 0)
    _same(g, gs, os_)
    coeffs = F.cheb_step_coeffs(63, 0.3)
    for d1 in (2, 8):
        gy = g.chebyshev_eval(kg, gs, coeffs, d1)
        oy = o.chebyshev(ko, os_, coeffs, d1)
        _same(g, gy, oy)
    exact = c["wl"].exact_scores()
    dec = g.decrypt_decode(kg, gs)
    assert np.max(np.abs(dec[: len(exact)] - exact)) <= 2 ** -20
    assert np.max(np.abs(dec[len(exact):])) <= 2 ** -20


@pytest.mark.timeout(900)
def test_full_hoisted_bitexact(F, gctx, config2):
    """The product with the baby steps held over Q_l U P (one ModDown per
    inner sum) at N = 2^16 over one group of 512 diagonals: the oracle's
    words, and scores within 2^-20."""
    g, c = gctx, config2
    gdb = c["gdb"].extend()
    gs = g.bsgs_matvec_hoisted(c["kg"], c["gq"], gdb, 0)
    os_ = c["o"].bsgs_matvec_hoisted(c["ko"], c["oq"], c["odb"], 0)
    _same(g, gs, os_)
    exact = c["wl"].exact_scores()
    dec = g.decrypt_decode(c["kg"], gs)
    assert np.max(np.abs(dec[: len(exact)] - exact)) <= 2 ** -20
    assert np.max(np.abs(dec[len(exact):])) <= 2 ** -20


@pytest.mark.timeout(900)
def test_tuning_knobs_keep_the_words(F, gctx, config2):
    """The tuning knobs choose launches only: with every knob away from its
    default (each NTT pass always / never in its 4-word form, the ModUp
    always / never merged over the digits, the Chebyshev groups in recorded
    or critical-first order, the baby steps written by their own launch or
    formed inside the MAC, the giant steps' keys staged in LDS or loaded
    per lane) the hoisted product and the Chebyshev step at
    d1 = 8 give the oracle's words."""
    g, c = gctx, config2
    gdb = c["gdb"].extend()
    os_ = c["o"].bsgs_matvec_hoisted(c["ko"], c["oq"], c["odb"], 0)
    coeffs = F.cheb_step_coeffs(63, 0.3)
    oy = c["o"].chebyshev(c["ko"], os_, coeffs, 8)
    ntt = ("ntt_fwd_cols4", "ntt_fwd_rows4", "ntt_inv_rows4", "ntt_inv_cols4")
    settings = [dict({k: 0 for k in ntt}, modup_merge=48, cheb_sched=0, ksmac=0, ks_lds=0),
                dict({k: 1 << 20 for k in ntt}, modup_merge=0, cheb_sched=1, ksmac=2, ks_lds=1)]
    start = g.tune_state()
    try:
        for kn in settings:
            for k, v in kn.items():
                g.set_tune(k, v)
            gs = g.bsgs_matvec_hoisted(c["kg"], c["gq"], gdb, 0)
            _same(g, gs, os_)
            _same(g, g.chebyshev_eval(c["kg"], gs, coeffs, 8), oy)
    finally:
        for k, v in start.items():
            g.set_tune(k, v)


def test_full_size_encoder_within_one(F, gctx, config2):
    """Device encoder of the pre-rotated diagonals vs the oracle's, sampled diagonals."""
    g, c = gctx, config2
    gdb = g.db_load(c["wl"].templates, ELL, c["B"], N1, g.L, 2.0 ** 40)
    q0 = g.q[0]
    for d in (0, 33, 257, 511):
        a = gdb.export(0, d)[0].astype(object)
        b = c["odb"].export(0, d)[0].astype(object)
        diff = (a - b) % q0
        diff = np.where(diff > q0 // 2, diff - q0, diff)
        assert np.max(np.abs(diff)) <= 1


@pytest.mark.timeout(600)
def test_identification_2p15(F, gctx):
    g = gctx
    wl = synth.make_workload(3, 2 ** 15, ELL, planted_frac=0.01)
    rots = sorted(set(F.bsgs_rotation_set(ELL, N1)) | set(F.power_of_two_rotations(g.N)))
    keys = g.keygen(synth.int_seed(3, synth.SUB_KEYS), rots)
    B = g.N // 2 // ELL
    db = g.db_load(wl.templates, ELL, B, N1, g.L, 2.0 ** 40)
    assert db.G == 1
    q = g.encrypt(keys, g.encode(synth.replicate_query(wl.query, g.N // 2), g.L, 2.0 ** 40),
                  synth.int_seed(3, synth.SUB_ENC))
    baby = [q] + g.rotate_hoisted(keys, q, range(1, N1))
    S = g.bsgs_diag_matvec(keys, baby, db, 0)
    exact = wl.exact_scores()
    dec = g.decrypt_decode(keys, S)
    assert np.max(np.abs(dec - exact)) <= 2 ** -20
    coeffs = F.cheb_step_coeffs(63, 0.3)
    for d1 in (2, 8):
        Y = g.chebyshev_eval(keys, S, coeffs, d1)
        y = g.decrypt_decode(keys, Y)
        assert np.max(np.abs(y - np.polynomial.chebyshev.chebval(exact, coeffs))) <= 2 ** -12
        assert np.array_equal(np.nonzero(y >= 0.5)[0], wl.planted)
    # the hoisted product (baby steps over Q_l U P) scores the same
    H = g.bsgs_matvec_hoisted(keys, q, db.extend(), 0)
    assert np.max(np.abs(g.decrypt_decode(keys, H) - exact)) <= 2 ** -20
    YH = g.decrypt_decode(keys, g.chebyshev_eval(keys, H, coeffs, 8))
    assert np.array_equal(np.nonzero(YH >= 0.5)[0], wl.planted)
    # membership: the sum of the polynomial over all 2^15 slots in every slot
    # (328 planted matches plus the ripple of the degree-63 step elsewhere)
    count = g.decrypt_decode(keys, g.membership_aggregate(keys, [Y]))
    want = np.polynomial.chebyshev.chebval(exact, coeffs).sum()
    assert np.max(np.abs(count - want)) < 0.5


@pytest.mark.timeout(600)
def test_batched_path_equals_alone_2p15(F, gctx):
    """Three queries through the batched hot path at N = 2^16 against the
    2^15-template database: each query's baby steps, score and Chebyshev
    ciphertexts are the words the one-query path gives for it."""
    g = gctx
    wl = synth.make_workload(3, 2 ** 15, ELL, planted_frac=0.01)
    rots = F.bsgs_rotation_set(ELL, N1)
    keys = g.keygen(synth.int_seed(3, synth.SUB_KEYS), rots)
    db = g.db_load(wl.templates, ELL, g.N // 2 // ELL, N1, g.L, 2.0 ** 40)
    Q = np.vstack([wl.query[None, :], synth.query_batch(3, 2, ELL)])
    qs = [g.encrypt(keys, g.encode(synth.replicate_query(Q[q], g.N // 2), g.L, 2.0 ** 40),
                    synth.int_seed(3, synth.SUB_ENC, q)) for q in range(3)]
    coeffs = F.cheb_step_coeffs(63, 0.3)
    rows = g.rotate_hoisted_batch(keys, qs, range(1, N1))
    babies = [[qs[q]] + rows[q] for q in range(3)]
    S = g.bsgs_diag_matvec_batch(keys, babies, db, 0)
    Y = g.chebyshev_eval_batch(keys, S, coeffs, 8)
    for q in range(3):
        alone = [qs[q]] + g.rotate_hoisted(keys, qs[q], range(1, N1))
        for i in (1, 16, 31):
            assert np.array_equal(g.ct_export(alone[i]), g.ct_export(babies[q][i]))
        s1 = g.bsgs_diag_matvec(keys, alone, db, 0)
        assert np.array_equal(g.ct_export(s1), g.ct_export(S[q]))
        y1 = g.chebyshev_eval(keys, s1, coeffs, 8)
        assert (y1.level, y1.scale) == (Y[q].level, Y[q].scale)
        assert np.array_equal(g.ct_export(y1), g.ct_export(Y[q]))
        exact = wl.templates.astype(np.float64) @ Q[q].astype(np.float64)
        assert np.max(np.abs(g.decrypt_decode(keys, S[q]) - exact)) <= 2 ** -20
    y0 = g.decrypt_decode(keys, Y[0])
    assert np.array_equal(np.nonzero(y0 >= 0.5)[0], wl.planted)
    # hoisted product, batched and alone
    db.extend()
    HB = g.bsgs_matvec_hoisted_batch(keys, qs, db, 0)
    for q in range(3):
        h1 = g.bsgs_matvec_hoisted(keys, qs[q], db, 0)
        assert (h1.level, h1.scale) == (HB[q].level, HB[q].scale)
        assert np.array_equal(g.ct_export(h1), g.ct_export(HB[q]))
        exact = wl.templates.astype(np.float64) @ Q[q].astype(np.float64)
        assert np.max(np.abs(g.decrypt_decode(keys, HB[q]) - exact)) <= 2 ** -20
