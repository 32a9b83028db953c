"""GPU parity of the BSGS product with the baby steps' ModDown hoisted past
the inner sums (baby steps held over Q_l U P; the inner sums' first
polynomials rotated and summed before one ModDown, one ModDown per second
polynomial).

Every score ciphertext is compared bit-exactly with the oracle's
or_bsgs_matvec_hoisted on the same keys, encryption seeds and integer
plaintexts, and decrypted scores are held to 2^-20 of the FP64 inner
products.  Rings N = 2^12: the paper-scale modulus chain (five special
primes, digits of five limbs) and the small chain (one special prime, one
limb per digit) with ragged and degenerate shapes.
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
    bad = np.argwhere(g.ct_export(a) != g.ct_export(b))
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:3].tolist()}"


def _same_oracle(g, gct, oct_):
    assert (gct.level, gct.scale) == (oct_.level, oct_.scale)
    bad = np.argwhere(g.ct_export(gct) != oct_.coeffs())
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:3].tolist()}"


@pytest.fixture(scope="module")
def H(oracle_mod):
    """Paper chain at N = 2^12; a one-group and a two-group database (the
    latter extended to the special primes on both sides), ten queries."""
    from paper_2604_00546_amd import fr
    p = fr.deep_small_params()
    g, o = fr.Context(**p), oracle_mod.Context(**_oparams(p))
    seed = synth.int_seed(5, synth.SUB_KEYS)
    kg, ko = g.keygen(seed, ROTS), o.keygen(seed, ROTS)
    wl = synth.make_workload(5, 3000, ELL)
    odb = o.db_build(wl.templates, wl.K, ELL, 16, N1, o.L, 2.0 ** 40)
    gdb = g.db_import(odb.export_all(), odb.G, ELL, 16, N1, g.L, 2.0 ** 40)
    assert gdb.G == 2
    before = gdb.export(1, 77)
    gdb.extend()
    assert np.array_equal(gdb.export(1, 77), before)
    gdb.extend()  # idempotent
    Q = synth.query_batch(5, NQ, ELL)
    gq, oq = [], []
    for q in range(NQ):
        opt = o.encode(synth.replicate_query(Q[q], g.N // 2), o.L, 2.0 ** 40)
        es = synth.int_seed(5, synth.SUB_ENC, q)
        gq.append(g.encrypt(kg, g.pt_import(opt.coeffs(), g.L, 2.0 ** 40), es))
        oq.append(o.encrypt(ko, opt, es))
    return dict(fr=fr, g=g, o=o, kg=kg, ko=ko, wl=wl, odb=odb, gdb=gdb, Q=Q, gq=gq, oq=oq)


@pytest.mark.parametrize("q,group,ksmac", [(0, 0, 1), (3, 1, 1), (3, 1, 0)])
def test_hoisted_bitexact_paper_chain(H, q, group, ksmac):
    """ksmac 1: baby steps formed inside the MAC; 0: written by the key
    inner product launch and read back."""
    g, o = H["g"], H["o"]
    keep = g.get_tune("ksmac")
    g.set_tune("ksmac", ksmac)
    try:
        gs = g.bsgs_matvec_hoisted(H["kg"], H["gq"][q], H["gdb"], group)
    finally:
        g.set_tune("ksmac", keep)
    os_ = o.bsgs_matvec_hoisted(H["ko"], H["oq"][q], H["odb"], group)
    _same_oracle(g, gs, os_)
    dec = g.decrypt_decode(H["kg"], gs)
    T = H["wl"].templates[group * 16 * ELL: (group + 1) * 16 * ELL]
    exact = T.astype(np.float64) @ H["Q"][q].astype(np.float64)
    assert np.max(np.abs(dec[: len(exact)] - exact)) <= 2 ** -20


@pytest.mark.parametrize("ksmac", [1, 2])
def test_hoisted_batch_equals_alone_and_oracle(H, ksmac):
    """Ten queries (a full chunk of eight and a ragged chunk of two) over both
    groups of one database, interleaved: each output is the one-query word
    set; two are checked against the oracle.  ksmac 2: the chunks' baby
    steps formed inside the MAC too (1: only one-query chunks)."""
    g, o = H["g"], H["o"]
    groups = [q % 2 for q in range(NQ)]
    keep = g.get_tune("ksmac")
    g.set_tune("ksmac", ksmac)
    try:
        outs = g.bsgs_matvec_hoisted_batch(H["kg"], H["gq"], H["gdb"], groups)
    finally:
        g.set_tune("ksmac", keep)
    for q in range(NQ):
        _same_ct(g, outs[q], g.bsgs_matvec_hoisted(H["kg"], H["gq"][q], H["gdb"], groups[q]))
    for q in (4, 9):
        _same_oracle(g, outs[q], o.bsgs_matvec_hoisted(H["ko"], H["oq"][q], H["odb"], groups[q]))


def test_hoisted_close_to_single_hoisted(H):
    """The same product through rotate_hoisted + bsgs_diag_matvec: other
    rounding, so other words, but the same scores to well inside 2^-20."""
    g = H["g"]
    a = g.bsgs_matvec_hoisted(H["kg"], H["gq"][1], H["gdb"], 0)
    baby = [H["gq"][1]] + g.rotate_hoisted(H["kg"], H["gq"][1], range(1, N1))
    b = g.bsgs_diag_matvec(H["kg"], baby, H["gdb"], 0)
    assert (a.level, a.scale) == (b.level, b.scale)
    da, db = g.decrypt_decode(H["kg"], a), g.decrypt_decode(H["kg"], b)
    assert np.max(np.abs(da - db)) <= 2 ** -22


def test_hoisted_rejects_bad_inputs(H):
    g, F = H["g"], H["fr"]
    plain = g.db_import(H["odb"].export_all(), H["odb"].G, ELL, 16, N1, g.L, 2.0 ** 40)
    with pytest.raises(F.FrError, match="not extended"):
        g.bsgs_matvec_hoisted(H["kg"], H["gq"][0], plain, 0)
    low = g.rescale(H["gq"][0])
    with pytest.raises(F.FrError, match="level"):
        g.bsgs_matvec_hoisted(H["kg"], low, H["gdb"], 0)
    with pytest.raises(F.FrError, match="group"):
        g.bsgs_matvec_hoisted(H["kg"], H["gq"][0], H["gdb"], 2)


# --------------------------------------------------------------------------
# ragged and degenerate shapes on the small chain (one special prime)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("K,ell,B,n1,group", [
    (300, 100, 20, 8, 0),    # n2 = 13: partial giant-step tile, diagonals past ell
    (1000, 128, 4, 40, 1),   # n1 > 32: baby steps in two MAC chunks; second of two groups
    (64, 64, 32, 64, 0),     # the diagonal method: n2 = 1, no giant step
    (20, 128, 1, 8, 0),      # B = 1: one block per plaintext
    (200, 96, 8, 7, 0),      # odd n1: an odd number of baby steps per MAC launch
    (500, 128, 4, 33, 0),    # n1 = 33: MAC chunks of 32 and 1 baby steps
])
def test_hoisted_ragged_shapes_bitexact(oracle_mod, K, ell, B, n1, group):
    from paper_2604_00546_amd import fr
    p = fr.small_params()
    g, o = fr.Context(**p), oracle_mod.Context(**_oparams(p))
    rots = fr.bsgs_rotation_set(ell, n1)
    seed = synth.int_seed(1, synth.SUB_KEYS, ell + n1)
    kg, ko = g.keygen(seed, rots), o.keygen(seed, rots)
    wl = synth.make_workload(1, K, ell, extra=ell + n1)
    odb = o.db_build(wl.templates, wl.K, ell, B, n1, o.L, 2.0 ** 40)
    gdb = g.db_import(odb.export_all(), odb.G, ell, B, n1, g.L, 2.0 ** 40).extend()
    opt = o.encode(synth.replicate_query(wl.query, g.N // 2), o.L, 2.0 ** 40)
    es = synth.int_seed(1, synth.SUB_ENC, ell + n1)
    gq, oq = g.encrypt(kg, g.pt_import(opt.coeffs(), g.L, 2.0 ** 40), es), o.encrypt(ko, opt, es)
    gs = g.bsgs_matvec_hoisted(kg, gq, gdb, group)
    _same_oracle(g, gs, o.bsgs_matvec_hoisted(ko, oq, odb, group))
    dec = g.decrypt_decode(kg, gs)
    exact = wl.exact_scores()
    lo, hi = group * B * ell, min(K, (group + 1) * B * ell)
    assert np.max(np.abs(dec[: hi - lo] - exact[lo:hi])) <= 2 ** -20


def test_many_digits_bitexact(oracle_mod):
    """Five digits of one limb each (dnum = 5 on a five-limb chain): the key
    inner products and the fused giant-step sum take their any-count form
    (five digits at the top level, four after the rescale).  Rotations, the
    relinearised product and the hoisted product are compared bit-exactly."""
    from paper_2604_00546_amd import fr
    p = dict(fr.small_params(), n_mid=4, dnum=5)
    g, o = fr.Context(**p), oracle_mod.Context(**_oparams(p))
    ell, n1 = 64, 8
    rots = fr.bsgs_rotation_set(ell, n1)
    seed = synth.int_seed(7, synth.SUB_KEYS)
    kg, ko = g.keygen(seed, rots), o.keygen(seed, rots)
    wl = synth.make_workload(7, 500, ell, extra=ell + n1)
    odb = o.db_build(wl.templates, wl.K, ell, 8, n1, o.L, 2.0 ** 40)
    gdb = g.db_import(odb.export_all(), odb.G, ell, 8, n1, g.L, 2.0 ** 40).extend()
    opt = o.encode(synth.replicate_query(wl.query, g.N // 2), o.L, 2.0 ** 40)
    es = synth.int_seed(7, synth.SUB_ENC)
    gq, oq = g.encrypt(kg, g.pt_import(opt.coeffs(), g.L, 2.0 ** 40), es), o.encrypt(ko, opt, es)
    for a, b in zip(g.rotate_hoisted(kg, gq, [1, 3, 8]), o.rotate_hoisted(ko, oq, [1, 3, 8])):
        _same_oracle(g, a, b)
    _same_oracle(g, g.mul_relin_rescale(kg, gq, gq), o.mul_relin_rescale(ko, oq, oq))
    gs = g.bsgs_matvec_hoisted(kg, gq, gdb, 0)
    _same_oracle(g, gs, o.bsgs_matvec_hoisted(ko, oq, odb, 0))
    dec = g.decrypt_decode(kg, gs)
    exact = wl.exact_scores()
    assert np.max(np.abs(dec[: min(wl.K, 8 * ell)] - exact[: 8 * ell])) <= 2 ** -20


def test_packed_special_primes_bitexact(oracle_mod):
    """Two 40-bit special primes: the special limbs of the keys and of the
    extended diagonals are stored packed (5 bytes per residue) as well.
    Rotations, the relinearised product and the hoisted product are compared
    bit-exactly."""
    from paper_2604_00546_amd import fr
    p = dict(fr.small_params(), n_special=2, special_bits=40)
    g, o = fr.Context(**p), oracle_mod.Context(**_oparams(p))
    ell, n1 = 64, 8
    rots = fr.bsgs_rotation_set(ell, n1)
    seed = synth.int_seed(8, synth.SUB_KEYS)
    kg, ko = g.keygen(seed, rots), o.keygen(seed, rots)
    wl = synth.make_workload(8, 400, ell, extra=ell + n1)
    odb = o.db_build(wl.templates, wl.K, ell, 8, n1, o.L, 2.0 ** 40)
    gdb = g.db_import(odb.export_all(), odb.G, ell, 8, n1, g.L, 2.0 ** 40).extend()
    opt = o.encode(synth.replicate_query(wl.query, g.N // 2), o.L, 2.0 ** 40)
    es = synth.int_seed(8, synth.SUB_ENC)
    gq, oq = g.encrypt(kg, g.pt_import(opt.coeffs(), g.L, 2.0 ** 40), es), o.encrypt(ko, opt, es)
    for a, b in zip(g.rotate_hoisted(kg, gq, [1, 5, 16]), o.rotate_hoisted(ko, oq, [1, 5, 16])):
        _same_oracle(g, a, b)
    _same_oracle(g, g.mul_relin_rescale(kg, gq, gq), o.mul_relin_rescale(ko, oq, oq))
    _same_oracle(g, g.bsgs_matvec_hoisted(kg, gq, gdb, 0), o.bsgs_matvec_hoisted(ko, oq, odb, 0))


@pytest.mark.parametrize("log_n", [11, 13])
def test_other_ring_sizes_bitexact(oracle_mod, log_n):
    """Rings other than 2^12 and 2^16 take the generic transform passes and
    the unfused relinearisation and ModUp paths: rotations, the relinearised
    product, the single-hoisted and the hoisted products are compared
    bit-exactly, and the decrypted scores held to 2^-20."""
    from paper_2604_00546_amd import fr
    p = dict(fr.small_params(), log_n=log_n)
    g, o = fr.Context(**p), oracle_mod.Context(**_oparams(p))
    ell, n1 = 64, 8
    B = (g.N // 2) // ell
    rots = fr.bsgs_rotation_set(ell, n1)
    seed = synth.int_seed(9, synth.SUB_KEYS)
    kg, ko = g.keygen(seed, rots), o.keygen(seed, rots)
    wl = synth.make_workload(9, 300, ell, extra=ell + n1)
    odb = o.db_build(wl.templates, wl.K, ell, B, n1, o.L, 2.0 ** 40)
    gdb = g.db_import(odb.export_all(), odb.G, ell, B, n1, g.L, 2.0 ** 40)
    opt = o.encode(synth.replicate_query(wl.query, g.N // 2), o.L, 2.0 ** 40)
    es = synth.int_seed(9, synth.SUB_ENC)
    gq, oq = g.encrypt(kg, g.pt_import(opt.coeffs(), g.L, 2.0 ** 40), es), o.encrypt(ko, opt, es)
    gr, orr = g.rotate_hoisted(kg, gq, range(1, n1)), o.rotate_hoisted(ko, oq, range(1, n1))
    for a, b in zip(gr, orr):
        _same_oracle(g, a, b)
    _same_oracle(g, g.mul_relin_rescale(kg, gq, gq), o.mul_relin_rescale(ko, oq, oq))
    _same_oracle(g, g.bsgs_diag_matvec(kg, [gq] + gr, gdb, 0), o.bsgs_matvec(ko, [oq] + orr, odb, 0))
    gdb.extend()
    gs = g.bsgs_matvec_hoisted(kg, gq, gdb, 0)
    _same_oracle(g, gs, o.bsgs_matvec_hoisted(ko, oq, odb, 0))
    dec = g.decrypt_decode(kg, gs)
    exact = wl.exact_scores()
    assert np.max(np.abs(dec[: wl.K] - exact)) <= 2 ** -20
