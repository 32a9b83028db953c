"""GPU parity of the encrypted-database BSGS product (BSGS-TBS and -TBE):
the server-side homomorphic pre-rotation of encrypted diagonals with
temporary negative giant-step keys, the enroller-side alternative
(encrypted pre-rotated plaintexts), the product with one relinearisation
per giant step, and the giant rotate-sum, each word for word against the
oracle's composition of the same steps."""
import numpy as np
import pytest

from paper_2604_00546_amd import synth

pytestmark = pytest.mark.gpu

ELL, N1, B = 128, 8, 16
ROTS = list(range(1, N1)) + [N1 * j for j in range(1, ELL // N1)]
NEG = [-N1 * j for j in range(1, ELL // N1)]


def _oparams(p):
    return dict(logN=p["log_n"], q0_bits=p["q0_bits"], n_mid=p["n_mid"], mid_bits=p["mid_bits"],
                n_special=p["n_special"], special_bits=p["special_bits"], dnum=p["dnum"])


def _same(g, gct, oct_):
    a, b = g.ct_export(gct), oct_.coeffs()
    assert (gct.level, gct.scale) == (oct_.level, oct_.scale)
    bad = np.argwhere(a != b)
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:3].tolist()}"


@pytest.fixture(scope="module")
def E(oracle_mod):
    from paper_2604_00546_amd import fr
    p = fr.deep_small_params()
    g, o = fr.Context(**p), oracle_mod.Context(**_oparams(p))
    seed = synth.int_seed(6, synth.SUB_KEYS)
    kg, ko = g.keygen(seed, ROTS), o.keygen(seed, ROTS)
    tg, to = g.keygen(seed, NEG), o.keygen(seed, NEG)  # temporary keys, same secret
    wl = synth.make_workload(6, 64, ELL)
    plain = o.db_build(wl.templates, wl.K, ELL, B, ELL, o.L, 2.0 ** 40)  # not pre-rotated
    pre = o.db_build(wl.templates, wl.K, ELL, B, N1, o.L, 2.0 ** 40)     # pre-rotated slots (TBE)
    enc_g, enc_o, tbe_g, tbe_o = [], [], [], []
    for d in range(ELL):
        m = plain.export(0, d)
        s = synth.int_seed(6, synth.SUB_ENC, d)
        enc_g.append(g.encrypt(kg, g.pt_import(m, g.L, 2.0 ** 40), s))
        enc_o.append(o.encrypt(ko, o.pt_import(m, o.L, 2.0 ** 40), s))
        m = pre.export(0, d)
        s = synth.int_seed(6, synth.SUB_ENC, 500 + d)
        tbe_g.append(g.encrypt(kg, g.pt_import(m, g.L, 2.0 ** 40), s))
        tbe_o.append(o.encrypt(ko, o.pt_import(m, o.L, 2.0 ** 40), s))
    qs = synth.int_seed(6, synth.SUB_ENC, 999)
    opt = o.encode(synth.replicate_query(wl.query, o.N // 2), o.L, 2.0 ** 40)
    qg, qo = g.encrypt(kg, g.pt_import(opt.coeffs(), g.L, 2.0 ** 40), qs), o.encrypt(ko, opt, qs)
    bg = [qg] + g.rotate_hoisted(kg, qg, range(1, N1))
    bo = [qo] + o.rotate_hoisted(ko, qo, range(1, N1))
    print("encrypted-database case: N=2^12, 64 templates x 128-d, n1=8", flush=True)
    return dict(g=g, o=o, kg=kg, ko=ko, tg=tg, to=to, wl=wl, enc_g=enc_g, enc_o=enc_o, tbe_g=tbe_g,
                tbe_o=tbe_o, bg=bg, bo=bo)


def test_tbs_prerotation_bitexact(E):
    """Server-side pre-rotation: the diagonals of giant step j rotated by
    -j n1 in one batched hoisted call per j."""
    g, o = E["g"], E["o"]
    tbs_g = list(E["enc_g"][:N1])
    for j in range(1, ELL // N1):
        blk = E["enc_g"][j * N1:(j + 1) * N1]
        tbs_g += [row[0] for row in g.rotate_hoisted_batch(E["tg"], blk, [-N1 * j])]
    tbs_o = [E["enc_o"][d] if d < N1 else o.rotate_hoisted(E["to"], E["enc_o"][d], [-N1 * (d // N1)])[0]
             for d in range(ELL)]
    for d in (0, 7, 8, 63, 127):
        _same(g, tbs_g[d], tbs_o[d])
    E["tbs_g"], E["tbs_o"] = tbs_g, tbs_o


@pytest.mark.parametrize("form", ["tbs", "tbe"])
def test_encrypted_bsgs_matvec_bitexact(E, form):
    g, o = E["g"], E["o"]
    if form == "tbs" and "tbs_g" not in E:
        test_tbs_prerotation_bitexact(E)
    dg, do = E[form + "_g"], E[form + "_o"]
    S = g.bsgs_encrypted_matvec(E["kg"], E["bg"], dg)
    P = [o.tensor_sum_relin_rescale(E["ko"], E["bo"], do[j * N1:(j + 1) * N1]) for j in range(ELL // N1)]
    So = o.rotate_sum(E["ko"], P, N1)
    _same(g, S, So)
    dec = g.decrypt_decode(E["kg"], S)
    assert np.max(np.abs(dec[:64] - E["wl"].exact_scores())) < 2 ** -19


def test_rotate_sum_bitexact(E):
    g, o = E["g"], E["o"]
    cts_g, cts_o = E["bg"][:4], E["bo"][:4]
    _same(g, g.rotate_sum(E["kg"], cts_g, N1), o.rotate_sum(E["ko"], cts_o, N1))
    # a single input comes back unchanged
    _same(g, g.rotate_sum(E["kg"], cts_g[:1], N1), cts_o[0])


def test_missing_keys_are_errors(E):
    from paper_2604_00546_amd import fr
    g = E["g"]
    with pytest.raises(fr.FrError) as e:
        g.rotate_sum(E["tg"], E["bg"][:3], N1)  # only negative rotations in the temporary keys
    assert e.value.code == fr.FR_ENOKEY
