"""Membership aggregation on the GPU (Alg. gpu-bsgs-membership, aggregation
step): the group Chebyshev ciphertexts are added and the slots summed by
power-of-two rotations.  Bit-exact against the oracle's same sequence, and
the decrypted count equals the FP64 sum of the threshold polynomial over every
slot (the planted matches plus the ripple of the degree-63 step elsewhere).

Ring N = 2^12 with the paper-scale modulus chain, 128-d templates, B = 16,
n1 = 8, 3000 templates in two groups (the second group ragged), 2% planted.
"""
import numpy as np
import pytest

from paper_2604_00546_amd import synth

pytestmark = pytest.mark.gpu

ELL, N1, K = 128, 8, 3000


def _oparams(p):
    return dict(logN=p["log_n"], q0_bits=p["q0_bits"], n_mid=p["n_mid"], mid_bits=p["mid_bits"],
                n_special=p["n_special"], special_bits=p["special_bits"], dnum=p["dnum"])


def test_membership_count_bitexact():
    from oracle import oracle as O
    from paper_2604_00546_amd import fr
    p = fr.deep_small_params()
    g, o = fr.Context(**p), O.Context(**_oparams(p))
    rots = sorted(set(fr.bsgs_rotation_set(ELL, N1)) | set(fr.power_of_two_rotations(g.N)))
    seed = synth.int_seed(6, synth.SUB_KEYS)
    kg, ko = g.keygen(seed, rots), o.keygen(seed, rots)
    wl = synth.make_workload(6, K, ELL, planted_frac=0.02)
    odb = o.db_build(wl.templates, wl.K, ELL, 16, N1, o.L, 2.0 ** 40)
    gdb = g.db_import(odb.export_all(), odb.G, ELL, 16, N1, g.L, 2.0 ** 40)
    assert gdb.G == 2
    opt = o.encode(synth.replicate_query(wl.query, g.N // 2), o.L, 2.0 ** 40)
    es = synth.int_seed(6, synth.SUB_ENC)
    gq, oq = g.encrypt(kg, g.pt_import(opt.coeffs(), g.L, 2.0 ** 40), es), o.encrypt(ko, opt, es)
    gb = [gq] + g.rotate_hoisted(kg, gq, range(1, N1))
    ob = [oq] + o.rotate_hoisted(ko, oq, range(1, N1))
    c = fr.cheb_step_coeffs(63, 0.3)
    gy = [g.chebyshev_eval(kg, g.bsgs_diag_matvec(kg, gb, gdb, grp), c, 8) for grp in range(2)]
    oy = [o.chebyshev(ko, o.bsgs_matvec(ko, ob, odb, grp), c, 8) for grp in range(2)]
    gm = g.membership_aggregate(kg, gy)
    om = o.membership_aggregate(ko, oy)
    assert (gm.level, gm.scale) == (om.level, om.scale)
    bad = np.argwhere(g.ct_export(gm) != om.coeffs())
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:3].tolist()}"
    count = g.decrypt_decode(kg, gm)
    # every slot of both groups is a template or a zero padding row; the
    # count is the sum of the polynomial over all of them (its ripple away
    # from the step included)
    pad = 2 * (g.N // 2) - K
    want = np.polynomial.chebyshev.chebval(wl.exact_scores(), c).sum() + pad * np.polynomial.chebyshev.chebval(0.0, c)
    assert np.max(np.abs(count - want)) < 0.1


def test_membership_needs_power_of_two_keys():
    from paper_2604_00546_amd import fr
    g = fr.Context(**fr.small_params())
    k = g.keygen(5, [1, 2])
    ct = g.encrypt(k, g.encode(np.zeros(g.N // 2), g.L, 2.0 ** 40), 3)
    with pytest.raises(fr.FrError):
        g.membership_aggregate(k, [ct])
