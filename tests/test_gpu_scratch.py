"""The boundary's error contract for device scratch: a call that needs more
scratch than the context's limit returns FR_ENOMEM (no abort), leaves its
output descriptor untouched, and the context works again, with the same
words, once the limit is lifted."""
import numpy as np
import pytest

from paper_2604_00546_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup(oracle_mod):
    from paper_2604_00546_amd import fr
    p = fr.deep_small_params()
    g = fr.Context(**p)
    ell, n1, B = 128, 8, 16
    rots = fr.bsgs_rotation_set(ell, n1)
    keys = g.keygen(synth.int_seed(1, synth.SUB_KEYS), rots)
    wl = synth.make_workload(1, 64, ell)
    q = g.encrypt(keys, g.encode(synth.replicate_query(wl.query, g.N // 2), g.L, 2.0 ** 40),
                  synth.int_seed(1, synth.SUB_ENC))
    db = g.db_load(wl.templates, ell, B, n1, g.L, 2.0 ** 40).extend()
    coeffs = fr.cheb_step_coeffs(63, 0.3)
    return fr, g, keys, q, db, coeffs


def test_matvec_over_the_limit_is_enomem(setup):
    fr, g, keys, q, db, coeffs = setup
    ref = g.ct_export(g.bsgs_matvec_hoisted(keys, q, db, 0))
    alloc, peak = g.scratch_info()
    assert peak > 0 and alloc >= peak
    g.set_scratch_limit(peak // 4)
    assert g.scratch_info()[0] <= peak // 4
    out = g.new_ct(q.level - 1)
    with pytest.raises(fr.FrError) as e:
        g.bsgs_matvec_hoisted(keys, q, db, 0, out=out)
    assert e.value.code == fr.FR_ENOMEM
    assert out.level == -1  # descriptor untouched
    # the same context, limit lifted: the same words
    g.set_scratch_limit(0)
    got = g.ct_export(g.bsgs_matvec_hoisted(keys, q, db, 0, out=out))
    assert np.array_equal(got, ref)


def test_chebyshev_over_the_limit_is_enomem(setup):
    fr, g, keys, q, db, coeffs = setup
    s = g.bsgs_matvec_hoisted(keys, q, db, 0)
    ref = g.ct_export(g.chebyshev_eval(keys, s, coeffs, 8))
    g.set_scratch_limit(1 << 20)
    with pytest.raises(fr.FrError) as e:
        g.chebyshev_eval(keys, s, coeffs, 8)
    assert e.value.code == fr.FR_ENOMEM
    g.set_scratch_limit(0)
    assert np.array_equal(g.ct_export(g.chebyshev_eval(keys, s, coeffs, 8)), ref)


def test_reserve_respects_the_limit(setup):
    fr, g, keys, q, db, coeffs = setup
    g.set_scratch_limit(256 << 20)
    with pytest.raises(fr.FrError) as e:
        g.reserve(512 << 20)
    assert e.value.code == fr.FR_ENOMEM
    g.reserve(200 << 20)
    assert g.scratch_info()[0] >= 200 << 20
    g.set_scratch_limit(0)
