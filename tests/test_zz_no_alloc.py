"""fr_rotate_hoisted_noalloc: the allocation-free hoisted rotation gives the
words of fr_rotate_hoisted, call after call on the same fixed scratch array
(the second call smaller than the first), at N = 2^12 and at the 2^16 ring
of the benchmark (where the rotations are taken in chunks that fit in the
array), and refuses, before any device work, an input whose one rotation
needs more than the array holds."""
import numpy as np
import pytest

from paper_2604_00546_amd import synth

pytestmark = pytest.mark.gpu


def _fresh(g, keys, level, seed):
    z = np.random.default_rng(seed).uniform(-1.0, 1.0, g.N // 2)
    return g.encrypt(keys, g.encode(z, level, 2.0 ** 40), synth.int_seed(seed, synth.SUB_ENC))


def _same(g, keys, ct, rots):
    ref = [g.ct_export(o) for o in g.rotate_hoisted(keys, ct, rots)]
    outs = g.rotate_hoisted_noalloc(keys, ct, rots)
    for r, o, want in zip(rots, outs, ref):
        assert o.level == ct.level and o.scale == ct.scale
        assert np.array_equal(g.ct_export(o), want), f"rotation {r} differs"


@pytest.mark.parametrize("which", ["deep_small_params", "paper_params"])
def test_noalloc_equals_rotate_hoisted_twice(which):
    from paper_2604_00546_amd import fr
    p = getattr(fr, which)()
    g = fr.Context(**p)
    rots = [0, 1, 2, 3, 5, 8, 32]
    keys = g.keygen(synth.int_seed(7, synth.SUB_KEYS), [r for r in rots if r])
    # first call: a fresh query at the top level, every rotation of the set
    print(f"noalloc {which}: level {g.L}, rotations {rots}", flush=True)
    _same(g, keys, _fresh(g, keys, g.L, 11), rots)
    # second call on the same array: a smaller input (fewer limbs, fewer rotations)
    low = g.drop_to(_fresh(g, keys, g.L, 12), 3)
    print(f"noalloc {which}: level 3, rotations [3, 1]", flush=True)
    _same(g, keys, low, [3, 1])
    g.sync()


def test_noalloc_refuses_more_than_the_array():
    from paper_2604_00546_amd import fr
    # one rotation at 25 Q limbs, 5 special primes, dnum 5 needs 147.5 MiB
    g = fr.Context(log_n=16, q0_bits=60, n_mid=24, mid_bits=40, n_special=5, special_bits=60, dnum=5)
    keys = g.keygen(synth.int_seed(8, synth.SUB_KEYS), [1])
    ct = _fresh(g, keys, g.L, 13)
    out = g.new_ct(g.L)
    with pytest.raises(fr.FrError) as e:
        g.rotate_hoisted_noalloc(keys, ct, [1], outs=[out])
    assert e.value.code == fr.FR_ENOMEM
    assert out.level == -1  # descriptor untouched
    # the same input at level 14 (three digits) needs 77.5 MiB: it fits and
    # matches the allocating call
    _same(g, keys, g.drop_to(ct, 14), [1])
    g.sync()
