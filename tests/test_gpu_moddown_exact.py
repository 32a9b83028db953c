"""GPU parity of ModDown's rounding where an FP64 estimate cannot decide it.

Integers U = P w + r with r = U mod P at (P -+ 1)/2 (+- d) or across the
2^-40 band around P/2 go through the device's three ModDown paths via the
parity hook (the key switch of a rotation, the inner sums' merged ModDown +
rescale, the relinearised product's merged ModDown + rescale) and are
compared word for word with the oracle's ModDown (exact big-integer
rounding), and on the key-switch path also with round(U / P) itself.
"""
import math

import numpy as np
import pytest

import moddown_cases as mc

pytestmark = pytest.mark.gpu


def _oparams(p):
    return dict(logN=p["log_n"], q0_bits=p["q0_bits"], n_mid=p["n_mid"], mid_bits=p["mid_bits"],
                n_special=p["n_special"], special_bits=p["special_bits"], dnum=p["dnum"])


@pytest.fixture(scope="module", params=["small", "deep", "paper"])
def case(request, oracle_mod):
    from paper_2604_00546_amd import fr
    p = {"small": fr.small_params, "deep": fr.deep_small_params, "paper": fr.paper_params}[request.param]()
    g, o = fr.Context(**p), oracle_mod.Context(**_oparams(p))
    level = g.L
    n_adv = 1024 if request.param != "paper" else 2048
    u, Us, P = mc.build_u(g.moduli, level, g.L, g.nP, g.N, n_adv, seed=23)
    rnd = np.random.default_rng(24)
    d = np.stack([np.stack([rnd.integers(0, q, g.N, dtype=np.uint64) for q in g.q[: level + 1]]) for _ in range(2)])
    print(f"moddown parity case {request.param}: N={g.N} level={level} nP={g.nP}", flush=True)
    return request.param, g, o, level, u, Us, P, d


def _oracle_moddown_ct(o, level, u):
    m = np.stack([o.moddown(level, u[0]), o.moddown(level, u[1])])
    return o.ct_import(m, level, 1.0)


def test_inputs_reach_the_undecidable_band(case):
    name, g, o, level, u, Us, P, d = case
    if name == "paper":
        pytest.skip("coverage is counted on the N = 2^12 rings (same primes as the paper chain)")
    assert mc.fp64_rule_differs(u[0], g.moduli, level, g.L, g.nP) > 0


def test_key_switch_moddown_exact(case):
    name, g, o, level, u, Us, P, d = case
    got = g.ct_export(g.moddown_parity(0, u, level))
    want = _oracle_moddown_ct(o, level, u).coeffs()
    bad = np.argwhere(got != want)
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:3].tolist()}"
    for k in list(range(0, 64)) + list(range(64, g.N, 257)):
        r = (2 * Us[0][k] + P) // (2 * P)
        assert [int(got[0][i][k]) for i in range(level + 1)] == [r % q for q in g.q[: level + 1]], k


def test_inner_sum_moddown_rescale_exact(case):
    name, g, o, level, u, Us, P, d = case
    got = g.ct_export(g.moddown_parity(1, u, level))
    want = o.rescale(_oracle_moddown_ct(o, level, u)).coeffs()
    bad = np.argwhere(got != want)
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:3].tolist()}"


def test_relin_moddown_rescale_exact(case):
    name, g, o, level, u, Us, P, d = case
    got = g.ct_export(g.moddown_parity(2, u, level, d))
    want = o.rescale(o.add(o.ct_import(d, level, 1.0), _oracle_moddown_ct(o, level, u))).coeffs()
    bad = np.argwhere(got != want)
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:3].tolist()}"


def test_hook_rejects_bad_input(case):
    name, g, o, level, u, Us, P, d = case
    from paper_2604_00546_amd import fr
    bad = u.copy()
    bad[0, 0, 0] = g.q[0]
    with pytest.raises(fr.FrError) as e:
        g.moddown_parity(0, bad, level)
    assert e.value.code == fr.FR_EINVAL
    with pytest.raises(fr.FrError) as e:
        g.moddown_parity(1, u[:, : 1 + g.nP].copy(), 0)
    assert e.value.code == fr.FR_ELEVEL
