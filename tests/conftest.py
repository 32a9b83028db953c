import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU oracle case")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    O.lib()
    return O


@pytest.fixture(scope="session")
def small_ctx(oracle_mod):
    """N = 2^12; Q = 50 + 40 + 40 bits; P = one 60-bit prime; dnum 3."""
    return oracle_mod.Context(**oracle_mod.small_params())


@pytest.fixture(scope="session")
def deep_ctx(oracle_mod):
    """N = 2^12 with the paper-scale modulus chain (60 + 14 x 40 bits, P = 5 x 60,
    dnum 3): room for the Chebyshev ladder at a ring size the oracle runs fast."""
    return oracle_mod.Context(logN=12, q0_bits=60, n_mid=14, mid_bits=40, n_special=5, special_bits=60, dnum=3)
