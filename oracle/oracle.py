"""ctypes wrapper of the plain CPU oracle (oracle/ckks_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product path.  It
marshals arguments and copies results into numpy arrays -- all arithmetic is
in the C oracle.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")


class _Ct(C.Structure):
    _fields_ = [("level", C.c_int), ("scale", C.c_double), ("c", C.POINTER(C.c_uint64))]


class _Pt(C.Structure):
    _fields_ = [("level", C.c_int), ("scale", C.c_double), ("m", C.POINTER(C.c_uint64))]


_P = C.c_void_p
_CT = C.POINTER(_Ct)
_PT = C.POINTER(_Pt)
_U64P = C.POINTER(C.c_uint64)
_I64P = C.POINTER(C.c_int64)
_DP = C.POINTER(C.c_double)
_I32P = C.POINTER(C.c_int32)

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # type: ignore
        _b.build()
    L = C.CDLL(_LIB_PATH)
    sig = {
        "or_ctx_create": (_P, [C.c_int] * 7),
        "or_ctx_free": (None, [_P]),
        "or_ctx_N": (C.c_int, [_P]),
        "or_ctx_L": (C.c_int, [_P]),
        "or_ctx_nspecial": (C.c_int, [_P]),
        "or_ctx_alpha": (C.c_int, [_P]),
        "or_ctx_modulus": (C.c_uint64, [_P, C.c_int]),
        "or_last_error": (C.c_char_p, []),
        "or_set_threads": (None, [C.c_int]),
        "or_get_threads": (C.c_int, []),
        "or_philox4x64_10": (None, [_U64P, _U64P, _U64P]),
        "or_gauss_cdt": (None, [_U64P]),
        "or_sample_uniform": (None, [C.c_uint64, C.c_uint64, C.c_int, C.c_uint64, C.c_int, _U64P]),
        "or_sample_ternary": (None, [C.c_uint64, C.c_uint64, C.c_int, _I64P]),
        "or_sample_gauss": (None, [C.c_uint64, C.c_uint64, C.c_int, _I64P]),
        "or_galois_element": (C.c_uint64, [_P, C.c_int]),
        "or_polymul": (C.c_int, [_P, C.c_int, _U64P, _U64P, _U64P]),
        "or_automorphism": (None, [_P, C.c_int, C.c_uint64, _U64P, _U64P]),
        "or_modup_digit": (C.c_int, [_P, C.c_int, C.c_int, _U64P, _U64P]),
        "or_moddown": (C.c_int, [_P, C.c_int, _U64P, _U64P]),
        "or_keygen": (_P, [_P, C.c_uint64, _I32P, C.c_int]),
        "or_keys_free": (None, [_P]),
        "or_keys_secret": (_I64P, [_P]),
        "or_keys_pk": (_U64P, [_P]),
        "or_keys_ksk": (_U64P, [_P, C.c_uint64]),
        "or_encode": (_PT, [_P, _DP, C.c_int, C.c_int, C.c_double]),
        "or_encode_direct": (_PT, [_P, _DP, C.c_int, C.c_int, C.c_double]),
        "or_encode_fft": (_PT, [_P, _DP, C.c_int, C.c_int, C.c_double]),
        "or_pt_import": (_PT, [_P, _U64P, C.c_int, C.c_double]),
        "or_pt_free": (None, [_PT]),
        "or_encrypt": (_CT, [_P, _P, _PT, C.c_uint64]),
        "or_decrypt": (_PT, [_P, _P, _CT]),
        "or_pt_lift": (C.c_int, [_P, _PT, _DP]),
        "or_decode": (C.c_int, [_P, _PT, _DP]),
        "or_decode_direct": (C.c_int, [_P, _PT, _DP]),
        "or_decode_fft": (C.c_int, [_P, _PT, _DP]),
        "or_ct_import": (_CT, [_P, _U64P, C.c_int, C.c_double]),
        "or_ct_copy": (_CT, [_P, _CT]),
        "or_ct_free": (None, [_CT]),
        "or_rotate_hoisted": (C.c_int, [_P, _P, _CT, _I32P, C.c_int, C.POINTER(_CT)]),
        "or_rescale": (_CT, [_P, _CT]),
        "or_rotate_sum": (_CT, [_P, _P, C.POINTER(_CT), C.c_int, C.c_int]),
        "or_add": (_CT, [_P, _CT, _CT]),
        "or_sub": (_CT, [_P, _CT, _CT]),
        "or_mul_plain": (_CT, [_P, _CT, _PT]),
        "or_mul_relin_rescale": (_CT, [_P, _P, _CT, _CT]),
        "or_tensor_sum_relin_rescale": (_CT, [_P, _P, C.POINTER(_CT), C.POINTER(_CT), C.c_int]),
        "or_mul_int": (_CT, [_P, _CT, C.c_int64]),
        "or_add_const": (_CT, [_P, _CT, C.c_double]),
        "or_drop_to": (_CT, [_P, _CT, C.c_int]),
        "or_db_build": (_P, [_P, C.POINTER(C.c_float), C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                             C.c_double]),
        "or_db_import": (_P, [_P, _U64P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double]),
        "or_db_free": (None, [_P]),
        "or_db_groups": (C.c_int, [_P]),
        "or_db_export": (C.c_int, [_P, C.c_int, C.c_int, _U64P]),
        "or_db_slots": (C.c_int, [_P, C.POINTER(C.c_float), C.c_int, C.c_int, C.c_int, C.c_int,
                                  C.c_int, C.c_int, _DP]),
        "or_bsgs_matvec": (_CT, [_P, _P, C.POINTER(_CT), C.c_int, _P, C.c_int]),
        "or_bsgs_matvec_hoisted": (_CT, [_P, _P, _CT, C.c_int, _P, C.c_int]),
        "or_db_export_special": (C.c_int, [_P, _P, C.c_int, C.c_int, _U64P]),
        "or_db_extend": (C.c_int, [_P, _P]),
        "or_cheb_step_coeffs": (None, [C.c_int, C.c_double, _DP]),
        "or_cheb_clenshaw": (C.c_double, [_DP, C.c_int, C.c_double]),
        "or_chebyshev": (_CT, [_P, _P, _CT, _DP, C.c_int, C.c_int]),
        "or_chebyshev_count_mults": (C.c_int, [C.c_int, C.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class OracleError(RuntimeError):
    pass


def _err(what: str):
    raise OracleError(f"{what}: {lib().or_last_error().decode()}")


def _u64(a: np.ndarray):
    return a.ctypes.data_as(_U64P)


def _f64(a: np.ndarray):
    return a.ctypes.data_as(_DP)


# --------------------------------------------------------------------------
# plain functions
# --------------------------------------------------------------------------
def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(_u64(c), _u64(k), _u64(out))
    return out


def gauss_cdt() -> np.ndarray:
    out = np.zeros(20, dtype=np.uint64)
    lib().or_gauss_cdt(_u64(out))
    return out


def sample_uniform(seed, poly, gidx, q, N) -> np.ndarray:
    out = np.zeros(N, dtype=np.uint64)
    lib().or_sample_uniform(seed, poly, gidx, q, N, _u64(out))
    return out


def sample_ternary(seed, poly, N) -> np.ndarray:
    out = np.zeros(N, dtype=np.int64)
    lib().or_sample_ternary(seed, poly, N, out.ctypes.data_as(_I64P))
    return out


def sample_gauss(seed, poly, N) -> np.ndarray:
    out = np.zeros(N, dtype=np.int64)
    lib().or_sample_gauss(seed, poly, N, out.ctypes.data_as(_I64P))
    return out


def cheb_step_coeffs(n: int, delta: float) -> np.ndarray:
    out = np.zeros(n + 1, dtype=np.float64)
    lib().or_cheb_step_coeffs(n, delta, _f64(out))
    return out


def cheb_clenshaw(c, x: float) -> float:
    c = np.ascontiguousarray(c, dtype=np.float64)
    return lib().or_cheb_clenshaw(_f64(c), len(c) - 1, x)


def cheb_count_mults(n: int, d1: int) -> int:
    return lib().or_chebyshev_count_mults(n, d1)


# --------------------------------------------------------------------------
# objects
# --------------------------------------------------------------------------
class Ct:
    def __init__(self, ctx: "Context", ptr):
        if not ptr:
            _err("ciphertext")
        self.ctx, self.ptr = ctx, ptr

    def __del__(self):
        try:
            if self.ptr:
                lib().or_ct_free(self.ptr)
        except Exception:
            pass

    @property
    def level(self) -> int:
        return self.ptr.contents.level

    @property
    def scale(self) -> float:
        return self.ptr.contents.scale

    @scale.setter
    def scale(self, v: float):
        self.ptr.contents.scale = v

    def coeffs(self) -> np.ndarray:
        """[2][level+1][N] canonical coefficient residues (a copy)."""
        n = 2 * (self.level + 1) * self.ctx.N
        a = np.ctypeslib.as_array(self.ptr.contents.c, shape=(n,)).copy()
        return a.reshape(2, self.level + 1, self.ctx.N)


class Pt:
    def __init__(self, ctx: "Context", ptr):
        if not ptr:
            _err("plaintext")
        self.ctx, self.ptr = ctx, ptr

    def __del__(self):
        try:
            if self.ptr:
                lib().or_pt_free(self.ptr)
        except Exception:
            pass

    @property
    def level(self) -> int:
        return self.ptr.contents.level

    @property
    def scale(self) -> float:
        return self.ptr.contents.scale

    def coeffs(self) -> np.ndarray:
        n = (self.level + 1) * self.ctx.N
        a = np.ctypeslib.as_array(self.ptr.contents.m, shape=(n,)).copy()
        return a.reshape(self.level + 1, self.ctx.N)


class Keys:
    def __init__(self, ctx: "Context", ptr, rots):
        if not ptr:
            _err("keygen")
        self.ctx, self.ptr, self.rots = ctx, ptr, list(rots)

    def __del__(self):
        try:
            lib().or_keys_free(self.ptr)
        except Exception:
            pass

    def secret(self) -> np.ndarray:
        return np.ctypeslib.as_array(lib().or_keys_secret(self.ptr), shape=(self.ctx.N,)).copy()

    def pk(self) -> np.ndarray:
        c = self.ctx
        return np.ctypeslib.as_array(lib().or_keys_pk(self.ptr),
                                     shape=(2 * (c.L + 1) * c.N,)).copy().reshape(2, c.L + 1, c.N)

    def ksk(self, kid: int) -> np.ndarray:
        c = self.ctx
        p = lib().or_keys_ksk(self.ptr, kid)
        if not p:
            raise KeyError(kid)
        nm = c.L + 1 + c.nP
        return np.ctypeslib.as_array(p, shape=(c.dnum * 2 * nm * c.N,)).copy().reshape(c.dnum, 2, nm, c.N)


class Db:
    def __init__(self, ctx, ptr, ell, B, n1, level, scale):
        if not ptr:
            _err("db")
        self.ctx, self.ptr = ctx, ptr
        self.ell, self.B, self.n1, self.level, self.scale = ell, B, n1, level, scale
        self.G = lib().or_db_groups(ptr)

    def __del__(self):
        try:
            lib().or_db_free(self.ptr)
        except Exception:
            pass

    def export(self, g: int, d: int) -> np.ndarray:
        out = np.zeros((self.level + 1) * self.ctx.N, dtype=np.uint64)
        if lib().or_db_export(self.ptr, g, d, _u64(out)):
            _err("db_export")
        return out.reshape(self.level + 1, self.ctx.N)

    def export_all(self) -> np.ndarray:
        return np.stack([np.stack([self.export(g, d) for d in range(self.ell)]) for g in range(self.G)])

    def extend(self) -> "Db":
        """Build the special-prime limbs of every diagonal now."""
        lib().or_db_extend(self.ctx.ptr, self.ptr)
        return self

    def export_special(self, g: int, d: int) -> np.ndarray:
        """Residues of plaintext (g, d)'s centered coefficients mod the special primes, [nP][N]."""
        out = np.zeros(self.ctx.nP * self.ctx.N, dtype=np.uint64)
        if lib().or_db_export_special(self.ctx.ptr, self.ptr, g, d, _u64(out)):
            _err("db_export_special")
        return out.reshape(self.ctx.nP, self.ctx.N)


class Context:
    """Parameter set and every oracle operation on it."""

    def __init__(self, logN, q0_bits, n_mid, mid_bits, n_special, special_bits, dnum):
        self.ptr = lib().or_ctx_create(logN, q0_bits, n_mid, mid_bits, n_special, special_bits, dnum)
        if not self.ptr:
            _err("ctx_create")
        self.logN = logN
        self.N = lib().or_ctx_N(self.ptr)
        self.L = lib().or_ctx_L(self.ptr)
        self.nP = lib().or_ctx_nspecial(self.ptr)
        self.alpha = lib().or_ctx_alpha(self.ptr)
        self.dnum = dnum
        self.moduli = [int(lib().or_ctx_modulus(self.ptr, i)) for i in range(self.L + 1 + self.nP)]
        self.q = self.moduli[: self.L + 1]
        self.p = self.moduli[self.L + 1:]

    def __del__(self):
        try:
            lib().or_ctx_free(self.ptr)
        except Exception:
            pass

    # helpers --------------------------------------------------------------
    def galois(self, rot: int) -> int:
        return int(lib().or_galois_element(self.ptr, rot))

    def polymul(self, gidx, a, b) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        out = np.zeros(self.N, dtype=np.uint64)
        if lib().or_polymul(self.ptr, gidx, _u64(a), _u64(b), _u64(out)):
            _err("polymul")
        return out

    def automorphism(self, gidx, g, a) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint64)
        out = np.zeros(self.N, dtype=np.uint64)
        lib().or_automorphism(self.ptr, gidx, g, _u64(a), _u64(out))
        return out

    def modup_digit(self, level, t, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.uint64)
        out = np.zeros((level + 1 + self.nP, self.N), dtype=np.uint64)
        if lib().or_modup_digit(self.ptr, level, t, _u64(x), _u64(out)):
            _err("modup")
        return out

    def moddown(self, level, u) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.uint64)
        out = np.zeros((level + 1, self.N), dtype=np.uint64)
        if lib().or_moddown(self.ptr, level, _u64(u), _u64(out)):
            _err("moddown")
        return out

    # keys / encoding ---------------------------------------------------------
    def keygen(self, seed: int, rots) -> Keys:
        r = np.ascontiguousarray(list(rots), dtype=np.int32)
        return Keys(self, lib().or_keygen(self.ptr, seed, r.ctypes.data_as(_I32P), len(r)), rots)

    def encode(self, z, level, scale, method: str = "auto") -> Pt:
        z = np.ascontiguousarray(z, dtype=np.float64)
        f = {"auto": lib().or_encode, "direct": lib().or_encode_direct, "fft": lib().or_encode_fft}[method]
        return Pt(self, f(self.ptr, _f64(z), len(z), level, scale))

    def pt_import(self, m, level, scale) -> Pt:
        m = np.ascontiguousarray(m, dtype=np.uint64)
        return Pt(self, lib().or_pt_import(self.ptr, _u64(m), level, scale))

    def ct_import(self, c, level, scale) -> Ct:
        c = np.ascontiguousarray(c, dtype=np.uint64)
        return Ct(self, lib().or_ct_import(self.ptr, _u64(c), level, scale))

    def encrypt(self, keys: Keys, pt: Pt, seed: int) -> Ct:
        return Ct(self, lib().or_encrypt(self.ptr, keys.ptr, pt.ptr, seed))

    def decrypt(self, keys: Keys, ct: Ct) -> Pt:
        return Pt(self, lib().or_decrypt(self.ptr, keys.ptr, ct.ptr))

    def lift(self, pt: Pt) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.float64)
        lib().or_pt_lift(self.ptr, pt.ptr, _f64(out))
        return out

    def decode(self, pt: Pt, method: str = "auto") -> np.ndarray:
        out = np.zeros(self.N // 2, dtype=np.float64)
        f = {"auto": lib().or_decode, "direct": lib().or_decode_direct, "fft": lib().or_decode_fft}[method]
        f(self.ptr, pt.ptr, _f64(out))
        return out

    def decrypt_decode(self, keys: Keys, ct: Ct) -> np.ndarray:
        return self.decode(self.decrypt(keys, ct))

    # homomorphic ops ------------------------------------------------------------
    def rotate_hoisted(self, keys: Keys, ct: Ct, rots) -> list:
        r = np.ascontiguousarray(list(rots), dtype=np.int32)
        outs = (_CT * len(r))()
        if lib().or_rotate_hoisted(self.ptr, keys.ptr, ct.ptr, r.ctypes.data_as(_I32P), len(r), outs):
            _err("rotate_hoisted")
        return [Ct(self, outs[i]) for i in range(len(r))]

    def rescale(self, ct: Ct) -> Ct:
        return Ct(self, lib().or_rescale(self.ptr, ct.ptr))

    def membership_aggregate(self, keys: Keys, cts) -> Ct:
        """Aggregation step of Alg. gpu-bsgs-membership (Alg. membership of the
        appendix: EvalAddMany, then EvalSum over all slots): the group
        ciphertexts are added in order, then x <- x + Rot_{2^i}(x) for
        i < log2(N/2), after which every slot holds the sum of all slots."""
        x = cts[0]
        for c in cts[1:]:
            x = self.add(x, c)
        for i in range(self.logN - 1):
            x = self.add(x, self.rotate_hoisted(keys, x, [1 << i])[0])
        return x

    def add(self, a: Ct, b: Ct) -> Ct:
        return Ct(self, lib().or_add(self.ptr, a.ptr, b.ptr))

    def sub(self, a: Ct, b: Ct) -> Ct:
        return Ct(self, lib().or_sub(self.ptr, a.ptr, b.ptr))

    def mul_plain(self, a: Ct, p: Pt) -> Ct:
        return Ct(self, lib().or_mul_plain(self.ptr, a.ptr, p.ptr))

    def mul_relin_rescale(self, keys: Keys, a: Ct, b: Ct) -> Ct:
        return Ct(self, lib().or_mul_relin_rescale(self.ptr, keys.ptr, a.ptr, b.ptr))

    def tensor_sum_relin_rescale(self, keys: Keys, a, b) -> Ct:
        """Sum of the tensor products of the pairs (a[k], b[k]), one
        relinearisation, rescale (the encrypted-database product)."""
        n = len(a)
        pa = (_CT * n)(*[x.ptr for x in a])
        pb = (_CT * n)(*[x.ptr for x in b])
        r = lib().or_tensor_sum_relin_rescale(self.ptr, keys.ptr, pa, pb, n)
        if not r:
            _err("tensor_sum_relin_rescale")
        return Ct(self, r)

    def rotate_sum(self, keys: Keys, cts, stride: int) -> Ct:
        """cts[0] + sum_{j >= 1} Rot_{j stride}(cts[j]), one shared ModDown."""
        n = len(cts)
        p = (_CT * n)(*[x.ptr for x in cts])
        r = lib().or_rotate_sum(self.ptr, keys.ptr, p, n, stride)
        if not r:
            _err("rotate_sum")
        return Ct(self, r)

    def mul_int(self, a: Ct, k: int) -> Ct:
        return Ct(self, lib().or_mul_int(self.ptr, a.ptr, k))

    def add_const(self, a: Ct, c: float) -> Ct:
        return Ct(self, lib().or_add_const(self.ptr, a.ptr, c))

    def drop_to(self, a: Ct, level: int) -> Ct:
        return Ct(self, lib().or_drop_to(self.ptr, a.ptr, level))

    # database / matvec / chebyshev ---------------------------------------------------
    def db_build(self, T, K, ell, B, n1, level, scale_d) -> Db:
        T = np.ascontiguousarray(T, dtype=np.float32)
        return Db(self, lib().or_db_build(self.ptr, T.ctypes.data_as(C.POINTER(C.c_float)), K, ell, B, n1,
                                          level, scale_d), ell, B, n1, level, scale_d)

    def db_import(self, coeffs, G, ell, B, n1, level, scale_d) -> Db:
        c = np.ascontiguousarray(coeffs, dtype=np.uint64)
        return Db(self, lib().or_db_import(self.ptr, _u64(c), G, ell, B, n1, level, scale_d),
                  ell, B, n1, level, scale_d)

    def db_slots(self, T, K, ell, B, n1, g, d) -> np.ndarray:
        T = np.ascontiguousarray(T, dtype=np.float32)
        v = np.zeros(self.N // 2, dtype=np.float64)
        if lib().or_db_slots(self.ptr, T.ctypes.data_as(C.POINTER(C.c_float)), K, ell, B, n1, g, d, _f64(v)):
            _err("db_slots")
        return v

    def bsgs_matvec(self, keys: Keys, baby: list, db: Db, group: int) -> Ct:
        arr = (_CT * len(baby))(*[b.ptr for b in baby])
        return Ct(self, lib().or_bsgs_matvec(self.ptr, keys.ptr, arr, len(baby), db.ptr, group))

    def bsgs_matvec_hoisted(self, keys: Keys, ct: Ct, db: Db, group: int) -> Ct:
        """The product from the query itself, baby steps held over Q_l U P (the inner sums' first
        polynomials rotated and summed before one ModDown, one ModDown per second polynomial)."""
        return Ct(self, lib().or_bsgs_matvec_hoisted(self.ptr, keys.ptr, ct.ptr, db.n1, db.ptr, group))

    def chebyshev(self, keys: Keys, x: Ct, coeffs, d1: int) -> Ct:
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        return Ct(self, lib().or_chebyshev(self.ptr, keys.ptr, x.ptr, _f64(c), len(c) - 1, d1))


# parameter sets of the two ring sizes the tests and the benchmark use
def set_threads(n: int):
    """OpenMP threads the oracle's parallel loops use from now on."""
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def small_params():
    """N = 2^12; Q = one 50-bit + two 40-bit primes; P = one 60-bit prime; dnum 3."""
    return dict(logN=12, q0_bits=50, n_mid=2, mid_bits=40, n_special=1, special_bits=60, dnum=3)


def paper_params():
    """N = 2^16; Q = one 60-bit + fourteen 40-bit primes; P = five 60-bit primes; dnum 3."""
    return dict(logN=16, q0_bits=60, n_mid=14, mid_bits=40, n_special=5, special_bits=60, dnum=3)
