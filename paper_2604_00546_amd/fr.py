"""Python binding of the gfx950 library (include/fr.h), same names as the C ABI.

Argument marshalling only: every homomorphic step runs in libfrhip.so's
kernels.  PyTorch provides the device buffers of ciphertexts and plaintexts
(int64 tensors holding the uint64 words) and the stream.  There is no
fallback: if the built library is missing this module raises on first use.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfrhip.so")


class FrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


FR_OK, FR_EINVAL, FR_ENOMEM, FR_ELEVEL, FR_ENOKEY, FR_EHIP, FR_ERANGE = 0, -1, -2, -3, -4, -5, -6


class Params(C.Structure):
    _fields_ = [("log_n", C.c_int32), ("q0_bits", C.c_int32), ("n_mid", C.c_int32), ("mid_bits", C.c_int32),
                ("n_special", C.c_int32), ("special_bits", C.c_int32), ("dnum", C.c_int32)]


class CtDesc(C.Structure):
    _fields_ = [("data", C.c_void_p), ("level", C.c_int32), ("cap", C.c_int32), ("scale", C.c_double)]


PtDesc = CtDesc  # same layout (data, level, cap, scale)

_P = C.c_void_p
_U64P = C.POINTER(C.c_uint64)
_DP = C.POINTER(C.c_double)
_I32P = C.POINTER(C.c_int32)
_CTP = C.POINTER(CtDesc)
_lib = None

# symbol -> (restype, argtypes); every symbol declared in include/fr.h
SIGNATURES = {
    "fr_last_error": (C.c_char_p, []),
    "fr_ctx_create": (C.c_int, [C.POINTER(Params), C.POINTER(_P)]),
    "fr_ctx_destroy": (None, [_P]),
    "fr_ctx_set_stream": (C.c_int, [_P, _P]),
    "fr_ctx_sync": (C.c_int, [_P]),
    "fr_ctx_dims": (C.c_int, [_P, _I32P, _I32P, _I32P, _I32P, _I32P]),
    "fr_ctx_set_scratch_limit": (C.c_int, [_P, C.c_uint64]),
    "fr_ctx_set_tune": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "fr_ctx_get_tune": (C.c_int, [_P, C.c_int32, _I32P]),
    "fr_ctx_scratch_info": (C.c_int, [_P, _U64P, _U64P]),
    "fr_ctx_reserve": (C.c_int, [_P, C.c_uint64]),
    "fr_ctx_modulus": (C.c_uint64, [_P, C.c_int32]),
    "fr_keygen": (C.c_int, [_P, C.c_uint64, _I32P, C.c_int32, C.POINTER(_P)]),
    "fr_keys_destroy": (None, [_P]),
    "fr_keys_export": (C.c_int, [_P, _P, C.c_int32, C.c_uint64, _U64P]),
    "fr_encode": (C.c_int, [_P, _DP, C.c_int32, C.c_int32, C.c_double, _CTP]),
    "fr_encode_device": (C.c_int, [_P, _P, C.c_int32, C.c_int32, C.c_double, _CTP]),
    "fr_pt_import": (C.c_int, [_P, _U64P, C.c_int32, C.c_double, _CTP]),
    "fr_pt_export": (C.c_int, [_P, _CTP, _U64P]),
    "fr_encrypt": (C.c_int, [_P, _P, _CTP, C.c_uint64, _CTP]),
    "fr_decrypt": (C.c_int, [_P, _P, _CTP, _CTP]),
    "fr_decode": (C.c_int, [_P, _CTP, _DP, C.c_int32]),
    "fr_ct_import": (C.c_int, [_P, _U64P, C.c_int32, C.c_double, _CTP]),
    "fr_ct_export": (C.c_int, [_P, _CTP, _U64P]),
    "fr_rotate_hoisted": (C.c_int, [_P, _P, _CTP, _I32P, C.c_int32, _CTP]),
    "fr_rescale": (C.c_int, [_P, _CTP, _CTP]),
    "fr_add": (C.c_int, [_P, _CTP, _CTP, _CTP]),
    "fr_sub": (C.c_int, [_P, _CTP, _CTP, _CTP]),
    "fr_mul_plain": (C.c_int, [_P, _CTP, _CTP, _CTP]),
    "fr_mul_relin_rescale": (C.c_int, [_P, _P, _CTP, _CTP, _CTP]),
    "fr_mul_int": (C.c_int, [_P, _CTP, C.c_int64, _CTP]),
    "fr_add_const": (C.c_int, [_P, _CTP, C.c_double, _CTP]),
    "fr_drop_to": (C.c_int, [_P, _CTP, C.c_int32, _CTP]),
    "fr_db_load": (C.c_int, [_P, C.POINTER(C.c_float), C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                             C.c_double, C.POINTER(_P)]),
    "fr_db_import": (C.c_int, [_P, _U64P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                               C.POINTER(_P)]),
    "fr_db_export": (C.c_int, [_P, _P, C.c_int32, C.c_int32, _U64P]),
    "fr_db_extend": (C.c_int, [_P, _P]),
    "fr_bsgs_matvec_hoisted": (C.c_int, [_P, _P, _CTP, _P, C.c_int32, _CTP]),
    "fr_bsgs_matvec_hoisted_batch": (C.c_int, [_P, _P, _CTP, C.c_int32, _P, _I32P, _CTP]),
    "fr_db_groups": (C.c_int, [_P]),
    "fr_db_destroy": (None, [_P]),
    "fr_bsgs_diag_matvec": (C.c_int, [_P, _P, _CTP, C.c_int32, _P, C.c_int32, _CTP]),
    "fr_chebyshev_eval": (C.c_int, [_P, _P, _CTP, _DP, C.c_int32, C.c_int32, _CTP]),
    "fr_rotate_hoisted_batch": (C.c_int, [_P, _P, _CTP, C.c_int32, _I32P, C.c_int32, _CTP]),
    "fr_rotate_hoisted_noalloc": (C.c_int, [_P, _P, _CTP, _I32P, C.c_int32, _CTP]),
    "fr_membership_aggregate": (C.c_int, [_P, _P, _CTP, C.c_int32, _CTP]),
    "fr_tensor_sum_relin_rescale": (C.c_int, [_P, _P, _CTP, _CTP, C.c_int32, _CTP]),
    "fr_rotate_sum": (C.c_int, [_P, _P, _CTP, C.c_int32, C.c_int32, _CTP]),
    "fr_bsgs_encrypted_matvec": (C.c_int, [_P, _P, _CTP, C.c_int32, _CTP, C.c_int32, _CTP]),
    "fr_bsgs_diag_matvec_batch": (C.c_int, [_P, _P, _CTP, C.c_int32, C.c_int32, _P, _I32P, _CTP]),
    "fr_chebyshev_eval_batch": (C.c_int, [_P, _P, _CTP, C.c_int32, _DP, C.c_int32, C.c_int32, _CTP]),
    "fr_moddown_parity": (C.c_int, [_P, C.c_int32, _U64P, _U64P, C.c_int32, _CTP]),
    "fr_graph_begin": (C.c_int, [_P]),
    "fr_graph_end": (C.c_int, [_P, C.POINTER(_P)]),
    "fr_graph_launch": (C.c_int, [_P, _P]),
    "fr_graph_destroy": (None, [_P]),
    "fr_prof_begin": (C.c_int, [_P, C.c_int32]),
    "fr_prof_end": (C.c_int, [_P, _I32P, _DP, _DP]),
    "fr_cheb_step_coeffs": (C.c_int, [C.c_int32, C.c_double, _DP]),
    "fr_cheb_ps_params": (C.c_int, [C.c_int32, _I32P, _I32P]),
    "fr_cheb_out_level": (C.c_int, [C.c_int32, C.c_int32, C.c_int32]),
    "fr_cheb_mult_count": (C.c_int, [C.c_int32, C.c_int32]),
    "fr_stream_pool_size": (C.c_int, [C.c_int32, C.c_double, C.c_double]),
    "fr_bsgs_rotation_set": (C.c_int, [C.c_int32, C.c_int32, _I32P, C.c_int32]),
}


def lib():
    """Load libfrhip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc for gfx950) first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != FR_OK:
        raise FrError(rc, f"{what}: {lib().fr_last_error().decode()}")


def _u64(a: np.ndarray):
    return a.ctypes.data_as(_U64P)


# ---------------------------------------------------------------------------
# host-only helpers
# ---------------------------------------------------------------------------
def cheb_step_coeffs(degree: int, delta: float) -> np.ndarray:
    c = np.zeros(degree + 1)
    _check(lib().fr_cheb_step_coeffs(degree, delta, c.ctypes.data_as(_DP)), "fr_cheb_step_coeffs")
    return c


def cheb_ps_params(degree: int):
    a, b = C.c_int32(), C.c_int32()
    _check(lib().fr_cheb_ps_params(degree, C.byref(a), C.byref(b)), "fr_cheb_ps_params")
    return a.value, b.value


def cheb_out_level(in_level: int, degree: int, d1: int) -> int:
    return lib().fr_cheb_out_level(in_level, degree, d1)


def cheb_mult_count(degree: int, d1: int) -> int:
    return lib().fr_cheb_mult_count(degree, d1)


def stream_pool_size(compute_units: int, free_bytes: float, ct_bytes: float) -> int:
    return lib().fr_stream_pool_size(compute_units, free_bytes, ct_bytes)


def power_of_two_rotations(N: int) -> List[int]:
    """Rotation indices 2^i, i < log2(N/2): the keys of the slot-sum doublings."""
    return [1 << i for i in range(int(N).bit_length() - 2)]


def bsgs_rotation_set(ell: int, n1: int) -> List[int]:
    n = lib().fr_bsgs_rotation_set(ell, n1, None, 0)
    out = (C.c_int32 * max(n, 1))()
    lib().fr_bsgs_rotation_set(ell, n1, out, n)
    return list(out[:n])


# ---------------------------------------------------------------------------
# device objects
# ---------------------------------------------------------------------------
class Ct:
    """A ciphertext in a torch int64 buffer [2][cap+1][N] on the device."""

    def __init__(self, ctx: "Context", cap: int):
        import torch
        self.ctx = ctx
        self.buf = torch.empty((2 * (cap + 1) * ctx.N,), dtype=torch.int64, device=ctx.device)
        self.desc = CtDesc(self.buf.data_ptr(), -1, cap, 0.0)

    @property
    def level(self) -> int:
        return self.desc.level

    @property
    def scale(self) -> float:
        return self.desc.scale

    @property
    def ref(self):
        return C.byref(self.desc)


class Pt(Ct):
    """A plaintext in a torch int64 buffer [cap+1][N] on the device."""

    def __init__(self, ctx: "Context", cap: int):
        import torch
        self.ctx = ctx
        self.buf = torch.empty(((cap + 1) * ctx.N,), dtype=torch.int64, device=ctx.device)
        self.desc = CtDesc(self.buf.data_ptr(), -1, cap, 0.0)


class Keys:
    def __init__(self, ctx, ptr, rots):
        self.ctx, self.ptr, self.rots = ctx, ptr, list(rots)

    def __del__(self):
        try:
            lib().fr_keys_destroy(self.ptr)
        except Exception:
            pass

    def export_secret(self) -> np.ndarray:
        out = np.zeros(self.ctx.N, dtype=np.uint64)
        _check(lib().fr_keys_export(self.ctx.ptr, self.ptr, 0, 0, _u64(out)), "fr_keys_export")
        return out.view(np.int64)

    def export_pk(self) -> np.ndarray:
        c = self.ctx
        out = np.zeros(2 * (c.L + 1) * c.N, dtype=np.uint64)
        _check(lib().fr_keys_export(c.ptr, self.ptr, 1, 0, _u64(out)), "fr_keys_export")
        return out.reshape(2, c.L + 1, c.N)

    def export_ksk(self, kid: int) -> np.ndarray:
        c = self.ctx
        nm = c.L + 1 + c.nP
        out = np.zeros(c.dnum * 2 * nm * c.N, dtype=np.uint64)
        _check(lib().fr_keys_export(c.ptr, self.ptr, 2, kid, _u64(out)), "fr_keys_export")
        return out.reshape(c.dnum, 2, nm, c.N)


class Db:
    def __init__(self, ctx, ptr, ell, B, n1, level, scale):
        self.ctx, self.ptr = ctx, ptr
        self.ell, self.B, self.n1, self.level, self.scale = ell, B, n1, level, scale
        self.G = lib().fr_db_groups(ptr)
        self.extended = False

    def __del__(self):
        try:
            lib().fr_db_destroy(self.ptr)
        except Exception:
            pass

    def export(self, g: int, d: int) -> np.ndarray:
        out = np.zeros((self.level + 1) * self.ctx.N, dtype=np.uint64)
        _check(lib().fr_db_export(self.ctx.ptr, self.ptr, g, d, _u64(out)), "fr_db_export")
        return out.reshape(self.level + 1, self.ctx.N)

    def extend(self) -> "Db":
        """Append every diagonal's residues mod the special primes (needed by
        the hoisted product; idempotent)."""
        _check(lib().fr_db_extend(self.ctx.ptr, self.ptr), "fr_db_extend")
        self.extended = True
        return self


class Graph:
    """A recorded call sequence (fr_graph); launch() replays it on the
    context's stream."""

    def __init__(self, ctx, ptr):
        self.ctx, self.ptr = ctx, ptr

    def launch(self):
        _check(lib().fr_graph_launch(self.ctx.ptr, self.ptr), "fr_graph_launch")

    def __del__(self):
        try:
            lib().fr_graph_destroy(self.ptr)
        except Exception:
            pass


class Context:
    """fr_ctx: parameter set, tables and stream (torch's current stream)."""

    def __init__(self, log_n, q0_bits, n_mid, mid_bits, n_special, special_bits, dnum, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("paper_2604_00546_amd needs a ROCm GPU (gfx950); none is visible")
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        L = lib()
        p = Params(log_n, q0_bits, n_mid, mid_bits, n_special, special_bits, dnum)
        ptr = _P()
        _check(L.fr_ctx_create(C.byref(p), C.byref(ptr)), "fr_ctx_create")
        self.ptr = ptr
        n, l, ns, a, d = (C.c_int32() for _ in range(5))
        L.fr_ctx_dims(ptr, C.byref(n), C.byref(l), C.byref(ns), C.byref(a), C.byref(d))
        self.N, self.L, self.nP, self.alpha, self.dnum = n.value, l.value, ns.value, a.value, d.value
        self.moduli = [int(L.fr_ctx_modulus(ptr, i)) for i in range(self.L + 1 + self.nP)]
        self.q, self.p = self.moduli[: self.L + 1], self.moduli[self.L + 1:]
        self.set_stream()

    def __del__(self):
        try:
            lib().fr_ctx_destroy(self.ptr)
        except Exception:
            pass

    def set_stream(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(lib().fr_ctx_set_stream(self.ptr, C.c_void_p(s.cuda_stream)), "fr_ctx_set_stream")

    def sync(self):
        _check(lib().fr_ctx_sync(self.ptr), "fr_ctx_sync")

    # tuning knobs ------------------------------------------------------------------
    TUNE_KNOBS = {"ntt_fwd_cols4": 0, "ntt_fwd_rows4": 1, "ntt_inv_rows4": 2, "ntt_inv_cols4": 3,
                  "modup_merge": 4, "matvec_chunk": 5, "cheb_chunk": 6, "cheb_sched": 7, "ksmac": 8, "ks_lds": 9}

    def set_tune(self, knob: str, value: int):
        _check(lib().fr_ctx_set_tune(self.ptr, self.TUNE_KNOBS[knob], int(value)), "fr_ctx_set_tune")

    def get_tune(self, knob: str) -> int:
        v = C.c_int32()
        _check(lib().fr_ctx_get_tune(self.ptr, self.TUNE_KNOBS[knob], C.byref(v)), "fr_ctx_get_tune")
        return v.value

    def tune_state(self) -> dict:
        return {k: self.get_tune(k) for k in self.TUNE_KNOBS}

    # device scratch ---------------------------------------------------------------
    def set_scratch_limit(self, nbytes: int):
        """At most nbytes of device scratch (0: no limit); calls beyond it raise FR_ENOMEM."""
        _check(lib().fr_ctx_set_scratch_limit(self.ptr, int(nbytes)), "fr_ctx_set_scratch_limit")

    def scratch_info(self):
        """(bytes allocated now, most bytes one call has used)."""
        a, p = C.c_uint64(), C.c_uint64()
        _check(lib().fr_ctx_scratch_info(self.ptr, C.byref(a), C.byref(p)), "fr_ctx_scratch_info")
        return a.value, p.value

    def reserve(self, nbytes: int):
        _check(lib().fr_ctx_reserve(self.ptr, int(nbytes)), "fr_ctx_reserve")

    # kernel timing hook ------------------------------------------------------
    KERNEL_CLASSES = {"ntt": 1, "modup": 2, "ks_inner": 3, "moddown": 4, "mac": 5, "rescale": 6, "tensor": 7,
                      "elementwise": 8}

    def prof_begin(self, kernel_class: str):
        _check(lib().fr_prof_begin(self.ptr, self.KERNEL_CLASSES[kernel_class]), "fr_prof_begin")

    def prof_end(self):
        n, ms, b = C.c_int32(), C.c_double(), C.c_double()
        _check(lib().fr_prof_end(self.ptr, C.byref(n), C.byref(ms), C.byref(b)), "fr_prof_end")
        return n.value, ms.value, b.value

    # graph capture ------------------------------------------------------------
    def graph_begin(self):
        _check(lib().fr_graph_begin(self.ptr), "fr_graph_begin")

    def graph_end(self) -> Graph:
        ptr = _P()
        _check(lib().fr_graph_end(self.ptr, C.byref(ptr)), "fr_graph_end")
        return Graph(self, ptr)

    def capture(self, fn) -> Graph:
        """Record the device calls fn() makes on this context as one graph."""
        self.graph_begin()
        try:
            fn()
        except Exception:
            try:
                self.graph_end()
            except FrError:
                pass
            raise
        return self.graph_end()

    # parity hook -------------------------------------------------------------
    def moddown_parity(self, mode: int, u, level: int, d=None) -> Ct:
        """mode 0: ModDown(u); 1: Rescale(ModDown(u)); 2: Rescale(d + ModDown(u)),
        u over Q_level U P and d over Q_level in coefficient form, through the
        device paths of the hot path."""
        u = np.ascontiguousarray(u, dtype=np.uint64)
        dd = None if d is None else np.ascontiguousarray(d, dtype=np.uint64)
        out = self.new_ct(level if mode == 0 else level - 1)
        _check(lib().fr_moddown_parity(self.ptr, mode, _u64(u), None if dd is None else _u64(dd), level, out.ref),
               "fr_moddown_parity")
        return out

    # allocation -------------------------------------------------------------
    def new_ct(self, cap: int) -> Ct:
        return Ct(self, cap)

    def new_pt(self, cap: int) -> Pt:
        return Pt(self, cap)

    # keys ------------------------------------------------------------------------
    def keygen(self, seed: int, rots: Sequence[int]) -> Keys:
        r = np.ascontiguousarray(list(rots), dtype=np.int32)
        ptr = _P()
        _check(lib().fr_keygen(self.ptr, seed, r.ctypes.data_as(_I32P), len(r), C.byref(ptr)), "fr_keygen")
        return Keys(self, ptr, rots)

    # encode / encrypt -----------------------------------------------------------------
    def encode(self, z, level: int, scale: float) -> Pt:
        z = np.ascontiguousarray(z, dtype=np.float64)
        pt = self.new_pt(level)
        _check(lib().fr_encode(self.ptr, z.ctypes.data_as(_DP), len(z), level, scale, pt.ref), "fr_encode")
        return pt

    def pt_import(self, coeffs, level: int, scale: float) -> Pt:
        m = np.ascontiguousarray(coeffs, dtype=np.uint64)
        pt = self.new_pt(level)
        _check(lib().fr_pt_import(self.ptr, _u64(m), level, scale, pt.ref), "fr_pt_import")
        return pt

    def pt_export(self, pt: Pt) -> np.ndarray:
        out = np.zeros((pt.level + 1) * self.N, dtype=np.uint64)
        _check(lib().fr_pt_export(self.ptr, pt.ref, _u64(out)), "fr_pt_export")
        return out.reshape(pt.level + 1, self.N)

    def ct_import(self, coeffs, level: int, scale: float) -> Ct:
        m = np.ascontiguousarray(coeffs, dtype=np.uint64)
        ct = self.new_ct(level)
        _check(lib().fr_ct_import(self.ptr, _u64(m), level, scale, ct.ref), "fr_ct_import")
        return ct

    def ct_export(self, ct: Ct) -> np.ndarray:
        out = np.zeros(2 * (ct.level + 1) * self.N, dtype=np.uint64)
        _check(lib().fr_ct_export(self.ptr, ct.ref, _u64(out)), "fr_ct_export")
        return out.reshape(2, ct.level + 1, self.N)

    def encrypt(self, keys: Keys, pt: Pt, seed: int) -> Ct:
        ct = self.new_ct(pt.level)
        _check(lib().fr_encrypt(self.ptr, keys.ptr, pt.ref, seed, ct.ref), "fr_encrypt")
        return ct

    def decrypt(self, keys: Keys, ct: Ct) -> Pt:
        pt = self.new_pt(ct.level)
        _check(lib().fr_decrypt(self.ptr, keys.ptr, ct.ref, pt.ref), "fr_decrypt")
        return pt

    def decode(self, pt: Pt, n: int | None = None) -> np.ndarray:
        n = self.N // 2 if n is None else n
        out = np.zeros(n, dtype=np.float64)
        _check(lib().fr_decode(self.ptr, pt.ref, out.ctypes.data_as(_DP), n), "fr_decode")
        return out

    def decrypt_decode(self, keys: Keys, ct: Ct, n: int | None = None) -> np.ndarray:
        return self.decode(self.decrypt(keys, ct), n)

    # homomorphic ops ----------------------------------------------------------------------
    def rotate_hoisted(self, keys: Keys, ct: Ct, rots: Sequence[int], outs: List[Ct] | None = None) -> List[Ct]:
        rots = list(rots)
        if outs is None:
            outs = [self.new_ct(ct.level) for _ in rots]
        arr = (CtDesc * len(rots))(*[o.desc for o in outs])
        r = np.ascontiguousarray(rots, dtype=np.int32)
        _check(lib().fr_rotate_hoisted(self.ptr, keys.ptr, ct.ref, r.ctypes.data_as(_I32P), len(r), arr),
               "fr_rotate_hoisted")
        for o, d in zip(outs, arr):
            o.desc.level, o.desc.scale = d.level, d.scale
        return outs

    def rotate_hoisted_noalloc(self, keys: Keys, ct: Ct, rots: Sequence[int],
                               outs: List[Ct] | None = None) -> List[Ct]:
        """fr_rotate_hoisted with the library's fixed per-GPU scratch array (no device allocation)."""
        rots = list(rots)
        if outs is None:
            outs = [self.new_ct(ct.level) for _ in rots]
        arr = (CtDesc * max(len(rots), 1))(*[o.desc for o in outs])
        r = np.ascontiguousarray(rots, dtype=np.int32)
        _check(lib().fr_rotate_hoisted_noalloc(self.ptr, keys.ptr, ct.ref, r.ctypes.data_as(_I32P), len(r), arr),
               "fr_rotate_hoisted_noalloc")
        for o, d in zip(outs, arr):
            o.desc.level, o.desc.scale = d.level, d.scale
        return outs

    def rotate_hoisted_batch(self, keys: Keys, cts: Sequence[Ct], rots: Sequence[int],
                             outs: List[List[Ct]] | None = None) -> List[List[Ct]]:
        """outs[q][r] = Rot_{rots[r]}(cts[q]); one key read per rotation for the whole batch."""
        rots, cts = list(rots), list(cts)
        if outs is None:
            outs = [[self.new_ct(ct.level) for _ in rots] for ct in cts]
        ins = (CtDesc * len(cts))(*[c.desc for c in cts])
        flat = [o for row in outs for o in row]
        arr = (CtDesc * max(len(flat), 1))(*[o.desc for o in flat])
        r = np.ascontiguousarray(rots, dtype=np.int32)
        _check(lib().fr_rotate_hoisted_batch(self.ptr, keys.ptr, ins, len(cts), r.ctypes.data_as(_I32P), len(r),
                                             arr), "fr_rotate_hoisted_batch")
        for o, d in zip(flat, arr):
            o.desc.level, o.desc.scale = d.level, d.scale
        return outs

    def rescale(self, ct: Ct) -> Ct:
        out = self.new_ct(max(ct.level - 1, 0))
        _check(lib().fr_rescale(self.ptr, ct.ref, out.ref), "fr_rescale")
        return out

    def add(self, a: Ct, b: Ct) -> Ct:
        out = self.new_ct(a.level)
        _check(lib().fr_add(self.ptr, a.ref, b.ref, out.ref), "fr_add")
        return out

    def sub(self, a: Ct, b: Ct) -> Ct:
        out = self.new_ct(a.level)
        _check(lib().fr_sub(self.ptr, a.ref, b.ref, out.ref), "fr_sub")
        return out

    def mul_plain(self, a: Ct, p: Pt) -> Ct:
        out = self.new_ct(min(a.level, p.level))
        _check(lib().fr_mul_plain(self.ptr, a.ref, p.ref, out.ref), "fr_mul_plain")
        return out

    def mul_relin_rescale(self, keys: Keys, a: Ct, b: Ct) -> Ct:
        out = self.new_ct(max(a.level - 1, 0))
        _check(lib().fr_mul_relin_rescale(self.ptr, keys.ptr, a.ref, b.ref, out.ref), "fr_mul_relin_rescale")
        return out

    def mul_int(self, a: Ct, k: int) -> Ct:
        out = self.new_ct(a.level)
        _check(lib().fr_mul_int(self.ptr, a.ref, k, out.ref), "fr_mul_int")
        return out

    def add_const(self, a: Ct, c: float) -> Ct:
        out = self.new_ct(a.level)
        _check(lib().fr_add_const(self.ptr, a.ref, c, out.ref), "fr_add_const")
        return out

    def drop_to(self, a: Ct, level: int) -> Ct:
        out = self.new_ct(level)
        _check(lib().fr_drop_to(self.ptr, a.ref, level, out.ref), "fr_drop_to")
        return out

    # database / matvec / chebyshev -------------------------------------------------------------
    def db_load(self, T, ell: int, B: int, n1: int, level: int, scale: float) -> Db:
        T = np.ascontiguousarray(T, dtype=np.float32)
        ptr = _P()
        _check(lib().fr_db_load(self.ptr, T.ctypes.data_as(C.POINTER(C.c_float)), T.shape[0], ell, B, n1, level,
                                scale, C.byref(ptr)), "fr_db_load")
        return Db(self, ptr, ell, B, n1, level, scale)

    def db_import(self, coeffs, G: int, ell: int, B: int, n1: int, level: int, scale: float) -> Db:
        m = np.ascontiguousarray(coeffs, dtype=np.uint64)
        ptr = _P()
        _check(lib().fr_db_import(self.ptr, _u64(m), G, ell, B, n1, level, scale, C.byref(ptr)), "fr_db_import")
        return Db(self, ptr, ell, B, n1, level, scale)

    def bsgs_diag_matvec(self, keys: Keys, baby: Sequence[Ct], db: Db, group: int, out: Ct | None = None) -> Ct:
        arr = (CtDesc * len(baby))(*[b.desc for b in baby])
        if out is None:
            out = self.new_ct(max(min(baby[0].level, db.level) - 1, 0))
        _check(lib().fr_bsgs_diag_matvec(self.ptr, keys.ptr, arr, len(baby), db.ptr, group, out.ref),
               "fr_bsgs_diag_matvec")
        return out

    def bsgs_diag_matvec_batch(self, keys: Keys, babies: Sequence[Sequence[Ct]], db, group=0,
                               outs: List[Ct] | None = None) -> List[Ct]:
        """babies[q] = the n1 baby steps of query q; db / group: one database
        and group for every query, or one per query.  One score ciphertext
        per query."""
        nq, n1 = len(babies), len(babies[0])
        dbs = list(db) if isinstance(db, (list, tuple)) else [db] * nq
        grp = np.ascontiguousarray(list(group) if isinstance(group, (list, tuple)) else [group] * nq,
                                   dtype=np.int32)
        flat = [b for row in babies for b in row]
        arr = (CtDesc * len(flat))(*[b.desc for b in flat])
        if outs is None:
            outs = [self.new_ct(max(min(row[0].level, d.level) - 1, 0)) for row, d in zip(babies, dbs)]
        oarr = (CtDesc * nq)(*[o.desc for o in outs])
        dptr = (C.c_void_p * nq)(*[d.ptr for d in dbs])
        _check(lib().fr_bsgs_diag_matvec_batch(self.ptr, keys.ptr, arr, nq, n1, dptr, grp.ctypes.data_as(_I32P),
                                               oarr), "fr_bsgs_diag_matvec_batch")
        for o, d in zip(outs, oarr):
            o.desc.level, o.desc.scale = d.level, d.scale
        return outs

    def bsgs_matvec_hoisted(self, keys: Keys, query: Ct, db: Db, group: int = 0, out: Ct | None = None) -> Ct:
        """Score ciphertext from the query itself, baby steps held over Q_l U P
        (db extended)."""
        if out is None:
            out = self.new_ct(max(query.level - 1, 0))
        _check(lib().fr_bsgs_matvec_hoisted(self.ptr, keys.ptr, query.ref, db.ptr, group, out.ref),
               "fr_bsgs_matvec_hoisted")
        return out

    def bsgs_matvec_hoisted_batch(self, keys: Keys, queries: Sequence[Ct], db, group=0,
                                  outs: List[Ct] | None = None) -> List[Ct]:
        """One score ciphertext per query; db / group: one for all, or one per query."""
        queries = list(queries)
        nq = len(queries)
        dbs = list(db) if isinstance(db, (list, tuple)) else [db] * nq
        grp = np.ascontiguousarray(list(group) if isinstance(group, (list, tuple)) else [group] * nq,
                                   dtype=np.int32)
        arr = (CtDesc * nq)(*[q.desc for q in queries])
        if outs is None:
            outs = [self.new_ct(max(q.level - 1, 0)) for q in queries]
        oarr = (CtDesc * nq)(*[o.desc for o in outs])
        dptr = (C.c_void_p * nq)(*[d.ptr for d in dbs])
        _check(lib().fr_bsgs_matvec_hoisted_batch(self.ptr, keys.ptr, arr, nq, dptr, grp.ctypes.data_as(_I32P),
                                                  oarr), "fr_bsgs_matvec_hoisted_batch")
        for o, d in zip(outs, oarr):
            o.desc.level, o.desc.scale = d.level, d.scale
        return outs

    def chebyshev_eval_batch(self, keys: Keys, cts: Sequence[Ct], coeffs, d1: int,
                             outs: List[Ct] | None = None) -> List[Ct]:
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        cts = list(cts)
        if outs is None:
            outs = [self.new_ct(max(cheb_out_level(ct.level, len(c) - 1, d1), 0)) for ct in cts]
        ins = (CtDesc * len(cts))(*[x.desc for x in cts])
        oarr = (CtDesc * len(outs))(*[o.desc for o in outs])
        _check(lib().fr_chebyshev_eval_batch(self.ptr, keys.ptr, ins, len(cts), c.ctypes.data_as(_DP), len(c) - 1,
                                             d1, oarr), "fr_chebyshev_eval_batch")
        for o, d in zip(outs, oarr):
            o.desc.level, o.desc.scale = d.level, d.scale
        return outs

    def tensor_sum_relin_rescale(self, keys: Keys, a: Sequence[Ct], b: Sequence[Ct], out: Ct | None = None) -> Ct:
        """Rescale(Relin(sum_k a[k] (x) b[k])): the encrypted-database product."""
        a, b = list(a), list(b)
        if out is None:
            out = self.new_ct(max(a[0].level - 1, 0))
        pa = (CtDesc * len(a))(*[x.desc for x in a])
        pb = (CtDesc * len(b))(*[x.desc for x in b])
        _check(lib().fr_tensor_sum_relin_rescale(self.ptr, keys.ptr, pa, pb, len(a), out.ref),
               "fr_tensor_sum_relin_rescale")
        return out

    def rotate_sum(self, keys: Keys, cts: Sequence[Ct], stride: int, out: Ct | None = None) -> Ct:
        """cts[0] + sum_{j >= 1} Rot_{j stride}(cts[j]), one shared ModDown."""
        cts = list(cts)
        if out is None:
            out = self.new_ct(cts[0].level)
        ins = (CtDesc * len(cts))(*[x.desc for x in cts])
        _check(lib().fr_rotate_sum(self.ptr, keys.ptr, ins, len(cts), stride, out.ref), "fr_rotate_sum")
        return out

    def bsgs_encrypted_matvec(self, keys: Keys, baby: Sequence[Ct], diag: Sequence[Ct],
                              out: Ct | None = None) -> Ct:
        """BSGS product with pre-rotated encrypted diagonals: one
        relinearisation per giant step, then the giant rotate-sum."""
        baby, diag = list(baby), list(diag)
        if out is None:
            out = self.new_ct(max(baby[0].level - 1, 0))
        pb = (CtDesc * len(baby))(*[x.desc for x in baby])
        pd = (CtDesc * len(diag))(*[x.desc for x in diag])
        _check(lib().fr_bsgs_encrypted_matvec(self.ptr, keys.ptr, pb, len(baby), pd, len(diag), out.ref),
               "fr_bsgs_encrypted_matvec")
        return out

    def membership_aggregate(self, keys: Keys, cts: Sequence[Ct], out: Ct | None = None) -> Ct:
        """Sum of the inputs, then the sum of all slots in every slot."""
        cts = list(cts)
        if out is None:
            out = self.new_ct(cts[0].level)
        ins = (CtDesc * len(cts))(*[x.desc for x in cts])
        _check(lib().fr_membership_aggregate(self.ptr, keys.ptr, ins, len(cts), out.ref), "fr_membership_aggregate")
        return out

    def chebyshev_eval(self, keys: Keys, ct: Ct, coeffs, d1: int, out: Ct | None = None) -> Ct:
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        if out is None:
            out = self.new_ct(max(cheb_out_level(ct.level, len(c) - 1, d1), 0))
        _check(lib().fr_chebyshev_eval(self.ptr, keys.ptr, ct.ref, c.ctypes.data_as(_DP), len(c) - 1, d1, out.ref),
               "fr_chebyshev_eval")
        return out


def small_params():
    """N = 2^12; Q = one 50-bit + two 40-bit primes; P = one 60-bit prime; dnum 3."""
    return dict(log_n=12, q0_bits=50, n_mid=2, mid_bits=40, n_special=1, special_bits=60, dnum=3)


def deep_small_params():
    """N = 2^12 with the paper-scale modulus chain (room for the Chebyshev ladder)."""
    return dict(log_n=12, q0_bits=60, n_mid=14, mid_bits=40, n_special=5, special_bits=60, dnum=3)


def paper_params():
    """N = 2^16; Q = one 60-bit + fourteen 40-bit primes; P = five 60-bit primes; dnum 3."""
    return dict(log_n=16, q0_bits=60, n_mid=14, mid_bits=40, n_special=5, special_bits=60, dnum=3)
