"""Integer VALU issue rates of the GPU (denominator of the NTT roofline).

Runs the probes of csrc/microbench.hip: 8 independent chains per thread of
one instruction kind, on a grid that covers every compute unit many times,
and prints instructions (or 64-bit Shoup modular multiplies) per second,
per compute unit per clock at 2.4 GHz, and per lane per clock.

usage: python -m paper_2604_00546_amd.microbench
"""
import ctypes as C
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KINDS = {0: "v_mad_u64_u32", 1: "v_mul_hi_u32", 2: "v_mul_lo_u32", 3: "v_add_u32", 4: "shoup_modmul_u64"}
CUS, CLOCK = 256, 2.4e9


def run(iters: int = 4096, blocks: int = 256 * 32) -> dict:
    lib = C.CDLL(os.path.join(HERE, "libfrmb.so"))
    lib.fr_mb_run.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double)]
    out = {}
    for k, name in KINDS.items():
        ms = C.c_double()
        rc = lib.fr_mb_run(k, iters, blocks, C.byref(ms))
        if rc:
            raise RuntimeError(f"probe {name} failed ({rc})")
        ops = 8.0 * iters * blocks * 256
        rate = ops / (ms.value * 1e-3)
        out[name] = {"ops_per_s": rate, "per_cu_per_clk": rate / (CUS * CLOCK),
                     "per_lane_per_clk": rate / (CUS * CLOCK * 64), "ms": ms.value}
    return out


if __name__ == "__main__":
    print(json.dumps(run(), indent=1))
