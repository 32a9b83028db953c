// microbench.hip -- issue-rate probes for the integer VALU of gfx950, the
// denominator of the NTT's arithmetic roofline.  Each thread runs 8
// independent dependency chains of one instruction kind for `iters`
// iterations; the grid covers every compute unit many times over.
//   kind 0: v_mad_u64_u32   acc = (u64)x * y + acc
//   kind 1: v_mul_hi_u32    x = mulhi(x, y) ^ c
//   kind 2: v_mul_lo_u32    x = x * y + c   (32-bit)
//   kind 3: v_add_u32       x = x + y
//   kind 4: 64-bit Shoup modular multiply  x = x * w - mulhi64(x, wp) * q
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kT = 256;

template <int KIND>
__global__ __launch_bounds__(kT) void k_probe(uint64_t *out, int iters, uint32_t y, uint64_t w, uint64_t wp,
                                              uint64_t q) {
    const uint32_t t = blockIdx.x * kT + threadIdx.x;
    uint64_t a[8];
    uint32_t b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = t * 7919u + j;
        b[j] = t * 104729u + 3u * j + 1u;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (KIND == 0) {
                uint64_t cc;
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(a[j]), "=s"(cc) : "v"(b[j]), "v"(y));
            }
            if (KIND == 1) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(b[j]) : "v"(y));
            if (KIND == 2) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(b[j]) : "v"(y));
            if (KIND == 3) asm volatile("v_add_u32 %0, %0, %1" : "+v"(b[j]) : "v"(y));
            if (KIND == 4) a[j] = a[j] * w - __umul64hi(a[j], wp) * q;
        }
    }
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j] + b[j];
    out[t] = s;
}

}  // namespace

extern "C" int fr_mb_run(int kind, int iters, int blocks, double *ms_out) {
    uint64_t *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * kT * 8) != hipSuccess) return -1;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const uint64_t q = 0xFFFFFFFFFFC0001ull, w = 0x123456789ABCull, wp = 0x1234567ull;
    for (int rep = 0; rep < 2; ++rep) {
        (void)hipEventRecord(e0, 0);
        switch (kind) {
            case 0: hipLaunchKernelGGL(k_probe<0>, dim3(blocks), dim3(kT), 0, 0, out, iters, 0x9E3779B9u, w, wp, q); break;
            case 1: hipLaunchKernelGGL(k_probe<1>, dim3(blocks), dim3(kT), 0, 0, out, iters, 0x9E3779B9u, w, wp, q); break;
            case 2: hipLaunchKernelGGL(k_probe<2>, dim3(blocks), dim3(kT), 0, 0, out, iters, 0x9E3779B9u, w, wp, q); break;
            case 3: hipLaunchKernelGGL(k_probe<3>, dim3(blocks), dim3(kT), 0, 0, out, iters, 0x9E3779B9u, w, wp, q); break;
            default: hipLaunchKernelGGL(k_probe<4>, dim3(blocks), dim3(kT), 0, 0, out, iters, 0x9E3779B9u, w, wp, q); break;
        }
        (void)hipEventRecord(e1, 0);
        (void)hipEventSynchronize(e1);
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *ms_out = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
