// peaks.h -- throughput probes for the two arithmetic units the trailing
// update runs on, so rooflines can be quoted against measured rates as well
// as published ones.  Each thread runs a fixed number of iterations of
// independent instruction chains and writes one checksum word (so nothing is
// optimised away); no other memory is touched.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpk {

// 8 independent chains of v_mad_u64_u32 (32x32->64 multiply, 64-bit add,
// carry out) per lane: 8 * iters multiply-adds per thread
__global__ void __launch_bounds__(256) k_peak_mad64(uint32_t iters, uint32_t seed, uint32_t *out) {
    uint64_t acc[8];
    uint32_t x = seed + threadIdx.x, y = seed * 2654435761u + blockIdx.x;
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = (uint64_t)(x + c) << 17;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            uint64_t cc;
            asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[c]), "=s"(cc) : "v"(x), "v"(y));
        }
    }
    uint64_t s = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s ^= acc[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(s ^ (s >> 32));
}

typedef int p4i __attribute__((ext_vector_type(4)));
typedef int p16i __attribute__((ext_vector_type(16)));

// 8 independent accumulator chains of v_mfma_i32_32x32x32_i8 per wave:
// 8 * iters * 32768 int8 multiply-adds per wave.  clk (may be null): the
// first wave of block 0 stores its shader-clock counter (s_memtime) and the
// constant 100 MHz counter (s_memrealtime) before and after its loop, which
// gives the clock the matrix cores ran at.
__global__ void __launch_bounds__(256) k_peak_mfma_i8(uint32_t iters, uint32_t seed, uint32_t *out, uint64_t *clk) {
    p16i acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = (p16i){0};
    const int v = (int)(seed + threadIdx.x);
    p4i a = {v, v + 1, v + 2, v + 3}, b = {v ^ 5, v ^ 7, v ^ 9, v ^ 11};
    const bool timer = clk != nullptr && blockIdx.x == 0 && threadIdx.x < 64;
    uint64_t t0 = 0, r0 = 0;
    if (timer) {
        t0 = __builtin_amdgcn_s_memtime();
        r0 = __builtin_amdgcn_s_memrealtime();
    }
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[c], 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) s ^= acc[c][r];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)s;
    if (timer) {
        // the loop's results are stored first, so the end stamps follow it
        const uint64_t t1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
        if (threadIdx.x == 0) {
            clk[0] = t0;
            clk[1] = t1;
            clk[2] = r0;
            clk[3] = r1;
        }
    }
}

}  // namespace mpk
