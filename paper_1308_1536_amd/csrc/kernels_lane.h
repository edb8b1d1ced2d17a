// kernels_lane.h -- the limb products of the trailing update (Algorithm 1
// step 2.2.2) on the VALU path with one lane per element, for P <= kLaneMaxP
// limbs with P a multiple of 4.
//
// A workgroup of kLaneRows waves owns kLaneRows rows i and kLaneFT = 64
// consecutive columns j of the trailing block.  The pivot-row limbs u_kj of
// those columns are shared by every row: the workgroup copies them into LDS
// limb-major (row x holds limb x of the 64 elements, rows padded to 65 words
// so the per-lane reads are free of bank conflicts), and each wave copies its
// multiplier l_i into a broadcast buffer.  Each lane then forms l_i u_j by
// column (Comba) accumulation: output columns r are taken eight at a time,
// every multiplier limb l[a] is multiplied into a window of eight pivot-row
// limbs u[r+c-a] that slides by one limb per step, and each column keeps a
// 96-bit sum of 32x32->64 products (v_mad_u64_u32 with its carry out, folded
// by v_addc_co_u32).  Zero rows below limb 0 and above limb P-1 let the
// window run over the band's edges without bounds checks.
//
// The product's top limbs P-1 .. 2P-1 go to the same record buffer, in the
// same limb-major layout, as the MFMA path's epilogue writes, and the same
// finish kernel forms a_ij = RZ_p(a_ij - RZ_p(l_i u_j)).
#pragma once

#include "kernels_mfma.h"

namespace mpk {

constexpr int kLaneMaxP = 128;
constexpr int kLaneFT = 64;    // columns per workgroup (one per lane)
constexpr int kLaneRows = 4;   // rows per workgroup (one per wave)
constexpr int kLaneW = 8;      // product columns per Comba block
constexpr int kPadLo = 8;      // zero tile rows below limb 0 ...
constexpr int kPadHi = 8;      // ... and above limb P-1, read instead of clamping

__host__ __device__ inline bool lane_update_ok(int P) { return P <= kLaneMaxP && P % 4 == 0; }
__host__ __device__ inline size_t lane_lds_bytes(int P) {
    return ((size_t)(P + kPadLo + kPadHi) * (kLaneFT + 1) + (size_t)kLaneRows * P) * 4u;
}
// workgroups for an m x m trailing block
__host__ __device__ inline int64_t lane_update_blocks(int64_t m) {
    return ((m + kLaneRows - 1) / kLaneRows) * ((m + kLaneFT - 1) / kLaneFT);
}

// s_c + h_c 2^64 += x y_c for c = 0..3: v_mad_u64_u32 adds the 64-bit
// accumulator in the same instruction and reports the carry out of bit 63,
// which v_addc_co_u32 folds into the high word
__device__ __forceinline__ void mac96x4(uint64_t (&s)[4], uint32_t (&h)[4], uint32_t x, const uint32_t (&y)[4]) {
    uint64_t c0, c1, c2, c3;
    asm volatile(
        "v_mad_u64_u32 %0, %8, %12, %13, %0\n\t"
        "v_mad_u64_u32 %1, %9, %12, %14, %1\n\t"
        "v_mad_u64_u32 %2, %10, %12, %15, %2\n\t"
        "v_mad_u64_u32 %3, %11, %12, %16, %3\n\t"
        "v_addc_co_u32_e64 %4, %8, 0, %4, %8\n\t"
        "v_addc_co_u32_e64 %5, %9, 0, %5, %9\n\t"
        "v_addc_co_u32_e64 %6, %10, 0, %6, %10\n\t"
        "v_addc_co_u32_e64 %7, %11, 0, %7, %11"
        : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(h[0]), "+v"(h[1]), "+v"(h[2]), "+v"(h[3]),
          "=&s"(c0), "=&s"(c1), "=&s"(c2), "=&s"(c3)
        : "v"(x), "v"(y[0]), "v"(y[1]), "v"(y[2]), "v"(y[3]));
}

// The record of element (i', j') (i' = i - k - 1, j' = j - k - 1) is word x
// at T[((i' njb + j' / 32) TP + x) 32 + j' % 32], x = 0..P: product limb P-1+x.
__device__ __forceinline__ void prod_lane_body(uint32_t *lds, MatDev A, uint32_t *T, const int32_t *info, int64_t k,
                                               int64_t n, int P, int64_t bx) {
    if (*info != 0) return;
    const int64_t m = n - k - 1;
    const int FT = kLaneFT, FTP = FT + 1;
    const int64_t ncol = (m + FT - 1) / FT;
    const int64_t rg = bx / ncol, j0 = (bx % ncol) * FT;
    if (rg * kLaneRows >= m) return;  // uniform over the workgroup
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = mpw::lane();
    const int64_t ip = rg * kLaneRows + wave;
    const int cnt = (int)min((int64_t)FT, m - j0);
    // tile rows -kPadLo .. P+kPadHi-1 of FTP words (limb x of element e at
    // row x, column e; rows outside 0..P-1 hold zeros)
    uint32_t *tile = lds + kPadLo * FTP;
    uint32_t *lsh = lds + (size_t)(P + kPadLo + kPadHi) * FTP + wave * P;  // this wave's multiplier
    const bool row_ok = ip < m;
    const uint32_t *lm = el(A, k + 1 + (row_ok ? ip : 0), k, P);
    for (int q = lane; q < P; q += MP_WAVE) lsh[q] = lm[q];
    {
        const int nt = (int)blockDim.x, tid = (int)threadIdx.x;
        for (int z = tid; z < kPadLo * FTP; z += nt) lds[z] = 0u;
        for (int z = tid; z < kPadHi * FTP; z += nt) tile[P * FTP + z] = 0u;
        // pivot-row limbs of the tile (cnt * P contiguous words) by the whole
        // workgroup, 8 loads per thread in flight; word w is limb w mod P of
        // element w / P, and for w < 2^13, P <= 128 the quotient is
        // (w * magic) >> 24 exactly.  Columns cnt..63 are never read.
        const uint32_t *urow = el(A, k, k + 1 + j0, P);
        const int nw = cnt * P;
        const uint32_t magic = (1u << 24) / (uint32_t)P + 1u;
        for (int w0 = 0; w0 < nw; w0 += 8 * nt) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = urow[min(w0 + u * nt + tid, nw - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int w = w0 + u * nt + tid;
                if (w < nw) {
                    const int ee = (int)(((uint64_t)w * magic) >> 24);
                    tile[(w - ee * P) * FTP + ee] = v[u];
                }
            }
        }
    }
    __syncthreads();
    const int e = lane;
    if (!row_ok || e >= cnt || lm[P - 1] == 0u) return;
    const int64_t jp = j0 + e;
    if (el(A, k, k + 1 + jp, P)[P - 1] == 0u) return;  // u_j = 0: a_ij is left as it is
    const int64_t njb = (m + 31) / 32;
    const int TP = mfma_geom(P).TP;
    uint32_t *rec = T + (ip * njb + jp / 32) * (int64_t)TP * 32 + (jp % 32);

    const uint32_t *col = tile + e;  // limb x at col[x * FTP], -kPadLo <= x < P + kPadHi
    uint64_t carry = 0;              // carry into the next column (< 2^40)
    constexpr int W = kLaneW;
    for (int r0 = 0; r0 < 2 * P; r0 += W) {
        const int alo = max(0, r0 - P + 1), ahi = min(r0 + W - 1, P - 1);
        // window w_c = u[r0 + c - a] at a = alo; r0 + c - alo <= P - 1 + c
        uint32_t wv[W];
#pragma unroll
        for (int c = 0; c < W; ++c) wv[c] = col[(r0 + c - alo) * FTP];
        uint64_t s[W];
        uint32_t h[W];
#pragma unroll
        for (int c = 0; c < W; ++c) {
            s[c] = 0;
            h[c] = 0;
        }
        // one step at a: multiply l[a] into the window, then slide it down by
        // one limb, u[r0 - a - 1] entering (>= -W: a zero pad row below limb 0)
        auto step = [&](uint32_t la, uint32_t vn) __attribute__((always_inline)) {
            uint64_t(&s0)[4] = *reinterpret_cast<uint64_t(*)[4]>(&s[0]);
            uint64_t(&s1)[4] = *reinterpret_cast<uint64_t(*)[4]>(&s[4]);
            uint32_t(&h0)[4] = *reinterpret_cast<uint32_t(*)[4]>(&h[0]);
            uint32_t(&h1)[4] = *reinterpret_cast<uint32_t(*)[4]>(&h[4]);
            const uint32_t(&w0)[4] = *reinterpret_cast<const uint32_t(*)[4]>(&wv[0]);
            const uint32_t(&w1)[4] = *reinterpret_cast<const uint32_t(*)[4]>(&wv[4]);
            mac96x4(s0, h0, la, w0);
            mac96x4(s1, h1, la, w1);
#pragma unroll
            for (int c = W - 1; c > 0; --c) wv[c] = wv[c - 1];
            wv[0] = vn;
        };
        const uint32_t *urd = col + (r0 - alo - 1) * FTP;  // row of the limb entering at step alo
        // groups of four steps, ping-pong buffered: a group's LDS reads are
        // issued while the previous group computes
        int a = alo;
        uint32_t la[4], ua[4], lb[4], ubf[4];
        auto load4 = [&](uint32_t (&l)[4], uint32_t (&u)[4], int a0) __attribute__((always_inline)) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                l[t] = lsh[a0 + t];
                u[t] = urd[-(a0 - alo + t) * FTP];
            }
        };
        auto run4 = [&](const uint32_t (&l)[4], const uint32_t (&u)[4]) __attribute__((always_inline)) {
#pragma unroll
            for (int t = 0; t < 4; ++t) step(l[t], u[t]);
        };
        const int nfull = (ahi + 1 - alo) / 4;  // full groups
        int g = 0;
        if (nfull > 0) {
            load4(la, ua, a);
            for (; g + 2 < nfull; g += 2, a += 8) {
                load4(lb, ubf, a + 4);
                run4(la, ua);
                load4(la, ua, a + 8);
                run4(lb, ubf);
            }
            if (g + 1 < nfull) {
                load4(lb, ubf, a + 4);
                run4(la, ua);
                run4(lb, ubf);
                a += 8;
            } else {
                run4(la, ua);
                a += 4;
            }
        }
        for (; a <= ahi; ++a) step(lsh[a], urd[-(a - alo) * FTP]);
        // resolve the W columns; the record keeps limbs P-1 .. 2P-1
#pragma unroll
        for (int c = 0; c < W; ++c) {
            const int r = r0 + c;
            const uint64_t lo = s[c] + carry;
            const uint32_t hi = h[c] + (lo < s[c] ? 1u : 0u);
            carry = (lo >> 32) | ((uint64_t)hi << 32);
            const int x = r - (P - 1);
            if (x >= 0 && r < 2 * P) rec[(int64_t)x * 32] = (uint32_t)lo;
        }
    }
}

__global__ void __launch_bounds__(64 * kLaneRows) k_prod_lane(MatDev A, uint32_t *T, const int32_t *info, int64_t k,
                                                              int64_t n, int P) {
    extern __shared__ uint32_t lds_raw[];
    prod_lane_body(lds_raw, A, T, info, k, n, P, flat_block());
}

}  // namespace mpk
