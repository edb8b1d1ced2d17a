// kernels_lane.h -- the limb products of the trailing update (Algorithm 1
// step 2.2.2) on the VALU path with one lane per element, for P <= kLaneMaxP
// limbs with P a multiple of 4.
//
// A workgroup of kLaneRows waves owns kLaneRows rows i and kLaneFT = 64
// consecutive columns j of the trailing block.  The product is formed in
// radix 2^28: both operands are cut into ND = ceil(32P / 28) digits of 28
// bits, so a digit product is below 2^56 and a whole column sum of at most ND
// <= 147 products stays below 2^64 -- one 64-bit accumulator per column and
// no carry handling inside the accumulation (v_mad_u64_u32 only).  The
// pivot-row digits of the workgroup's 64 columns sit in LDS digit-major (row d
// holds digit d of the 64 elements, rows padded to 65 words so the per-lane
// reads are free of bank conflicts); each wave keeps its multiplier's digits
// in a broadcast buffer.  Each lane forms l_i u_j by column (Comba)
// accumulation: output columns r are taken eight at a time, every multiplier
// digit l[a] is multiplied into a window of eight pivot-row digits u[r+c-a]
// that slides by one digit per step.  Zero rows below digit 0 and above digit
// ND-1 let the window run over the band's edges without bounds checks.  The
// column sums are then carried in radix 2^28 and repacked into 32-bit limbs.
//
// The product's top limbs P-1 .. 2P-1 go to the same record buffer, in the
// same limb-major layout, as the MFMA path's epilogue writes, and the same
// finish kernel forms a_ij = RZ_p(a_ij - RZ_p(l_i u_j)).
//
// Only those limbs are kept, so the columns below c0 = lane_short_start(P)
// are not formed at all (a truncated, or "short", product: about 47% fewer
// multiply-adds at P = 128).  What they would add, E = sum_{r < c0} s_r
// 2^(28r), is below ND 2^56 2^(28 c0) / (2^28 - 1) < 2^(28 c0 + 36), so the
// kept limbs of the sum from c0 up are exact unless every bit of it from
// 28 c0 + 36 up to bit 32 (P - 1) is a one (a carry out of E could then run
// into limb P-1).  c0 leaves at least 32 such guard bits; when a lane finds
// them all ones the wave forms the whole product again from column 0.
#pragma once

#include "kernels_mfma.h"

namespace mpk {

constexpr int kLaneMaxP = 128;
constexpr int kLaneFT = 64;    // columns per workgroup (one per lane)
constexpr int kLaneRows = 4;   // rows per workgroup (one per wave): the default of 2, 4 or 8
constexpr int kLaneW = 8;      // product columns per Comba block
constexpr int kDigit = 28;     // bits per digit of the product
constexpr int kPadLo = 24;     // zero tile rows below digit 0 ...
constexpr int kPadHi = 8;      // ... and above digit ND-1, read instead of clamping
constexpr int kPadL = 16;      // zero multiplier digits above digit ND-1

__host__ __device__ inline bool lane_update_ok(int P) { return P <= kLaneMaxP && P % 4 == 0; }
__host__ __device__ inline int lane_digits(int P) { return (32 * P + kDigit - 1) / kDigit; }
__host__ __device__ inline size_t lane_lds_bytes(int P, int rows = kLaneRows) {
    const int nd = lane_digits(P);
    return ((size_t)(nd + kPadLo + kPadHi) * (kLaneFT + 1) + (size_t)rows * (nd + kPadL)) * 4u;
}
// first product column formed (0: the whole product): the largest c0 with
// 28 c0 + 36 + 32 <= 32 (P - 1), when that skips at least one Comba block
__host__ __device__ inline int lane_short_start(int P) {
    const int c0 = (32 * (P - 1) - 36 - 32) / kDigit;
    return c0 >= kLaneW ? c0 : 0;
}
// workgroups for an mr x mc block (an m x m trailing block: mr = mc = m)
__host__ __device__ inline int64_t lane_update_blocks(int64_t mr, int64_t mc, int rows = kLaneRows) {
    return ((mr + rows - 1) / rows) * ((mc + kLaneFT - 1) / kLaneFT);
}
__host__ __device__ inline int64_t lane_update_blocks(int64_t m) { return lane_update_blocks(m, m); }

// digit d (bits 28d .. 28d+27) of a P-limb mantissa
__device__ __forceinline__ uint32_t digit28(const uint32_t *m, int P, int d) {
    const int bit = kDigit * d, k = bit >> 5, sh = bit & 31;
    const uint32_t lo = m[k], hi = k + 1 < P ? m[k + 1] : 0u;
    return __builtin_amdgcn_alignbit(hi, lo, sh) & ((1u << kDigit) - 1u);
}

// The record of element (i', j') of the rank-1 update R (i' < R.mr, j' <
// R.mc) is word x at T[((i' njb + j' / 32) TP + x) 32 + j' % 32], njb =
// ceil(R.mc / 32), x = 0..P: limb P-1+x of x_i' y_j'.
// ROWS: rows (= waves) of the workgroup's tile; any value gives the same bits.
template <int ROWS = kLaneRows>
__device__ __forceinline__ void prod_lane_body(uint32_t *lds, const Rank1 &R, uint32_t *T, const int32_t *info,
                                               int P, int64_t bx) {
    if (*info != 0) return;
    const int FT = kLaneFT, FTP = FT + 1;
    const int ND = lane_digits(P);
    const int64_t ncol = (R.mc + FT - 1) / FT;
    const int64_t rg = bx / ncol, j0 = (bx % ncol) * FT;
    if (rg * ROWS >= R.mr) return;  // uniform over the workgroup
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = mpw::lane();
    const int64_t ip = rg * ROWS + wave;
    const int cnt = (int)min((int64_t)FT, R.mc - j0);
    // tile rows -kPadLo .. ND+kPadHi-1 of FTP words (digit d of element e at
    // row d, column e; rows outside 0..ND-1 hold zeros)
    uint32_t *tile = lds + kPadLo * FTP;
    // this wave's multiplier digits, kPadL zeros above
    uint32_t *lsh = lds + (size_t)(ND + kPadLo + kPadHi) * FTP + wave * (ND + kPadL);
    const bool row_ok = ip < R.mr;
    const uint32_t *lm = r1x(R, row_ok ? ip : 0, P);
    for (int d = lane; d < ND + kPadL; d += MP_WAVE) lsh[d] = d < ND ? digit28(lm, P, d) : 0u;
    {
        const int nt = (int)blockDim.x, tid = (int)threadIdx.x;
        for (int z = tid; z < kPadLo * FTP; z += nt) lds[z] = 0u;
        for (int z = tid; z < kPadHi * FTP; z += nt) tile[ND * FTP + z] = 0u;
        // pivot-row digits of the tile: item w is digit w mod ND of element
        // w / ND (8 items per thread in flight; the two limbs a digit spans are
        // neighbours of the next item's, so the loads mostly hit the cache).
        // For w < 2^14, ND <= 147 the quotient is (w * magic) >> 24 exactly.
        // Columns cnt..63 are never read.
        // element b of the tile at ub + b * ustep (a row of Y or a column)
        const uint32_t *ub = r1y(R, j0, P);
        const int64_t ustep = (R.ydr * R.Y.ld + R.ydc) * (int64_t)P;
        const int nw = cnt * ND;
        const uint32_t magic = (1u << 24) / (uint32_t)ND + 1u;
        for (int w0 = 0; w0 < nw; w0 += 8 * nt) {
            uint32_t v[8];
            int ee[8], dd[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int w = min(w0 + u * nt + tid, nw - 1);
                ee[u] = (int)(((uint64_t)w * magic) >> 24);
                dd[u] = w - ee[u] * ND;
                v[u] = digit28(ub + (int64_t)ee[u] * ustep, P, dd[u]);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (w0 + u * nt + tid < nw) tile[dd[u] * FTP + ee[u]] = v[u];
        }
    }
    __syncthreads();
    const int e = lane;
    if (!row_ok || e >= cnt || lm[P - 1] == 0u) return;
    const int64_t jp = j0 + e;
    if (r1y(R, jp, P)[P - 1] == 0u) return;  // u_j = 0: a_ij is left as it is
    const int64_t njb = (R.mc + 31) / 32;
    const int TP = mfma_geom(P).TP;
    uint32_t *rec = T + (ip * njb + jp / 32) * (int64_t)TP * 32 + (jp % 32);

    const uint32_t *col = tile + e;  // digit x at col[x * FTP], -kPadLo <= x < ND + kPadHi
    constexpr int W = kLaneW;
    for (int c0 = lane_short_start(P);; c0 = 0) {
    // the guard bits 28 c0 + 36 .. 32 (P - 1) - 1 lie in limbs tw .. P-2
    const int tb = kDigit * c0 + 36, tw = tb >> 5;
    const uint32_t tmask = (1u << (tb & 31)) - 1u;
    uint32_t ones = 0xffffffffu;     // AND of the guard bits (bits below tb forced to one)
    uint64_t carry = 0;              // carry into the next column (< 2^37)
    uint64_t pk = 0;                 // bits of the product not yet emitted as a limb
    int pkn = (kDigit * c0) & 31;    // their count (zeros stand below bit 28 c0)
    int lout = (kDigit * c0) >> 5;   // index of the next limb
    for (int r0 = c0; r0 < 2 * ND; r0 += W) {
        const int alo = max(0, r0 - ND + 1), ahi = min(r0 + W - 1, ND - 1);
        // Steps a = alo .. ahi, padded to nb whole blocks of W: a padding step
        // multiplies a zero digit (a >= ND) or reads only zero rows below digit
        // 0 (a > r0 + W - 1), so it adds nothing.  In a block starting at a0,
        // ring slot y & 7 holds u[r0 - a0 + y] for the window y = c - t of step
        // a0 + t; the slot that column 7 frees receives the next digit down, so
        // the window turns by renaming and is back in place after W steps.
        const int nb = (ahi - alo + W) / W;
        uint32_t R[W];
#pragma unroll
        for (int c = 0; c < W; ++c) R[c] = col[(r0 + c - alo) * FTP];
        uint64_t s[W];
#pragma unroll
        for (int c = 0; c < W; ++c) s[c] = 0;
        // a block's digits: l[a0 + t] at lp[t]; the digit entering at step
        // a0 + t, u[r0 - a0 - t - 1], at up[(W - 1 - t) FTP]; each block moves
        // lp up and up down by W digits.  Up to one block past the last is
        // fetched: a <= ahi + 2W - 1 <= ND + 2W - 2 and r0 - a - 1 >= -3W.
        const uint32_t *lp = lsh + alo;
        const uint32_t *up = col + (r0 - alo - W) * FTP;
        auto fetch = [&](uint32_t (&l)[W], uint32_t (&u)[W]) __attribute__((always_inline)) {
#pragma unroll
            for (int t = 0; t < W; ++t) {
                l[t] = lp[t];
                u[t] = up[(W - 1 - t) * FTP];
            }
            lp += W;
            up -= W * FTP;
        };
        auto run = [&](const uint32_t (&l)[W], const uint32_t (&u)[W]) __attribute__((always_inline)) {
#pragma unroll
            for (int t = 0; t < W; ++t) {
#pragma unroll
                for (int c = 0; c < W; ++c) s[c] += (uint64_t)l[t] * R[(c - t) & (W - 1)];
                R[(W - 1 - t) & (W - 1)] = u[t];
            }
        };
        // two blocks per iteration, each one's LDS reads issued while the
        // other computes; the barriers keep a buffer's refill after its use
        uint32_t lA[W], uA[W], lB[W], uB[W];
        fetch(lA, uA);
        int b = 0;
        for (; b + 2 <= nb; b += 2) {
            fetch(lB, uB);
            run(lA, uA);
            __builtin_amdgcn_sched_barrier(0);
            fetch(lA, uA);
            run(lB, uB);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (b < nb) run(lA, uA);
        // carry the W columns in radix 2^28 (every sum and carry fits 64 bits)
        // and repack the digits into 32-bit limbs; the record keeps limbs
        // P-1 .. 2P-1
#pragma unroll
        for (int c = 0; c < W; ++c) {
            const uint64_t t = s[c] + carry;
            carry = t >> kDigit;
            pk |= (t & ((1u << kDigit) - 1u)) << pkn;
            pkn += kDigit;
            if (pkn >= 32) {  // the same on every lane
                if (lout >= P - 1 && lout < 2 * P)
                    rec[(int64_t)(lout - (P - 1)) * 32] = (uint32_t)pk;
                else if (lout >= tw && lout < P - 1)
                    ones &= (uint32_t)pk | (lout == tw ? tmask : 0u);
                pk >>= 32;
                pkn -= 32;
                ++lout;
            }
        }
    }
    // a short product whose guard bits are all ones may be missing a carry
    if (c0 == 0 || !__any(ones == 0xffffffffu)) break;
    }
}

template <int ROWS>
__global__ void __launch_bounds__(64 * ROWS) k_prod_lane(MatDev A, uint32_t *T, const int32_t *info, int64_t k,
                                                         int64_t n, int P) {
    extern __shared__ uint32_t lds_raw[];
    prod_lane_body<ROWS>(lds_raw, elim_rank1(A, k, n), T, info, P, flat_block());
}

// the products of any rank-1 update (k_finish_r1 completes it)
template <int ROWS>
__global__ void __launch_bounds__(64 * ROWS) k_prod_lane_r1(Rank1 R, uint32_t *T, const int32_t *info, int P) {
    extern __shared__ uint32_t lds_raw[];
    prod_lane_body<ROWS>(lds_raw, R, T, info, P, flat_block());
}

}  // namespace mpk
