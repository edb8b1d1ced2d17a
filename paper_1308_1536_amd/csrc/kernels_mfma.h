// kernels_mfma.h -- the trailing update (Algorithm 1 step 2.2.2) with the limb
// products on INT8 MFMA (v_mfma_i32_32x32x32_i8, gfx950).
//
// Exactness.  Each mantissa m (P8 = 4P little-endian bytes) is rewritten in
// balanced base 256: m = sum_{c=0..P8} d_c 256^c with d_c in [-128, 127] for
// c < P8 and d_P8 in {0, 1} (a carry-lookahead over the bytes: a byte >= 128
// borrows 256 from itself and carries 1 up).  Signed int8 operands then hold
// the digits exactly, and every column sum S_r = sum_c dl[r-c] du[c] obeys
// |S_r| <= (P8+1) 2^14 < 2^31, so int32 accumulation is exact.
//
// Contraction.  For a fixed row i the products l_i u_j for all j are one
// integer matrix product: S[r][j] = sum_c T_i[r][c] U[c][j] with the Toeplitz
// matrix T_i[r][c] = dl_i[r-c] (M = byte position r, K = digit c) and
// U[c][j] = du_j[c] (N = column j).  A 64-lane wave owns (row i, 32 columns)
// and sweeps r in chunks of 8 output tiles of 32 rows; the A fragment of a tile
// depends only on d = r0 - c0, so moving one K-step along the diagonal turns
// tile t's fragment into tile t+1's and only one new fragment is read from LDS
// per K-step (the row's digits are staged there reversed).  Fragments outside
// the band 0 <= r - c <= P8 are zero; every MFMA of a K-step is issued.
//
// Epilogue.  The signed column sums of a limb's four byte positions form
// V = sum_b S_b 256^b = lo + hi 2^32 (three v_mad_i64_i32); with
// y_L = lo_L + hi_{L-1}, limb L of the product is (y_L + c_L) mod 2^32 for a
// carry c_L in {-1, 0, 1}.  The fast path takes c_{L+1} = floor(y_L / 2^32),
// exact unless some y_L + c_L leaves [0, 2^32) in its low word; one ballot
// per chunk detects that, and such a chunk redoes its carries limb by limb
// (see update_mfma_body).  The top limbs of each product, from limb P-1 up,
// go to a record buffer; the finish kernel truncates the product to p bits
// and forms RZ_p(a_ij - RZ_p(l_i u_j)).
//
// Truncated product.  Only the byte positions r >= R0 = mfma_short_start(P)
// are formed, in chunks of 256 from R0 (a multiple of the 32-row tile; at
// 32K bits R0 = 4064 of 8192, about half the MFMAs skipped).  The skipped
// columns add E = sum_{r < R0} S_r 256^r, of either sign,
// |E| < (P8+1) 2^14 256^R0 / 255 < 2^(8 R0 + 22) for P8 < 2^15; the kept
// limbs of the formed sum are those of the whole product unless its bits
// 8 R0 + 24 .. 32 (P - 1) - 1 (at least 32 of them) are all ones (E > 0 could
// carry through) or all zeros (E < 0 could borrow through).  A wave in which
// some column's guard bits are like that forms its products again from
// R0 = 0.
#pragma once

#include <type_traits>

#include "kernels_valu.h"

namespace mpk {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

struct MfmaGeom {
    int P, P8;
    int K8;       // bytes per pivot-row digit string (digits 0..P8, zero padded)
    int LR;       // bytes per reversed multiplier digit string
    int Q;        // reversal origin: Lr[x] = dl[Q - x]
    int TP;       // limbs per product-top record in the scratch buffer
    int nchunks;  // chunks of 256 product bytes covering r < 2 P8
};

__host__ __device__ inline MfmaGeom mfma_geom(int P) {
    MfmaGeom g;
    g.P = P;
    g.P8 = 4 * P;
    g.K8 = g.P8 + 32;
    // the zero padding on both sides covers every diagonal offset d the
    // K-loop reads (-256 <= d <= P8 + 255), so out-of-band fragments read zeros
    g.LR = g.P8 + 608;
    g.Q = g.P8 + 291;  // Q = 3 mod 4: reversed limbs land on aligned words
    g.TP = P + 4;
    g.nchunks = (2 * g.P8 + 255) / 256;
    return g;
}

__host__ __device__ inline bool mfma_shape_ok(int P) { return P >= 8 && P % 8 == 0; }

// first product byte position formed (0: all): the largest multiple R0 of 32
// with 8 R0 + 24 + 32 <= 32 (P - 1), i.e. at least 32 guard bits
__host__ __device__ inline int mfma_short_start(int P) {
    if (4 * P >= (1 << 15)) return 0;  // the bound on E above needs P8 < 2^15
    const int r = (4 * P - 11) / 32 * 32;
    return r > 0 ? r : 0;
}

// Pivot-row digits in fragment-major order: digit c of column j' = 32 jb + j
// is byte c % 16 of the 16-byte fragment at ((jb NF + c / 16) 32 + j) 16,
// NF = K8 / 16, so the B fragments of one K-step of a 32-column block (lane
// (j, h) takes digits c0 + 16h .. c0 + 16h + 15) are one contiguous 1 KB run.
// Sized for whole 32-column blocks.
__host__ __device__ inline size_t ub_bytes(int64_t m, int P) {
    return (size_t)((m + 31) / 32) * 32u * (size_t)mfma_geom(P).K8;
}

constexpr int64_t kXcds = 8;  // MI355X: 8 accelerator complex dies, one L2 each
// word 3 of a raw (untyped, unswizzled) buffer resource on gfx9-class GPUs
constexpr int kBufferRsrcWord3 = 0x00020000;

// Waves per workgroup of k_update_mfma: the waves take consecutive rows i of
// the same 32-column block, so the pivot-row digit fragments they stream are
// the same cache lines and are fetched into the CU's L1 once for all of them.
constexpr int kMfmaWaves = 2;  // the default of 1, 2 or 4
// LDS one workgroup of k_update_mfma may take
constexpr size_t kMfmaLdsMax = 64 * 1024;

// workgroups of k_update_mfma for `rows` rows of an m x m trailing block
__host__ __device__ inline int64_t mfma_update_blocks(int64_t rows, int64_t m, int waves = kMfmaWaves) {
    const int64_t njb = (m + 31) / 32, nrg = (rows + waves - 1) / waves;
    return njb >= kXcds ? kXcds * nrg * ((njb + kXcds - 1) / kXcds) : nrg * njb;
}


// bit k of v -> bit 2k
__device__ __forceinline__ uint64_t spread_bits(uint32_t v) {
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

// ---------------------------------------------------------------------------
// Balanced digits of one mantissa (all lanes of the wave): dw[0..P] receive the
// digit words (digit 4q+b in byte b of word q; word P holds d_P8 in byte 0).
// ---------------------------------------------------------------------------
__device__ void balanced_digit_words(uint32_t *dw, const uint32_t *m, int P) {
    uint32_t carry = 0;
    for (int base = 0; base < P; base += MP_WAVE) {
        const int q = base + mpw::lane();
        const int cnt = min(MP_WAVE, P - base);
        const uint32_t w = q < P ? m[q] : 0u;
        // carry out of the limb's four bytes for carry-in 0 and 1
        uint32_t co0 = 0, co1 = 1;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            uint32_t by = (w >> (8 * b)) & 0xFFu;
            co0 = (by + co0) >= 128u;
            co1 = (by + co1) >= 128u;
        }
        const uint64_t valid = cnt == 64 ? ~0ull : ((1ull << cnt) - 1ull);
        const uint64_t G = __ballot(co0 != 0u) & valid;
        const uint64_t Pm = __ballot(co1 != 0u && co0 == 0u) & valid;
        const uint64_t C = mpw::lookahead(G, Pm, carry);
        uint32_t c = (uint32_t)((C >> mpw::lane()) & 1ull);
        uint32_t out = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            uint32_t t = ((w >> (8 * b)) & 0xFFu) + c;
            c = t >= 128u;
            out |= ((t - 256u * c) & 0xFFu) << (8 * b);
        }
        if (q < P) dw[q] = out;
        carry = mpw::block_carry_out(G, Pm, C, cnt);
    }
    if (mpw::lane() == 0) dw[P] = carry;
    mpw::wsync();
}

// Per step: block b < m -> reversed multiplier digits of row k+1+b (Lr),
// block b >= m -> digits of pivot-row element k+1+(b-m) (Ub).
__device__ __forceinline__ void mfma_prep_body(uint32_t *lds_raw, MatDev A, uint8_t *Lr, uint8_t *Ub, const int32_t *info,
                               int64_t k, int64_t n, int P, int64_t b) {
    if (*info != 0) return;
    const MfmaGeom g = mfma_geom(P);
    const int64_t m = n - k - 1;
    const bool is_row = b < m;
    const uint32_t *src = is_row ? el(A, k + 1 + b, k, P) : el(A, k, k + 1 + (b - m), P);
    if (src[P - 1] == 0u && is_row) return;  // zero multiplier: its row is skipped
    uint32_t *dw = lds_raw;                  // P + 1 words
    balanced_digit_words(dw, src, P);
    if (is_row) {
        // word w of the reversed row holds digit word (Q - 3) / 4 - w, bytes reversed
        uint32_t *out = (uint32_t *)(Lr + b * (int64_t)g.LR);
        for (int w = mpw::lane(); w < g.LR / 4; w += MP_WAVE) {
            int qd = (g.Q - 3) / 4 - w;
            uint32_t v = 0;
            if (qd >= 0 && qd <= P) v = __builtin_bswap32(dw[qd]);
            out[w] = v;
        }
    } else {
        const int64_t jp = b - m;
        const int NF = g.K8 / 16;
        uint8_t *col = Ub + ((jp / 32) * NF * 32 + jp % 32) * 16;
        // word w holds digits 4w .. 4w+3: fragment w / 4, bytes 4 (w % 4) on
        for (int w = mpw::lane(); w < g.K8 / 4; w += MP_WAVE)
            *(uint32_t *)(col + (int64_t)(w >> 2) * 512 + (w & 3) * 4) = w <= P ? dw[w] : 0u;
    }
}

// Row order inside a 32-row output tile.  The MFMA's C fragment gives lane
// (j, h) the rows 8gq + 4h + b (gq, b = 0..3) of column j; the tile's A rows
// are permuted so that row 8gq + 4h + b is byte position 16h + 4gq + b of the
// tile, and a lane then holds four whole consecutive limbs (4h + gq) of each
// tile.  A row r of the A fragment is byte position tile_pos(r).
__device__ __forceinline__ int tile_pos(int r) { return 16 * ((r >> 2) & 1) + 4 * (r >> 3) + (r & 3); }

// LDS of one wave: NC copies of its reversed digit row, copy a shifted down by
// a bytes (copy_a[x] = Lr[x + a]).  A fragment (16 consecutive bytes of the
// row, starting at a lane-dependent byte) is read as four aligned words from
// the copy whose shift cancels the start's misalignment; with NC = 1 the lane
// reads the five words around its bytes and shifts them into place
// (v_alignbyte_b32).  Byte-misaligned 16-byte LDS reads stall the LDS pipeline.
// p: the aligned word at or below the fragment's first byte, in the copy the
// lane reads (a_word below)
template <int NC>
__device__ __forceinline__ v4i load_a(const uint32_t *p, uint32_t sh) {
    v4i v;
    if constexpr (NC == 4) {
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = (int)p[t];
    } else {
        uint32_t w[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) w[t] = p[t];
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = (int)__builtin_amdgcn_alignbyte(w[t + 1], w[t], sh);
    }
    return v;
}
// the aligned word of byte s - sh (s = first byte of a fragment, sh = s mod 4)
template <int NC>
__device__ __forceinline__ const uint32_t *a_word(const uint8_t *lr, int LR, int s, uint32_t sh) {
    return (const uint32_t *)(lr + (NC == 4 ? (int)sh * LR : 0) + (s - (int)sh));
}

// LDS copies of the digit row that fit a workgroup (0: the MFMA update does not fit)
__host__ __device__ inline int mfma_copies(int P, int waves = kMfmaWaves) {
    const size_t lr = (size_t)mfma_geom(P).LR * waves;
    return 4 * lr <= kMfmaLdsMax ? 4 : (lr <= kMfmaLdsMax ? 1 : 0);
}
__host__ __device__ inline size_t mfma_lds_bytes(int P, int waves = kMfmaWaves) {
    return (size_t)mfma_geom(P).LR * waves * (size_t)mfma_copies(P, waves);
}
__host__ __device__ inline bool mfma_supported(int P) { return mfma_shape_ok(P) && mfma_copies(P) > 0; }

// Exchange word of a tile between the lanes of a column: bits 0..23 the
// signed high part of the tile's top limb sum, bits 24..25 the signed carry
// out of that limb's low word.
__device__ __forceinline__ uint32_t xw_pack(int32_t hi, int32_t c) {
    return ((uint32_t)hi & 0xFFFFFFu) | (((uint32_t)c & 3u) << 24);
}
__device__ __forceinline__ int32_t xw_hi(uint32_t w) { return (int32_t)(w << 8) >> 8; }
__device__ __forceinline__ int32_t xw_c(uint32_t w) { return (int32_t)(w << 6) >> 30; }

// sum_b s_b 256^b over the four signed byte-column sums of one limb, exactly
// (three v_mad_i64_i32 onto the sign-extended s_0)
__device__ __forceinline__ int64_t limb_sum(int32_t s0, int32_t s1, int32_t s2, int32_t s3) {
    int64_t v = (int64_t)s0;
    uint64_t cc;
    asm volatile("v_mad_i64_i32 %0, %1, %2, %3, %0" : "+v"(v), "=s"(cc) : "v"(s1), "s"(256));
    asm volatile("v_mad_i64_i32 %0, %1, %2, %3, %0" : "+v"(v), "=s"(cc) : "v"(s2), "s"(65536));
    asm volatile("v_mad_i64_i32 %0, %1, %2, %3, %0" : "+v"(v), "=s"(cc) : "v"(s3), "s"(16777216));
    return v;
}

// value of the partner lane (lane ^ 32): h = 1 lanes receive b of lane j,
// h = 0 lanes receive a of lane j + 32 (v_permlane32_swap_b32)
__device__ __forceinline__ uint32_t partner_of(uint32_t a, uint32_t b, int h) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    return h ? r[0] : r[1];
}

// Product top limbs: for every row i' (multiplier l = a_{k+1+i', k}) and
// column block jb of 32, word x <= P of the record of column j' = 32 jb + j is
// limb P-1+x of l * u_{j'}, stored limb-major across the block's 32 columns:
// T[((i' njb + jb) TP + x) 32 + j].
// WAVES: waves (= consecutive rows of one column block) per workgroup; any
// value gives the same bits.
template <int NE>
__device__ __forceinline__ void finish_stream_tile(uint32_t *lds, MatDev A, uint32_t *__restrict__ T, int64_t k,
                                                   int64_t n, int P, int64_t ip0, int64_t ip, int64_t j0, int cnt);

template <int NC>
__device__ __forceinline__ void mfma_task(uint8_t *lr, MatDev A, const uint8_t *Lr, const uint8_t *Ub, uint32_t *T,
                                          int64_t k, int64_t n, int P, int64_t ip0, int64_t ip, int64_t jb);

// FUSE (P > kFinStreamMinP): each wave then finishes its own 32 elements
// from its records (finish_stream_tile), so no finish launch follows; the
// finish of one wave (vector ALU, memory) can run beside the products of
// another on the same SIMD.
template <int NC, int WAVES = kMfmaWaves, bool FUSE = false>
__device__ __forceinline__ void update_mfma_body(uint32_t *lds_raw, MatDev A, const uint8_t *Lr, const uint8_t *Ub,
                                                 uint32_t *T, const int32_t *info, int64_t k, int64_t n, int P,
                                                 int64_t ip0, int64_t rows, int64_t bx, bool xcd_aware) {
    if (*info != 0) return;
    const MfmaGeom g = mfma_geom(P);
    const int64_t m = n - k - 1;
    const int64_t njb = (m + 31) / 32, nrg = (rows + WAVES - 1) / WAVES;
    int64_t rg, jb;
    if (xcd_aware && njb >= kXcds) {
        // workgroups go to the 8 XCDs round-robin: XCD x takes the column
        // blocks jb = x (mod 8), so each XCD's L2 holds only its share of the
        // pivot-row digits
        const int64_t xcd = bx % kXcds, loc = bx / kXcds;
        const int64_t cnt = (njb - xcd + kXcds - 1) / kXcds;
        if (loc >= nrg * cnt) return;
        rg = loc / cnt;
        jb = xcd + kXcds * (loc % cnt);
    } else {
        if (bx >= nrg * njb) return;
        rg = bx / njb;
        jb = bx % njb;
    }
    // wave w of the workgroup takes row i' = ip0 + WAVES rg + w of the
    // panel [ip0, ip0 + rows)
    const int wave = (int)(threadIdx.x >> 6);
    const int64_t ip = ip0 + rg * WAVES + wave;
    const bool valid = ip < ip0 + rows && ip < m;
    uint8_t *lr = (uint8_t *)lds_raw + (size_t)wave * NC * g.LR;
    if (!valid) return;
    mfma_task<NC>(lr, A, Lr, Ub, T, k, n, P, ip0, ip, jb);
    if constexpr (FUSE) {
        // the records are complete and visible to every lane of the wave,
        // and the wave's LDS is free
        __builtin_amdgcn_s_waitcnt(0);
        mpw::wsync();
        finish_stream_tile<32>((uint32_t *)lr, A, T, k, n, P, ip0, ip, jb * 32, (int)min((int64_t)32, m - jb * 32));
    }
}

// One task of the update: row i' = ip of the trailing block (its record slot
// ip - ip0 of the panel) times the 32 columns of block jb, in one wave with
// its own LDS (NC copies of the row's digits).
template <int NC>
__device__ __forceinline__ void mfma_task(uint8_t *lr, MatDev A, const uint8_t *Lr, const uint8_t *Ub, uint32_t *T,
                                          int64_t k, int64_t n, int P, int64_t ip0, int64_t ip, int64_t jb) {
    const MfmaGeom g = mfma_geom(P);
    const int64_t m = n - k - 1;
    const int64_t njb = (m + 31) / 32;
    // a zero multiplier leaves the row as it is
    if (el(A, k + 1 + ip, k, P)[P - 1] == 0u) return;
    const int LR = g.LR;
    {
        const uint32_t *src = (const uint32_t *)(Lr + ip * (int64_t)LR);
        const int nw = LR / 4;
        for (int w = mpw::lane(); w < nw; w += MP_WAVE) {
            const uint32_t x0 = src[w], x1 = w + 1 < nw ? src[w + 1] : 0u;
#pragma unroll
            for (int a = 0; a < NC; ++a) ((uint32_t *)(lr + a * LR))[w] = __builtin_amdgcn_alignbyte(x1, x0, a);
        }
    }
    mpw::wsync();

    const int lane = mpw::lane();
    const int j = lane & 31, h = lane >> 5;
    const int64_t jp = jb * 32 + j;
    const bool jvalid = jp < m;
    // this lane's B fragment of the K-step at c0 is at ubs + 32 c0 + boff (a
    // column past m reads its block's unused, allocated slot; its results are
    // dropped); ubs is the same for the whole wave
    // (read through a buffer resource: per-lane offset in a VGPR, the step's
    // offset in an SGPR, no 64-bit address arithmetic per step)
    const uint8_t *ubs = Ub + jb * (int64_t)(g.K8 / 16) * 512;
    const uint32_t boff = (uint32_t)(h * 32 + j) * 16u;
    const __amdgpu_buffer_rsrc_t brs =
        __builtin_amdgcn_make_buffer_rsrc((void *)ubs, (short)0, 32 * g.K8, kBufferRsrcWord3);
    auto load_b = [&](int c0) __attribute__((always_inline)) {
        return __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(brs, boff, 32 * c0, 0));
    };
    uint32_t *tcol = T + ((ip - ip0) * njb + jb) * (int64_t)g.TP * 32 + j;
    const int P8 = g.P8;
    const int bmax = g.K8 - 32;  // last K-step offset c0 inside the digit strings
    // A fragment of diagonal offset d = r0 - c0 for this lane (row r = j of the
    // A operand, K half h): the 16 bytes of the reversed row from byte
    // sa - d on, sa = Q - tile_pos(j) + 16h; ash = the start's byte offset mod 4
    const int sa = g.Q - tile_pos(j) + 16 * h;
    const uint32_t ash = (uint32_t)sa & 3u;
    for (int rb = mfma_short_start(P);; rb = 0) {
    uint32_t xw_prev = 0;  // exchange word of tile 7 of the chunk below (carry into this chunk)
    // guard limbs tw .. P-2 (bits below 24 of limb tw excluded): AND and OR
    // of this lane's share
    const int tw = rb / 4;
    uint32_t g_and = 0xffffffffu, g_or = 0u;
    const int nch = (2 * g.P8 - rb + 255) / 256;  // chunks of 256 rows from rb

    for (int chunk = 0; chunk < nch; ++chunk) {
        const int r0 = rb + chunk * 256;
        v16i acc[8];
        int c_lo = r0 - 31 - P8;
        c_lo = c_lo <= 0 ? 0 : ((c_lo + 31) & ~31);
        const int c_hi = min(P8, r0 + 224);
        const int nsteps = (c_hi - c_lo) / 32 + 1;
        // Step n, tile t uses the A fragment with d = r0 + 32(t - n) - c_lo,
        // kept in window slot (t - n) mod 8; the slot of tile 7 is refilled with
        // the next step's tile-0 fragment, so slots rotate by renaming inside
        // the 8-way unrolled loop.  B fragments sit in an 8-deep register ring
        // (prefetch distance 8 steps).  All 8 MFMAs run every step: a fragment
        // outside the band is zero.
        v4i W[8], BR[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) W[t] = load_a<NC>(a_word<NC>(lr, LR, sa - (r0 + 32 * t - c_lo), ash), ash);
        // B loads are unconditional: offsets are clamped into the column's
        // digit string, and a fragment fetched for a step >= nsteps is never used
#pragma unroll
        for (int u = 0; u < 8; ++u) BR[u] = load_b(min(c_lo + 32 * u, bmax));
        // word of the tile-0 fragment of step 1 (the first one the loop reads);
        // step n's is 8 (n - 1) words further on
        const uint32_t *a1 = a_word<NC>(lr, LR, sa - (r0 - c_lo - 32), ash);
        // one K-step: tile 7's MFMA frees its window slot, which is refilled at
        // once with the next step's tile-0 fragment (its LDS latency hides
        // behind tiles 0..6); the slot's next B fragment is fetched after the
        // step's MFMAs, so the ring keeps its registers and 7 loads stay in
        // flight
        // (first: the chunk's first step, whose MFMAs start from zero)
        auto kstep = [&](auto first, const uint32_t *ablk, int n, int u) __attribute__((always_inline)) {
            const int c0 = c_lo + 32 * n;
            acc[7] = __builtin_amdgcn_mfma_i32_32x32x32_i8(W[(7 - u) & 7], BR[u], first ? (v16i){0} : acc[7], 0, 0, 0);
            W[(7 - u) & 7] = load_a<NC>(ablk + 8 * u, ash);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < 7; ++t)
                acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(W[(t - u) & 7], BR[u], first ? (v16i){0} : acc[t], 0,
                                                               0, 0);
            BR[u] = load_b(min(c0 + 256, bmax));
            // keep each step's loads in their step: the scheduler would
            // otherwise sink a block's 8 loads to its end
            __builtin_amdgcn_sched_barrier(0);
        };
        // full blocks of 8 steps (no exit inside, so the load count at the loop
        // edge is the same on every path), then the partial block
        constexpr std::true_type kFirst{};
        constexpr std::false_type kNext{};
        int n8 = 0;
        if (nsteps >= 8) {
            kstep(kFirst, a1, 0, 0);
#pragma unroll
            for (int u = 1; u < 8; ++u) kstep(kNext, a1, u, u);
            n8 = 8;
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) acc[t] = (v16i){0};
        }
        for (; n8 + 8 <= nsteps; n8 += 8) {
            const uint32_t *ablk = a1 + 8 * n8;
#pragma unroll
            for (int u = 0; u < 8; ++u) kstep(kNext, ablk, n8 + u, u);
        }
        {
            const uint32_t *ablk = a1 + 8 * n8;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (n8 + u >= nsteps) break;
                kstep(kNext, ablk, n8 + u, u);
            }
        }

        // Epilogue, in registers.  Lane (j, h) holds, for tile t and gq = 0..3,
        // the signed column sums S of the four bytes of chunk limb
        // L = 8t + 4h + gq of column j; V = sum_b S_b 256^b = lo + hi 2^32
        // (lo unsigned, hi signed) and y_L = lo_L + hi_{L-1} leave a carry
        // c_L in {-1, 0, 1} into each limb: limb_L = (y_L + c_L) mod 2^32,
        // c_{L+1} = floor((y_L + c_L) / 2^32).  Fast path: c_{L+1} is taken as
        // floor(y_L / 2^32), which is exact unless some y_L + c_L leaves
        // [0, 2^32) in its low word (all-ones plus 1, or zero minus 1); the
        // wave checks that and, if it happened anywhere, redoes the chunk's
        // carries one limb after another.  The limbs of tile t's top limb
        // (gq = 3) reach the partner lane through one exchange word per tile.
        uint32_t ylo[32];
        int32_t yhi[32];
        uint32_t xw[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            int32_t hi[4];
            uint32_t lo[4];
#pragma unroll
            for (int gq = 0; gq < 4; ++gq) {
                const int64_t V = limb_sum(acc[t][4 * gq], acc[t][4 * gq + 1], acc[t][4 * gq + 2], acc[t][4 * gq + 3]);
                lo[gq] = (uint32_t)V;
                hi[gq] = (int32_t)(V >> 32);
            }
            // limbs 1..3 of the group take the high part of the limb below
#pragma unroll
            for (int gq = 1; gq < 4; ++gq) {
                const int64_t y = (int64_t)lo[gq] + hi[gq - 1];
                ylo[4 * t + gq] = (uint32_t)y;
                yhi[4 * t + gq] = (int32_t)(y >> 32);
            }
            ylo[4 * t] = lo[0];  // the high part from below arrives with the exchange
            xw[t] = xw_pack(hi[3], yhi[4 * t + 3]);
        }
        // limb 4h of tile t: below it is limb 3 of the partner's tile t (h = 1)
        // or of the partner's tile t - 1 (h = 0; for t = 0 the chunk below)
        bool danger = false;
        uint32_t limb[32];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const uint32_t in = partner_of(t ? xw[t - 1] : xw_prev, xw[t], h);
            const int64_t y = (int64_t)ylo[4 * t] + xw_hi(in);
            ylo[4 * t] = (uint32_t)y;
            yhi[4 * t] = (int32_t)(y >> 32);
            int32_t c = xw_c(in);
#pragma unroll
            for (int gq = 0; gq < 4; ++gq) {
                const int64_t z = (int64_t)ylo[4 * t + gq] + c;
                limb[4 * t + gq] = (uint32_t)z;
                danger |= (z >> 32) != 0;
                c = yhi[4 * t + gq];
            }
        }
        // the top limb of the chunk (h = 1, tile 7, gq = 3) carries into the next
        // chunk's first limb (h = 0, tile 0): the h = 1 lanes keep its word
        uint32_t next_prev = xw[7];
        if (__builtin_amdgcn_ballot_w64(danger) != 0ull) {
            // exact carries, limb after limb: per tile, the h = 0 lanes take
            // their four limbs, then hand the carry to the h = 1 lanes, which
            // hand theirs to the h = 0 lanes' next tile
            int32_t c0 = xw_c(partner_of(xw_prev, xw_prev, h));  // carry into limb 0 (h = 0 lanes)
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                int32_t cin = c0;
                // h = 0 lanes: limbs 8t .. 8t+3
#pragma unroll
                for (int gq = 0; gq < 4; ++gq) {
                    const int64_t z = (int64_t)ylo[4 * t + gq] + cin;
                    if (h == 0) limb[4 * t + gq] = (uint32_t)z;
                    cin = yhi[4 * t + gq] + (int32_t)(z >> 32);
                }
                // carry out of the h = 0 group to the h = 1 lanes
                const int32_t c1 = (int32_t)partner_of(0u, (uint32_t)cin, h);
                cin = c1;
#pragma unroll
                for (int gq = 0; gq < 4; ++gq) {
                    const int64_t z = (int64_t)ylo[4 * t + gq] + cin;
                    if (h == 1) limb[4 * t + gq] = (uint32_t)z;
                    cin = yhi[4 * t + gq] + (int32_t)(z >> 32);
                }
                // carry out of the h = 1 group back to the h = 0 lanes
                c0 = (int32_t)partner_of((uint32_t)cin, 0u, h);
                if (t == 7 && h == 1) next_prev = xw_pack(xw_hi(xw[7]), cin);
            }
        }
        xw_prev = next_prev;
        // limb q = r0/4 + 8t + 4h + gq of the product; the record keeps P-1 .. 2P-1
        const int qbase = r0 / 4;
        if (rb > 0 && qbase <= P - 2 && qbase + 63 >= tw) {
#pragma unroll
            for (int t = 0; t < 8; ++t)
#pragma unroll
                for (int gq = 0; gq < 4; ++gq) {
                    const int q = qbase + 8 * t + 4 * h + gq;
                    if (q >= tw && q <= P - 2) {
                        const uint32_t low = q == tw ? 0x00ffffffu : 0u;
                        g_and &= limb[4 * t + gq] | low;
                        g_or |= limb[4 * t + gq] & ~low;
                    }
                }
        }
        if (qbase + 63 >= P - 1 && jvalid) {
            if (qbase >= P - 1 && qbase + 63 < 2 * P) {
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int gq = 0; gq < 4; ++gq)
                        tcol[(int64_t)(qbase + 8 * t + 4 * h + gq - (P - 1)) * 32] = limb[4 * t + gq];
            } else {
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int gq = 0; gq < 4; ++gq) {
                        const int q = qbase + 8 * t + 4 * h + gq;
                        if (q >= P - 1 && q < 2 * P) tcol[(int64_t)(q - (P - 1)) * 32] = limb[4 * t + gq];
                    }
            }
        }
    }
    if (rb == 0) break;
    // column j's guard limbs are split between lanes j and j + 32; a column
    // past m or with u_j = 0 has no product to keep
    const uint32_t p_and = partner_of(g_and, g_and, h), p_or = partner_of(g_or, g_or, h);
    const bool live = jvalid && el(A, k, k + 1 + jp, P)[P - 1] != 0u;
    const bool unsure = live && ((g_and & p_and) == 0xffffffffu || (g_or | p_or) == 0u);
    if (__builtin_amdgcn_ballot_w64(unsure) == 0ull) break;
    }
}

// ---------------------------------------------------------------------------
// Finish of the update: a_ij = RZ_p(a_ij - t), t = RZ_p(l_i u_j) rebuilt from
// the record (word x = product limb P-1+x, x = 0..P).  One workgroup (one
// wave) takes FT consecutive elements of a row, which are one contiguous run
// in HBM: it copies their limbs into LDS limb-major (row q holds limb q of the
// FT elements, rows padded to FT+1 words, so both the coalesced copy and the
// per-lane walk are free of bank conflicts), each lane finishes one element
// in place with the case analysis of mpw::addsub (pass 1 forms the exact
// p+2-bit sum or difference G over the element's own LDS column, pass 2
// normalises G to p bits), and the tile is copied back.  Every pass walks the
// limbs in an order that never reads a location after writing it.
// ---------------------------------------------------------------------------
// Streaming variant (finish_stream_body), for P above kFinStreamMinP: the tile
// is always 64 elements and LDS holds one 32-limb chunk of each, so occupancy
// and lane use no longer fall with P.
constexpr int kFinStreamMinP = 256;
constexpr int kFinC = 32;   // limbs per chunk of the streaming finish
constexpr int kFinCP = 36;  // LDS words per element row of a chunk (one spare, 16-byte aligned)
// LDS of the streaming finish of NE elements per wave: NE + 1 element rows, two
// words per lane
__host__ __device__ inline size_t finish_tile_lds(int NE) { return (size_t)((NE + 1) * kFinCP + 128) * 4u; }
// the update launch can finish its own products (FUSE): the streaming finish
// applies and the LDS of a wave (its digit-row copies) holds a 32-element
// finish tile
__host__ __device__ inline bool mfma_fuse_ok(int P, int waves) {
    const size_t per_wave = (size_t)mfma_copies(P, waves) * (size_t)mfma_geom(P).LR;
    return P > kFinStreamMinP && per_wave >= finish_tile_lds(32);
}
__host__ __device__ inline bool finish_streams(int P) { return P > kFinStreamMinP; }
__host__ __device__ inline int finish_tile(int P) {
    return finish_streams(P) ? 64 : (P <= 256 ? 64 : (P <= 512 ? 32 : 16));
}
__host__ __device__ inline size_t finish_lds_bytes(int P) {
    if (finish_streams(P)) return finish_tile_lds(64);
    return (size_t)(P + 1) * (size_t)(finish_tile(P) + 1) * 4u;
}
// workgroups of the finish for `rows` rows of an m x m trailing block
__host__ __device__ inline int64_t finish_blocks(int64_t rows, int64_t m, int P) {
    const int ft = finish_tile(P);
    return rows * ((m + ft - 1) / ft);
}
// record slots of `rows` rows of an m x m trailing block: rows x njb blocks of 32 columns
__host__ __device__ inline int64_t rec_slots(int64_t rows, int64_t m) { return rows * ((m + 31) / 32) * 32; }

// Length of G = X 2^gsh +- (Y >> (32w + b)) (-+ a sticky unit) from the top
// three limbs of both terms (leading-zero anticipation); xl(q), yl(q) give
// limb q of X and Y (0 outside 0..P-1).  H, the same combination of limbs
// P-2 .. P alone, differs from G's limbs P-2 .. P by the carry (+1) or borrow
// (-1, sticky included) out of the limbs below, which changes H's length only
// if H is all ones (addition) or a power of two (subtraction).  Outside those
// cases, and if H has at least 32 bits (the normalised result then starts no
// more than one limb below G's limb order, so it can be written while G is
// formed), *len = G's bit length and the result is true.
template <typename XL, typename YL>
__device__ __forceinline__ bool lza_length(int P, int gsh, int w, int b, bool subtract, XL xl, YL yl, int *len) {
    uint32_t hx[3], hy[3];
#pragma unroll
    for (int z = 0; z < 3; ++z) {
        const int q = P - 2 + z;
        hx[z] = gsh ? __builtin_amdgcn_alignbit(xl(q), xl(q - 1), 32 - gsh) : xl(q);
        hy[z] = __builtin_amdgcn_alignbit(yl(q + w + 1), yl(q + w), b);
    }
    // H as one 96-bit value: two 64-bit words
    const uint64_t xlo = ((uint64_t)hx[1] << 32) | hx[0], ylo64 = ((uint64_t)hy[1] << 32) | hy[0];
    uint64_t hlo, hhi;
    if (subtract) {
        hlo = xlo - ylo64;
        hhi = (uint64_t)hx[2] - hy[2] - (xlo < ylo64 ? 1u : 0u);
    } else {
        hlo = xlo + ylo64;
        hhi = (uint64_t)hx[2] + hy[2] + (hlo < xlo ? 1u : 0u);
    }
    const int hbits = hhi ? 64 + 64 - __clzll(hhi) : (hlo ? 64 - __clzll(hlo) : 0);
    bool ambiguous;
    if (subtract) {  // a power of two
        const uint64_t mlo = hlo - 1, mhi = hhi - (hlo == 0 ? 1u : 0u);
        ambiguous = (hlo & mlo) == 0 && (hhi & mhi) == 0;
    } else {  // all ones below the top bit: H + 1 is a power of two
        const uint64_t plo = hlo + 1, phi = hhi + (plo == 0 ? 1u : 0u);
        ambiguous = (hlo & plo) == 0 && (hhi & phi) == 0;
    }
    *len = 32 * (P - 2) + hbits;
    return !ambiguous && hbits >= 32;
}

// A rank-1 update z_ab <- RZ_p(z_ab - RZ_p(x_a s y_b)), s = -1 if yneg else 1,
// over a block of mr rows and mc columns: x_a = X[xr + a xdr][xc + a xdc],
// y_b = Y[yr + b ydr][yc + b ydc], z_ab = Z[zr + a][zc + b] (RZ is odd, so
// yneg gives z + RZ_p(x y)).  Step k of the elimination is X = Y = Z = A with
// x the multipliers of column k, y the pivot row and z the trailing block;
// the row sweeps of L^-1 and the adjugate's back substitution and
// accumulation are other instances.  The z block must not overlap x or y.
struct Rank1 {
    MatDev X, Y, Z;
    int64_t xr, xc, xdr, xdc, yr, yc, ydr, ydc, zr, zc, mr, mc;
    int32_t yneg;
};
__host__ __device__ inline Rank1 elim_rank1(MatDev A, int64_t k, int64_t n) {
    const int64_t m = n - k - 1;
    return Rank1{A, A, A, k + 1, k, 1, 0, k, k + 1, 0, 1, k + 1, k + 1, m, m, 0};
}
// x_a and y_b of a rank-1 update: limbs, exponent and sign
__device__ __forceinline__ uint32_t *r1x(const Rank1 &R, int64_t a, int P) {
    return el(R.X, R.xr + a * R.xdr, R.xc + a * R.xdc, P);
}
__device__ __forceinline__ int64_t r1x_e(const Rank1 &R, int64_t a) { return ex(R.X, R.xr + a * R.xdr, R.xc + a * R.xdc); }
__device__ __forceinline__ int32_t r1x_s(const Rank1 &R, int64_t a) { return sg(R.X, R.xr + a * R.xdr, R.xc + a * R.xdc); }
__device__ __forceinline__ uint32_t *r1y(const Rank1 &R, int64_t b, int P) {
    return el(R.Y, R.yr + b * R.ydr, R.yc + b * R.ydc, P);
}
__device__ __forceinline__ int64_t r1y_e(const Rank1 &R, int64_t b) { return ex(R.Y, R.yr + b * R.ydr, R.yc + b * R.ydc); }
__device__ __forceinline__ int32_t r1y_s(const Rank1 &R, int64_t b) { return sg(R.Y, R.yr + b * R.ydr, R.yc + b * R.ydc); }

__device__ __forceinline__ void finish_tile_body(uint32_t *lds, const Rank1 &R, const uint32_t *__restrict__ T,
                                                 int P, int64_t ip0, int64_t rows, int64_t bx) {
    const MfmaGeom g = mfma_geom(P);
    const int64_t njb = (R.mc + 31) / 32;
    const int FT = finish_tile(P), FTP = FT + 1;
    const int64_t ntile = (R.mc + FT - 1) / FT;
    const int64_t ip = ip0 + bx / ntile, j0 = (bx % ntile) * FT;
    if (bx / ntile >= rows || ip >= R.mr) return;
    const int64_t i = R.zr + ip;
    if (r1x(R, ip, P)[P - 1] == 0u) return;  // zero multiplier: the row keeps its values
    const int cnt = (int)min((int64_t)FT, R.mc - j0);
    uint32_t *arow = el(R.Z, i, R.zc + j0, P);  // cnt elements, cnt * P contiguous limbs
    const int lane = mpw::lane();
    const int e = lane;
    const bool live = e < cnt;
    const int64_t jp = j0 + (live ? e : 0), j = R.zc + jp;
    // per-lane scalars first, so their latency overlaps the tile copy
    const uint32_t *raw = T + ((ip - ip0) * njb + jp / 32) * (int64_t)g.TP * 32 + (jp % 32);
    const uint32_t utop = r1y(R, jp, P)[P - 1];
    const uint32_t rtop = raw[(int64_t)P * 32];
    const int64_t eik = r1x_e(R, ip), ekj = r1y_e(R, jp), ea = ex(R.Z, i, j);
    const int32_t sik = r1x_s(R, ip), skj = r1y_s(R, jp) ^ R.yneg, sa = sg(R.Z, i, j);

    // tile copy in 16-byte chunks, 16 per lane in flight: chunk c holds limbs
    // 4(c mod cpe) .. +3 of element c / cpe, cpe = P / 4 (c < 4096, so the
    // quotient is (c * magic) >> 24 exactly)
    const int cpe = P / 4;
    const uint32_t magic = (1u << 24) / (uint32_t)cpe + 1u;
    const int nch = cnt * cpe;
    {
        const uint4 *src = (const uint4 *)arow;
        for (int c0 = 0; c0 < nch; c0 += 16 * MP_WAVE) {
            uint4 v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int c = c0 + u * MP_WAVE + lane;
                v[u] = c < nch ? src[c] : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int c = c0 + u * MP_WAVE + lane;
                if (c < nch) {
                    const int ee = (int)(((uint64_t)c * magic) >> 24);
                    uint32_t *d = lds + 4 * (c - ee * cpe) * FTP + ee;
                    d[0] = v[u].x;
                    d[FTP] = v[u].y;
                    d[2 * FTP] = v[u].z;
                    d[3 * FTP] = v[u].w;
                }
            }
        }
    }
    mpw::wsync();

    if (live && utop != 0u) {
        uint32_t *col = lds + e;  // limb q at col[q * FTP], q = 0..P
        const int top = (int)(rtop >> 31);
        const int sh = 1 - top;
        // word x of the record (0 outside 0..P) and limb q of t (0 outside 0..P-1);
        // all indices here are below 2P + 40 and fit int
        auto rw = [&](int x) -> uint32_t { return (x >= 0 && x <= P) ? raw[x * 32] : 0u; };
        auto tl = [&](int q) -> uint32_t {
            if (q < 0 || q >= P) return 0u;
            const uint32_t hi = rw(q + 1);
            return sh ? (hi << 1) | (rw(q) >> 31) : hi;
        };
        auto al = [&](int q) -> uint32_t { return (q >= 0 && q < P) ? col[q * FTP] : 0u; };
        const int64_t et = eik + ekj - 1 + top;
        const int32_t sy = sik ^ skj ^ 1;  // sign of -t
        int64_t *eo = &ex(R.Z, i, j);
        int32_t *so = &sg(R.Z, i, j);
        if (col[(P - 1) * FTP] == 0u) {  // 0 - t
            for (int q = 0; q < P; ++q) col[q * FTP] = tl(q);
            *eo = et;
            *so = sy;
        } else {
            const bool subtract = sa != sy;
            bool a_is_x = ea > et || (ea == et && !subtract);
            bool zero = false;
            if (ea == et && subtract) {
                int c = 0;
                for (int q = P - 1; q >= 0 && c == 0; --q) {
                    const uint32_t x = al(q), y = tl(q);
                    c = x > y ? 1 : (x < y ? -1 : 0);
                }
                zero = c == 0;
                a_is_x = c > 0;
            }
            if (zero) {
                for (int q = 0; q < P; ++q) col[q * FTP] = 0u;
                *eo = 0;
                *so = 0;
            } else {
                const int pbits = 32 * P;
                const int64_t eX = a_is_x ? ea : et, eY = a_is_x ? et : ea;
                const int32_t sX = a_is_x ? sa : sy;
                const uint64_t d = (uint64_t)eX - (uint64_t)eY;
                const int gsh = subtract ? (int)(d < 2 ? d : 2) : 0;      // left shift of X
                const uint64_t rsu = subtract ? (d < 2 ? 0 : d - 2) : d;  // right shift of Y
                const int rs = (int)(rsu > (uint64_t)(pbits + 64) ? (uint64_t)(pbits + 64) : rsu);
                const int w = rs / 32;
                const int b = rs % 32;
                uint32_t st = 0;  // sticky: any bit of Y below bit rs (subtraction only)
                if (subtract && rs > 0) {
                    bool any = false;
                    for (int q = 0; q < P && q <= w && !any; ++q) {
                        const uint32_t v = a_is_x ? tl(q) : al(q);
                        if (q < w) any = v != 0u;
                        else if (b) any = (v & ((1u << b) - 1u)) != 0u;
                    }
                    st = any ? 1u : 0u;
                }
                // pass 1: G = X 2^gsh +- (Y >> rs) -+ sticky over P + 1 limbs, in
                // place; a difference is X + ~Y' + (1 - sticky) in two's
                // complement, so both cases are one carry chain.  Step q reads X
                // limb q and Y limb w+q+1 (both at or above the limb it writes).
                const int oa = a_is_x ? 0 : w + 1, ot = a_is_x ? w + 1 : 0;
                const uint32_t ymask = subtract ? 0xFFFFFFFFu : 0u;
                uint32_t c = subtract ? 1u - st : 0u;
                uint32_t xprev = 0, gprev = 0;
                // single pass where G's length is known from its top limbs: step
                // q writes result limb q - w0 - 1 (at or below the limb it reads)
                // instead of G limb q; result limb -1 goes to the unused row P
                int flen = 0;
                const bool fast = lza_length(P, gsh, w, b, subtract, [&](int q) { return a_is_x ? al(q) : tl(q); },
                                             [&](int q) { return a_is_x ? tl(q) : al(q); }, &flen);
                const int fw0 = flen - pbits >= 0 ? 0 : -1, fbb = flen - pbits - 32 * fw0;
                uint32_t ylo = a_is_x ? tl(w) : al(w);
                uint32_t wlo = rw(ot);  // record word of t limb q + ot, streamed upwards
                // record words W(ot + 1 + q), q = 0..P, in a ring of PF registers
                // fetched PF steps ahead, so the loads overlap the carry chain.
                // The loads are unconditional (the record buffer is padded past
                // its last record) and words past P are zeroed where they are used.
                constexpr int PF = 32;
                uint32_t ring[PF];
                const int xlim = P - ot - 1;  // step q uses a real word iff q <= xlim
                const uint32_t *rp = raw + (ot + 1) * 32;
#pragma unroll
                for (int u = 0; u < PF; ++u) ring[u] = rp[u * 32];
                const int na = P - oa;  // step q reads a real limb of a iff q < na
                const int arow_max = P * FTP;  // LDS offset of row P (reads clamp there)
                int abase = oa * FTP;           // LDS offset of a's limb q0 + oa
                auto step1 = [&](int q, int u, uint32_t ar) __attribute__((always_inline)) {
                    const uint32_t whi = q <= xlim ? ring[u] : 0u;
                    ring[u] = rp[(q + PF) * 32];
                    const uint32_t tsh = sh ? __builtin_amdgcn_alignbit(whi, wlo, 31) : whi;
                    const uint32_t tv = q + ot < P ? tsh : 0u;
                    wlo = whi;
                    const uint32_t av = q < na ? ar : 0u;
                    const uint32_t xq = a_is_x ? av : tv;
                    const uint32_t yhi = a_is_x ? tv : av;
                    const uint32_t xg = gsh ? __builtin_amdgcn_alignbit(xq, xprev, 32 - gsh) : xq;
                    const uint32_t ysh = __builtin_amdgcn_alignbit(yhi, ylo, b);
                    const uint64_t t = (uint64_t)xg + (ysh ^ ymask) + c;
                    const uint32_t gq = (uint32_t)t;
                    const int row = fast ? (q - fw0 - 1 >= 0 ? q - fw0 - 1 : P) : q;
                    col[row * FTP] = fast ? __builtin_amdgcn_alignbit(gq, gprev, fbb) : gq;
                    gprev = gq;
                    c = (uint32_t)(t >> 32);
                    xprev = xq;
                    ylo = yhi;
                };
                // full blocks (one load per step on every path), then the rest.
                // A block's limbs of a are read from LDS before its steps
                // write: step u reads row q0 + oa + u and writes row q0 + u or
                // q0 + u - 1, so no row is read after the block writes it, and
                // the reads need not wait for the writes.
                int q0 = 0;
                for (; q0 + PF <= P + 1; q0 += PF, abase += PF * FTP) {
                    uint32_t ab[PF];
#pragma unroll
                    for (int u = 0; u < PF; ++u) ab[u] = col[min(abase + u * FTP, arow_max)];
#pragma unroll
                    for (int u = 0; u < PF; ++u) step1(q0 + u, u, ab[u]);
                }
                {
                    uint32_t ab[PF];
#pragma unroll
                    for (int u = 0; u < PF; ++u) ab[u] = col[min(abase + u * FTP, arow_max)];
#pragma unroll
                    for (int u = 0; u < PF; ++u) {
                        if (q0 + u > P) break;
                        step1(q0 + u, u, ab[u]);
                    }
                }
                // pass 2: normalise G (limbs 0..P, G < 2^(p+2)) to p bits, in place
                int qt = P;
                if (fast) {
                    *eo = eX - gsh - pbits + flen;
                    *so = sX;
                } else {
                while (qt >= 0 && col[qt * FTP] == 0u) --qt;
                if (qt < 0) {
                    for (int q = 0; q < P; ++q) col[q * FTP] = 0u;
                    *eo = 0;
                    *so = 0;
                } else {
                    const int L = 32 * qt + 32 - __clz(col[qt * FTP]);
                    const int sr = L - pbits;  // bits to drop (negative: shift left)
                    if (sr >= 0) {
                        // sr <= 2: limb q = bits of G limbs q and q + 1, ascending
                        uint32_t lo = col[0];
                        for (int q = 0; q < P; ++q) {
                            const uint32_t hi = col[(q + 1) * FTP];
                            col[q * FTP] = __builtin_amdgcn_alignbit(hi, lo, sr);
                            lo = hi;
                        }
                    } else {  // cancellation: shift left, reading at or below: descending
                        const int w0 = -((-sr + 31) / 32);
                        const int bb = sr - 32 * w0;
                        auto gl = [&](int idx) -> uint32_t { return (idx >= 0 && idx <= P) ? col[idx * FTP] : 0u; };
                        for (int q = P - 1; q >= 0; --q) {
                            const uint32_t lo = gl(q + w0), hi = gl(q + w0 + 1);
                            col[q * FTP] = __builtin_amdgcn_alignbit(hi, lo, bb);
                        }
                    }
                    *eo = eX - gsh - pbits + L;
                    *so = sX;
                }
                }
            }
        }
    }
    mpw::wsync();
    {
        uint4 *dst = (uint4 *)arow;
        for (int c = lane; c < nch; c += MP_WAVE) {
            const int ee = (int)(((uint64_t)c * magic) >> 24);
            const uint32_t *d = lds + 4 * (c - ee * cpe) * FTP + ee;
            dst[c] = make_uint4(d[0], d[FTP], d[2 * FTP], d[3 * FTP]);
        }
    }
}

__global__ void __launch_bounds__(64) k_mfma_prep(MatDev A, uint8_t *Lr, uint8_t *Ub, const int32_t *info,
                                                  int64_t k, int64_t n, int P) {
    extern __shared__ uint32_t lds_raw[];
    mfma_prep_body(lds_raw, A, Lr, Ub, info, k, n, P, flat_block());
}

template <int NC, int WAVES, bool FUSE = false>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_update_mfma(MatDev A, const uint8_t *Lr, const uint8_t *Ub, uint32_t *T, const int32_t *info, int64_t k, int64_t n,
              int P, int64_t ip0, int64_t rows) {
    extern __shared__ uint32_t lds_raw[];
    update_mfma_body<NC, WAVES, FUSE>(lds_raw, A, Lr, Ub, T, info, k, n, P, ip0, rows, flat_block(), true);
}

// The finish of step k, and the first part of step k+1: the workgroup that
// holds a_{k+1,k+1} (block 0) goes on, once its tile is stored, to the next
// pivot's reciprocal and D_{k+1} (pivot_recip_body), while the other
// workgroups of the launch are still finishing -- the reciprocal leaves the
// chain of dependent launches.  Its zero / overflow code goes to the pending
// word rw[P + 2] rather than to info, which the launch's other workgroups are
// reading; step k+1's divide kernel moves it into info.  rw == nullptr: no
// look-ahead.
// The same finish for any P, up to 64 elements per wave: lane e carries the
// chain of element j0 + e, and the elements' limbs move between HBM and LDS in
// chunks of 32 limbs (8 lanes move one element's chunk as four 16-byte
// pieces, so 8 elements share one load or store instruction and every line
// is used whole).  Step q of the chain forms G limb q and emits result limb
// q - 1, so chunk c (steps 32c + 1 .. 32c + 32) holds the limbs of a it
// consumes and, in the same LDS cells, the result limbs 32c .. 32c + 31 it
// produces.  The next chunk's limbs of a are loaded into registers while a
// chunk is computed, and the record words come from a ring of 32 registers
// filled 31 steps ahead (lanes of one 32-column block read one line).  No
// limb of a is stored before its load has been consumed.  An element whose
// result length is not known from the top limbs keeps G in its record (word
// q written after every read of it) and is normalised by a second pass.
typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));
typedef u32x4v u32x4u __attribute__((aligned(4)));  // 16 bytes at a 4-byte offset

// NE (64 or 32) elements of the trailing block, the columns j0 .. j0 + cnt - 1
// (cnt <= NE) of row ip, records of panel [ip0, ...).  LDS finish_tile_lds(NE)
// bytes.
template <int NE>
__device__ __forceinline__ void finish_stream_tile(uint32_t *lds, MatDev A, uint32_t *__restrict__ T, int64_t k,
                                                   int64_t n, int P, int64_t ip0, int64_t ip, int64_t j0, int cnt) {
    const MfmaGeom g = mfma_geom(P);
    const int64_t m = n - k - 1;
    const int64_t njb = (m + 31) / 32;
    constexpr int FT = 64, CP = kFinCP, C = kFinC;
    static_assert(C == 32 && (NE == 64 || NE == 32), "a chunk move is 8 lanes x 4 limbs per element, 8 elements per pass");
    const int64_t i = k + 1 + ip;
    if (el(A, i, k, P)[P - 1] == 0u) return;  // zero multiplier: the row keeps its values
    // element e2's limbs (e2 < cnt)
    auto eptr = [&](int e2) -> uint32_t * { return el(A, i, k + 1 + j0 + e2, P); };
    // LDS: element e's chunk at chunk + e CP (limbs 0..C-1, then a spare
    // word); rows of 36 words keep the 16-byte accesses of 8 lanes on
    // distinct banks; lanes past NE use row NE
    uint32_t *chunk = lds;
    int32_t *eoff = (int32_t *)(lds + (NE + 1) * CP);  // per element (lane): 1 + its offset into a, or -1: not live
    int32_t *sflag = eoff + FT;                  // per element: its result is stored from the chunks
    const int e = mpw::lane();
    const bool in = e < cnt;
    const int ee = in ? e : 0;
    const int64_t jp = j0 + ee, j = k + 1 + jp;
    uint32_t *am = eptr(ee);
    uint32_t *trow = T + (ip - ip0) * njb * (int64_t)g.TP * 32;  // the row's records
    uint32_t *raw = trow + (jp / 32) * (int64_t)g.TP * 32 + (jp % 32);
    const bool live = in && el(A, k, j, P)[P - 1] != 0u;  // u_j = 0: a_ij is left as it is
    const int pbits = 32 * P;

    // ---- operands, alignment, sticky ----
    int oa = 0, ot = 0, gsh = 0, b = 0, w = 0, sh = 0;
    bool a_is_x = true;
    uint32_t ymask = 0u, cy = 0u;
    int64_t eX = 0;
    int32_t sX = 0;
    auto rw = [&](int x) -> uint32_t { return (x >= 0 && x <= P) ? raw[(int64_t)x * 32] : 0u; };
    auto tl = [&](int q) -> uint32_t {
        if (q < 0 || q >= P) return 0u;
        const uint32_t hi = rw(q + 1);
        return sh ? __builtin_amdgcn_alignbit(hi, rw(q), 31) : hi;
    };
    auto al = [&](int q) -> uint32_t { return (q >= 0 && q < P) ? am[q] : 0u; };
    uint32_t ylo = 0u, wlo = 0u;
    bool fast = false;
    int flen = 0;
    if (live) {
        const int top = (int)(rw(P) >> 31);
        sh = 1 - top;
        const int64_t et = ex(A, i, k) + ex(A, k, j) - 1 + top;
        const int32_t sy = sg(A, i, k) ^ sg(A, k, j) ^ 1;  // sign of -t
        const int64_t ea = ex(A, i, j);
        const int32_t sa = sg(A, i, j);
        bool subtract = false;
        uint32_t st = 0u;
        if (am[P - 1] == 0u) {  // 0 - t: X = t, Y = a = 0 shifted out
            a_is_x = false;
            eX = et;
            sX = sy;
            w = P + 2;
        } else {
            subtract = sa != sy;
            a_is_x = ea > et || (ea == et && !subtract);
            if (ea == et && subtract) {
                int c = 0;
                for (int q = P - 1; q >= 0 && c == 0; --q) {
                    const uint32_t x = al(q), y = tl(q);
                    c = x > y ? 1 : (x < y ? -1 : 0);
                }
                a_is_x = c >= 0;  // c == 0: a = t exactly, X = a, Y = t, G = 0
            }
            eX = a_is_x ? ea : et;
            const int64_t eY = a_is_x ? et : ea;
            sX = a_is_x ? sa : sy;
            const uint64_t d = (uint64_t)eX - (uint64_t)eY;
            gsh = subtract ? (int)(d < 2 ? d : 2) : 0;
            const uint64_t rsu = subtract ? (d < 2 ? 0 : d - 2) : d;
            const int rs = (int)(rsu > (uint64_t)(pbits + 64) ? (uint64_t)(pbits + 64) : rsu);
            w = rs / 32;
            b = rs % 32;
            if (subtract && rs > 0) {
                bool any = false;
                for (int q = 0; q < P && q <= w && !any; ++q) {
                    const uint32_t v = a_is_x ? tl(q) : al(q);
                    if (q < w) any = v != 0u;
                    else if (b) any = (v & ((1u << b) - 1u)) != 0u;
                }
                st = any ? 1u : 0u;
            }
        }
        oa = a_is_x ? 0 : w + 1;
        ot = a_is_x ? w + 1 : 0;
        ymask = subtract ? 0xFFFFFFFFu : 0u;
        cy = subtract ? 1u - st : 0u;
        ylo = a_is_x ? tl(w) : al(w);
        wlo = rw(ot + 1 - sh);
        fast = lza_length(P, gsh, w, b, subtract, [&](int q) { return a_is_x ? al(q) : tl(q); },
                          [&](int q) { return a_is_x ? tl(q) : al(q); }, &flen);
    }
    // single pass: result limb r = bits of G limbs r + fw0 + 1 and r + fw0
    // (fw0 = 0 or -1) shifted right by fbb; it is emitted at step r + 1
    const int fsr = flen - pbits;  // -32 .. 3
    const bool f0 = fsr >= 0;      // fw0 == 0
    const int fbb = f0 ? fsr : fsr + 32;
    if (!live) fast = true;  // (stores nothing: sflag is 0)
    const bool keep_g = __builtin_amdgcn_ballot_w64(!fast) != 0ull;  // some element needs pass 2
    eoff[e] = live ? 1 + oa : -1;
    sflag[e] = live && fast ? 1 : 0;

    // ---- pass 1: G = X 2^gsh +- (Y >> rs) -+ sticky, limbs 0..P ----
    // Limb q of t is bits 31 sh .. of the record words ot + 1 + q and
    // ot + 2 + q, that is alignbit(w_hi, w_lo, 31 sh) of the words
    // ot + 2 - sh + q (w_hi) and ot + 1 - sh + q (w_lo): the lane reads its
    // words from ot + 2 - sh on, so one alignbit serves both cases.  Words
    // past P count as 0.  The words come through a buffer resource over the
    // row's records: the lane's offset in a VGPR, the step's in an SGPR, no
    // address arithmetic per step, and a read past the records returns 0.
    const int rbase = ot + 2 - sh;
    const uint32_t sb = sh ? 31u : 0u;
    const __amdgpu_buffer_rsrc_t trs =
        __builtin_amdgcn_make_buffer_rsrc((void *)trow, (short)0, (int)(njb * g.TP * 32 * 4), kBufferRsrcWord3);
    const uint32_t roff = (uint32_t)(((jp / 32) * (int64_t)g.TP * 32 + (jp % 32) + (int64_t)rbase * 32) * 4);
    auto recw = [&](int q) -> uint32_t { return __builtin_amdgcn_raw_buffer_load_b32(trs, roff, q * 128, 0); };
    uint32_t xprev = 0u, gprev = 0u, hprev = 0u;
    // one step of the chain: G limb q from record word wr and a limb ar;
    // returns result limb q - 1.  INTERIOR: q + ot + 2 <= P and q + oa < P,
    // so no operand needs masking.
    // (wr, wl: the words for steps q and q - 1, i.e. record words rbase + q
    // and rbase + q - 1)
    auto step = [&](int q, uint32_t wr, uint32_t wl, uint32_t ar, auto store_g, auto interior)
                    __attribute__((always_inline)) -> uint32_t {
        const uint32_t whi = (decltype(interior)::value || rbase + q <= P) ? wr : 0u;
        const uint32_t wlo = (decltype(interior)::value || rbase + q - 1 <= P) ? wl : 0u;
        const uint32_t tsh = __builtin_amdgcn_alignbit(whi, wlo, sb);
        const uint32_t tv = (decltype(interior)::value || q + ot < P) ? tsh : 0u;
        const uint32_t av = (decltype(interior)::value || q + oa < P) ? ar : 0u;
        const uint32_t xq = a_is_x ? av : tv;
        const uint32_t yhi = a_is_x ? tv : av;
        const uint32_t xg = gsh ? __builtin_amdgcn_alignbit(xq, xprev, 32 - gsh) : xq;
        const uint32_t ysh = __builtin_amdgcn_alignbit(yhi, ylo, b);
        const uint64_t t = (uint64_t)xg + (ysh ^ ymask) + cy;
        const uint32_t gq = (uint32_t)t;
        cy = (uint32_t)(t >> 32);
        xprev = xq;
        ylo = yhi;
        // result limb q - 1: G limbs q, q - 1 (fw0 = 0) or q - 1, q - 2
        const uint32_t hq = f0 ? gq : gprev;
        const uint32_t r = __builtin_amdgcn_alignbit(hq, hprev, fbb);
        // G limb q to record word q (read at step q - ot - 2 or before)
        if (decltype(store_g)::value && !fast && q <= P) raw[(int64_t)q * 32] = gq;
        hprev = hq;
        gprev = gq;
        return r;
    };
    // Every lane runs the chain, and every chunk, the last included, issues
    // the same loads (addresses clamped into the element; record reads past
    // the row's records return 0; what lies past limb P - 1 or word P is
    // never used): no branch around the loads, so the ring stays in its
    // registers and each step waits only for its own word.  A lane with no
    // element is "fast" and stores nothing.
    // Chunks whose steps need no masking on any lane of the wave come first.
    const int need = __builtin_amdgcn_readfirstlane(mpw::wave_max(live ? max(ot + 2, oa + 1) : 0));
    mpw::wsync();  // eoff and sflag are visible
    // this lane moves limbs 4 sub .. 4 sub + 3 of the chunks of elements
    // 8 s + grp, s < NE / 8
    constexpr int NS = NE / 8;
    const int sub = e & 7, grp = e >> 3;
    int aoff[NS];
    uint32_t st_mask = 0u;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        aoff[s] = eoff[8 * s + grp];
        st_mask |= sflag[8 * s + grp] ? 1u << s : 0u;
    }
    // element 8 s + grp's limbs of a for the chunk whose first step is q0:
    // limbs x .. x + 3, x = q0 + oa + 4 sub, read from x - d (d > 0 only where
    // x > P - 4, so that every address stays inside the element; limbs at or
    // past P are masked by the step).  One 16-byte load per element and no
    // branch, so no load waits for another.
    auto a_at = [&](int s, int q0) -> int { return q0 - 1 + aoff[s] + 4 * sub; };
    auto load_a = [&](u32x4v *v, int q0) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            // (columns past the block are not read)
            v[s] = *(const u32x4u *)(eptr(min(8 * s + grp, cnt - 1)) + min(a_at(s, q0), P - 4));
        }
    };
    // the first chunk's limbs of a, then the record words (the order in
    // which every later chunk issues them)
    u32x4v va[NS];
    load_a(va, 1);
    uint32_t ring[C];
    using no_g = std::integral_constant<bool, false>;
    using with_g = std::integral_constant<bool, true>;
    using masked = std::integral_constant<bool, false>;
    using inner = std::integral_constant<bool, true>;
    // ring slot u holds the word of step q0 + u of the current chunk, slot
    // C - 1 that of step q0 - 1 until step q0 has read it (as w_lo); after
    // step q0 + u the slot read as w_lo, (u + C - 1) mod C, takes the word of
    // step q0 + u + C - 1 (a word is read as w_hi, then as w_lo, then
    // replaced, so no register is needed twice)
    if (keep_g) (void)step(0, recw(0), wlo, al(oa), with_g{}, masked{});
    else (void)step(0, recw(0), wlo, al(oa), no_g{}, masked{});
    // in the order in which the chunks reload them (the wait for a word
    // then counts the loads issued after it)
    ring[C - 1] = recw(0);
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < C - 1; ++u) {
        ring[u] = recw(1 + u);
        asm volatile("" ::: "memory");
    }
    // the chunks: a loop of its own for waves that keep G (no branch on it
    // inside the loop, whose registers then stay put)
    auto chunk_at = [&](int q0, auto store_g, auto interior) __attribute__((always_inline)) {
        {
            mpw::wsync();  // the previous chunk's results have left LDS
    #pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int d = a_at(s, q0) - min(a_at(s, q0), P - 4);
                uint32_t *row = chunk + (8 * s + grp) * CP;
                if (__builtin_amdgcn_ballot_w64(d != 0) == 0ull) {
                    *(u32x4v *)(row + 4 * sub) = va[s];
                } else {
                    // limb x - d + z belongs at 4 sub + z - d; limbs before the
                    // chunk (consumed already) go to the spare word C
                    const int rb = 4 * sub - d;
                    row[rb >= 0 ? rb : C] = va[s].x;
                    row[rb + 1 >= 0 ? rb + 1 : C] = va[s].y;
                    row[rb + 2 >= 0 ? rb + 2 : C] = va[s].z;
                    row[rb + 3 >= 0 ? rb + 3 : C] = va[s].w;
                }
            }
            load_a(va, q0 + C);
            mpw::wsync();
            // four steps per 16-byte LDS read and write of the lane's own row
            // (steps past P, in the last chunk, produce limbs that are not stored)
            uint32_t *mine = chunk + min(e, NE) * CP;
    #pragma unroll
            for (int t4 = 0; t4 < C / 4; ++t4) {
                const u32x4v a4 = *(const u32x4v *)(mine + 4 * t4);
                u32x4v r4;
    #pragma unroll
                for (int z = 0; z < 4; ++z) {
                    const int u = 4 * t4 + z, q = q0 + u;
                    const int ul = (u + C - 1) % C;
                    r4[z] = step(q, ring[u], ring[ul], a4[z], store_g, interior);
                    ring[ul] = recw(q + C - 1);
                    // one reload per step, in step order: the ring keeps its
                    // registers across the loop edge, so no wait gathers there
                    __builtin_amdgcn_sched_barrier(0);
                }
                *(u32x4v *)(mine + 4 * t4) = r4;
            }
            mpw::wsync();
            // results: limbs q0 - 1 + 4 sub .. + 3 of the single-pass elements
            const int r0 = q0 - 1 + 4 * sub;
    #pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (!(st_mask >> s & 1u) || r0 >= P) continue;
                const u32x4v c = *(const u32x4v *)(chunk + (8 * s + grp) * CP + 4 * sub);
                uint32_t *dst = eptr(8 * s + grp) + r0;
                if (r0 + 3 < P) {
                    *(u32x4u *)dst = c;
                } else {
    #pragma unroll
                    for (int z = 0; z < 4; ++z)
                        if (r0 + z < P) dst[z] = c[z];
                }
            }
        }
    };
    auto chunks = [&](auto store_g) __attribute__((always_inline)) {
        int q0 = 1;
        for (; q0 + C - 1 + need <= P; q0 += C) chunk_at(q0, store_g, inner{});
        for (; q0 <= P; q0 += C) chunk_at(q0, store_g, masked{});
    };
    if (keep_g) chunks(with_g{});
    else chunks(no_g{});
    if (live && fast) {
        ex(A, i, j) = eX - gsh - pbits + flen;
        sg(A, i, j) = sX;
    }
    if (!keep_g) return;

    // ---- pass 2: normalise G (record words 0..P) to p bits, per element ----
    mpw::wsync();  // G's stores precede these loads
    if (!live || fast) return;
    auto gw = [&](int x) -> uint32_t { return (x >= 0 && x <= P) ? raw[(int64_t)x * 32] : 0u; };
    int qt = P;
    while (qt >= 0 && gw(qt) == 0u) --qt;
    if (qt < 0) {
        for (int r = 0; r < P; ++r) am[r] = 0u;
        ex(A, i, j) = 0;
        sg(A, i, j) = 0;
        return;
    }
    const int L = 32 * qt + 32 - __clz(gw(qt));
    const int sr = L - pbits;  // bits to drop (negative: shift left)
    const int w0 = sr >= 0 ? 0 : -((-sr + 31) / 32);
    const int bb = sr - 32 * w0;
    for (int r0 = 0; r0 < P; r0 += C) {
        uint32_t gv[C + 1];
#pragma unroll
        for (int u = 0; u <= C; ++u) gv[u] = gw(r0 + u + w0);  // result limb r = G limbs r + w0, r + w0 + 1
#pragma unroll
        for (int u = 0; u < C; ++u)
            if (r0 + u < P) am[r0 + u] = __builtin_amdgcn_alignbit(gv[u + 1], gv[u], bb);
    }
    ex(A, i, j) = eX - gsh - pbits + L;
    sg(A, i, j) = sX;
}

// the finish launch: workgroup bx takes 64 consecutive elements of a row
__device__ __forceinline__ void finish_stream_body(uint32_t *lds, MatDev A, uint32_t *__restrict__ T, int64_t k,
                                                   int64_t n, int P, int64_t ip0, int64_t rows, int64_t bx) {
    const int64_t m = n - k - 1;
    const int64_t ntile = (m + 63) / 64;
    const int64_t ip = ip0 + bx / ntile, j0 = (bx % ntile) * 64;
    if (bx / ntile >= rows || ip >= m) return;
    finish_stream_tile<64>(lds, A, T, k, n, P, ip0, ip, j0, (int)min((int64_t)64, m - j0));
}

// STREAM must equal finish_streams(P); the two forms are separate kernels so
// that each gets its own register allocation.
template <bool STREAM>
__device__ __forceinline__ void finish_body(uint32_t *lds, MatDev A, uint32_t *__restrict__ T,
                                            const int32_t *info, int64_t k, int64_t n, int P, int64_t ip0,
                                            int64_t rows, int64_t bx, MatDev D, uint32_t *rw) {
    if (*info != 0) return;
    if constexpr (STREAM) finish_stream_body(lds, A, T, k, n, P, ip0, rows, bx);
    else finish_tile_body(lds, elim_rank1(A, k, n), T, P, ip0, rows, bx);
    // (block 0 of the panel holding row k+1 holds a_{k+1,k+1})
    if (rw != nullptr && ip0 == 0 && bx == 0 && k + 1 < n) {
        mpw::wsync();  // the tile's stores are visible to the wave, its LDS is free
        int32_t *pend = (int32_t *)(rw + P + 2);
        pivot_recip_body(lds, A, D, info, pend, rw, k + 1, n, P, 1);
        mpw::wsync();
        pivot_recip_body(lds, A, D, info, pend, rw, k + 1, n, P, 0);
    }
}

// Look-ahead pays while the pivot's LDS scratch does not crowd the finish
// launch (P <= 256 or so); beyond, the pivot keeps a launch of its own.
__host__ __device__ inline bool finish_lookahead_ok(int P) { return pivot_lds_bytes(P) <= 36u * 1024u; }
// LDS of the finish launch: the tile, or the pivot's scratch if larger
__host__ __device__ inline size_t finish_launch_lds(int P) {
    const size_t a = finish_lds_bytes(P), b = finish_lookahead_ok(P) ? pivot_lds_bytes(P) : 0;
    return a > b ? a : b;
}

template <bool STREAM>
__global__ void __launch_bounds__(64) k_finish(MatDev A, uint32_t *T, const int32_t *info, int64_t k,
                                               int64_t n, int P, int64_t ip0, int64_t rows, MatDev D, uint32_t *rw) {
    extern __shared__ uint32_t lds_raw[];
    finish_body<STREAM>(lds_raw, A, T, info, k, n, P, ip0, rows, flat_block(), D, rw);
}

// The LDS-tile finish of any rank-1 update (P <= 256): all R.mr rows, the
// records from k_prod_lane_r1; nothing when info != 0.
__global__ void __launch_bounds__(64) k_finish_r1(Rank1 R, const uint32_t *T, const int32_t *info, int P) {
    extern __shared__ uint32_t lds_raw[];
    if (*info != 0) return;
    finish_tile_body(lds_raw, R, T, P, 0, R.mr, flat_block());
}

}  // namespace mpk
