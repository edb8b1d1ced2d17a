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
// per K-step (the row's digits are staged there reversed).  Tiles outside the
// band 0 <= r - c <= P8 are skipped.
//
// Epilogue.  Column sums are biased, S'_r = S_r + 2^27 - 2^19 [r >= 1], which
// makes them positive (< 2^28) and adds sum_r bias_r 256^r = 2^27 256^R -- a
// multiple of 2^(2p) -- to the total, invisible in the low 2p bits.  Four
// consecutive S' form a 64-bit limb column V_q < 2^53, and one lane per column
// runs the carry chain limb_q = (V_q + c) mod 2^32, c = (V_q + c) >> 32 from
// the lowest limb up.  Limbs P-1 .. 2P-1 of each product go to a scratch
// buffer; a wave-cooperative kernel then truncates the product to p bits and
// forms RZ_p(a_ij - RZ_p(l_i u_j)).
#pragma once

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
    g.LR = g.P8 + 192;
    g.Q = g.P8 + 67;  // Q = 3 mod 4: reversed limbs land on aligned words
    g.TP = P + 4;
    g.nchunks = (2 * g.P8 + 255) / 256;
    return g;
}

__host__ __device__ inline bool mfma_supported(int P) { return P >= 8 && P % 8 == 0; }

constexpr int64_t kXcds = 8;  // MI355X: 8 accelerator complex dies, one L2 each

// workgroups of k_update_mfma for an m x m trailing block
__host__ __device__ inline int64_t mfma_update_blocks(int64_t m) {
    const int64_t njb = (m + 31) / 32;
    return njb >= kXcds ? kXcds * m * ((njb + kXcds - 1) / kXcds) : m * njb;
}

// LDS for k_update_mfma: the reversed digit row, then 32 columns x 65 uint64
__host__ __device__ inline size_t mfma_lds_bytes(int P) {
    MfmaGeom g = mfma_geom(P);
    return (size_t)g.LR + 32u * 65u * 8u;
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
        // word w of the reversed row holds digit word P + 16 - w, bytes reversed
        uint32_t *out = (uint32_t *)(Lr + b * (int64_t)g.LR);
        for (int w = mpw::lane(); w < g.LR / 4; w += MP_WAVE) {
            int qd = P + 16 - w;
            uint32_t v = 0;
            if (qd >= 0 && qd <= P) v = __builtin_bswap32(dw[qd]);
            out[w] = v;
        }
    } else {
        uint32_t *out = (uint32_t *)(Ub + (b - m) * (int64_t)g.K8);
        for (int w = mpw::lane(); w < g.K8 / 4; w += MP_WAVE) out[w] = w <= P ? dw[w] : 0u;
    }
}

// A fragment of the Toeplitz block with diagonal offset d = r0 - c0: lane
// (r = lane % 32, h = lane / 32) holds T[r0 + r][c0 + 16h + b], b = 0..15.
__device__ __forceinline__ v4i load_a(const uint8_t *lr, int d, int P8, int Q) {
    v4i v = {0, 0, 0, 0};
    if (d >= -31 && d <= P8 + 31) {
        const int r = mpw::lane() & 31, h = mpw::lane() >> 5;
        __builtin_memcpy(&v, lr + (Q - d - r + 16 * h), 16);
    }
    return v;
}

// Product top limbs: for every row i' (multiplier l = a_{k+1+i', k}) and
// column block jb of 32, word x <= P of the record of column j' = 32 jb + j is
// limb P-1+x of l * u_{j'}, stored limb-major across the block's 32 columns:
// T[((i' njb + jb) TP + x) 32 + j].
__device__ __forceinline__ void update_mfma_body(uint32_t *lds_raw, MatDev A, const uint8_t *Lr, const uint8_t *Ub, uint32_t *T,
                                 const int32_t *info, int64_t k, int64_t n, int P, int64_t bx, bool xcd_aware) {
    if (*info != 0) return;
    const MfmaGeom g = mfma_geom(P);
    const int64_t m = n - k - 1;
    const int64_t njb = (m + 31) / 32;
    int64_t ip, jb;
    if (xcd_aware && njb >= kXcds) {
        // workgroups go to the 8 XCDs round-robin: XCD x takes the column
        // blocks jb = x (mod 8), so each XCD's L2 holds only its share of the
        // pivot-row digits
        const int64_t xcd = bx % kXcds, loc = bx / kXcds;
        const int64_t cnt = (njb - xcd + kXcds - 1) / kXcds;
        if (loc >= m * cnt) return;
        ip = loc / cnt;
        jb = xcd + kXcds * (loc % cnt);
    } else {
        if (bx >= m * njb) return;
        ip = bx / njb;
        jb = bx % njb;
    }
    if (el(A, k + 1 + ip, k, P)[P - 1] == 0u) return;

    uint8_t *lr = (uint8_t *)lds_raw;
    uint64_t *vbuf = (uint64_t *)(lds_raw + g.LR / 4);
    {
        const uint4 *src = (const uint4 *)(Lr + ip * (int64_t)g.LR);
        uint4 *dst = (uint4 *)lr;
        for (int w = mpw::lane(); w < g.LR / 16; w += MP_WAVE) dst[w] = src[w];
    }
    mpw::wsync();

    const int lane = mpw::lane();
    const int j = lane & 31, h = lane >> 5;
    const int64_t jp = jb * 32 + j;
    const bool jvalid = jp < m;
    const uint8_t *ub = Ub + (jvalid ? jp : 0) * (int64_t)g.K8 + 16 * h;
    uint32_t *tcol = T + (ip * njb + jb) * (int64_t)g.TP * 32 + j;
    const int P8 = g.P8, Q = g.Q;
    uint64_t carry = 0;

    for (int chunk = 0; chunk < g.nchunks; ++chunk) {
        const int r0 = chunk * 256;
        v16i acc[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] = (v16i){0};
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
        for (int t = 0; t < 8; ++t) W[t] = load_a(lr, r0 + 32 * t - c_lo, P8, Q);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            BR[u] = (v4i){0, 0, 0, 0};
            if (jvalid && u < nsteps) BR[u] = *(const v4i *)(ub + c_lo + 32 * u);
        }
        for (int n8 = 0; n8 < nsteps; n8 += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int n = n8 + u;
                const int c0 = c_lo + 32 * n;
                const v4i bv = BR[u];
                BR[u] = (v4i){0, 0, 0, 0};
                if (jvalid && n + 8 < nsteps) BR[u] = *(const v4i *)(ub + c0 + 256);
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(W[(t - u) & 7], bv, acc[t], 0, 0, 0);
                W[(7 - u) & 7] = load_a(lr, r0 - c0 - 32, P8, Q);
            }
        }
        // biased 64-bit limb columns: lane (j, h), tile t, group gq holds r =
        // r0 + 32t + 8gq + 4h + {0..3}, i.e. limb q = r0/4 + 8t + 2gq + h
#pragma unroll
        for (int t = 0; t < 8; ++t) {
#pragma unroll
            for (int gq = 0; gq < 4; ++gq) {
                const int rb = r0 + 32 * t + 8 * gq + 4 * h;
                uint64_t V = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int r = rb + b;
                    const uint32_t bias = r == 0 ? (1u << 27) : ((1u << 27) - (1u << 19));
                    const uint32_t s = (uint32_t)acc[t][4 * gq + b] + bias;
                    V += (uint64_t)s << (8 * b);
                }
                vbuf[j * 65 + 8 * t + 2 * gq + h] = V;
            }
        }
        mpw::wsync();
        if (h == 0) {
            const int qbase = r0 / 4;
            const int qend = min(64, 2 * P - qbase);  // limbs of this chunk below 2P
            for (int q8 = 0; q8 < qend; q8 += 8) {
                uint64_t v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = vbuf[j * 65 + q8 + u];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = qbase + q8 + u;
                    const uint64_t x = v[u] + carry;
                    carry = x >> 32;
                    if (q8 + u < qend && q >= P - 1 && jvalid) tcol[(int64_t)(q - (P - 1)) * 32] = (uint32_t)x;
                }
            }
        }
        mpw::wsync();
    }
}

// ---------------------------------------------------------------------------
// Finish of the update, one lane per element: a_ij = RZ_p(a_ij - t) with
// t = RZ_p(l_i u_j) rebuilt from the product's top limbs (raw word x = product
// limb P-1+x, x = 0..P, in the limb-major record above).  Same case analysis
// as mpw::addsub, run by one lane over the limbs from low to high with
// one-limb register windows: pass 1 writes G, the exact p+2-bit intermediate,
// to its own limb-major buffer (no location is read after it is written), and
// pass 2 normalises G into a_ij.  Lanes of a wave take consecutive columns, so
// the record and G accesses are coalesced.
// ---------------------------------------------------------------------------

// limb q (0..P-1) of a or t through a strided word view (0 outside)
struct LimbSrc {
    const uint32_t *p;  // raw words, word idx at p[idx * stride]
    int64_t stride;
    int off;            // limb q uses words q+off and q+off-1
    int sh;             // 0: limb = w[q+off]; 1: limb = (w[q+off] << 1) | (w[q+off-1] >> 31)
    int P;
    __device__ __forceinline__ uint32_t word(int64_t idx) const {
        return (idx >= 0 && idx < (int64_t)P + off) ? p[idx * stride] : 0u;
    }
    __device__ __forceinline__ uint32_t limb(int64_t q) const {
        if (q < 0 || q >= P) return 0u;
        const uint32_t hi = word(q + off);
        if (!sh) return hi;
        return (hi << 1) | (word(q + off - 1) >> 31);
    }
};

__device__ __forceinline__ void sub_lane_body(MatDev A, const uint32_t *__restrict__ T, uint32_t *__restrict__ Gb,
                              const int32_t *info, int64_t k, int64_t n, int P, int64_t slot) {
    if (*info != 0) return;
    const MfmaGeom g = mfma_geom(P);
    const int64_t m = n - k - 1;
    const int64_t njb = (m + 31) / 32;
    const int64_t ip = slot / (njb * 32), jp = slot % (njb * 32);
    if (ip >= m || jp >= m) return;
    const int64_t i = k + 1 + ip, j = k + 1 + jp;
    if (el(A, i, k, P)[P - 1] == 0u || el(A, k, j, P)[P - 1] == 0u) return;
    const int64_t rec = (ip * njb + jp / 32) * (int64_t)g.TP * 32 + (jp % 32);
    const uint32_t *__restrict__ raw = T + rec;
    uint32_t *__restrict__ G = Gb + rec;
    uint32_t *__restrict__ am = el(A, i, j, P);
    const int64_t p = 32LL * P;
    const int top = (int)(raw[(int64_t)P * 32] >> 31);
    const LimbSrc ts{raw, 32, 1, 1 - top, P};
    const LimbSrc as{am, 1, 0, 0, P};
    const int64_t et = ex(A, i, k) + ex(A, k, j) - 1 + top;
    const int32_t sy = sg(A, i, k) ^ sg(A, k, j) ^ 1;  // sign of -t
    const int64_t ea = ex(A, i, j);
    const int32_t sa = sg(A, i, j);
    int64_t *eo = &ex(A, i, j);
    int32_t *so = &sg(A, i, j);
    if (am[P - 1] == 0u) {  // 0 - t
        for (int q = 0; q < P; ++q) am[q] = ts.limb(q);
        *eo = et;
        *so = sy;
        return;
    }
    const bool subtract = sa != sy;
    bool a_is_x = ea > et || (ea == et && !subtract);
    if (ea == et && subtract) {
        int c = 0;
        for (int q = P - 1; q >= 0 && c == 0; --q) {
            const uint32_t x = as.limb(q), y = ts.limb(q);
            c = x > y ? 1 : (x < y ? -1 : 0);
        }
        if (c == 0) {
            for (int q = 0; q < P; ++q) am[q] = 0u;
            *eo = 0;
            *so = 0;
            return;
        }
        a_is_x = c > 0;
    }
    const LimbSrc X = a_is_x ? as : ts, Y = a_is_x ? ts : as;
    const int64_t eX = a_is_x ? ea : et, eY = a_is_x ? et : ea;
    const int32_t sX = a_is_x ? sa : sy;
    const uint64_t d = (uint64_t)eX - (uint64_t)eY;
    const int gsh = subtract ? (int)(d < 2 ? d : 2) : 0;       // left shift of X
    const uint64_t rsu = subtract ? (d < 2 ? 0 : d - 2) : d;   // right shift of Y
    const int64_t rs = (int64_t)(rsu > (uint64_t)(p + 64) ? (uint64_t)(p + 64) : rsu);
    const int64_t w = rs / 32;
    const int b = (int)(rs % 32);
    uint32_t cb = 0;  // carry (sum) or borrow (difference)
    if (subtract && rs > 0) {  // sticky: any bit of Y below bit rs
        bool st = false;
        for (int64_t q = 0; q < P && q <= w && !st; ++q) {
            const uint32_t v = Y.limb(q);
            if (q < w) st = v != 0u;
            else if (b) st = (v & ((1u << b) - 1u)) != 0u;
        }
        cb = st ? 1u : 0u;
    }
    // pass 1: G = X 2^gsh +- (Y >> rs) -+ sticky, P + 1 limbs
    uint32_t xprev = 0;
    uint32_t ylo = Y.limb(w);
    for (int q = 0; q <= P; ++q) {
        const uint32_t xq = X.limb(q);
        const uint32_t yhi = Y.limb(w + q + 1);
        const uint32_t xg = gsh ? ((xq << gsh) | (xprev >> (32 - gsh))) : xq;
        const uint32_t ysh = b ? ((ylo >> b) | (yhi << (32 - b))) : ylo;
        uint32_t gq;
        if (!subtract) {
            const uint64_t sum = (uint64_t)xg + ysh + cb;
            gq = (uint32_t)sum;
            cb = (uint32_t)(sum >> 32);
        } else {
            const int64_t df = (int64_t)xg - (int64_t)ysh - (int64_t)cb;
            gq = (uint32_t)df;
            cb = df < 0 ? 1u : 0u;
        }
        G[(int64_t)q * 32] = gq;
        xprev = xq;
        ylo = yhi;
    }
    // pass 2: normalise G to p bits into a_ij
    int qt = P;
    while (qt >= 0 && G[(int64_t)qt * 32] == 0u) --qt;
    if (qt < 0) {
        for (int q = 0; q < P; ++q) am[q] = 0u;
        *eo = 0;
        *so = 0;
        return;
    }
    const int64_t L = 32LL * qt + 32 - __clz(G[(int64_t)qt * 32]);
    const int64_t sr = L - p;  // bits to drop (negative: shift left)
    const int64_t w0 = sr >= 0 ? sr / 32 : -((-sr + 31) / 32);
    const int bb = (int)(sr - 32 * w0);
    for (int q = 0; q < P; ++q) {
        const int64_t lo_i = q + w0, hi_i = q + w0 + 1;
        const uint32_t lo = (lo_i >= 0 && lo_i <= P) ? G[lo_i * 32] : 0u;
        const uint32_t hi = (hi_i >= 0 && hi_i <= P) ? G[hi_i * 32] : 0u;
        am[q] = bb ? ((lo >> bb) | (hi << (32 - bb))) : lo;
    }
    *eo = eX - gsh - p + L;
    *so = sX;
}

// elements of the m x m trailing block in lane slots (m rows x njb*32 columns)
__host__ __device__ inline int64_t sub_lane_slots(int64_t m) { return m * ((m + 31) / 32) * 32; }

__global__ void __launch_bounds__(64) k_mfma_prep(MatDev A, uint8_t *Lr, uint8_t *Ub, const int32_t *info,
                                                  int64_t k, int64_t n, int P) {
    extern __shared__ uint32_t lds_raw[];
    mfma_prep_body(lds_raw, A, Lr, Ub, info, k, n, P, flat_block());
}

__global__ void __launch_bounds__(64) k_update_mfma(MatDev A, const uint8_t *Lr, const uint8_t *Ub, uint32_t *T,
                                                    const int32_t *info, int64_t k, int64_t n, int P) {
    extern __shared__ uint32_t lds_raw[];
    update_mfma_body(lds_raw, A, Lr, Ub, T, info, k, n, P, flat_block(), true);
}

__global__ void __launch_bounds__(64) k_sub_lane(MatDev A, const uint32_t *T, uint32_t *G, const int32_t *info,
                                                 int64_t k, int64_t n, int P) {
    sub_lane_body(A, T, G, info, k, n, P, flat_block() * 64 + threadIdx.x);
}

}  // namespace mpk
