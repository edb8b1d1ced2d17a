// wave_mp.h -- wave-cooperative multiprecision arithmetic for gfx950.
//
// One 64-lane wavefront owns one multiprecision operation.  Operands live in
// LDS; lane t works on limbs t, t+64, t+128, ...  Carries and borrows between
// limbs are resolved with a carry-lookahead over the wave: per block of 64
// limbs each lane forms its generate/propagate bits, two ballots give 64-bit
// masks G and P, and the carry into every lane is read off the integer sum
// (G|P) + G + c_in (the carries of an addition whose generate and propagate
// vectors are G and P).  Every routine is called by all 64 lanes of a
// single-wave workgroup and returns wave-uniform results.
//
// Number format: value = (-1)^s * m * 2^(e - 32P), m with P limbs and the top
// bit set, zero = (m = 0, e = 0, s = 0).  Every result is RZ_p (truncation
// toward zero of the exact result).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MP_WAVE 64

namespace mpw {

__device__ __forceinline__ int lane() { return (int)(threadIdx.x & 63u); }

// LDS visibility between lanes of the (single-wave) workgroup.
__device__ __forceinline__ void wsync() { __syncthreads(); }

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

struct Hdr {
    int64_t e;
    int32_t s;
    bool zero;
};

__device__ __forceinline__ Hdr zero_hdr() { return Hdr{0, 0, true}; }

// ---------------------------------------------------------------------------
// limb vectors in LDS
// ---------------------------------------------------------------------------

__device__ __forceinline__ void fill(uint32_t *d, int n, uint32_t v) {
    for (int q = lane(); q < n; q += MP_WAVE) d[q] = v;
}

__device__ __forceinline__ void copy(uint32_t *d, const uint32_t *s, int n) {
    for (int q = lane(); q < n; q += MP_WAVE) d[q] = s[q];
}

// highest q < n with a[q] != 0, or -1
__device__ __forceinline__ int top_nonzero(const uint32_t *a, int n) {
    int best = -1;
    for (int q = lane(); q < n; q += MP_WAVE)
        if (a[q]) best = q;
    return wave_max(best);
}

// number of significant bits of a (0 when a == 0)
__device__ __forceinline__ int64_t bitlen(const uint32_t *a, int n) {
    int q = top_nonzero(a, n);
    if (q < 0) return 0;
    return 32LL * q + 32 - __clz(a[q]);
}

// d[0..nd) = floor(s * 2^sh) mod 2^(32 nd); sh < 0 shifts right.  d != s.
__device__ __forceinline__ void shift(uint32_t *d, int nd, const uint32_t *s, int ns, int64_t sh) {
    const int64_t hi_clamp = 32LL * (nd + 2), lo_clamp = -32LL * (ns + 2);
    if (sh > hi_clamp) sh = hi_clamp;
    if (sh < lo_clamp) sh = lo_clamp;
    for (int q = lane(); q < nd; q += MP_WAVE) {
        int64_t pos = 32LL * q - sh;  // bit of s that lands on bit 0 of d[q]
        int64_t w = pos >= 0 ? pos / 32 : -((-pos + 31) / 32);
        int b = (int)(pos - 32 * w);
        uint32_t lo = (w >= 0 && w < ns) ? s[w] : 0u;
        uint32_t hi = (w + 1 >= 0 && w + 1 < ns) ? s[w + 1] : 0u;
        d[q] = b ? ((lo >> b) | (hi << (32 - b))) : lo;
    }
}

// any bit of a below bit position `bits` set
__device__ __forceinline__ bool low_bits_nonzero(const uint32_t *a, int n, int64_t bits) {
    bool any = false;
    if (bits > 0) {
        int64_t w = bits / 32;
        int b = (int)(bits % 32);
        for (int q = lane(); q < n; q += MP_WAVE) {
            uint32_t v = a[q];
            if (q < w) any |= (v != 0u);
            else if (q == w && b) any |= ((v & ((1u << b) - 1u)) != 0u);
        }
    }
    return __ballot(any) != 0ull;
}

// carry/borrow into each lane of a 64-limb block from generate/propagate masks
__device__ __forceinline__ uint64_t lookahead(uint64_t G, uint64_t Pm, uint32_t cin) {
    uint64_t A = G | Pm;
    uint64_t S = A + G + (uint64_t)cin;
    return S ^ A ^ G;  // bit t = carry into lane t
}

__device__ __forceinline__ uint32_t block_carry_out(uint64_t G, uint64_t Pm, uint64_t C, int cnt) {
    if (cnt == 64) return (uint32_t)(((G >> 63) | ((Pm >> 63) & (C >> 63))) & 1ull);
    return (uint32_t)((C >> cnt) & 1ull);
}

// d = a + b + cin over n limbs; returns the carry out.  d may alias a or b.
__device__ __forceinline__ uint32_t add(uint32_t *d, const uint32_t *a, const uint32_t *b, int n,
                                        uint32_t cin) {
    uint32_t carry = cin;
    for (int base = 0; base < n; base += MP_WAVE) {
        int q = base + lane();
        int cnt = min(MP_WAVE, n - base);
        uint32_t x = q < n ? a[q] : 0u, y = q < n ? b[q] : 0u;
        uint32_t s = x + y;
        uint64_t valid = cnt == 64 ? ~0ull : ((1ull << cnt) - 1ull);
        uint64_t G = __ballot(s < x) & valid;
        uint64_t Pm = __ballot(s == 0xFFFFFFFFu) & valid;
        uint64_t C = lookahead(G, Pm, carry);
        if (q < n) d[q] = s + (uint32_t)((C >> lane()) & 1ull);
        carry = block_carry_out(G, Pm, C, cnt);
    }
    return carry;
}

// d = a - b - bin over n limbs; returns the borrow out.  d may alias a or b.
__device__ __forceinline__ uint32_t sub(uint32_t *d, const uint32_t *a, const uint32_t *b, int n,
                                        uint32_t bin) {
    uint32_t borrow = bin;
    for (int base = 0; base < n; base += MP_WAVE) {
        int q = base + lane();
        int cnt = min(MP_WAVE, n - base);
        uint32_t x = q < n ? a[q] : 0u, y = q < n ? b[q] : 0u;
        uint64_t valid = cnt == 64 ? ~0ull : ((1ull << cnt) - 1ull);
        uint64_t G = __ballot(x < y) & valid;
        uint64_t Pm = __ballot(x == y) & valid;
        uint64_t C = lookahead(G, Pm, borrow);
        if (q < n) d[q] = x - y - (uint32_t)((C >> lane()) & 1ull);
        borrow = block_carry_out(G, Pm, C, cnt);
    }
    return borrow;
}

// sign of a - b (n limbs each)
__device__ __forceinline__ int cmp(const uint32_t *a, const uint32_t *b, int n) {
    int best = -1;
    for (int q = lane(); q < n; q += MP_WAVE)
        if (a[q] != b[q]) best = q;
    best = wave_max(best);
    if (best < 0) return 0;
    return a[best] > b[best] ? 1 : -1;
}

// ---------------------------------------------------------------------------
// full product of two P-limb integers: prod[0..2P) = x * y
//   x: LDS, P limbs;  ypad: LDS, P + 128 limbs with y at ypad + 64 and 64 zero
//   limbs on each side;  t0..t3: LDS scratch of 2P limbs each.
// Lane t accumulates the product columns r = t, t+64, ... (96-bit sums of
// x[a] * y[r-a]); the columns are then folded into limbs by carry passes that
// never write a buffer they read.
// ---------------------------------------------------------------------------
__device__ void mul_full(uint32_t *prod, const uint32_t *x, const uint32_t *ypad, int P,
                         uint32_t *t0, uint32_t *t1, uint32_t *t2, uint32_t *t3) {
    const int R = 2 * P;
    const uint32_t *y = ypad + MP_WAVE;
    for (int base = 0; base < R; base += MP_WAVE) {
        int r = base + lane();
        int a0 = max(0, base - P + 1), a1 = min(base + MP_WAVE - 1, P - 1);
        uint64_t acc = 0;
        uint32_t acc_hi = 0;
        for (int a = a0; a <= a1; ++a) {
            uint64_t pr = (uint64_t)x[a] * (uint64_t)y[r - a];
            acc += pr;
            acc_hi += (acc < pr) ? 1u : 0u;
        }
        if (r < R) {
            t0[r] = (uint32_t)acc;
            t1[r] = (uint32_t)(acc >> 32);
            t2[r] = acc_hi;
        }
    }
    wsync();
    // column r holds t0 + t1*2^32 + t2*2^64; v_r = t0_r + t1_{r-1} + t2_{r-2} < 3*2^32
    for (int r = lane(); r < R; r += MP_WAVE) {
        uint64_t v = (uint64_t)t0[r] + (r >= 1 ? t1[r - 1] : 0u) + (r >= 2 ? t2[r - 2] : 0u);
        prod[r] = (uint32_t)v;
        t3[r] = (uint32_t)(v >> 32);
    }
    wsync();
    // w_r = (v_r mod 2^32) + (v_{r-1} >> 32) <= 2^32 + 1; its carry bit goes one limb up
    for (int r = lane(); r < R; r += MP_WAVE) {
        uint64_t w = (uint64_t)prod[r] + (r >= 1 ? t3[r - 1] : 0u);
        prod[r] = (uint32_t)w;
        t0[r] = (uint32_t)(w >> 32);
    }
    wsync();
    for (int r = lane(); r < R; r += MP_WAVE) t1[r] = r >= 1 ? t0[r - 1] : 0u;
    wsync();
    add(prod, prod, t1, R, 0u);
    wsync();
}

// Scratch for the number routines: every buffer is in LDS.
struct Scratch {
    uint32_t *x;     // P
    uint32_t *ypad;  // P + 128
    uint32_t *prod;  // 2P + 2
    uint32_t *t0, *t1, *t2, *t3;  // 2P + 2 each
};

// load a number from global memory into LDS (P limbs); returns its header
__device__ __forceinline__ Hdr load(uint32_t *dst, const uint32_t *src, int64_t e, int32_t s, int P) {
    for (int q = lane(); q < P; q += MP_WAVE) dst[q] = src[q];
    wsync();
    bool z = dst[P - 1] == 0u;
    return z ? zero_hdr() : Hdr{e, s, false};
}

__device__ __forceinline__ void store(uint32_t *dst_limbs, int64_t *dst_e, int32_t *dst_s,
                                      const uint32_t *src, Hdr h, int P) {
    for (int q = lane(); q < P; q += MP_WAVE) dst_limbs[q] = h.zero ? 0u : src[q];
    if (lane() == 0) {
        *dst_e = h.zero ? 0 : h.e;
        *dst_s = h.zero ? 0 : h.s;
    }
}

// out = RZ_p(x * y).  x in sc.x, y in sc.ypad + 64 (pads must be zero).
__device__ Hdr mul(uint32_t *out, Hdr hx, Hdr hy, int P, const Scratch &sc) {
    if (hx.zero || hy.zero) return zero_hdr();
    mul_full(sc.prod, sc.x, sc.ypad, P, sc.t0, sc.t1, sc.t2, sc.t3);
    int top = (int)(sc.prod[2 * P - 1] >> 31);
    shift(out, P, sc.prod, 2 * P, -(32LL * P - 1 + top));
    wsync();
    return Hdr{hx.e + hy.e - 1 + top, hx.s ^ hy.s, false};
}

// Normalise the (n)-limb integer G (value G * 2^(scale)) to P limbs: RZ_p.
__device__ __forceinline__ Hdr normalise(uint32_t *out, const uint32_t *G, int n, int64_t scale,
                                         int32_t sign, int P) {
    int64_t L = bitlen(G, n);
    if (L == 0) return zero_hdr();
    shift(out, P, G, n, 32LL * P - L);
    wsync();
    return Hdr{scale + L, sign, false};
}

// out = RZ_p(x + y) for signed x (LDS, P limbs) and y (LDS, P limbs).
// G, Y2: LDS scratch of P + 2 limbs.  out must differ from x, y, G, Y2.
//
// With X the operand of larger exponent (larger magnitude when the exponents
// are equal and the signs differ) and d = e_X - e_Y:
//  * same signs:      G = m_X + floor(m_Y / 2^d)                (scale e_X - p)
//  * opposite, d<=1:  G = m_X 2^d - m_Y, exact                  (scale e_X - d - p)
//  * opposite, d>=2:  G = 4 m_X - ceil(m_Y / 2^(d-2))            (scale e_X - 2 - p)
// then RZ_p(G * 2^scale).  Truncating a sum never needs the dropped bits of Y;
// for a difference the two guard bits and the ceiling (sticky) give the exact
// truncation because the result keeps at least p+1 bits of G.
__device__ Hdr addsub(uint32_t *out, const uint32_t *xm, Hdr hx, const uint32_t *ym, Hdr hy,
                      uint32_t *G, uint32_t *Y2, int P) {
    if (hy.zero) {
        if (hx.zero) return zero_hdr();
        copy(out, xm, P);
        wsync();
        return hx;
    }
    if (hx.zero) {
        copy(out, ym, P);
        wsync();
        return hy;
    }
    const bool subtract = hx.s != hy.s;
    bool swap = hy.e > hx.e;
    if (subtract && hx.e == hy.e) swap = cmp(ym, xm, P) > 0;
    const uint32_t *X = swap ? ym : xm;
    const uint32_t *Y = swap ? xm : ym;
    const Hdr hX = swap ? hy : hx, hY = swap ? hx : hy;
    const uint64_t d = (uint64_t)hX.e - (uint64_t)hY.e;
    const int n = P + 1;
    int64_t g;
    if (!subtract) {
        g = 0;
        shift(G, n, X, P, 0);
        shift(Y2, n, Y, P, -(int64_t)(d > (uint64_t)(32 * P + 64) ? (uint64_t)(32 * P + 64) : d));
        wsync();
        add(G, G, Y2, n, 0u);
    } else if (d <= 1) {
        g = (int64_t)d;
        shift(G, n, X, P, g);
        shift(Y2, n, Y, P, 0);
        wsync();
        sub(G, G, Y2, n, 0u);
    } else {
        g = 2;
        const uint64_t dm2 = d - 2;
        const int64_t rs = (int64_t)(dm2 > (uint64_t)(32 * P + 64) ? (uint64_t)(32 * P + 64) : dm2);
        shift(G, n, X, P, 2);
        shift(Y2, n, Y, P, -rs);
        bool sticky = low_bits_nonzero(Y, P, rs);
        wsync();
        sub(G, G, Y2, n, sticky ? 1u : 0u);
    }
    wsync();
    return normalise(out, G, n, hX.e - g - 32LL * P, hX.s, P);
}

// out = RZ_p(a / b), b != 0 with its top bit set.
// Knuth's Algorithm D in base 2^32 on U = m_a * 2^(p+1) (2P+1 limbs, plus a
// zero limb on top) and V = m_b (already normalised); the quotient Q has
// p+1 or p+2 bits and is truncated to p bits.
//   U: LDS 2P+2 limbs; LO, HI: LDS P+1 limbs; Q: LDS P+2 limbs.
__device__ Hdr div(uint32_t *out, const uint32_t *am, Hdr ha, const uint32_t *bm, Hdr hb,
                   uint32_t *U, uint32_t *LO, uint32_t *HI, uint32_t *Q, int P) {
    if (ha.zero) return zero_hdr();
    const int m = 2 * P + 1;
    shift(U, m + 1, am, P, 32LL * P + 1);
    fill(Q, P + 2, 0u);
    wsync();
    const uint64_t B = 1ull << 32;
    const uint64_t v1 = bm[P - 1], v2 = bm[P - 2];
    for (int j = m - P; j >= 0; --j) {
        uint64_t num = ((uint64_t)U[j + P] << 32) | U[j + P - 1];
        uint64_t qhat = num / v1;
        uint64_t rhat = num - qhat * v1;
        while (qhat >= B || qhat * v2 > ((rhat << 32) | U[j + P - 2])) {
            qhat--;
            rhat += v1;
            if (rhat >= B) break;
        }
        if (qhat) {
            for (int q = lane(); q < P + 1; q += MP_WAVE) {
                uint64_t pr = q < P ? qhat * (uint64_t)bm[q] : 0ull;
                LO[q] = (uint32_t)pr;
                if (q < P) HI[q + 1] = (uint32_t)(pr >> 32);
            }
            if (lane() == 0) HI[0] = 0u;
            wsync();
            uint32_t b1 = sub(U + j, U + j, LO, P + 1, 0u);
            wsync();
            uint32_t b2 = sub(U + j, U + j, HI, P + 1, 0u);
            wsync();
            if (b1 + b2) {
                qhat--;
                for (int q = lane(); q < P + 1; q += MP_WAVE) LO[q] = q < P ? bm[q] : 0u;
                wsync();
                add(U + j, U + j, LO, P + 1, 0u);
                wsync();
            }
        }
        if (lane() == 0) Q[j] = (uint32_t)qhat;
        wsync();
    }
    return normalise(out, Q, P + 2, ha.e - hb.e - 32LL * P - 1, ha.s ^ hb.s, P);
}

}  // namespace mpw
