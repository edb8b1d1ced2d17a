// kernels_valu.h -- elimination, leading determinants, minors and output
// conversion with wave-cooperative 32x32->64-bit VALU limb arithmetic.
//
// Every kernel runs single-wave (64-thread) workgroups; one workgroup owns one
// multiprecision operation and keeps its operands in LDS (layout `Lds`).
#pragma once

#include "wave_mp.h"

namespace mpk {

struct MatDev {
    uint32_t *limbs;  // [rows][ld][P]
    int64_t *exp;     // [rows][ld]
    int32_t *sign;    // [rows][ld]
    int64_t ld;
};

__device__ __forceinline__ uint32_t *el(const MatDev &A, int64_t i, int64_t j, int P) {
    return A.limbs + (i * A.ld + j) * (int64_t)P;
}
__device__ __forceinline__ int64_t &ex(const MatDev &A, int64_t i, int64_t j) { return A.exp[i * A.ld + j]; }
__device__ __forceinline__ int32_t &sg(const MatDev &A, int64_t i, int64_t j) { return A.sign[i * A.ld + j]; }

constexpr int64_t kExpLimit = 1LL << 62;

// LDS carve-up shared by all VALU kernels (12P + 2*MP_YPAD + 10 limbs).
struct Lds {
    mpw::Scratch sc;  // x, ypad, prod, t0..t3
    __device__ Lds(uint32_t *base, int P) {
        sc.x = base;
        sc.ypad = sc.x + P;
        sc.prod = sc.ypad + P + 2 * MP_YPAD;
        sc.t0 = sc.prod + 2 * P + 2;
        sc.t1 = sc.t0 + 2 * P + 2;
        sc.t2 = sc.t1 + 2 * P + 2;
        sc.t3 = sc.t2 + 2 * P + 2;
    }
};

__host__ __device__ constexpr size_t lds_bytes(int P) { return (size_t)(12 * P + 2 * MP_YPAD + 10) * 4u; }

// y operand of a product: value at ypad + MP_YPAD, zero limbs around it
__device__ __forceinline__ mpw::Hdr load_y(uint32_t *ypad, const uint32_t *src, int64_t e, int32_t s,
                                           int P) {
    for (int q = mpw::lane(); q < MP_YPAD; q += MP_WAVE) {
        ypad[q] = 0u;
        ypad[MP_YPAD + P + q] = 0u;
    }
    mpw::gload(ypad + MP_YPAD, src, P);
    mpw::wsync();
    const bool z = __builtin_amdgcn_readfirstlane(ypad[MP_YPAD + P - 1]) == 0u;
    return z ? mpw::zero_hdr() : mpw::Hdr{e, s, false};
}

__device__ void store_zero(uint32_t *l, int64_t *e, int32_t *s, int P) {
    for (int q = mpw::lane(); q < P; q += MP_WAVE) l[q] = 0u;
    if (mpw::lane() == 0) {
        *e = 0;
        *s = 0;
    }
}

// ---------------------------------------------------------------------------
// Step k, part 1 (Algorithm 1 steps 2.1 and 2.2.1), with one shared reciprocal.
// k_pivot_recip: block 0 = D_k = RZ_p(D_{k-1} a_kk) (D_1 = a_11) and the zero /
// overflow checks that set info; block 1 = R = floor(2^(2p) / m_pivot) into rw[0..P], with
// rw[P+1] = 1 when the reciprocal is exact (0: callers use long division).
// k_divide: block b -> l_ik = RZ_p(a_ik / a_kk) for i = k+1+b.
// ---------------------------------------------------------------------------
__host__ __device__ inline size_t pivot_lds_bytes(int P) {
    size_t a = lds_bytes(P), b = mpw::div_lds_limbs(P) * 4u;
    return a > b ? a : b;
}

// LDS of k_divide (and k_divide_from): the lean layout from 16 limbs on
__host__ __device__ inline size_t divide_lds_bytes(int P) {
    return P >= 16 ? mpw::div_lean_words(P) * 4u : pivot_lds_bytes(P);
}

// Waves of k_pivot_recip, k_divide and k_minors_sweep (a team, see
// wave_mp.h): one per round
// of 64 windows of a P x P product, at most 4 (one below 224 limbs or so).
__host__ __device__ inline int team_waves(int P) {
    const int cols = (64 * P + 27) / 28, windows = (cols + 7) / 8, rounds = (windows + 63) / 64;
    return rounds < 1 ? 1 : (rounds > 4 ? 4 : rounds);
}

// a wave-uniform copy of a value every lane read from the same address
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// info_out receives the zero-pivot / overflow code (info itself, or a pending
// word when this runs inside the previous step's launch, see finish_body)
// tm: the team forming the products with this wave (nullptr: it alone)
__device__ __forceinline__ void pivot_recip_body(uint32_t *lds_raw, MatDev A, MatDev D, const int32_t *info,
                                                 int32_t *info_out, uint32_t *rw, int64_t k, int64_t n, int P,
                                                 int role, mpw::TeamCtl *tm = nullptr) {
    if (uni((uint32_t)*info) != 0u) return;
    const uint32_t *pm = el(A, k, k, P);
    const bool piv_zero = uni(pm[P - 1]) == 0u;
    const int64_t pe = ex(A, k, k);
    const int32_t ps = sg(A, k, k);
    if (role == 0) {
        Lds L(lds_raw, P);
        L.sc.team = tm;
        bool bad = false;
        int32_t code = 0;
        mpw::Hdr hd{0, 0, true};
        if (piv_zero) {
            bad = true;
            code = (int32_t)(k + 1);
        } else {
            mpw::Hdr hp = load_y(L.sc.ypad, pm, pe, ps, P);
            if (k == 0) {
                mpw::copy(L.sc.t3, L.sc.ypad + MP_YPAD, P);
                mpw::wsync();
                hd = hp;
            } else {
                mpw::Hdr hprev = mpw::load(L.sc.x, el(D, 0, k - 1, P), ex(D, 0, k - 1), sg(D, 0, k - 1), P);
                hd = mpw::mul(L.sc.t3, hprev, hp, P, L.sc);
            }
            if (pe > kExpLimit || pe < -kExpLimit || (!hd.zero && (hd.e > kExpLimit || hd.e < -kExpLimit))) {
                bad = true;
                code = -1;
            }
        }
        if (bad) {
            if (mpw::lane() == 0) *info_out = code;
            for (int64_t t = k; t < n; ++t) store_zero(el(D, 0, t, P), &ex(D, 0, t), &sg(D, 0, t), P);
        } else {
            mpw::store(el(D, 0, k, P), &ex(D, 0, k), &sg(D, 0, k), L.sc.t3, hd, P);
        }
        return;
    }
    if (piv_zero || n - k - 1 <= 0) return;
    mpw::DivBufs B = mpw::div_bufs(lds_raw, P);
    B.team = tm;
    mpw::gload(B.v, pm, P);
    mpw::wsync();
    const bool ok = mpw::recip(B, P);
    for (int q = mpw::lane(); q < P + 1; q += MP_WAVE) rw[q] = B.x[q];
    if (mpw::lane() == 0) rw[P + 1] = ok ? 1u : 0u;
}

// rw[P + 2] is the pending code of step k's pivot when that pivot was
// examined inside the previous step's launch: a nonzero code stops the step,
// and block 0 moves it into info for the launches that follow.  long_div:
// every row by long division (the reciprocal's fallback; same bits).
__device__ __forceinline__ void divide_body(uint32_t *lds_raw, MatDev A, const uint32_t *rw, int32_t *info, int64_t k,
                                            int64_t n, int P, int64_t blk, mpw::TeamCtl *tm = nullptr,
                                            bool long_div = false) {
    const int32_t pend = (int32_t)uni(rw[P + 2]);
    if (uni((uint32_t)*info) != 0u || pend != 0) {
        if (blk == 0 && mpw::lane() == 0 && *info == 0) *info = pend;
        return;
    }
    const uint32_t *pm = el(A, k, k, P);
    if (uni(pm[P - 1]) == 0u) return;
    const int64_t i = k + 1 + blk;
    uint32_t *am = el(A, i, k, P);
    if (P >= 16) {  // the lean layout (divide_lds_bytes)
        mpw::DivLean L = mpw::div_lean(lds_raw, P);
        L.team = tm;
        mpw::Hdr ha = mpw::load(L.a, am, ex(A, i, k), sg(A, i, k), P);
        mpw::Hdr hp = mpw::load(L.v, pm, ex(A, k, k), sg(A, k, k), P);
        mpw::Hdr hq;
        bool done = false;
        if (!long_div && uni(rw[P + 1]) != 0u) done = mpw::div_by_recip_lean(hq, ha, hp, rw, L, P);
        // long division: U = prod (2P+2), Q = the scratch's first P + 2 words
        if (!done) hq = mpw::div(L.out, L.a, ha, L.v, hp, L.prod, L.ws, L.ws, L.ws, P);
        mpw::store(am, &ex(A, i, k), &sg(A, i, k), L.out, hq, P);
        return;
    }
    mpw::DivBufs B = mpw::div_bufs(lds_raw, P);
    B.team = tm;
    mpw::Hdr ha = mpw::load(B.a, am, ex(A, i, k), sg(A, i, k), P);
    mpw::Hdr hp = mpw::load(B.v, pm, ex(A, k, k), sg(A, k, k), P);
    mpw::Hdr hq;
    bool done = false;
    if (!long_div && uni(rw[P + 1]) != 0u) done = mpw::div_by_recip(B.t3, hq, ha, hp, rw, B, P);
    if (!done) {
        // long division: U = prod (2P+2), LO = t0, HI = t1, Q = t2, out = t3
        hq = mpw::div(B.t3, B.a, ha, B.v, hp, B.prod, B.t0, B.t1, B.t2, P);
    }
    mpw::store(am, &ex(A, i, k), &sg(A, i, k), B.t3, hq, P);
}

// ---------------------------------------------------------------------------
// Step k, part 2 (Algorithm 1 step 2.2.2): a_ij = RZ_p(a_ij - RZ_p(l_ik u_kj))
// for k < i, j < n; block (bx) -> i = k+1 + bx / m, j = k+1 + bx % m.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void update_valu_body(uint32_t *lds_raw, MatDev A, const int32_t *info, int64_t k, int64_t n, int P,
                                 int64_t bx) {
    if (*info != 0) return;
    const int64_t m = n - k - 1;
    if (bx >= m * m) return;
    const int64_t i = k + 1 + bx / m, j = k + 1 + bx % m;
    const uint32_t *lm = el(A, i, k, P);
    const uint32_t *um = el(A, k, j, P);
    if (lm[P - 1] == 0u || um[P - 1] == 0u) return;  // a_ij - 0 = a_ij
    Lds L(lds_raw, P);
    mpw::Hdr hl = mpw::load(L.sc.x, lm, ex(A, i, k), sg(A, i, k), P);
    mpw::Hdr hu = load_y(L.sc.ypad, um, ex(A, k, j), sg(A, k, j), P);
    mpw::Hdr ht = mpw::mul(L.sc.t3, hl, hu, P, L.sc);
    ht.s ^= 1;  // subtract
    uint32_t *am = el(A, i, j, P);
    mpw::Hdr ha = mpw::load(L.sc.x, am, ex(A, i, j), sg(A, i, j), P);
    mpw::Hdr hr = mpw::addsub(L.sc.t2, L.sc.x, ha, L.sc.t3, ht, L.sc.t0, L.sc.t1, P);
    mpw::store(am, &ex(A, i, j), &sg(A, i, j), L.sc.t2, hr, P);
}

// The factors are complete when elimination ran all its steps: info == 0, or
// info == n (only the last pivot, u_nn, is zero -- det = D_n = 0, but the
// minors and the adjugate never divide by u_nn and stay defined; eq. (minors)
// needs them exactly where det vanishes).
__host__ __device__ __forceinline__ bool factors_complete(int32_t info, int64_t n) {
    return info == 0 || (int64_t)info == n;
}

// ---------------------------------------------------------------------------
// Last-column minors (Sec. 3, [A I] derivation): x^T L = e_n^T by sweeps.
// ---------------------------------------------------------------------------
__global__ void k_minors_init(MatDev c, int64_t n, int P) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = n * (int64_t)P;
    if (t < total) c.limbs[(t / P) * (int64_t)P + t % P] = 0u;  // vector: ld irrelevant for row 0
    if (t < n) {
        c.exp[t] = 0;
        c.sign[t] = 0;
    }
}

// sweep j: s_i = RZ_p(s_i - RZ_p(x_j l_ji)), i < j; x_{n-1} = 1, x_j = s_j otherwise
// (nothing unless the factors are complete; k_minors_init wrote zeros)
// (tm: the team forming the product with this wave; nullptr: it alone)
__device__ __forceinline__ void minors_sweep_body(uint32_t *lds_raw, MatDev LU, MatDev c, const int32_t *info, int64_t j,
                                  int64_t n, int P, int64_t i, mpw::TeamCtl *tm = nullptr) {
    if (!factors_complete((int32_t)uni((uint32_t)*info), n)) return;
    Lds L(lds_raw, P);
    L.sc.team = tm;
    const uint32_t *lm = el(LU, j, i, P);
    if (uni(lm[P - 1]) == 0u) return;
    mpw::Hdr ht;
    if (j == n - 1) {
        ht = mpw::load(L.sc.t3, lm, ex(LU, j, i), sg(LU, j, i), P);  // 1 * l_ji, exact
    } else {
        mpw::Hdr hx = mpw::load(L.sc.x, el(c, 0, j, P), ex(c, 0, j), sg(c, 0, j), P);
        if (hx.zero) return;
        mpw::Hdr hl = load_y(L.sc.ypad, lm, ex(LU, j, i), sg(LU, j, i), P);
        ht = mpw::mul(L.sc.t3, hx, hl, P, L.sc);
    }
    ht.s ^= 1;
    uint32_t *sm = el(c, 0, i, P);
    mpw::Hdr hs = mpw::load(L.sc.x, sm, ex(c, 0, i), sg(c, 0, i), P);
    mpw::Hdr hr = mpw::addsub(L.sc.t2, L.sc.x, hs, L.sc.t3, ht, L.sc.t0, L.sc.t1, P);
    mpw::store(sm, &ex(c, 0, i), &sg(c, 0, i), L.sc.t2, hr, P);
}

// c_i = RZ_p(D_{n-1} x_i) for i < n-1 (block i), c_{n-1} = D_{n-1}; n == 1: c = 1
__device__ __forceinline__ void minors_final_body(uint32_t *lds_raw, MatDev D, MatDev c, const int32_t *info, int64_t n, int P,
                                  int64_t i) {
    if (!factors_complete(*info, n)) return;
    uint32_t *cm = el(c, 0, i, P);
    if (n == 1) {
        for (int q = mpw::lane(); q < P; q += MP_WAVE) cm[q] = (q == P - 1) ? 0x80000000u : 0u;
        if (mpw::lane() == 0) {
            ex(c, 0, 0) = 1;
            sg(c, 0, 0) = 0;
        }
        return;
    }
    const uint32_t *dm = el(D, 0, n - 2, P);
    if (i == n - 1) {
        for (int q = mpw::lane(); q < P; q += MP_WAVE) cm[q] = dm[q];
        if (mpw::lane() == 0) {
            ex(c, 0, i) = ex(D, 0, n - 2);
            sg(c, 0, i) = sg(D, 0, n - 2);
        }
        return;
    }
    Lds L(lds_raw, P);
    mpw::Hdr hd = mpw::load(L.sc.x, dm, ex(D, 0, n - 2), sg(D, 0, n - 2), P);
    mpw::Hdr hx = load_y(L.sc.ypad, cm, ex(c, 0, i), sg(c, 0, i), P);
    mpw::Hdr hr = mpw::mul(L.sc.t3, hd, hx, P, L.sc);
    mpw::store(cm, &ex(c, 0, i), &sg(c, 0, i), L.sc.t3, hr, P);
}

// ---------------------------------------------------------------------------
// single-matrix launches (one block per unit of work)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t flat_block() {
    return (int64_t)blockIdx.x + (int64_t)blockIdx.y * (int64_t)gridDim.x;
}

// A wave that runs out of a team wait (never in a correct run: the bound is
// the handle's wait limit, 10 s by default) stops the factorisation with
// info = -2 instead of hanging the launch.
__device__ __forceinline__ void team_report(mpw::TeamCtl *tm, int32_t *info) {
    if (!mpw::team_close(tm) && mpw::lane() == 0) atomicCAS(info, 0, -2);
}

// blockDim.x = 64 team_waves(P) (or 64: one wave)
__global__ void __launch_bounds__(256) k_pivot_recip(MatDev A, MatDev D, int32_t *info, uint32_t *rw, int64_t k,
                                                     int64_t n, int P, uint64_t wait_ticks) {
    extern __shared__ uint32_t lds_raw[];
    __shared__ mpw::TeamCtl ctl;
    mpw::team_open(&ctl, wait_ticks);
    if (mpw::team_wave() != 0) {
        mpw::team_serve(&ctl);
        return;
    }
    pivot_recip_body(lds_raw, A, D, info, info, rw, k, n, P, (int)blockIdx.x, &ctl);
    team_report(&ctl, info);
}

// clear the pending pivot code (rw[P + 2]) before a factorisation, and move a
// code still pending after the last step into info
__global__ void k_pend_clear(uint32_t *rw, int P) {
    if (threadIdx.x == 0 && blockIdx.x == 0) rw[P + 2] = 0u;
}
__global__ void k_pend_promote(int32_t *info, const uint32_t *rw, int P) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && *info == 0) *info = (int32_t)rw[P + 2];
}

// blockDim.x = 64 team_waves(P) (or 64: one wave)
__global__ void __launch_bounds__(256) k_divide(MatDev A, const uint32_t *rw, int32_t *info, int64_t k,
                                                int64_t n, int P, uint64_t wait_ticks, int long_div) {
    extern __shared__ uint32_t lds_raw[];
    __shared__ mpw::TeamCtl ctl;
    mpw::team_open(&ctl, wait_ticks);
    if (mpw::team_wave() != 0) {
        mpw::team_serve(&ctl);
        return;
    }
    divide_body(lds_raw, A, rw, info, k, n, P, flat_block(), &ctl, long_div != 0);
    team_report(&ctl, info);
}

// multipliers of rows row0 .. n-1 only (growing a factorisation: the rows
// added after the leading block was factored); blockDim.x as for k_divide
__global__ void __launch_bounds__(256) k_divide_from(MatDev A, const uint32_t *rw, int32_t *info, int64_t k,
                                                     int64_t n, int P, int64_t row0, uint64_t wait_ticks,
                                                     int long_div) {
    extern __shared__ uint32_t lds_raw[];
    __shared__ mpw::TeamCtl ctl;
    mpw::team_open(&ctl, wait_ticks);
    if (mpw::team_wave() != 0) {
        mpw::team_serve(&ctl);
        return;
    }
    divide_body(lds_raw, A, rw, info, k, n, P, row0 - k - 1 + (int64_t)blockIdx.x, &ctl, long_div != 0);
    team_report(&ctl, info);
}

__global__ void __launch_bounds__(64) k_update_valu(MatDev A, const int32_t *info, int64_t k, int64_t n, int P) {
    extern __shared__ uint32_t lds_raw[];
    update_valu_body(lds_raw, A, info, k, n, P, flat_block());
}

// blockDim.x = 64 team_waves(P) (or 64: one wave)
__global__ void __launch_bounds__(256) k_minors_sweep(MatDev LU, MatDev c, int32_t *info, int64_t j, int64_t n,
                                                      int P, uint64_t wait_ticks) {
    extern __shared__ uint32_t lds_raw[];
    __shared__ mpw::TeamCtl ctl;
    mpw::team_open(&ctl, wait_ticks);
    if (mpw::team_wave() != 0) {
        mpw::team_serve(&ctl);
        return;
    }
    minors_sweep_body(lds_raw, LU, c, info, j, n, P, flat_block(), &ctl);
    team_report(&ctl, info);
}

__global__ void __launch_bounds__(64) k_minors_final(MatDev D, MatDev c, const int32_t *info, int64_t n, int P) {
    extern __shared__ uint32_t lds_raw[];
    minors_final_body(lds_raw, D, c, info, n, P, flat_block());
}

// ---------------------------------------------------------------------------
// Output conversion: (-1)^s RZ_53(m / 2^p) and the exponent.
// ---------------------------------------------------------------------------
__global__ void k_to_f64(MatDev x, int64_t rows, int64_t cols, int P, double *mant, int64_t *eo) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * cols) return;
    int64_t i = t / cols, j = t % cols;
    const uint32_t *m = el(x, i, j, P);
    uint32_t top = m[P - 1];
    if (top == 0u) {
        mant[t] = 0.0;
        eo[t] = 0;
        return;
    }
    // top 53 bits: 32 from limb P-1, 21 from limb P-2
    uint64_t v = ((uint64_t)top << 21) | (uint64_t)(m[P - 2] >> 11);
    double d = ldexp((double)v, -53);
    mant[t] = sg(x, i, j) ? -d : d;
    eo[t] = ex(x, i, j);
}

// val = RZ_53 mantissa * 2^(exp - *shift), one IEEE rounding (ldexp: nearest
// even) where the result lands in float64's subnormal range; the exponent
// difference is clamped to +-2200, beyond which the result is 0 or inf anyway.
__global__ void k_to_f64_scaled(MatDev x, int64_t rows, int64_t cols, int P, const int64_t *shift, double *val) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * cols) return;
    int64_t i = t / cols, j = t % cols;
    const uint32_t *m = el(x, i, j, P);
    uint32_t top = m[P - 1];
    if (top == 0u) {
        val[t] = 0.0;
        return;
    }
    uint64_t v = ((uint64_t)top << 21) | (uint64_t)(m[P - 2] >> 11);
    int64_t s = ex(x, i, j) - *shift;
    s = s < -2200 ? -2200 : (s > 2200 ? 2200 : s);
    // v 2^(s-53) in two exact-or-once-rounded steps: v 2^-53 is exact
    double d = ldexp(ldexp((double)v, -53), (int)s);
    val[t] = sg(x, i, j) ? -d : d;
}

// RZ to 32 P2 bits of a rows x cols block (P2 <= P): a nonzero mantissa has
// its top bit set, so that is its top P2 limbs, same exponent and sign.  One
// thread per output limb.
__global__ void k_truncate(MatDev X, MatDev Y, int64_t rows, int64_t cols, int P, int P2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + (int64_t)blockIdx.y * gridDim.x * blockDim.x;
    const int64_t total = rows * cols * (int64_t)P2;
    if (t >= total) return;
    const int64_t e = t / P2, q = t % P2, i = e / cols, j = e % cols;
    el(Y, i, j, P2)[q] = el(X, i, j, P)[P - P2 + q];
    if (q == 0) {
        ex(Y, i, j) = ex(X, i, j);
        sg(Y, i, j) = sg(X, i, j);
    }
}

__global__ void k_set_info(int32_t *info, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *info = v;
}

}  // namespace mpk
