// kernels_ball.h -- rigorous error bounds for the elimination (ball
// arithmetic; the rigorous results the paper's future-work section asks for,
// with a radius carried beside every number instead of interval endpoints).
//
// Every number x of the elimination gets a radius r(x) with
// |x - x*| <= r(x), where x* is the value the same sequence of operations
// gives in exact arithmetic on the exact input.  Radii are small floating
// point numbers m 2^e (m a 32-bit integer, 0 or in [2^31, 2^32); e int64),
// every operation on them rounded up, so each bound is rigorous; they are
// integer arithmetic, so the oracle reproduces them bit for bit.
//
// With p = 32P and ulp(y) = 2^(e_y - p) for a nonzero result y (|y| < 2^e_y),
// step k of the elimination (pivot u = a_kk, l_i = RZ(a_ik / u)) gives:
//   D_k = RZ(D_{k-1} u):  r(D_k) = |D_{k-1}| r(u) + |u| r(D_{k-1})
//                                  + r(D_{k-1}) r(u) + ulp(D_k)   (D_1 = a_11)
//   l_i:  r(l_i) = (r(a_ik) + |q| r(u)) / (|u| - r(u)) + ulp(l_i),
//         |q| <= 2^e_l, |u| - r(u) >= 2^(e_u - 2) when r(u) <= 2^(e_u - 2)
//         (else the ball of u may hold 0 and no bound follows: r = infinite)
//   a_ij = RZ(a_ij - RZ(l_i u_kj)):
//         r += |l_i| r(u_kj) + |u_kj| r(l_i) + r(l_i) r(u_kj)
//              + ulp(l_i u_kj) + ulp(new a_ij)
// with |x| <= 2^e_x (0 for an exact zero); the product's and the difference's
// rounding terms are left out where the operation is skipped (a zero factor)
// or exact (a zero result).
#pragma once

#include "kernels_valu.h"

namespace mpk {

// radius m 2^e; m == 0: zero; e == kRadInf: no bound
constexpr int64_t kRadInf = INT64_MAX;
struct Rad {
    uint32_t m;
    int64_t e;
};

__host__ __device__ inline Rad rad_zero() { return Rad{0u, 0}; }
__host__ __device__ inline Rad rad_inf() { return Rad{0xFFFFFFFFu, kRadInf}; }
__host__ __device__ inline bool rad_is_inf(Rad a) { return a.e == kRadInf; }

__host__ __device__ inline int bitlen64(uint64_t v) {
#if defined(__HIP_DEVICE_COMPILE__)
    return v ? 64 - __clzll(v) : 0;
#else
    return v ? 64 - __builtin_clzll(v) : 0;
#endif
}

// v 2^e rounded up to a 32-bit mantissa
__host__ __device__ inline Rad rad_norm(uint64_t v, int64_t e) {
    if (v == 0) return rad_zero();
    const int n = bitlen64(v);
    if (n > 32) {
        const int s = n - 32;
        uint64_t m = v >> s;
        if (v & ((1ull << s) - 1ull)) ++m;
        int64_t ee = e + s;
        if (m >> 32) {
            m >>= 1;  // 2^32 -> 2^31, exact
            ++ee;
        }
        return Rad{(uint32_t)m, ee};
    }
    return Rad{(uint32_t)(v << (32 - n)), e - (32 - n)};
}

__host__ __device__ inline Rad rad_pow2(int64_t k) { return Rad{0x80000000u, k - 31}; }

__host__ __device__ inline Rad rad_add(Rad a, Rad b) {
    if (rad_is_inf(a) || rad_is_inf(b)) return rad_inf();
    if (a.m == 0) return b;
    if (b.m == 0) return a;
    if (a.e < b.e) {
        const Rad t = a;
        a = b;
        b = t;
    }
    const uint64_t d = (uint64_t)(a.e - b.e);
    const uint64_t A = (uint64_t)a.m << 31;
    uint64_t B;
    if (d >= 63) {
        B = 1;  // below one unit of A's scale: one unit bounds it
    } else {
        const uint64_t bb = (uint64_t)b.m << 31;
        B = bb >> d;
        if (bb & ((1ull << d) - 1ull)) ++B;
    }
    return rad_norm(A + B, a.e - 31);
}

__host__ __device__ inline Rad rad_mul(Rad a, Rad b) {
    if (a.m == 0 || b.m == 0) return rad_zero();
    if (rad_is_inf(a) || rad_is_inf(b)) return rad_inf();
    return rad_norm((uint64_t)a.m * (uint64_t)b.m, a.e + b.e);
}

// a 2^k (exact)
__host__ __device__ inline Rad rad_scale(Rad a, int64_t k) {
    if (a.m == 0 || rad_is_inf(a)) return a;
    return Rad{a.m, a.e + k};
}

// r <= 2^k ?  (r < 2^(e + 32))
__host__ __device__ inline bool rad_le_pow2(Rad r, int64_t k) { return r.m == 0 || (!rad_is_inf(r) && r.e + 32 <= k); }

// |x| <= 2^e_x for a nonzero number, 0 for zero
__host__ __device__ inline Rad rad_mag(bool zero, int64_t e) { return zero ? rad_zero() : rad_pow2(e); }

// ulp of a nonzero result (p bits), 0 for an exact zero
__host__ __device__ inline Rad rad_ulp(bool zero, int64_t e, int P) { return zero ? rad_zero() : rad_pow2(e - 32 * (int64_t)P); }

// the radius of one multiplier from the radii of a_ik and u before the division
__host__ __device__ inline Rad rad_multiplier(Rad ra, Rad ru, bool lzero, int64_t el, bool uzero, int64_t eu, int P) {
    if (uzero || !rad_le_pow2(ru, eu - 2)) return rad_inf();
    const Rad num = rad_add(ra, rad_mul(rad_mag(lzero, el), ru));
    return rad_add(rad_scale(num, 2 - eu), rad_ulp(lzero, el, P));
}

// step k (0-based) ran to its end: no stop so far, or a zero pivot found at a
// later step (the previous step's finish examines the next pivot, so info can
// name step k+2 while step k's radii are formed); an overflow (info < 0)
// leaves every radius unbounded (k_ball_end)
__host__ __device__ inline bool ball_step_done(int32_t info, int64_t k) { return info == 0 || info > k + 1; }

struct RadMat {
    uint32_t *m;  // [n][n]
    int64_t *e;
    int64_t ld;
};

__device__ __forceinline__ Rad rad_at(const RadMat &R, int64_t i, int64_t j) {
    return Rad{R.m[i * R.ld + j], R.e[i * R.ld + j]};
}
__device__ __forceinline__ void rad_put(const RadMat &R, int64_t i, int64_t j, Rad r) {
    R.m[i * R.ld + j] = r.m;
    R.e[i * R.ld + j] = r.e;
}
__device__ __forceinline__ bool is_zero_num(const MatDev &A, int64_t i, int64_t j, int P) {
    return el(A, i, j, P)[P - 1] == 0u;
}

// the input's radii: 0 (exact) or one ulp of each entry.  A step at or after
// an elimination that stopped (info != 0) gets no bound.
__global__ void k_ball_init(MatDev A, RadMat R, int64_t n, int P, int ulp) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    const int64_t i = t / n, j = t % n;
    rad_put(R, i, j, ulp ? rad_ulp(is_zero_num(A, i, j, P), ex(A, i, j), P) : rad_zero());
}

// Step k, after its elimination step: the radius of D_k (thread 0) and of
// the multipliers l_i, i > k (one thread each, into LR: column k of R still
// holds the radii before the division, which these threads read, and
// k_ball_update moves LR into it).  The pivot's radius is R_kk.
__global__ void k_ball_mult(MatDev A, MatDev D, RadMat R, uint32_t *LRm, int64_t *LRe, uint32_t *RDm, int64_t *RDe,
                            const int32_t *info, int64_t k, int64_t n, int P) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!ball_step_done(*info, k)) {  // the elimination stopped at or before step k: no bound
        if (t == 0) {
            RDm[k] = 0xFFFFFFFFu;
            RDe[k] = kRadInf;
        }
        return;
    }
    const Rad ru = rad_at(R, k, k);
    const bool uz = is_zero_num(A, k, k, P);
    const int64_t eu = ex(A, k, k);
    if (t == 0) {
        Rad rd;
        if (k == 0) {
            rd = ru;
        } else {
            const Rad rp = Rad{RDm[k - 1], RDe[k - 1]};
            const bool dz = el(D, 0, k - 1, P)[P - 1] == 0u, kz = el(D, 0, k, P)[P - 1] == 0u;
            rd = rad_add(rad_add(rad_mul(rad_mag(dz, ex(D, 0, k - 1)), ru), rad_mul(rad_mag(uz, eu), rp)),
                         rad_add(rad_mul(rp, ru), rad_ulp(kz, ex(D, 0, k), P)));
        }
        RDm[k] = rd.m;
        RDe[k] = rd.e;
    }
    const int64_t i = k + 1 + t;
    if (i >= n) return;
    const Rad rl = rad_multiplier(rad_at(R, i, k), ru, is_zero_num(A, i, k, P), ex(A, i, k), uz, eu, P);
    LRm[i] = rl.m;
    LRe[i] = rl.e;
}

// the trailing block's radii after step k (thread per element), then column k
// takes the multipliers' radii
__global__ void k_ball_update(MatDev A, RadMat R, const uint32_t *LRm, const int64_t *LRe, const int32_t *info,
                              int64_t k, int64_t n, int P) {
    if (!ball_step_done(*info, k)) return;
    const int64_t m = n - k - 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * (m + 1)) return;
    const int64_t i = k + 1 + t / (m + 1), c = t % (m + 1);
    const Rad rl = Rad{LRm[i], LRe[i]};
    if (c == m) {  // the multiplier itself
        rad_put(R, i, k, rl);
        return;
    }
    const int64_t j = k + 1 + c;
    const bool lz = is_zero_num(A, i, k, P), uz = is_zero_num(A, k, j, P);
    const int64_t el_ = ex(A, i, k), eu = ex(A, k, j);
    const Rad ru = rad_at(R, k, j);
    Rad r = rad_at(R, i, j);
    r = rad_add(r, rad_mul(rad_mag(lz, el_), ru));
    r = rad_add(r, rad_mul(rad_mag(uz, eu), rl));
    r = rad_add(r, rad_mul(rl, ru));
    if (!lz && !uz) {  // the product and the difference were formed, each rounded
        r = rad_add(r, rad_pow2(el_ + eu - 32 * (int64_t)P));
        r = rad_add(r, rad_ulp(is_zero_num(A, i, j, P), ex(A, i, j), P));
    }
    rad_put(R, i, j, r);
}

// after the elimination: an exponent overflow (info = -1) leaves no bound
__global__ void k_ball_end(const int32_t *info, uint32_t *RDm, int64_t *RDe, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && *info < 0) {
        RDm[t] = 0xFFFFFFFFu;
        RDe[t] = kRadInf;
    }
}

}  // namespace mpk
