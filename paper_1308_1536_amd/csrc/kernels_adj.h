// kernels_adj.h -- adj(A)^T = d det / d A from the stored factors (the
// backward of the determinant; Sec. 3: by Baur-Strassen every (N-1)x(N-1)
// minor is a partial derivative of det, d det / d a_ij = C_ij).
//
// With A = L U (L unit lower, holding the multipliers), adj(A) = adj(U) W,
// W = L^-1, in this fixed order (the oracle follows the same one):
//   W:      row r solves x^T L = e_r^T; sweeps j = n-1..1 (all rows r >= j in
//           one launch): W_ri <- RZ(W_ri - RZ(W_rj l_ji)), i < j;
//   adj(U): S_n = 1, S_i = RZ(u_ii S_{i+1}); adj(U)_ii = RZ(D_{i-1} S_{i+1});
//           strictly upper part by right-looking back substitution of
//           U x = det(U) e_j: for k = n-1..1, t_i <- RZ(t_i - RZ(u_ik x_k))
//           (i < k, all columns j >= k in one launch), then
//           x_{k-1} = RZ(t_{k-1} / u_{k-1,k-1});
//   adj(A): for k = 0..n-1, acc_im <- RZ(acc_im + RZ(adj(U)_ik W_km)) for
//           i, m <= k (each entry sums its terms in ascending k).
// The kernels here take one wave per number operation (wave-cooperative
// limbs).  Where the lane product applies (P <= 128, P a multiple of 4) the
// host runs the three O(n^3) phases -- the W sweeps, the back substitution's
// updates and the accumulation -- as rank-1 updates on the lane product and
// the tile finish instead (k_prod_lane_r1, k_finish_r1): the same operation
// on every element, in the same order, so the same bits.
// Row n-1 of adj(A) is RZ(D_{n-2} W_{n-1,m}), the last-column minors.
#pragma once

#include "kernels_mfma.h"

namespace mpk {

// zero a matrix block of n x n numbers; diag_one puts 1 on the diagonal
__global__ void k_adj_init(MatDev X, int64_t n, int P, int diag_one) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = n * n;
    if (t >= total) return;
    const int64_t i = t / n, j = t % n;
    uint32_t *m = el(X, i, j, P);
    const bool one = diag_one && i == j;
    for (int q = 0; q < P; ++q) m[q] = (one && q == P - 1) ? 0x80000000u : 0u;
    ex(X, i, j) = one ? 1 : 0;
    sg(X, i, j) = 0;
}

// c = RZ(c + s * RZ(x * y)), s = -1 (subtract) or +1, all through LDS
__device__ __forceinline__ void fma_like(uint32_t *cm, int64_t *ce, int32_t *cs, const uint32_t *xm,
                                         int64_t xe, int32_t xs, const uint32_t *ym, int64_t ye, int32_t ys,
                                         bool subtract, Lds &L, int P) {
    mpw::Hdr hx = mpw::load(L.sc.x, xm, xe, xs, P);
    mpw::Hdr hy = load_y(L.sc.ypad, ym, ye, ys, P);
    if (hx.zero || hy.zero) return;  // c +- 0 = c
    mpw::Hdr ht = mpw::mul(L.sc.t3, hx, hy, P, L.sc);
    if (subtract) ht.s ^= 1;
    mpw::Hdr hc = mpw::load(L.sc.x, cm, *ce, *cs, P);
    mpw::Hdr hr = mpw::addsub(L.sc.t2, L.sc.x, hc, L.sc.t3, ht, L.sc.t0, L.sc.t1, P);
    mpw::store(cm, ce, cs, L.sc.t2, hr, P);
}

// W sweep j: unit b -> (r, i) = (j + b / j, b % j)
__device__ __forceinline__ void adj_w_body(uint32_t *lds_raw, MatDev LU, MatDev W, const int32_t *info, int64_t j,
                                           int64_t n, int P, int64_t b) {
    if (*info != 0) return;
    if (b >= (n - j) * j) return;
    const int64_t r = j + b / j, i = b % j;
    Lds L(lds_raw, P);
    fma_like(el(W, r, i, P), &ex(W, r, i), &sg(W, r, i), el(W, r, j, P), ex(W, r, j), sg(W, r, j),
             el(LU, j, i, P), ex(LU, j, i), sg(LU, j, i), true, L, P);
}
__global__ void __launch_bounds__(64) k_adj_w(MatDev LU, MatDev W, const int32_t *info, int64_t j, int64_t n,
                                              int P) {
    extern __shared__ uint32_t lds_raw[];
    adj_w_body(lds_raw, LU, W, info, j, n, P, (int64_t)blockIdx.x + (int64_t)blockIdx.y * (int64_t)gridDim.x);
}

// S_n = 1, S_i = RZ(u_ii S_{i+1}) (one wave, sequential), then the diagonal
// of adj(U) is written by k_adj_diag
__device__ __forceinline__ void adj_s_body(uint32_t *lds_raw, MatDev LU, MatDev S, const int32_t *info, int64_t n,
                                           int P) {
    if (*info != 0) return;
    Lds L(lds_raw, P);
    // the running product stays in LDS as the y operand (S_n = 1)
    for (int q = mpw::lane(); q < P + 2 * MP_YPAD; q += MP_WAVE)
        L.sc.ypad[q] = (q == MP_YPAD + P - 1) ? 0x80000000u : 0u;
    for (int q = mpw::lane(); q < P; q += MP_WAVE) el(S, 0, n, P)[q] = (q == P - 1) ? 0x80000000u : 0u;
    if (mpw::lane() == 0) {
        ex(S, 0, n) = 1;
        sg(S, 0, n) = 0;
    }
    mpw::wsync();
    mpw::Hdr hs{1, 0, false};
    for (int64_t i = n - 1; i >= 0; --i) {
        mpw::Hdr hu = mpw::load(L.sc.x, el(LU, i, i, P), ex(LU, i, i), sg(LU, i, i), P);
        mpw::Hdr hr = mpw::mul(L.sc.t3, hu, hs, P, L.sc);
        mpw::store(el(S, 0, i, P), &ex(S, 0, i), &sg(S, 0, i), L.sc.t3, hr, P);
        mpw::copy(L.sc.ypad + MP_YPAD, L.sc.t3, P);
        mpw::wsync();
        hs = hr;
    }
}
__global__ void __launch_bounds__(64) k_adj_s(MatDev LU, MatDev S, const int32_t *info, int64_t n, int P) {
    extern __shared__ uint32_t lds_raw[];
    adj_s_body(lds_raw, LU, S, info, n, P);
}

// adj(U)_ii = RZ(D_{i-1} S_{i+1}), D_0 = 1 (so adj(U)_00 = S_1)
__device__ __forceinline__ void adj_diag_body(uint32_t *lds_raw, MatDev D, MatDev S, MatDev J, const int32_t *info,
                                              int P, int64_t i) {
    if (*info != 0) return;
    Lds L(lds_raw, P);
    mpw::Hdr hs = mpw::load(L.sc.t3, el(S, 0, i + 1, P), ex(S, 0, i + 1), sg(S, 0, i + 1), P);
    mpw::Hdr hr = hs;
    if (i > 0) {
        mpw::Hdr hd = mpw::load(L.sc.x, el(D, 0, i - 1, P), ex(D, 0, i - 1), sg(D, 0, i - 1), P);
        mpw::Hdr hs2 = load_y(L.sc.ypad, el(S, 0, i + 1, P), ex(S, 0, i + 1), sg(S, 0, i + 1), P);
        hr = mpw::mul(L.sc.t3, hd, hs2, P, L.sc);
    }
    mpw::store(el(J, i, i, P), &ex(J, i, i), &sg(J, i, i), L.sc.t3, hr, P);
}
__global__ void __launch_bounds__(64) k_adj_diag(MatDev D, MatDev S, MatDev J, const int32_t *info, int64_t n,
                                                 int P) {
    extern __shared__ uint32_t lds_raw[];
    (void)n;
    adj_diag_body(lds_raw, D, S, J, info, P, blockIdx.x);
}

// reciprocals of the pivots u_ii (block i), as k_pivot_recip's block 1
__device__ __forceinline__ void adj_recip_body(uint32_t *lds_raw, MatDev LU, uint32_t *rw, const int32_t *info,
                                               int P, int64_t i) {
    if (*info != 0) return;
    uint32_t *r = rw + i * (int64_t)(P + 2);
    if (el(LU, i, i, P)[P - 1] == 0u) {  // u_nn = 0 (info == n): never a divisor
        if (mpw::lane() == 0) r[P + 1] = 0u;
        return;
    }
    mpw::DivBufs B = mpw::div_bufs(lds_raw, P);
    mpw::gload(B.v, el(LU, i, i, P), P);
    mpw::wsync();
    const bool ok = mpw::recip(B, P);
    for (int q = mpw::lane(); q < P + 1; q += MP_WAVE) r[q] = B.x[q];
    if (mpw::lane() == 0) r[P + 1] = ok ? 1u : 0u;
}
__global__ void __launch_bounds__(64) k_adj_recips(MatDev LU, uint32_t *rw, const int32_t *info, int64_t n,
                                                   int P) {
    extern __shared__ uint32_t lds_raw[];
    (void)n;
    adj_recip_body(lds_raw, LU, rw, info, P, blockIdx.x);
}

// back substitution step k, part 1: block b -> (i, j) = (b % k, k + b / k):
// J_ij <- RZ(J_ij - RZ(u_ik J_kj))
__device__ __forceinline__ void adj_u_upd_body(uint32_t *lds_raw, MatDev LU, MatDev J, const int32_t *info, int64_t k,
                                               int64_t n, int P, int64_t b) {
    if (*info != 0) return;
    if (b >= k * (n - k)) return;
    const int64_t i = b % k, j = k + b / k;
    Lds L(lds_raw, P);
    fma_like(el(J, i, j, P), &ex(J, i, j), &sg(J, i, j), el(LU, i, k, P), ex(LU, i, k), sg(LU, i, k),
             el(J, k, j, P), ex(J, k, j), sg(J, k, j), true, L, P);
}
__global__ void __launch_bounds__(64) k_adj_u_upd(MatDev LU, MatDev J, const int32_t *info, int64_t k, int64_t n,
                                                  int P) {
    extern __shared__ uint32_t lds_raw[];
    adj_u_upd_body(lds_raw, LU, J, info, k, n, P, (int64_t)blockIdx.x + (int64_t)blockIdx.y * (int64_t)gridDim.x);
}

// part 2: unit b -> j = k + b: J_{k-1,j} <- RZ(J_{k-1,j} / u_{k-1,k-1})
__device__ __forceinline__ void adj_u_div_body(uint32_t *lds_raw, MatDev LU, MatDev J, const uint32_t *rw,
                                               const int32_t *info, int64_t k, int P, int64_t b) {
    if (*info != 0) return;
    const int64_t j = k + b;
    const int64_t i = k - 1;
    mpw::DivBufs B = mpw::div_bufs(lds_raw, P);
    uint32_t *tm = el(J, i, j, P);
    mpw::Hdr ht = mpw::load(B.a, tm, ex(J, i, j), sg(J, i, j), P);
    mpw::Hdr hu = mpw::load(B.v, el(LU, i, i, P), ex(LU, i, i), sg(LU, i, i), P);
    const uint32_t *R = rw + i * (int64_t)(P + 2);
    mpw::Hdr hq;
    bool done = false;
    if (R[P + 1] != 0u) done = mpw::div_by_recip(B.t3, hq, ht, hu, R, B, P);
    if (!done) hq = mpw::div(B.t3, B.a, ht, B.v, hu, B.prod, B.t0, B.t1, B.t2, P);
    mpw::store(tm, &ex(J, i, j), &sg(J, i, j), B.t3, hq, P);
}
__global__ void __launch_bounds__(64) k_adj_u_div(MatDev LU, MatDev J, const uint32_t *rw, const int32_t *info,
                                                  int64_t k, int64_t n, int P) {
    extern __shared__ uint32_t lds_raw[];
    (void)n;
    adj_u_div_body(lds_raw, LU, J, rw, info, k, P, blockIdx.x);
}

// Any rank-1 update R, one wave per element: unit b -> (a, c) = (b / R.mc,
// b % R.mc), z_ac <- RZ(z_ac - RZ(x_a (+-y_c))) (fma_like: the operations of
// the elimination's update, a product then a difference, each truncated).
__device__ __forceinline__ void rank1_wave_body(uint32_t *lds_raw, const Rank1 &R, const int32_t *info, int P,
                                                int64_t b) {
    if (*info != 0) return;
    if (b >= R.mr * R.mc) return;
    const int64_t a = b / R.mc, c = b % R.mc;
    const int64_t zi = R.zr + a, zj = R.zc + c;
    Lds L(lds_raw, P);
    fma_like(el(R.Z, zi, zj, P), &ex(R.Z, zi, zj), &sg(R.Z, zi, zj), r1x(R, a, P), r1x_e(R, a), r1x_s(R, a),
             r1y(R, c, P), r1y_e(R, c), r1y_s(R, c), R.yneg == 0, L, P);
}
__global__ void __launch_bounds__(64) k_rank1_wave(Rank1 R, const int32_t *info, int P) {
    extern __shared__ uint32_t lds_raw[];
    rank1_wave_body(lds_raw, R, info, P, (int64_t)blockIdx.x + (int64_t)blockIdx.y * (int64_t)gridDim.x);
}

// The gate the adjugate's and all-minors' kernels test instead of info: 0
// when the factors are complete (info 0, or info == n: only u_nn is zero),
// else info (those kernels then write zeros or nothing).
__global__ void k_factors_gate(const int32_t *info, int64_t n, int32_t *gate) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *gate = factors_complete(*info, n) ? 0 : *info;
}

// adj(A) accumulation step k: block b -> (i, m) = (b / (k+1), b % (k+1)):
// adjT_mi <- RZ(adjT_mi + RZ(J_ik W_km))
__device__ __forceinline__ void adj_prod_body(uint32_t *lds_raw, MatDev J, MatDev W, MatDev T, const int32_t *info,
                                              int64_t k, int P, int64_t b) {
    if (*info != 0) return;
    const int64_t k1 = k + 1;
    if (b >= k1 * k1) return;
    const int64_t i = b / k1, m = b % k1;
    Lds L(lds_raw, P);
    fma_like(el(T, m, i, P), &ex(T, m, i), &sg(T, m, i), el(J, i, k, P), ex(J, i, k), sg(J, i, k),
             el(W, k, m, P), ex(W, k, m), sg(W, k, m), false, L, P);
}
__global__ void __launch_bounds__(64) k_adj_prod(MatDev J, MatDev W, MatDev T, const int32_t *info, int64_t k,
                                                 int P) {
    extern __shared__ uint32_t lds_raw[];
    adj_prod_body(lds_raw, J, W, T, info, k, P, (int64_t)blockIdx.x + (int64_t)blockIdx.y * (int64_t)gridDim.x);
}

// The last-column minors of every leading block (mp_det_all_minors): row r
// of W, after the sweeps above, is the minors solve of the leading
// (r+1) x (r+1) block (its multipliers are the leading block of L), so
// C[r][i] = RZ(D_r W[r][i]) for i < r, C[r][r] = D_r (D_r the determinant of
// the leading r x r block, D_0 = 1), and 0 above the diagonal -- the same
// operations, in the same order, as the minors of that block alone.  Block b
// -> element (b / n, b % n); info != 0 writes zeros.
__global__ void __launch_bounds__(64) k_all_minors_final(MatDev D, MatDev W, MatDev C, const int32_t *info,
                                                         int64_t n, int P) {
    extern __shared__ uint32_t lds_raw[];
    const int64_t b = (int64_t)blockIdx.x + (int64_t)blockIdx.y * (int64_t)gridDim.x;
    if (b >= n * n) return;
    const int64_t r = b / n, i = b % n;
    uint32_t *cm = el(C, r, i, P);
    const bool one = *info == 0 && r == 0 && i == 0;
    if (*info != 0 || i > r || one) {
        for (int q = mpw::lane(); q < P; q += MP_WAVE) cm[q] = (one && q == P - 1) ? 0x80000000u : 0u;
        if (mpw::lane() == 0) {
            ex(C, r, i) = one ? 1 : 0;
            sg(C, r, i) = 0;
        }
        return;
    }
    const uint32_t *dm = el(D, 0, r - 1, P);
    if (i == r) {
        for (int q = mpw::lane(); q < P; q += MP_WAVE) cm[q] = dm[q];
        if (mpw::lane() == 0) {
            ex(C, r, i) = ex(D, 0, r - 1);
            sg(C, r, i) = sg(D, 0, r - 1);
        }
        return;
    }
    Lds L(lds_raw, P);
    mpw::Hdr hd = mpw::load(L.sc.x, dm, ex(D, 0, r - 1), sg(D, 0, r - 1), P);
    mpw::Hdr hx = load_y(L.sc.ypad, el(W, r, i, P), ex(W, r, i), sg(W, r, i), P);
    mpw::Hdr hr = mpw::mul(L.sc.t3, hd, hx, P, L.sc);
    mpw::store(cm, &ex(C, r, i), &sg(C, r, i), L.sc.t3, hr, P);
}

// Normalised minors (eq. (minors)): O[r][i] = RZ_p(C[r][i] / C[r][0]), each
// row divided by its first entry (for mp_det_minors' vector, delta_{N,n}; for
// mp_det_all_minors' rows, the same for every leading block).  A row whose
// first entry is zero is written as zeros.  O must not overlap C.  Block b ->
// (b / cols, b % cols).
__global__ void __launch_bounds__(64) k_norm_minors(MatDev C, MatDev O, int64_t rows, int64_t cols, int P) {
    extern __shared__ uint32_t lds_raw[];
    const int64_t b = (int64_t)blockIdx.x + (int64_t)blockIdx.y * (int64_t)gridDim.x;
    if (b >= rows * cols) return;
    const int64_t r = b / cols, i = b % cols;
    uint32_t *om = el(O, r, i, P);
    const uint32_t *ym = el(C, r, 0, P);
    if (ym[P - 1] == 0u) {
        for (int q = mpw::lane(); q < P; q += MP_WAVE) om[q] = 0u;
        if (mpw::lane() == 0) {
            ex(O, r, i) = 0;
            sg(O, r, i) = 0;
        }
        return;
    }
    mpw::DivBufs B = mpw::div_bufs(lds_raw, P);
    mpw::Hdr hx = mpw::load(B.a, el(C, r, i, P), ex(C, r, i), sg(C, r, i), P);
    mpw::Hdr hy = mpw::load(B.v, ym, ex(C, r, 0), sg(C, r, 0), P);
    mpw::Hdr hq = mpw::div(B.t3, B.a, hx, B.v, hy, B.prod, B.t0, B.t1, B.t2, P);
    mpw::store(om, &ex(O, r, i), &sg(O, r, i), B.t3, hq, P);
}

}  // namespace mpk
