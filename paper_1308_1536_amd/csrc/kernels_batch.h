// kernels_batch.h -- many matrices of uneven n, one launch per phase per step.
//
// The host sorts the batch by n (largest first), so the matrices still active
// at step k (n > k) are a prefix of that order.  Each batched launch covers
// every active matrix: off[0..cnt] are prefix sums of the matrices' block
// counts for this (step, phase), block bx belongs to the t-th active matrix
// with off[t] <= bx < off[t+1] (binary search), and runs the same per-block
// body as the single-matrix kernels with that matrix's descriptor.
#pragma once

#include "kernels_lane.h"
#include "kernels_mfma.h"

namespace mpk {

struct BatchMat {
    MatDev A, D, c;
    int32_t *info;
    int64_t n;
    uint8_t *Lr, *Ub;  // MFMA digit strings (null on the VALU path)
    uint32_t *T;       // product-top records (MFMA path, and the VALU path for P <= 128)
    uint32_t *rw;      // the pivot's reciprocal (P + 2 limbs) and the pending pivot code
};

// largest t in [0, cnt) with off[t] <= bx
__device__ __forceinline__ int locate(const int64_t *off, int cnt, int64_t bx) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= bx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

#define MPK_BATCH_PROLOGUE                                   \
    extern __shared__ uint32_t lds_raw[];                    \
    const int64_t bx = flat_block();                         \
    if (bx >= off[cnt]) return;                              \
    const int t = locate(off, cnt, bx);                      \
    const BatchMat M = mats[order[t]];                       \
    const int64_t loc = bx - off[t];

__global__ void __launch_bounds__(64) k_batch_pivot(const BatchMat *mats, const int32_t *order, const int64_t *off,
                                                    int cnt, int64_t k, int P) {
    MPK_BATCH_PROLOGUE
    pivot_recip_body(lds_raw, M.A, M.D, M.info, M.info, M.rw, k, M.n, P, (int)loc);
}

__global__ void __launch_bounds__(64) k_batch_divide(const BatchMat *mats, const int32_t *order, const int64_t *off,
                                                     int cnt, int64_t k, int P) {
    MPK_BATCH_PROLOGUE
    divide_body(lds_raw, M.A, M.rw, M.info, k, M.n, P, loc);
}

__global__ void __launch_bounds__(64) k_batch_update_valu(const BatchMat *mats, const int32_t *order,
                                                          const int64_t *off, int cnt, int64_t k, int P) {
    MPK_BATCH_PROLOGUE
    update_valu_body(lds_raw, M.A, M.info, k, M.n, P, loc);
}

template <int ROWS>
__global__ void __launch_bounds__(64 * ROWS) k_batch_prod_lane(const BatchMat *mats, const int32_t *order,
                                                               const int64_t *off, int cnt, int64_t k, int P) {
    MPK_BATCH_PROLOGUE
    prod_lane_body<ROWS>(lds_raw, elim_rank1(M.A, k, M.n), M.T, M.info, P, loc);
}

__global__ void __launch_bounds__(64) k_batch_prep(const BatchMat *mats, const int32_t *order, const int64_t *off,
                                                   int cnt, int64_t k, int P) {
    MPK_BATCH_PROLOGUE
    mfma_prep_body(lds_raw, M.A, M.Lr, M.Ub, M.info, k, M.n, P, loc);
}

template <int NC, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_batch_update_mfma(const BatchMat *mats, const int32_t *order, const int64_t *off, int cnt, int64_t k, int P) {
    MPK_BATCH_PROLOGUE
    // every matrix's block count is a multiple of 8, so loc and bx agree mod 8
    // and the XCD-aware column mapping holds inside each matrix
    update_mfma_body<NC, WAVES>(lds_raw, M.A, M.Lr, M.Ub, M.T, M.info, k, M.n, P, 0, M.n - k - 1, loc, true);
}

template <bool STREAM>
__global__ void __launch_bounds__(64) k_batch_finish(const BatchMat *mats, const int32_t *order,
                                                     const int64_t *off, int cnt, int64_t k, int P) {
    MPK_BATCH_PROLOGUE
    // the look-ahead pivot runs only where the host launches no pivot phase
    finish_body<STREAM>(lds_raw, M.A, M.T, M.info, k, M.n, P, 0, M.n - k - 1, loc, M.D,
                        finish_lookahead_ok(P) ? M.rw : nullptr);
}

// minors sweep number s: matrix of size n processes j = n - 1 - s (blocks i < j)
__global__ void __launch_bounds__(64) k_batch_msweep(const BatchMat *mats, const int32_t *order, const int64_t *off,
                                                     int cnt, int64_t s, int P) {
    MPK_BATCH_PROLOGUE
    minors_sweep_body(lds_raw, M.A, M.c, M.info, M.n - 1 - s, M.n, P, loc);
}

__global__ void __launch_bounds__(64) k_batch_mfinal(const BatchMat *mats, const int32_t *order, const int64_t *off,
                                                     int cnt, int64_t unused, int P) {
    MPK_BATCH_PROLOGUE
    (void)unused;
    minors_final_body(lds_raw, M.D, M.c, M.info, M.n, P, loc);
}

// zero the minors accumulators of every matrix (one block per 256 limbs), and
// clear info
__global__ void k_batch_minit(const BatchMat *mats, const int32_t *order, const int64_t *off, int cnt, int P) {
    const int64_t bx = flat_block();
    if (bx >= off[cnt]) return;
    const int t = locate(off, cnt, bx);
    const BatchMat M = mats[order[t]];
    const int64_t e = (bx - off[t]) * 256 + threadIdx.x;
    if (e < M.n * (int64_t)P) M.c.limbs[e] = 0u;
    if (e < M.n) {
        M.c.exp[e] = 0;
        M.c.sign[e] = 0;
    }
}

__global__ void k_batch_zero_info(int32_t *info, int64_t batch) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < batch) info[i] = 0;
}

// clear (promote = 0) or move into info (promote = 1) every matrix's pending
// pivot code
__global__ void k_batch_pend(const BatchMat *mats, int64_t batch, int P, int promote) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const BatchMat M = mats[b];
    if (!promote) M.rw[P + 2] = 0u;
    else if (*M.info == 0) *M.info = (int32_t)M.rw[P + 2];
}

#undef MPK_BATCH_PROLOGUE

}  // namespace mpk
