// mpdet_api.hip -- C-ABI of libmpdet.so (declared in include/mpdet.h).
//
// Host side: argument validation, the step loop of the elimination, and
// kernel launches on the caller's stream.  Every arithmetic step runs in the
// HIP kernels of kernels_valu.h / kernels_mfma.h.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "mpdet.h"
#include "kernels_valu.h"
#include "kernels_mfma.h"
#include "kernels_adj.h"
#include "kernels_batch.h"
#include "kernels_lane.h"
#include "kernels_persist.h"
#include "kernels_ball.h"
#include "peaks.h"
#include <algorithm>
#include <mutex>
#include <numeric>
#include <vector>

// Per-kernel timing (off by default): each launch is bracketed by two HIP
// events recorded on the launch stream; mpdet_profile_end folds the elapsed
// times into per-kernel totals.
enum KernelId { K_PIVOT_DIVIDE = 0, K_DIVIDE, K_UPDATE_VALU, K_UPDATE_MFMA, K_MFMA_PREP, K_MINORS_SWEEP,
                K_MINORS_FINAL, K_UPDATE_FINISH, K_ADJUGATE, K_ALL_MINORS, K_BATCH_PERSIST, K_OTHER, K_COUNT };
static const char *kKernelNames[K_COUNT] = {"pivot_divide", "divide",       "update_valu",   "update_mfma",
                                            "mfma_prep",    "minors_sweep", "minors_final",  "update_finish",
                                            "adjugate",     "all_minors",   "batch_persistent", "other"};

struct ProfRec {
    int kernel;
    hipEvent_t start, stop;
};

struct mpdet_handle {
    int device;
    bool profiling;
    ProfRec *recs;
    int64_t nrec, caprec;
    hipEvent_t *pool;
    int64_t npool, cappool;
    double total_ms[K_COUNT];
    int64_t launches[K_COUNT];
    // MFMA-path workspace (grown on demand, freed by mpdet_destroy)
    void *ws;
    size_t ws_bytes;
    // rows per panel of the trailing update (0: from kRecBudget)
    int64_t panel_rows;
    // the pivot's reciprocal
    void *rw;
    size_t rw_bytes;
    // adjugate workspace
    void *aw;
    size_t aw_bytes;
    // batched launches: device workspace, pinned staging of the tables, and
    // the event of the last staging copy
    void *bw;
    size_t bw_bytes;
    void *bh;
    size_t bh_bytes;
    hipEvent_t bh_done;
    bool bh_pending;
    // radii of the ball-arithmetic factorisation: R (n x n) and the
    // multipliers' radii (n)
    void *radw;
    size_t radw_bytes;
    // MFMA path: row panels per step whose finish runs on a second stream
    // beside the next panel's update (0 or 1: off), that stream and its events
    int32_t overlap_panels;
    hipStream_t side;
    hipEvent_t ev_upd[2], ev_fin[2], ev_join;
    // tuning (0: the defaults): rows per workgroup of the VALU lane product
    // (2, 4, 8) and waves per workgroup of the MFMA update (1, 2, 4)
    int32_t lane_rows, mfma_waves;
    // the bound on each wait inside a launch (the persistent batched launch,
    // the teams of the step-serial kernels) in seconds (10 s before the first
    // setting), and the wall clock's rate
    double wait_limit_s;
    bool wait_limit_set;
    int wall_khz;
    // every multiplier by long division (mpdet_set_long_division)
    int32_t long_div;
};

namespace {

constexpr int kMaxLimbs = 1024;

int check(hipError_t e) { return e == hipSuccess ? MPDET_OK : MPDET_EHIP; }

// the handle's wait limit in wall-clock ticks (no handle: 10 s on the
// current device's clock)
uint64_t wait_ticks(const mpdet_handle *h) {
    const double lim_s = h && h->wait_limit_set ? h->wait_limit_s : 10.0;
    int khz = h ? h->wall_khz : 0;
    if (khz < 1) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz < 1)
            khz = 100000;
    }
    return (uint64_t)(lim_s * (double)khz * 1000.0);
}

bool mat_ok(const mpdet_mat &m, bool need_ptrs) {
    if (m.rows < 0 || m.cols < 0 || m.ld < m.cols || m.nlimbs < 2 || m.nlimbs > kMaxLimbs) return false;
    if (need_ptrs && (!m.limbs || !m.exp || !m.sign)) return false;
    return true;
}

mpk::MatDev dev(const mpdet_mat &m) { return mpk::MatDev{m.limbs, m.exp, m.sign, m.ld}; }

// the byte ranges a rows x cols matrix spans (limbs, exponents, signs) of x
// and y intersect anywhere (addresses compared as integers; rows, cols > 0)
bool mats_overlap(const mpdet_mat &x, const mpdet_mat &y) {
    auto span = [](const void *p, int64_t rows, int64_t ld, int64_t cols, size_t elem, uintptr_t *lo,
                   uintptr_t *hi) {
        *lo = (uintptr_t)p;
        *hi = *lo + (size_t)((rows - 1) * ld + cols) * elem;
    };
    const void *px[3] = {x.limbs, x.exp, x.sign}, *py[3] = {y.limbs, y.exp, y.sign};
    const size_t ex_[3] = {(size_t)x.nlimbs * 4u, 8u, 4u}, ey_[3] = {(size_t)y.nlimbs * 4u, 8u, 4u};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            uintptr_t l1, h1, l2, h2;
            span(px[a], x.rows, x.ld, x.cols, ex_[a], &l1, &h1);
            span(py[b], y.rows, y.ld, y.cols, ey_[b], &l2, &h2);
            if (l1 < h2 && l2 < h1) return true;
        }
    return false;
}
mpk::MatDev dev_mat(const mpdet_mat &m) { return dev(m); }

dim3 grid_for(int64_t blocks) {
    // gridDim.x <= 2^31-1; fold into y beyond that
    const int64_t maxx = 1 << 30;
    if (blocks <= maxx) return dim3((unsigned)blocks, 1, 1);
    return dim3((unsigned)maxx, (unsigned)((blocks + maxx - 1) / maxx), 1);
}

int last_launch() { return check(hipGetLastError()); }

hipEvent_t pool_event(mpdet_handle *h) {
    if (h->npool == h->cappool) {
        int64_t cap = h->cappool ? 2 * h->cappool : 256;
        hipEvent_t *p = (hipEvent_t *)realloc(h->pool, sizeof(hipEvent_t) * (size_t)cap);
        if (!p) return nullptr;
        h->pool = p;
        for (int64_t i = h->cappool; i < cap; ++i)
            if (hipEventCreate(&h->pool[i]) != hipSuccess) h->pool[i] = nullptr;
        h->cappool = cap;
    }
    return h->pool[h->npool++];
}

// Bracket one launch with events when profiling is on.
struct Prof {
    mpdet_handle *h;
    hipStream_t s;
    int kernel;
    hipEvent_t stop = nullptr;
    Prof(mpdet_handle *h_, hipStream_t s_, int k) : h(h_), s(s_), kernel(k) {
        if (!h || !h->profiling) return;
        hipEvent_t start = pool_event(h);
        stop = pool_event(h);
        if (!start || !stop) {
            stop = nullptr;
            return;
        }
        if (h->nrec == h->caprec) {
            int64_t cap = h->caprec ? 2 * h->caprec : 256;
            ProfRec *p = (ProfRec *)realloc(h->recs, sizeof(ProfRec) * (size_t)cap);
            if (!p) {
                stop = nullptr;
                return;
            }
            h->recs = p;
            h->caprec = cap;
        }
        h->recs[h->nrec++] = ProfRec{kernel, start, stop};
        (void)hipEventRecord(start, s);
    }
    ~Prof() {
        if (stop) (void)hipEventRecord(stop, s);
    }
};

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int d) {
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(d) == hipSuccess) ok = true;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// A fixed device region the factorisation's workspace is carved from instead
// of the handle's allocations (the allocation-free entry point's scratch): the
// pivot's reciprocal first, then the update's digits and records.
struct Arena {
    uint8_t *base;
    size_t cap;
};

size_t recip_bytes(int P) { return ((size_t)(P + 3) * 4u + 255) & ~(size_t)255; }

// Scratch for the pivot's reciprocal: P + 2 limbs (R and its exactness flag),
// then the pending pivot code (see finish_body).
int recip_ws(mpdet_handle *h, int P, uint32_t **rw, const Arena *ar = nullptr) {
    const size_t need = recip_bytes(P);
    if (ar) {
        if (need > ar->cap) return MPDET_ERANGE;
        *rw = (uint32_t *)ar->base;
        return MPDET_OK;
    }
    if (need > h->rw_bytes) {
        if (h->rw) (void)hipFree(h->rw);
        h->rw = nullptr;
        h->rw_bytes = 0;
        if (hipMalloc(&h->rw, need) != hipSuccess) {
            h->rw = nullptr;
            (void)hipGetLastError();
            return MPDET_ENOMEM;
        }
        h->rw_bytes = need;
    }
    *rw = (uint32_t *)h->rw;
    return MPDET_OK;
}

// Algorithm 1 steps 2.1 and 2.2.1 for step k: D_k and the pivot's reciprocal
// (unless the previous step's finish launch already examined this pivot),
// then the multipliers of rows k+1..n-1.
int pivot_step(mpdet_handle *h, const mpk::MatDev &a, const mpk::MatDev &d, int32_t *info, uint32_t *rw, int64_t k,
               int64_t n, int P, bool pivot_done, hipStream_t s) {
    int rc;
    const size_t lds = mpk::pivot_lds_bytes(P);
    if (!pivot_done) {
        {
            Prof pr(h, s, K_PIVOT_DIVIDE);
            hipLaunchKernelGGL(mpk::k_pivot_recip, dim3(2), dim3(64 * mpk::team_waves(P)), lds, s, a, d, info, rw,
                               k, n, P, wait_ticks(h));
        }
        if ((rc = last_launch())) return rc;
    }
    const int64_t m = n - k - 1;
    if (m <= 0) return MPDET_OK;
    {
        Prof pr(h, s, K_DIVIDE);
        hipLaunchKernelGGL(mpk::k_divide, dim3((unsigned)m), dim3(64 * mpk::team_waves(P)), mpk::divide_lds_bytes(P), s, a,
                           (const uint32_t *)rw, info, k, n, P, wait_ticks(h), h ? h->long_div : 0);
    }
    return last_launch();
}

// the pending pivot code: cleared before a factorisation, moved into info after it
int pend_clear(uint32_t *rw, int P, hipStream_t s) {
    hipLaunchKernelGGL(mpk::k_pend_clear, dim3(1), dim3(64), 0, s, rw, P);
    return last_launch();
}
int pend_promote(int32_t *info, const uint32_t *rw, int P, hipStream_t s) {
    hipLaunchKernelGGL(mpk::k_pend_promote, dim3(1), dim3(64), 0, s, info, rw, P);
    return last_launch();
}


// Workspace of the MFMA path for trailing blocks up to m x m: reversed
// multiplier digits, pivot-row digits and product-top records.
struct MfmaWs {
    uint8_t *Lr, *Ub;
    uint32_t *T;
};

// bytes of the product-top records for an m x m trailing block, plus the
// padding the finish kernel's unconditional read-ahead may touch past the
// last record ((P + 40) * 32 words)
size_t mfma_rec_bytes(int64_t rows, int64_t m, int P) {
    return ((size_t)mpk::rec_slots(rows, m) * (size_t)mpk::mfma_geom(P).TP + (size_t)(P + 40) * 32u) * 4u;
}

// Bytes the product-top records of one panel may take: the trailing update
// runs over row panels of at most this size, so the workspace stays bounded
// (a 6144 x 6144 matrix of 32768-bit numbers alone takes 155 GB).
constexpr size_t kRecBudget = (size_t)24 << 30;

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// bytes of the reversed multiplier digits and the pivot-row digits for an
// m x m trailing block (the MFMA path only)
size_t mfma_digit_bytes(int64_t m, int P) {
    return up256((size_t)m * mpk::mfma_geom(P).LR) + up256(mpk::ub_bytes(m, P));
}

// rows per panel for trailing blocks up to m x m: the handle's setting, else
// as many as fit kRecBudget; from a fixed arena, as many as fit what the
// reciprocal and the digits leave of it (0 if not one row fits)
int64_t panel_rows(const mpdet_handle *h, int64_t m, int P, const Arena *ar = nullptr) {
    const size_t per_row = (size_t)((m + 31) / 32) * 32u * (size_t)mpk::mfma_geom(P).TP * 4u;
    if (ar) {
        const size_t fixed = recip_bytes(P) + mfma_digit_bytes(m, P) + up256(mfma_rec_bytes(0, m, P)) + 256u;
        if (fixed + per_row > ar->cap) return 0;
        const int64_t r = (int64_t)((ar->cap - fixed) / per_row);
        return r < m ? r : m;
    }
    if (h->panel_rows > 0) return h->panel_rows < m ? h->panel_rows : m;
    const int64_t r = (int64_t)(kRecBudget / per_row);
    return r < 1 ? 1 : (r < m ? r : m);
}

// digits: the MFMA path's digit strings are needed (the lane product reads
// only the records)
int mfma_workspace(mpdet_handle *h, int64_t m, int P, int64_t rows, MfmaWs *w, bool digits = true,
                   const Arena *ar = nullptr) {
    const mpk::MfmaGeom g = mpk::mfma_geom(P);
    auto up = up256;
    const size_t lr = digits ? up((size_t)m * g.LR) : 0, ub = digits ? up(mpk::ub_bytes(m, P)) : 0;
    const size_t t = up(mfma_rec_bytes(rows, m, P));
    const size_t need = lr + ub + t;
    if (ar) {
        const size_t off = recip_bytes(P);
        if (off > ar->cap || need > ar->cap - off) return MPDET_ERANGE;
        uint8_t *base = ar->base + off;
        w->Lr = digits ? base : nullptr;
        w->Ub = digits ? base + lr : nullptr;
        w->T = (uint32_t *)(base + lr + ub);
        return MPDET_OK;
    }
    if (need > h->ws_bytes) {
        if (h->ws) (void)hipFree(h->ws);
        h->ws = nullptr;
        h->ws_bytes = 0;
        if (hipMalloc(&h->ws, need) != hipSuccess) {
            h->ws = nullptr;
            (void)hipGetLastError();
            return MPDET_ENOMEM;
        }
        h->ws_bytes = need;
    }
    uint8_t *base = (uint8_t *)h->ws;
    w->Lr = digits ? base : nullptr;
    w->Ub = digits ? base + lr : nullptr;
    w->T = (uint32_t *)(base + lr + ub);
    return MPDET_OK;
}

// The tuned variants (every one gives the same bits).
int lane_rows_of(const mpdet_handle *h) { return h && h->lane_rows ? h->lane_rows : mpk::kLaneRows; }
int mfma_waves_of(const mpdet_handle *h) { return h && h->mfma_waves ? h->mfma_waves : mpk::kMfmaWaves; }

using LaneKernel = void (*)(mpk::MatDev, uint32_t *, const int32_t *, int64_t, int64_t, int);
using LaneR1Kernel = void (*)(mpk::Rank1, uint32_t *, const int32_t *, int);
using MfmaKernel = void (*)(mpk::MatDev, const uint8_t *, const uint8_t *, uint32_t *, const int32_t *, int64_t,
                            int64_t, int, int64_t, int64_t);
using BatchKernel = void (*)(const mpk::BatchMat *, const int32_t *, const int64_t *, int, int64_t, int);

LaneKernel lane_kernel(int rows) {
    return rows == 2 ? mpk::k_prod_lane<2> : rows == 8 ? mpk::k_prod_lane<8> : mpk::k_prod_lane<4>;
}
LaneR1Kernel lane_r1_kernel(int rows) {
    return rows == 2 ? mpk::k_prod_lane_r1<2> : rows == 8 ? mpk::k_prod_lane_r1<8> : mpk::k_prod_lane_r1<4>;
}
BatchKernel batch_lane_kernel(int rows) {
    return rows == 2 ? mpk::k_batch_prod_lane<2> : rows == 8 ? mpk::k_batch_prod_lane<8> : mpk::k_batch_prod_lane<4>;
}
MfmaKernel mfma_kernel(int copies, int waves, bool fuse = false) {
    if (fuse) {
        if (copies == 4)
            return waves == 1 ? mpk::k_update_mfma<4, 1, true>
                              : waves == 4 ? mpk::k_update_mfma<4, 4, true> : mpk::k_update_mfma<4, 2, true>;
        return waves == 1 ? mpk::k_update_mfma<1, 1, true>
                          : waves == 4 ? mpk::k_update_mfma<1, 4, true> : mpk::k_update_mfma<1, 2, true>;
    }
    if (copies == 4) return waves == 1 ? mpk::k_update_mfma<4, 1> : waves == 4 ? mpk::k_update_mfma<4, 4>
                                                                                : mpk::k_update_mfma<4, 2>;
    return waves == 1 ? mpk::k_update_mfma<1, 1> : waves == 4 ? mpk::k_update_mfma<1, 4> : mpk::k_update_mfma<1, 2>;
}
BatchKernel batch_mfma_kernel(int copies, int waves) {
    if (copies == 4)
        return waves == 1 ? mpk::k_batch_update_mfma<4, 1>
                          : waves == 4 ? mpk::k_batch_update_mfma<4, 4> : mpk::k_batch_update_mfma<4, 2>;
    return waves == 1 ? mpk::k_batch_update_mfma<1, 1>
                      : waves == 4 ? mpk::k_batch_update_mfma<1, 4> : mpk::k_batch_update_mfma<1, 2>;
}

// one rank-1 update on the lane product and the tile finish (records in T)
int lane_rank1(const mpdet_handle *h, const mpk::Rank1 &R, uint32_t *T, const int32_t *info, int P,
               hipStream_t s) {
    if (R.mr <= 0 || R.mc <= 0) return MPDET_OK;
    const int rows = lane_rows_of(h);
    hipLaunchKernelGGL(lane_r1_kernel(rows), grid_for(mpk::lane_update_blocks(R.mr, R.mc, rows)), dim3(64 * rows),
                       mpk::lane_lds_bytes(P, rows), s, R, T, info, P);
    hipLaunchKernelGGL(mpk::k_finish_r1, grid_for(mpk::finish_blocks(R.mr, R.mc, P)), dim3(64),
                       mpk::finish_lds_bytes(P), s, R, (const uint32_t *)T, info, P);
    return last_launch();
}

// VALU path.  For P <= 128 (P a multiple of 4) each step runs the
// lane-per-element product kernel into the record buffer, then the finish
// kernel the MFMA path uses; otherwise one wave per element update.
int factor_valu(mpdet_handle *h, const mpdet_mat &A, const mpdet_mat &D, int32_t *info, int64_t k_begin,
                int64_t k_end, hipStream_t s, const Arena *ar = nullptr) {
    const int64_t n = A.rows;
    const int P = A.nlimbs;
    const size_t lds = mpk::lds_bytes(P);
    const bool lane = mpk::lane_update_ok(P);
    MfmaWs w{};
    if (lane) {
        const int64_t m0 = n > 1 ? n - 1 : 1;
        int rc = mfma_workspace(h, m0, P, m0, &w, false, ar);
        if (rc) return rc;
    }
    const int lrows = lane_rows_of(h);
    const size_t lds_prod = mpk::lane_lds_bytes(P, lrows), lds_fin = mpk::finish_launch_lds(P);
    auto fin_kernel = mpk::finish_streams(P) ? mpk::k_finish<true> : mpk::k_finish<false>;
    mpk::MatDev a = dev(A), d = dev(D);
    const int32_t *cinfo = info;
    uint32_t *rw = nullptr;
    const bool ahead = lane && mpk::finish_lookahead_ok(P);  // the finish launch examines the next pivot
    int rc0 = recip_ws(h, P, &rw, ar);
    if (rc0 || (rc0 = pend_clear(rw, P, s))) return rc0;
    for (int64_t k = k_begin; k < k_end; ++k) {
        // with the finish kernel, step k's pivot was examined by step k-1's finish launch
        int rc = pivot_step(h, a, d, info, rw, k, n, P, ahead && k > k_begin, s);
        if (rc) return rc;
        const int64_t m = n - k - 1;
        if (m <= 0) continue;
        if (lane) {
            {
                Prof pr(h, s, K_UPDATE_VALU);
                hipLaunchKernelGGL(lane_kernel(lrows), grid_for(mpk::lane_update_blocks(m, m, lrows)), dim3(64 * lrows),
                                   lds_prod, s, a, w.T, cinfo, k, n, P);
            }
            if ((rc = last_launch())) return rc;
            {
                Prof pr(h, s, K_UPDATE_FINISH);
                hipLaunchKernelGGL(fin_kernel, grid_for(mpk::finish_blocks(m, m, P)), dim3(64), lds_fin, s, a, w.T,
                                   cinfo, k, n, P, (int64_t)0, m, d, ahead ? rw : nullptr);
            }
        } else {
            Prof pr(h, s, K_UPDATE_VALU);
            hipLaunchKernelGGL(mpk::k_update_valu, grid_for(m * m), dim3(64), lds, s, a, cinfo, k, n, P);
        }
        if ((rc = last_launch())) return rc;
    }
    return pend_promote(info, rw, P, s);
}

// the second stream and events of the overlapped MFMA schedule
int overlap_ready(mpdet_handle *h) {
    if (!h->side && hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) {
        h->side = nullptr;
        return MPDET_EHIP;
    }
    for (int t = 0; t < 2; ++t) {
        if (!h->ev_upd[t] && hipEventCreateWithFlags(&h->ev_upd[t], hipEventDisableTiming) != hipSuccess)
            return MPDET_EHIP;
        if (!h->ev_fin[t] && hipEventCreateWithFlags(&h->ev_fin[t], hipEventDisableTiming) != hipSuccess)
            return MPDET_EHIP;
    }
    if (!h->ev_join && hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) return MPDET_EHIP;
    return MPDET_OK;
}

int factor_mfma(mpdet_handle *h, const mpdet_mat &A, const mpdet_mat &D, int32_t *info, int64_t k_begin,
                int64_t k_end, hipStream_t s, const Arena *ar = nullptr) {
    const int64_t n = A.rows;
    const int P = A.nlimbs;
    MfmaWs w;
    const int64_t m0 = n - k_begin - 1 > 1 ? n - k_begin - 1 : 1;
    // overlapped schedule: S row panels per step, the finish of panel p on a
    // second stream while the update of panel p + 1 runs, two record buffers
    const int S = (!ar && h && h->overlap_panels > 1) ? h->overlap_panels : 1;
    // the finish inside the update launch (the default where it applies;
    // overlap setting 1 keeps it a launch of its own)
    const int mw = mfma_waves_of(h);
    const bool fuse = S == 1 && !(h && h->overlap_panels == 1) && mpk::mfma_fuse_ok(P, mw);
    int64_t R = panel_rows(h, m0, P, ar);
    if (R < 1) return MPDET_ERANGE;
    if (S > 1) R = std::min<int64_t>(R, (m0 + S - 1) / S);
    int rc = mfma_workspace(h, m0, P, S > 1 ? 2 * R : R, &w, true, ar);
    if (rc) return rc;
    if (S > 1 && (rc = overlap_ready(h))) return rc;
    uint32_t *Tbuf[2] = {w.T, w.T + (size_t)mpk::rec_slots(R, m0) * (size_t)mpk::mfma_geom(P).TP};
    if (mpk::mfma_copies(P, mw) == 0) return MPDET_ENOTSUP;
    const size_t lds_mfma = mpk::mfma_lds_bytes(P, mw), lds_prep = (size_t)(P + 1) * 4;
    const size_t lds_fin = mpk::finish_launch_lds(P);
    auto fin_kernel = mpk::finish_streams(P) ? mpk::k_finish<true> : mpk::k_finish<false>;
    auto upd_kernel = mfma_kernel(mpk::mfma_copies(P, mw), mw, fuse);
    mpk::MatDev a = dev(A), d = dev(D);
    const int32_t *cinfo = info;
    uint32_t *rw = nullptr;
    if ((rc = recip_ws(h, P, &rw, ar)) || (rc = pend_clear(rw, P, s))) return rc;
    const bool ahead = !fuse && mpk::finish_lookahead_ok(P);  // the finish launch examines the next pivot
    for (int64_t k = k_begin; k < k_end; ++k) {
        if ((rc = pivot_step(h, a, d, info, rw, k, n, P, ahead && k > k_begin, s))) return rc;
        const int64_t m = n - k - 1;
        if (m <= 0) continue;
        {
            Prof pr(h, s, K_MFMA_PREP);
            hipLaunchKernelGGL(mpk::k_mfma_prep, grid_for(2 * m), dim3(64), lds_prep, s, a, w.Lr, w.Ub, cinfo, k,
                               n, P);
        }
        if ((rc = last_launch())) return rc;
        if (S == 1) {
            // row panels [ip0, ip0 + rows) share the record buffer, one after another
            for (int64_t ip0 = 0; ip0 < m; ip0 += R) {
                const int64_t rows = m - ip0 < R ? m - ip0 : R;
                {
                    Prof pr(h, s, K_UPDATE_MFMA);
                    hipLaunchKernelGGL(upd_kernel, grid_for(mpk::mfma_update_blocks(rows, m, mw)),
                                       dim3(64 * mw), lds_mfma, s, a, (const uint8_t *)w.Lr,
                                       (const uint8_t *)w.Ub, w.T, cinfo, k, n, P, ip0, rows);
                }
                if ((rc = last_launch())) return rc;
                if (fuse) continue;
                {
                    Prof pr(h, s, K_UPDATE_FINISH);
                    hipLaunchKernelGGL(fin_kernel, grid_for(mpk::finish_blocks(rows, m, P)), dim3(64), lds_fin, s,
                                       a, w.T, cinfo, k, n, P, ip0, rows, d, ahead ? rw : nullptr);
                }
                if ((rc = last_launch())) return rc;
            }
            continue;
        }
        // overlapped: update p on s into buffer p % 2, then its finish on the
        // side stream; update p + 2 waits for finish p to release the buffer;
        // the step ends when s has waited for the last finish
        const int64_t Rk = std::min<int64_t>(R, (m + S - 1) / S);
        int64_t p = 0;
        for (int64_t ip0 = 0; ip0 < m; ip0 += Rk, ++p) {
            const int64_t rows = m - ip0 < Rk ? m - ip0 : Rk;
            const int b = (int)(p & 1);
            if (p >= 2 && hipStreamWaitEvent(s, h->ev_fin[b], 0) != hipSuccess) return MPDET_EHIP;
            {
                Prof pr(h, s, K_UPDATE_MFMA);
                hipLaunchKernelGGL(upd_kernel, grid_for(mpk::mfma_update_blocks(rows, m, mw)), dim3(64 * mw),
                                   lds_mfma, s, a, (const uint8_t *)w.Lr, (const uint8_t *)w.Ub, Tbuf[b], cinfo, k,
                                   n, P, ip0, rows);
            }
            if ((rc = last_launch())) return rc;
            if (hipEventRecord(h->ev_upd[b], s) != hipSuccess ||
                hipStreamWaitEvent(h->side, h->ev_upd[b], 0) != hipSuccess)
                return MPDET_EHIP;
            {
                Prof pr(h, h->side, K_UPDATE_FINISH);
                hipLaunchKernelGGL(fin_kernel, grid_for(mpk::finish_blocks(rows, m, P)), dim3(64), lds_fin, h->side,
                                   a, Tbuf[b], cinfo, k, n, P, ip0, rows, d, ahead ? rw : nullptr);
            }
            if ((rc = last_launch())) return rc;
            if (hipEventRecord(h->ev_fin[b], h->side) != hipSuccess) return MPDET_EHIP;
        }
        if (hipEventRecord(h->ev_join, h->side) != hipSuccess || hipStreamWaitEvent(s, h->ev_join, 0) != hipSuccess)
            return MPDET_EHIP;
    }
    return pend_promote(info, rw, P, s);
}

// The allocation-free entry point's workspace: one static array per device,
// loaded with the code object and held until the process ends.  Host code
// never uses the array's name as an address: each device's address comes from
// hipGetSymbolAddress, taken once with that device current.
__device__ __align__(256) uint8_t scratch[MPDET_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices];

// the scratch array's address on `device` (which must be current), resolved
// on first use; nullptr if the runtime cannot give it
uint8_t *scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[device] = (uint8_t *)ptr;
    }
    return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

const char *mpdet_strerror(int status) {
    switch (status) {
        case MPDET_OK: return "ok";
        case MPDET_EINVAL: return "invalid argument";
        case MPDET_ENOMEM: return "out of device memory";
        case MPDET_EHIP: return "HIP runtime error";
        case MPDET_ENOTSUP: return "not supported";
        case MPDET_ERANGE: return "workspace exceeds the allocation-free entry point's scratch";
        default: return "unknown status";
    }
}

int mpdet_create(mpdet_handle **h, int device) {
    if (!h) return MPDET_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return MPDET_EHIP;
    if (device < 0 || device >= count) return MPDET_EINVAL;
    mpdet_handle *p = (mpdet_handle *)calloc(1, sizeof(mpdet_handle));
    if (!p) return MPDET_ENOMEM;
    p->device = device;
    {
        // resolve the device's scratch address for mp_det_factor_noalloc
        DeviceGuard g(device);
        if (!g.ok || !scratch_on(device) ||
            hipDeviceGetAttribute(&p->wall_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess ||
            p->wall_khz < 1) {
            free(p);
            return MPDET_EHIP;
        }
    }
    *h = p;
    return MPDET_OK;
}

int mpdet_destroy(mpdet_handle *h) {
    if (!h) return MPDET_EINVAL;
    DeviceGuard g(h->device);
    (void)hipDeviceSynchronize();
    for (int64_t i = 0; i < h->cappool; ++i)
        if (h->pool[i]) (void)hipEventDestroy(h->pool[i]);
    free(h->pool);
    free(h->recs);
    if (h->ws) (void)hipFree(h->ws);
    if (h->rw) (void)hipFree(h->rw);
    if (h->aw) (void)hipFree(h->aw);
    if (h->bw) (void)hipFree(h->bw);
    if (h->radw) (void)hipFree(h->radw);
    if (h->bh) (void)hipHostFree(h->bh);
    if (h->bh_done) (void)hipEventDestroy(h->bh_done);
    for (int t = 0; t < 2; ++t) {
        if (h->ev_upd[t]) (void)hipEventDestroy(h->ev_upd[t]);
        if (h->ev_fin[t]) (void)hipEventDestroy(h->ev_fin[t]);
    }
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->side) (void)hipStreamDestroy(h->side);
    free(h);
    return MPDET_OK;
}

int mpdet_measure_peak(mpdet_handle *h, int kind, double *per_second) {
    if (!h || !per_second || (kind != MPDET_PEAK_MAD64 && kind != MPDET_PEAK_MFMA_I8 && kind != MPDET_PEAK_MFMA_CLOCK))
        return MPDET_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus <= 0)
        return MPDET_EHIP;
    const unsigned blocks = (unsigned)cus * 8u, threads = 256u;
    uint32_t *out = nullptr;
    // the checksum words, then 4 clock stamps (8-byte aligned)
    const size_t out_bytes = (size_t)blocks * threads * 4u;
    if (hipMalloc(&out, out_bytes + 32u) != hipSuccess) {
        (void)hipGetLastError();
        return MPDET_ENOMEM;
    }
    uint64_t *clk = (uint64_t *)((char *)out + out_bytes);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = MPDET_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = MPDET_EHIP;
    const uint32_t iters = kind == MPDET_PEAK_MAD64 ? 8192u : 512u;
    const bool clock = kind == MPDET_PEAK_MFMA_CLOCK;
    float ms = 0.f;
    for (int pass = 0; pass < 2 && rc == MPDET_OK; ++pass) {  // pass 0 warms up
        if (hipEventRecord(e0, nullptr) != hipSuccess) rc = MPDET_EHIP;
        if (kind == MPDET_PEAK_MAD64)
            hipLaunchKernelGGL(mpk::k_peak_mad64, dim3(blocks), dim3(threads), 0, nullptr, iters, 12345u, out);
        else
            hipLaunchKernelGGL(mpk::k_peak_mfma_i8, dim3(blocks), dim3(threads), 0, nullptr, iters, 12345u, out,
                               clock ? clk : nullptr);
        if (rc == MPDET_OK) rc = last_launch();
        if (rc == MPDET_OK && hipEventRecord(e1, nullptr) != hipSuccess) rc = MPDET_EHIP;
        if (rc == MPDET_OK && hipEventSynchronize(e1) != hipSuccess) rc = MPDET_EHIP;
        if (rc == MPDET_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = MPDET_EHIP;
    }
    if (rc == MPDET_OK && clock) {
        uint64_t c[4] = {0, 0, 0, 0};
        if (hipMemcpy(c, clk, sizeof c, hipMemcpyDeviceToHost) != hipSuccess) rc = MPDET_EHIP;
        // shader clocks over 100 MHz real-time ticks
        *per_second = (rc == MPDET_OK && c[3] > c[2]) ? (double)(c[1] - c[0]) / (double)(c[3] - c[2]) * 1e8 : 0.0;
    } else if (rc == MPDET_OK) {
        const double threads_total = (double)blocks * threads;
        const double ops = kind == MPDET_PEAK_MAD64 ? threads_total * 8.0 * iters
                                                    : threads_total / 64.0 * 8.0 * iters * 32768.0;
        *per_second = ms > 0.f ? ops / (ms * 1e-3) : 0.0;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}

int mpdet_profile_begin(mpdet_handle *h) {
    if (!h) return MPDET_EINVAL;
    h->profiling = true;
    h->nrec = 0;
    h->npool = 0;
    for (int k = 0; k < K_COUNT; ++k) {
        h->total_ms[k] = 0.0;
        h->launches[k] = 0;
    }
    return MPDET_OK;
}

int mpdet_profile_end(mpdet_handle *h) {
    if (!h) return MPDET_EINVAL;
    DeviceGuard g(h->device);
    h->profiling = false;
    int rc = MPDET_OK;
    for (int64_t i = 0; i < h->nrec; ++i) {
        const ProfRec &r = h->recs[i];
        if (hipEventSynchronize(r.stop) != hipSuccess) {
            rc = MPDET_EHIP;
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) {
            rc = MPDET_EHIP;
            continue;
        }
        h->total_ms[r.kernel] += ms;
        h->launches[r.kernel] += 1;
    }
    h->nrec = 0;
    h->npool = 0;
    return rc;
}

int mpdet_profile_get(mpdet_handle *h, const char *kernel, double *total_ms, int64_t *launches) {
    if (!h || !kernel || !total_ms || !launches) return MPDET_EINVAL;
    for (int k = 0; k < K_COUNT; ++k) {
        if (strcmp(kernel, kKernelNames[k]) == 0) {
            *total_ms = h->total_ms[k];
            *launches = h->launches[k];
            return MPDET_OK;
        }
    }
    return MPDET_EINVAL;
}

// MPDET_PATH_AUTO: the MFMA path where it applies, except at 64 limbs or
// fewer, where the VALU lane product is faster (2048 bits, 256 matrices of
// N in [16, 384]: 544 against 636 ms; at 4096 bits MFMA leads, 139 against
// 161 ms for two N = 512 matrices)
static bool auto_uses_mfma(int P) {
    return mpk::mfma_supported(P) && !(P <= 64 && mpk::lane_update_ok(P));
}

}  // extern "C"

namespace {
// argument checks shared by mp_det_factor_steps and mp_det_factor_noalloc;
// *use_mfma receives the path taken
int factor_args(const mpdet_mat &A, const mpdet_mat &D, const int32_t *info_dev, int64_t k_begin, int64_t k_end,
                int path, bool *use_mfma) {
    if (!info_dev) return MPDET_EINVAL;
    if (!mat_ok(A, A.rows > 0) || !mat_ok(D, A.rows > 0)) return MPDET_EINVAL;
    if (A.rows != A.cols || D.nlimbs != A.nlimbs || D.rows < 1 || D.cols < A.rows) return MPDET_EINVAL;
    if (k_begin < 0 || k_end < k_begin || k_end > A.rows) return MPDET_EINVAL;
    if (path != MPDET_PATH_AUTO && path != MPDET_PATH_VALU && path != MPDET_PATH_MFMA) return MPDET_EINVAL;
    const bool mfma_ok = mpk::mfma_supported(A.nlimbs);
    if (path == MPDET_PATH_MFMA && !mfma_ok) return MPDET_ENOTSUP;
    *use_mfma = path == MPDET_PATH_MFMA || (path == MPDET_PATH_AUTO && auto_uses_mfma(A.nlimbs));
    return MPDET_OK;
}
}  // namespace

extern "C" {

int mp_det_factor_steps(mpdet_handle *h, mpdet_mat A, mpdet_mat D, int32_t *info_dev, int64_t k_begin,
                        int64_t k_end, int path, void *stream) {
    if (!h) return MPDET_EINVAL;
    bool use_mfma = false;
    if (int rc = factor_args(A, D, info_dev, k_begin, k_end, path, &use_mfma)) return rc;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    hipStream_t s = (hipStream_t)stream;
    if (k_begin == 0) {
        hipLaunchKernelGGL(mpk::k_set_info, dim3(1), dim3(64), 0, s, info_dev, 0);
        int rc = last_launch();
        if (rc) return rc;
    }
    if (k_end == k_begin) return MPDET_OK;
    return use_mfma ? factor_mfma(h, A, D, info_dev, k_begin, k_end, s)
                    : factor_valu(h, A, D, info_dev, k_begin, k_end, s);
}

int mp_det_factor(mpdet_handle *h, mpdet_mat A, mpdet_mat D, int32_t *info_dev, int path, void *stream) {
    return mp_det_factor_steps(h, A, D, info_dev, 0, A.rows, path, stream);
}

int mp_det_extend(mpdet_handle *h, mpdet_mat A, mpdet_mat D, int32_t *info_dev, int64_t n_old, int path,
                  void *stream) {
    if (!h) return MPDET_EINVAL;
    bool use_mfma = false;
    if (int rc = factor_args(A, D, info_dev, 0, A.rows, path, &use_mfma)) return rc;
    const int64_t N = A.rows;
    if (n_old < 0 || n_old > N) return MPDET_EINVAL;
    if (n_old == N) return MPDET_OK;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    hipStream_t s = (hipStream_t)stream;
    const int P = A.nlimbs;
    int rc;
    if (n_old > 0) {
        // Steps 0 .. n_old-1 were applied to the leading block; apply them to
        // the rest in step order: the new rows' multipliers, then the two
        // regions each step updates outside the leading block -- (a) the new
        // rows right of column k, (b) the leading rows below row k in the new
        // columns.  Neither reads what the other writes in the same step.
        uint32_t *rw = nullptr;
        if ((rc = recip_ws(h, P, &rw)) || (rc = pend_clear(rw, P, s))) return rc;
        const bool lane = mpk::lane_update_ok(P);
        MfmaWs w{};
        if (lane) {  // records of the larger region: (N - n_old) x (N - 1) or n_old x (N - n_old)
            const int64_t rows = std::max(N - n_old, n_old), cols = N;
            if ((rc = mfma_workspace(h, cols, P, rows, &w, false))) return rc;
        }
        mpk::MatDev a = dev(A), d = dev(D);
        const size_t lds = mpk::pivot_lds_bytes(P);
        auto rank1 = [&](const mpk::Rank1 &R) -> int {
            if (R.mr <= 0 || R.mc <= 0) return MPDET_OK;
            if (lane) {
                return lane_rank1(h, R, w.T, info_dev, P, s);
            } else {
                hipLaunchKernelGGL(mpk::k_rank1_wave, grid_for(R.mr * R.mc), dim3(64), mpk::lds_bytes(P), s, R,
                                   (const int32_t *)info_dev, P);
            }
            return last_launch();
        };
        for (int64_t k = 0; k < n_old; ++k) {
            // the pivot's reciprocal (D_k is written again with the same bits)
            hipLaunchKernelGGL(mpk::k_pivot_recip, dim3(2), dim3(64 * mpk::team_waves(P)), lds, s, a, d, info_dev,
                               rw, k, N, P, wait_ticks(h));
            if ((rc = last_launch())) return rc;
            hipLaunchKernelGGL(mpk::k_divide_from, dim3((unsigned)(N - n_old)), dim3(64 * mpk::team_waves(P)),
                               mpk::divide_lds_bytes(P), s,
                               a, (const uint32_t *)rw, info_dev, k, N, P, n_old, wait_ticks(h), h->long_div);
            if ((rc = last_launch())) return rc;
            // (a) rows n_old.. x columns k+1..: x = column k below, y = row k
            if ((rc = rank1(mpk::Rank1{a, a, a, n_old, k, 1, 0, k, k + 1, 0, 1, n_old, k + 1, N - n_old, N - k - 1, 0})))
                return rc;
            // (b) rows k+1..n_old-1 x columns n_old..
            if ((rc = rank1(mpk::Rank1{a, a, a, k + 1, k, 1, 0, k, n_old, 0, 1, k + 1, n_old, n_old - k - 1, N - n_old,
                                       0})))
                return rc;
        }
    }
    // steps n_old .. N-1 as a factorisation continued from n_old
    return use_mfma ? factor_mfma(h, A, D, info_dev, n_old, N, s) : factor_valu(h, A, D, info_dev, n_old, N, s);
}

}  // extern "C"
namespace {
int grow_device(void **p, size_t *have, size_t need);
}
extern "C" {

int mp_det_factor_ball(mpdet_handle *h, mpdet_mat A, mpdet_mat D, uint32_t *rad_mant_dev, int64_t *rad_exp_dev,
                       int32_t *info_dev, int flags, int path, void *stream) {
    if (!h) return MPDET_EINVAL;
    bool use_mfma = false;
    if (int rc = factor_args(A, D, info_dev, 0, A.rows, path, &use_mfma)) return rc;
    if (flags & ~MPDET_BALL_INPUT_ULP) return MPDET_EINVAL;
    const int64_t n = A.rows;
    if (n > 0 && (!rad_mant_dev || !rad_exp_dev)) return MPDET_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if (n == 0) return mp_det_factor_steps(h, A, D, info_dev, 0, 0, path, stream);
    const size_t nn = (size_t)n * (size_t)n;
    const size_t need = up256(nn * 4u) + up256(nn * 8u) + up256((size_t)n * 4u) + up256((size_t)n * 8u);
    if ((rc = grow_device(&h->radw, &h->radw_bytes, need))) return rc;
    uint8_t *base = (uint8_t *)h->radw;
    mpk::RadMat R{(uint32_t *)base, (int64_t *)(base + up256(nn * 4u)), n};
    uint32_t *LRm = (uint32_t *)(base + up256(nn * 4u) + up256(nn * 8u));
    int64_t *LRe = (int64_t *)((uint8_t *)LRm + up256((size_t)n * 4u));
    mpk::MatDev a = dev(A), d = dev(D);
    hipLaunchKernelGGL(mpk::k_ball_init, grid_for(((int64_t)nn + 255) / 256), dim3(256), 0, s, a, R, n, A.nlimbs,
                       (flags & MPDET_BALL_INPUT_ULP) ? 1 : 0);
    if ((rc = last_launch())) return rc;
    // one elimination step at a time, each followed by its radii (same bits as
    // one mp_det_factor call: every range continues the state)
    for (int64_t k = 0; k < n; ++k) {
        if ((rc = mp_det_factor_steps(h, A, D, info_dev, k, k + 1, path, stream))) return rc;
        const int64_t m = n - k - 1;
        hipLaunchKernelGGL(mpk::k_ball_mult, grid_for((std::max<int64_t>(m, 1) + 255) / 256), dim3(256), 0, s, a, d,
                           R, LRm, LRe, rad_mant_dev, rad_exp_dev, (const int32_t *)info_dev, k, n, A.nlimbs);
        if (m > 0)
            hipLaunchKernelGGL(mpk::k_ball_update, grid_for((m * (m + 1) + 255) / 256), dim3(256), 0, s, a, R,
                               (const uint32_t *)LRm, (const int64_t *)LRe, (const int32_t *)info_dev, k, n,
                               A.nlimbs);
        if ((rc = last_launch())) return rc;
    }
    hipLaunchKernelGGL(mpk::k_ball_end, grid_for((n + 255) / 256), dim3(256), 0, s, (const int32_t *)info_dev,
                       rad_mant_dev, rad_exp_dev, n);
    return last_launch();
}

int mp_truncate(mpdet_handle *h, mpdet_mat x, mpdet_mat y, void *stream) {
    if (!h) return MPDET_EINVAL;
    const int64_t cnt = x.rows * x.cols;
    if (!mat_ok(x, cnt > 0) || !mat_ok(y, cnt > 0) || y.rows != x.rows || y.cols != x.cols ||
        y.nlimbs > x.nlimbs)
        return MPDET_EINVAL;
    if (cnt == 0) return MPDET_OK;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    const int64_t total = cnt * y.nlimbs;
    hipLaunchKernelGGL(mpk::k_truncate, grid_for((total + 255) / 256), dim3(256), 0, (hipStream_t)stream, dev(x),
                       dev(y), x.rows, x.cols, x.nlimbs, y.nlimbs);
    return last_launch();
}

int mp_det_factor_reduced(mpdet_handle *h, mpdet_mat A, mpdet_mat D, mpdet_mat A2, mpdet_mat D2, int32_t *info_dev,
                          int64_t k_switch, int path, int path2, void *stream) {
    if (!h) return MPDET_EINVAL;
    bool m1 = false, m2 = false;
    if (int rc = factor_args(A, D, info_dev, 0, A.rows, path, &m1)) return rc;
    if (int rc = factor_args(A2, D2, info_dev, 0, A2.rows, path2, &m2)) return rc;
    if (A2.rows != A.rows || A2.nlimbs > A.nlimbs || k_switch < 0 || k_switch > A.rows) return MPDET_EINVAL;
    int rc;
    if ((rc = mp_det_factor_steps(h, A, D, info_dev, 0, k_switch, path, stream))) return rc;
    mpdet_mat Dk = D, Dk2 = D2;  // the leading determinants computed so far
    Dk.rows = Dk2.rows = 1;
    if ((rc = mp_truncate(h, A, A2, stream))) return rc;
    if (k_switch > 0) {
        Dk.cols = Dk2.cols = k_switch;
        if ((rc = mp_truncate(h, Dk, Dk2, stream))) return rc;
    }
    return mp_det_factor_steps(h, A2, D2, info_dev, k_switch, A.rows, path2, stream);
}

int mp_det_factor_noalloc(mpdet_mat A, mpdet_mat D, int32_t *info_dev, int path, void *stream) {
    bool use_mfma = false;
    if (int rc = factor_args(A, D, info_dev, 0, A.rows, path, &use_mfma)) return rc;
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess) return MPDET_EHIP;
    uint8_t *base = scratch_on(device);
    if (!base) return MPDET_EHIP;
    const Arena ar{base, (size_t)MPDET_NOALLOC_SCRATCH_BYTES};
    // the workspace must fit before anything is launched
    const int P = A.nlimbs;
    const int64_t m0 = A.rows > 1 ? A.rows - 1 : 1;
    if (use_mfma ? A.rows > 1 && panel_rows(nullptr, m0, P, &ar) < 1
                 : recip_bytes(P) + (mpk::lane_update_ok(P) && A.rows > 1 ? up256(mfma_rec_bytes(m0, m0, P)) : 0) >
                       ar.cap)
        return MPDET_ERANGE;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(mpk::k_set_info, dim3(1), dim3(64), 0, s, info_dev, 0);
    if (int rc = last_launch()) return rc;
    if (A.rows == 0) return MPDET_OK;
    return use_mfma ? factor_mfma(nullptr, A, D, info_dev, 0, A.rows, s, &ar)
                    : factor_valu(nullptr, A, D, info_dev, 0, A.rows, s, &ar);
}

int mpdet_workspace_size(mpdet_handle *h, int64_t n, int32_t nlimbs, int path, size_t *bytes) {
    if (!bytes || n < 0 || nlimbs < 2 || nlimbs > kMaxLimbs) return MPDET_EINVAL;
    if (path != MPDET_PATH_AUTO && path != MPDET_PATH_VALU && path != MPDET_PATH_MFMA) return MPDET_EINVAL;
    if (path == MPDET_PATH_MFMA && !mpk::mfma_supported(nlimbs)) return MPDET_ENOTSUP;
    const bool use_mfma = path == MPDET_PATH_MFMA || (path == MPDET_PATH_AUTO && auto_uses_mfma(nlimbs));
    const int P = nlimbs;
    const int64_t m0 = n > 1 ? n - 1 : 1;
    mpdet_handle dflt{};  // the default panel setting when no handle is given
    size_t total = n > 0 ? recip_bytes(P) : 0;
    if (n > 1 && use_mfma)
        total += mfma_digit_bytes(m0, P) + up256(mfma_rec_bytes(h ? panel_rows(h, m0, P) : panel_rows(&dflt, m0, P),
                                                               m0, P));
    else if (n > 1 && mpk::lane_update_ok(P))
        total += up256(mfma_rec_bytes(m0, m0, P));
    *bytes = total;
    return MPDET_OK;
}

int mpdet_set_panel_rows(mpdet_handle *h, int64_t rows) {
    if (!h || rows < 0) return MPDET_EINVAL;
    h->panel_rows = rows;
    return MPDET_OK;
}

int mp_det_minors(mpdet_handle *h, mpdet_mat LU, mpdet_mat D, mpdet_mat c, int32_t *info_dev, void *stream) {
    if (!h || !info_dev) return MPDET_EINVAL;
    const int64_t n = LU.rows;
    if (n < 1 || !mat_ok(LU, true) || !mat_ok(D, true) || !mat_ok(c, true)) return MPDET_EINVAL;
    if (LU.cols != n || D.cols < n || c.cols < n || D.nlimbs != LU.nlimbs || c.nlimbs != LU.nlimbs)
        return MPDET_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    hipStream_t s = (hipStream_t)stream;
    const int P = LU.nlimbs;
    const size_t lds = mpk::lds_bytes(P);
    mpk::MatDev lu = dev(LU), d = dev(D), cv = dev(c);
    const int64_t total = n * (int64_t)P;
    hipLaunchKernelGGL(mpk::k_minors_init, grid_for((total + 255) / 256), dim3(256), 0, s, cv, n, P);
    int rc = last_launch();
    if (rc) return rc;
    for (int64_t j = n - 1; j >= 1; --j) {
        {
            Prof pr(h, s, K_MINORS_SWEEP);
            hipLaunchKernelGGL(mpk::k_minors_sweep, dim3((unsigned)j), dim3(64 * mpk::team_waves(P)), lds, s, lu, cv,
                               info_dev, j, n, P, wait_ticks(h));
        }
        rc = last_launch();
        if (rc) return rc;
    }
    {
        Prof pr(h, s, K_MINORS_FINAL);
        hipLaunchKernelGGL(mpk::k_minors_final, dim3((unsigned)n), dim3(64), lds, s, d, cv, info_dev, n, P);
    }
    return last_launch();
}

namespace {

enum BatchPhase { BP_PIVOT = 0, BP_DIVIDE, BP_UPD, BP_PREP, BP_SUB, BP_COUNT };

int grow_device(void **p, size_t *have, size_t need) {
    if (need <= *have) return MPDET_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
    if (hipMalloc(p, need) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return MPDET_ENOMEM;
    }
    *have = need;
    return MPDET_OK;
}

}  // namespace

}  // extern "C"

namespace {

// The persistent launch's schedule (kernels_persist.h): phase records of every
// matrix, ordered by (virtual time, phase slot, rank in the size order), each
// with the count of its matrix's tickets that must be complete before it runs;
// pre[r] = tickets before record r, pre[nrec] = all tickets.
struct PersistPlan {
    std::vector<mpk::PersistRec> recs;
    std::vector<int64_t> pre;
};

struct PlanKey {
    int64_t vt;
    int32_t slot, rank;
    mpk::PersistRec rec;
};

// order the records by (virtual time, phase slot, rank) and give each its
// matrix's count of earlier tickets; wg(kind): one ticket per unit
template <typename WgKind>
void persist_order(std::vector<PlanKey> &keys, size_t nmat, WgKind wg, PersistPlan *out) {
    std::sort(keys.begin(), keys.end(), [](const PlanKey &a, const PlanKey &b) {
        if (a.vt != b.vt) return a.vt < b.vt;
        if (a.slot != b.slot) return a.slot < b.slot;
        return a.rank < b.rank;
    });
    std::vector<int64_t> doneb(nmat, 0);
    out->recs.clear();
    out->pre.assign(1, 0);
    out->recs.reserve(keys.size());
    out->pre.reserve(keys.size() + 1);
    for (const PlanKey &kk : keys) {
        mpk::PersistRec r = kk.rec;
        const int64_t tk = wg(r.kind) ? r.units : (r.units + mpk::kPersistWaves - 1) / mpk::kPersistWaves;
        r.need = doneb[(size_t)r.mat];
        doneb[(size_t)r.mat] += tk;
        out->recs.push_back(r);
        out->pre.push_back(out->pre.back() + tk);
    }
}

// n[b]: sizes; order: matrices by size, largest first
void persist_plan(const std::vector<int64_t> &n, const std::vector<int32_t> &order, int P, bool lane,
                  bool lookahead, bool minors, PersistPlan *out) {
    using Key = PlanKey;
    std::vector<Key> keys;
    for (int32_t t = 0; t < (int32_t)order.size(); ++t) {
        const int32_t b = order[(size_t)t];
        const int64_t nb = n[(size_t)b];
        auto add = [&](int64_t vt, int32_t slot, int32_t kind, int64_t k, int64_t units) {
            if (units > 0) keys.push_back(Key{vt, slot, t, mpk::PersistRec{0, units, k, b, kind}});
        };
        add(0, 0, mpk::PK_INIT, 0, 1);
        for (int64_t k = 0; k < nb; ++k) {
            const int64_t m = nb - k - 1;
            if (!lookahead || k == 0) add(k, 1, mpk::PK_PIVOT, k, 2);
            if (m <= 0) continue;
            add(k, 2, mpk::PK_DIVIDE, k, m);
            if (lane) {
                add(k, 3, mpk::PK_PROD, k, mpk::lane_update_blocks(m));
                add(k, 4, mpk::PK_FINISH, k, mpk::finish_blocks(m, m, P));
            } else {
                add(k, 3, mpk::PK_UPDV, k, m * m);
            }
        }
        add(nb - 1, 5, mpk::PK_PEND, nb - 1, 1);
        if (minors) {
            for (int64_t sw = 0; sw + 2 <= nb; ++sw) add(nb + sw, 6, mpk::PK_MSWEEP, nb - 1 - sw, nb - 1 - sw);
            add(2 * nb - 1, 7, mpk::PK_MFINAL, 0, nb);
        }
    }
    persist_order(keys, n.size(), [](int kind) { return mpk::persist_wg_kind(kind); }, out);
}

// The backward's schedule: per matrix the phases of mp_det_adjugate in order
// (virtual times: W sweeps 1..n-1, S and the diagonal n, back substitution
// n+1..2n-1, accumulation 2n..3n-1)
void persist_plan_adj(const std::vector<int64_t> &n, const std::vector<int32_t> &order, int P, bool lane,
                      PersistPlan *out) {
    std::vector<PlanKey> keys;
    for (int32_t t = 0; t < (int32_t)order.size(); ++t) {
        const int32_t b = order[(size_t)t];
        const int64_t nb = n[(size_t)b];
        auto add = [&](int64_t vt, int32_t slot, int32_t kind, int64_t k, int64_t units) {
            if (units > 0) keys.push_back(PlanKey{vt, slot, t, mpk::PersistRec{0, units, k, b, kind}});
        };
        add(0, 0, mpk::AK_INIT, 0, nb);
        for (int64_t j = nb - 1; j >= 1; --j) {
            const int64_t vt = nb - j;
            if (lane) {
                add(vt, 1, mpk::AK_WPROD, j, mpk::lane_update_blocks(nb - j, j));
                add(vt, 2, mpk::AK_WFIN, j, mpk::finish_blocks(nb - j, j, P));
            } else {
                add(vt, 1, mpk::AK_WONE, j, (nb - j) * j);
            }
        }
        add(nb, 1, mpk::AK_S, 0, 1);
        add(nb, 2, mpk::AK_DIAGREC, 0, 2 * nb);
        for (int64_t k = nb - 1; k >= 1; --k) {
            const int64_t vt = nb + (nb - k);
            if (lane) {
                add(vt, 1, mpk::AK_UPROD, k, mpk::lane_update_blocks(k, nb - k));
                add(vt, 2, mpk::AK_UFIN, k, mpk::finish_blocks(k, nb - k, P));
            } else {
                add(vt, 1, mpk::AK_UONE, k, k * (nb - k));
            }
            add(vt, 3, mpk::AK_UDIV, k, nb - k);
        }
        for (int64_t k = 0; k < nb; ++k) {
            const int64_t vt = 2 * nb + k;
            if (lane) {
                add(vt, 1, mpk::AK_APROD, k, mpk::lane_update_blocks(k + 1, k + 1));
                add(vt, 2, mpk::AK_AFIN, k, mpk::finish_blocks(k + 1, k + 1, P));
            } else {
                add(vt, 1, mpk::AK_AONE, k, (k + 1) * (k + 1));
            }
        }
    }
    persist_order(keys, n.size(), [](int kind) { return mpk::adj_wg_kind(kind); }, out);
}

// LDS words of one wave's slice in the persistent kernel, and the workgroup's bytes
int64_t persist_lds_wave(int P, bool lane) {
    size_t b = mpk::pivot_lds_bytes(P);
    b = std::max(b, mpk::lds_bytes(P));
    if (lane) b = std::max(b, mpk::finish_launch_lds(P));
    return (int64_t)((b / 4 + 3) / 4 * 4);
}
size_t persist_lds_bytes(int P, bool lane) {
    const size_t waves = (size_t)mpk::kPersistWaves * (size_t)persist_lds_wave(P, lane) * 4u;
    return lane ? std::max(waves, mpk::lane_lds_bytes(P)) : waves;
}

// Device workspace of a persistent launch, in the handle's batch buffer:
// [descriptors | records | prefix] (staged from the pinned host buffer), then
// the per-matrix ticket counts and marks, the queue control word and the
// per-matrix scratch.
struct PersistStage {
    uint8_t *host_desc;  // pinned: the caller writes its descriptors here
    uint8_t *dev_desc;
    const mpk::PersistRec *recs;
    const int64_t *pre;
    int64_t *done;
    int32_t *skipped;
    mpk::PersistCtl *ctl;
    uint8_t *scratch;
    size_t desc_bytes, rec_bytes, pre_bytes;
};

int persist_alloc(mpdet_handle *h, size_t desc_raw, const PersistPlan &plan, int64_t batch, size_t scratch_bytes,
                  PersistStage *st) {
    const size_t nrec = plan.recs.size();
    st->desc_bytes = up256(desc_raw);
    st->rec_bytes = up256(sizeof(mpk::PersistRec) * nrec);
    st->pre_bytes = up256(sizeof(int64_t) * (nrec + 1));
    const size_t host_bytes = st->desc_bytes + st->rec_bytes + st->pre_bytes;
    const size_t done_bytes = up256(sizeof(int64_t) * (size_t)batch), skip_bytes = up256(sizeof(int32_t) * (size_t)batch);
    const size_t ctl_bytes = up256(sizeof(mpk::PersistCtl));
    int rc = grow_device(&h->bw, &h->bw_bytes, host_bytes + done_bytes + skip_bytes + ctl_bytes + scratch_bytes);
    if (rc) return rc;
    if (h->bh_pending) {  // the pinned buffer is still being copied from
        (void)hipEventSynchronize(h->bh_done);
        h->bh_pending = false;
    }
    if (host_bytes > h->bh_bytes) {
        if (h->bh) (void)hipHostFree(h->bh);
        h->bh = nullptr;
        h->bh_bytes = 0;
        if (hipHostMalloc(&h->bh, host_bytes, hipHostMallocDefault) != hipSuccess) {
            h->bh = nullptr;
            (void)hipGetLastError();
            return MPDET_ENOMEM;
        }
        h->bh_bytes = host_bytes;
    }
    if (!h->bh_done && hipEventCreateWithFlags(&h->bh_done, hipEventDisableTiming) != hipSuccess) return MPDET_EHIP;
    uint8_t *dev = (uint8_t *)h->bw;
    st->host_desc = (uint8_t *)h->bh;
    st->dev_desc = dev;
    st->recs = (const mpk::PersistRec *)(dev + st->desc_bytes);
    st->pre = (const int64_t *)(dev + st->desc_bytes + st->rec_bytes);
    st->done = (int64_t *)(dev + host_bytes);
    st->skipped = (int32_t *)(dev + host_bytes + done_bytes);
    st->ctl = (mpk::PersistCtl *)(dev + host_bytes + done_bytes + skip_bytes);
    st->scratch = dev + host_bytes + done_bytes + skip_bytes + ctl_bytes;
    return MPDET_OK;
}

// copy the descriptors (already in the pinned buffer), records and prefix to the device
int persist_upload(mpdet_handle *h, const PersistPlan &plan, PersistStage *st, hipStream_t s) {
    uint8_t *hst = st->host_desc;
    memcpy(hst + st->desc_bytes, plan.recs.data(), sizeof(mpk::PersistRec) * plan.recs.size());
    memcpy(hst + st->desc_bytes + st->rec_bytes, plan.pre.data(), sizeof(int64_t) * plan.pre.size());
    const size_t host_bytes = st->desc_bytes + st->rec_bytes + st->pre_bytes;
    if (hipMemcpyAsync(st->dev_desc, hst, host_bytes, hipMemcpyHostToDevice, s) != hipSuccess) return MPDET_EHIP;
    if (hipEventRecord(h->bh_done, s) != hipSuccess) return MPDET_EHIP;
    h->bh_pending = true;
    return MPDET_OK;
}

// grid: every workgroup that fits on the device at once (at most one per
// ticket); limit: the wait bound in wall-clock ticks
int persist_shape(mpdet_handle *h, const void *kernel, size_t lds, int64_t tickets, int64_t *grid, uint64_t *limit) {
    if (lds > 64u * 1024u &&
        hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return MPDET_EHIP;
    int per_cu = 0, cus = 0, khz = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64 * mpk::kPersistWaves, lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device) != hipSuccess)
        return MPDET_EHIP;
    if (per_cu < 1 || cus < 1 || khz < 1) return MPDET_ENOTSUP;
    *grid = std::max<int64_t>(1, std::min<int64_t>(tickets, (int64_t)per_cu * cus));
    const double lim_s = h->wait_limit_set ? h->wait_limit_s : 10.0;
    *limit = (uint64_t)(lim_s * (double)khz * 1000.0);
    return MPDET_OK;
}

}  // namespace

extern "C" {

int mpdet_set_overlap(mpdet_handle *h, int32_t panels) {
    if (!h || panels < 0 || panels > 64) return MPDET_EINVAL;
    h->overlap_panels = panels;
    return MPDET_OK;
}

int mpdet_set_tuning(mpdet_handle *h, int32_t lane_rows, int32_t mfma_waves) {
    if (!h) return MPDET_EINVAL;
    if (lane_rows != 0 && lane_rows != 2 && lane_rows != 4 && lane_rows != 8) return MPDET_EINVAL;
    if (mfma_waves != 0 && mfma_waves != 1 && mfma_waves != 2 && mfma_waves != 4) return MPDET_EINVAL;
    h->lane_rows = lane_rows;
    h->mfma_waves = mfma_waves;
    return MPDET_OK;
}

int mpdet_set_long_division(mpdet_handle *h, int32_t on) {
    if (!h || (on != 0 && on != 1)) return MPDET_EINVAL;
    h->long_div = on;
    return MPDET_OK;
}

int mpdet_set_wait_limit(mpdet_handle *h, double seconds) {
    if (!h || !(seconds >= 0.0) || seconds > 3600.0) return MPDET_EINVAL;
    h->wait_limit_s = seconds;
    h->wait_limit_set = true;
    return MPDET_OK;
}

int mpdet_batched_plan(int64_t batch, const int64_t *n_host, int32_t nlimbs, int path, int flags, void *recs_out,
                       int64_t cap, int64_t *nrec, int64_t *ntickets) {
    if (batch < 0 || (batch > 0 && !n_host) || !nrec || !ntickets || nlimbs < 2 || nlimbs > kMaxLimbs)
        return MPDET_EINVAL;
    if (path != MPDET_PATH_AUTO && path != MPDET_PATH_VALU && path != MPDET_PATH_MFMA) return MPDET_EINVAL;
    if (path == MPDET_PATH_MFMA || (path == MPDET_PATH_AUTO && auto_uses_mfma(nlimbs))) return MPDET_ENOTSUP;
    std::vector<int64_t> n((size_t)batch);
    for (int64_t b = 0; b < batch; ++b) {
        if (n_host[b] < 1) return MPDET_EINVAL;
        n[(size_t)b] = n_host[b];
    }
    std::vector<int32_t> order((size_t)batch);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return n[(size_t)a] > n[(size_t)b]; });
    const bool lane = mpk::lane_update_ok(nlimbs);
    PersistPlan plan;
    persist_plan(n, order, nlimbs, lane, lane && mpk::finish_lookahead_ok(nlimbs), (flags & MPDET_WANT_MINORS) != 0,
                 &plan);
    *nrec = (int64_t)plan.recs.size();
    *ntickets = plan.pre.back();
    if (recs_out) {
        if (cap < *nrec) return MPDET_EINVAL;
        memcpy(recs_out, plan.recs.data(), plan.recs.size() * sizeof(mpk::PersistRec));
    }
    return MPDET_OK;
}

int mp_det_batched(mpdet_handle *h, int64_t batch, const mpdet_mat *A_arr, const mpdet_mat *D_arr,
                   const mpdet_mat *c_arr, int32_t *info_dev, int flags, int path, void *stream) {
    if (!h || batch < 0) return MPDET_EINVAL;
    if (batch == 0) return MPDET_OK;
    if (!A_arr || !D_arr || !info_dev) return MPDET_EINVAL;
    if (flags & ~(MPDET_WANT_MINORS | MPDET_BATCH_LOCKSTEP | MPDET_BATCH_PERSISTENT)) return MPDET_EINVAL;
    if ((flags & MPDET_BATCH_LOCKSTEP) && (flags & MPDET_BATCH_PERSISTENT)) return MPDET_EINVAL;
    const bool minors = (flags & MPDET_WANT_MINORS) != 0;
    if (minors && !c_arr) return MPDET_EINVAL;
    if (path != MPDET_PATH_AUTO && path != MPDET_PATH_VALU && path != MPDET_PATH_MFMA) return MPDET_EINVAL;
    const int P = A_arr[0].nlimbs;
    int64_t nmax = 0;
    for (int64_t b = 0; b < batch; ++b) {
        const mpdet_mat &A = A_arr[b], &D = D_arr[b];
        const int64_t n = A.rows;
        if (n < 1 || A.cols != n || !mat_ok(A, true) || !mat_ok(D, true) || A.nlimbs != P || D.nlimbs != P ||
            D.cols < n)
            return MPDET_EINVAL;
        if (minors && (!mat_ok(c_arr[b], true) || c_arr[b].nlimbs != P || c_arr[b].cols < n))
            return MPDET_EINVAL;
        nmax = n > nmax ? n : nmax;
    }
    const bool mfma_ok = mpk::mfma_supported(P);
    if (path == MPDET_PATH_MFMA && !mfma_ok) return MPDET_ENOTSUP;
    const bool use_mfma = path == MPDET_PATH_MFMA || (path == MPDET_PATH_AUTO && auto_uses_mfma(P));
    const bool lane_valu = !use_mfma && mpk::lane_update_ok(P);
    const int lrows = lane_rows_of(h), mw = mfma_waves_of(h);
    if (use_mfma && mpk::mfma_copies(P, mw) == 0) return MPDET_ENOTSUP;
    if (use_mfma && (flags & MPDET_BATCH_PERSISTENT)) return MPDET_ENOTSUP;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    hipStream_t s = (hipStream_t)stream;

    // largest first: the matrices active at step k are a prefix of `order`
    std::vector<int32_t> order((size_t)batch);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return A_arr[a].rows > A_arr[b].rows; });
    // the persistent schedule on request (measured slower than lockstep on
    // config 4's forward: 1.25 s against 0.57 s)
    const bool persistent = !use_mfma && (flags & MPDET_BATCH_PERSISTENT);
    if (persistent) {
        // one persistent launch over the whole schedule (kernels_persist.h)
        const bool lookahead = lane_valu && mpk::finish_lookahead_ok(P);
        std::vector<int64_t> nv((size_t)batch);
        for (int64_t b = 0; b < batch; ++b) nv[(size_t)b] = A_arr[b].rows;
        PersistPlan plan;
        persist_plan(nv, order, P, lane_valu, lookahead, minors, &plan);
        std::vector<size_t> scratch((size_t)batch);
        size_t total_scratch = 0;
        for (int64_t b = 0; b < batch; ++b) {
            const int64_t n = A_arr[b].rows, m = n > 1 ? n - 1 : 1;
            scratch[(size_t)b] = recip_bytes(P) + (lane_valu ? up256(mfma_rec_bytes(m, m, P)) : 0);
            total_scratch += scratch[(size_t)b];
        }
        PersistStage st;
        int rc = persist_alloc(h, sizeof(mpk::BatchMat) * (size_t)batch, plan, batch, total_scratch, &st);
        if (rc) return rc;
        mpk::BatchMat *hm = (mpk::BatchMat *)st.host_desc;
        uint8_t *sp = st.scratch;
        for (int64_t b = 0; b < batch; ++b) {
            mpk::BatchMat &M = hm[b];
            M.A = dev_mat(A_arr[b]);
            M.D = dev_mat(D_arr[b]);
            M.c = minors ? dev_mat(c_arr[b]) : mpk::MatDev{nullptr, nullptr, nullptr, 0};
            M.info = info_dev + b;
            M.n = A_arr[b].rows;
            M.rw = (uint32_t *)sp;
            M.Lr = M.Ub = nullptr;
            M.T = lane_valu ? (uint32_t *)(sp + recip_bytes(P)) : nullptr;
            sp += scratch[(size_t)b];
        }
        const size_t lds = persist_lds_bytes(P, lane_valu);
        int64_t grid = 0;
        uint64_t limit = 0;
        if ((rc = persist_upload(h, plan, &st, s)) ||
            (rc = persist_shape(h, (const void *)mpk::k_persist, lds, plan.pre.back(), &grid, &limit)))
            return rc;
        const unsigned bb = (unsigned)((batch + 255) / 256);
        hipLaunchKernelGGL(mpk::k_persist_begin, dim3(bb), dim3(256), 0, s, st.ctl, st.done, st.skipped, batch);
        if ((rc = last_launch())) return rc;
        const mpk::BatchMat *dmats = (const mpk::BatchMat *)st.dev_desc;
        {
            Prof pr(h, s, K_BATCH_PERSIST);
            hipLaunchKernelGGL(mpk::k_persist, dim3((unsigned)grid), dim3(64 * mpk::kPersistWaves), lds, s, dmats,
                               st.recs, st.pre, (int64_t)plan.recs.size(), st.done, st.skipped, st.ctl, P,
                               lookahead ? 1 : 0, minors ? 1 : 0, persist_lds_wave(P, lane_valu), limit);
        }
        if ((rc = last_launch())) return rc;
        hipLaunchKernelGGL(mpk::k_persist_end, dim3(bb), dim3(256), 0, s, dmats, (const int32_t *)st.skipped, batch);
        return last_launch();
    }
    auto nof = [&](int t) { return A_arr[order[(size_t)t]].rows; };

    // block counts per (step, phase) -> prefix offsets, all in one table
    auto blocks = [&](int phase, int64_t n, int64_t k) -> int64_t {
        const int64_t m = n - k - 1;
        switch (phase) {
            case BP_PIVOT: return 2;
            case BP_DIVIDE: return m;
            case BP_UPD:
                if (use_mfma) return (mpk::mfma_update_blocks(m, m, mw) + 7) / 8 * 8;
                return lane_valu ? mpk::lane_update_blocks(m, m, lrows) : m * m;
            case BP_PREP: return 2 * m;
            case BP_SUB: return mpk::finish_blocks(m, m, P);
        }
        return 0;
    };
    std::vector<int64_t> table;
    std::vector<int64_t> start((size_t)(nmax * BP_COUNT + nmax + 2), -1);
    std::vector<int32_t> count((size_t)(nmax * BP_COUNT + nmax + 2), 0);
    int cnt = (int)batch;
    for (int64_t k = 0; k < nmax; ++k) {
        while (cnt > 0 && nof(cnt - 1) <= k) --cnt;
        for (int ph = 0; ph < BP_COUNT; ++ph) {
            const size_t slot = (size_t)(k * BP_COUNT + ph);
            start[slot] = (int64_t)table.size();
            count[slot] = cnt;
            int64_t acc = 0;
            table.push_back(0);
            for (int t = 0; t < cnt; ++t) {
                acc += blocks(ph, nof(t), k);
                table.push_back(acc);
            }
        }
    }
    // minors: sweep s (active: n >= s + 2), then final and init (all)
    const size_t mbase = (size_t)(nmax * BP_COUNT);
    if (minors) {
        for (int64_t sw = 0; sw + 2 <= nmax; ++sw) {
            int c2 = 0;
            while (c2 < (int)batch && nof(c2) >= sw + 2) ++c2;
            start[mbase + (size_t)sw] = (int64_t)table.size();
            count[mbase + (size_t)sw] = c2;
            int64_t acc = 0;
            table.push_back(0);
            for (int t = 0; t < c2; ++t) {
                acc += nof(t) - 1 - sw;
                table.push_back(acc);
            }
        }
        for (int which = 0; which < 2; ++which) {  // 0: final (n blocks), 1: init
            const size_t slot = mbase + (size_t)nmax + (size_t)which;
            start[slot] = (int64_t)table.size();
            count[slot] = (int)batch;
            int64_t acc = 0;
            table.push_back(0);
            for (int t = 0; t < (int)batch; ++t) {
                acc += which == 0 ? nof(t) : (nof(t) * P + 255) / 256;
                table.push_back(acc);
            }
        }
    }

    // device workspace: descriptors, order, table, then per-matrix scratch
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const mpk::MfmaGeom geo = mpk::mfma_geom(P);
    std::vector<size_t> scratch((size_t)batch);
    size_t total_scratch = 0;
    for (int64_t b = 0; b < batch; ++b) {
        const int64_t n = A_arr[b].rows, m = n > 1 ? n - 1 : 1;
        size_t need = up((size_t)(P + 3) * 4u);
        if (use_mfma)
            need += up((size_t)m * geo.LR) + up(mpk::ub_bytes(m, P)) + up(mfma_rec_bytes(m, m, P));
        else if (lane_valu)
            need += up(mfma_rec_bytes(m, m, P));
        scratch[(size_t)b] = need;
        total_scratch += need;
    }
    const size_t desc_bytes = up(sizeof(mpk::BatchMat) * (size_t)batch);
    const size_t order_bytes = up(sizeof(int32_t) * (size_t)batch);
    const size_t table_bytes = up(sizeof(int64_t) * table.size());
    const size_t host_bytes = desc_bytes + order_bytes + table_bytes;
    int rc = grow_device(&h->bw, &h->bw_bytes, host_bytes + total_scratch);
    if (rc) return rc;
    if (h->bh_pending) {
        (void)hipEventSynchronize(h->bh_done);
        h->bh_pending = false;
    }
    if (host_bytes > h->bh_bytes) {
        if (h->bh) (void)hipHostFree(h->bh);
        h->bh = nullptr;
        h->bh_bytes = 0;
        if (hipHostMalloc(&h->bh, host_bytes, hipHostMallocDefault) != hipSuccess) {
            h->bh = nullptr;
            (void)hipGetLastError();
            return MPDET_ENOMEM;
        }
        h->bh_bytes = host_bytes;
    }
    if (!h->bh_done && hipEventCreateWithFlags(&h->bh_done, hipEventDisableTiming) != hipSuccess) return MPDET_EHIP;
    uint8_t *dev = (uint8_t *)h->bw;
    uint8_t *hst = (uint8_t *)h->bh;
    mpk::BatchMat *hm = (mpk::BatchMat *)hst;
    uint8_t *sp = dev + host_bytes;
    for (int64_t b = 0; b < batch; ++b) {
        const int64_t n = A_arr[b].rows, m = n > 1 ? n - 1 : 1;
        mpk::BatchMat &M = hm[b];
        M.A = dev_mat(A_arr[b]);
        M.D = dev_mat(D_arr[b]);
        M.c = minors ? dev_mat(c_arr[b]) : mpk::MatDev{nullptr, nullptr, nullptr, 0};
        M.info = info_dev + b;
        M.n = n;
        uint8_t *q = sp;
        M.rw = (uint32_t *)q;
        q += up((size_t)(P + 3) * 4u);
        M.Lr = M.Ub = nullptr;
        M.T = nullptr;
        if (use_mfma) {
            M.Lr = q;
            q += up((size_t)m * geo.LR);
            M.Ub = q;
            q += up(mpk::ub_bytes(m, P));
            M.T = (uint32_t *)q;
        } else if (lane_valu) {
            M.T = (uint32_t *)q;
        }
        sp += scratch[(size_t)b];
    }
    memcpy(hst + desc_bytes, order.data(), sizeof(int32_t) * order.size());
    memcpy(hst + desc_bytes + order_bytes, table.data(), sizeof(int64_t) * table.size());
    if (hipMemcpyAsync(dev, hst, host_bytes, hipMemcpyHostToDevice, s) != hipSuccess) return MPDET_EHIP;
    if (hipEventRecord(h->bh_done, s) != hipSuccess) return MPDET_EHIP;
    h->bh_pending = true;
    const mpk::BatchMat *dmats = (const mpk::BatchMat *)dev;
    const int32_t *dorder = (const int32_t *)(dev + desc_bytes);
    const int64_t *dtable = (const int64_t *)(dev + desc_bytes + order_bytes);

    hipLaunchKernelGGL(mpk::k_batch_zero_info, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, info_dev,
                       batch);
    if ((rc = last_launch())) return rc;
    const size_t lds_piv = mpk::pivot_lds_bytes(P), lds = mpk::lds_bytes(P);
    const size_t lds_mfma = mpk::mfma_lds_bytes(P, mw), lds_prep = (size_t)(P + 1) * 4;
    const size_t lds_fin = mpk::finish_launch_lds(P);
    auto bfin_kernel = mpk::finish_streams(P) ? mpk::k_batch_finish<true> : mpk::k_batch_finish<false>;
    auto bupd_kernel = batch_mfma_kernel(mpk::mfma_copies(P, mw), mw);
    // with the finish kernel, step k's pivot is examined by step k-1's finish launch
    const bool lookahead = (use_mfma || lane_valu) && mpk::finish_lookahead_ok(P);
    hipLaunchKernelGGL(mpk::k_batch_pend, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, dmats, batch, P, 0);
    if ((rc = last_launch())) return rc;
    auto launch = [&](int kernel_id, auto kern, size_t slot, size_t shmem, int64_t arg, int threads = 64) -> int {
        const int c = count[slot];
        if (c <= 0) return MPDET_OK;
        const int64_t total = table[(size_t)start[slot] + (size_t)c];
        if (total <= 0) return MPDET_OK;
        Prof pr(h, s, kernel_id);
        hipLaunchKernelGGL(kern, grid_for(total), dim3(threads), shmem, s, dmats, dorder, dtable + start[slot], c,
                           arg, P);
        return last_launch();
    };
    for (int64_t k = 0; k < nmax; ++k) {
        const size_t base = (size_t)(k * BP_COUNT);
        if (!(lookahead && k > 0) && (rc = launch(K_PIVOT_DIVIDE, mpk::k_batch_pivot, base + BP_PIVOT, lds_piv, k)))
            return rc;
        if ((rc = launch(K_DIVIDE, mpk::k_batch_divide, base + BP_DIVIDE, lds_piv, k))) return rc;
        if (use_mfma) {
            if ((rc = launch(K_MFMA_PREP, mpk::k_batch_prep, base + BP_PREP, lds_prep, k))) return rc;
            if ((rc = launch(K_UPDATE_MFMA, bupd_kernel, base + BP_UPD, lds_mfma, k,
                             64 * mw)))
                return rc;
            if ((rc = launch(K_UPDATE_FINISH, bfin_kernel, base + BP_SUB, lds_fin, k))) return rc;
        } else {
            if (lane_valu) {
                if ((rc = launch(K_UPDATE_VALU, batch_lane_kernel(lrows), base + BP_UPD, mpk::lane_lds_bytes(P, lrows),
                                 k, 64 * lrows)))
                    return rc;
                if ((rc = launch(K_UPDATE_FINISH, bfin_kernel, base + BP_SUB, lds_fin, k))) return rc;
            } else if ((rc = launch(K_UPDATE_VALU, mpk::k_batch_update_valu, base + BP_UPD, lds, k))) {
                return rc;
            }
        }
    }
    hipLaunchKernelGGL(mpk::k_batch_pend, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, dmats, batch, P, 1);
    if ((rc = last_launch())) return rc;
    if (minors) {
        const size_t islot = mbase + (size_t)nmax + 1;
        const int64_t itotal = table[(size_t)start[islot] + (size_t)count[islot]];
        hipLaunchKernelGGL(mpk::k_batch_minit, grid_for(itotal), dim3(256), 0, s, dmats, dorder,
                           dtable + start[islot], count[islot], P);
        if ((rc = last_launch())) return rc;
        for (int64_t sw = 0; sw + 2 <= nmax; ++sw)
            if ((rc = launch(K_MINORS_SWEEP, mpk::k_batch_msweep, mbase + (size_t)sw, lds, sw))) return rc;
        if ((rc = launch(K_MINORS_FINAL, mpk::k_batch_mfinal, mbase + (size_t)nmax, lds, 0))) return rc;
    }
    return MPDET_OK;
}

// Row sweeps of W = L^-1, j = n-1..1: W_ri <- RZ(W_ri - RZ(W_rj l_ji)) for
// every row r >= j and column i < j.  Sweep j is a rank-1 update of the
// (n - j) x j block of W at (j, 0), x the column j of W and y the row j of
// L, so where the lane product applies it runs on the lane product and the
// tile finish (the factorisation's record workspace holds its records);
// otherwise one wave per multiply-subtract (k_adj_w).  Either way every
// element sees the same operations in the same order.
static int w_sweeps(mpdet_handle *h, mpk::MatDev lu, mpk::MatDev W, const int32_t *info, int64_t n, int P,
             hipStream_t s) {
    int rc;
    if (mpk::lane_update_ok(P) && n > 1) {
        MfmaWs w{};
        if ((rc = mfma_workspace(h, n, P, n, &w))) return rc;
        for (int64_t j = n - 1; j >= 1; --j) {
            // x_r = W[r][j] (r >= j), y_i = l_ji (i < j), z = W[r][i]
            const mpk::Rank1 R{W, lu, W, j, j, 1, 0, j, 0, 0, 1, j, 0, n - j, j, 0};
            if ((rc = lane_rank1(h, R, w.T, info, P, s))) return rc;
        }
        return MPDET_OK;
    }
    const size_t lds = mpk::pivot_lds_bytes(P);
    for (int64_t j = n - 1; j >= 1; --j) {
        hipLaunchKernelGGL(mpk::k_adj_w, grid_for((n - j) * j), dim3(64), lds, s, lu, W, info, j, n, P);
        if ((rc = last_launch())) return rc;
    }
    return MPDET_OK;
}

int mp_det_all_minors(mpdet_handle *h, mpdet_mat LU, mpdet_mat D, mpdet_mat C, const int32_t *info_dev,
                      void *stream) {
    if (!h || !info_dev) return MPDET_EINVAL;
    const int64_t n = LU.rows;
    if (n < 1 || !mat_ok(LU, true) || !mat_ok(D, true) || !mat_ok(C, true)) return MPDET_EINVAL;
    if (LU.cols != n || D.cols < n || C.rows != n || C.cols != n || D.nlimbs != LU.nlimbs ||
        C.nlimbs != LU.nlimbs)
        return MPDET_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    hipStream_t s = (hipStream_t)stream;
    const int P = LU.nlimbs;
    // workspace: W (n x n), in the adjugate's buffer
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t nn = (size_t)n * (size_t)n;
    const size_t ml = up(nn * (size_t)P * 4u), me = up(nn * 8u), ms = up(nn * 4u);
    const size_t need = ml + me + ms + 256;  // + the factors gate
    if (need > h->aw_bytes) {
        if (h->aw) (void)hipFree(h->aw);
        h->aw = nullptr;
        h->aw_bytes = 0;
        if (hipMalloc(&h->aw, need) != hipSuccess) {
            h->aw = nullptr;
            (void)hipGetLastError();
            return MPDET_ENOMEM;
        }
        h->aw_bytes = need;
    }
    uint8_t *base = (uint8_t *)h->aw;
    mpk::MatDev W{(uint32_t *)base, (int64_t *)(base + ml), (int32_t *)(base + ml + me), n};
    int32_t *gate = (int32_t *)(base + ml + me + ms);
    mpk::MatDev lu = dev(LU), d = dev(D), cm = dev(C);
    const size_t lds = mpk::pivot_lds_bytes(P);
    int rc;
    hipLaunchKernelGGL(mpk::k_factors_gate, dim3(1), dim3(64), 0, s, info_dev, n, gate);
    hipLaunchKernelGGL(mpk::k_adj_init, grid_for(((int64_t)nn + 255) / 256), dim3(256), 0, s, W, n, P, 1);
    if ((rc = last_launch())) return rc;
    {
        Prof pr(h, s, K_ALL_MINORS);
        if ((rc = w_sweeps(h, lu, W, gate, n, P, s))) return rc;
        hipLaunchKernelGGL(mpk::k_all_minors_final, grid_for((int64_t)nn), dim3(64), lds, s, d, W, cm, gate, n, P);
    }
    return last_launch();
}

int mp_det_normalize_minors(mpdet_handle *h, mpdet_mat C, mpdet_mat out, void *stream) {
    if (!h) return MPDET_EINVAL;
    const int64_t cnt = C.rows * C.cols;
    if (!mat_ok(C, cnt > 0) || !mat_ok(out, cnt > 0)) return MPDET_EINVAL;
    if (out.rows != C.rows || out.cols != C.cols || out.nlimbs != C.nlimbs) return MPDET_EINVAL;
    if (cnt == 0) return MPDET_OK;
    if (mats_overlap(C, out)) return MPDET_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    const int P = C.nlimbs;
    hipLaunchKernelGGL(mpk::k_norm_minors, grid_for(cnt), dim3(64), mpk::pivot_lds_bytes(P), (hipStream_t)stream,
                       dev(C), dev(out), C.rows, C.cols, P);
    return last_launch();
}

int mp_det_adjugate(mpdet_handle *h, mpdet_mat LU, mpdet_mat D, mpdet_mat adjT, const int32_t *info_dev,
                    void *stream) {
    if (!h || !info_dev) return MPDET_EINVAL;
    const int64_t n = LU.rows;
    if (n < 1 || !mat_ok(LU, true) || !mat_ok(D, true) || !mat_ok(adjT, true)) return MPDET_EINVAL;
    if (LU.cols != n || D.cols < n || adjT.rows != n || adjT.cols != n || D.nlimbs != LU.nlimbs ||
        adjT.nlimbs != LU.nlimbs)
        return MPDET_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    hipStream_t s = (hipStream_t)stream;
    const int P = LU.nlimbs;
    // workspace: W, adj(U) (n x n each), S (n + 1), reciprocals (n x (P + 2))
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t nn = (size_t)n * (size_t)n;
    const size_t ml = up(nn * (size_t)P * 4u), me = up(nn * 8u), ms = up(nn * 4u);
    const size_t sl = up((size_t)(n + 1) * P * 4u), se = up((size_t)(n + 1) * 8u), ss = up((size_t)(n + 1) * 4u);
    const size_t rb = up((size_t)n * (P + 2) * 4u);
    const size_t need = 2 * (ml + me + ms) + sl + se + ss + rb + 256;  // + the factors gate
    if (need > h->aw_bytes) {
        if (h->aw) (void)hipFree(h->aw);
        h->aw = nullptr;
        h->aw_bytes = 0;
        if (hipMalloc(&h->aw, need) != hipSuccess) {
            h->aw = nullptr;
            (void)hipGetLastError();
            return MPDET_ENOMEM;
        }
        h->aw_bytes = need;
    }
    uint8_t *base = (uint8_t *)h->aw;
    auto carve = [&](size_t bytes) {
        uint8_t *p = base;
        base += bytes;
        return p;
    };
    mpk::MatDev W{(uint32_t *)carve(ml), (int64_t *)carve(me), (int32_t *)carve(ms), n};
    mpk::MatDev J{(uint32_t *)carve(ml), (int64_t *)carve(me), (int32_t *)carve(ms), n};
    mpk::MatDev S{(uint32_t *)carve(sl), (int64_t *)carve(se), (int32_t *)carve(ss), n + 1};
    uint32_t *rw = (uint32_t *)carve(rb);
    int32_t *gate = (int32_t *)carve(256);
    mpk::MatDev lu = dev(LU), d = dev(D), t = dev(adjT);
    const size_t lds = mpk::pivot_lds_bytes(P);
    int rc;
    const int64_t cells = (int64_t)nn;
    hipLaunchKernelGGL(mpk::k_factors_gate, dim3(1), dim3(64), 0, s, info_dev, n, gate);
    hipLaunchKernelGGL(mpk::k_adj_init, grid_for((cells + 255) / 256), dim3(256), 0, s, W, n, P, 1);
    hipLaunchKernelGGL(mpk::k_adj_init, grid_for((cells + 255) / 256), dim3(256), 0, s, J, n, P, 0);
    hipLaunchKernelGGL(mpk::k_adj_init, grid_for((cells + 255) / 256), dim3(256), 0, s, t, n, P, 0);
    if ((rc = last_launch())) return rc;
    {
        Prof pr(h, s, K_ADJUGATE);
        if ((rc = w_sweeps(h, lu, W, gate, n, P, s))) return rc;
        hipLaunchKernelGGL(mpk::k_adj_s, dim3(1), dim3(64), lds, s, lu, S, gate, n, P);
        hipLaunchKernelGGL(mpk::k_adj_diag, dim3((unsigned)n), dim3(64), lds, s, d, S, J, gate, n, P);
        hipLaunchKernelGGL(mpk::k_adj_recips, dim3((unsigned)n), dim3(64), lds, s, lu, rw, gate, n, P);
        if ((rc = last_launch())) return rc;
        // Where the lane product applies, the back substitution's updates and
        // the accumulation are rank-1 updates on the lane product and the
        // tile finish (the same operation on every element, in the same
        // order, as k_adj_u_upd and k_adj_prod)
        const bool lane = mpk::lane_update_ok(P);
        MfmaWs ws{};
        if (lane && (rc = mfma_workspace(h, n, P, n, &ws))) return rc;
        auto rank1 = [&](const mpk::Rank1 &R) { (void)lane_rank1(h, R, ws.T, gate, P, s); };
        for (int64_t k = n - 1; k >= 1; --k) {
            if (lane)  // x_i = u_ik (i < k), y_j = J_kj (j >= k), z = J_ij
                rank1(mpk::Rank1{lu, J, J, 0, k, 1, 0, k, k, 0, 1, 0, k, k, n - k, 0});
            else
                hipLaunchKernelGGL(mpk::k_adj_u_upd, grid_for(k * (n - k)), dim3(64), lds, s, lu, J, gate, k, n,
                                   P);
            hipLaunchKernelGGL(mpk::k_adj_u_div, dim3((unsigned)(n - k)), dim3(64), lds, s, lu, J,
                               (const uint32_t *)rw, gate, k, n, P);
            if ((rc = last_launch())) return rc;
        }
        for (int64_t k = 0; k < n; ++k) {
            if (lane)  // x_m = W_km, y_i = J_ik (negated: an addition), z = adjT_mi (m, i <= k)
                rank1(mpk::Rank1{W, J, t, k, 0, 0, 1, 0, k, 1, 0, 0, 0, k + 1, k + 1, 1});
            else
                hipLaunchKernelGGL(mpk::k_adj_prod, grid_for((k + 1) * (k + 1)), dim3(64), lds, s, J, W, t,
                                   gate, k, P);
            if ((rc = last_launch())) return rc;
        }
    }
    return MPDET_OK;
}

}  // extern "C"

namespace {
// status[b] of the batched backward when it runs one call per matrix
__global__ void k_adj_status(const int32_t *info, const int64_t *n, int32_t *status, int64_t batch) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < batch) status[b] = mpk::factors_complete(info[b], n[b]) ? 0 : info[b];
}
}  // namespace

extern "C" {

int mp_det_adjugate_batched(mpdet_handle *h, int64_t batch, const mpdet_mat *LU_arr, const mpdet_mat *D_arr,
                            const mpdet_mat *adjT_arr, const int32_t *info_dev, int32_t *status_dev, int flags,
                            void *stream) {
    if (!h || batch < 0) return MPDET_EINVAL;
    if (batch == 0) return MPDET_OK;
    if (!LU_arr || !D_arr || !adjT_arr || !info_dev) return MPDET_EINVAL;
    if (flags & ~MPDET_BATCH_LOCKSTEP) return MPDET_EINVAL;
    const int P = LU_arr[0].nlimbs;
    for (int64_t b = 0; b < batch; ++b) {
        const mpdet_mat &LU = LU_arr[b], &D = D_arr[b], &T = adjT_arr[b];
        const int64_t n = LU.rows;
        if (n < 1 || LU.cols != n || !mat_ok(LU, true) || !mat_ok(D, true) || !mat_ok(T, true) || LU.nlimbs != P ||
            D.nlimbs != P || T.nlimbs != P || D.cols < n || T.rows != n || T.cols != n)
            return MPDET_EINVAL;
    }
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if (flags & MPDET_BATCH_LOCKSTEP) {  // one mp_det_adjugate call per matrix
        for (int64_t b = 0; b < batch; ++b)
            if ((rc = mp_det_adjugate(h, LU_arr[b], D_arr[b], adjT_arr[b], info_dev + b, stream))) return rc;
        if (!status_dev) return MPDET_OK;
        int64_t *nd = nullptr;
        std::vector<int64_t> nv((size_t)batch);
        for (int64_t b = 0; b < batch; ++b) nv[(size_t)b] = LU_arr[b].rows;
        if ((rc = grow_device(&h->bw, &h->bw_bytes, sizeof(int64_t) * (size_t)batch))) return rc;
        nd = (int64_t *)h->bw;
        if (hipMemcpyAsync(nd, nv.data(), sizeof(int64_t) * (size_t)batch, hipMemcpyHostToDevice, s) != hipSuccess)
            return MPDET_EHIP;
        hipLaunchKernelGGL(k_adj_status, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, info_dev, nd,
                           status_dev, batch);
        rc = last_launch();
        if (rc == MPDET_OK && hipStreamSynchronize(s) != hipSuccess) rc = MPDET_EHIP;  // nv is a host vector
        return rc;
    }
    // one persistent launch over every matrix's phases (kernels_persist.h)
    const bool lane = mpk::lane_update_ok(P);
    std::vector<int32_t> order((size_t)batch);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return LU_arr[a].rows > LU_arr[b].rows; });
    std::vector<int64_t> nv((size_t)batch);
    for (int64_t b = 0; b < batch; ++b) nv[(size_t)b] = LU_arr[b].rows;
    PersistPlan plan;
    persist_plan_adj(nv, order, P, lane, &plan);
    // per matrix: W and J (n x n each), S (n + 1), reciprocals (n x (P + 2)), gate, records
    auto sizes = [&](int64_t n, size_t *ml, size_t *me, size_t *ms, size_t *sl, size_t *se, size_t *ss, size_t *rb,
                     size_t *tb) {
        const size_t nn = (size_t)n * (size_t)n;
        *ml = up256(nn * (size_t)P * 4u);
        *me = up256(nn * 8u);
        *ms = up256(nn * 4u);
        *sl = up256((size_t)(n + 1) * P * 4u);
        *se = up256((size_t)(n + 1) * 8u);
        *ss = up256((size_t)(n + 1) * 4u);
        *rb = up256((size_t)n * (P + 2) * 4u);
        *tb = lane ? up256(mfma_rec_bytes(n, n, P)) : 0;
        return 2 * (*ml + *me + *ms) + *sl + *se + *ss + *rb + 256 + *tb;
    };
    std::vector<size_t> scratch((size_t)batch);
    size_t total_scratch = 0;
    for (int64_t b = 0; b < batch; ++b) {
        size_t a[8];
        scratch[(size_t)b] = sizes(nv[(size_t)b], &a[0], &a[1], &a[2], &a[3], &a[4], &a[5], &a[6], &a[7]);
        total_scratch += scratch[(size_t)b];
    }
    PersistStage st;
    if ((rc = persist_alloc(h, sizeof(mpk::AdjMat) * (size_t)batch, plan, batch, total_scratch, &st))) return rc;
    mpk::AdjMat *hm = (mpk::AdjMat *)st.host_desc;
    uint8_t *sp = st.scratch;
    for (int64_t b = 0; b < batch; ++b) {
        const int64_t n = nv[(size_t)b];
        size_t ml, me, ms, sl, se, ss, rb, tb;
        (void)sizes(n, &ml, &me, &ms, &sl, &se, &ss, &rb, &tb);
        uint8_t *q = sp;
        auto carve = [&](size_t bytes) {
            uint8_t *p = q;
            q += bytes;
            return p;
        };
        mpk::AdjMat &M = hm[b];
        M.LU = dev_mat(LU_arr[b]);
        M.D = dev_mat(D_arr[b]);
        M.adjT = dev_mat(adjT_arr[b]);
        M.W = mpk::MatDev{(uint32_t *)carve(ml), (int64_t *)carve(me), (int32_t *)carve(ms), n};
        M.J = mpk::MatDev{(uint32_t *)carve(ml), (int64_t *)carve(me), (int32_t *)carve(ms), n};
        M.S = mpk::MatDev{(uint32_t *)carve(sl), (int64_t *)carve(se), (int32_t *)carve(ss), n + 1};
        M.rw = (uint32_t *)carve(rb);
        M.gate = (int32_t *)carve(256);
        M.T = lane ? (uint32_t *)carve(tb) : nullptr;
        M.info = info_dev + b;
        M.n = n;
        sp += scratch[(size_t)b];
    }
    const size_t lds = persist_lds_bytes(P, lane);
    int64_t grid = 0;
    uint64_t limit = 0;
    if ((rc = persist_upload(h, plan, &st, s)) ||
        (rc = persist_shape(h, (const void *)mpk::k_persist_adj, lds, plan.pre.back(), &grid, &limit)))
        return rc;
    const unsigned bb = (unsigned)((batch + 255) / 256);
    hipLaunchKernelGGL(mpk::k_persist_begin, dim3(bb), dim3(256), 0, s, st.ctl, st.done, st.skipped, batch);
    if ((rc = last_launch())) return rc;
    const mpk::AdjMat *dmats = (const mpk::AdjMat *)st.dev_desc;
    {
        Prof pr(h, s, K_BATCH_PERSIST);
        hipLaunchKernelGGL(mpk::k_persist_adj, dim3((unsigned)grid), dim3(64 * mpk::kPersistWaves), lds, s, dmats,
                           st.recs, st.pre, (int64_t)plan.recs.size(), st.done, st.skipped, st.ctl, P,
                           persist_lds_wave(P, lane), limit);
    }
    if ((rc = last_launch())) return rc;
    if (status_dev) {
        hipLaunchKernelGGL(mpk::k_persist_adj_end, dim3(bb), dim3(256), 0, s, dmats, (const int32_t *)st.skipped,
                           status_dev, batch);
        rc = last_launch();
    }
    return rc;
}

int mp_to_f64(mpdet_handle *h, mpdet_mat x, double *mant_dev, int64_t *exp_dev, void *stream) {
    if (!h || !mat_ok(x, x.rows * x.cols > 0)) return MPDET_EINVAL;
    const int64_t cnt = x.rows * x.cols;
    if (cnt == 0) return MPDET_OK;
    if (!mant_dev || !exp_dev) return MPDET_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    hipLaunchKernelGGL(mpk::k_to_f64, grid_for((cnt + 255) / 256), dim3(256), 0, (hipStream_t)stream, dev(x),
                       x.rows, x.cols, x.nlimbs, mant_dev, exp_dev);
    return last_launch();
}

int mp_to_f64_scaled(mpdet_handle *h, mpdet_mat x, const int64_t *shift_dev, double *val_dev, void *stream) {
    if (!h || !mat_ok(x, x.rows * x.cols > 0)) return MPDET_EINVAL;
    const int64_t cnt = x.rows * x.cols;
    if (cnt == 0) return MPDET_OK;
    if (!shift_dev || !val_dev) return MPDET_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    hipLaunchKernelGGL(mpk::k_to_f64_scaled, grid_for((cnt + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       dev(x), x.rows, x.cols, x.nlimbs, shift_dev, val_dev);
    return last_launch();
}

}  // extern "C"
