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

// Per-kernel timing (off by default): each launch is bracketed by two HIP
// events recorded on the launch stream; mpdet_profile_end folds the elapsed
// times into per-kernel totals.
enum KernelId { K_PIVOT_DIVIDE = 0, K_DIVIDE, K_UPDATE_VALU, K_UPDATE_MFMA, K_MFMA_PREP, K_MINORS_SWEEP,
                K_MINORS_FINAL, K_OTHER, K_COUNT };
static const char *kKernelNames[K_COUNT] = {"pivot_divide", "divide", "update_valu", "update_mfma", "mfma_prep",
                                            "minors_sweep", "minors_final", "other"};

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
    // the pivot's reciprocal
    void *rw;
    size_t rw_bytes;
};

namespace {

constexpr int kMaxLimbs = 1024;

int check(hipError_t e) { return e == hipSuccess ? MPDET_OK : MPDET_EHIP; }

bool mat_ok(const mpdet_mat &m, bool need_ptrs) {
    if (m.rows < 0 || m.cols < 0 || m.ld < m.cols || m.nlimbs < 2 || m.nlimbs > kMaxLimbs) return false;
    if (need_ptrs && (!m.limbs || !m.exp || !m.sign)) return false;
    return true;
}

mpk::MatDev dev(const mpdet_mat &m) { return mpk::MatDev{m.limbs, m.exp, m.sign, m.ld}; }

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

// Scratch for the pivot's reciprocal: P + 2 limbs (R and its exactness flag).
int recip_ws(mpdet_handle *h, int P, uint32_t **rw) {
    const size_t need = ((size_t)(P + 2) * 4u + 255) & ~(size_t)255;
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

// Algorithm 1 steps 2.1 and 2.2.1 for step k: D_k and the pivot's reciprocal,
// then the multipliers of rows k+1..n-1.
int pivot_step(mpdet_handle *h, const mpk::MatDev &a, const mpk::MatDev &d, int32_t *info, int64_t k, int64_t n,
               int P, hipStream_t s) {
    uint32_t *rw = nullptr;
    int rc = recip_ws(h, P, &rw);
    if (rc) return rc;
    const size_t lds = mpk::pivot_lds_bytes(P);
    {
        Prof pr(h, s, K_PIVOT_DIVIDE);
        hipLaunchKernelGGL(mpk::k_pivot_recip, dim3(2), dim3(64), lds, s, a, d, info, rw, k, n, P);
    }
    if ((rc = last_launch())) return rc;
    const int64_t m = n - k - 1;
    if (m <= 0) return MPDET_OK;
    {
        Prof pr(h, s, K_DIVIDE);
        hipLaunchKernelGGL(mpk::k_divide, dim3((unsigned)m), dim3(64), lds, s, a, (const uint32_t *)rw,
                           (const int32_t *)info, k, n, P);
    }
    return last_launch();
}

int factor_valu(mpdet_handle *h, const mpdet_mat &A, const mpdet_mat &D, int32_t *info, hipStream_t s) {
    const int64_t n = A.rows;
    const int P = A.nlimbs;
    const size_t lds = mpk::lds_bytes(P);
    mpk::MatDev a = dev(A), d = dev(D);
    for (int64_t k = 0; k < n; ++k) {
        int rc = pivot_step(h, a, d, info, k, n, P, s);
        if (rc) return rc;
        const int64_t m = n - k - 1;
        if (m > 0) {
            {
                Prof pr(h, s, K_UPDATE_VALU);
                hipLaunchKernelGGL(mpk::k_update_valu, grid_for(m * m), dim3(64), lds, s, a, (const int32_t *)info,
                                   k, n, P);
            }
            rc = last_launch();
            if (rc) return rc;
        }
    }
    return MPDET_OK;
}

// Workspace of the MFMA path for trailing blocks up to m x m: reversed
// multiplier digits, pivot-row digits and product-top records.
struct MfmaWs {
    uint8_t *Lr, *Ub;
    uint32_t *T;
};

int mfma_workspace(mpdet_handle *h, int64_t m, int P, MfmaWs *w) {
    const mpk::MfmaGeom g = mpk::mfma_geom(P);
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t lr = up((size_t)m * g.LR), ub = up((size_t)m * g.K8);
    const size_t t = up((size_t)m * (size_t)m * (size_t)g.TP * 4u);
    const size_t need = lr + ub + t;
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
    w->Lr = base;
    w->Ub = base + lr;
    w->T = (uint32_t *)(base + lr + ub);
    return MPDET_OK;
}

int factor_mfma(mpdet_handle *h, const mpdet_mat &A, const mpdet_mat &D, int32_t *info, hipStream_t s) {
    const int64_t n = A.rows;
    const int P = A.nlimbs;
    MfmaWs w;
    int rc = mfma_workspace(h, n > 1 ? n - 1 : 1, P, &w);
    if (rc) return rc;
    const size_t lds_mfma = mpk::mfma_lds_bytes(P), lds_prep = (size_t)(P + 1) * 4;
    mpk::MatDev a = dev(A), d = dev(D);
    const int32_t *cinfo = info;
    for (int64_t k = 0; k < n; ++k) {
        if ((rc = pivot_step(h, a, d, info, k, n, P, s))) return rc;
        const int64_t m = n - k - 1;
        if (m <= 0) continue;
        {
            Prof pr(h, s, K_MFMA_PREP);
            hipLaunchKernelGGL(mpk::k_mfma_prep, grid_for(2 * m), dim3(64), lds_prep, s, a, w.Lr, w.Ub, cinfo, k,
                               n, P);
        }
        if ((rc = last_launch())) return rc;
        {
            Prof pr(h, s, K_UPDATE_MFMA);
            hipLaunchKernelGGL(mpk::k_update_mfma, grid_for(m * ((m + 31) / 32)), dim3(64), lds_mfma, s, a,
                               (const uint8_t *)w.Lr, (const uint8_t *)w.Ub, w.T, cinfo, k, n, P);
        }
        if ((rc = last_launch())) return rc;
        {
            Prof pr(h, s, K_OTHER);
            hipLaunchKernelGGL(mpk::k_sub_mfma, grid_for(m * m), dim3(64), mpk::lds_bytes(P), s, a,
                               (const uint32_t *)w.T, cinfo, k, n, P);
        }
        if ((rc = last_launch())) return rc;
    }
    return MPDET_OK;
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
    free(h);
    return MPDET_OK;
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

int mp_det_factor(mpdet_handle *h, mpdet_mat A, mpdet_mat D, int32_t *info_dev, int path, void *stream) {
    if (!h || !info_dev) return MPDET_EINVAL;
    if (!mat_ok(A, A.rows > 0) || !mat_ok(D, A.rows > 0)) return MPDET_EINVAL;
    if (A.rows != A.cols || D.nlimbs != A.nlimbs || D.rows < 1 || D.cols < A.rows) return MPDET_EINVAL;
    if (path != MPDET_PATH_AUTO && path != MPDET_PATH_VALU && path != MPDET_PATH_MFMA) return MPDET_EINVAL;
    const bool mfma_ok = mpk::mfma_supported(A.nlimbs);
    if (path == MPDET_PATH_MFMA && !mfma_ok) return MPDET_ENOTSUP;
    const bool use_mfma = path == MPDET_PATH_MFMA || (path == MPDET_PATH_AUTO && mfma_ok);
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(mpk::k_set_info, dim3(1), dim3(64), 0, s, info_dev, 0);
    int rc = last_launch();
    if (rc) return rc;
    if (A.rows == 0) return MPDET_OK;
    return use_mfma ? factor_mfma(h, A, D, info_dev, s) : factor_valu(h, A, D, info_dev, s);
}

int mp_det_minors(mpdet_handle *h, mpdet_mat LU, mpdet_mat D, mpdet_mat c, const int32_t *info_dev,
                  void *stream) {
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
            hipLaunchKernelGGL(mpk::k_minors_sweep, dim3((unsigned)j), dim3(64), lds, s, lu, cv, info_dev, j, n,
                               P);
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

}  // extern "C"
