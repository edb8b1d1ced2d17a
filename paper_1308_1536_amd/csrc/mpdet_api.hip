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

struct mpdet_handle {
    int device;
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

int factor_valu(const mpdet_mat &A, const mpdet_mat &D, int32_t *info, hipStream_t s) {
    const int64_t n = A.rows;
    const int P = A.nlimbs;
    const size_t lds = mpk::lds_bytes(P);
    mpk::MatDev a = dev(A), d = dev(D);
    for (int64_t k = 0; k < n; ++k) {
        hipLaunchKernelGGL(mpk::k_pivot_divide, dim3((unsigned)(n - k)), dim3(64), lds, s, a, d, info, k, n, P);
        int rc = last_launch();
        if (rc) return rc;
        const int64_t m = n - k - 1;
        if (m > 0) {
            hipLaunchKernelGGL(mpk::k_update_valu, grid_for(m * m), dim3(64), lds, s, a, (const int32_t *)info, k,
                               n, P);
            rc = last_launch();
            if (rc) return rc;
        }
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
    free(h);
    return MPDET_OK;
}

int mp_det_factor(mpdet_handle *h, mpdet_mat A, mpdet_mat D, int32_t *info_dev, int path, void *stream) {
    if (!h || !info_dev) return MPDET_EINVAL;
    if (!mat_ok(A, A.rows > 0) || !mat_ok(D, A.rows > 0)) return MPDET_EINVAL;
    if (A.rows != A.cols || D.nlimbs != A.nlimbs || D.rows < 1 || D.cols < A.rows) return MPDET_EINVAL;
    if (path != MPDET_PATH_AUTO && path != MPDET_PATH_VALU && path != MPDET_PATH_MFMA) return MPDET_EINVAL;
    if (path == MPDET_PATH_MFMA) return MPDET_ENOTSUP;
    DeviceGuard g(h->device);
    if (!g.ok) return MPDET_EHIP;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(mpk::k_set_info, dim3(1), dim3(64), 0, s, info_dev, 0);
    int rc = last_launch();
    if (rc) return rc;
    if (A.rows == 0) return MPDET_OK;
    return factor_valu(A, D, info_dev, s);
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
        hipLaunchKernelGGL(mpk::k_minors_sweep, dim3((unsigned)j), dim3(64), lds, s, lu, cv, info_dev, j, n, P);
        rc = last_launch();
        if (rc) return rc;
    }
    hipLaunchKernelGGL(mpk::k_minors_final, dim3((unsigned)n), dim3(64), lds, s, d, cv, info_dev, n, P);
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
