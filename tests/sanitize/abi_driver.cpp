// Runs the C-ABI's host-side code under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_sanitizers.py with the
// sanitizers on the host pass only): argument checks of every entry point,
// the workspace query and the persistent launch's schedule builder on large
// batches.  Nothing here needs a GPU.  Exit status 0 and no sanitizer report
// is a pass.
#include <stdint.h>
#include <stdio.h>

#include <vector>

#include "mpdet.h"

#define EXPECT(cond)                                                  \
    do {                                                              \
        if (!(cond)) {                                                \
            printf("abi driver: failed %s (line %d)\n", #cond, __LINE__); \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main() {
    mpdet_mat m{nullptr, nullptr, nullptr, 4, 4, 4, 8};
    EXPECT(mp_det_factor(nullptr, m, m, nullptr, 0, nullptr) == MPDET_EINVAL);
    EXPECT(mp_det_factor_steps(nullptr, m, m, nullptr, 0, 4, 0, nullptr) == MPDET_EINVAL);
    EXPECT(mp_det_minors(nullptr, m, m, m, nullptr, nullptr) == MPDET_EINVAL);
    EXPECT(mp_det_batched(nullptr, 3, &m, &m, &m, nullptr, 0, 0, nullptr) == MPDET_EINVAL);
    EXPECT(mp_det_adjugate(nullptr, m, m, m, nullptr, nullptr) == MPDET_EINVAL);
    EXPECT(mp_det_adjugate_batched(nullptr, 1, &m, &m, &m, nullptr, nullptr, 0, nullptr) == MPDET_EINVAL);
    EXPECT(mp_det_all_minors(nullptr, m, m, m, nullptr, nullptr) == MPDET_EINVAL);
    EXPECT(mp_det_normalize_minors(nullptr, m, m, nullptr) == MPDET_EINVAL);
    EXPECT(mp_det_extend(nullptr, m, m, nullptr, 2, 0, nullptr) == MPDET_EINVAL);
    EXPECT(mp_det_factor_ball(nullptr, m, m, nullptr, nullptr, nullptr, 0, 0, nullptr) == MPDET_EINVAL);
    EXPECT(mp_truncate(nullptr, m, m, nullptr) == MPDET_EINVAL);
    EXPECT(mp_to_f64(nullptr, m, nullptr, nullptr, nullptr) == MPDET_EINVAL);
    EXPECT(mp_det_factor_noalloc(m, m, nullptr, 0, nullptr) == MPDET_EINVAL);
    EXPECT(mpdet_create(nullptr, 0) == MPDET_EINVAL);
    EXPECT(mpdet_destroy(nullptr) == MPDET_EINVAL);
    mpdet_handle *h = nullptr;
    const int rc = mpdet_create(&h, 0);  // no GPU in this container
    EXPECT(rc == MPDET_OK || rc == MPDET_EHIP || rc == MPDET_EINVAL);
    if (rc == MPDET_OK) mpdet_destroy(h);
    // the workspace query over shapes and paths
    size_t bytes = 0;
    for (int64_t n : {0, 1, 2, 63, 64, 65, 511, 2048, 6144})
        for (int32_t P : {2, 3, 8, 64, 128, 129, 1024})
            for (int path : {0, 1, 2}) {
                const int r = mpdet_workspace_size(nullptr, n, P, path, &bytes);
                EXPECT(r == MPDET_OK || (path == 2 && r == MPDET_ENOTSUP));
            }
    EXPECT(mpdet_workspace_size(nullptr, -1, 8, 0, &bytes) == MPDET_EINVAL);
    // the persistent launch's schedule on a config-4-sized batch and on edge sizes
    std::vector<int64_t> sizes;
    for (int b = 0; b < 256; ++b) sizes.push_back(16 + (b * 367) % 369);
    int64_t nrec = 0, ntk = 0;
    EXPECT(mpdet_batched_plan((int64_t)sizes.size(), sizes.data(), 64, 1, MPDET_WANT_MINORS, nullptr, 0, &nrec,
                              &ntk) == MPDET_OK);
    std::vector<unsigned char> recs((size_t)nrec * 32);
    EXPECT(mpdet_batched_plan((int64_t)sizes.size(), sizes.data(), 64, 1, MPDET_WANT_MINORS, recs.data(), nrec,
                              &nrec, &ntk) == MPDET_OK);
    EXPECT(mpdet_batched_plan((int64_t)sizes.size(), sizes.data(), 64, 1, 0, recs.data(), 1, &nrec, &ntk) ==
           MPDET_EINVAL);  // too small a buffer
    const int64_t one = 1;
    EXPECT(mpdet_batched_plan(1, &one, 6, 1, MPDET_WANT_MINORS, nullptr, 0, &nrec, &ntk) == MPDET_OK);
    EXPECT(mpdet_batched_plan(0, nullptr, 6, 1, 0, nullptr, 0, &nrec, &ntk) == MPDET_OK && nrec == 0);
    EXPECT(mpdet_batched_plan(2, sizes.data(), 128, 2, 0, nullptr, 0, &nrec, &ntk) == MPDET_ENOTSUP);
    EXPECT(mpdet_strerror(MPDET_ERANGE) != nullptr && mpdet_strerror(12345) != nullptr);
    printf("abi driver: ok\n");
    return 0;
}
