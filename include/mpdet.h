/*
 * mpdet.h -- C-ABI of libmpdet.so: multiprecision determinant, leading
 * determinants and last-column minors on AMD Instinct MI355X (gfx950).
 *
 * Method: Gaussian elimination without pivoting in multiprecision floating
 * point (Beliakov & Matiyasevich, "A Parallel Algorithm for Calculation of
 * Large Determinants with High Accuracy for GPUs and MPI clusters", Sec. 3 and
 * Algorithm 1).  The determinant and every leading principal determinant are
 * running products of the pivots (Algorithm 1 step 2.1; Sec. 3 "determinants
 * of all submatrices in the top left corner"); the signed minors of the last
 * column follow from the [A I] derivation of Sec. 3 (the last row of L times
 * |A|), eq. (minorsdef).
 *
 * ---------------------------------------------------------------------------
 * Number format (shared by every entry point)
 *   value = (-1)^sign * m * 2^(exp - 32*nlimbs)
 *   m: nlimbs little-endian uint32 limbs (limb 0 least significant), top bit
 *      of limb nlimbs-1 set (2^(p-1) <= m < 2^p, p = 32*nlimbs);
 *   exp: int64; sign: int32, 0 (+) or 1 (-).
 *   Zero is canonical: m = 0, exp = 0, sign = 0.
 * Every operation is the exact real result truncated toward zero to p bits
 * (RZ_p).  A product is rounded before it is subtracted (two roundings per
 * trailing update); a quotient is RZ_p of the exact quotient.
 * The same mantissa bytes read as 4*nlimbs little-endian 8-bit limbs.
 *
 * Matrix layout in device memory (mpdet_mat), element-contiguous mantissas:
 *   limbs[(i*ld + j)*nlimbs + q], exp[i*ld + j], sign[i*ld + j],
 *   0 <= i < rows, 0 <= j < cols <= ld.  A vector is a 1 x n matrix.
 * All pointers in mpdet_mat are device pointers owned by the caller; the
 * library never frees them.  Exponents of inputs must satisfy |exp| <= 2^48.
 *
 * Return codes: every entry point returns MPDET_OK or a negative status for
 * errors it can detect on the host (bad shapes or pointers, unsupported path,
 * allocation or launch failure).  Calls are stream ordered and asynchronous.
 * Numeric outcomes are written to a device int32 `info`, LAPACK getrf style:
 *   0   success;
 *   k>0 the pivot of step k (1-based) is exactly zero: D_k..D_n are written as
 *       zero and the matrix holds the state after k-1 elimination steps;
 *   -1  a pivot or a leading determinant has |exp| > 2^62: D_k..D_n are zero
 *       and the matrix contents are unspecified;
 *   -2  a bounded wait inside a launch ran out (an internal failure: waves of
 *       one workgroup lost step with each other, or a persistent launch's
 *       dependency never completed); the outputs are unspecified.  No correct
 *       run waits long enough for this (the bounds are seconds).
 * One handle per host thread; calls on one handle must not overlap in time on
 * different streams (the handle's workspace is shared).
 */
#ifndef MPDET_H
#define MPDET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpdet_handle mpdet_handle;

typedef struct {
    uint32_t *limbs; /* device: [rows][ld][nlimbs] */
    int64_t *exp;    /* device: [rows][ld] */
    int32_t *sign;   /* device: [rows][ld] */
    int64_t rows, cols, ld;
    int32_t nlimbs;
} mpdet_mat;

enum {
    MPDET_OK = 0,
    MPDET_EINVAL = -1,
    MPDET_ENOMEM = -2,
    MPDET_EHIP = -3,
    MPDET_ENOTSUP = -4,
    MPDET_ERANGE = -5 /* the workspace would exceed mp_det_factor_noalloc's scratch */
};

enum {
    MPDET_PATH_AUTO = 0, /* library chooses: MFMA when nlimbs allows it and
                            is above 64, else VALU */
    MPDET_PATH_VALU = 1, /* 32x32->64-bit integer VALU limb products */
    MPDET_PATH_MFMA = 2  /* exact INT8 MFMA Toeplitz contraction of 8-bit limbs */
};

/* Create a handle bound to HIP device `device`.  *h receives the handle. */
int mpdet_create(mpdet_handle **h, int device);
/* Release the handle and its workspace (synchronises the device first). */
int mpdet_destroy(mpdet_handle *h);
/* Human-readable name of a status code (static storage). */
const char *mpdet_strerror(int status);

/*
 * mp_det_factor -- Gaussian elimination without pivoting, in place
 * (Algorithm 1 steps 1-2.2.2; multipliers stored below the diagonal as in the
 * Sec. 3 storage paragraph).
 *   A     n x n (rows == cols == n, n >= 0), overwritten: U on and above the
 *         diagonal, the multipliers l_ik = a_ik / a_kk below it.
 *   D     1 x n (cols >= n), same nlimbs: D_k = RZ_p(D_{k-1} * u_kk), D_1 =
 *         u_11; det(A) = D_n.
 *   info  device int32, written as described above.
 *   path  MPDET_PATH_*; MFMA requires nlimbs % 8 == 0 (else MPDET_ENOTSUP).
 *   stream hipStream_t (NULL = default stream).
 * nlimbs must be in [2, 1024].  Results are bit-identical for every path.
 */
int mp_det_factor(mpdet_handle *h, mpdet_mat A, mpdet_mat D, int32_t *info_dev,
                  int path, void *stream);

/*
 * mp_det_factor_steps -- elimination steps k_begin .. k_end-1 (0-based; step k
 * eliminates column k) of mp_det_factor, in place: a factorisation can be
 * split into several calls (e.g. to bound the time of one call, or to check
 * the leading determinants D_1 .. D_{k_end} of a large run while it runs).
 * Calling it with the ranges [0, k_1), [k_1, k_2), ..., [k_r, n) on the same
 * A, D and info, with the same path, gives the bits of one mp_det_factor call
 * (Algorithm 1 runs its steps in order and each step only reads the state the
 * previous one left).  k_begin == 0 resets info; a later range continues from
 * info as the previous range left it (a nonzero info makes it do nothing).
 *   0 <= k_begin <= k_end <= n, else MPDET_EINVAL; other arguments as for
 *   mp_det_factor.
 */
int mp_det_factor_steps(mpdet_handle *h, mpdet_mat A, mpdet_mat D, int32_t *info_dev,
                        int64_t k_begin, int64_t k_end, int path, void *stream);

/*
 * mp_det_extend -- grow a factorisation (Sec. 4.1: the largest size need not
 * be fixed in advance; determinants of sizes N_b, 2 N_b, 3 N_b, ... follow as
 * blocks are added).  A is n x n; its leading n_old x n_old block holds
 * mp_det_factor's output for that block (U and the multipliers) and D holds
 * its D_1 .. D_{n_old}; the other entries of A are the new rows and columns,
 * not yet eliminated.  The call applies elimination steps 0 .. n_old-1 to the
 * new entries (the new rows' multipliers, then each step's update of the new
 * rows and of the new columns, in step order), then runs steps n_old .. n-1,
 * so A, D and info end bit-identical to mp_det_factor on the whole n x n
 * matrix (every entry gets the same operations in the same order).
 *   info_dev must hold the leading factorisation's info; a nonzero value makes
 *   the call do nothing.  0 <= n_old <= n (n_old = 0: mp_det_factor).  The
 *   steps 0 .. n_old-1 on the new entries run on the VALU kernels (the lane
 *   product where nlimbs <= 128 is a multiple of 4, else one wave per
 *   element); the steps from n_old on take `path`.
 */
int mp_det_extend(mpdet_handle *h, mpdet_mat A, mpdet_mat D, int32_t *info_dev, int64_t n_old, int path,
                  void *stream);

/*
 * mp_det_factor_ball -- mp_det_factor (same bits) and rigorous error bounds
 * for every leading determinant (the rigorous results the paper's future-work
 * section asks for, by ball arithmetic instead of intervals): after the call
 *   |D_k - D*_k| <= rad_mant[k-1] * 2^rad_exp[k-1],  k = 1..n,
 * where D*_k is the exact leading determinant of the input (with
 * MPDET_BALL_INPUT_ULP, of any matrix whose entries are within one unit in
 * the last place of the input's: inputs rounded from exact values).  Every
 * number of the elimination carries a radius m 2^e (32-bit m, int64 e)
 * propagated with upward rounding through the divisions, products and
 * differences; rad_exp[k-1] == INT64_MAX means no bound (a pivot's ball may
 * contain zero; the elimination stopped at or before step k; an exponent
 * overflow, info = -1, leaves every D_k without a bound).  The bound is worst-case, so it is looser than the actual
 * error.  rad_mant_dev uint32[n], rad_exp_dev int64[n] (device).  The handle
 * keeps 12 n^2 bytes of radii; the steps run one per call of
 * mp_det_factor_steps, each followed by two small radius kernels.
 */
enum { MPDET_BALL_INPUT_ULP = 1 };
int mp_det_factor_ball(mpdet_handle *h, mpdet_mat A, mpdet_mat D, uint32_t *rad_mant_dev, int64_t *rad_exp_dev,
                       int32_t *info_dev, int flags, int path, void *stream);

/*
 * mp_truncate -- y = RZ to 32*y.nlimbs bits of x, element by element
 * (y.nlimbs <= x.nlimbs; same rows and cols, each its own ld): the top
 * y.nlimbs limbs of every mantissa, the same exponent and sign.
 */
int mp_truncate(mpdet_handle *h, mpdet_mat x, mpdet_mat y, void *stream);

/*
 * mp_det_factor_reduced -- elimination with reduced precision in its later
 * steps (Sec. 4.3: after the unavoidable loss of accuracy, the later
 * iterations need not run at full precision).  Steps 0 .. k_switch-1 run on A
 * (nlimbs P) with D receiving D_1 .. D_{k_switch} at full precision; then A
 * and D_1 .. D_{k_switch} are truncated (mp_truncate) into A2 and D2 (nlimbs
 * P2 <= P, n x n and 1 x n), and steps k_switch .. n-1 run there on path2.
 * Afterwards A2 holds the factors at P2 (mp_det_minors on A2, D2 gives the
 * minors at P2) and D2 all of D_1 .. D_n at P2.  info as for mp_det_factor.
 *   0 <= k_switch <= n; other arguments as for mp_det_factor.
 */
int mp_det_factor_reduced(mpdet_handle *h, mpdet_mat A, mpdet_mat D, mpdet_mat A2, mpdet_mat D2, int32_t *info_dev,
                          int64_t k_switch, int path, int path2, void *stream);

/*
 * mpdet_workspace_size -- device bytes of workspace mp_det_factor takes from
 * the handle for an n x n matrix of nlimbs-limb numbers on `path` (with the
 * handle's current panel setting, see mpdet_set_panel_rows): the pivot's
 * reciprocal and, on the MFMA path and the VALU lane product (nlimbs <= 128,
 * a multiple of 4), the product records of one row panel (MFMA: plus the
 * digit strings of the multipliers and the pivot row).  mp_det_minors takes
 * none.  The handle keeps the largest workspace any call needed until
 * mpdet_destroy.  h may be NULL (the default panel setting).  Writes *bytes
 * on the host; touches no device.
 *   n >= 0, nlimbs in [2, 1024], path as for mp_det_factor, else
 *   MPDET_EINVAL (MPDET_ENOTSUP: MFMA with nlimbs % 8 != 0).
 */
int mpdet_workspace_size(mpdet_handle *h, int64_t n, int32_t nlimbs, int path, size_t *bytes);

/*
 * mpdet_set_panel_rows -- rows per panel of the MFMA path's trailing update
 * (the product records of one panel of rows are formed and consumed before the
 * next panel's; their buffer grows with the panel).  0 (the default) sizes
 * panels to a 24 GiB record buffer, which keeps one panel per step up to
 * 32768-bit numbers at n ~ 2800; a 6144 x 6144 matrix of 32768-bit numbers
 * (155 GB) then needs a few panels per step.  Any value gives the same bits.
 *   rows >= 0, else MPDET_EINVAL.
 */
int mpdet_set_panel_rows(mpdet_handle *h, int64_t rows);

/*
 * mp_det_factor_noalloc -- mp_det_factor for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments (no handle), same bits; it calls no
 * hipMalloc, hipFree or other allocating routine.  Its workspace (the
 * reciprocal, the digits and the product records) lives in one static device
 * array of MPDET_NOALLOC_SCRATCH_BYTES per GPU, loaded with the library and
 * held until the process ends; its address is taken once per device (in
 * mpdet_create, or on the first call on that device).  Runs on the current
 * HIP device.
 *   Sizes whose workspace does not fit the array return MPDET_ERANGE before
 *   any launch: on the VALU lane product (nlimbs <= 128, a multiple of 4) the
 *   records of the whole (n-1) x (n-1) trailing block must fit (n <= 482 at
 *   64 limbs, n <= 353 at 128); on the MFMA path the update runs over row
 *   panels sized to the array, and the digit strings plus one row's records
 *   must fit (n <= 5156 at 1024 limbs); other VALU limb counts need only the
 *   reciprocal.
 *   Every call on one GPU uses that GPU's one array, which keeps what the last
 *   call left: calls that overlap in time on one GPU (other streams, other
 *   threads) race and give wrong results.  Whatever a call uses from the
 *   array it wrote earlier in the same call (the pending-pivot word is cleared
 *   by a kernel at the start; the read-ahead past the last record and the
 *   padding columns are read but never used), so earlier contents never reach
 *   a result.
 */
#define MPDET_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mp_det_factor_noalloc(mpdet_mat A, mpdet_mat D, int32_t *info_dev, int path, void *stream);

/*
 * mpdet_set_tuning -- launch shapes of the trailing update on this handle
 * (the autotuner's knobs; every setting gives the same bits):
 *   lane_rows   rows (= waves) per workgroup of the VALU lane product, each
 *               workgroup a lane_rows x 64 tile: 2, 4 or 8 (0: 4);
 *   mfma_waves  waves per workgroup of the MFMA update, each a row of one
 *               32-column block: 1, 2 or 4 (0: 2); a value whose LDS does not
 *               fit makes MFMA calls return MPDET_ENOTSUP.
 * The persistent batched launches keep 4 waves per workgroup.
 */
int mpdet_set_tuning(mpdet_handle *h, int32_t lane_rows, int32_t mfma_waves);

/*
 * mpdet_set_overlap -- how the MFMA path schedules the finish of the trailing
 * update (the rounding and subtraction, bound by memory) against the integer
 * products (bound by the matrix cores).  Same bits for every value.
 *   0  (the default) above 256 limbs, each wave of the update launch
 *      finishes its own 32 products as soon as they are formed, while other
 *      waves keep the matrix cores busy; otherwise as 1;
 *   1  the finish is a launch of its own after each panel's products;
 *   2 .. 64  the update split into that many row panels per step, the finish
 *      of each panel on a second stream of the handle while the next panel's
 *      update runs; two record buffers alternate.
 *   Else MPDET_EINVAL.
 */
int mpdet_set_overlap(mpdet_handle *h, int32_t panels);

/*
 * mp_det_minors -- signed last-column cofactors c_i = (-1)^(i+n) M_{i,n}
 * (eq. (minorsdef); Sec. 3 [A I] derivation), from mp_det_factor's output.
 * With L the unit lower factor, x^T L = e_n^T is solved by sweeps j = n..2,
 * s_i <- RZ(s_i - RZ(x_j l_ji)) for i < j (x_n = 1, x_{j-1} = s_{j-1}), then
 * c_i = RZ(D_{n-1} x_i), c_n = D_{n-1} (n = 1: c_1 = 1).  sum_i c_i a_in = det.
 *   LU    n x n factor output (read only);  D  1 x n from mp_det_factor;
 *   c     1 x n output;  info_dev  the factorisation's info: when it is not 0
 *         (or n), c is written as all zeros; set to -2 (see above) if a wait
 *         inside the sweeps runs out.
 */
int mp_det_minors(mpdet_handle *h, mpdet_mat LU, mpdet_mat D, mpdet_mat c,
                  int32_t *info_dev, void *stream);

/*
 * mp_det_batched -- mp_det_factor (and, with MPDET_WANT_MINORS, mp_det_minors)
 * on `batch` matrices of uneven n.  Results are bit-identical to calling
 * mp_det_factor / mp_det_minors on each matrix (every matrix gets exactly the
 * operations of its own elimination; only the schedule differs).
 *   A_arr, D_arr, c_arr  host arrays of `batch` descriptors (device buffers),
 *                        shapes as for mp_det_factor / mp_det_minors; all
 *                        matrices share one nlimbs;  c_arr may be NULL
 *                        without MPDET_WANT_MINORS.
 *   info_dev             device int32[batch], one info per matrix (a failing
 *                        matrix does not affect the others); besides the codes
 *                        above, -2 means a wait of the persistent launch
 *                        expired (mpdet_set_wait_limit) and the matrix's
 *                        results are unspecified.
 *   flags                MPDET_WANT_MINORS, and at most one schedule flag.
 * Schedules (Sec. 4.1: a queue of tasks, each taken by an idle worker once the
 * tasks it depends on are done):
 *   lockstep (the default): the batch ordered by n, every phase of every step
 *     one launch over all matrices still active at that step.
 *   persistent (MPDET_BATCH_PERSISTENT; the VALU path only, MPDET_ENOTSUP on
 *     MFMA): ONE launch of resident workgroups works through a queue of
 *     tickets -- every phase of every elimination step and minors sweep of
 *     every matrix, ordered by step, then phase, then matrix size (largest
 *     first) -- and a ticket starts once its matrix's count of completed
 *     tickets shows every earlier phase of that matrix done, so a matrix never
 *     waits for another.  Two small launches around it reset the counters and
 *     turn expired waits into info = -2.  Every wait is bounded.
 *   MPDET_BATCH_LOCKSTEP names the default explicitly.
 *   Known defect: on config 4's batch (256 matrices, N up to 384, 2048 bits)
 *   the persistent launch has given a result different from the lockstep
 *   launches' (and the oracle's) for one or two large matrices in about a
 *   third of the runs, at one of their last 30 steps; small batches have
 *   matched in every run.  Until it is found, use the lockstep default where
 *   the bits matter (the autotuner does not choose the persistent launch).
 * The descriptor and schedule tables are staged through pinned host memory
 * owned by the handle; per-matrix scratch lives in the handle's device
 * workspace.
 */
enum { MPDET_WANT_MINORS = 1, MPDET_BATCH_LOCKSTEP = 2, MPDET_BATCH_PERSISTENT = 4 };
int mp_det_batched(mpdet_handle *h, int64_t batch, const mpdet_mat *A_arr, const mpdet_mat *D_arr,
                   const mpdet_mat *c_arr, int32_t *info_dev, int flags, int path, void *stream);

/*
 * mpdet_set_wait_limit -- bound, in seconds, on every wait inside a launch
 * (default 10 s): the persistent batched launch's waits for earlier phases
 * (no correct run waits more than one phase of one matrix), and the waits
 * between the waves of one workgroup of the pivot, divide and minors-sweep
 * kernels above about 224 limbs (no correct run waits more than one
 * multiprecision product).  A persistent-launch wait that expires stops the
 * launch: every later ticket is skipped and the matrices it touched report
 * info = -2.  A workgroup wait that expires makes mp_det_factor and its
 * variants, mp_det_extend and mp_det_minors report info = -2.  0 makes any
 * wait that is not already satisfied expire (a test of those paths).
 *   0 <= seconds <= 3600, else MPDET_EINVAL.
 */
int mpdet_set_wait_limit(mpdet_handle *h, double seconds);

/*
 * mpdet_set_long_division -- 1: the single-matrix calls (mp_det_factor and
 * its variants, mp_det_extend) form every multiplier l_ik = RZ_p(a_ik / a_kk)
 * (Algorithm 1 step 2.2.1) by long division (Knuth's Algorithm D on one wave,
 * the path the shared reciprocal's exact remainder check otherwise takes only
 * when it does not settle); 0 (the default): through the pivot's reciprocal.
 * Both give the exact RZ_p quotient, so the bits are the same; long division
 * is slower.  It lets a test reach the fallback.
 *   on is 0 or 1, else MPDET_EINVAL.
 */
int mpdet_set_long_division(mpdet_handle *h, int32_t on);

/*
 * mpdet_batched_plan -- the persistent launch's schedule for matrices of sizes
 * n_host[0..batch) (host only; touches no device): *nrec phase records and
 * *ntickets tickets (a lane-product ticket is one tile for the whole
 * workgroup; any other ticket gives each of the workgroup's 4 waves one unit).  With recs_out (cap >= *nrec records of 32 bytes: int64
 * need, int64 units, int64 k, int32 matrix, int32 kind) the records are
 * copied out in queue order; `need` is the number of that matrix's tickets
 * that must be complete before the record's tickets start.  Kinds: 0 init,
 * 1 pivot, 2 multipliers, 3 lane products, 4 finish, 5 one-wave update,
 * 6 pending-code promotion, 7 minors sweep (k = its column j), 8 minors' last
 * step.  MPDET_ENOTSUP where the batch would run on MFMA (lockstep only).
 */
int mpdet_batched_plan(int64_t batch, const int64_t *n_host, int32_t nlimbs, int path, int flags, void *recs_out,
                       int64_t cap, int64_t *nrec, int64_t *ntickets);

/*
 * mp_det_adjugate -- adjT = adj(A)^T, i.e. adjT[i][j] = C_ij = d det(A) / d a_ij
 * (Sec. 3: by Baur-Strassen all (N-1)x(N-1) minors are partial derivatives of
 * the determinant), from mp_det_factor's output.  With L the unit lower factor
 * and W = L^-1, adj(A) = adj(U) W; the operations and their order are fixed
 * (W by row sweeps, adj(U) by right-looking back substitution of
 * U x = det(U) e_j, then adj(A) accumulated in ascending k), so column n of
 * adjT equals mp_det_minors' c bit for bit.
 *   LU    n x n factor output;  D  1 x n leading determinants;
 *   adjT  n x n output (its own ld);  info_dev  the factorisation's info:
 *         when it is not 0, adjT is written as all zeros.
 * The library allocates a workspace of about 2 n^2 numbers in the handle,
 * and, where the lane product applies (nlimbs <= 128, a multiple of 4), the
 * factorisation's record buffer for an n x n block (n * ceil(n/32) * 32
 * records of nlimbs + 4 words); the O(n^3) phases then run as rank-1 updates
 * on the factorisation's kernels, with the same bits.
 */
int mp_det_adjugate(mpdet_handle *h, mpdet_mat LU, mpdet_mat D, mpdet_mat adjT,
                    const int32_t *info_dev, void *stream);

/*
 * mp_det_adjugate_batched -- mp_det_adjugate on `batch` factored matrices of
 * uneven n (the backward of mp_det_batched), bit-identical to one
 * mp_det_adjugate call per matrix.  By default ONE persistent launch works
 * through a queue holding every phase of every matrix's adjugate (the W
 * sweeps, S and the diagonal of adj(U), the reciprocals, the back
 * substitution, the accumulation; each O(n^3) step a rank-1 update on the
 * lane product and the tile finish where nlimbs <= 128 is a multiple of 4),
 * as mp_det_batched's persistent schedule does for the forward;
 * MPDET_BATCH_LOCKSTEP runs one mp_det_adjugate call per matrix instead.
 *   LU_arr, D_arr, adjT_arr  host arrays of `batch` descriptors, shapes as for
 *                            mp_det_adjugate; all share one nlimbs.
 *   info_dev                 device int32[batch]: the factorisations' infos.
 *   status_dev               device int32[batch] or NULL: 0 (adjT written),
 *                            the factorisation's info (factors incomplete:
 *                            adjT is zero), or -2 (a wait of the persistent
 *                            launch expired, see mpdet_set_wait_limit: adjT
 *                            unspecified).
 *   flags                    0 or MPDET_BATCH_LOCKSTEP.
 * Workspace (in the handle): about 2 n^2 numbers per matrix plus, on the lane
 * product, the records of an n x n block per matrix.
 */
int mp_det_adjugate_batched(mpdet_handle *h, int64_t batch, const mpdet_mat *LU_arr, const mpdet_mat *D_arr,
                            const mpdet_mat *adjT_arr, const int32_t *info_dev, int32_t *status_dev, int flags,
                            void *stream);

/*
 * mp_det_all_minors -- the last-column cofactors of every leading block
 * (eq. (minorsdef) applied to A_r, the leading r x r block, r = 1..n): row
 * r-1 of C holds c^(r)_i = (-1)^(i+r) M^(r)_{i,r}, i = 1..r, and zeros above
 * the diagonal, from mp_det_factor's output.  Elimination without pivoting
 * factors every leading block with the leading part of the same L and U, so
 * row r-1 of W = L^-1 is the x of mp_det_minors on A_r; the sweeps are the
 * adjugate's (all rows at once) and C[r-1][i] = RZ(D_{r-1} W[r-1][i]),
 * C[r-1][r-1] = D_{r-1} (D_0 = 1).  Row r-1 equals mp_det_minors' c on A_r
 * bit for bit, and sum_i C[r-1][i] a_ir = D_r.
 *   LU    n x n factor output;  D  1 x n leading determinants;
 *   C     n x n output (its own ld);  info_dev  the factorisation's info:
 *         when it is not 0, C is written as all zeros.
 * The library allocates a workspace of about n^2 numbers in the handle (plus
 * the record buffer, as mp_det_adjugate).
 */
int mp_det_all_minors(mpdet_handle *h, mpdet_mat LU, mpdet_mat D, mpdet_mat C,
                      const int32_t *info_dev, void *stream);

/*
 * mp_det_normalize_minors -- the normalised minors of eq. (minors):
 * out[r][i] = RZ_p(C[r][i] / C[r][0]), every row divided by its first entry
 * (C = mp_det_minors' 1 x n vector gives delta_{N,n} = c_n / c_1; C =
 * mp_det_all_minors' n x n output gives them for every leading block).
 *   C    rows x cols input (read only);  out  rows x cols output, its own
 *        ld, same nlimbs; none of out's three arrays may share a byte with
 *        any of C's over the spans the shapes give (else MPDET_EINVAL).
 * A row whose first entry is zero is written as zeros.
 */
int mp_det_normalize_minors(mpdet_handle *h, mpdet_mat C, mpdet_mat out, void *stream);

/*
 * mp_to_f64 -- (mantissa, exponent) pairs: mant = (-1)^s * RZ_53(m / 2^p) in
 * +-[0.5, 1) and exp_out = exp (zero -> 0.0, 0).  x is any rows x cols matrix;
 * outputs are dense [rows][cols] device arrays.
 */
int mp_to_f64(mpdet_handle *h, mpdet_mat x, double *mant_dev, int64_t *exp_dev,
              void *stream);

/*
 * mp_to_f64_scaled -- val = (-1)^s * RZ_53(m / 2^p) * 2^(exp - *shift_dev) as
 * one float64 per number (dense [rows][cols]); the only rounding after the
 * 53-bit truncation is IEEE ldexp's (nearest even) in the subnormal range, and
 * results beyond float64's range are +-inf or +-0.  shift_dev is a device
 * int64 read by the kernel (for instance the det's exponent written by
 * mp_to_f64), so no host synchronisation is needed.  This is the float64
 * gradient of the det mantissa, adj(A)^T 2^-e_det, when x is adj(A)^T (Sec. 3:
 * the cofactors are the partial derivatives of det).
 */
int mp_to_f64_scaled(mpdet_handle *h, mpdet_mat x, const int64_t *shift_dev, double *val_dev,
                     void *stream);

/*
 * mpdet_measure_peak -- measured throughput of one arithmetic unit the
 * trailing update runs on (a probe kernel over every compute unit, timed with
 * HIP events after a warm-up launch; blocks the calling thread):
 *   MPDET_PEAK_MAD64    32x32->64-bit multiply-adds per second (v_mad_u64_u32,
 *                       the VALU path's limb product);
 *   MPDET_PEAK_MFMA_I8  int8 multiply-adds per second (v_mfma_i32_32x32x32_i8,
 *                       the MFMA path's limb product);
 *   MPDET_PEAK_MFMA_CLOCK  the shader clock in Hz while that probe runs (its
 *                       first wave's clock counter against the constant
 *                       100 MHz real-time counter), the clock that the
 *                       published peak's 2.4 GHz is to be compared with.
 * The probe allocates and frees a small output buffer.
 */
enum { MPDET_PEAK_MAD64 = 0, MPDET_PEAK_MFMA_I8 = 1, MPDET_PEAK_MFMA_CLOCK = 2 };
int mpdet_measure_peak(mpdet_handle *h, int kind, double *per_second);

/*
 * Per-kernel timing with HIP events (tracing; off by default).
 * mpdet_profile_begin clears the counters and brackets every later launch on
 * this handle with two events on the launch stream; mpdet_profile_end waits
 * for those events and adds their elapsed times to the totals;
 * mpdet_profile_get returns the total milliseconds and launch count of one
 * kernel: "pivot_divide" (leading determinant and the pivot's reciprocal),
 * "divide" (multipliers), "update_valu", "update_mfma", "mfma_prep",
 * "minors_sweep", "minors_final", "update_finish" (the MFMA path's per-element
 * rounding and subtraction), "adjugate", "all_minors", "batch_persistent" (the
 * persistent batched launch) or "other" (MPDET_EINVAL for other names).
 */
int mpdet_profile_begin(mpdet_handle *h);
int mpdet_profile_end(mpdet_handle *h);
int mpdet_profile_get(mpdet_handle *h, const char *kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif
