// kernels_persist.h -- a batch of matrices of uneven n in ONE persistent
// launch over a queue of tasks (the task queue of Sec. 4.1: a task is taken
// by an idle worker once every task it depends on has been processed).
//
// The host lays out the whole schedule as a list of phase records, one per
// (matrix, phase of a step): initialise, pivot (where the previous step's
// finish did not already examine it), multipliers, products, finish (or the
// one-wave update), the promotion of the pending pivot code, the minors
// sweeps and the minors' last step.  A record is cut into tickets: a product
// ticket is one workgroup-wide tile of the lane product; every other ticket
// gives each of the workgroup's waves one unit (a row, a 64-element finish
// tile, an element) of that phase.  Records are ordered by a virtual time
// (elimination step k, then the minors sweeps after a matrix's last step),
// then by phase, then by matrix size (largest first); within a matrix that
// order is its own phase order.
//
// Workgroups take tickets from one atomic counter in that order.  Before a
// ticket runs, its matrix's count of completed tickets must reach the
// record's `need` (every ticket of that matrix's earlier phases); a finished
// ticket adds one to the count.  A ticket is taken only after every earlier
// ticket was taken by a running workgroup, and it waits only for earlier
// tickets, so the earliest unfinished ticket can always run: the queue
// drains whatever number of workgroups is resident.  Every wait is bounded
// (wall clock): a wait that expires sets an abort flag, every later ticket
// is skipped, and the matrices with skipped tickets are marked (k_persist_end
// turns the marks into info = -2).
//
// Each matrix gets exactly the operations of its own elimination in the same
// order per element, so results are bit-identical to the per-matrix calls.
#pragma once

#include "kernels_adj.h"
#include "kernels_batch.h"

namespace mpk {

enum PersistKind : int32_t {
    PK_INIT = 0,   // workgroup: info = 0, pending code cleared, minors accumulators zeroed
    PK_PIVOT,      // waves, 2 units: D_k (unit 0) and the pivot's reciprocal (unit 1)
    PK_DIVIDE,     // waves, m units: multipliers of rows k+1 ..
    PK_PROD,       // workgroup, lane_update_blocks(m) units: lane products into the records
    PK_FINISH,     // waves, finish_blocks(m, m, P) units: a_ij = RZ(a_ij - RZ(l u)) (+ look-ahead pivot)
    PK_UPDV,       // waves, m^2 units: one-wave update of one element
    PK_PEND,       // workgroup: the last pending pivot code moves into info
    PK_MSWEEP,     // waves, j units: minors sweep j = n - 1 - s
    PK_MFINAL,     // waves, n units: c_i = RZ(D_{n-1} x_i)
    PK_COUNT
};

__host__ __device__ inline bool persist_wg_kind(int kind) {
    return kind == PK_INIT || kind == PK_PROD || kind == PK_PEND;
}

struct PersistRec {
    int64_t need;   // completed tickets of this matrix before the record may run
    int64_t units;  // units of work of the phase
    int64_t k;      // elimination step, or the minors sweep's column j
    int32_t mat;    // index into the descriptor array
    int32_t kind;   // PersistKind
};

struct PersistCtl {
    int64_t head;       // next ticket
    int32_t abort_flag; // a bounded wait expired
    int32_t pad;
};

constexpr int kPersistWaves = kLaneRows;  // waves per workgroup (the lane product's rows)

// largest r in [from, nrec) with pre[r] <= t, given pre[from] <= t: a
// workgroup's tickets only grow, so the search gallops forward from the record
// of its previous ticket (a few steps) instead of bisecting the whole table
__device__ __forceinline__ int64_t persist_locate(const int64_t *pre, int64_t nrec, int64_t t, int64_t from) {
    int64_t lo = from, step = 1;
    while (lo + step < nrec && pre[lo + step] <= t) {
        lo += step;
        step <<= 1;
    }
    int64_t hi = min(lo + step, nrec) - 1;  // pre[hi + 1] > t, or hi = nrec - 1
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Wait (one thread) until *cnt >= need.  Returns false when the abort flag is
// set or the wait outlives `limit` wall-clock ticks (then it sets the flag).
__device__ bool persist_wait(const int64_t *cnt, int64_t need, int32_t *abort_flag, uint64_t limit) {
    if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return true;
    const uint64_t t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(2);
        if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return true;
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        if (wall_clock64() - t0 > limit) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
}

// One wave's unit of a ticket: base + wave, if below the phase's unit count
// (one unit per wave: a loop around the bodies makes the compiler keep far
// more registers live).
template <typename F>
__device__ __forceinline__ void persist_wave_unit(int64_t base, int64_t units, F body) {
    const int64_t u = base + (int64_t)(threadIdx.x >> 6);
    if (u < units) body(u);
}

// The queue loop shared by the persistent kernels: take a ticket, wait until
// its matrix's earlier phases are done, run it (exec), count it.  lds: the
// workgroup's dynamic LDS; lds_wave: words of one wave's slice of it (the
// one-wave bodies); the workgroup-wide bodies use the whole allocation.
// exec(R, tk, base, lw, P): record, ticket within the record, first unit of
// the ticket for one-wave kinds (tk * waves), this wave's LDS slice.
template <typename Exec>
__device__ __forceinline__ void persist_queue(uint32_t *lds, const PersistRec *recs, const int64_t *pre,
                                              int64_t nrec, int64_t *done, int32_t *skipped, PersistCtl *ctl,
                                              int P_arg, int64_t lds_wave, uint64_t limit, Exec exec) {
    __shared__ int64_t s_ticket;
    __shared__ int32_t s_ok;
    const int64_t total = pre[nrec];
    int64_t r = 0;  // record of the previous ticket
    for (;;) {
        // P and the LDS slice are made opaque in every round of the queue loop:
        // otherwise the compiler hoists what the bodies derive from them out of
        // the loop, and the values it keeps live across it cost ~100 registers
        int P = P_arg;
        asm volatile("" : "+s"(P));
        int64_t lwo = lds_wave;
        asm volatile("" : "+s"(lwo));
        uint32_t *lw = lds + (int64_t)(threadIdx.x >> 6) * lwo;
        if (threadIdx.x == 0) s_ticket = __hip_atomic_fetch_add(&ctl->head, (int64_t)1, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        // the ticket is the same for the whole workgroup: keep it (and all that
        // is derived from it) in scalar registers
        const int64_t t = uniform64(s_ticket);
        if (t >= total) break;
        r = persist_locate(pre, nrec, t, r);
        const PersistRec R = recs[r];
        if (threadIdx.x == 0) {
            bool ok = __hip_atomic_load(&ctl->abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
                      persist_wait(&done[R.mat], R.need, &ctl->abort_flag, limit);
            // every earlier phase of the matrix is complete: see its writes
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_ok = ok ? 1 : 0;
            if (!ok) skipped[R.mat] = 1;
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(s_ok)) {
            const int64_t tk = t - pre[r];  // ticket within the record
            exec(R, tk, tk * (int64_t)kPersistWaves, lw, P);
        }
        // every wave's memory operations are complete (a workgroup barrier
        // alone waits only for LDS) before one release at device scope makes
        // them visible and counts the ticket
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&done[R.mat], (int64_t)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void __launch_bounds__(64 * kPersistWaves) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_persist(const BatchMat *mats, const PersistRec *recs, const int64_t *pre, int64_t nrec, int64_t *done,
          int32_t *skipped, PersistCtl *ctl, int P, int lookahead, int minors, int64_t lds_wave,
          uint64_t limit) {
    extern __shared__ uint32_t lds_raw[];
    persist_queue(lds_raw, recs, pre, nrec, done, skipped, ctl, P, lds_wave, limit,
                  [&](const PersistRec &R, int64_t tk, int64_t base, uint32_t *lw, int P) {
        const BatchMat M = mats[R.mat];
        const int64_t k = R.k, n = M.n, m = n - k - 1;
        switch (R.kind) {
            case PK_INIT: {
                const int64_t nl = minors ? n * (int64_t)P : 0;
                for (int64_t e = threadIdx.x; e < nl; e += blockDim.x) M.c.limbs[e] = 0u;
                if (minors)
                    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
                        M.c.exp[e] = 0;
                        M.c.sign[e] = 0;
                    }
                if (threadIdx.x == 0) {
                    *M.info = 0;
                    M.rw[P + 2] = 0u;
                }
                break;
            }
            case PK_PIVOT:
                persist_wave_unit(base, R.units, [&](int64_t u) {
                    pivot_recip_body(lw, M.A, M.D, M.info, M.info, M.rw, k, n, P, (int)u);
                });
                break;
            case PK_DIVIDE:
                persist_wave_unit(base, R.units, [&](int64_t u) { divide_body(lw, M.A, M.rw, M.info, k, n, P, u); });
                break;
            case PK_PROD: prod_lane_body(lds_raw, elim_rank1(M.A, k, n), M.T, M.info, P, tk); break;
            case PK_FINISH:
                persist_wave_unit(base, R.units, [&](int64_t u) {
                    finish_body<false>(lw, M.A, M.T, M.info, k, n, P, 0, m, u, M.D, lookahead ? M.rw : nullptr);
                });
                break;
            case PK_UPDV:
                persist_wave_unit(base, R.units, [&](int64_t u) { update_valu_body(lw, M.A, M.info, k, n, P, u); });
                break;
            case PK_PEND:
                if (threadIdx.x == 0 && *M.info == 0) *M.info = (int32_t)M.rw[P + 2];
                break;
            case PK_MSWEEP:
                persist_wave_unit(base, R.units,
                                  [&](int64_t u) { minors_sweep_body(lw, M.A, M.c, M.info, k, n, P, u); });
                break;
            case PK_MFINAL:
                persist_wave_unit(base, R.units, [&](int64_t u) { minors_final_body(lw, M.D, M.c, M.info, n, P, u); });
                break;
            default: break;
        }
    });
}

// ---------------------------------------------------------------------------
// The determinant's backward, adj(A)^T, for a batch in one persistent launch:
// the phases of mp_det_adjugate (kernels_adj.h: W by row sweeps, S and the
// diagonal of adj(U), the pivots' reciprocals, the back substitution, the
// ascending-k accumulation) as records of the same queue, per matrix in that
// order.  Where the lane product applies, each O(n^3) step is a rank-1 update
// (lane product tile, then tile finish); otherwise one wave per element.
// ---------------------------------------------------------------------------
struct AdjMat {
    MatDev LU, D, adjT;  // the caller's factors, leading determinants and output
    MatDev W, J, S;      // workspace: L^-1, adj(U), the products S_i
    uint32_t *rw;        // the pivots' reciprocals, n x (P + 2) words
    uint32_t *T;         // product records of one rank-1 update (lane product)
    const int32_t *info; // the factorisation's info
    int32_t *gate;       // 0 when the factors are complete, else info
    int64_t n;
};

enum AdjKind : int32_t {
    AK_INIT = 0,  // waves, n units: row r of W (1 on the diagonal), J and adjT zeroed; unit 0 sets the gate
    AK_WPROD,     // workgroup: W sweep j = k, lane products
    AK_WFIN,      // waves: its tile finish
    AK_WONE,      // waves: W sweep j = k, one wave per element
    AK_S,         // one wave: S_n = 1, S_i = RZ(u_ii S_{i+1})
    AK_DIAGREC,   // waves, 2n units: adj(U)_ii (unit i) and the reciprocal of u_ii (unit n + i)
    AK_UPROD,     // workgroup: back substitution step k, lane products
    AK_UFIN,      // waves: its tile finish
    AK_UONE,      // waves: back substitution step k, one wave per element
    AK_UDIV,      // waves, n - k units: J_{k-1,j} / u_{k-1,k-1}
    AK_APROD,     // workgroup: accumulation step k, lane products
    AK_AFIN,      // waves: its tile finish
    AK_AONE,      // waves: accumulation step k, one wave per element
    AK_COUNT
};

__host__ __device__ inline bool adj_wg_kind(int kind) {
    return kind == AK_WPROD || kind == AK_UPROD || kind == AK_APROD;
}

// the rank-1 update of a family (W sweep, back substitution, accumulation) at step s
__host__ __device__ inline Rank1 adj_rank1(const AdjMat &M, int kind, int64_t s) {
    const int64_t n = M.n;
    if (kind == AK_WPROD || kind == AK_WFIN)  // x_r = W[r][j] (r >= j), y_i = l_ji (i < j), z = W[r][i]
        return Rank1{M.W, M.LU, M.W, s, s, 1, 0, s, 0, 0, 1, s, 0, n - s, s, 0};
    if (kind == AK_UPROD || kind == AK_UFIN)  // x_i = u_ik (i < k), y_j = J_kj (j >= k), z = J_ij
        return Rank1{M.LU, M.J, M.J, 0, s, 1, 0, s, s, 0, 1, 0, s, s, n - s, 0};
    // x_m = W_km, y_i = J_ik (negated: an addition), z = adjT_mi (m, i <= k)
    return Rank1{M.W, M.J, M.adjT, s, 0, 0, 1, 0, s, 1, 0, 0, 0, s + 1, s + 1, 1};
}

__global__ void __launch_bounds__(64 * kPersistWaves) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_persist_adj(const AdjMat *mats, const PersistRec *recs, const int64_t *pre, int64_t nrec, int64_t *done,
              int32_t *skipped, PersistCtl *ctl, int P, int64_t lds_wave, uint64_t limit) {
    extern __shared__ uint32_t lds_raw[];
    persist_queue(lds_raw, recs, pre, nrec, done, skipped, ctl, P, lds_wave, limit,
                  [&](const PersistRec &R, int64_t tk, int64_t base, uint32_t *lw, int P) {
        const AdjMat M = mats[R.mat];
        const int64_t k = R.k, n = M.n;
        switch (R.kind) {
            case AK_INIT:
                persist_wave_unit(base, R.units, [&](int64_t r) {
                    if (r == 0 && mpw::lane() == 0) *M.gate = factors_complete(*M.info, n) ? 0 : *M.info;
                    for (int64_t j = 0; j < n; ++j) {
                        const bool one = r == j;
                        uint32_t *w = el(M.W, r, j, P), *jm = el(M.J, r, j, P), *t = el(M.adjT, r, j, P);
                        for (int q = mpw::lane(); q < P; q += MP_WAVE) {
                            w[q] = (one && q == P - 1) ? 0x80000000u : 0u;
                            jm[q] = 0u;
                            t[q] = 0u;
                        }
                        if (mpw::lane() == 0) {
                            ex(M.W, r, j) = one ? 1 : 0;
                            sg(M.W, r, j) = 0;
                            ex(M.J, r, j) = 0;
                            sg(M.J, r, j) = 0;
                            ex(M.adjT, r, j) = 0;
                            sg(M.adjT, r, j) = 0;
                        }
                    }
                });
                break;
            case AK_WPROD:
            case AK_UPROD:
            case AK_APROD: prod_lane_body(lds_raw, adj_rank1(M, R.kind, k), M.T, M.gate, P, tk); break;
            case AK_WFIN:
            case AK_UFIN:
            case AK_AFIN: {
                const Rank1 R1 = adj_rank1(M, R.kind, k);
                persist_wave_unit(base, R.units, [&](int64_t u) {
                    if (*M.gate == 0) finish_tile_body(lw, R1, M.T, P, 0, R1.mr, u);
                });
                break;
            }
            case AK_WONE:
                persist_wave_unit(base, R.units, [&](int64_t u) { adj_w_body(lw, M.LU, M.W, M.gate, k, n, P, u); });
                break;
            case AK_S:
                persist_wave_unit(base, R.units, [&](int64_t) { adj_s_body(lw, M.LU, M.S, M.gate, n, P); });
                break;
            case AK_DIAGREC:
                persist_wave_unit(base, R.units, [&](int64_t u) {
                    if (u < n) adj_diag_body(lw, M.D, M.S, M.J, M.gate, P, u);
                    else adj_recip_body(lw, M.LU, M.rw, M.gate, P, u - n);
                });
                break;
            case AK_UONE:
                persist_wave_unit(base, R.units, [&](int64_t u) { adj_u_upd_body(lw, M.LU, M.J, M.gate, k, n, P, u); });
                break;
            case AK_UDIV:
                persist_wave_unit(base, R.units,
                                  [&](int64_t u) { adj_u_div_body(lw, M.LU, M.J, M.rw, M.gate, k, P, u); });
                break;
            case AK_AONE:
                persist_wave_unit(base, R.units, [&](int64_t u) { adj_prod_body(lw, M.J, M.W, M.adjT, M.gate, k, P, u); });
                break;
            default: break;
        }
    });
}

// after the backward's launch: status[b] = 0 (done), the factorisation's info
// (factors incomplete: adjT is zero), or -2 (a wait expired)
__global__ void k_persist_adj_end(const AdjMat *mats, const int32_t *skipped, int32_t *status, int64_t batch) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < batch && status) status[b] = skipped[b] ? -2 : *mats[b].gate;
}

// before the persistent launch: the queue head, the abort flag, the per-matrix
// counts and marks
__global__ void k_persist_begin(PersistCtl *ctl, int64_t *done, int32_t *skipped, int64_t batch) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b == 0) {
        ctl->head = 0;
        ctl->abort_flag = 0;
    }
    if (b < batch) {
        done[b] = 0;
        skipped[b] = 0;
    }
}

// after it: a matrix with a skipped ticket reports info = -2
__global__ void k_persist_end(const BatchMat *mats, const int32_t *skipped, int64_t batch) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < batch && skipped[b]) *mats[b].info = -2;
}

}  // namespace mpk
