// wave_mp.h -- wave-cooperative multiprecision arithmetic for gfx950.
//
// One 64-lane wavefront owns one multiprecision operation.  Operands live in
// LDS; lane t works on limbs t, t+64, t+128, ...  Carries and borrows between
// limbs are resolved with a carry-lookahead over the wave: per block of 64
// limbs each lane forms its generate/propagate bits, two ballots give 64-bit
// masks G and P, and the carry into every lane is read off the integer sum
// (G|P) + G + c_in (the carries of an addition whose generate and propagate
// vectors are G and P).  Every routine is called by all 64 lanes of a
// single-wave workgroup and returns wave-uniform results.
//
// Number format: value = (-1)^s * m * 2^(e - 32P), m with P limbs and the top
// bit set, zero = (m = 0, e = 0, s = 0).  Every result is RZ_p (truncation
// toward zero of the exact result).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MP_WAVE 64
// zero limbs on each side of the y operand of a product (covers r - a - 3 >= -66)
#define MP_YPAD 72

namespace mpw {

__device__ __forceinline__ int lane() { return (int)(threadIdx.x & 63u); }

// LDS and memory visibility between the lanes of one wave: the memory fences
// of a workgroup barrier without the barrier itself, so a wave can run these
// routines on its own while the other waves of its workgroup run something
// else (in a one-wave workgroup this is exactly __syncthreads()).
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

struct Hdr {
    int64_t e;
    int32_t s;
    bool zero;
};

__device__ __forceinline__ Hdr zero_hdr() { return Hdr{0, 0, true}; }

// ---------------------------------------------------------------------------
// limb vectors in LDS
// ---------------------------------------------------------------------------

__device__ __forceinline__ void fill(uint32_t *d, int n, uint32_t v) {
    for (int q = lane(); q < n; q += MP_WAVE) d[q] = v;
}

__device__ __forceinline__ void copy(uint32_t *d, const uint32_t *s, int n) {
    for (int q = lane(); q < n; q += MP_WAVE) d[q] = s[q];
}

// highest q < n with a[q] != 0, or -1
__device__ __forceinline__ int top_nonzero(const uint32_t *a, int n) {
    int best = -1;
    for (int q = lane(); q < n; q += MP_WAVE)
        if (a[q]) best = q;
    return __builtin_amdgcn_readfirstlane(wave_max(best));  // the same in every lane
}

// number of significant bits of a (0 when a == 0)
__device__ __forceinline__ int64_t bitlen(const uint32_t *a, int n) {
    int q = top_nonzero(a, n);
    if (q < 0) return 0;
    return 32LL * q + 32 - __clz(a[q]);
}

// d[0..nd) = floor(s * 2^sh) mod 2^(32 nd); sh < 0 shifts right.  d != s.
__device__ __forceinline__ void shift(uint32_t *d, int nd, const uint32_t *s, int ns, int64_t sh) {
    const int64_t hi_clamp = 32LL * (nd + 2), lo_clamp = -32LL * (ns + 2);
    if (sh > hi_clamp) sh = hi_clamp;
    if (sh < lo_clamp) sh = lo_clamp;
    for (int q = lane(); q < nd; q += MP_WAVE) {
        int64_t pos = 32LL * q - sh;  // bit of s that lands on bit 0 of d[q]
        int64_t w = pos >= 0 ? pos / 32 : -((-pos + 31) / 32);
        int b = (int)(pos - 32 * w);
        uint32_t lo = (w >= 0 && w < ns) ? s[w] : 0u;
        uint32_t hi = (w + 1 >= 0 && w + 1 < ns) ? s[w + 1] : 0u;
        d[q] = b ? ((lo >> b) | (hi << (32 - b))) : lo;
    }
}

// any bit of a below bit position `bits` set
__device__ __forceinline__ bool low_bits_nonzero(const uint32_t *a, int n, int64_t bits) {
    bool any = false;
    if (bits > 0) {
        int64_t w = bits / 32;
        int b = (int)(bits % 32);
        for (int q = lane(); q < n; q += MP_WAVE) {
            uint32_t v = a[q];
            if (q < w) any |= (v != 0u);
            else if (q == w && b) any |= ((v & ((1u << b) - 1u)) != 0u);
        }
    }
    return __ballot(any) != 0ull;
}

// carry/borrow into each lane of a 64-limb block from generate/propagate masks
__device__ __forceinline__ uint64_t lookahead(uint64_t G, uint64_t Pm, uint32_t cin) {
    uint64_t A = G | Pm;
    uint64_t S = A + G + (uint64_t)cin;
    return S ^ A ^ G;  // bit t = carry into lane t
}

__device__ __forceinline__ uint32_t block_carry_out(uint64_t G, uint64_t Pm, uint64_t C, int cnt) {
    if (cnt == 64) return (uint32_t)(((G >> 63) | ((Pm >> 63) & (C >> 63))) & 1ull);
    return (uint32_t)((C >> cnt) & 1ull);
}

// d = a + b + cin over n limbs; returns the carry out.  d may alias a or b.
__device__ __forceinline__ uint32_t add(uint32_t *d, const uint32_t *a, const uint32_t *b, int n,
                                        uint32_t cin) {
    uint32_t carry = cin;
    for (int base = 0; base < n; base += MP_WAVE) {
        int q = base + lane();
        int cnt = min(MP_WAVE, n - base);
        uint32_t x = q < n ? a[q] : 0u, y = q < n ? b[q] : 0u;
        uint32_t s = x + y;
        uint64_t valid = cnt == 64 ? ~0ull : ((1ull << cnt) - 1ull);
        uint64_t G = __ballot(s < x) & valid;
        uint64_t Pm = __ballot(s == 0xFFFFFFFFu) & valid;
        uint64_t C = lookahead(G, Pm, carry);
        if (q < n) d[q] = s + (uint32_t)((C >> lane()) & 1ull);
        carry = block_carry_out(G, Pm, C, cnt);
    }
    return carry;
}

// d = a - b - bin over n limbs; returns the borrow out.  d may alias a or b.
__device__ __forceinline__ uint32_t sub(uint32_t *d, const uint32_t *a, const uint32_t *b, int n,
                                        uint32_t bin) {
    uint32_t borrow = bin;
    for (int base = 0; base < n; base += MP_WAVE) {
        int q = base + lane();
        int cnt = min(MP_WAVE, n - base);
        uint32_t x = q < n ? a[q] : 0u, y = q < n ? b[q] : 0u;
        uint64_t valid = cnt == 64 ? ~0ull : ((1ull << cnt) - 1ull);
        uint64_t G = __ballot(x < y) & valid;
        uint64_t Pm = __ballot(x == y) & valid;
        uint64_t C = lookahead(G, Pm, borrow);
        if (q < n) d[q] = x - y - (uint32_t)((C >> lane()) & 1ull);
        borrow = block_carry_out(G, Pm, C, cnt);
    }
    return borrow;
}

// sign of a - b (n limbs each)
__device__ __forceinline__ int cmp(const uint32_t *a, const uint32_t *b, int n) {
    int best = -1;
    for (int q = lane(); q < n; q += MP_WAVE)
        if (a[q] != b[q]) best = q;
    best = wave_max(best);
    if (best < 0) return 0;
    return a[best] > b[best] ? 1 : -1;
}

// ---------------------------------------------------------------------------
// full product of two P-limb integers: prod[0..2P) = x * y
//   x: LDS, P limbs;  ypad: LDS, P + 2*MP_YPAD limbs with y at ypad + MP_YPAD
//   and zero limbs on each side;  t0..t3: LDS scratch of 2P limbs each.
// Lane t accumulates the product columns r = t, t+64, ... (96-bit sums of
// x[a] * y[r-a]); the columns are then folded into limbs by carry passes that
// never write a buffer they read.
// ---------------------------------------------------------------------------
// prod[0..ncols) = (x * y) mod 2^(32 ncols) for x of nx limbs and y of ny
// limbs (ncols <= nx + ny).  x: LDS; ypad: LDS, y at ypad + MP_YPAD with
// MP_YPAD zero limbs on each side; t0..t3: LDS scratch of ncols limbs each.
__device__ void mul_cols(uint32_t *prod, int ncols, const uint32_t *x, int nx, const uint32_t *ypad, int ny,
                         uint32_t *t0, uint32_t *t1, uint32_t *t2, uint32_t *t3) {
    const int R = ncols;
    const uint32_t *y = ypad + MP_YPAD;
    for (int base = 0; base < R; base += MP_WAVE) {
        const int r = base + lane();
        const int a0 = max(0, base - ny + 1), a1 = min(base + MP_WAVE - 1, nx - 1);
        // two independent 96-bit accumulators break the add dependency chain
        uint64_t acc0 = 0, acc1 = 0;
        uint32_t hi0 = 0, hi1 = 0;
        int a = a0;
        for (; a + 3 <= a1; a += 4) {
            uint4 xv, yv;  // x[a..a+3] (same for all lanes), y[r-a-3 .. r-a]
            __builtin_memcpy(&xv, x + a, 16);
            __builtin_memcpy(&yv, y + (r - a - 3), 16);
            uint64_t p0 = (uint64_t)xv.x * yv.w, p1 = (uint64_t)xv.y * yv.z;
            uint64_t p2 = (uint64_t)xv.z * yv.y, p3 = (uint64_t)xv.w * yv.x;
            acc0 += p0;
            hi0 += acc0 < p0;
            acc1 += p1;
            hi1 += acc1 < p1;
            acc0 += p2;
            hi0 += acc0 < p2;
            acc1 += p3;
            hi1 += acc1 < p3;
        }
        for (; a <= a1; ++a) {
            uint64_t pr = (uint64_t)x[a] * (uint64_t)y[r - a];
            acc0 += pr;
            hi0 += acc0 < pr;
        }
        uint64_t acc = acc0 + acc1;
        uint32_t acc_hi = hi0 + hi1 + (acc < acc0 ? 1u : 0u);
        if (r < R) {
            t0[r] = (uint32_t)acc;
            t1[r] = (uint32_t)(acc >> 32);
            t2[r] = acc_hi;
        }
    }
    wsync();
    // column r holds t0 + t1*2^32 + t2*2^64; v_r = t0_r + t1_{r-1} + t2_{r-2} < 3*2^32
    for (int r = lane(); r < R; r += MP_WAVE) {
        uint64_t v = (uint64_t)t0[r] + (r >= 1 ? t1[r - 1] : 0u) + (r >= 2 ? t2[r - 2] : 0u);
        prod[r] = (uint32_t)v;
        t3[r] = (uint32_t)(v >> 32);
    }
    wsync();
    // w_r = (v_r mod 2^32) + (v_{r-1} >> 32) <= 2^32 + 1; its carry bit goes one limb up
    for (int r = lane(); r < R; r += MP_WAVE) {
        uint64_t w = (uint64_t)prod[r] + (r >= 1 ? t3[r - 1] : 0u);
        prod[r] = (uint32_t)w;
        t0[r] = (uint32_t)(w >> 32);
    }
    wsync();
    for (int r = lane(); r < R; r += MP_WAVE) t1[r] = r >= 1 ? t0[r - 1] : 0u;
    wsync();
    add(prod, prod, t1, R, 0u);
    wsync();
}


// ---------------------------------------------------------------------------
// Teams: the waves of one workgroup forming the products of one operation
// together.  Wave 0 runs the operation as a single wave would; for each
// windowed product (mul_win) it posts the arguments in an LDS command block,
// and waves 1..nw-1, waiting in team_serve, join it: every wave converts its
// share of the digits and takes the rounds of 64 windows whose index is its
// own modulo nw.  Which wave forms a window does not change its bits.  The
// waves meet at team barriers (an LDS arrival counter); every wait is
// bounded by wall-clock time (the caller's limit), and a wait that runs out
// sets `fail` (which every later wait sees at once), so a lost wave cannot
// hang the launch.
// Wave 0 posts and waits only in uniform control flow and closes the team
// (team_close) on every path.
// ---------------------------------------------------------------------------
struct TeamCtl {
    uint32_t seq;   // commands posted
    uint32_t op;    // 1: a product, 0: close
    uint32_t bar;   // arrivals at team barriers (two per product)
    uint32_t fail;  // a wait ran out
    int32_t ncols, nx, ny, wlo;
    uint64_t prod, x, y, ws;  // LDS addresses of the product's operands
    uint64_t limit;           // bound on each wait, in wall-clock ticks
};

__device__ __forceinline__ int team_size() { return (int)(blockDim.x / MP_WAVE); }
__device__ __forceinline__ int team_wave() { return (int)__builtin_amdgcn_readfirstlane(threadIdx.x / MP_WAVE); }

__device__ __forceinline__ uint32_t team_read(const uint32_t *p) {
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
}

// wait until *p - v >= 0 (mod 2^32); false when it, or an earlier wait, ran out
__device__ __forceinline__ bool team_wait(TeamCtl *c, const uint32_t *p, uint32_t v) {
    if (team_read(&c->fail) != 0u) return false;
    if ((int32_t)(team_read(p) - v) >= 0) return true;
    const uint32_t *lw = (const uint32_t *)&c->limit;
    const uint64_t limit = ((uint64_t)team_read(lw + 1) << 32) | team_read(lw);
    const uint64_t t0 = wall_clock64();
    for (;;) {
        if (wall_clock64() - t0 >= limit) {
            if (lane() == 0) __hip_atomic_store(&c->fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
        if ((int32_t)(team_read(p) - v) >= 0) return true;
        if (team_read(&c->fail) != 0u) return false;
    }
}

// the team barrier that completes when the arrival count reaches `target`:
// every wave's LDS writes before it are visible to every wave after it
__device__ __forceinline__ void team_bar(TeamCtl *c, uint32_t target) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane() == 0) __hip_atomic_fetch_add(&c->bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    (void)team_wait(c, &c->bar, target);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// every wave, at the start of the kernel: the team is the whole workgroup;
// limit bounds each wait (wall-clock ticks; 0: any wait not already
// satisfied runs out)
__device__ __forceinline__ void team_open(TeamCtl *c, uint64_t limit) {
    if (threadIdx.x == 0) {
        c->seq = 0u;
        c->op = 0u;
        c->bar = 0u;
        c->fail = 0u;
        c->limit = limit;
    }
    __syncthreads();
}

// wave 0: post a command (op 1 with a product's arguments, op 0: close);
// returns its number (1, 2, ...)
__device__ __forceinline__ uint32_t team_post(TeamCtl *c, uint32_t op, uint32_t *prod, int ncols, const uint32_t *x,
                                              int nx, const uint32_t *y, int ny, uint32_t *ws, int wlo) {
    const uint32_t cmd = team_read(&c->seq) + 1u;  // wave 0 is the only writer
    if (lane() == 0) {
        c->op = op;
        c->ncols = ncols;
        c->nx = nx;
        c->ny = ny;
        c->wlo = wlo;
        c->prod = (uint64_t)(uintptr_t)prod;
        c->x = (uint64_t)(uintptr_t)x;
        c->y = (uint64_t)(uintptr_t)y;
        c->ws = (uint64_t)(uintptr_t)ws;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane() == 0) __hip_atomic_store(&c->seq, cmd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return cmd;
}

// wave 0, on every path: release the other waves; true when no wait ran out
__device__ __forceinline__ bool team_close(TeamCtl *c) {
    if (team_size() > 1) (void)team_post(c, 0u, nullptr, 0, nullptr, 0, nullptr, 0, nullptr, 0);
    return team_read(&c->fail) == 0u;
}

// ---------------------------------------------------------------------------
// The same product in radix 2^28 with register windows (the form every
// product of a few dozen limbs or more takes).  Both operands are cut into
// 28-bit digits in LDS, so a digit product is below 2^56 and one
// v_mad_u64_u32 adds it into a 64-bit column sum; every 128 steps the sums
// fold their bits above 28 into a second word, so they never overflow.
// Lane t owns a window of 8 consecutive digit columns r0 = 8w .. 8w+7 (64
// windows per round) and forms them by columns (Comba): at step a it adds
// x_a * y_{r0+c-a} for c = 0..7, where x_a is the same for every lane (a
// broadcast LDS read) and the y digits come from a 16-register ring that
// moves by one digit per step -- y is stored reversed, so one aligned 16-byte
// read brings the digits of four steps, issued one group of four steps
// ahead.  The steps of a round run over the union of its windows' ranges;
// digits outside y read as zero (the read index is clamped into zero guard
// words).  A window's column sums are carried into 8 digits plus a carry
// (224 + 41 bits), i.e. 7 whole limbs and two overlapping the next window:
// the 7 go to prod, the 2 to an overflow vector, and one carry-lookahead
// addition merges the two.  Needs the scratch words mul_win_words()
// reports; callers fall back to mul_cols where they do not fit.
// ---------------------------------------------------------------------------
constexpr uint32_t kDigMask = (1u << 28) - 1u;

// bits [28d, 28d + 28) of the n-limb integer a
__device__ __forceinline__ uint32_t digit_of(const uint32_t *a, int n, int d) {
    const int bit = 28 * d, q = bit >> 5, sh = bit & 31;
    uint32_t v = (q < n ? a[q] : 0u) >> sh;
    if (sh > 4) v |= (q + 1 < n ? a[q + 1] : 0u) << (32 - sh);
    return v & kDigMask;
}

// WinGeom(ncols, nx, ny).words(), also on the host
__host__ __device__ constexpr int win_words(int ncols, int nx, int ny) {
    const int nc = (32 * ncols + 27) / 28;
    const int nxd = (32 * nx + 27) / 28 < nc ? (32 * nx + 27) / 28 : nc;
    const int nyd = (32 * ny + 27) / 28 < nc ? (32 * ny + 27) / 28 : nc;
    return 3 + ((ncols + 3) & ~3) + ((nxd + 15 + 3) & ~3) + ((nyd + 3 + 3) & ~3) + 8;
}

struct WinGeom {
    int NC, NXd, NYd, W;   // digit columns, digits of x and y taken, windows
    int ov, dx, K, len;    // words: overflow vector, x digits, reversed y (DYR[K - b] = y_b), its length
    __device__ WinGeom(int ncols, int nx, int ny) {
        NC = (32 * ncols + 27) / 28;
        NXd = min((32 * nx + 27) / 28, NC);
        NYd = min((32 * ny + 27) / 28, NC);
        W = (NC + 7) / 8;
        ov = (ncols + 3) & ~3;
        dx = (NXd + 15 + 3) & ~3;       // the last block's x reads end below NXd + 15
        K = (NYd + 3 + 3) & ~3;         // at least 4 zero words below y's lowest stored digit
        len = K + 8;                    // and 7 above its highest
    }
    __device__ int words() const { return 3 + ov + dx + len; }  // 3: 16-byte alignment of the base
};

// One wave's share of the windowed product (tm == nullptr: all of it): the
// digits t with t / 64 = wv mod nw, then the rounds of 64 windows from window
// wlo on with the same property; it leaves the window limbs in prod and the
// overflow vector at the aligned start of ws.  cmd: the product's command
// number (team barriers 2 cmd - 1 and 2 cmd).
__device__ __forceinline__ void mul_win_part(uint32_t *prod, int ncols, const uint32_t *x, int nx, const uint32_t *y,
                                             int ny, uint32_t *ws, TeamCtl *tm, uint32_t cmd, int wlo) {
    const WinGeom g(ncols, nx, ny);
    const int nw = tm ? team_size() : 1, wv = tm ? team_wave() : 0;
    uint32_t *base = (uint32_t *)(((uintptr_t)ws + 15u) & ~(uintptr_t)15u);
    uint32_t *OV = base, *DX = base + g.ov, *DY = DX + g.dx;
    for (int t = wv * MP_WAVE + lane(); t < g.dx; t += nw * MP_WAVE) DX[t] = t < g.NXd ? digit_of(x, nx, t) : 0u;
    for (int t = wv * MP_WAVE + lane(); t < g.len; t += nw * MP_WAVE) {
        const int b = g.K - t;
        DY[t] = (b >= 0 && b < g.NYd) ? digit_of(y, ny, b) : 0u;
    }
    if (tm) team_bar(tm, (2u * cmd - 1u) * (uint32_t)nw);
    else wsync();
    // a 16-byte read DY[t..t+3] with t clamped into [lo_c, hi_c]: outside
    // that range every digit it stands for is zero, and so are the clamped words
    const int lo_c = ((g.K - g.NYd + 1) & ~3) - 4, hi_c = g.K + 4;
    for (int w0 = wlo + wv * MP_WAVE; w0 < g.W; w0 += nw * MP_WAVE) {
        const int w = w0 + lane();
        const int r0 = 8 * w;
        const int wl = min(g.W, w0 + MP_WAVE) - 1;
        const int A0 = max(0, 8 * w0 - g.NYd + 1) & ~15;
        const int A1 = min(g.NXd - 1, 8 * wl + 7);
        const int nblocks = A1 >= A0 ? (A1 - A0 + 16) / 16 : 0;
        uint64_t acc[8], hi[8];
        uint32_t ring[16];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = hi[c] = 0;
        auto load4 = [&](int slot, int a) {
            int t = g.K - r0 + a;
            t = min(max(t, lo_c), hi_c);
            const uint4 v = *(const uint4 *)(DY + t);
            ring[slot] = v.x;
            ring[slot + 1] = v.y;
            ring[slot + 2] = v.z;
            ring[slot + 3] = v.w;
        };
        // the digit of step j is y_{r0 - j}, kept in slot (j - A0) mod 16
        load4(8, A0 - 8);
        load4(12, A0 - 4);
        load4(0, A0);
#pragma unroll 1
        for (int blk = 0; blk < nblocks; ++blk) {
            const int a0 = A0 + 16 * blk;
            const uint4 *xq = (const uint4 *)(DX + a0);
            const uint4 xv0 = xq[0], xv1 = xq[1], xv2 = xq[2], xv3 = xq[3];
            const uint32_t xs[16] = {xv0.x, xv0.y, xv0.z, xv0.w, xv1.x, xv1.y, xv1.z, xv1.w,
                                     xv2.x, xv2.y, xv2.z, xv2.w, xv3.x, xv3.y, xv3.z, xv3.w};
#pragma unroll
            for (int gq = 0; gq < 4; ++gq) {
                load4(((gq + 1) & 3) * 4, a0 + 4 * gq + 4);  // the next group's digits
#pragma unroll
                for (int u4 = 0; u4 < 4; ++u4) {
                    const int u = 4 * gq + u4;
#pragma unroll
                    for (int c = 0; c < 8; ++c) acc[c] += (uint64_t)xs[u] * (uint64_t)ring[(u - c) & 15];
                }
            }
            if ((blk & 7) == 7) {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    hi[c] += acc[c] >> 28;
                    acc[c] &= kDigMask;
                }
            }
        }
        if (w < g.W) {
            uint32_t d[8];
            uint64_t carry = 0;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const uint64_t sm = acc[c] + carry;
                d[c] = (uint32_t)sm & kDigMask;
                carry = (sm >> 28) + hi[c];
            }
            const uint32_t L[9] = {d[0] | (d[1] << 28),         (d[1] >> 4) | (d[2] << 24),
                                   (d[2] >> 8) | (d[3] << 20),  (d[3] >> 12) | (d[4] << 16),
                                   (d[4] >> 16) | (d[5] << 12), (d[5] >> 20) | (d[6] << 8),
                                   (d[6] >> 24) | (d[7] << 4),  (uint32_t)carry,
                                   (uint32_t)(carry >> 32)};
            const int q0 = 7 * w;
#pragma unroll
            for (int i = 0; i < 7; ++i)
                if (q0 + i < ncols) prod[q0 + i] = L[i];
#pragma unroll
            for (int i = 2; i < 9; ++i)
                if (q0 + i < ncols) OV[q0 + i] = i >= 7 ? L[i] : 0u;
            if (w == wlo) {  // nothing carries in from below the first window
                OV[q0] = 0u;
                if (q0 + 1 < ncols) OV[q0 + 1] = 0u;
            }
        }
    }
    if (tm) team_bar(tm, 2u * cmd * (uint32_t)nw);
    else wsync();
}

// the waves of team tm (nullptr: this wave alone) form it; called by wave 0.
// wlo > 0 (7 wlo < ncols): only the digit columns from 8 wlo on are formed, so
// limbs 7 wlo .. ncols - 1 of prod hold (x y - E) / 2^(224 wlo) mod
// 2^(32 (ncols - 7 wlo)) for the dropped part 0 <= E < 2^(224 wlo) m 2^56
// (m: digits of the shorter operand), and limbs below 7 wlo are left as they
// are.
__device__ __forceinline__ void mul_win(uint32_t *prod, int ncols, const uint32_t *x, int nx, const uint32_t *y, int ny,
                        uint32_t *ws, TeamCtl *tm = nullptr, int wlo = 0) {
    uint32_t cmd = 0u;
    if (tm != nullptr && team_size() > 1) cmd = team_post(tm, 1u, prod, ncols, x, nx, y, ny, ws, wlo);
    else tm = nullptr;
    mul_win_part(prod, ncols, x, nx, y, ny, ws, tm, cmd, wlo);
    uint32_t *OV = (uint32_t *)(((uintptr_t)ws + 15u) & ~(uintptr_t)15u);
    add(prod + 7 * wlo, prod + 7 * wlo, OV + 7 * wlo, ncols - 7 * wlo, 0u);
    wsync();
}

// waves 1..nw-1 of a team: join wave 0's products until it closes the team
__device__ __forceinline__ void team_serve(TeamCtl *c) {
    uint32_t seen = 0u;
    for (;;) {
        if (!team_wait(c, &c->seq, seen + 1u)) return;
        seen += 1u;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (team_read(&c->op) == 0u) return;
        auto ptr = [&](const uint64_t *f) -> uint32_t * {
            const uint32_t *w = (const uint32_t *)f;
            return (uint32_t *)(uintptr_t)(((uint64_t)team_read(w + 1) << 32) | team_read(w));
        };
        const int ncols = (int)team_read((const uint32_t *)&c->ncols);
        const int nx = (int)team_read((const uint32_t *)&c->nx);
        const int ny = (int)team_read((const uint32_t *)&c->ny);
        const int wlo = (int)team_read((const uint32_t *)&c->wlo);
        mul_win_part(ptr(&c->prod), ncols, ptr(&c->x), nx, ptr(&c->y), ny, ptr(&c->ws), c, seen, wlo);
    }
}

// prod[0..ncols) = (x * y) mod 2^(32 ncols); t0..t3 are one contiguous
// scratch block of 4 * tsz words (the layouts in use place them so).
// wlo: as for mul_win (the column form forms every column, which is always
// allowed)
__device__ __forceinline__ void mul_gen(uint32_t *prod, int ncols, const uint32_t *x, int nx, const uint32_t *ypad,
                                        int ny, uint32_t *t0, uint32_t *t1, uint32_t *t2, uint32_t *t3, int tsz,
                                        TeamCtl *tm = nullptr, int wlo = 0) {
    if (WinGeom(ncols, nx, ny).words() <= 4 * tsz && ncols >= 16)
        mul_win(prod, ncols, x, nx, ypad + MP_YPAD, ny, t0, tm, wlo);
    else
        mul_cols(prod, ncols, x, nx, ypad, ny, t0, t1, t2, t3);
}

// prod[0..2P) = x * y for two P-limb integers
__device__ __forceinline__ void mul_full(uint32_t *prod, const uint32_t *x, const uint32_t *ypad, int P,
                                         uint32_t *t0, uint32_t *t1, uint32_t *t2, uint32_t *t3, TeamCtl *tm = nullptr) {
    mul_gen(prod, 2 * P, x, P, ypad, P, t0, t1, t2, t3, 2 * P + 2, tm);
}

// place n limbs of src as the y operand of mul_gen (zero pads around)
__device__ __forceinline__ void set_y(uint32_t *ypad, const uint32_t *src, int n, int cap) {
    for (int q = lane(); q < cap + 2 * MP_YPAD; q += MP_WAVE) {
        int k = q - MP_YPAD;
        ypad[q] = (k >= 0 && k < n) ? src[k] : 0u;
    }
}

// Scratch for the number routines: every buffer is in LDS.
struct Scratch {
    uint32_t *x;     // P
    uint32_t *ypad;  // P + 2*MP_YPAD
    uint32_t *prod;  // 2P + 2
    uint32_t *t0, *t1, *t2, *t3;  // 2P + 2 each
    TeamCtl *team = nullptr;         // the waves that form the products with this one
};

// Copy n limbs global -> LDS.  Lanes move 16-byte chunks when both sides
// allow it (n % 4 == 0 and 16-byte aligned addresses); all of a lane's loads
// are issued before its LDS stores.
__device__ __forceinline__ void gload(uint32_t *dst, const uint32_t *src, int n) {
    if ((n & 3) == 0 && (((uintptr_t)src | (uintptr_t)dst) & 15u) == 0) {
        const int nc = n >> 2;
        const uint4 *s4 = (const uint4 *)src;
        uint4 *d4 = (uint4 *)dst;
        int c = lane();
        for (; c + 3 * MP_WAVE < nc; c += 4 * MP_WAVE) {
            uint4 v0 = s4[c], v1 = s4[c + MP_WAVE], v2 = s4[c + 2 * MP_WAVE], v3 = s4[c + 3 * MP_WAVE];
            d4[c] = v0;
            d4[c + MP_WAVE] = v1;
            d4[c + 2 * MP_WAVE] = v2;
            d4[c + 3 * MP_WAVE] = v3;
        }
        for (; c < nc; c += MP_WAVE) d4[c] = s4[c];
    } else {
        for (int q = lane(); q < n; q += MP_WAVE) dst[q] = src[q];
    }
}

__device__ __forceinline__ void gstore(uint32_t *dst, const uint32_t *src, int n) {
    if ((n & 3) == 0 && (((uintptr_t)src | (uintptr_t)dst) & 15u) == 0) {
        const int nc = n >> 2;
        const uint4 *s4 = (const uint4 *)src;
        uint4 *d4 = (uint4 *)dst;
        for (int c = lane(); c < nc; c += MP_WAVE) d4[c] = s4[c];
    } else {
        for (int q = lane(); q < n; q += MP_WAVE) dst[q] = src[q];
    }
}

// load a number from global memory into LDS (P limbs); returns its header
__device__ __forceinline__ Hdr load(uint32_t *dst, const uint32_t *src, int64_t e, int32_t s, int P) {
    gload(dst, src, P);
    wsync();
    const bool z = __builtin_amdgcn_readfirstlane(dst[P - 1]) == 0u;
    return z ? zero_hdr() : Hdr{e, s, false};
}

__device__ __forceinline__ void store(uint32_t *dst_limbs, int64_t *dst_e, int32_t *dst_s,
                                      const uint32_t *src, Hdr h, int P) {
    if (h.zero) {
        for (int q = lane(); q < P; q += MP_WAVE) dst_limbs[q] = 0u;
    } else {
        gstore(dst_limbs, src, P);
    }
    if (lane() == 0) {
        *dst_e = h.zero ? 0 : h.e;
        *dst_s = h.zero ? 0 : h.s;
    }
}

// out = RZ_p(x * y).  x in sc.x, y in sc.ypad + MP_YPAD (pads must be zero).
__device__ Hdr mul(uint32_t *out, Hdr hx, Hdr hy, int P, const Scratch &sc) {
    if (hx.zero || hy.zero) return zero_hdr();
    mul_full(sc.prod, sc.x, sc.ypad, P, sc.t0, sc.t1, sc.t2, sc.t3, sc.team);
    int top = (int)(sc.prod[2 * P - 1] >> 31);
    shift(out, P, sc.prod, 2 * P, -(32LL * P - 1 + top));
    wsync();
    return Hdr{hx.e + hy.e - 1 + top, hx.s ^ hy.s, false};
}

// Normalise the (n)-limb integer G (value G * 2^(scale)) to P limbs: RZ_p.
__device__ __forceinline__ Hdr normalise(uint32_t *out, const uint32_t *G, int n, int64_t scale,
                                         int32_t sign, int P) {
    int64_t L = bitlen(G, n);
    if (L == 0) return zero_hdr();
    shift(out, P, G, n, 32LL * P - L);
    wsync();
    return Hdr{scale + L, sign, false};
}

// out = RZ_p(x + y) for signed x (LDS, P limbs) and y (LDS, P limbs).
// G, Y2: LDS scratch of P + 2 limbs.  out must differ from x, y, G, Y2.
//
// With X the operand of larger exponent (larger magnitude when the exponents
// are equal and the signs differ) and d = e_X - e_Y:
//  * same signs:      G = m_X + floor(m_Y / 2^d)                (scale e_X - p)
//  * opposite, d<=1:  G = m_X 2^d - m_Y, exact                  (scale e_X - d - p)
//  * opposite, d>=2:  G = 4 m_X - ceil(m_Y / 2^(d-2))            (scale e_X - 2 - p)
// then RZ_p(G * 2^scale).  Truncating a sum never needs the dropped bits of Y;
// for a difference the two guard bits and the ceiling (sticky) give the exact
// truncation because the result keeps at least p+1 bits of G.
__device__ Hdr addsub(uint32_t *out, const uint32_t *xm, Hdr hx, const uint32_t *ym, Hdr hy,
                      uint32_t *G, uint32_t *Y2, int P) {
    if (hy.zero) {
        if (hx.zero) return zero_hdr();
        copy(out, xm, P);
        wsync();
        return hx;
    }
    if (hx.zero) {
        copy(out, ym, P);
        wsync();
        return hy;
    }
    const bool subtract = hx.s != hy.s;
    bool swap = hy.e > hx.e;
    if (subtract && hx.e == hy.e) swap = cmp(ym, xm, P) > 0;
    const uint32_t *X = swap ? ym : xm;
    const uint32_t *Y = swap ? xm : ym;
    const Hdr hX = swap ? hy : hx, hY = swap ? hx : hy;
    const uint64_t d = (uint64_t)hX.e - (uint64_t)hY.e;
    const int n = P + 1;
    int64_t g;
    if (!subtract) {
        g = 0;
        shift(G, n, X, P, 0);
        shift(Y2, n, Y, P, -(int64_t)(d > (uint64_t)(32 * P + 64) ? (uint64_t)(32 * P + 64) : d));
        wsync();
        add(G, G, Y2, n, 0u);
    } else if (d <= 1) {
        g = (int64_t)d;
        shift(G, n, X, P, g);
        shift(Y2, n, Y, P, 0);
        wsync();
        sub(G, G, Y2, n, 0u);
    } else {
        g = 2;
        const uint64_t dm2 = d - 2;
        const int64_t rs = (int64_t)(dm2 > (uint64_t)(32 * P + 64) ? (uint64_t)(32 * P + 64) : dm2);
        shift(G, n, X, P, 2);
        shift(Y2, n, Y, P, -rs);
        bool sticky = low_bits_nonzero(Y, P, rs);
        wsync();
        sub(G, G, Y2, n, sticky ? 1u : 0u);
    }
    wsync();
    return normalise(out, G, n, hX.e - g - 32LL * P, hX.s, P);
}

// floor(num / v1) for v1 >= 2^31 and num < v1 * 2^32: a float64 estimate
// (error below one unit) fixed up with exact 64-bit remainders.
__device__ __forceinline__ uint64_t udiv_2by1(uint64_t num, uint32_t v1) {
    uint64_t q = (uint64_t)((double)num / (double)v1);
    if (q > 0xFFFFFFFFull) q = 0xFFFFFFFFull;
    int64_t r = (int64_t)(num - q * (uint64_t)v1);
    while (r < 0) {
        q--;
        r += v1;
    }
    while (r >= (int64_t)v1) {
        q++;
        r -= v1;
    }
    return q;
}

// out = RZ_p(a / b), b != 0 with its top bit set.
// Knuth's Algorithm D in base 2^32 on U = m_a * 2^(p+1) (2P+1 limbs, plus a
// zero limb on top) and V = m_b (already normalised); the quotient Q has
// p+1 or p+2 bits and is truncated to p bits.  Per quotient digit the
// remainder window U[j..j+P] -= qhat * V runs block by block: lane t owns
// window limbs t, t+64, ...; the product's high words and the first-stage
// borrows (0..2) move one limb up by lane shuffles, and the remaining 1-bit
// borrows are resolved by the ballot lookahead.  One LDS barrier per digit.
//   U: LDS 2P+2 limbs; LO, HI: unused (kept for the layout); Q: LDS P+2 limbs.
__device__ Hdr div(uint32_t *out, const uint32_t *am, Hdr ha, const uint32_t *bm, Hdr hb,
                   uint32_t *U, uint32_t *LO, uint32_t *HI, uint32_t *Q, int P) {
    (void)LO;
    (void)HI;
    if (ha.zero) return zero_hdr();
    const int m = 2 * P + 1;
    const int n1 = P + 1;  // window limbs
    const int S = (n1 + MP_WAVE - 1) / MP_WAVE;
    shift(U, m + 1, am, P, 32LL * P + 1);
    fill(Q, P + 2, 0u);
    wsync();
    const uint64_t B = 1ull << 32;
    const uint32_t v1 = bm[P - 1], v2 = bm[P - 2];
    for (int j = m - P; j >= 0; --j) {
        const uint32_t u2 = U[j + P], u1 = U[j + P - 1], u0 = U[j + P - 2];
        const uint64_t num = ((uint64_t)u2 << 32) | u1;
        uint64_t qhat, rhat;
        if (u2 >= v1) {
            qhat = B - 1;
            rhat = num - qhat * v1;
        } else {
            qhat = udiv_2by1(num, v1);
            rhat = num - qhat * v1;
        }
        while (rhat < B && qhat * v2 > ((rhat << 32) | u0)) {
            qhat--;
            rhat += v1;
        }
        if (qhat) {
            uint32_t hi_in = 0, b1_in = 0, b2_in = 0;  // entering lane 0 of a block
            uint32_t neg = 0;
#pragma unroll 1
            for (int s = 0; s < S; ++s) {
                {
                    const int q = s * MP_WAVE + lane();
                    const int cnt = min(MP_WAVE, n1 - s * MP_WAVE);
                    const uint64_t pr = qhat * (uint64_t)(q < P ? bm[q] : 0u);
                    const uint32_t lo = (uint32_t)pr, hi = (uint32_t)(pr >> 32);
                    uint32_t hi_prev = __shfl_up(hi, 1);
                    if (lane() == 0) hi_prev = hi_in;
                    const uint32_t u = q < n1 ? U[j + q] : 0u;
                    const int64_t diff = (int64_t)u - (int64_t)lo - (int64_t)hi_prev;
                    const uint32_t limb = (uint32_t)diff;
                    const uint32_t b1 = (uint32_t)(-(diff >> 32));  // 0, 1 or 2
                    uint32_t b1_prev = __shfl_up(b1, 1);
                    if (lane() == 0) b1_prev = b1_in;
                    const int64_t t = (int64_t)limb - (int64_t)b1_prev;
                    const uint32_t limb2 = (uint32_t)t;
                    const bool gb = t < 0;
                    const uint64_t valid = cnt == 64 ? ~0ull : ((1ull << cnt) - 1ull);
                    const uint64_t G = __ballot(gb) & valid;
                    const uint64_t Pm = __ballot(!gb && limb2 == 0u) & valid;
                    const uint64_t C = lookahead(G, Pm, b2_in);
                    const uint32_t cin = (uint32_t)((C >> lane()) & 1ull);
                    if (q < n1) U[j + q] = limb2 - cin;
                    b2_in = block_carry_out(G, Pm, C, cnt);
                    hi_in = __shfl(hi, cnt - 1);
                    b1_in = __shfl(b1, cnt - 1);
                }
            }
            // the top window limb's first-stage borrow and the chain's borrow
            // leave the window: the difference is negative
            neg = b1_in + b2_in;
            wsync();
            if (neg) {
                qhat--;
                uint32_t carry = 0;
#pragma unroll 1
                for (int s = 0; s < S; ++s) {
                    {
                        const int q = s * MP_WAVE + lane();
                        const int cnt = min(MP_WAVE, n1 - s * MP_WAVE);
                        const uint32_t x = q < n1 ? U[j + q] : 0u, y = q < P ? bm[q] : 0u;
                        const uint32_t sm = x + y;
                        const uint64_t valid = cnt == 64 ? ~0ull : ((1ull << cnt) - 1ull);
                        const uint64_t G = __ballot(sm < x) & valid;
                        const uint64_t Pm = __ballot(sm == 0xFFFFFFFFu) & valid;
                        const uint64_t C = lookahead(G, Pm, carry);
                        if (q < n1) U[j + q] = sm + (uint32_t)((C >> lane()) & 1ull);
                        carry = block_carry_out(G, Pm, C, cnt);
                    }
                }
                wsync();
            }
        }
        if (lane() == 0) Q[j] = (uint32_t)qhat;
    }
    wsync();
    return normalise(out, Q, P + 2, ha.e - hb.e - 32LL * P - 1, ha.s ^ hb.s, P);
}

// ---------------------------------------------------------------------------
// Division through one shared reciprocal.
//
// recip(): R = floor(2^(2p) / v) for v of P limbs with its top bit set.
// Newton's iteration X <- X + X (1 - V X) on scaled integers: X_f ~ 2^(p+f)/v
// carries f bits; one step goes from f to f' = min(2f - 8, p) using the top
// g = f' + 16 bits of v:  T = V_g X_f ~ 2^(f+g)(1 - eps),  e = 2^(f+g) - T,
// X_f' = X_f 2^(f'-f) + floor(X_f e / 2^(2f+g-f')).  The seed (f = 48) comes
// from a float64 quotient of the top 64 bits of v.  The result is then made
// exact by the remainder E = 2^(2p) - v R (R moves by one while E < 0 or
// E >= v).  Correctness rests only on this final exact check; the error
// analysis (about 8 units left) only bounds its trip count.  Returns false
// when the correction did not settle within the bound (callers then fall back
// to long division).
// ---------------------------------------------------------------------------
struct DivBufs {
    uint32_t *x;     // P + 4
    uint32_t *ypad;  // P + 4 + 2*MP_YPAD
    uint32_t *prod;  // 2P + 4
    uint32_t *t0, *t1, *t2, *t3;  // 2P + 4 each
    uint32_t *a;     // P + 4
    uint32_t *v;     // P + 4
    TeamCtl *team = nullptr;  // the waves that form the products with this one
};

__host__ __device__ constexpr size_t div_lds_limbs(int P) { return (size_t)(14 * P + 2 * MP_YPAD + 36); }

__device__ __forceinline__ DivBufs div_bufs(uint32_t *base, int P) {
    DivBufs b;
    b.x = base;
    b.ypad = b.x + P + 4;
    b.prod = b.ypad + P + 4 + 2 * MP_YPAD;
    b.t0 = b.prod + 2 * P + 4;
    b.t1 = b.t0 + 2 * P + 4;
    b.t2 = b.t1 + 2 * P + 4;
    b.t3 = b.t2 + 2 * P + 4;
    b.a = b.t3 + 2 * P + 4;
    b.v = b.a + P + 4;
    return b;
}

__device__ __forceinline__ int limbs_for_bits(int64_t bits) { return (int)((bits + 31) / 32); }

// v must be in B.v (P limbs, top bit set); R (P + 1 limbs) is written to B.x.
__device__ bool recip(const DivBufs &B, int P) {
    const int64_t p = 32LL * P;
    // seed: X_48 ~ 2^(p+48) / v = 2^112 / (top 64 bits of v)
    if (lane() == 0) {
        const uint64_t vt = ((uint64_t)B.v[P - 1] << 32) | B.v[P - 2];
        const double q = 5192296858534827628530496329220096.0 / (double)vt;  // 2^112 / vt
        const uint64_t X0 = (uint64_t)q;
        B.x[0] = (uint32_t)X0;
        B.x[1] = (uint32_t)(X0 >> 32);
    }
    wsync();
    int64_t f = 48;
    int nX = 2;
    while (f < p) {
        const int64_t f2 = min(2 * f - 8, p);
        const int64_t gb = f2 + 16;
        const int nV = limbs_for_bits(gb) + 1;
        // V_g = floor(v * 2^(g - p)) into ypad (as the y operand)
        shift(B.ypad + MP_YPAD, nV, B.v, P, gb - p);
        for (int q = lane(); q < MP_YPAD; q += MP_WAVE) {
            B.ypad[q] = 0u;
            B.ypad[MP_YPAD + nV + q] = 0u;
        }
        wsync();
        const int nT = nV + nX;
        mul_gen(B.prod, nT, B.x, nX, B.ypad, nV, B.t0, B.t1, B.t2, B.t3, 2 * P + 4, B.team);
        // e = 2^(f+g) - T modulo 2^(32 nT): power of two minus the product
        fill(B.t0, nT, 0u);
        wsync();
        if (lane() == 0) B.t0[(f + gb) / 32] = 1u << ((f + gb) % 32);
        wsync();
        sub(B.prod, B.t0, B.prod, nT, 0u);
        wsync();
        const bool eneg = (B.prod[nT - 1] >> 31) != 0u;
        if (eneg) {  // |e| = -e
            fill(B.t0, nT, 0u);
            wsync();
            sub(B.prod, B.t0, B.prod, nT, 0u);
            wsync();
        }
        // |e| ~ 2^(g+8): keep its limbs as the y operand
        const int ne = min(nT, limbs_for_bits(gb + 12) + 1);
        if (top_nonzero(B.prod, nT) >= ne) return false;
        set_y(B.ypad, B.prod, ne, max(nV, ne));
        wsync();
        const int nD = nX + ne;
        mul_gen(B.prod, nD, B.x, nX, B.ypad, ne, B.t0, B.t1, B.t2, B.t3, 2 * P + 4, B.team);
        // X' = X 2^(f'-f) +- (X |e|) >> (2f + g - f')
        const int nX2 = limbs_for_bits(f2 + 2) + 1;
        shift(B.t0, nX2, B.x, nX, f2 - f);
        shift(B.t1, nX2, B.prod, nD, -(2 * f + gb - f2));
        wsync();
        if (eneg) sub(B.x, B.t0, B.t1, nX2, 0u);
        else add(B.x, B.t0, B.t1, nX2, 0u);
        wsync();
        f = f2;
        nX = nX2;
    }
    // exact correction with E = 2^(2p) - v X over 2P + 2 limbs
    const int nE = 2 * P + 2;
    fill(B.x + nX, P + 4 - nX, 0u);
    set_y(B.ypad, B.v, P, P + 4);
    wsync();
    mul_gen(B.prod, nE, B.x, P + 2, B.ypad, P, B.t0, B.t1, B.t2, B.t3, 2 * P + 4, B.team);
    fill(B.t0, nE, 0u);
    wsync();
    if (lane() == 0) B.t0[2 * P] = 1u;
    wsync();
    sub(B.prod, B.t0, B.prod, nE, 0u);  // E (two's complement over nE limbs)
    wsync();
    // v padded to nE limbs in t1, one in t2 (for X -+ 1)
    fill(B.t1, nE, 0u);
    fill(B.t2, nE, 0u);
    wsync();
    copy(B.t1, B.v, P);
    if (lane() == 0) B.t2[0] = 1u;
    wsync();
    for (int it = 0; it < 24; ++it) {
        const bool neg = (B.prod[nE - 1] >> 31) != 0u;
        if (neg) {  // X -= 1, E += v
            sub(B.x, B.x, B.t2, P + 2, 0u);
            add(B.prod, B.prod, B.t1, nE, 0u);
            wsync();
            continue;
        }
        if (cmp(B.prod, B.t1, nE) >= 0) {  // X += 1, E -= v
            add(B.x, B.x, B.t2, P + 2, 0u);
            sub(B.prod, B.prod, B.t1, nE, 0u);
            wsync();
            continue;
        }
        return true;  // 0 <= E < v
    }
    return false;
}

// out = RZ_p(a / b) given R = floor(2^(2p) / m_b) (P + 1 limbs, in global
// memory).  Q = floor(m_a 2^(p+1) / m_b) lies in [Q0, Q0 + 2] for
// Q0 = floor(m_a R / 2^(p-1)).  The product m_a R is formed only from digit
// window wlo on (mul_win), which leaves out less than 2^(p-1), so the Q0' it
// gives is Q0 or Q0 - 1 and Q lies in [Q0', Q0' + 3]; the remainder
// m_a 2^(p+1) - Q0' m_b (in [0, 4 m_b)), formed modulo 2^(32(P+2)) from the
// low half of Q0' m_b, moves Q0' up to Q.  a (P limbs) must be in B.a, b in
// B.v.  Returns false if the remainder check did not settle (callers then fall
// back to long division).
__device__ bool div_by_recip(uint32_t *out, Hdr &hq, Hdr ha, Hdr hb, const uint32_t *R, const DivBufs &B,
                             int P) {
    const int64_t p = 32LL * P;
    if (ha.zero) {
        hq = zero_hdr();
        return true;
    }
    const int n2 = P + 2;
    // Q0 = (m_a R) >> (p - 1)
    copy(B.x, B.a, P);
    for (int q = lane(); q < P + 1 + 2 * MP_YPAD; q += MP_WAVE) {
        int kq = q - MP_YPAD;
        B.ypad[q] = (kq >= 0 && kq < P + 1) ? R[kq] : 0u;
    }
    wsync();
    // windows below wlo hold digit columns below 8 wlo: what they leave out is
    // below 2^(224 wlo + 68) <= 2^(p - 1) (column sums below 2^67 for up to
    // 2^11 digits), and the limbs read below (from P - 1 on) are above 7 wlo
    const int wlo = P <= 1024 ? max(0, (32 * P - 69) / 224) : 0;
    mul_gen(B.prod, 2 * P + 1, B.x, P, B.ypad, P + 1, B.t0, B.t1, B.t2, B.t3, 2 * P + 4, B.team, wlo);
    shift(B.x, n2, B.prod, 2 * P + 1, -(p - 1));  // Q0' (P + 2 limbs)
    set_y(B.ypad, B.v, P, P + 4);
    wsync();
    // low half of Q0 m_b
    mul_gen(B.prod, n2, B.x, n2, B.ypad, P, B.t0, B.t1, B.t2, B.t3, 2 * P + 4, B.team);
    // rem = (m_a 2^(p+1) - Q0 m_b) mod 2^(32 n2)
    shift(B.t0, n2, B.a, P, p + 1);
    fill(B.t1, n2, 0u);
    fill(B.t2, n2, 0u);
    wsync();
    sub(B.t0, B.t0, B.prod, n2, 0u);
    copy(B.t1, B.v, P);  // v padded to n2 limbs
    if (lane() == 0) B.t2[0] = 1u;
    wsync();
    bool ok = false;
    for (int it = 0; it < 6; ++it) {
        if ((B.t0[n2 - 1] >> 31) != 0u) break;  // negative: R was not exact
        if (cmp(B.t0, B.t1, n2) < 0) {
            ok = true;
            break;
        }
        add(B.x, B.x, B.t2, n2, 0u);
        sub(B.t0, B.t0, B.t1, n2, 0u);
        wsync();
    }
    if (!ok) return false;
    hq = normalise(out, B.x, n2, ha.e - hb.e - p - 1, ha.s ^ hb.s, P);
    return true;
}

// The multipliers' own layout (k_divide): a, v, Q0 and the product in LDS,
// the windowed products' scratch (digits, overflow vector) reused afterwards
// for the remainder, v padded, one, the quotient and the result; R is read
// from global memory where the digits are formed.  About 9.3P words against
// the 14P of DivBufs, so twice as many workgroups of the launch share a CU.
// Needs P >= 16 (every product windowed).
struct DivLean {
    uint32_t *a, *v, *x;  // P + 4 each (x: Q0, P + 2 limbs)
    uint32_t *prod;       // 2P + 4
    uint32_t *ws;         // ws_words(P): the products' scratch, then t0 t1 t2 (P + 2 each) and out (P)
    uint32_t *out;
    TeamCtl *team = nullptr;
};
__host__ __device__ constexpr int div_lean_ws_words(int P) {
    const int w = win_words(2 * P + 1, P, P + 1), t = 4 * P + 8;
    return ((w > t ? w : t) + 3) & ~3;
}
__host__ __device__ constexpr size_t div_lean_words(int P) {
    return (size_t)(3 * ((P + 4 + 3) & ~3) + ((2 * P + 4 + 3) & ~3) + div_lean_ws_words(P));
}
__device__ __forceinline__ DivLean div_lean(uint32_t *base, int P) {
    const int n1 = (P + 4 + 3) & ~3, n2 = (2 * P + 4 + 3) & ~3;
    DivLean L;
    L.a = base;
    L.v = L.a + n1;
    L.x = L.v + n1;
    L.prod = L.x + n1;
    L.ws = L.prod + n2;
    L.out = L.ws + 3 * (P + 2);
    return L;
}

// div_by_recip on the lean layout: the same steps and bits.  a in L.a, b in
// L.v; the quotient goes to L.out.
__device__ bool div_by_recip_lean(Hdr &hq, Hdr ha, Hdr hb, const uint32_t *R, const DivLean &L, int P) {
    const int64_t p = 32LL * P;
    if (ha.zero) {
        hq = zero_hdr();
        return true;
    }
    const int n2 = P + 2;
    // Q0' = (m_a R) >> (p - 1), the product from digit window wlo on (the bound
    // as in div_by_recip)
    const int wlo = P <= 1024 ? max(0, (32 * P - 69) / 224) : 0;
    mul_win(L.prod, 2 * P + 1, L.a, P, R, P + 1, L.ws, L.team, wlo);
    shift(L.x, n2, L.prod, 2 * P + 1, -(p - 1));
    wsync();
    // low half of Q0' m_b
    mul_win(L.prod, n2, L.x, n2, L.v, P, L.ws, L.team);
    // rem = (m_a 2^(p+1) - Q0' m_b) mod 2^(32 n2), in [0, 4 m_b)
    uint32_t *t0 = L.ws, *t1 = t0 + n2, *t2 = t1 + n2;
    shift(t0, n2, L.a, P, p + 1);
    fill(t1, n2, 0u);
    fill(t2, n2, 0u);
    wsync();
    sub(t0, t0, L.prod, n2, 0u);
    copy(t1, L.v, P);  // v padded to n2 limbs
    if (lane() == 0) t2[0] = 1u;
    wsync();
    bool ok = false;
    for (int it = 0; it < 6; ++it) {
        if ((t0[n2 - 1] >> 31) != 0u) break;  // negative: R was not exact
        if (cmp(t0, t1, n2) < 0) {
            ok = true;
            break;
        }
        add(L.x, L.x, t2, n2, 0u);
        sub(t0, t0, t1, n2, 0u);
        wsync();
    }
    if (!ok) return false;
    hq = normalise(L.out, L.x, n2, ha.e - hb.e - p - 1, ha.s ^ hb.s, P);
    return true;
}

}  // namespace mpw
