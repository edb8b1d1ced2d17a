/*
 * mpref.c -- CPU oracle: multiprecision Gaussian elimination without pivoting,
 * leading determinants, last-column cofactors and the adjugate.
 *
 * TEST INFRASTRUCTURE ONLY (see mpref.h).  Written to be read against the
 * paper, not to be fast: every operation is the exact integer result followed
 * by one truncation toward zero (RZ_p), every loop follows the order the
 * method states, and the only parallelism is the paper's shared-memory scheme
 * (rows of the trailing block split into equal contiguous blocks, one per
 * thread, re-split at every step; Sec. 4.1).
 *
 * Paper references:
 *   Sec. 3 / Algorithm 1 step 2.1   Det = Det * a_ii (leading determinants)
 *   Algorithm 1 step 2.2.1          z = a_ji / a_ii
 *   Algorithm 1 step 2.2.2          a_jk = a_jk - z * a_ik
 *   Sec. 3 ([A I] derivation)       L A = U; |A| times the last row of L gives
 *                                   the signed minors of the last column
 *   Sec. 3 (storage paragraph)      multipliers stored below the diagonal
 *   Sec. 3 (Baur-Strassen remark)   all (N-1)x(N-1) minors are d det / d a_ij
 *   Eq. (minorsdef)                 signed minors (-1)^(N+n) M_{n,N}
 */
#include "mpref.h"

#include <stdlib.h>
#include <string.h>
#include <math.h>

#define EXP_LIMIT (((int64_t)1) << 62)

/* ------------------------------------------------------------------------- */
/* Unsigned big integers: little-endian arrays of uint32 limbs.              */
/* ------------------------------------------------------------------------- */

static int clz32(uint32_t x)
{
    int n = 0;
    if (x == 0) return 32;
    while (!(x & 0x80000000u)) { x <<= 1; n++; }
    return n;
}

/* number of significant bits of a (0 for a == 0) */
static int64_t bn_bitlen(const uint32_t *a, int64_t n)
{
    for (int64_t i = n - 1; i >= 0; i--)
        if (a[i]) return 32 * i + (32 - clz32(a[i]));
    return 0;
}

/* out[0..na+nb) = a * b, schoolbook */
void mpref_bn_mul(uint32_t *out, const uint32_t *a, int32_t na,
                  const uint32_t *b, int32_t nb)
{
    memset(out, 0, sizeof(uint32_t) * (size_t)(na + nb));
    for (int32_t i = 0; i < na; i++) {
        uint64_t carry = 0;
        for (int32_t j = 0; j < nb; j++) {
            uint64_t t = (uint64_t)a[i] * b[j] + out[i + j] + carry;
            out[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        out[i + nb] = (uint32_t)carry;
    }
}

/* out[0..nout) = a << bits (the caller guarantees the result fits) */
static void bn_shl(uint32_t *out, int64_t nout, const uint32_t *a, int64_t na, int64_t bits)
{
    int64_t w = bits / 32, b = bits % 32;
    memset(out, 0, sizeof(uint32_t) * (size_t)nout);
    for (int64_t i = 0; i < na; i++) {
        if (i + w < nout) out[i + w] |= a[i] << b;
        if (b && i + w + 1 < nout) out[i + w + 1] |= a[i] >> (32 - b);
    }
}

/* out[0..nout) = floor(a / 2^bits), low nout limbs */
static void bn_shr(uint32_t *out, int64_t nout, const uint32_t *a, int64_t na, int64_t bits)
{
    int64_t w = bits / 32, b = bits % 32;
    for (int64_t i = 0; i < nout; i++) {
        uint64_t lo = (i + w < na) ? a[i + w] : 0;
        uint64_t hi = (i + w + 1 < na) ? a[i + w + 1] : 0;
        out[i] = (uint32_t)(((hi << 32) | lo) >> b);
    }
}

static int bn_cmp(const uint32_t *a, const uint32_t *b, int64_t n)
{
    for (int64_t i = n - 1; i >= 0; i--)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}

/* out = a + b, n limbs each; returns the carry out */
static uint32_t bn_add(uint32_t *out, const uint32_t *a, const uint32_t *b, int64_t n)
{
    uint64_t c = 0;
    for (int64_t i = 0; i < n; i++) {
        c += (uint64_t)a[i] + b[i];
        out[i] = (uint32_t)c;
        c >>= 32;
    }
    return (uint32_t)c;
}

/* out = a - b, n limbs each, requires a >= b */
static void bn_sub(uint32_t *out, const uint32_t *a, const uint32_t *b, int64_t n)
{
    int64_t br = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t t = (int64_t)a[i] - b[i] - br;
        br = t < 0;
        out[i] = (uint32_t)(t + (br ? ((int64_t)1 << 32) : 0));
    }
}

/*
 * Long division in base 2^32 (Knuth, TAOCP vol. 2, Sec. 4.3.1, Algorithm D).
 * u has m limbs, v has n limbs with v[n-1] != 0 and m >= n.
 * q receives m - n + 1 limbs, r (if not NULL) receives n limbs.
 * Returns -1 on a bad argument.
 */
int mpref_bn_divmod(uint32_t *q, uint32_t *r, const uint32_t *u, int32_t m,
                    const uint32_t *v, int32_t n)
{
    const uint64_t B = (uint64_t)1 << 32;
    if (n < 1 || m < n || v[n - 1] == 0) return -1;
    if (n == 1) {
        uint64_t k = 0;
        for (int32_t j = m - 1; j >= 0; j--) {
            uint64_t cur = (k << 32) | u[j];
            q[j] = (uint32_t)(cur / v[0]);
            k = cur - (uint64_t)q[j] * v[0];
        }
        if (r) r[0] = (uint32_t)k;
        return 0;
    }
    int s = clz32(v[n - 1]);
    uint32_t *vn = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *un = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(m + 1));
    /* D1: normalize so that the divisor's top bit is set */
    for (int32_t i = n - 1; i > 0; i--)
        vn[i] = (v[i] << s) | (s ? v[i - 1] >> (32 - s) : 0);
    vn[0] = v[0] << s;
    un[m] = s ? u[m - 1] >> (32 - s) : 0;
    for (int32_t i = m - 1; i > 0; i--)
        un[i] = (u[i] << s) | (s ? u[i - 1] >> (32 - s) : 0);
    un[0] = u[0] << s;
    for (int32_t j = m - n; j >= 0; j--) {
        /* D3: estimate the quotient digit from the top two remainder limbs */
        uint64_t num = ((uint64_t)un[j + n] << 32) | un[j + n - 1];
        uint64_t qhat = num / vn[n - 1];
        uint64_t rhat = num - qhat * vn[n - 1];
        while (qhat >= B || qhat * vn[n - 2] > ((rhat << 32) | un[j + n - 2])) {
            qhat--;
            rhat += vn[n - 1];
            if (rhat >= B) break;
        }
        /* D4: multiply and subtract */
        int64_t k = 0, t;
        for (int32_t i = 0; i < n; i++) {
            uint64_t p = qhat * vn[i];
            t = (int64_t)un[i + j] - k - (int64_t)(p & 0xFFFFFFFFu);
            un[i + j] = (uint32_t)t;
            k = (int64_t)(p >> 32) - (t >> 32);
        }
        t = (int64_t)un[j + n] - k;
        un[j + n] = (uint32_t)t;
        q[j] = (uint32_t)qhat;
        /* D6: add back when the estimate was one too large */
        if (t < 0) {
            q[j]--;
            uint64_t c = 0;
            for (int32_t i = 0; i < n; i++) {
                c += (uint64_t)un[i + j] + vn[i];
                un[i + j] = (uint32_t)c;
                c >>= 32;
            }
            un[j + n] += (uint32_t)c;
        }
    }
    if (r) {
        for (int32_t i = 0; i < n - 1; i++)
            r[i] = (un[i] >> s) | (s ? un[i + 1] << (32 - s) : 0);
        r[n - 1] = un[n - 1] >> s;
    }
    free(vn);
    free(un);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Numbers in the format, and the single truncation rule RZ_p.               */
/* ------------------------------------------------------------------------- */

typedef struct {
    uint32_t *m; /* P limbs */
    int64_t e;
    int32_t s;
} num;

static int num_is_zero(const uint32_t *m, int32_t P)
{
    for (int32_t i = 0; i < P; i++)
        if (m[i]) return 0;
    return 1;
}

static void set_zero(uint32_t *m, int64_t *e, int32_t *s, int32_t P)
{
    memset(m, 0, sizeof(uint32_t) * (size_t)P);
    *e = 0;
    *s = 0;
}

static void set_one(uint32_t *m, int64_t *e, int32_t *s, int32_t P)
{
    memset(m, 0, sizeof(uint32_t) * (size_t)P);
    m[P - 1] = 0x80000000u; /* 1 = 2^(p-1) * 2^(1-p) */
    *e = 1;
    *s = 0;
}

/*
 * RZ_p of the exact value (-1)^sign * V * 2^E, V an unsigned integer of nV
 * limbs.  With L = bitlen(V): m = floor(V / 2^(L-p)) (or V * 2^(p-L) when
 * L < p) and e = E + L, so that m * 2^(e-p) = V * 2^E up to the truncation.
 */
static void rz_round(uint32_t *m, int64_t *e, int32_t *s, int32_t P,
                     int32_t sign, const uint32_t *V, int64_t nV, int64_t E)
{
    int64_t p = 32 * (int64_t)P;
    int64_t L = bn_bitlen(V, nV);
    if (L == 0) {
        set_zero(m, e, s, P);
        return;
    }
    if (L >= p) bn_shr(m, P, V, nV, L - p);
    else bn_shl(m, P, V, nV, p - L);
    *e = E + L;
    *s = sign;
}

/* RZ_p(a * b): the exact product has 2P limbs. */
static void rz_mul(int32_t P, const uint32_t *am, int64_t ae, int32_t as,
                   const uint32_t *bm, int64_t be, int32_t bs,
                   uint32_t *rm, int64_t *re, int32_t *rs)
{
    int64_t p = 32 * (int64_t)P;
    if (num_is_zero(am, P) || num_is_zero(bm, P)) {
        set_zero(rm, re, rs, P);
        return;
    }
    uint32_t V[2 * P];
    mpref_bn_mul(V, am, P, bm, P);
    rz_round(rm, re, rs, P, as ^ bs, V, 2 * (int64_t)P, ae + be - 2 * p);
}

/*
 * RZ_p(a + (-1)^negb * b).
 *
 * Let X be the operand with the larger exponent and Y the other, d = e_X - e_Y.
 * The exact value is (m_X * 2^d +- m_Y) * 2^(e_Y - p).  When d exceeds
 * 2p + 4 it is clamped to dc = 2p + 4, i.e. Y is replaced by a value of the
 * same sign whose magnitude is still below ulp(X)/4.  That does not change the
 * result: for 0 < |y| < ulp(x)/4, RZ_p(x + y) is x when y has the sign of x,
 * and the next representable number toward zero from x when it has the
 * opposite sign (x - ulp(x), or x - ulp(x)/2 when |x| is a power of two), for
 * every such y.  Below the clamp the integer arithmetic is exact.
 */
static void rz_addsub(int32_t P, const uint32_t *am, int64_t ae, int32_t as,
                      const uint32_t *bm, int64_t be, int32_t bs, int negb,
                      uint32_t *rm, int64_t *re, int32_t *rs)
{
    int64_t p = 32 * (int64_t)P;
    int32_t sb = bs ^ (negb ? 1 : 0);
    int az = num_is_zero(am, P), bz = num_is_zero(bm, P);
    if (az && bz) {
        set_zero(rm, re, rs, P);
        return;
    }
    if (bz) {
        memmove(rm, am, sizeof(uint32_t) * (size_t)P);
        *re = ae;
        *rs = as;
        return;
    }
    if (az) {
        memmove(rm, bm, sizeof(uint32_t) * (size_t)P);
        *re = be;
        *rs = sb;
        return;
    }
    const uint32_t *xm, *ym;
    int64_t xe, ye;
    int32_t xs, ys;
    if (ae >= be) {
        xm = am; xe = ae; xs = as; ym = bm; ye = be; ys = sb;
    } else {
        xm = bm; xe = be; xs = sb; ym = am; ye = ae; ys = as;
    }
    int64_t d = xe - ye;
    int64_t dc = d < 2 * p + 4 ? d : 2 * p + 4;
    int64_t n = P + (dc + 31) / 32 + 2;
    uint32_t VX[n], VY[n], V[n];
    bn_shl(VX, n, xm, P, dc);
    memset(VY, 0, sizeof(uint32_t) * (size_t)n);
    memcpy(VY, ym, sizeof(uint32_t) * (size_t)P);
    int32_t sign;
    if (xs == ys) {
        bn_add(V, VX, VY, n); /* n has a spare limb: no carry out */
        sign = xs;
    } else {
        int c = bn_cmp(VX, VY, n);
        if (c == 0) {
            set_zero(rm, re, rs, P);
            return;
        }
        if (c > 0) {
            bn_sub(V, VX, VY, n);
            sign = xs;
        } else {
            bn_sub(V, VY, VX, n);
            sign = ys;
        }
    }
    rz_round(rm, re, rs, P, sign, V, n, xe - dc - p);
}

/*
 * RZ_p(a / b), b != 0: Q = floor(m_a * 2^(p+1) / m_b) has p+1 or p+2 bits
 * (m_a / m_b lies in (1/2, 2)); rz_round truncates the remaining one or two
 * bits, and floor(floor(x) / 2^k) = floor(x / 2^k).
 */
static void rz_div(int32_t P, const uint32_t *am, int64_t ae, int32_t as,
                   const uint32_t *bm, int64_t be, int32_t bs,
                   uint32_t *rm, int64_t *re, int32_t *rs)
{
    int64_t p = 32 * (int64_t)P;
    if (num_is_zero(am, P)) {
        set_zero(rm, re, rs, P);
        return;
    }
    int32_t nu = 2 * P + 1;
    uint32_t U[nu], Q[nu - P + 1];
    bn_shl(U, nu, am, P, p + 1);
    mpref_bn_divmod(Q, NULL, U, nu, bm, P);
    rz_round(rm, re, rs, P, as ^ bs, Q, nu - P + 1, ae - be - p - 1);
}

void mpref_mul(int32_t P, const uint32_t *am, int64_t ae, int32_t as,
               const uint32_t *bm, int64_t be, int32_t bs,
               uint32_t *rm, int64_t *re, int32_t *rs)
{
    rz_mul(P, am, ae, as, bm, be, bs, rm, re, rs);
}

void mpref_add(int32_t P, const uint32_t *am, int64_t ae, int32_t as,
               const uint32_t *bm, int64_t be, int32_t bs,
               uint32_t *rm, int64_t *re, int32_t *rs)
{
    rz_addsub(P, am, ae, as, bm, be, bs, 0, rm, re, rs);
}

void mpref_sub(int32_t P, const uint32_t *am, int64_t ae, int32_t as,
               const uint32_t *bm, int64_t be, int32_t bs,
               uint32_t *rm, int64_t *re, int32_t *rs)
{
    rz_addsub(P, am, ae, as, bm, be, bs, 1, rm, re, rs);
}

int mpref_div(int32_t P, const uint32_t *am, int64_t ae, int32_t as,
              const uint32_t *bm, int64_t be, int32_t bs,
              uint32_t *rm, int64_t *re, int32_t *rs)
{
    if (num_is_zero(bm, P)) return -1;
    rz_div(P, am, ae, as, bm, be, bs, rm, re, rs);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Gaussian elimination without pivoting (Algorithm 1, steps 1-2.2.2).       */
/* ------------------------------------------------------------------------- */

#define EL(i, j) (limbs + ((size_t)(i) * (size_t)n + (size_t)(j)) * (size_t)P)
#define EE(i, j) (exp[(size_t)(i) * (size_t)n + (size_t)(j)])
#define ES(i, j) (sign[(size_t)(i) * (size_t)n + (size_t)(j)])

static int64_t iabs64(int64_t x) { return x < 0 ? -x : x; }

int mpref_factor(int64_t n, int32_t P, uint32_t *limbs, int64_t *exp, int32_t *sign,
                 uint32_t *Dl, int64_t *De, int32_t *Ds, int32_t *info, int32_t threads)
{
    if (!info) return -1;
    *info = 0;
    return mpref_factor_range(n, P, limbs, exp, sign, Dl, De, Ds, info, 0, n, threads);
}

/*
 * Steps k_begin .. k_end-1 of the elimination above, continuing from the
 * state an earlier range left (the matrix, D_1..D_{k_begin} and *info; a
 * nonzero *info means the elimination already stopped).  Ranges [0, k_1),
 * [k_1, k_2), ... applied in order are the whole elimination: each step reads
 * only what the steps before it left.
 */
int mpref_factor_range(int64_t n, int32_t P, uint32_t *limbs, int64_t *exp, int32_t *sign,
                       uint32_t *Dl, int64_t *De, int32_t *Ds, int32_t *info, int64_t k_begin,
                       int64_t k_end, int32_t threads)
{
    if (n < 0 || P < 1 || !info || (n > 0 && (!limbs || !exp || !sign || !Dl || !De || !Ds)))
        return -1;
    if (k_begin < 0 || k_end < k_begin || k_end > n) return -1;
    if (threads < 1) threads = 1;
    if (*info != 0) return 0;
    for (int64_t k = k_begin; k < k_end; k++) {
        /* step 2.1: the pivot is a_kk after k-1 elimination steps */
        if (num_is_zero(EL(k, k), P)) {
            *info = (int32_t)(k + 1);
            for (int64_t t = k; t < n; t++) set_zero(Dl + t * P, De + t, Ds + t, P);
            return 0;
        }
        if (k == 0) {
            memcpy(Dl, EL(0, 0), sizeof(uint32_t) * (size_t)P);
            De[0] = EE(0, 0);
            Ds[0] = ES(0, 0);
        } else {
            rz_mul(P, Dl + (k - 1) * P, De[k - 1], Ds[k - 1], EL(k, k), EE(k, k), ES(k, k),
                   Dl + k * P, De + k, Ds + k);
        }
        if (iabs64(EE(k, k)) > EXP_LIMIT || iabs64(De[k]) > EXP_LIMIT) {
            *info = -1;
            for (int64_t t = k; t < n; t++) set_zero(Dl + t * P, De + t, Ds + t, P);
            return 0;
        }
        /* step 2.2.1: multipliers l_ik = a_ik / a_kk, stored in place */
#pragma omp parallel for num_threads(threads) schedule(static)
        for (int64_t i = k + 1; i < n; i++)
            rz_div(P, EL(i, k), EE(i, k), ES(i, k), EL(k, k), EE(k, k), ES(k, k),
                   EL(i, k), &EE(i, k), &ES(i, k));
        /* step 2.2.2: a_ij = a_ij - l_ik * a_kj (product rounded, then difference) */
#pragma omp parallel for num_threads(threads) schedule(static)
        for (int64_t i = k + 1; i < n; i++) {
            uint32_t tm[P];
            int64_t te;
            int32_t ts;
            for (int64_t j = k + 1; j < n; j++) {
                rz_mul(P, EL(i, k), EE(i, k), ES(i, k), EL(k, j), EE(k, j), ES(k, j),
                       tm, &te, &ts);
                rz_addsub(P, EL(i, j), EE(i, j), ES(i, j), tm, te, ts, 1,
                          EL(i, j), &EE(i, j), &ES(i, j));
            }
        }
    }
    return 0;
}

/*
 * Last-column cofactors (Sec. 3, [A I] derivation).  With A = L_std U and
 * L_std unit lower triangular holding the multipliers, e_n^T L_std^-1 A =
 * u_nn e_n^T, so c = D_{n-1} * (e_n^T L_std^-1) satisfies c . A_{:,j} = 0 for
 * j < n and c . A_{:,n} = det.  x^T = e_n^T L_std^-1 solves x^T L_std = e_n^T:
 * x_n = 1 and, sweeping j from n down to 2, s_i <- s_i - x_j l_ji for i < j,
 * after which x_{j-1} = s_{j-1}.  Then c_i = D_{n-1} x_i and c_n = D_{n-1}.
 */
int mpref_minors(int64_t n, int32_t P, const uint32_t *limbs, const int64_t *exp,
                 const int32_t *sign, const uint32_t *Dl, const int64_t *De,
                 const int32_t *Ds, uint32_t *cl, int64_t *ce, int32_t *cs,
                 int32_t threads)
{
    if (n < 1 || P < 1 || !limbs || !exp || !sign || !Dl || !De || !Ds || !cl || !ce || !cs)
        return -1;
    if (threads < 1) threads = 1;
    if (n == 1) { /* the cofactor of a 1x1 matrix is the empty determinant, 1 */
        set_one(cl, ce, cs, P);
        return 0;
    }
    /* s_i accumulates in c's storage: entries 0..n-2 */
    for (int64_t i = 0; i < n - 1; i++) set_zero(cl + i * P, ce + i, cs + i, P);
    uint32_t one_m[P];
    int64_t one_e;
    int32_t one_s;
    set_one(one_m, &one_e, &one_s, P);
    uint32_t xm[P];
    int64_t xe;
    int32_t xs;
    for (int64_t j = n - 1; j >= 1; j--) {
        if (j == n - 1) {
            memcpy(xm, one_m, sizeof(uint32_t) * (size_t)P);
            xe = one_e;
            xs = one_s;
        } else {
            memcpy(xm, cl + j * P, sizeof(uint32_t) * (size_t)P);
            xe = ce[j];
            xs = cs[j];
        }
#pragma omp parallel for num_threads(threads) schedule(static)
        for (int64_t i = 0; i < j; i++) {
            uint32_t tm[P];
            int64_t te;
            int32_t ts;
            rz_mul(P, xm, xe, xs, EL(j, i), EE(j, i), ES(j, i), tm, &te, &ts);
            rz_addsub(P, cl + i * P, ce[i], cs[i], tm, te, ts, 1, cl + i * P, ce + i, cs + i);
        }
    }
    /* c_i = D_{n-1} x_i for i < n, c_n = D_{n-1} */
    const uint32_t *dm = Dl + (n - 2) * P;
#pragma omp parallel for num_threads(threads) schedule(static)
    for (int64_t i = 0; i < n - 1; i++)
        rz_mul(P, dm, De[n - 2], Ds[n - 2], cl + i * P, ce[i], cs[i], cl + i * P, ce + i, cs + i);
    memcpy(cl + (n - 1) * P, dm, sizeof(uint32_t) * (size_t)P);
    ce[n - 1] = De[n - 2];
    cs[n - 1] = Ds[n - 2];
    return 0;
}

/*
 * Adjugate from the stored factors (Sec. 3: by Baur-Strassen all the
 * (N-1)x(N-1) minors are the partial derivatives of the determinant, so
 * d det / d a_ij = C_ij and the gradient is adj(A)^T).  With A = L_std U,
 * adj(A) = adj(U) adj(L_std) = adj(U) W, W = L_std^-1, computed in this fixed
 * order:
 *   W row r: x^T L_std = e_r^T, solved exactly as in mpref_minors with r in
 *     place of n (so row n of W is the minors' x, bit for bit);
 *   adj(U)_ii = D_{i-1} * S_{i+1}, S_{n+1} = 1, S_i = u_ii * S_{i+1};
 *   adj(U)_ij (i < j) = t / u_ii, t = -sum_{k=i+1..j} u_ik adj(U)_kj
 *     (U adj(U) = det(U) I, row i, column j), accumulated in descending k:
 *     the right-looking back substitution of each column;
 *   adj(A)_im = sum_{k >= max(i,m)} adj(U)_ik W_km, ascending k.
 * Row n of adj(A) is then D_{n-1} x_m = c_m, identical to mpref_minors.
 * Output: adjT[i][m] = adj(A)[m][i].
 */
int mpref_adjugate_t(int64_t n, int32_t P, const uint32_t *limbs, const int64_t *exp,
                     const int32_t *sign, const uint32_t *Dl, const int64_t *De,
                     const int32_t *Ds, uint32_t *tl, int64_t *te, int32_t *ts,
                     int32_t threads)
{
    if (n < 1 || P < 1 || !limbs || !exp || !sign || !Dl || !De || !Ds || !tl || !te || !ts)
        return -1;
    if (threads < 1) threads = 1;
    size_t nn = (size_t)n * (size_t)n;
    uint32_t *Wl = (uint32_t *)calloc(nn * (size_t)P, sizeof(uint32_t));
    int64_t *We = (int64_t *)calloc(nn, sizeof(int64_t));
    int32_t *Ws = (int32_t *)calloc(nn, sizeof(int32_t));
    uint32_t *Jl = (uint32_t *)calloc(nn * (size_t)P, sizeof(uint32_t)); /* adj(U) */
    int64_t *Je = (int64_t *)calloc(nn, sizeof(int64_t));
    int32_t *Js = (int32_t *)calloc(nn, sizeof(int32_t));
    uint32_t *Sl = (uint32_t *)calloc((size_t)(n + 1) * (size_t)P, sizeof(uint32_t));
    int64_t *Se = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int32_t *Ss = (int32_t *)calloc((size_t)(n + 1), sizeof(int32_t));
    if (!Wl || !We || !Ws || !Jl || !Je || !Js || !Sl || !Se || !Ss) {
        free(Wl); free(We); free(Ws); free(Jl); free(Je); free(Js);
        free(Sl); free(Se); free(Ss);
        return -1;
    }
#define W_(i, j) (Wl + ((size_t)(i) * (size_t)n + (size_t)(j)) * (size_t)P)
#define WE(i, j) (We[(size_t)(i) * (size_t)n + (size_t)(j)])
#define WS(i, j) (Ws[(size_t)(i) * (size_t)n + (size_t)(j)])
#define J_(i, j) (Jl + ((size_t)(i) * (size_t)n + (size_t)(j)) * (size_t)P)
#define JE(i, j) (Je[(size_t)(i) * (size_t)n + (size_t)(j)])
#define JS(i, j) (Js[(size_t)(i) * (size_t)n + (size_t)(j)])
#define T_(i, j) (tl + ((size_t)(i) * (size_t)n + (size_t)(j)) * (size_t)P)
#define TE(i, j) (te[(size_t)(i) * (size_t)n + (size_t)(j)])
#define TS(i, j) (ts[(size_t)(i) * (size_t)n + (size_t)(j)])

    /* W = L_std^-1, one row per solve (rows are independent) */
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
    for (int64_t r = 0; r < n; r++) {
        uint32_t xm[P], tm[P];
        int64_t xe, tE;
        int32_t xs, tS;
        set_one(W_(r, r), &WE(r, r), &WS(r, r), P);
        for (int64_t j = r; j >= 1; j--) {
            memcpy(xm, W_(r, j), sizeof(uint32_t) * (size_t)P);
            xe = WE(r, j);
            xs = WS(r, j);
            for (int64_t i = 0; i < j; i++) {
                rz_mul(P, xm, xe, xs, EL(j, i), EE(j, i), ES(j, i), tm, &tE, &tS);
                rz_addsub(P, W_(r, i), WE(r, i), WS(r, i), tm, tE, tS, 1,
                          W_(r, i), &WE(r, i), &WS(r, i));
            }
        }
    }
    /* S_i = u_ii S_{i+1}, S_{n+1} = 1 (0-based: S[n] = 1) */
    set_one(Sl + (size_t)n * P, Se + n, Ss + n, P);
    for (int64_t i = n - 1; i >= 0; i--)
        rz_mul(P, EL(i, i), EE(i, i), ES(i, i), Sl + (size_t)(i + 1) * P, Se[i + 1], Ss[i + 1],
               Sl + (size_t)i * P, Se + i, Ss + i);
    /* adj(U) diagonal: D_{i-1} S_{i+1}, D_0 = 1 */
    for (int64_t i = 0; i < n; i++) {
        if (i == 0) {
            memcpy(J_(0, 0), Sl + P, sizeof(uint32_t) * (size_t)P);
            JE(0, 0) = Se[1];
            JS(0, 0) = Ss[1];
        } else {
            rz_mul(P, Dl + (i - 1) * P, De[i - 1], Ds[i - 1], Sl + (size_t)(i + 1) * P,
                   Se[i + 1], Ss[i + 1], J_(i, i), &JE(i, i), &JS(i, i));
        }
    }
    /* adj(U) strictly upper part: back substitution in U x = det(U) e_j for
     * every column j, right-looking: once x_k is final, t_i <- t_i - u_ik x_k
     * for all i < k (k descending), then x_{k-1} = t_{k-1} / u_{k-1,k-1}.
     * The accumulators t_i live in J(i, j), which starts at zero (calloc). */
    for (int64_t k = n - 1; k >= 1; k--) {
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
        for (int64_t j = k; j < n; j++) {
            uint32_t tm[P];
            int64_t tE;
            int32_t tS;
            for (int64_t i = 0; i < k; i++) {
                rz_mul(P, EL(i, k), EE(i, k), ES(i, k), J_(k, j), JE(k, j), JS(k, j), tm, &tE, &tS);
                rz_addsub(P, J_(i, j), JE(i, j), JS(i, j), tm, tE, tS, 1, J_(i, j), &JE(i, j), &JS(i, j));
            }
            rz_div(P, J_(k - 1, j), JE(k - 1, j), JS(k - 1, j), EL(k - 1, k - 1), EE(k - 1, k - 1),
                   ES(k - 1, k - 1), J_(k - 1, j), &JE(k - 1, j), &JS(k - 1, j));
        }
    }
    /* adj(A)_im = sum_{k >= max(i,m)} adj(U)_ik W_km; stored transposed */
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
    for (int64_t i = 0; i < n; i++) {
        uint32_t acc[P], tm[P];
        int64_t ae, tE;
        int32_t as, tS;
        for (int64_t m = 0; m < n; m++) {
            set_zero(acc, &ae, &as, P);
            for (int64_t k = (i > m ? i : m); k < n; k++) {
                rz_mul(P, J_(i, k), JE(i, k), JS(i, k), W_(k, m), WE(k, m), WS(k, m),
                       tm, &tE, &tS);
                rz_addsub(P, acc, ae, as, tm, tE, tS, 0, acc, &ae, &as);
            }
            memcpy(T_(m, i), acc, sizeof(uint32_t) * (size_t)P);
            TE(m, i) = ae;
            TS(m, i) = as;
        }
    }
    free(Wl); free(We); free(Ws); free(Jl); free(Je); free(Js);
    free(Sl); free(Se); free(Ss);
    return 0;
}

/* mant = (-1)^s * RZ_53(m / 2^p): the top 53 bits of m, exactly a double */
void mpref_to_f64(int64_t count, int32_t P, const uint32_t *limbs, const int64_t *exp,
                  const int32_t *sign, double *mant, int64_t *eout)
{
    int64_t p = 32 * (int64_t)P;
    for (int64_t t = 0; t < count; t++) {
        const uint32_t *m = limbs + t * P;
        if (num_is_zero(m, P)) {
            mant[t] = 0.0;
            eout[t] = 0;
            continue;
        }
        uint32_t top[2];
        if (p >= 53) bn_shr(top, 2, m, P, p - 53);
        else bn_shl(top, 2, m, P, 53 - p);
        uint64_t v = ((uint64_t)top[1] << 32) | top[0];
        double x = ldexp((double)v, -53);
        mant[t] = sign[t] ? -x : x;
        eout[t] = exp[t];
    }
}

/*
 * RZ to p2 = 32 P2 bits of numbers held with P >= P2 limbs: the exact value
 * truncated toward zero.  A nonzero mantissa has its top bit set, so that is
 * its top P2 limbs with the same exponent and sign (value m' 2^(e - 32 P2)).
 */
int mpref_truncate(int64_t count, int32_t P, int32_t P2, const uint32_t *limbs, const int64_t *exp,
                   const int32_t *sign, uint32_t *ol, int64_t *oe, int32_t *os)
{
    if (count < 0 || P2 < 1 || P2 > P || (count > 0 && (!limbs || !exp || !sign || !ol || !oe || !os)))
        return -1;
    for (int64_t t = 0; t < count; t++) {
        memcpy(ol + t * P2, limbs + t * P + (P - P2), sizeof(uint32_t) * (size_t)P2);
        oe[t] = exp[t];
        os[t] = sign[t];
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Rigorous error bounds by ball arithmetic (the future-work section's
 * rigorous results: instead of the interval endpoints of MPFI, each number
 * carries a radius bounding its distance to the value the same sequence of
 * operations gives in exact arithmetic on the exact input).
 *
 * A radius is m 2^e with m a 32-bit integer (0, or 2^31 <= m < 2^32), e an
 * int64; every operation on radii rounds up, so every bound holds; the
 * arithmetic is integer, so it is reproducible bit for bit.  e == RAD_INF:
 * no bound (a pivot whose ball may contain zero).
 * ---------------------------------------------------------------------- */
#define RAD_INF INT64_MAX

typedef struct {
    uint32_t m;
    int64_t e;
} rad_t;

static rad_t rad_make(uint32_t m, int64_t e) { rad_t r; r.m = m; r.e = e; return r; }
static rad_t rad_zero(void) { return rad_make(0u, 0); }
static rad_t rad_inf(void) { return rad_make(0xFFFFFFFFu, RAD_INF); }
static int rad_isinf(rad_t a) { return a.e == RAD_INF; }

/* the 64-bit value v 2^e, rounded up to a 32-bit mantissa */
static rad_t rad_round_up(uint64_t v, int64_t e)
{
    if (v == 0) return rad_zero();
    int n = 0;
    for (uint64_t t = v; t; t >>= 1) n++;
    if (n <= 32) return rad_make((uint32_t)(v << (32 - n)), e - (32 - n));
    int s = n - 32;
    uint64_t m = v >> s;
    if (v & ((((uint64_t)1) << s) - 1)) m++;   /* a dropped bit: round up */
    if (m == (((uint64_t)1) << 32)) { m >>= 1; s++; }
    return rad_make((uint32_t)m, e + s);
}

static rad_t rad_two_to(int64_t k) { return rad_make(0x80000000u, k - 31); }

static rad_t rad_sum(rad_t a, rad_t b)
{
    if (rad_isinf(a) || rad_isinf(b)) return rad_inf();
    if (a.m == 0) return b;
    if (b.m == 0) return a;
    if (a.e < b.e) { rad_t t = a; a = b; b = t; }
    uint64_t gap = (uint64_t)(a.e - b.e);
    /* both on the scale 2^(a.e - 31): a exactly, b rounded up */
    uint64_t A = (uint64_t)a.m << 31, B;
    if (gap >= 63) {
        B = 1;
    } else {
        uint64_t bb = (uint64_t)b.m << 31;
        B = bb >> gap;
        if (bb & ((((uint64_t)1) << gap) - 1)) B++;
    }
    return rad_round_up(A + B, a.e - 31);
}

static rad_t rad_prod(rad_t a, rad_t b)
{
    if (a.m == 0 || b.m == 0) return rad_zero();
    if (rad_isinf(a) || rad_isinf(b)) return rad_inf();
    return rad_round_up((uint64_t)a.m * (uint64_t)b.m, a.e + b.e);
}

/* |x| < 2^e for a nonzero number of exponent e; 0 for zero */
static rad_t rad_abs_bound(const uint32_t *m, int64_t e, int32_t P)
{
    return num_is_zero(m, P) ? rad_zero() : rad_two_to(e);
}

/* the truncation error of a result: below one unit in its last place, 0 if it is zero */
static rad_t rad_unit(const uint32_t *m, int64_t e, int32_t P)
{
    return num_is_zero(m, P) ? rad_zero() : rad_two_to(e - 32 * (int64_t)P);
}

/*
 * mpref_factor_ball: mpref_factor, and for every leading determinant D_k a
 * radius rd[k] = rdm[k] 2^rde[k] with |D_k - D*_k| <= rd[k], D*_k the exact
 * leading determinant of the input (input_ulp: each input entry is itself
 * within one unit in its last place of an exact value).  Per step k, with
 * u = a_kk, l_i the multiplier of row i and q_i = a_ik / u before rounding:
 *   r(D_1) = r(a_11);  r(D_k) = |D_{k-1}| r(u) + |u| r(D_{k-1}) + r(D_{k-1}) r(u) + ulp(D_k);
 *   r(l_i) = (r(a_ik) + |q_i| r(u)) / (|u| - r(u)) + ulp(l_i), where
 *            |q_i| <= 2^e(l_i) and |u| - r(u) >= 2^(e(u) - 2) provided
 *            r(u) <= 2^(e(u) - 2) (otherwise no bound);
 *   r(a_ij) += |l_i| r(u_kj) + |u_kj| r(l_i) + r(l_i) r(u_kj)
 *              [+ ulp of the product + ulp of the new a_ij, where both were formed].
 */
int mpref_factor_ball(int64_t n, int32_t P, uint32_t *limbs, int64_t *exp, int32_t *sign,
                      uint32_t *Dl, int64_t *De, int32_t *Ds, int32_t *info, int32_t input_ulp,
                      uint32_t *rdm, int64_t *rde, int32_t threads)
{
    if (n < 0 || P < 1 || !info || (n > 0 && (!limbs || !exp || !sign || !Dl || !De || !Ds || !rdm || !rde)))
        return -1;
    rad_t *R = (rad_t *)malloc(sizeof(rad_t) * (size_t)(n > 0 ? n * n : 1));
    rad_t *LR = (rad_t *)malloc(sizeof(rad_t) * (size_t)(n > 0 ? n : 1));
    if (!R || !LR) { free(R); free(LR); return -1; }
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = 0; j < n; j++)
            R[i * n + j] = input_ulp ? rad_unit(EL(i, j), EE(i, j), P) : rad_zero();
    *info = 0;
    for (int64_t k = 0; k < n; k++) {
        /* the radii of the pivot and of column k before the step */
        rad_t ru = R[k * n + k];
        int64_t eu = EE(k, k);
        int uz = num_is_zero(EL(k, k), P);
        int rc = mpref_factor_range(n, P, limbs, exp, sign, Dl, De, Ds, info, k, k + 1, threads);
        if (rc != 0) { free(R); free(LR); return rc; }
        if (*info != 0) {  /* the elimination stopped: no bound from here on */
            for (int64_t t = k; t < n; t++) { rdm[t] = 0xFFFFFFFFu; rde[t] = RAD_INF; }
            break;
        }
        /* D_k */
        rad_t rd;
        if (k == 0) {
            rd = ru;
        } else {
            rad_t rp = rad_make(rdm[k - 1], rde[k - 1]);
            rad_t t1 = rad_prod(rad_abs_bound(Dl + (k - 1) * P, De[k - 1], P), ru);
            rad_t t2 = rad_prod(uz ? rad_zero() : rad_two_to(eu), rp);
            rad_t t3 = rad_prod(rp, ru);
            rd = rad_sum(rad_sum(t1, t2), rad_sum(t3, rad_unit(Dl + k * P, De[k], P)));
        }
        rdm[k] = rd.m;
        rde[k] = rd.e;
        /* the multipliers (now in column k) */
        for (int64_t i = k + 1; i < n; i++) {
            if (uz || !(ru.m == 0 || (!rad_isinf(ru) && ru.e + 32 <= eu - 2))) {
                LR[i] = rad_inf();
                continue;
            }
            rad_t num = rad_sum(R[i * n + k], rad_prod(rad_abs_bound(EL(i, k), EE(i, k), P), ru));
            if (num.m != 0 && !rad_isinf(num)) num.e += 2 - eu;   /* times 2^(2 - e(u)), exact */
            LR[i] = rad_sum(num, rad_unit(EL(i, k), EE(i, k), P));
        }
        /* the trailing block */
        for (int64_t i = k + 1; i < n; i++) {
            rad_t rl = LR[i];
            int lz = num_is_zero(EL(i, k), P);
            for (int64_t j = k + 1; j < n; j++) {
                int ukz = num_is_zero(EL(k, j), P);
                rad_t ruj = R[k * n + j];
                rad_t r = R[i * n + j];
                r = rad_sum(r, rad_prod(lz ? rad_zero() : rad_two_to(EE(i, k)), ruj));
                r = rad_sum(r, rad_prod(ukz ? rad_zero() : rad_two_to(EE(k, j)), rl));
                r = rad_sum(r, rad_prod(rl, ruj));
                if (!lz && !ukz) {
                    r = rad_sum(r, rad_two_to(EE(i, k) + EE(k, j) - 32 * (int64_t)P));
                    r = rad_sum(r, rad_unit(EL(i, j), EE(i, j), P));
                }
                R[i * n + j] = r;
            }
            R[i * n + k] = rl;
        }
    }
    if (*info < 0)  /* an exponent overflow: no bound anywhere */
        for (int64_t t = 0; t < n; t++) { rdm[t] = 0xFFFFFFFFu; rde[t] = RAD_INF; }
    free(R);
    free(LR);
    return 0;
}
