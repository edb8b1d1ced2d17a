/*
 * mpref.h -- CPU oracle for multiprecision Gaussian elimination without
 * pivoting (Beliakov & Matiyasevich, "A Parallel Algorithm for Calculation
 * of Large Determinants with High Accuracy for GPUs and MPI clusters").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the GPU library
 * against a plain, slow, independently written reference.  The product path
 * never links, loads or calls it, and it shares no code, header or table with
 * the GPU library.
 *
 * Number format (same definition as the GPU library, written out again here):
 *   value = (-1)^s * m * 2^(e - 32P),  m an integer with P little-endian
 *   uint32 limbs, 2^(32P-1) <= m < 2^(32P) (top bit set), e int64, s in {0,1}.
 *   Zero is canonical: s = 0, e = 0, m = 0.
 * Every arithmetic result is the exact real result truncated toward zero to
 * p = 32P significant bits (RZ_p).
 *
 * Host layouts used by this oracle (element-contiguous):
 *   matrix limbs [n][n][P] uint32, exp [n][n] int64, sign [n][n] int32;
 *   vector limbs [n][P],          exp [n],      sign [n].
 *
 * Return codes: 0 ok, -1 bad argument.  Numeric outcomes go to *info:
 *   0 ok; k > 0 the pivot of step k (1-based) is exactly zero; -1 a pivot or
 *   leading determinant has |exponent| > 2^62.
 */
#ifndef MPREF_H
#define MPREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Single-number primitives (exact result, then RZ_p). */
void mpref_mul(int32_t P, const uint32_t *am, int64_t ae, int32_t as,
               const uint32_t *bm, int64_t be, int32_t bs,
               uint32_t *rm, int64_t *re, int32_t *rs);
void mpref_add(int32_t P, const uint32_t *am, int64_t ae, int32_t as,
               const uint32_t *bm, int64_t be, int32_t bs,
               uint32_t *rm, int64_t *re, int32_t *rs);
void mpref_sub(int32_t P, const uint32_t *am, int64_t ae, int32_t as,
               const uint32_t *bm, int64_t be, int32_t bs,
               uint32_t *rm, int64_t *re, int32_t *rs);
/* returns -1 (and writes nothing) when b is zero */
int mpref_div(int32_t P, const uint32_t *am, int64_t ae, int32_t as,
              const uint32_t *bm, int64_t be, int32_t bs,
              uint32_t *rm, int64_t *re, int32_t *rs);

/* Exact unsigned big-integer helpers, exported so tests can pin them. */
void mpref_bn_mul(uint32_t *out, const uint32_t *a, int32_t na,
                  const uint32_t *b, int32_t nb);
int mpref_bn_divmod(uint32_t *q, uint32_t *r, const uint32_t *u, int32_t m,
                    const uint32_t *v, int32_t n);

/* Gaussian elimination without pivoting, in place (Algorithm 1, steps 1-2.2.2).
 * On return the matrix holds U on and above the diagonal and the multipliers
 * l_ik = a_ik / a_kk below it; D receives the leading determinants D_1..D_n. */
int mpref_factor(int64_t n, int32_t P, uint32_t *limbs, int64_t *exp, int32_t *sign,
                 uint32_t *Dl, int64_t *De, int32_t *Ds, int32_t *info, int32_t threads);
/* Steps k_begin .. k_end-1 of the same elimination, continuing from the state
 * (matrix, D, *info) an earlier range left; *info is not reset. */
int mpref_factor_range(int64_t n, int32_t P, uint32_t *limbs, int64_t *exp, int32_t *sign,
                       uint32_t *Dl, int64_t *De, int32_t *Ds, int32_t *info, int64_t k_begin,
                       int64_t k_end, int32_t threads);
/* mpref_factor and, for every leading determinant, a rigorous radius:
 * |D_k - D*_k| <= rdm[k] 2^rde[k] with D*_k the exact leading determinant of
 * the input (input_ulp: every input entry within one unit in its last place of
 * an exact value); rde[k] == INT64_MAX: no bound.  Ball arithmetic with
 * radii rounded up (see mpref.c). */
int mpref_factor_ball(int64_t n, int32_t P, uint32_t *limbs, int64_t *exp, int32_t *sign,
                      uint32_t *Dl, int64_t *De, int32_t *Ds, int32_t *info, int32_t input_ulp,
                      uint32_t *rdm, int64_t *rde, int32_t threads);
/* RZ to 32*P2 bits (P2 <= P) of `count` numbers: the top P2 limbs. */
int mpref_truncate(int64_t count, int32_t P, int32_t P2, const uint32_t *limbs, const int64_t *exp,
                   const int32_t *sign, uint32_t *ol, int64_t *oe, int32_t *os);

/* Signed last-column cofactors c_i = (-1)^(i+n) M_{i,n} from factor's output. */
int mpref_minors(int64_t n, int32_t P, const uint32_t *limbs, const int64_t *exp,
                 const int32_t *sign, const uint32_t *Dl, const int64_t *De,
                 const int32_t *Ds, uint32_t *cl, int64_t *ce, int32_t *cs,
                 int32_t threads);

/* Full adjugate from factor's output: adjT[i][j] = C_ij = d det / d a_ij. */
int mpref_adjugate_t(int64_t n, int32_t P, const uint32_t *limbs, const int64_t *exp,
                     const int32_t *sign, const uint32_t *Dl, const int64_t *De,
                     const int32_t *Ds, uint32_t *tl, int64_t *te, int32_t *ts,
                     int32_t threads);

/* (mantissa, exponent) pair: mant = (-1)^s * RZ_53(m / 2^p), in [0.5, 1). */
void mpref_to_f64(int64_t count, int32_t P, const uint32_t *limbs, const int64_t *exp,
                  const int32_t *sign, double *mant, int64_t *eout);

#ifdef __cplusplus
}
#endif
#endif
