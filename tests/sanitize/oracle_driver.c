/* Runs the CPU oracle's entry points under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_sanitizers.py): the
 * factorisation, minors, adjugate, ball bounds, step ranges and truncation
 * at small and at the largest limb counts (the arithmetic keeps arrays of up
 * to ~37 KB on the stacks of its worker threads at 1024 limbs), plus the
 * argument checks.  Exit status 0 and no sanitizer report is a pass. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mpref.h"

static uint64_t rng = 88172645463325252ull;
static uint32_t next32(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (uint32_t)rng;
}

static int run(int64_t n, int32_t P, int threads) {
    size_t nn = (size_t)(n * n);
    uint32_t *l = malloc(sizeof(uint32_t) * nn * (size_t)P);
    int64_t *e = malloc(sizeof(int64_t) * nn);
    int32_t *s = malloc(sizeof(int32_t) * nn);
    uint32_t *Dl = malloc(sizeof(uint32_t) * (size_t)(n * P));
    int64_t *De = malloc(sizeof(int64_t) * (size_t)n);
    int32_t *Ds = malloc(sizeof(int32_t) * (size_t)n);
    uint32_t *cl = malloc(sizeof(uint32_t) * (size_t)(n * P));
    int64_t *ce = malloc(sizeof(int64_t) * (size_t)n);
    int32_t *cs = malloc(sizeof(int32_t) * (size_t)n);
    uint32_t *tl = malloc(sizeof(uint32_t) * nn * (size_t)P);
    int64_t *te = malloc(sizeof(int64_t) * nn);
    int32_t *ts = malloc(sizeof(int32_t) * nn);
    uint32_t *rm = malloc(sizeof(uint32_t) * (size_t)n);
    int64_t *re = malloc(sizeof(int64_t) * (size_t)n);
    for (size_t t = 0; t < nn; t++) {
        for (int q = 0; q < P; q++) l[t * P + q] = next32();
        l[t * P + P - 1] |= 0x80000000u;
        e[t] = (int64_t)(next32() % 9) - 4;
        s[t] = (int32_t)(next32() & 1);
    }
    int32_t info = 0;
    int rc = 0;
    uint32_t *l2 = malloc(sizeof(uint32_t) * nn * (size_t)P);
    int64_t *e2 = malloc(sizeof(int64_t) * nn);
    int32_t *s2 = malloc(sizeof(int32_t) * nn);
    memcpy(l2, l, sizeof(uint32_t) * nn * (size_t)P);
    memcpy(e2, e, sizeof(int64_t) * nn);
    memcpy(s2, s, sizeof(int32_t) * nn);
    rc |= mpref_factor_ball(n, P, l2, e2, s2, Dl, De, Ds, &info, 1, rm, re, threads);
    rc |= mpref_factor(n, P, l, e, s, Dl, De, Ds, &info, threads);
    rc |= mpref_minors(n, P, l, e, s, Dl, De, Ds, cl, ce, cs, threads);
    rc |= mpref_adjugate_t(n, P, l, e, s, Dl, De, Ds, tl, te, ts, threads);
    rc |= mpref_truncate((int64_t)nn, P, P > 2 ? P / 2 : P, l, e, s, tl, te, ts);
    free(l); free(e); free(s); free(Dl); free(De); free(Ds); free(cl); free(ce); free(cs);
    free(tl); free(te); free(ts); free(rm); free(re); free(l2); free(e2); free(s2);
    return rc;
}

int main(void) {
    int rc = 0;
    rc |= run(1, 1, 1);
    rc |= run(7, 3, 2);
    rc |= run(12, 64, 4);
    rc |= run(5, 1024, 4);
    /* argument checks: every one must refuse, not touch memory */
    int32_t info = 0;
    if (mpref_factor(-1, 4, NULL, NULL, NULL, NULL, NULL, NULL, &info, 1) != -1) rc |= 1;
    if (mpref_factor_range(3, 4, NULL, NULL, NULL, NULL, NULL, NULL, &info, 0, 1, 1) != -1) rc |= 1;
    if (mpref_truncate(2, 2, 3, NULL, NULL, NULL, NULL, NULL, NULL) != -1) rc |= 1;
    if (mpref_factor_ball(2, 0, NULL, NULL, NULL, NULL, NULL, NULL, &info, 0, NULL, NULL, 1) != -1) rc |= 1;
    printf("oracle driver: %s\n", rc ? "FAILED" : "ok");
    return rc ? 1 : 0;
}
