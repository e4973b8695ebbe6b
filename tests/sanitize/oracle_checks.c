/*
 * The CPU oracle under the address and undefined-behaviour sanitizers: random
 * rule lists (prefix lengths 0 to 32, so both shift edges are taken) and
 * packets, every thread count from 1 to 17 over batches of 0, 1 and 5,000
 * packets, plus an empty rule list.  Results must agree across thread counts
 * and with the rule-check count the oracle reports.  Exit status 0 on success.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/fwref.c"

static uint64_t state = 99;
static uint64_t next(void)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint32_t below(uint32_t n) { return (uint32_t)((next() >> 11) % n); }

int main(void)
{
    enum { R = 700, N = 5000 };
    uint32_t *src = malloc(R * 4), *dst = malloc(R * 4);
    uint8_t *sl = malloc(R), *dl = malloc(R), *pr = malloc(R), *pa = malloc(R), *ac = malloc(R);
    uint16_t *slo = malloc(R * 2), *shi = malloc(R * 2), *dlo = malloc(R * 2), *dhi = malloc(R * 2);
    for (int r = 0; r < R; ++r) {
        src[r] = (uint32_t)next();
        dst[r] = (uint32_t)next();
        sl[r] = (uint8_t)below(33);
        dl[r] = (uint8_t)below(33);
        slo[r] = (uint16_t)below(65536);
        shi[r] = (uint16_t)(slo[r] + below(65536 - slo[r]));
        dlo[r] = (uint16_t)below(65536);
        dhi[r] = (uint16_t)(dlo[r] + below(65536 - dlo[r]));
        pr[r] = (uint8_t)below(256);
        pa[r] = (uint8_t)(below(3) == 0);
        ac[r] = (uint8_t)below(2);
    }
    uint32_t *ps = malloc(N * 4), *pd = malloc(N * 4);
    uint16_t *pss = malloc(N * 2), *pds = malloc(N * 2);
    uint8_t *pp = malloc(N);
    for (int i = 0; i < N; ++i) {
        int k = (int)below(R);
        ps[i] = below(2) ? src[k] : (uint32_t)next();
        pd[i] = below(2) ? dst[k] : (uint32_t)next();
        pss[i] = (uint16_t)below(65536);
        pds[i] = (uint16_t)below(65536);
        pp[i] = (uint8_t)below(256);
    }
    int32_t *want = malloc(N * 4), *got = malloc(N * 4);
    uint8_t *wa = malloc(N), *ga = malloc(N);
    int failures = 0;
    for (int rules = 0; rules <= R; rules += R) {   /* an empty list, then all of them */
        ref_rules rs = {(uint32_t)rules, src, dst, sl, dl, slo, shi, dlo, dhi, pr, pa, ac, 1};
        const uint64_t sizes[3] = {0, 1, N};
        for (int s = 0; s < 3; ++s) {
            ref_packets pk = {sizes[s], ps, pd, pss, pds, pp};
            uint64_t st0[2] = {0, 0};
            if (ref_classify(&rs, &pk, want, wa, 1, st0) != 0) return 2;
            uint64_t checks = 0;
            for (uint64_t i = 0; i < sizes[s]; ++i) {
                checks += want[i] < 0 ? (uint64_t)rules : (uint64_t)want[i] + 1;
                if (want[i] < -1 || want[i] >= rules) ++failures;
                if (want[i] < 0 && wa[i] != 1) ++failures;   /* default action */
            }
            if (checks != st0[0]) {
                fprintf(stderr, "rule checks %llu, counted %llu\n", (unsigned long long)st0[0],
                        (unsigned long long)checks);
                ++failures;
            }
            for (int t = 2; t <= 17; ++t) {
                memset(got, 0x5A, N * 4);
                uint64_t st[2];
                if (ref_classify(&rs, &pk, got, ga, t, st) != 0) return 2;
                if (sizes[s] && (memcmp(got, want, sizes[s] * 4) || memcmp(ga, wa, sizes[s]))) {
                    fprintf(stderr, "threads %d differ (rules %d, packets %llu)\n", t, rules,
                            (unsigned long long)sizes[s]);
                    ++failures;
                }
                if (st[0] != st0[0] || st[1] != st0[1]) ++failures;
            }
        }
    }
    free(src); free(dst); free(sl); free(dl); free(pr); free(pa); free(ac);
    free(slo); free(shi); free(dlo); free(dhi);
    free(ps); free(pd); free(pss); free(pds); free(pp);
    free(want); free(got); free(wa); free(ga);
    if (failures) {
        fprintf(stderr, "%d oracle check(s) failed\n", failures);
        return 1;
    }
    printf("oracle checks passed\n");
    return 0;
}
