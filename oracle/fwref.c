/*
 * Sequential CPU first-match oracle.  TEST INFRASTRUCTURE ONLY: the tests, the
 * smoke check and the benchmark's CPU-baseline leg use it to check the GPU
 * path; the product never calls it.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * What it computes (paper, Section I and Section IV): a packet filter holds an
 * ordered list of rules; each rule is a 5-tuple (source address, destination
 * address, source port, destination port, protocol) plus an action, and a
 * field that a rule leaves unspecified matches every value.  Rules are tried
 * in insertion order and the first one that matches decides the packet's
 * fate ("first match"); a packet that no rule matches is denied ("default
 * deny").  Packets are processed one after the other.
 *
 * Readings where the paper is silent:
 *  - addresses are CIDR prefixes (base, length); length 0 is the wildcard
 *    and the bits of the base below the prefix are ignored;
 *  - ports are inclusive ranges [lo, hi]; the wildcard is [0, 65535];
 *  - protocol is either one value or "any" (a separate flag, so protocol 0
 *    is an ordinary value);
 *  - ports are compared for every protocol (a plain 5-dimensional box);
 *  - no match gives rule index -1 and the default action.
 *
 * The address test is written in the prefix/XOR form, not as a range, so the
 * GPU path's range normalisation is checked by an independent formulation.
 */
#include <pthread.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

typedef struct ref_rules {
    uint32_t n;
    const uint32_t *src_ip, *dst_ip;
    const uint8_t *src_plen, *dst_plen;
    const uint16_t *sport_lo, *sport_hi, *dport_lo, *dport_hi;
    const uint8_t *proto, *proto_any, *action;
    uint8_t default_action;
} ref_rules;

typedef struct ref_packets {
    uint64_t n;
    const uint32_t *src_ip, *dst_ip;
    const uint16_t *sport, *dport;
    const uint8_t *proto;
} ref_packets;

/* Address `ip` lies in prefix (base, len): the top `len` bits agree. */
static int in_prefix(uint32_t ip, uint32_t base, unsigned len)
{
    if (len == 0)
        return 1;                         /* unspecified field: all values */
    return ((ip ^ base) >> (32u - len)) == 0;
}

/*
 * First matching rule of one packet; -1 when none matches.  `*tests`, when
 * given, receives the number of field tests evaluated with the short-circuit
 * order destination, source, ports, protocol (ports count as one test).
 */
static int32_t first_match(const ref_rules *rs, uint32_t src, uint32_t dst,
                           uint16_t sport, uint16_t dport, uint8_t proto,
                           uint64_t *tests)
{
    uint64_t t = 0;
    for (uint32_t r = 0; r < rs->n; ++r) {
        ++t;
        if (!in_prefix(dst, rs->dst_ip[r], rs->dst_plen[r]))
            continue;
        ++t;
        if (!in_prefix(src, rs->src_ip[r], rs->src_plen[r]))
            continue;
        ++t;
        if (!(rs->sport_lo[r] <= sport && sport <= rs->sport_hi[r] &&
              rs->dport_lo[r] <= dport && dport <= rs->dport_hi[r]))
            continue;
        ++t;
        if (!(rs->proto_any[r] || rs->proto[r] == proto))
            continue;
        if (tests)
            *tests += t;
        return (int32_t)r;
    }
    if (tests)
        *tests += t;
    return -1;
}

typedef struct job {
    const ref_rules *rs;
    const ref_packets *pk;
    uint64_t begin, end;
    int32_t *out_idx;
    uint8_t *out_act;
    uint64_t checks, tests;
} job;

static void *run_job(void *arg)
{
    job *j = (job *)arg;
    uint64_t checks = 0, tests = 0;
    for (uint64_t i = j->begin; i < j->end; ++i) {
        int32_t r = first_match(j->rs, j->pk->src_ip[i], j->pk->dst_ip[i],
                                j->pk->sport[i], j->pk->dport[i], j->pk->proto[i],
                                &tests);
        j->out_idx[i] = r;
        j->out_act[i] = r < 0 ? j->rs->default_action : j->rs->action[r];
        checks += r < 0 ? (uint64_t)j->rs->n : (uint64_t)r + 1;
    }
    j->checks = checks;
    j->tests = tests;
    return NULL;
}

/*
 * Classify pk->n packets.  Packets are independent, so `threads` workers each
 * take a contiguous chunk; every packet is still scanned sequentially.
 * `stats`, when given, receives {rule checks, field tests}: a rule check per
 * rule visited (first-match index + 1, or the rule count when unmatched).
 * Returns 0, or -1 when a worker thread could not be started.
 */
int ref_classify(const ref_rules *rs, const ref_packets *pk, int32_t *out_idx,
                 uint8_t *out_act, int threads, uint64_t *stats)
{
    if (threads < 1)
        threads = 1;
    if ((uint64_t)threads > pk->n)
        threads = pk->n ? (int)pk->n : 1;
    job *jobs = (job *)calloc((size_t)threads, sizeof(job));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs);
        free(tid);
        return -1;
    }
    uint64_t chunk = (pk->n + (uint64_t)threads - 1) / (uint64_t)threads;
    int rc = 0, started = 0;
    for (int t = 0; t < threads; ++t) {
        jobs[t].rs = rs;
        jobs[t].pk = pk;
        jobs[t].begin = (uint64_t)t * chunk < pk->n ? (uint64_t)t * chunk : pk->n;
        jobs[t].end = jobs[t].begin + chunk < pk->n ? jobs[t].begin + chunk : pk->n;
        jobs[t].out_idx = out_idx;
        jobs[t].out_act = out_act;
    }
    if (threads == 1) {
        run_job(&jobs[0]);
    } else {
        for (int t = 0; t < threads; ++t) {
            if (pthread_create(&tid[t], NULL, run_job, &jobs[t]) != 0) {
                rc = -1;
                break;
            }
            ++started;
        }
        for (int t = 0; t < started; ++t)
            pthread_join(tid[t], NULL);
    }
    if (stats && rc == 0) {
        stats[0] = stats[1] = 0;
        for (int t = 0; t < threads; ++t) {
            stats[0] += jobs[t].checks;
            stats[1] += jobs[t].tests;
        }
    }
    free(jobs);
    free(tid);
    return rc;
}
