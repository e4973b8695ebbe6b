/*
 * fw.h -- C interface of the MI355X (gfx950) first-match packet classifier.
 *
 * The operation (paper, Section I): an ordered list of filtering rules is
 * consulted in insertion order; the first rule that matches a packet decides
 * its action ("first match"); a packet that no rule matches is denied
 * ("default deny").  Each rule (paper, Section IV) is a 5-tuple -- source and
 * destination IPv4 address, source and destination port, protocol -- plus an
 * action, and a field that a rule leaves unspecified matches every value.
 *
 * Four ways to compute the same result are offered:
 *  - packet split: every GPU lane owns whole packets and walks the whole
 *    rule list (the paper's data-parallel firewall, Section IV-A: each node
 *    holds a duplicate of the policy, each packet goes to one node);
 *  - rule split: the rule list is cut into P contiguous partitions, one wave
 *    per partition and group of 16 packets (8 for batches under 2,097,152
 *    packets) holds 64 of its rules in its lanes, and the partial first matches are merged by a minimum over rule
 *    indices, within the wave as the lowest matching lane and across
 *    partitions by an atomic minimum (the paper's function-parallel firewall, Section IV-B,
 *    where each node holds a part of the policy; the paper merges on the CPU,
 *    here the merge runs on the GPU);
 *  - learned index: a small network trained on the rule list's destination
 *    interval boundaries locates each packet's destination interval, and
 *    only exact candidate lists are scanned: the interval's own list, the
 *    list of the packet's source interval among destination-wildcard rules,
 *    and a port/protocol bit-vector table for rules that leave both
 *    addresses unspecified.  Not in the paper; its results are identical to
 *    the scan by construction.
 *  - hybrid: a work-group per 64 packets whose waves split the rule list
 *    (the paper's Section IV-C).
 *
 * Conventions for every entry point:
 *  - all integers are host byte order: 10.0.0.1 is 0x0A000001;
 *  - packet and output buffers are DEVICE pointers owned by the caller, each
 *    16-byte aligned; they must stay valid until the work on the given HIP
 *    stream has completed;
 *  - classification calls are asynchronous on the given stream (the null
 *    stream when none is given) and return once the work is enqueued;
 *  - errors come back as an fw_status; fw_last_error() then describes the
 *    most recent failure of the calling thread.  Errors found while
 *    enqueueing are reported at once; a device fault in earlier asynchronous
 *    work is reported by a later call as FW_E_DEVICE;
 *  - a ruleset is immutable once loaded (building its learned index aside)
 *    and may be used concurrently by classification calls on different
 *    streams.
 */
#ifndef FW_H
#define FW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fw_status {
    FW_OK = 0,
    FW_E_INVAL = -1,    /* bad argument or invalid rule */
    FW_E_ALIGN = -2,    /* a device buffer is not 16-byte aligned */
    FW_E_NOMEM = -3,    /* device or host allocation failed, or over a memory budget */
    FW_E_DEVICE = -4,   /* a HIP runtime call or kernel failed */
    FW_E_NOINDEX = -5   /* learned mode asked for, but no learned index is built */
} fw_status;

typedef enum fw_action { FW_DROP = 0, FW_ACCEPT = 1 } fw_action;

typedef enum fw_mode {
    FW_MODE_AUTO = 0,          /* learned index when built; else by batch size: packet
                                  split from 262,144 packets, below that rule split over 64
                                  partitions for batches up to 4,096 packets with at least
                                  2,048 reachable rules, else the hybrid over 16 partitions
                                  (the split forms wait for a fraction of the rule list per
                                  packet, which is what a small batch's latency needs) */
    FW_MODE_PACKET_SPLIT = 1,  /* data-parallel scan (paper Section IV-A) */
    FW_MODE_RULE_SPLIT = 2,    /* function-parallel scan (paper Section IV-B) */
    FW_MODE_LEARNED = 3,       /* learned destination index + candidate scan */
    FW_MODE_HYBRID = 4         /* a workgroup per packet group, its waves split the rules
                                  (paper Section IV-C) */
} fw_mode;

/*
 * One rule, 24 bytes, host memory.  Fields (paper Section IV):
 *  src_ip/src_plen, dst_ip/dst_plen: CIDR prefix; length 0..32, 0 matches
 *      every address; bits of the base below the prefix are ignored;
 *  sport_lo..sport_hi, dport_lo..dport_hi: inclusive port ranges; [0, 65535]
 *      matches every port; ports are compared for every protocol;
 *  proto, proto_any: proto_any != 0 matches every protocol, else the packet's
 *      protocol must equal proto (0 is an ordinary value);
 *  action: FW_DROP or FW_ACCEPT (the paper's QUEUE target is not supported).
 */
typedef struct fw_rule {
    uint32_t src_ip, dst_ip;
    uint8_t src_plen, dst_plen;
    uint8_t proto, proto_any;
    uint16_t sport_lo, sport_hi, dport_lo, dport_hi;
    uint8_t action;
    uint8_t _pad[3];
} fw_rule;

/* A batch of packet headers as five device arrays (structure of arrays),
 * each 16-byte aligned, element i of each array belonging to packet i. */
typedef struct fw_packets {
    const uint32_t *src_ip;
    const uint32_t *dst_ip;
    const uint16_t *src_port;
    const uint16_t *dst_port;
    const uint8_t *proto;
} fw_packets;

/* Opaque ruleset handle: the library owns its host and device memory. */
typedef struct fw_ruleset fw_ruleset;

typedef struct fw_classify_opts {
    uint32_t mode;          /* fw_mode */
    uint32_t partitions;    /* rule split / hybrid: partition count P >= 1; 0 means 16 */
    void *stream;           /* hipStream_t to enqueue on; NULL = null stream */
    uint32_t lookup;        /* learned mode: 0 = network + error window (default),
                               1 = full binary search with the network skipped */
    uint32_t packets_per_lane; /* packet split, learned and hybrid mode: 1, 2 or 4 (rule
                                  split ignores it); 0 = library default: the most (up to 4
                                  for packet split, 2 for learned) that still gives the
                                  launch 8,192 waves, so small batches use fewer per lane;
                                  hybrid: 1 while n * partitions / 64 <= 8,192, else 4 */
    uint64_t *window_misses;   /* learned mode, optional HOST pointer: the call's statistics.
                                  When given, the call counts in memory of its own how many
                                  packets' error window missed (they fell back to a full
                                  search), waits for its work (the call is then synchronous)
                                  and stores the count; NULL keeps the call asynchronous.
                                  The other modes store 0. */
} fw_classify_opts;

/*
 * Compile `n_rules` rules into a device-resident ruleset (paper Section I: the
 * list's order is its priority, the first match decides, and packets no rule
 * matches take the default action, deny in the paper; Section IV: each rule
 * is a 5-tuple plus an action, an unspecified field matching every value).
 * Rule i keeps index i.  Every field becomes an unsigned range [lo, lo + w]
 * (a prefix of length L keeps the top L bits of its base), packed into a
 * 32-byte device record; the list is also grouped by each rule's most
 * selective field and cut after its first rule that matches every packet
 * (rules past it can never be a first match).  The rules are
 * copied; the caller may free `rules` on return.  `default_action` (FW_DROP
 * or FW_ACCEPT) applies to packets no rule matches.  n_rules may be 0 (every
 * packet then takes the default) and at most 16,777,216.
 * Errors: FW_E_INVAL for a null `out`, null `rules` with n_rules > 0, a
 * prefix length above 32, a port range with lo > hi, or an action or
 * default_action above 1; FW_E_NOMEM / FW_E_DEVICE from the device.  On any
 * error *out is left NULL.
 */
fw_status fw_load_ruleset(const fw_rule *rules, uint32_t n_rules, uint8_t default_action,
                          fw_ruleset **out);

/* Free a ruleset and its learned index.  Waits for all device work first.
 * NULL is accepted and ignored. */
fw_status fw_free_ruleset(fw_ruleset *rs);

/* Number of rules in a ruleset (0 for NULL). */
uint32_t fw_ruleset_size(const fw_ruleset *rs);

/*
 * First match of `n` packets (paper Sections I and IV): out_rule_idx[i] is the
 * lowest index of a rule matching packet i, or -1; out_action[i] is that
 * rule's action, or the ruleset's default.  Every i < n is written exactly
 * once.  Mode FW_MODE_AUTO on the null stream.  n == 0 enqueues nothing.
 * Errors: FW_E_INVAL (null ruleset, packets or outputs with n > 0),
 * FW_E_ALIGN (a buffer not 16-byte aligned), FW_E_DEVICE (launch failure or
 * an earlier device fault).
 */
fw_status fw_classify(const fw_ruleset *rs, const fw_packets *pk, size_t n,
                      int32_t *out_rule_idx, uint8_t *out_action);

/* As fw_classify, with a mode, a partition count, a stream and learned-index
 * options (`opts` may be NULL).  FW_E_NOINDEX when FW_MODE_LEARNED is asked
 * for before fw_build_learned_index succeeded; FW_E_INVAL for an unknown
 * mode, partitions above the rule count's limit of 65,536, or a
 * packets_per_lane other than 0, 1, 2 or 4. */
fw_status fw_classify_ex(const fw_ruleset *rs, const fw_packets *pk, size_t n,
                         int32_t *out_rule_idx, uint8_t *out_action,
                         const fw_classify_opts *opts);

/* ------------------------------------------------------------------ learned index
 * Not in the paper.  Destination elementary intervals: B is {0} with every
 * rule's destination range start and every range end + 1 (when below 2^32),
 * sorted and de-duplicated; interval j is [B[j], B[j+1]).  Candidate list C_j
 * is the ascending list of rules whose destination range contains interval j;
 * the first match over C_j equals the first match over all rules.  A
 * two-stage recursive model index (one stage-1 network routing to `experts`
 * stage-2 networks, each 1 -> hidden -> 1 with ReLU) predicts j from a
 * destination address; a per-expert maximum error bounds the search window,
 * and a window miss falls back to a full binary search, so results never
 * depend on the network's accuracy. */

typedef struct fw_index_opts {
    uint32_t experts;       /* stage-2 experts, 1..256; 0 = 64 */
    uint32_t hidden;        /* hidden units of every network, 1..32; 0 = 32 */
    uint32_t epochs1;       /* stage-1 Adam steps; 0 = library default */
    uint32_t epochs2;       /* stage-2 Adam steps; 0 = library default */
    float lr;               /* Adam learning rate; 0 = library default */
    uint32_t seed;          /* weight initialisation seed */
    uint32_t train;         /* 0 = keep the random initial weights (ablation) */
    uint32_t use_mfma;      /* 1 = bf16 MFMA for the weight-gradient products (default),
                               0 = plain fp32 reduction (for checking) */
    uint32_t zero_error_bounds; /* testing only: store every error bound as 0, so most
                                   lookups miss their window and take the full search */
    uint64_t mem_budget;    /* device bytes the index may use; 0 = no limit */
    void *stream;           /* hipStream_t; NULL = null stream.  The build waits for it. */
} fw_index_opts;

typedef struct fw_index_stats {
    uint32_t n_boundaries;  /* |B| */
    uint32_t n_global;      /* destination-wildcard candidates kept (shared by all intervals) */
    uint64_t n_list_entries;/* per-interval candidate entries kept */
    uint32_t max_list;      /* longest per-interval list */
    uint32_t err_max;       /* largest per-expert error bound (positions) */
    float err_mean;         /* mean per-expert error bound */
    float loss1, loss2;     /* final training losses of stage 1 and stage 2 */
    float train_ms;         /* wall time of the GPU training */
    uint32_t weights_rounded; /* stage-2 weights that IEEE half, the lookup's storage
                               * for them, does not hold exactly even with each hidden
                               * unit's exact power-of-two scaling chosen to avoid it;
                               * rounded to nearest (an input weight whose unit has a
                               * zero output weight is not counted: that unit adds
                               * nothing); 0: the lookup's products are those of the
                               * bf16 network */
    uint64_t device_bytes;  /* device memory held by the index */
} fw_index_stats;

/* Build (or rebuild) the learned index of `rs`: intervals and candidate lists
 * on the host, network training on the GPU with the library's own forward,
 * backward and Adam kernels, bf16 quantisation, and error bounds measured
 * with the inference kernel itself.  `opts` and `stats` may be NULL.
 * Synchronous.  Must not run concurrently with other calls on `rs`; work
 * they enqueued earlier may still be running: a rebuild waits for the device
 * to finish it before it frees the previous index.
 * Errors: FW_E_INVAL (bad options), FW_E_NOMEM (over mem_budget or
 * allocation failure; `rs` stays usable in the scan modes), FW_E_DEVICE. */
fw_status fw_build_learned_index(fw_ruleset *rs, const fw_index_opts *opts,
                                 fw_index_stats *stats);

/* Interval index j of each destination address in `keys` (device, n entries,
 * 16-byte aligned), written to `out_interval` (device int32), through the
 * learned lookup (network + window, or binary search when `lookup` == 1).
 * Asynchronous on `stream`.  FW_E_NOINDEX without an index. */
fw_status fw_index_lookup(const fw_ruleset *rs, const uint32_t *keys, size_t n,
                          int32_t *out_interval, uint32_t lookup, void *stream);

/* Copy parts of the learned index to host memory.  `what`:
 *  0 = boundaries B (uint32, |B| entries);
 *  1 = per-interval list offsets (uint32, |B| + 1 entries);
 *  2 = per-interval list entries (uint32 rule indices);
 *  3 = global list (uint32 rule indices of destination-wildcard candidates);
 *  4 = per-expert error bounds (uint32, `experts` entries);
 *  5 = network weights as float (stage 1 then the experts, each
 *      [w1 (H), b1 (H), w2 (H), b2]), after bf16 quantisation;
 *  6 = source boundaries of the destination-wildcard candidates that specify a
 *      source (uint32);
 *  7 = their per-source-interval list offsets (uint32, count of 6 + 1);
 *  8 = their per-source-interval list entries (uint32 rule indices);
 *  9 = the candidates with source and destination both unspecified (uint32
 *      rule indices), tested for every packet: the first 64 that are not
 *      catch-alls through a port/protocol bit-vector table, the rest by a scan;
 * 10 = that table as bytes: uint64 protocol masks [256], source-port interval
 *      masks [130], destination-port interval masks [130], uint32 interval
 *      starts per port field [132] each (unused entries 0x10000), uint32 rule
 *      entries [68] (rule index | action << 24, 0xFFFFFFFF = none), uint8
 *      high-byte tables [256] per port field (source first); bit r of a mask
 *      stands for the table's r-th rule;
 * 11 = lookup-table shapes (uint32 [5]: rules in the port/protocol table, its
 *      walk steps per source port and per destination port; bits and walk
 *      steps of the source-address bucket table, bits 0 = none);
 * 12 = the source-address bucket table (uint16 [2^bits]): entry h is the
 *      source interval (of 6) holding address h << (32 - bits).
 * Lists 2, 8 and 9 are cut where no later entry can be a first match (after a
 * rule that matches every packet reaching the list, and past the shared
 * list's first catch-all).
 * At most `cap` bytes are written; *size receives the full size in bytes.
 * FW_E_NOINDEX without an index. */
fw_status fw_index_export(const fw_ruleset *rs, uint32_t what, void *host, size_t cap,
                          size_t *size);

/* Closed-loop latency probe: classify n_batches batches one after another,
 * batch k being packets [start[k], start[k] + count[k]) of the DEVICE arrays
 * `pk` (each start a multiple of 16, so every slice stays 16-byte aligned),
 * with `opts` (mode, partitions, stream, ...), waiting for each to complete
 * before the next is enqueued.  seconds[k] (HOST) receives batch k's time from
 * the start of its fw_classify_ex call to the end of the stream
 * synchronisation: the library's own enqueue-to-completion latency, with no
 * binding in between.  Results go to out_rule_idx / out_action at offset 0
 * (at least max(count) entries each).  Errors: those of fw_classify_ex,
 * FW_E_INVAL for a NULL argument or packet field, and FW_E_ALIGN for a start
 * that is not a multiple of 16. */
fw_status fw_closed_loop(const fw_ruleset *rs, const fw_packets *pk, uint32_t n_batches,
                         const size_t *start, const size_t *count, int32_t *out_rule_idx,
                         uint8_t *out_action, const fw_classify_opts *opts, double *seconds);

/* ------------------------------------------------------------------ network kernels
 * Direct access to the training kernels, for checking them against a CPU
 * reference.  One stage of E networks 1 -> H -> 1 (ReLU), parameters laid out
 * per network as [w1 (H), b1 (H), w2 (H), b2]; sample n has input u[n],
 * target t[n] and trains network expert[n].  The loss is the sum over
 * networks of each network's mean squared error over its own samples.  All
 * pointers are HOST memory; the call copies in, runs forward and backward on
 * the device (with bf16 MFMA weight-gradient products when use_mfma != 0)
 * and copies the gradient (E * (3H + 1) floats) and per-network loss (E
 * floats, may be NULL) back.  Synchronous.  Errors: FW_E_INVAL (E or H out
 * of range, NULL argument, an expert index >= E, n above 2^31). */
fw_status fw_rmi_gradients(uint32_t E, uint32_t H, const float *params, size_t n,
                           const float *u, const float *t, const uint32_t *expert,
                           uint32_t use_mfma, float *grad, float *loss);

/* One Adam step (Kingma and Ba, bias-corrected) on `count` parameters with the
 * library's optimiser kernel.  Host pointers; params, m and v are updated in
 * place.  `step` counts from 1.  Synchronous.  Errors: FW_E_INVAL (NULL
 * argument, step 0, count above 2^31). */
fw_status fw_rmi_adam_step(size_t count, float *params, const float *grad, float *m,
                           float *v, uint32_t step, float lr, float beta1, float beta2,
                           float eps);

/* ------------------------------------------------------------------ many chains
 * Not in the paper.  Many independent rulesets ("chains"), each with its own
 * packet batch, classified in one persistent launch: work items (tiles of a
 * chain's packets) are handed out from a device work queue, the most
 * expensive chains first.  Results are exactly those of fw_classify on each
 * chain alone. */

typedef struct fw_chain_batch {
    const fw_ruleset *rs;
    fw_packets pk;           /* device arrays, 16-byte aligned */
    size_t n;
    int32_t *out_rule_idx;   /* device, 16-byte aligned */
    uint8_t *out_action;     /* device, 16-byte aligned */
} fw_chain_batch;

typedef struct fw_multi_opts {
    void *stream;              /* hipStream_t; NULL = null stream */
    uint32_t packets_per_lane; /* 1, 2 or 4; 0 = tuned choice for this batch shape, else 2 */
    uint32_t placement;        /* 0 = tuned (else 4); 4 = each chain as fw_classify_ex
                                  classifies a large batch in mode AUTO: through its learned
                                  index when one is built, else the packet-split scan of its
                                  rules grouped by first test and cut at the first rule that
                                  matches every packet.  The plain rule list in rule order
                                  (the paper's Section IV-A placement study): 1 = rules
                                  through the scalar cache, 2 = rules staged in LDS tiles,
                                  3 = rules read by vector loads (every lane the same
                                  address) */
    uint32_t rule_tile;        /* LDS tile in rules: 256 or 1024; 0 = tuned or 1024 */
    uint32_t _reserved;
} fw_multi_opts;

/* Classify every chain's batch in one persistent launch (asynchronous on the
 * stream).  Chains with n == 0 are skipped.  Errors: FW_E_INVAL (NULL
 * ruleset or buffer, bad option), FW_E_ALIGN, FW_E_DEVICE. */
fw_status fw_classify_multi(const fw_chain_batch *batches, uint32_t n_chains,
                            const fw_multi_opts *opts);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * launch as fw_classify_multi with the same options and results, but its
 * chain descriptor table and work-queue counter live in a static device array
 * the library holds on each GPU it runs on (about 104 KiB, kept until the
 * process ends) instead of memory allocated for the call.  It calls no
 * hipMalloc, hipFree or other device-allocating routine; the array's address
 * is looked up once per device on the first call there.  Every call on one
 * GPU shares that array: calls that overlap on a GPU (on different streams,
 * or from different threads before the earlier launch has finished) race and
 * may give wrong results, so the caller orders them (one stream, or events).
 * The counter is cleared by a kernel at the start of each call.
 * Errors: those of fw_classify_multi, and FW_E_INVAL for more than 1,024
 * chains. */
fw_status fw_classify_multi_noalloc(const fw_chain_batch *batches, uint32_t n_chains,
                                    const fw_multi_opts *opts);

/* Time every packets-per-lane x placement configuration on these batches
 * (each run really classifies them), remember the fastest for this batch
 * shape (rule and packet counts of every chain) so later calls with tuned
 * options use it, and report it in *best (may be NULL) with its time in
 * *best_ms (may be NULL).  Synchronous. */
fw_status fw_autotune_multi(const fw_chain_batch *batches, uint32_t n_chains, void *stream,
                            fw_multi_opts *best, float *best_ms);

/* ------------------------------------------------------------------ serving
 * Not in the paper (its Section V names asynchronous launches as future
 * work).  A server keeps rulesets resident and classifies packet batches that
 * arrive over time with continuous batching.  Each of `slots` host threads
 * owns a HIP stream; a free slot admits, in arrival order, every queued
 * request that fits its share of the memory budget (up to max_group
 * requests) as one group, and classifies the whole group with one
 * multi-chain launch (one entry per request: the chain's learned index where
 * one is built, else the packet-split scan of its grouped rule list).  Each
 * request's result is the same as classifying it alone. */

typedef struct fw_server fw_server;

typedef struct fw_server_opts {
    uint32_t slots;         /* groups in flight at once, each with its own host thread and HIP
                               stream, 1..16; 0 = 4 (the hardware queues a process gets) */
    uint32_t mode;          /* FW_MODE_AUTO (learned index where built, else the grouped scan),
                               FW_MODE_PACKET_SPLIT (indexes ignored) or FW_MODE_LEARNED (every
                               chain must have an index: FW_E_NOINDEX otherwise) */
    uint32_t max_group;     /* requests coalesced into one launch, 1..1024; 0 = 1024 */
    uint32_t ingest;        /* 0 = copies: a group's requests under 4,096 packets are packed
                               into page-locked staging and moved by one copy per field, the
                               larger ones copied straight from and to their own buffers
                               (any host memory works; page-locked memory copies fastest);
                               1 = mapped: every buffer given to the server is page-locked
                               host memory mapped into the device's address space (from
                               hipHostMalloc, as torch's pinned memory is) and 16-byte aligned;
                               the kernel reads the packets and writes the results in place */
    uint64_t mem_budget;    /* bytes of packets and results in flight (18 per packet, each
                               request rounded up to 16 packets, each array to 256 bytes);
                               with copies it is also the device memory and the page-locked
                               staging the server holds; 0 = 256 MiB */
    uint64_t max_group_packets; /* packets coalesced into one launch (a larger request still
                                   runs, alone); every request of a group completes when the
                                   group does; 0 = 1,048,576 */
} fw_server_opts;

/* A batch of packet headers in HOST memory (structure of arrays): any host
 * memory with copy ingest, page-locked mapped memory with mapped ingest. */
typedef struct fw_host_packets {
    const uint32_t *src_ip;
    const uint32_t *dst_ip;
    const uint16_t *src_port;
    const uint16_t *dst_port;
    const uint8_t *proto;
} fw_host_packets;

/* Timestamps of one request, seconds on a monotonic clock. */
typedef struct fw_request_times {
    double submit, admit, done;
} fw_request_times;

/* Start a server over `n_chains` loaded rulesets (they must outlive it; mode
 * AUTO uses the learned index a chain has when a group is launched).
 * Errors: FW_E_INVAL (no chains, NULL chain, bad options, a mode other than
 * AUTO, PACKET_SPLIT or LEARNED), FW_E_NOINDEX (mode LEARNED and a chain
 * without an index), FW_E_NOMEM, FW_E_DEVICE. */
fw_status fw_server_create(fw_ruleset *const *chains, uint32_t n_chains,
                           const fw_server_opts *opts, fw_server **out);

/* Queue `n` packets (host memory) for chain `chain`; results go to the HOST
 * arrays out_rule_idx / out_action.  All buffers must stay valid until
 * fw_server_wait returns for *ticket.  FW_E_NOMEM if the request alone
 * exceeds the memory budget (it could never be admitted); FW_E_ALIGN with
 * mapped ingest for a buffer that is not 16-byte aligned. */
fw_status fw_server_submit(fw_server *sv, uint32_t chain, const fw_host_packets *pk, size_t n,
                           int32_t *out_rule_idx, uint8_t *out_action, uint64_t *ticket);

/* Block until request `ticket` has completed; `times` may be NULL.  Returns
 * the request's own status (a failed launch is reported here). */
fw_status fw_server_wait(fw_server *sv, uint64_t ticket, fw_request_times *times);

/* Wait for every request, stop the server and free its resources. */
fw_status fw_server_destroy(fw_server *sv);

/* Load generator: replay an arrival trace against a server.  Request k is
 * submitted at t0 + arrival_s[k] (t0 = when the call starts; arrival_s
 * non-decreasing) for chain[k], with packets [offset[k], offset[k] + n[k]) of
 * the HOST pool arrays and results written at the same offsets of out_idx and
 * out_action.  Returns once every request has completed; times[k] (may be
 * NULL) receives the request's scheduled arrival as `submit`, so queueing
 * behind a late generator still counts toward its latency. */
fw_status fw_server_replay(fw_server *sv, uint32_t n_req, const double *arrival_s,
                           const uint32_t *chain, const size_t *offset, const size_t *n,
                           const fw_host_packets *pool, int32_t *out_idx, uint8_t *out_action,
                           fw_request_times *times);

/* Description of the calling thread's most recent error ("" if none). */
const char *fw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FW_H */
