// C interface: argument checks, ruleset compilation and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <chrono>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fw.h"
#include "fw_internal.h"
#include "index.h"
#include "guard.h"

struct fw_ruleset {
    uint32_t n_rules = 0;
    uint8_t default_action = FW_DROP;
    int device = 0;
    fw::RuleRec* d_rules = nullptr;          // n_rules records (at least one allocated)
    uint2* d_pairs = nullptr;                // (dst_lo, dst_w) per rule, + kPairPadding
    fw::DevicePlan plan;                     // grouped scan plan (packet split)
    std::vector<fw::RuleRec> h_rules;        // host copy of the compiled records
    std::vector<fw_rule> source;             // the rules as given
    fw::LearnedIndex* index = nullptr;       // null until built
    fw::ChainView h_view{};                  // what the multi-chain kernels read ...
    fw::ChainView* d_view = nullptr;         // ... and its device copy
};

namespace fw {

thread_local std::string g_last_error;  // read by fw_last_error()

fw_status fail(fw_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

fw_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? FW_E_NOMEM : FW_E_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

// Prefix (base, len) -> [lo, lo + w]: the top `len` bits of the base, all low bits free.
static inline void prefix_to_range(uint32_t base, uint32_t len, uint32_t* lo, uint32_t* w) {
    const uint32_t mask = len == 0 ? 0u : (0xFFFFFFFFu << (32u - len));
    *lo = base & mask;
    *w = ~mask;
}

RuleRec compile_rule(const fw_rule& r, uint32_t idx) {
    RuleRec q{};
    prefix_to_range(r.src_ip, r.src_plen, &q.src_lo, &q.src_w);
    prefix_to_range(r.dst_ip, r.dst_plen, &q.dst_lo, &q.dst_w);
    q.port_lo = (uint32_t(r.sport_lo) << 16) | r.dport_lo;
    q.port_w = (uint32_t(r.sport_hi - r.sport_lo) << 16) | uint32_t(r.dport_hi - r.dport_lo);
    const uint32_t plo = r.proto_any ? 0u : r.proto;
    const uint32_t pw = r.proto_any ? 255u : 0u;
    q.proto = plo | (pw << 8) | (uint32_t(r.action & 1u) << 16);
    q.idx = idx;
    return q;
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

static fw_status check_classify_args(const fw_ruleset* rs, const fw_packets* pk, size_t n,
                                     int32_t* out_idx, uint8_t* out_act) {
    if (!rs) return fail(FW_E_INVAL, "ruleset is NULL");
    if (n == 0) return FW_OK;
    if (!pk) return fail(FW_E_INVAL, "packets is NULL");
    if (!pk->src_ip || !pk->dst_ip || !pk->src_port || !pk->dst_port || !pk->proto)
        return fail(FW_E_INVAL, "a packet field pointer is NULL");
    if (!out_idx || !out_act) return fail(FW_E_INVAL, "an output pointer is NULL");
    if (!aligned16(pk->src_ip) || !aligned16(pk->dst_ip) || !aligned16(pk->src_port) ||
        !aligned16(pk->dst_port) || !aligned16(pk->proto))
        return fail(FW_E_ALIGN, "packet arrays must be 16-byte aligned");
    if (!aligned16(out_idx) || !aligned16(out_act))
        return fail(FW_E_ALIGN, "output arrays must be 16-byte aligned");
    if (n > (size_t(1) << 40)) return fail(FW_E_INVAL, "n too large");
    return FW_OK;
}

PacketsDev to_dev(const fw_packets* pk) {
    return PacketsDev{pk->src_ip, pk->dst_ip, pk->src_port, pk->dst_port, pk->proto};
}

const ChainView* ruleset_chain_view(const fw_ruleset* rs, const ChainView** host) {
    if (host) *host = &rs->h_view;
    return rs->d_view;
}

// Write the ruleset's ChainView to its device copy.  Callers make sure no
// kernel is reading it (at load nothing can; an index build waits for the
// device first).
static hipError_t upload_view(fw_ruleset* rs) {
    return hipMemcpy(rs->d_view, &rs->h_view, sizeof(ChainView), hipMemcpyHostToDevice);
}

// Packets per lane when the caller leaves it to the library: the most (up to
// `most`) that still gives the launch 8,192 waves (8 per SIMD on 256 CUs), so
// small batches spread over more waves and each wave's scan is shorter.
static uint32_t default_packets_per_lane(size_t n, uint32_t most) {
    uint32_t k = most;
    while (k > 1 && n < size_t(8192) * 64u * k) k /= 2;
    return k;
}

// Hybrid default: one packet per lane while the batch's waves (P per 64
// packets) fit the GPU at once, about 8,192 of them; four above that, where
// fewer, longer waves finish sooner (measured at 10,000 and 1,000 rules: at
// 65,536 packets and 16 partitions four per lane take 52 us against 61 us for
// one, at 16,384 packets one takes 29 us against 51 us).
static uint32_t hybrid_packets_per_lane(size_t n, uint32_t partitions) {
    return double(n) * partitions / 64.0 <= 8192.0 ? 1u : 4u;
}

// Mode AUTO without a learned index, by batch size (closed-loop latencies
// measured on one MI355X, 64 to 1,048,576 packets at 1,000 and 10,000 rules):
// packet split from 262,144 packets, where the batch fills the GPU and its
// total work is the least; below that the split forms, whose waves share the
// rule list, so a packet waits for a fraction of the reachable rules instead
// of all of them: rule split over 64 partitions for batches up to 4,096
// packets when at least 2,048 rules are reachable (20-28 us at 10,000 rules
// against 28-29 us for the hybrid and 88-89 us for packet split), the hybrid
// over 16 partitions otherwise (at 65,536 packets 52 us against 90 us).
struct AutoChoice {
    uint32_t mode, partitions;
};
constexpr size_t kAutoScanFrom = 262144;
constexpr size_t kAutoRuleSplitUpTo = 4096;
constexpr uint32_t kAutoRuleSplitRules = 2048;
static AutoChoice auto_scan_mode(size_t n, uint32_t reachable) {
    if (n >= kAutoScanFrom) return {FW_MODE_PACKET_SPLIT, 0u};
    if (n <= kAutoRuleSplitUpTo && reachable >= kAutoRuleSplitRules)
        return {FW_MODE_RULE_SPLIT, 64u};
    return {FW_MODE_HYBRID, 16u};
}

// A device fault in earlier asynchronous work is sticky; report it before new work.
static fw_status check_device_state() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "earlier device work failed");
    return FW_OK;
}

}  // namespace fw

using namespace fw;

extern "C" {

fw_status fw_load_ruleset(const fw_rule* rules, uint32_t n_rules, uint8_t default_action,
                          fw_ruleset** out) {
    return guarded([&]() -> fw_status {
        if (!out) return fail(FW_E_INVAL, "out is NULL");
        *out = nullptr;
        if (n_rules > 0 && !rules) return fail(FW_E_INVAL, "rules is NULL");
        if (n_rules > kMaxRules) return fail(FW_E_INVAL, "at most %u rules", kMaxRules);
        if (default_action > 1) return fail(FW_E_INVAL, "default_action must be 0 or 1");
        for (uint32_t i = 0; i < n_rules; ++i) {
            const fw_rule& r = rules[i];
            if (r.src_plen > 32 || r.dst_plen > 32)
                return fail(FW_E_INVAL, "rule %u: prefix length above 32", i);
            if (r.sport_lo > r.sport_hi || r.dport_lo > r.dport_hi)
                return fail(FW_E_INVAL, "rule %u: port range with lo > hi", i);
            if (r.action > 1) return fail(FW_E_INVAL, "rule %u: action must be 0 or 1", i);
        }
        fw_ruleset* rs = new fw_ruleset();
        ScopeExit undo([rs] {   // a failed or throwing step below frees what was made
            if (rs->d_view) (void)hipFree(rs->d_view);
            if (rs->d_rules) (void)hipFree(rs->d_rules);
            if (rs->d_pairs) (void)hipFree(rs->d_pairs);
            free_plan(&rs->plan);
            delete rs;
        });
        rs->source.assign(rules, rules + n_rules);
        rs->h_rules.resize(n_rules);
        for (uint32_t i = 0; i < n_rules; ++i) rs->h_rules[i] = compile_rule(rules[i], i);
        rs->n_rules = n_rules;
        rs->default_action = default_action;
        std::vector<uint2> pairs(size_t(n_rules) + kPairPadding, uint2{0u, 0u});
        for (uint32_t i = 0; i < n_rules; ++i)
            pairs[i] = uint2{rs->h_rules[i].dst_lo, rs->h_rules[i].dst_w};
        hipError_t e = hipGetDevice(&rs->device);
        if (e == hipSuccess)
            e = hipMalloc(&rs->d_rules, sizeof(RuleRec) * (n_rules ? n_rules : 1));
        if (e == hipSuccess) e = hipMalloc(&rs->d_pairs, sizeof(uint2) * pairs.size());
        if (e == hipSuccess && n_rules)
            e = hipMemcpy(rs->d_rules, rs->h_rules.data(), sizeof(RuleRec) * n_rules,
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(rs->d_pairs, pairs.data(), sizeof(uint2) * pairs.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess) e = make_plan(rs->h_rules.data(), n_rules, &rs->plan);
        if (e == hipSuccess) {
            ChainView& v = rs->h_view;
            v.rules = rs->d_rules;
            v.pairs = rs->d_pairs;
            v.n_rules = n_rules;
            v.dflt = default_action;
            v.plan = rs->plan.plan;
            e = hipMalloc(&rs->d_view, sizeof(ChainView));
        }
        if (e == hipSuccess) e = upload_view(rs);
        if (e != hipSuccess) return hip_fail(e, "uploading the ruleset");
        undo.dismiss();
        *out = rs;
        return FW_OK;
    });
}

fw_status fw_free_ruleset(fw_ruleset* rs) {
    return guarded([&]() -> fw_status {
        if (!rs) return FW_OK;
        hipError_t e = hipDeviceSynchronize();
        destroy_index(rs->index);
        rs->index = nullptr;
        free_plan(&rs->plan);
        for (void* p : {static_cast<void*>(rs->d_rules), static_cast<void*>(rs->d_pairs),
                        static_cast<void*>(rs->d_view)}) {
            if (!p) continue;
            const hipError_t e2 = hipFree(p);
            if (e == hipSuccess) e = e2;
        }
        delete rs;
        if (e != hipSuccess) return hip_fail(e, "freeing the ruleset");
        return FW_OK;
    });
}

uint32_t fw_ruleset_size(const fw_ruleset* rs) { return rs ? rs->n_rules : 0u; }

fw_status fw_classify_ex(const fw_ruleset* rs, const fw_packets* pk, size_t n,
                         int32_t* out_rule_idx, uint8_t* out_action,
                         const fw_classify_opts* opts) {
    return guarded([&]() -> fw_status {
        fw_classify_opts o{};
        if (opts) o = *opts;
        fw_status st = check_classify_args(rs, pk, n, out_rule_idx, out_action);
        if (st != FW_OK) return st;
        if (o.mode > FW_MODE_HYBRID) return fail(FW_E_INVAL, "unknown mode %u", o.mode);
        if (o.packets_per_lane != 0 && o.packets_per_lane != 1 && o.packets_per_lane != 2 &&
            o.packets_per_lane != 4)
            return fail(FW_E_INVAL, "packets_per_lane must be 0, 1, 2 or 4");
        uint32_t P = o.partitions ? o.partitions : 16u;
        if (P > kMaxPartitions) return fail(FW_E_INVAL, "at most %u partitions", kMaxPartitions);
        if (o.mode == FW_MODE_HYBRID && P > 16)
            return fail(FW_E_INVAL, "hybrid mode takes 1..16 partitions (one wave each)");
        if (o.mode == FW_MODE_LEARNED && !rs->index)
            return fail(FW_E_NOINDEX, "no learned index: call fw_build_learned_index first");
        if (n == 0) {
            if (o.window_misses) *o.window_misses = 0;
            return FW_OK;
        }
        st = check_device_state();
        if (st != FW_OK) return st;
        hipStream_t stream = static_cast<hipStream_t>(o.stream);
        const PacketsDev pd = to_dev(pk);
        uint32_t mode = o.mode;
        // the split forms partition the rules up to and including the first catch-all: later
        // rules can never be a first match
        const uint32_t reachable =
            rs->plan.plan.tail_idx == kNoMatch ? rs->n_rules : rs->plan.plan.tail_idx + 1u;
        if (mode == FW_MODE_AUTO) {
            if (rs->index) {
                mode = FW_MODE_LEARNED;
            } else {
                const AutoChoice c = auto_scan_mode(n, reachable);
                mode = c.mode;
                if (c.partitions) P = c.partitions;
            }
        }
        hipError_t e = hipSuccess;
        switch (mode) {
            case FW_MODE_PACKET_SPLIT:
                e = launch_packet_split(rs->plan.plan, pd, n, out_rule_idx, out_action,
                                        rs->default_action,
                                        o.packets_per_lane ? int(o.packets_per_lane)
                                                           : int(default_packets_per_lane(n, 4)),
                                        stream);
                break;
            case FW_MODE_RULE_SPLIT:
                e = launch_rule_split(rs->d_rules, reachable, P, pd, n, out_rule_idx, out_action,
                                      rs->default_action, stream);
                break;
            case FW_MODE_HYBRID:
                e = launch_hybrid(rs->d_pairs, rs->d_rules, reachable, P, pd, n, out_rule_idx,
                                  out_action, rs->default_action,
                                  o.packets_per_lane ? int(o.packets_per_lane)
                                                     : int(hybrid_packets_per_lane(n, P)),
                                  stream);
                break;
            case FW_MODE_LEARNED:
                return classify_learned(rs->index, rs->default_action, pd, n, out_rule_idx,
                                        out_action, o.lookup,
                                        o.packets_per_lane ? o.packets_per_lane
                                                           : default_packets_per_lane(n, 2),
                                        stream, o.window_misses);
            default:
                return fail(FW_E_INVAL, "unknown mode %u", mode);
        }
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        if (o.window_misses) *o.window_misses = 0;
        return FW_OK;
    });
}

fw_status fw_classify(const fw_ruleset* rs, const fw_packets* pk, size_t n,
                      int32_t* out_rule_idx, uint8_t* out_action) {
    return guarded([&]() -> fw_status {
        return fw_classify_ex(rs, pk, n, out_rule_idx, out_action, nullptr);
    });
}

fw_status fw_closed_loop(const fw_ruleset* rs, const fw_packets* pk, uint32_t n_batches,
                         const size_t* start, const size_t* count, int32_t* out_rule_idx,
                         uint8_t* out_action, const fw_classify_opts* opts, double* seconds) {
    return guarded([&]() -> fw_status {
        if (!rs || !pk) return fail(FW_E_INVAL, "ruleset or packets is NULL");
        if (n_batches == 0) return FW_OK;
        if (!start || !count || !seconds) return fail(FW_E_INVAL, "NULL argument");
        // checked here, before the slices are offset (an offset NULL is not NULL)
        if (!pk->src_ip || !pk->dst_ip || !pk->src_port || !pk->dst_port || !pk->proto)
            return fail(FW_E_INVAL, "a packet field pointer is NULL");
        fw_classify_opts o{};
        if (opts) o = *opts;
        hipStream_t stream = static_cast<hipStream_t>(o.stream);
        for (uint32_t k = 0; k < n_batches; ++k) {
            if (start[k] % 16u)
                return fail(FW_E_ALIGN, "batch %u starts at %zu, not a multiple of 16", k,
                            start[k]);
            const size_t s0 = start[k];
            const fw_packets sub{pk->src_ip + s0, pk->dst_ip + s0, pk->src_port + s0,
                                 pk->dst_port + s0, pk->proto + s0};
            const auto t0 = std::chrono::steady_clock::now();
            const fw_status st = fw_classify_ex(rs, &sub, count[k], out_rule_idx, out_action, &o);
            if (st != FW_OK) return st;
            const hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "closed-loop batch");
            seconds[k] =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        return FW_OK;
    });
}

fw_status fw_build_learned_index(fw_ruleset* rs, const fw_index_opts* opts,
                                 fw_index_stats* stats) {
    return guarded([&]() -> fw_status {
        if (!rs) return fail(FW_E_INVAL, "ruleset is NULL");
        fw_index_opts o{};
        if (opts) o = *opts;
        LearnedIndex* built = nullptr;
        const fw_status st = build_index(rs->source.data(), rs->h_rules.data(), rs->n_rules, o,
                                         stats, &built);
        if (st != FW_OK) return st;
        // classifications enqueued earlier may still read the old index or the ruleset's view
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            destroy_index(built);
            return hip_fail(e, "waiting for work on the previous index");
        }
        ChainView v = rs->h_view;
        index_chain_view(built, &v);
        const ChainView old_view = rs->h_view;
        rs->h_view = v;
        e = upload_view(rs);
        if (e != hipSuccess) {
            rs->h_view = old_view;
            (void)upload_view(rs);
            destroy_index(built);
            return hip_fail(e, "publishing the learned index");
        }
        if (rs->index) destroy_index(rs->index);
        rs->index = built;
        return FW_OK;
    });
}

fw_status fw_index_lookup(const fw_ruleset* rs, const uint32_t* keys, size_t n,
                          int32_t* out_interval, uint32_t lookup, void* stream) {
    return guarded([&]() -> fw_status {
        if (!rs) return fail(FW_E_INVAL, "ruleset is NULL");
        if (!rs->index) return fail(FW_E_NOINDEX, "no learned index");
        if (n == 0) return FW_OK;
        if (!keys || !out_interval) return fail(FW_E_INVAL, "NULL buffer");
        if (!aligned16(keys) || !aligned16(out_interval))
            return fail(FW_E_ALIGN, "buffers must be 16-byte aligned");
        if (lookup > 1) return fail(FW_E_INVAL, "lookup must be 0 or 1");
        const fw_status st = check_device_state();
        if (st != FW_OK) return st;
        return index_lookup(rs->index, keys, n, out_interval, lookup,
                            static_cast<hipStream_t>(stream));
    });
}

fw_status fw_index_export(const fw_ruleset* rs, uint32_t what, void* host, size_t cap,
                          size_t* size) {
    return guarded([&]() -> fw_status {
        if (!rs) return fail(FW_E_INVAL, "ruleset is NULL");
        if (!rs->index) return fail(FW_E_NOINDEX, "no learned index");
        return index_export(rs->index, what, host, cap, size);
    });
}

const char* fw_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
