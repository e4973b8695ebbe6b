// Internal declarations shared by the library's host and device sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "host_types.h"

namespace fw {

// A rule list cut at its first catch-all and split into up to four groups by
// the field each rule is tested on first (the most selective one): the
// destination prefix, the source prefix, the port pair, or the protocol.
// Each group keeps rule order and holds, per rule, the first test's (lo, w)
// pair (padded by kPairPadding) and the full record (whose idx field is the
// rule's position in the original list).  Rules after the first catch-all can
// never be a first match and are dropped; the catch-all itself becomes the
// `tail`, the answer for packets no earlier rule matches.

struct ScanGroup {
    const uint2* pairs;
    const RuleRec* recs;
    uint32_t count;
    uint32_t kind;   // FirstTest
};

struct ScanPlan {
    ScanGroup g[4];
    uint32_t n_groups;
    uint32_t tail_idx;   // kNoMatch when the list has no catch-all
    uint32_t tail_act;
    uint32_t pad;
};

// Device memory of one plan (plan.cpp).
struct DevicePlan {
    void* mem = nullptr;
    ScanPlan plan{};
    uint64_t bytes = 0;
};
// Build and upload the plan of `n` records (each carrying its own idx), in order.
hipError_t make_plan(const RuleRec* recs, uint32_t n, DevicePlan* out);
void free_plan(DevicePlan* p);

struct PacketsDev {
    const uint32_t* src;
    const uint32_t* dst;
    const uint16_t* sport;
    const uint16_t* dport;
    const uint8_t* proto;
};

// ---- scan launchers (scan.hip); all asynchronous on `stream`
hipError_t launch_packet_split(const ScanPlan& plan, PacketsDev pk, size_t n, int32_t* out_idx,
                               uint8_t* out_act, uint8_t default_action, int packets_per_lane,
                               hipStream_t stream);
hipError_t launch_rule_split(const RuleRec* rules, uint32_t n_rules, uint32_t partitions,
                             PacketsDev pk, size_t n, int32_t* out_idx, uint8_t* out_act,
                             uint8_t default_action, hipStream_t stream);
hipError_t launch_hybrid(const uint2* pairs, const RuleRec* rules, uint32_t n_rules,
                         uint32_t partitions,
                         PacketsDev pk, size_t n, int32_t* out_idx, uint8_t* out_act,
                         uint8_t default_action, int packets_per_lane, hipStream_t stream);

}  // namespace fw
