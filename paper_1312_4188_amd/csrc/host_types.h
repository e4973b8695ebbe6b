// Plain data types shared by the library's host and device sources, with no
// HIP dependency (the host-only list construction compiles without it).
#pragma once

#include <cstdint>

namespace fw {

// Extra first-test pairs allocated past the end of every pair array, so a
// scan can fetch the block after the last one without a bounds test.
constexpr uint32_t kPairPadding = 8;

// A compiled rule as the kernels read it: 32 bytes, every field a range test
// (v - lo) <= w in unsigned arithmetic, so a prefix (base, len) becomes
// lo = base with the low 32-len bits cleared and w = 2^(32-len) - 1.
//   port_lo = sport_lo << 16 | dport_lo,  port_w = sport_w << 16 | dport_w
//   proto   = proto_lo | proto_w << 8 | action << 16   (any protocol: lo 0, w 255)
//   idx     = the rule's position in the original list
struct alignas(32) RuleRec {
    uint32_t src_lo, src_w;
    uint32_t dst_lo, dst_w;
    uint32_t port_lo, port_w;
    uint32_t proto;
    uint32_t idx;
};
static_assert(sizeof(RuleRec) == 32, "rule record must stay 32 bytes");

constexpr uint32_t kNoMatch = 0xFFFFFFFFu;
constexpr uint32_t kMaxRules = 1u << 24;
constexpr uint32_t kMaxPartitions = 65536;

// The field a rule is tested on first in a grouped scan plan (see ScanPlan).
enum FirstTest : uint32_t { kFirstDst = 0, kFirstSrc = 1, kFirstPorts = 2, kFirstProto = 3 };

// Port/protocol table of the first (up to 64) candidates that leave both
// addresses unspecified: such a rule matches a packet exactly when both of
// its port ranges and its protocol test pass.  Per port field, the rules'
// range ends cut [0, 65535] into elementary intervals (each range is a union
// of whole intervals) and interval i carries the 64-bit mask of the rules
// whose range contains it; the protocol gets a mask per value.  The AND of
// the packet's three masks is the set of these rules it matches, and the
// lowest set bit is the first of them (bits follow rule order).  A port's
// interval is found from a 256-entry table on its high byte plus at most
// `steps` forward steps.  Fixed size, so it is staged into LDS as one block.
constexpr uint32_t kPtRules = 64;
constexpr uint32_t kPtMaxIv = 2 * kPtRules + 2;       // intervals per port field, rounded up
struct alignas(16) PortTable {
    uint64_t mask_p[256];           // per protocol value
    uint64_t mask_s[kPtMaxIv];      // per source-port interval
    uint64_t mask_d[kPtMaxIv];      // per destination-port interval
    uint32_t b_s[kPtMaxIv + 2];     // interval starts; unused entries (and one past the last) 0x10000
    uint32_t b_d[kPtMaxIv + 2];
    uint32_t rule[kPtRules + 4];    // bit r -> rule index | action << 24; entry kPtRules = none
    uint8_t bucket_s[256];          // interval holding port h << 8
    uint8_t bucket_d[256];
};
static_assert(sizeof(PortTable) % 16 == 0, "staged as 16-byte words");
constexpr uint32_t kPtNone = 0xFFFFFFFFu;

}  // namespace fw
