// Device-side helpers shared by the scan and learned-index kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fw_internal.h"

namespace fw {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Index of the calling wave within its work-group, as a wave-uniform (scalar) value.
__device__ __forceinline__ uint32_t wave_in_group() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Unsigned range test: v lies in [lo, lo + w].
__device__ __forceinline__ bool in_range(uint32_t v, uint32_t lo, uint32_t w) {
    return (v - lo) <= w;
}

// Both ports at once: packed 16-bit subtract, packed 16-bit max, one compare.
// max(v - lo, w) == w holds in both halves exactly when both differences are <= w.
__device__ __forceinline__ bool ports_in(uint32_t pp, uint32_t lo, uint32_t w) {
    u16x2 d = __builtin_bit_cast(u16x2, pp) - __builtin_bit_cast(u16x2, lo);
    u16x2 m = __builtin_elementwise_max(d, __builtin_bit_cast(u16x2, w));
    return __builtin_bit_cast(uint32_t, m) == w;
}

__device__ __forceinline__ uint32_t proto_lo(uint32_t p) { return p & 0xFFu; }
__device__ __forceinline__ uint32_t proto_w(uint32_t p) { return (p >> 8) & 0xFFu; }
__device__ __forceinline__ uint32_t rule_action(uint32_t p) { return (p >> 16) & 1u; }

// Source, port and protocol tests (the destination test is implied by a candidate list).
__device__ __forceinline__ bool match_no_dst(const RuleRec& q, uint32_t src, uint32_t pp,
                                             uint32_t pr) {
    return in_range(src, q.src_lo, q.src_w) && ports_in(pp, q.port_lo, q.port_w) &&
           in_range(pr, proto_lo(q.proto), proto_w(q.proto));
}

}  // namespace fw
