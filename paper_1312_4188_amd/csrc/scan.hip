// First-match scan kernels for gfx950 (CDNA4, wave64).
//
// Paper Section I: rules are tried in insertion order and the first match
// decides; no match means the default action.  Section IV-A (data parallel):
// every node holds the whole policy and each packet goes to exactly one node;
// here a node is a GPU lane.  Section IV-B (function parallel): the policy is
// split into parts, every node sees every packet, and the partial results
// are combined; here the parts are contiguous rule partitions and the
// combination is a minimum over rule indices.  Section IV-C (hybrid): a block
// per packet group, its threads splitting the rules.
//
// Every field test is the unsigned range test (v - lo) <= w (see RuleRec).
#include "device_util.h"
#include "fw_internal.h"
#include "scan_core.h"

namespace fw {
namespace {

constexpr uint32_t kScanBlock = 256;   // threads per work-group of the scan kernels

// ------------------------------------------------------------------ packet split
// The packet-split kernel: each wave classifies 64*K packets against the
// ruleset's grouped scan plan.
template <int K>
__global__ __launch_bounds__(kScanBlock) void k_packet_split(ScanPlan plan, PacketsDev pk, size_t n,
                                                      int32_t* __restrict__ out_idx,
                                                      uint8_t* __restrict__ out_act,
                                                      uint32_t dflt) {
    const size_t wave = size_t(blockIdx.x) * (kScanBlock / 64) + wave_in_group();
    const size_t wave_first = wave * 64u * K;
    if (wave_first >= n) return;  // wave-uniform
    WaveScan<K> w;
    w.init(pk, wave_first, n, dflt);
    w.scan_plan(plan);
    w.store(out_idx, out_act, n);
}

// ------------------------------------------------------------------ rule split
// Minimum over the LP lanes of one packet group, with DPP lane permutations
// (quad swaps, half-row and row mirrors), one swizzle across the two rows of a
// 32-lane half, and a readlane pair across the halves.  Every lane of the
// group receives the minimum.  Must be called with the whole wave active.
template <int LP>
__device__ __forceinline__ uint32_t group_min(uint32_t v) {
    if constexpr (LP >= 2)   // quad_perm [1,0,3,2]
        v = umin(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0xB1, 0xF, 0xF, false)));
    if constexpr (LP >= 4)   // quad_perm [2,3,0,1]
        v = umin(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x4E, 0xF, 0xF, false)));
    if constexpr (LP >= 8)   // row_half_mirror: lane i <-> 7 - i within each half row
        v = umin(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x141, 0xF, 0xF, false)));
    if constexpr (LP >= 16)  // row_mirror: lane i <-> 15 - i within each row
        v = umin(v, uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x140, 0xF, 0xF, false)));
    if constexpr (LP >= 32)  // swizzle, bit mode: lane ^ 16 within each 32-lane half
        v = umin(v, uint32_t(__builtin_amdgcn_ds_swizzle(int(v), 0x401F)));
    if constexpr (LP >= 64) {
        const uint32_t a = __builtin_amdgcn_readlane(int(v), 0);
        const uint32_t b = __builtin_amdgcn_readlane(int(v), 32);
        v = umin(a, b);
    }
    return v;
}

__device__ __forceinline__ bool full_match(const RuleRec& q, uint32_t src, uint32_t dst,
                                           uint32_t pp, uint32_t pr) {
    return in_range(dst, q.dst_lo, q.dst_w) && in_range(src, q.src_lo, q.src_w) &&
           ports_in(pp, q.port_lo, q.port_w) && in_range(pr, proto_lo(q.proto), proto_w(q.proto));
}

// Lane = (packet slot, partition).  LP lanes share one packet; lane `sub` of a
// slot scans partition blk*64 + sub, i.e. rules [part*S, min(R, part*S + S)).
// A lane stops at its partition's first match.  Every kPrune rules the group
// minimum is taken again and lanes whose next rule lies beyond it stop: no
// later find could win.  With more than 64 partitions a packet spans
// `wpp` waves whose minima meet through atomicMin on the 32-bit index.
constexpr int kPrune = 8;

template <int LP>
__global__ __launch_bounds__(kScanBlock) void k_rule_split(const RuleRec* __restrict__ rules,
                                                    uint32_t n_rules, uint32_t P, uint32_t S,
                                                    uint32_t wpp, PacketsDev pk, size_t n,
                                                    int32_t* __restrict__ out_idx,
                                                    uint8_t* __restrict__ out_act,
                                                    uint32_t dflt, int use_atomic) {
    const uint32_t lane = threadIdx.x & 63u;
    const size_t wave = size_t(blockIdx.x) * (kScanBlock / 64) + wave_in_group();
    const size_t group = wave / wpp;
    const uint32_t blk = uint32_t(wave % wpp);
    const uint32_t slot = lane / LP, sub = lane % LP;
    const size_t i = group * (64u / LP) + slot;
    if (group * (64u / LP) >= n) return;  // wave-uniform
    const uint32_t part = blk * 64u + sub;
    const bool valid = i < n && part < P;

    uint32_t src = 0, dst = 0, pp = 0, pr = 0;
    if (i < n) {
        src = pk.src[i];
        dst = pk.dst[i];
        pp = (uint32_t(pk.sport[i]) << 16) | pk.dport[i];
        pr = pk.proto[i];
    }
    const uint64_t r0 = valid ? uint64_t(part) * S : 0;
    const uint32_t begin = uint32_t(r0 < n_rules ? r0 : n_rules);
    const uint32_t end = uint32_t(r0 + S < n_rules ? r0 + S : n_rules);
    uint32_t r = begin;
    bool done = !valid || begin >= end;
    uint32_t best = kNoMatch;

    for (;;) {
#pragma unroll
        for (int t = 0; t < kPrune; ++t) {
            if (!done) {
                if (r >= end) {
                    done = true;
                } else {
                    const RuleRec q = rules[r];
                    if (full_match(q, src, dst, pp, pr)) {
                        best = r;
                        done = true;
                    }
                    ++r;
                }
            }
        }
        const uint32_t gm = group_min<LP>(best);
        if (gm < r) done = true;
        if (ballot(!done) == 0) break;
    }
    const uint32_t gm = group_min<LP>(best);
    if (sub == 0 && i < n) {
        if (use_atomic) {
            atomicMin(reinterpret_cast<uint32_t*>(out_idx) + i, gm);
        } else {
            out_idx[i] = int32_t(gm);
            out_act[i] = uint8_t(gm == kNoMatch ? dflt : rule_action(rules[gm].proto));
        }
    }
}

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Index -> action for the atomicMin path: 0xFFFFFFFF reads as -1 and takes the default.
__global__ void k_apply_action(const RuleRec* __restrict__ rules, const int32_t* idx, size_t n,
                               uint8_t* __restrict__ out_act, uint32_t dflt) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) {
        const uint32_t r = uint32_t(idx[i]);
        out_act[i] = uint8_t(r == kNoMatch ? dflt : rule_action(rules[r].proto));
    }
}

// ------------------------------------------------------------------ hybrid
// One work-group per 64 packets (paper Section IV-C: a block per packet, its
// threads splitting the rules; here a lane per packet and a wave per rule
// partition).  Wave w scans partition w with the packet-split wave scan, in
// chunks of kHybridChunk rules; after each chunk its lanes' first matches go
// into LDS through atomicMin, and lanes that another wave has already beaten
// (an LDS minimum below the next rule index) drop out.
constexpr uint32_t kHybridChunk = 64;

__global__ __launch_bounds__(1024) void k_hybrid(const uint2* __restrict__ pairs,
                                                 const RuleRec* __restrict__ rules,
                                                 uint32_t n_rules, uint32_t S, PacketsDev pk,
                                                 size_t n, int32_t* __restrict__ out_idx,
                                                 uint8_t* __restrict__ out_act, uint32_t dflt) {
    __shared__ uint32_t smin[64];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t w = wave_in_group();
    const size_t first = size_t(blockIdx.x) * 64u;
    if (w == 0) smin[lane] = kNoMatch;
    __syncthreads();

    WaveScan<1> ws;
    ws.init(pk, first, n, dflt);
    const uint64_t r0 = uint64_t(w) * S;
    const uint32_t begin = uint32_t(r0 < n_rules ? r0 : n_rules);
    const uint32_t end = uint32_t(r0 + S < n_rules ? r0 + S : n_rules);
    for (uint32_t c = begin; c < end && ws.any_live(); c += kHybridChunk) {
        const uint32_t cnt = min(kHybridChunk, end - c);
        ws.template scan<FirstField::Dst>(pairs + c, rules + c, cnt, c);
        if (ws.best[0] != kNoMatch) atomicMin(&smin[lane], ws.best[0]);
        const uint32_t cur = *reinterpret_cast<volatile uint32_t*>(&smin[lane]);
        ws.live[0] &= ballot(cur > c + cnt);
        ws.live_any = ws.live[0];
    }
    __syncthreads();
    const size_t i = first + lane;
    if (w == 0 && i < n) {
        const uint32_t b = smin[lane];
        out_idx[i] = int32_t(b);
        out_act[i] = uint8_t(b == kNoMatch ? dflt : rule_action(rules[b].proto));
    }
}

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return uint32_t((a + b - 1) / b); }

}  // namespace

hipError_t launch_packet_split(const ScanPlan& plan, PacketsDev pk, size_t n, int32_t* out_idx,
                               uint8_t* out_act, uint8_t default_action, int packets_per_lane,
                               hipStream_t stream) {
    if (n == 0) return hipSuccess;
    constexpr uint32_t kBlock = kScanBlock;
    const int K = packets_per_lane;
    const uint64_t per_block = uint64_t(kBlock) * K;
    const uint32_t grid = ceil_div(n, per_block);
    const uint32_t dflt = default_action;
    if (K == 4)
        hipLaunchKernelGGL(k_packet_split<4>, dim3(grid), dim3(kBlock), 0, stream, plan, pk, n,
                           out_idx, out_act, dflt);
    else if (K == 2)
        hipLaunchKernelGGL(k_packet_split<2>, dim3(grid), dim3(kBlock), 0, stream, plan, pk, n,
                           out_idx, out_act, dflt);
    else
        hipLaunchKernelGGL(k_packet_split<1>, dim3(grid), dim3(kBlock), 0, stream, plan, pk, n,
                           out_idx, out_act, dflt);
    return hipGetLastError();
}

hipError_t launch_rule_split(const RuleRec* rules, uint32_t n_rules, uint32_t P, PacketsDev pk,
                             size_t n, int32_t* out_idx, uint8_t* out_act,
                             uint8_t default_action, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    constexpr uint32_t kBlock = kScanBlock;
    const uint32_t S = n_rules == 0 ? 1u : ceil_div(n_rules, P);
    uint32_t LP = 1;
    while (LP < P && LP < 64) LP <<= 1;
    const uint32_t wpp = P > 64 ? ceil_div(P, 64) : 1u;
    const uint64_t groups = (n + (64 / LP) - 1) / (64 / LP);
    const uint64_t waves = groups * wpp;
    const uint32_t grid = ceil_div(waves * 64, kBlock);
    const int atomic = wpp > 1;
    if (atomic) {
        hipLaunchKernelGGL(k_fill_u32, dim3(ceil_div(n, 256)), dim3(256), 0, stream,
                           reinterpret_cast<uint32_t*>(out_idx), n, kNoMatch);
    }
#define FW_RS(L)                                                                          \
    hipLaunchKernelGGL(k_rule_split<L>, dim3(grid), dim3(kBlock), 0, stream, rules, n_rules, \
                       P, S, wpp, pk, n, out_idx, out_act, uint32_t(default_action), atomic)
    switch (LP) {
        case 1: FW_RS(1); break;
        case 2: FW_RS(2); break;
        case 4: FW_RS(4); break;
        case 8: FW_RS(8); break;
        case 16: FW_RS(16); break;
        case 32: FW_RS(32); break;
        default: FW_RS(64); break;
    }
#undef FW_RS
    if (atomic) {
        hipLaunchKernelGGL(k_apply_action, dim3(ceil_div(n, 256)), dim3(256), 0, stream, rules,
                           out_idx, n, out_act, uint32_t(default_action));
    }
    return hipGetLastError();
}

hipError_t launch_hybrid(const uint2* pairs, const RuleRec* rules, uint32_t n_rules, uint32_t P,
                         PacketsDev pk,
                         size_t n, int32_t* out_idx, uint8_t* out_act, uint8_t default_action,
                         hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t S = n_rules == 0 ? 1u : ceil_div(n_rules, P);
    hipLaunchKernelGGL(k_hybrid, dim3(ceil_div(n, 64)), dim3(64 * P), 0, stream, pairs, rules,
                       n_rules, S, pk, n, out_idx, out_act, uint32_t(default_action));
    return hipGetLastError();
}

}  // namespace fw
