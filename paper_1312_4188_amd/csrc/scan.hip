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
// The lanes whose rule matches a packet, as a wave mask: one ballot per field
// test (each compare already yields a lane mask), ANDed in scalar registers,
// so the vector work is the tests alone.
__device__ __forceinline__ uint64_t full_match_mask(const RuleRec& q, uint32_t src, uint32_t dst,
                                                    uint32_t pp, uint32_t pr) {
    return ballot(in_range(dst, q.dst_lo, q.dst_w)) & ballot(in_range(src, q.src_lo, q.src_w)) &
           ballot(ports_in(pp, q.port_lo, q.port_w)) &
           ballot(in_range(pr, proto_lo(q.proto), proto_w(q.proto)));
}

// Function-parallel scan (paper Section IV-B): every firewall node holds a
// part of the policy and sees every packet.  A node here is a wave holding
// partition p, the rules [p*S, min(R, (p+1)*S)); its 64 lanes take 64 of them
// at a time into registers, and G packets at a time are broadcast to
// all lanes through scalar registers, so each vector test checks one packet
// against 64 rules.  A packet is finished in this partition at the first
// 64-rule chunk where any lane matches; the rules sit in lane order, so the
// lowest lane of the match ballot is the partition's first match (a
// wave-uniform value, no per-lane bookkeeping), and the partitions meet
// through atomicMin on the 32-bit index (0xFFFFFFFF = none).
// Waves are numbered partition-major (all packet groups of partition 0, then
// of partition 1, ...), so on a large batch a wave of partition p starts after
// the lower partitions of its packets have finished.  It reads their merged
// index first and skips every packet already matched below its own first rule
// (the pruning across partitions): the index only decreases, so any value
// read bounds the final one from above, and a packet whose value lies below
// the partition start cannot take a rule of it.
// Packets per wave, G: their fields sit in scalar registers (four each), so
// G = 16 uses about 100 of them; the done mask is a 32-bit word.  Large
// batches take 16 (half the waves, and with the pruning most of them end at
// once); smaller ones 8, so that a small batch still spreads over many waves.
constexpr uint32_t kRsLargeBatch = 2097152;

template <uint32_t G>
__global__ __launch_bounds__(kScanBlock) void k_rule_split(const RuleRec* __restrict__ rules,
                                                          uint32_t n_rules, uint32_t P,
                                                          uint32_t S, PacketsDev pk, size_t n,
                                                          uint32_t* __restrict__ idx) {
    static_assert(G < 32, "packet masks are 32-bit words");
    const uint32_t lane = threadIdx.x & 63u;
    const size_t wave = size_t(blockIdx.x) * (kScanBlock / 64) + wave_in_group();
    const size_t groups = (n + G - 1) / G;
    const size_t part_sz = wave / groups;
    if (part_sz >= P) return;  // wave-uniform: past the last partition
    const uint32_t part = uint32_t(part_sz);
    const size_t p0 = (wave % groups) * G;
    const uint64_t b64 = uint64_t(part) * S;
    const uint32_t begin = uint32_t(b64 < n_rules ? b64 : n_rules);
    const uint32_t end = uint32_t(b64 + S < n_rules ? b64 + S : n_rules);
    if (begin >= end) return;  // empty partition

    // the packets, one per lane, then broadcast one at a time; with them the
    // index merged so far (a device-scope load, past the compute unit's cache)
    const size_t mine = p0 + (lane < G ? lane : 0u);
    const bool have = lane < G && mine < n;
    const uint32_t v_src = have ? pk.src[mine] : 0u, v_dst = have ? pk.dst[mine] : 0u;
    const uint32_t v_pp = have ? ((uint32_t(pk.sport[mine]) << 16) | pk.dport[mine]) : 0u;
    const uint32_t v_pr = have ? uint32_t(pk.proto[mine]) : 0u;
    const uint32_t v_cur = have ? __hip_atomic_load(idx + mine, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT)
                                : 0u;
    uint32_t src[G], dst[G], pp[G], pr[G];
    // done: packets past the batch end, and packets already matched below begin
    uint32_t done = uint32_t(ballot(!have || v_cur < begin)) & ((1u << G) - 1u);
#pragma unroll
    for (uint32_t g = 0; g < G; ++g) {
        src[g] = __builtin_amdgcn_readlane(int(v_src), int(g));
        dst[g] = __builtin_amdgcn_readlane(int(v_dst), int(g));
        pp[g] = __builtin_amdgcn_readlane(int(v_pp), int(g));
        pr[g] = __builtin_amdgcn_readlane(int(v_pr), int(g));
    }
    const uint32_t all = (1u << G) - 1u;
    uint32_t first[G];   // wave-uniform: this partition's first match per packet
#pragma unroll
    for (uint32_t g = 0; g < G; ++g) first[g] = kNoMatch;

    for (uint32_t k = begin; k < end && done != all; k += 64u) {
        const uint32_t r = k + lane;
        const bool ok = r < end;
        const RuleRec q = rules[ok ? r : begin];
        const uint64_t in_part = ballot(ok);
#pragma unroll
        for (uint32_t g = 0; g < G; ++g) {
            if ((done >> g) & 1u) continue;  // wave-uniform
            const uint64_t mb = full_match_mask(q, src[g], dst[g], pp[g], pr[g]) & in_part;
            if (mb != 0) {                   // at most one chunk per packet matches
                first[g] = k + uint32_t(__builtin_ctzll(mb));
                done |= 1u << g;
            }
        }
    }
    if (lane == 0) {
#pragma unroll
        for (uint32_t g = 0; g < G; ++g)
            if (first[g] != kNoMatch) atomicMin(idx + p0 + g, first[g]);
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
// One work-group per 64 K packets (paper Section IV-C: a block per packet, its
// threads splitting the rules; here K packets per lane and a wave per rule
// partition).  Wave w scans partition w with the packet-split wave scan, in
// chunks of kHybridChunk rules; after each chunk its lanes' first matches go
// into LDS through atomicMin, and packets that another wave has already beaten
// (an LDS minimum below the next rule index) drop out.
constexpr uint32_t kHybridChunk = 64;

template <int K>
__global__ __launch_bounds__(1024) void k_hybrid(const uint2* __restrict__ pairs,
                                                 const RuleRec* __restrict__ rules,
                                                 uint32_t n_rules, uint32_t S, PacketsDev pk,
                                                 size_t n, int32_t* __restrict__ out_idx,
                                                 uint8_t* __restrict__ out_act, uint32_t dflt) {
    __shared__ uint32_t smin[64 * K];   // packet first + K * lane + s at K * lane + s
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t w = wave_in_group();
    const size_t first = size_t(blockIdx.x) * 64u * K;
    if (w == 0) {
#pragma unroll
        for (int s = 0; s < K; ++s) smin[K * lane + s] = kNoMatch;
    }
    __syncthreads();

    // The per-rule form even with one packet per lane: taking a block's eight
    // first tests before one branch measured no faster here (the chunk merge
    // dominates), and its scalar registers would cost the launch its second
    // work-group per CU at four per lane.
    WaveScan<K, false> ws;
    ws.init(pk, first, n, dflt);
    const uint64_t r0 = uint64_t(w) * S;
    const uint32_t begin = uint32_t(r0 < n_rules ? r0 : n_rules);
    const uint32_t end = uint32_t(r0 + S < n_rules ? r0 + S : n_rules);
    for (uint32_t c = begin; c < end && ws.any_live(); c += kHybridChunk) {
        const uint32_t cnt = min(kHybridChunk, end - c);
        ws.template scan<FirstField::Dst>(pairs + c, rules + c, cnt, c);
        uint64_t live_any = 0;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (ws.best[s] != kNoMatch) atomicMin(&smin[K * lane + s], ws.best[s]);
            const uint32_t cur = *reinterpret_cast<volatile uint32_t*>(&smin[K * lane + s]);
            ws.live[s] &= ballot(cur > c + cnt);
            live_any |= ws.live[s];
        }
        ws.live_any = live_any;
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const size_t i = first + K * lane + s;
            if (i < n) {
                const uint32_t b = smin[K * lane + s];
                out_idx[i] = int32_t(b);
                out_act[i] = uint8_t(b == kNoMatch ? dflt : rule_action(rules[b].proto));
            }
        }
    }
}

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return uint32_t((a + b - 1) / b); }

// A dispatch's grid size is a 32-bit count of work-items per dimension, so
// one launch covers fewer than 2^32 of them.  Batches that would need more
// are launched in chunks; every chunk size is a multiple of 64 packets, so
// the offset arrays stay 16-byte aligned.
constexpr uint64_t kMaxLaunchItems = (uint64_t(1) << 32) - 1024;

PacketsDev advance(const PacketsDev& pk, size_t o) {
    return PacketsDev{pk.src + o, pk.dst + o, pk.sport + o, pk.dport + o, pk.proto + o};
}

// Largest chunk of packets (a multiple of 64) whose launch needs at most
// kMaxLaunchItems work-items when each packet costs items_per_packet of them.
size_t chunk_packets(double items_per_packet) {
    const double c = double(kMaxLaunchItems) / items_per_packet;
    const size_t k = size_t(c) / 64u * 64u;
    return k < 64u ? 64u : k;
}

template <class F>
hipError_t in_chunks(size_t n, size_t chunk, F launch) {
    for (size_t o = 0; o < n; o += chunk) {
        const hipError_t e = launch(o, n - o < chunk ? n - o : chunk);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t fill_no_match(uint32_t* idx, size_t n, hipStream_t stream) {
    return in_chunks(n, chunk_packets(1.0), [&](size_t o, size_t c) {
        hipLaunchKernelGGL(k_fill_u32, dim3(ceil_div(c, 256)), dim3(256), 0, stream, idx + o, c,
                           kNoMatch);
        return hipGetLastError();
    });
}

hipError_t apply_action(const RuleRec* rules, const int32_t* idx, size_t n, uint8_t* out_act,
                        uint8_t default_action, hipStream_t stream) {
    return in_chunks(n, chunk_packets(1.0), [&](size_t o, size_t c) {
        hipLaunchKernelGGL(k_apply_action, dim3(ceil_div(c, 256)), dim3(256), 0, stream, rules,
                           idx + o, c, out_act + o, uint32_t(default_action));
        return hipGetLastError();
    });
}

}  // namespace

hipError_t launch_packet_split(const ScanPlan& plan, PacketsDev pk, size_t n, int32_t* out_idx,
                               uint8_t* out_act, uint8_t default_action, int packets_per_lane,
                               hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const int K = packets_per_lane;
    const uint64_t per_block = uint64_t(kScanBlock) * K;
    const uint32_t dflt = default_action;
    return in_chunks(n, chunk_packets(1.0 / K), [&](size_t o, size_t c) {
        const uint32_t grid = ceil_div(c, per_block);
        const PacketsDev p = advance(pk, o);
        if (K == 4)
            hipLaunchKernelGGL(k_packet_split<4>, dim3(grid), dim3(kScanBlock), 0, stream, plan,
                               p, c, out_idx + o, out_act + o, dflt);
        else if (K == 2)
            hipLaunchKernelGGL(k_packet_split<2>, dim3(grid), dim3(kScanBlock), 0, stream, plan,
                               p, c, out_idx + o, out_act + o, dflt);
        else
            hipLaunchKernelGGL(k_packet_split<1>, dim3(grid), dim3(kScanBlock), 0, stream, plan,
                               p, c, out_idx + o, out_act + o, dflt);
        return hipGetLastError();
    });
}

hipError_t launch_rule_split(const RuleRec* rules, uint32_t n_rules, uint32_t P, PacketsDev pk,
                             size_t n, int32_t* out_idx, uint8_t* out_act,
                             uint8_t default_action, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    uint32_t* idx = reinterpret_cast<uint32_t*>(out_idx);
    hipError_t e = fill_no_match(idx, n, stream);
    if (e != hipSuccess) return e;
    if (n_rules > 0) {
        // Partitions of S rules; when they are shorter than a wave's 64 lanes,
        // one wave takes ceil(64 / S) consecutive partitions (their minimum is
        // merged inside the wave, exactly as across waves), so no lane idles
        // for want of a rule.
        const uint32_t S0 = ceil_div(n_rules, P);
        const uint32_t S = S0 >= 64u ? S0 : S0 * ceil_div(64u, S0);
        P = ceil_div(n_rules, S);
        // P waves of 64 lanes per G packets, numbered partition-major
        const uint32_t G = n >= kRsLargeBatch ? 16u : 8u;
        e = in_chunks(n, chunk_packets(64.0 * P / G), [&](size_t o, size_t c) {
            const uint64_t waves = uint64_t(P) * ((c + G - 1) / G);
            const uint64_t blocks = (waves + (kScanBlock / 64) - 1) / (kScanBlock / 64);
            if (G == 16)
                hipLaunchKernelGGL(k_rule_split<16>, dim3(uint32_t(blocks)), dim3(kScanBlock), 0,
                                   stream, rules, n_rules, P, S, advance(pk, o), c, idx + o);
            else
                hipLaunchKernelGGL(k_rule_split<8>, dim3(uint32_t(blocks)), dim3(kScanBlock), 0,
                                   stream, rules, n_rules, P, S, advance(pk, o), c, idx + o);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
    }
    return apply_action(rules, out_idx, n, out_act, default_action, stream);
}

hipError_t launch_hybrid(const uint2* pairs, const RuleRec* rules, uint32_t n_rules, uint32_t P,
                         PacketsDev pk,
                         size_t n, int32_t* out_idx, uint8_t* out_act, uint8_t default_action,
                         int packets_per_lane, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t S = n_rules == 0 ? 1u : ceil_div(n_rules, P);
    const uint32_t K = uint32_t(packets_per_lane);
    // a work-group of 64*P lanes per 64*K packets
    return in_chunks(n, chunk_packets(double(P) / K), [&](size_t o, size_t c) {
        const dim3 grid(ceil_div(c, 64u * K)), block(64 * P);
        const PacketsDev q = advance(pk, o);
        const uint32_t d = uint32_t(default_action);
        if (K == 4)
            hipLaunchKernelGGL(k_hybrid<4>, grid, block, 0, stream, pairs, rules, n_rules, S, q,
                               c, out_idx + o, out_act + o, d);
        else if (K == 2)
            hipLaunchKernelGGL(k_hybrid<2>, grid, block, 0, stream, pairs, rules, n_rules, S, q,
                               c, out_idx + o, out_act + o, d);
        else
            hipLaunchKernelGGL(k_hybrid<1>, grid, block, 0, stream, pairs, rules, n_rules, S, q,
                               c, out_idx + o, out_act + o, d);
        return hipGetLastError();
    });
}

}  // namespace fw
