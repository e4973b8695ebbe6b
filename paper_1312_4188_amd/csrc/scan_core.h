// The packet-split scan of one wave, shared by the single-chain and the
// multi-chain kernels.
#pragma once

#include "device_util.h"
#include "fw_internal.h"

namespace fw {

// Load K consecutive packets starting at p0 (p0 is a multiple of K).  Full
// groups use one 128-bit (K=4), 64-bit (K=2) or 32-bit load per address array;
// the ragged tail falls back to element loads.
template <int K>
__device__ __forceinline__ void load_packets(const PacketsDev& pk, size_t p0, size_t n,
                                             uint32_t (&src)[K], uint32_t (&dst)[K],
                                             uint32_t (&pp)[K], uint32_t (&pr)[K]) {
    if (p0 + K <= n) {
        if constexpr (K == 4) {
            const uint4 s = *reinterpret_cast<const uint4*>(pk.src + p0);
            const uint4 d = *reinterpret_cast<const uint4*>(pk.dst + p0);
            const uint2 sp = *reinterpret_cast<const uint2*>(pk.sport + p0);
            const uint2 dp = *reinterpret_cast<const uint2*>(pk.dport + p0);
            const uint32_t p = *reinterpret_cast<const uint32_t*>(pk.proto + p0);
            src[0] = s.x; src[1] = s.y; src[2] = s.z; src[3] = s.w;
            dst[0] = d.x; dst[1] = d.y; dst[2] = d.z; dst[3] = d.w;
            // packed pair = sport << 16 | dport
            pp[0] = (sp.x << 16) | (dp.x & 0xFFFFu);
            pp[1] = (sp.x & 0xFFFF0000u) | (dp.x >> 16);
            pp[2] = (sp.y << 16) | (dp.y & 0xFFFFu);
            pp[3] = (sp.y & 0xFFFF0000u) | (dp.y >> 16);
            pr[0] = p & 0xFFu; pr[1] = (p >> 8) & 0xFFu;
            pr[2] = (p >> 16) & 0xFFu; pr[3] = p >> 24;
            return;
        } else if constexpr (K == 2) {
            const uint2 s = *reinterpret_cast<const uint2*>(pk.src + p0);
            const uint2 d = *reinterpret_cast<const uint2*>(pk.dst + p0);
            const uint32_t sp = *reinterpret_cast<const uint32_t*>(pk.sport + p0);
            const uint32_t dp = *reinterpret_cast<const uint32_t*>(pk.dport + p0);
            const uint32_t p = *reinterpret_cast<const uint16_t*>(pk.proto + p0);
            src[0] = s.x; src[1] = s.y;
            dst[0] = d.x; dst[1] = d.y;
            pp[0] = (sp << 16) | (dp & 0xFFFFu);
            pp[1] = (sp & 0xFFFF0000u) | (dp >> 16);
            pr[0] = p & 0xFFu; pr[1] = p >> 8;
            return;
        }
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const size_t i = p0 + s;
        const bool ok = i < n;
        src[s] = ok ? pk.src[i] : 0u;
        dst[s] = ok ? pk.dst[i] : 0u;
        pp[s] = ok ? ((uint32_t(pk.sport[i]) << 16) | pk.dport[i]) : 0u;
        pr[s] = ok ? uint32_t(pk.proto[i]) : 0u;
    }
}

template <int K>
__device__ __forceinline__ void store_results(int32_t* out_idx, uint8_t* out_act, size_t p0,
                                              size_t n, const uint32_t (&best)[K],
                                              const uint32_t (&act)[K]) {
    if (p0 + K <= n) {
        if constexpr (K == 4) {
            *reinterpret_cast<int4*>(out_idx + p0) =
                make_int4(int(best[0]), int(best[1]), int(best[2]), int(best[3]));
            *reinterpret_cast<uint32_t*>(out_act + p0) =
                act[0] | (act[1] << 8) | (act[2] << 16) | (act[3] << 24);
            return;
        } else if constexpr (K == 2) {
            *reinterpret_cast<int2*>(out_idx + p0) = make_int2(int(best[0]), int(best[1]));
            *reinterpret_cast<uint16_t*>(out_act + p0) = uint16_t(act[0] | (act[1] << 8));
            return;
        }
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
        if (p0 + s < n) {
            out_idx[p0 + s] = int32_t(best[s]);
            out_act[p0 + s] = uint8_t(act[s]);
        }
    }
}

// Which packet field a rule is tested on first (see FirstTest).
enum class FirstField { Dst = kFirstDst, Src = kFirstSrc, Ports = kFirstPorts, Proto = kFirstProto };

// Rules per prefetch block of the first-test pairs: 8 pairs = 64 bytes, one
// scalar load.  Pair arrays carry kPairPadding extra entries so the block
// after the last one can be fetched without a bounds test.
constexpr uint32_t kPairBlock = 8;
static_assert(kPairPadding >= kPairBlock, "pair arrays must be padded by a whole block");

// First-match state of one wave over 64*K packets (K per lane).  Rule
// addresses are wave-uniform: the first-test pair (lo, w) of each rule arrives
// through scalar loads, 8 rules at a time and one block ahead, so the field
// test takes its rule operands from SGPRs without waiting.  A ballot turns
// the lanes' tests into a wave mask; when no live lane passes, the rule is
// done after 2K vector ops (3K for the port pair).  Otherwise the full record
// is read and the remaining fields are tested the same way; matched lanes
// take the rule through a select on the wave mask itself.
// Load through the vector memory path even when the address is wave-uniform:
// the empty asm moves the pointer into VGPRs, so the compiler can no longer
// use a scalar load.  Every lane reads the same bytes (one cache line per
// wave); the value lands in a VGPR.
template <class T>
__device__ __forceinline__ T vector_load(const T* p) {
    static_assert(sizeof(T) % 8 == 0 && alignof(T) >= 8, "whole 8-byte words");
    asm volatile("" : "+v"(p));
    using Word = const __attribute__((address_space(1))) uint64_t;   // global memory
    Word* g = (Word*)__builtin_assume_aligned(p, 8);
    uint64_t w[sizeof(T) / 8];
#pragma unroll
    for (size_t i = 0; i < sizeof(T) / 8; ++i) w[i] = g[i];
    T out;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}

// BATCH: with one packet per lane, a block's eight first tests are taken at
// once before its single branch (shorter dependence chains: a small batch,
// whose few waves cannot hide them, finishes sooner).  It costs 16 scalar
// registers, so a kernel short of them turns it off.
template <int K, bool BATCH = K == 1>
struct WaveScan {
    uint32_t src[K], dst[K], pp[K], pr[K];
    uint64_t valid[K];
    uint64_t live[K];
    uint64_t live_any;
    uint32_t best[K], act[K];
    size_t p0;

    __device__ __forceinline__ void init(const PacketsDev& pk, size_t wave_first, size_t n,
                                         uint32_t dflt) {
        p0 = wave_first + size_t(threadIdx.x & 63u) * K;
        load_packets<K>(pk, p0, n, src, dst, pp, pr);
        live_any = 0;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            valid[s] = ballot(p0 + s < n);
            live[s] = valid[s];
            live_any |= live[s];
            best[s] = kNoMatch;
            act[s] = dflt;
        }
    }

    // Single-packet-per-lane start from values already in registers.
    __device__ __forceinline__ void init_values(uint32_t s_, uint32_t d_, uint32_t pp_,
                                                uint32_t pr_, bool ok, uint32_t dflt) {
        static_assert(K == 1, "one packet per lane");
        src[0] = s_;
        dst[0] = d_;
        pp[0] = pp_;
        pr[0] = pr_;
        valid[0] = ballot(ok);
        live[0] = valid[0];
        live_any = live[0];
        best[0] = kNoMatch;
        act[0] = dflt;
        p0 = 0;
    }

    __device__ __forceinline__ bool any_live() const { return live_any != 0; }

    template <FirstField F>
    __device__ __forceinline__ bool first_test(int s, uint2 f) const {
        if constexpr (F == FirstField::Dst) return in_range(dst[s], f.x, f.y);
        if constexpr (F == FirstField::Src) return in_range(src[s], f.x, f.y);
        if constexpr (F == FirstField::Ports) return ports_in(pp[s], f.x, f.y);
        return in_range(pr[s], f.x, f.y);
    }

    // Remaining tests of a rule some live lane passed on its first field.  A
    // rule tested first on the ports has both addresses unspecified, one
    // tested first on the protocol has addresses and ports unspecified, so
    // those tests are skipped.  After an address, the other address is tested
    // on its own first: about half the rules some lane passes on one address
    // fail on the other in every lane, and leave without the port and protocol
    // tests.  With SEEDED, a lane takes the rule only if it beats the lane's
    // current answer.  Matched lanes leave the live masks.
    template <FirstField F, bool SEEDED>
    __device__ __forceinline__ void finish(const uint64_t (&c)[K], const RuleRec& q,
                                           uint32_t idx) {
        const uint32_t plo = proto_lo(q.proto), pw = proto_w(q.proto);
        uint64_t m[K];
        if constexpr (F == FirstField::Dst || F == FirstField::Src) {
            uint64_t some = 0;
#pragma unroll
            for (int s = 0; s < K; ++s) {
                m[s] = c[s] & live[s];
                if constexpr (F == FirstField::Src)
                    m[s] &= ballot(in_range(dst[s], q.dst_lo, q.dst_w));
                else
                    m[s] &= ballot(in_range(src[s], q.src_lo, q.src_w));
                some |= m[s];
            }
            if (some == 0) return;
        } else {
#pragma unroll
            for (int s = 0; s < K; ++s) m[s] = c[s] & live[s];
        }
        uint64_t any = 0;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if constexpr (F == FirstField::Dst || F == FirstField::Src)
                m[s] &= ballot(ports_in(pp[s], q.port_lo, q.port_w));
            if constexpr (F != FirstField::Proto) m[s] &= ballot(in_range(pr[s], plo, pw));
            if constexpr (SEEDED) m[s] &= ballot(best[s] > idx);
            any |= m[s];
        }
        if (any == 0) return;
        const uint32_t ra = rule_action(q.proto);
        live_any = 0;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (__builtin_amdgcn_inverse_ballot_w64(m[s])) {
                best[s] = idx;
                act[s] = ra;
            }
            live[s] &= ~m[s];
            live_any |= live[s];
        }
    }

    template <FirstField F, bool OWN_INDEX, bool SEEDED>
    __device__ __forceinline__ void step(uint2 f, const RuleRec* __restrict__ rules, uint32_t r,
                                         uint32_t base) {
        uint64_t c[K];
        uint64_t any = 0;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            c[s] = ballot(first_test<F>(s, f));
            any |= c[s];
        }
        if (__builtin_expect((any & live_any) != 0, 0)) {
            const RuleRec q = rules[r];
            finish<F, SEEDED>(c, q, OWN_INDEX ? q.idx : base + r);
        }
    }

    // Rules r = 0..count-1: first-test pair first[r], record rules[r], index
    // base + r (or the record's own index field with OWN_INDEX).  The pairs
    // come 8 at a time, one block ahead; the scan stops after the block in
    // which its last live lane matched.  Returns false once no lane is live.
    template <FirstField F, bool OWN_INDEX = false, bool SEEDED = false>
    __device__ __forceinline__ bool scan(const uint2* __restrict__ first,
                                         const RuleRec* __restrict__ rules, uint32_t count,
                                         uint32_t base) {
        if (live_any == 0) return false;
        uint32_t r = 0;
        if (count >= kPairBlock) {
            uint2 cur[kPairBlock];
#pragma unroll
            for (uint32_t u = 0; u < kPairBlock; ++u) cur[u] = first[u];
            for (; r + kPairBlock <= count; r += kPairBlock) {
                uint2 nxt[kPairBlock];
                if constexpr (K == 1 && BATCH) {
#pragma unroll
                    for (uint32_t u = 0; u < kPairBlock; ++u) nxt[u] = first[r + kPairBlock + u];
                    // the block's eight first tests at once (they do not depend
                    // on which lanes are live), then one branch; a block with a
                    // passing lane goes rule by rule in order, as step() does
                    uint64_t c8[kPairBlock];
                    uint64_t any = 0;
#pragma unroll
                    for (uint32_t u = 0; u < kPairBlock; ++u) {
                        c8[u] = ballot(first_test<F>(0, cur[u]));
                        any |= c8[u];
                    }
                    if (__builtin_expect((any & live_any) != 0, 0)) {
#pragma unroll
                        for (uint32_t u = 0; u < kPairBlock; ++u) {
                            if ((c8[u] & live_any) != 0) {
                                const RuleRec q = rules[r + u];
                                const uint64_t cu[1] = {c8[u]};
                                finish<F, SEEDED>(cu, q, OWN_INDEX ? q.idx : base + r + u);
                            }
                        }
                    }
                } else {
                    // the next block's pairs are requested after this block's
                    // first rule: the wait for a block's pairs (at the copy
                    // below) then finds them loaded behind seven rules of work,
                    // where a request at the top of the block would be waited
                    // for with the current block's own
                    step<F, OWN_INDEX, SEEDED>(cur[0], rules, r, base);
#pragma unroll
                    for (uint32_t u = 0; u < kPairBlock; ++u) nxt[u] = first[r + kPairBlock + u];
#pragma unroll
                    for (uint32_t u = 1; u < kPairBlock; ++u)
                        step<F, OWN_INDEX, SEEDED>(cur[u], rules, r + u, base);
                }
                if (live_any == 0) return false;
#pragma unroll
                for (uint32_t u = 0; u < kPairBlock; ++u) cur[u] = nxt[u];
            }
        }
        for (; r < count; ++r) {
            step<F, OWN_INDEX, SEEDED>(first[r], rules, r, base);
            if (live_any == 0) return false;
        }
        return true;
    }

    // The same first-match scan with the rule operands read by vector loads
    // (every lane the same address) instead of scalar loads: the pairs of
    // the next block of 8 rules are fetched while the current block is
    // tested, as in scan(), but they arrive in VGPRs through the vector
    // cache.  Destination-first, rule index = position.
    __device__ __forceinline__ bool scan_vector(const uint2* __restrict__ first,
                                                const RuleRec* __restrict__ rules,
                                                uint32_t count) {
        if (live_any == 0) return false;
        uint32_t r = 0;
        if (count >= kPairBlock) {
            uint2 cur[kPairBlock];
#pragma unroll
            for (uint32_t u = 0; u < kPairBlock; ++u) cur[u] = vector_load(first + u);
            for (; r + kPairBlock <= count; r += kPairBlock) {
                uint2 nxt[kPairBlock];
#pragma unroll
                for (uint32_t u = 0; u < kPairBlock; ++u)
                    nxt[u] = vector_load(first + r + kPairBlock + u);
#pragma unroll
                for (uint32_t u = 0; u < kPairBlock; ++u) vector_step(cur[u], rules, r + u);
                if (live_any == 0) return false;
#pragma unroll
                for (uint32_t u = 0; u < kPairBlock; ++u) cur[u] = nxt[u];
            }
        }
        for (; r < count; ++r) {
            vector_step(vector_load(first + r), rules, r);
            if (live_any == 0) return false;
        }
        return true;
    }

    __device__ __forceinline__ void vector_step(uint2 f, const RuleRec* __restrict__ rules,
                                                uint32_t r) {
        uint64_t c[K];
        uint64_t any = 0;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            c[s] = ballot(first_test<FirstField::Dst>(s, f));
            any |= c[s];
        }
        if (__builtin_expect((any & live_any) != 0, 0))
            finish<FirstField::Dst, false>(c, vector_load(rules + r), r);
    }

    // Grouped scan (ScanPlan).  The catch-all tail seeds every valid lane's
    // answer (when it beats what the lane already holds); then each group is
    // scanned in rule order by every valid lane whose answer could still
    // improve, taking a rule only when it beats the lane's answer.  The
    // answer is the minimum over groups of each group's first match, which is
    // the first match of the whole list.
    // The plan's catch-all tail seeds every valid lane whose answer it beats.
    __device__ __forceinline__ void seed_tail(const ScanPlan& plan) {
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (__builtin_amdgcn_inverse_ballot_w64(valid[s]) && plan.tail_idx < best[s]) {
                best[s] = plan.tail_idx;
                act[s] = plan.tail_act;
            }
        }
    }

    // Entering a group whose first rule has index first_idx: the live lanes
    // are the valid ones whose answer could still improve.
    __device__ __forceinline__ void enter_group(uint32_t first_idx) {
        live_any = 0;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            live[s] = valid[s] & ballot(best[s] > first_idx);
            live_any |= live[s];
        }
    }

    // ADDRESSES false: a plan of rules with both addresses unspecified (only
    // port- and protocol-first groups), whose address groups need no code.
    template <bool ADDRESSES = true>
    __device__ __forceinline__ void scan_plan(const ScanPlan& plan) {
        seed_tail(plan);
        for (uint32_t g = 0; g < plan.n_groups; ++g) {
            const ScanGroup& G = plan.g[g];
            enter_group(G.recs[0].idx);
            switch (G.kind) {
                case kFirstDst:
                    if constexpr (ADDRESSES)
                        scan<FirstField::Dst, true, true>(G.pairs, G.recs, G.count, 0u);
                    break;
                case kFirstSrc:
                    if constexpr (ADDRESSES)
                        scan<FirstField::Src, true, true>(G.pairs, G.recs, G.count, 0u);
                    break;
                case kFirstPorts:
                    scan<FirstField::Ports, true, true>(G.pairs, G.recs, G.count, 0u);
                    break;
                default:
                    scan<FirstField::Proto, true, true>(G.pairs, G.recs, G.count, 0u);
                    break;
            }
        }
    }

    __device__ __forceinline__ void store(int32_t* out_idx, uint8_t* out_act, size_t n) const {
        store_results<K>(out_idx, out_act, p0, n, best, act);
    }
};

// One wave classifies the 64*K packets starting at wave_first.
template <int K>
__device__ __forceinline__ void scan_wave(const uint2* __restrict__ first,
                                          const RuleRec* __restrict__ rules, uint32_t n_rules,
                                          const PacketsDev& pk, size_t wave_first, size_t n,
                                          int32_t* __restrict__ out_idx,
                                          uint8_t* __restrict__ out_act, uint32_t dflt) {
    WaveScan<K> w;
    w.init(pk, wave_first, n, dflt);
    w.template scan<FirstField::Dst>(first, rules, n_rules, 0u);
    w.store(out_idx, out_act, n);
}

}  // namespace fw
