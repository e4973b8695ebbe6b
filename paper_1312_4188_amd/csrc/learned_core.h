// The learned lookup shared by the single-chain kernels (rmi.hip) and the
// multi-chain kernel (multi.hip): network inference, the window search, the
// candidate-list walks, and the staging of an index's LDS image.
#pragma once

#include "device_util.h"
#include "fw_internal.h"
#include "index.h"
#include "scan_core.h"

namespace fw {

// ------------------------------------------------------------------ inference
// Stage 1 is kept as fp32 (the bf16 values widened) in four 32-slot segments
// [w1][b1][w2][b2]; stage 2 as rows of (half w1, b1) pair dwords and widened
// w2, b2 (see kRowDwords).  Hidden units past H carry zero weights and add nothing.
// Every routine below is shared by the error-bound kernel and the lookup
// kernels, so the recorded error bounds describe exactly the lookup's
// arithmetic.
constexpr uint32_t kSeg = 32;

// ReLU of a pre-activation the index build has scaled into (-inf, 1] (see
// the unit scaling at quantisation): max(z, 0) = clamp(z, 0, 1), which the
// compiler folds into the producing multiply-add's clamp modifier.
__device__ __forceinline__ float relu01(float z) { return __builtin_amdgcn_fmed3f(z, 0.0f, 1.0f); }

// Stage 1: u = x / 2^32 -> expert index in [0, E), for K keys at once: the
// weights are the same for every key, so each is read once and used K times;
// every key sees the same sequence of operations as on its own.
template <int K>
__device__ __forceinline__ void route(const float* w1, uint32_t E, const uint32_t (&x)[K],
                                      uint32_t (&e)[K]) {
    float u[K], y[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
        u[s] = float(x[s]) * 0x1p-32f;
        y[s] = w1[3 * kSeg];
    }
#pragma unroll
    for (uint32_t k = 0; k < kSeg; ++k) {
        const float a = w1[k], b = w1[kSeg + k], o = w1[2 * kSeg + k];
#pragma unroll
        for (int s = 0; s < K; ++s) y[s] = fmaf(o, relu01(fmaf(a, u[s], b)), y[s]);
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const float t = y[s] * float(E);
        // NaN and negatives go to expert 0, overflow to the last expert
        e[s] = t >= 1.0f ? (t < float(E) ? uint32_t(t) : E - 1u) : 0u;
    }
}

__device__ __forceinline__ uint32_t route(const float* w1, uint32_t E, uint32_t x) {
    const uint32_t k[1] = {x};
    uint32_t e[1];
    route<1>(w1, E, k, e);
    return e[0];
}

// Stage 2: position estimate of x inside expert e's range of positions (the
// row carries the expert's input scaling and position span; pos_lo is its
// first position).  Hidden unit k takes w1 as the fp16 value in the low half
// of its pair dword and its bias as the whole dword read as fp32 (the index
// build picks the high half for it), forms fp32 max(w1 v + b1, 0) as one
// clamped mixed-precision multiply-add (the half operand widened exactly, the
// arithmetic fp32), and adds its fp32 w2 share with a second: two
// instructions per unit.
__device__ __forceinline__ int32_t position(const uint32_t* row, int32_t pos_lo, uint32_t x) {
    const uint32_t key_lo = row[kRowKeyLo];
    const float inv_span = __uint_as_float(row[kRowInvSpan]);
    const float pos_span = __uint_as_float(row[kRowPosSpan]);
    const float v = x >= key_lo ? fminf(float(x - key_lo) * inv_span, 1.0f) : 0.0f;
    float y = __uint_as_float(row[kRowBias]);
#pragma unroll
    for (uint32_t c = 0; c < kSeg; c += 8) {
        const uint4 p0 = *reinterpret_cast<const uint4*>(row + kRowPairs + c);
        const uint4 p1 = *reinterpret_cast<const uint4*>(row + kRowPairs + c + 4);
        const uint4 o = *reinterpret_cast<const uint4*>(row + kRowOut + c / 2);
        const uint32_t pr[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
        const uint32_t oh[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float w1 = float(__builtin_bit_cast(_Float16, uint16_t(pr[i] & 0xFFFFu)));
            const float b1 = __uint_as_float(pr[i]);
            const uint32_t ob = oh[i / 2];
            const float w2 = float(__builtin_bit_cast(
                _Float16, uint16_t((i & 1) ? (ob >> 16) : (ob & 0xFFFFu))));
            y = fmaf(w2, relu01(fmaf(w1, v, b1)), y);
        }
    }
    const float q = fminf(fmaxf(y * pos_span, 0.0f), pos_span);  // NaN -> 0
    return pos_lo + int32_t(rintf(q));
}

// Largest j in [lo, hi] with B[j] <= x, assuming B[lo] <= x.
__device__ __forceinline__ uint32_t search_le(const uint32_t* B, uint32_t lo, uint32_t hi,
                                              uint32_t x) {
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1u) >> 1;
        if (B[mid] <= x)
            lo = mid;
        else
            hi = mid - 1u;
    }
    return lo;
}

// Interval of x among the M sorted starts B (B[0] = 0) through a bucket table
// over its top `bits` bits: the bucket's entry is the interval holding the
// bucket's first key, and `steps` forward steps (never past the last
// interval) reach x's interval.
__device__ __forceinline__ uint32_t bucket_walk(const uint16_t* bucket, const uint32_t* B,
                                                uint32_t M, uint32_t bits, uint32_t steps,
                                                uint32_t x) {
    uint32_t i = bucket[x >> (32u - bits)];
#pragma unroll 1   // serial steps (see port_table_first)
    for (uint32_t k = 0; k < steps; ++k) i += (i + 1u < M && B[i + 1u] <= x) ? 1u : 0u;
    return i;
}

// Interval of x, routed to expert e by stage 1: the window [p - err, p + err]
// of the predicted position first, checked by B[j] <= x < B[j+1]; a miss
// falls back to the full range.  `meta` holds each expert's first position and
// error bound (the rest of its record rides in its row).
__device__ __forceinline__ uint32_t locate(const uint32_t* B, uint32_t M, const uint32_t* w2,
                                           const LdsExpert* meta, uint32_t use_net, uint32_t e,
                                           uint32_t x, bool* miss) {
    if (use_net) {
        const LdsExpert m = meta[e];
        const int32_t p = position(w2 + size_t(e) * kRowDwords, m.pos_lo, x);
        const int64_t lo = int64_t(p) - int64_t(m.err), hi = int64_t(p) + int64_t(m.err);
        const uint32_t l = uint32_t(lo < 0 ? 0 : (lo >= int64_t(M) ? M - 1 : lo));
        const uint32_t h = uint32_t(hi < int64_t(l) ? l : (hi >= int64_t(M) ? M - 1 : hi));
        if (B[l] <= x) {
            const uint32_t j = search_le(B, l, h, x);
            if (j + 1u == M || x < B[j + 1u]) {
                *miss = false;
                return j;
            }
        }
        *miss = true;
    } else {
        *miss = false;
    }
    return search_le(B, 0, M - 1u, x);
}

// Per-lane list records through buffer loads.  The resource covers the
// list's bytes; a byte offset of kPastEnd (beyond any list the index
// accepts) is out of range, and an out-of-range buffer load returns zeros
// without touching memory.
constexpr uint32_t kPastEnd = kListPastEnd;
constexpr uint32_t kBufferDword3 = 0x00020000u;   // raw buffer, gfx9-family format bits

__device__ __forceinline__ __amdgpu_buffer_rsrc_t list_rsrc(const RuleRec* base, uint32_t count) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<RuleRec*>(base), 0,
                                             int(count * uint32_t(sizeof(RuleRec))),
                                             int(kBufferDword3));
}

__device__ __forceinline__ RuleRec list_record(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    const uint4 lo = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, int(byte_off), 0, 0));
    const uint4 hi = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, int(byte_off + 16u), 0, 0));
    RuleRec q;
    q.src_lo = lo.x;
    q.src_w = lo.y;
    q.dst_lo = lo.z;
    q.dst_w = lo.w;
    q.port_lo = hi.x;
    q.port_w = hi.y;
    q.proto = hi.z;
    q.idx = hi.w;
    return q;
}

// Only the second half (ports, protocol, index): enough for lists whose
// address tests are implied.
__device__ __forceinline__ RuleRec list_record_tail(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    const uint4 hi = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, int(byte_off + 16u), 0, 0));
    RuleRec q{};
    q.port_lo = hi.x;
    q.port_w = hi.y;
    q.proto = hi.z;
    q.idx = hi.w;
    return q;
}

// First rule of a port/protocol table that the packet matches, as
// rule index | action << 24, or kPtNone.  pp = source port << 16 | destination
// port.  Each port's interval: the high-byte table gives the interval holding
// the bucket's first port, then `steps` forward steps (an interval start past
// the port stops the walk; the entry after the last interval is 0x10000).
__device__ __forceinline__ uint32_t port_table_first(const PortTable& t, uint32_t steps_s,
                                                     uint32_t steps_d, uint32_t pp, uint32_t pr) {
    const uint32_t sp = pp >> 16, dp = pp & 0xFFFFu;
    uint32_t is = t.bucket_s[sp >> 8], id = t.bucket_d[dp >> 8];
    // Each step depends on the one before, so unrolling gains nothing; kept
    // rolled, the loops need no precomputed remainder masks in scalar registers.
#pragma unroll 1
    for (uint32_t k = 0; k < steps_s; ++k) is += t.b_s[is + 1u] <= sp ? 1u : 0u;
#pragma unroll 1
    for (uint32_t k = 0; k < steps_d; ++k) id += t.b_d[id + 1u] <= dp ? 1u : 0u;
    const uint64_t m = t.mask_s[is] & t.mask_d[id] & t.mask_p[pr & 0xFFu];
    return t.rule[m ? uint32_t(__builtin_ctzll(m)) : kPtRules];
}

// ------------------------------------------------------------------ lookup + candidate scan
// Persistent work-groups of 16 waves.  Each stages the stage-1 weights, the
// experts' records and bf16 weights, and (when it fits) the boundary array
// into LDS once; its waves then stride over tiles of 64*K packets:
//   1. locate each packet's destination interval j (network + window, else a
//      full binary search);
//   2. scan j's own candidate list per lane (ascending, stop at the first match);
//   3. locate the source interval i among the destination-wildcard candidates
//      that specify a source, and scan i's list per lane the same way (ports
//      and protocol tested; destination and source are implied);
//   4. the candidates with both addresses unspecified: the first 64 through
//      the port/protocol table (three masks ANDed, lowest bit), the rest
//      with the packet-split wave scan over a grouped plan; every step is
//      seeded with the best so far, so each lane keeps the smallest of the
//      partial first matches (the table runs before the lists, so they can
//      stop early);
//   5. write the index and action.
constexpr uint32_t kLearnedBlock = 1024;
constexpr uint32_t kLearnedK = 2;     // default packets per lane in the classify kernel

struct IndexView {
    const float* w1;
    const LdsExpert* meta;
    const uint32_t* w2;       // stage-2 rows, kRowDwords each
    const uint32_t* B;
    const uint32_t* Bs;
    const PortTable* pt;
    const uint16_t* bs_bucket;
    const uint32_t* off;
    const uint32_t* soff;
};

// Copy `words` 16-byte words from global memory to LDS.  Each thread issues
// all of its loads of a round (four words) before its stores, and the whole
// index image is one copy, so staging costs about one memory round trip
// instead of one per array and per stride of the loop.
__device__ __forceinline__ void stage_words(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                            uint32_t words) {
    constexpr uint32_t U = 4;
    for (uint32_t base = threadIdx.x; base < words; base += U * kLearnedBlock) {
        uint4 v[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t k = base + u * kLearnedBlock;
            v[u] = src[k < words ? k : words - 1u];
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t k = base + u * kLearnedBlock;
            if (k < words) dst[k] = v[u];
        }
    }
}

// Stage the index into LDS: the build wrote, for each placement, the exact
// LDS image (see LdsLayout), so staging is one copy.
// Where an index's arrays are once its image is in LDS (no copy).
template <bool B_LDS>
__device__ __forceinline__ IndexView index_view(const LookupArgs& a, const unsigned char* smem) {
    const LdsLayout L(a.E, a.M, a.Ms, a.bs_bits, B_LDS);
    return IndexView{reinterpret_cast<const float*>(smem + L.w1),
                     reinterpret_cast<const LdsExpert*>(smem + L.meta),
                     reinterpret_cast<const uint32_t*>(smem + L.w2),
                     B_LDS ? reinterpret_cast<const uint32_t*>(smem + L.b) : a.B,
                     B_LDS ? reinterpret_cast<const uint32_t*>(smem + L.bs) : a.Bs,
                     reinterpret_cast<const PortTable*>(smem + L.pt),
                     reinterpret_cast<const uint16_t*>(smem + L.bk),
                     B_LDS ? reinterpret_cast<const uint32_t*>(smem + L.off) : a.off,
                     B_LDS ? reinterpret_cast<const uint32_t*>(smem + L.soff) : a.soff};
}

template <bool B_LDS>
__device__ __forceinline__ IndexView stage_index(const LookupArgs& a, unsigned char* smem) {
    const LdsLayout L(a.E, a.M, a.Ms, a.bs_bits, B_LDS);
    stage_words(reinterpret_cast<uint4*>(smem), a.image[B_LDS], uint32_t(L.bytes / 16u));
    __syncthreads();
    return index_view<B_LDS>(a, smem);
}

// One wave's tile: the 64*K packets starting at `base` (base < n), through
// steps 1-5 above, with the index staged as `v`.  PLAN: the grouped plan of
// address-wildcard candidates beyond the port table may have groups to scan;
// without it only its catch-all tail is applied, and the code carries none of
// the plan scan's scalar state.
template <int K, bool PLAN>
__device__ __forceinline__ void learned_tile(const LookupArgs& a, const IndexView& v,
                                             const PacketsDev& pk, size_t base, size_t n,
                                             int32_t* __restrict__ out_idx,
                                             uint8_t* __restrict__ out_act, uint32_t dflt) {
    const uint32_t lane = threadIdx.x & 63u;
    WaveScan<K> w;
    w.init(pk, base, n, dflt);
    uint32_t lbest[K], lact[K], jj[K], si[K];
    // every packet's destination and source intervals first: stage 1
    // routes the K keys in one pass over its weights, and the K lookups
    // are independent, so their LDS round trips overlap
    uint32_t ex[K];
    if (a.use_net) route<K>(v.w1, a.E, w.dst, ex);
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const bool valid = w.p0 + s < n;
        bool miss = false;
        jj[s] = locate(v.B, a.M, v.w2, v.meta, a.use_net,
                                      a.use_net ? ex[s] : 0u, w.dst[s], &miss);
        if (a.miss) {
            const uint64_t mm = ballot(valid && miss);
            if (lane == 0 && mm) atomicAdd(a.miss, (unsigned long long)__popcll(mm));
        }
        si[s] = a.bs_bits ? bucket_walk(v.bs_bucket, v.Bs, a.Ms, a.bs_bits, a.bs_steps, w.src[s])
                          : search_le(v.Bs, 0, a.Ms - 1u, w.src[s]);
        lbest[s] = kNoMatch;
        lact[s] = dflt;
    }
    // the port/protocol table of the first address-wildcard candidates
    if (a.pt_count) {
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const uint32_t e = port_table_first(*v.pt, a.pt_steps_s, a.pt_steps_d, w.pp[s],
                                                w.pr[s]);
            if (e != kPtNone) {
                lbest[s] = e & 0xFFFFFFu;
                lact[s] = e >> 24;
            }
        }
    }
    // The per-lane lists: the destination-interval list, and the source-
    // interval list of the destination-wildcard candidates with a
    // specified source (a packet's source interval lists exactly those
    // whose source test it passes).  Each is ascending and ends at its
    // first match or at the first entry that can no longer beat the best
    // so far, so the answer is the minimum over lists.  All K packets'
    // lists advance together, one entry each per round, so a round's
    // record loads are in flight at once; a wave runs as many rounds as
    // its longest list needs, so the short source lists drop out of the
    // rounds once every lane is done with them.
    // The list cursors are byte offsets of the next record, or kPastEnd
    // (beyond every list end) once the list is done, so the cursor is the
    // load offset itself and the test "entries left" is cursor < end.
    const __amdgpu_buffer_rsrc_t rl = list_rsrc(a.L, a.nL);
    const __amdgpu_buffer_rsrc_t rs_ = list_rsrc(a.S, a.nS);
    constexpr uint32_t kRec = uint32_t(sizeof(RuleRec));
    uint32_t lk[K], le[K], sk[K], se[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {   // plain loads, all issued before the first use
        const uint32_t l0 = v.off[jj[s]], l1 = v.off[jj[s] + 1u];
        const uint32_t s0 = v.soff[si[s]], s1 = v.soff[si[s] + 1u];
        const bool valid = w.p0 + s < n;
        lk[s] = valid && l0 < l1 ? l0 * kRec : kPastEnd;
        le[s] = l1 * kRec;
        sk[s] = valid && s0 < s1 ? s0 * kRec : kPastEnd;
        se[s] = s1 * kRec;
    }
    // One entry of a packet's destination-interval list: the record's
    // source, port and protocol tests (its destination test is implied by
    // the list).  The list advances while its entries still beat the best
    // so far and do not match; otherwise it stops.  Straight-line selects,
    // no branches, so no load is sunk into a conditional block behind
    // another's wait.
    auto step_dst = [&](int s, const RuleRec& q) {
        const bool live = (unsigned(lk[s] < le[s]) & unsigned(q.idx < lbest[s])) != 0u;
        const bool t = (unsigned(in_range(w.src[s], q.src_lo, q.src_w)) &
                        unsigned(ports_in(w.pp[s], q.port_lo, q.port_w)) &
                        unsigned(in_range(w.pr[s], proto_lo(q.proto), proto_w(q.proto)))) != 0u;
        const bool m = live && t;
        lbest[s] = m ? q.idx : lbest[s];
        lact[s] = m ? rule_action(q.proto) : lact[s];
        const uint32_t next = lk[s] + kRec;
        lk[s] = live && !t && next < le[s] ? next : kPastEnd;
    };
    // One entry of its source-interval list (source test implied as well).
    auto step_src = [&](int s, const RuleRec& q) {
        const bool live = (unsigned(sk[s] < se[s]) & unsigned(q.idx < lbest[s])) != 0u;
        const bool t = (unsigned(ports_in(w.pp[s], q.port_lo, q.port_w)) &
                        unsigned(in_range(w.pr[s], proto_lo(q.proto), proto_w(q.proto)))) != 0u;
        const bool m = live && t;
        lbest[s] = m ? q.idx : lbest[s];
        lact[s] = m ? rule_action(q.proto) : lact[s];
        const uint32_t next = sk[s] + kRec;
        sk[s] = live && !t && next < se[s] ? next : kPastEnd;
    };
    // Buffer loads: a finished list loads at kPastEnd, out of the
    // buffer's range, so the load returns zeros without a memory access,
    // and no branch separates the loads.
    // Phase 1, while any lane has a source-interval entry left (those
    // lists are short): both lists of every packet advance each round.
    for (;;) {
        bool more = false;
#pragma unroll
        for (int s = 0; s < K; ++s) more = more || sk[s] < se[s];
        if (ballot(more) == 0) break;
        RuleRec ql[K], qs[K];
#pragma unroll
        for (int s = 0; s < K; ++s) {
            ql[s] = list_record(rl, lk[s]);
            qs[s] = list_record_tail(rs_, sk[s]);
        }
#pragma unroll
        for (int s = 0; s < K; ++s) {
            step_dst(s, ql[s]);
            step_src(s, qs[s]);
        }
    }
    // Phase 2: the rest of the destination-interval lists alone, at half
    // the cost per round.
    for (;;) {
        bool more = false;
#pragma unroll
        for (int s = 0; s < K; ++s) more = more || lk[s] < le[s];
        if (ballot(more) == 0) break;
        RuleRec ql[K];
#pragma unroll
        for (int s = 0; s < K; ++s) ql[s] = list_record(rl, lk[s]);
#pragma unroll
        for (int s = 0; s < K; ++s) step_dst(s, ql[s]);
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
        w.best[s] = lbest[s];
        w.act[s] = lact[s];
    }
    if constexpr (PLAN)
        w.template scan_plan<false>(a.G);   // both addresses unspecified in every rule
    else
        w.seed_tail(a.G);
    w.store(out_idx, out_act, n);
}

}  // namespace fw
