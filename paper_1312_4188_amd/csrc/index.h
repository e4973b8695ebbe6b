// Learned destination index: internal declarations.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fw.h"
#include "fw_internal.h"

namespace fw {

fw_status fail(fw_status st, const char* fmt, ...);
fw_status hip_fail(hipError_t e, const char* what);

struct LearnedIndex;

fw_status build_index(const fw_rule* rules, const RuleRec* recs, uint32_t n_rules,
                      const fw_index_opts& opts, fw_index_stats* stats, LearnedIndex** out);
void destroy_index(LearnedIndex* ix);
fw_status classify_learned(const LearnedIndex* ix, uint8_t default_action, PacketsDev pk,
                           size_t n, int32_t* out_idx, uint8_t* out_act, uint32_t lookup,
                           uint32_t packets_per_lane, hipStream_t stream,
                           uint64_t* window_misses);
fw_status index_lookup(const LearnedIndex* ix, const uint32_t* keys, size_t n,
                       int32_t* out_interval, uint32_t lookup, hipStream_t stream);
fw_status index_export(const LearnedIndex* ix, uint32_t what, void* host, size_t cap,
                       size_t* size);

}  // namespace fw

namespace fw {

// Per-expert data of the second stage (32 bytes).
struct ExpertMeta {
    uint32_t key_lo;    // smallest training key routed to the expert
    float inv_span;     // 1 / (largest key - key_lo + 1)
    int32_t pos_lo;     // smallest / largest target position of its keys
    int32_t pos_hi;
    float pos_span;     // pos_hi - pos_lo
    uint32_t err;       // max |predicted - true position| over its keys
    uint32_t pad[2];
};
static_assert(sizeof(ExpertMeta) == 32, "expert record must stay 32 bytes");

constexpr uint32_t kMaxHidden = 32;
constexpr uint32_t kMaxExperts = 256;
constexpr uint32_t kGradCols = 128;      // padded column count of the gradient product
constexpr uint32_t kNoExpert = 0xFFFFFFFFu;
// Inference layout of one stage-1 network (fp32): [w1][b1][w2][b2] in
// 32-slot segments, padded to 104 entries (a multiple of 8); hidden units past
// H are zero.  A stage-2 row (kRowDwords dwords) holds one expert: dword k
// pairs w1[k] (its bf16 value as IEEE half, low half) with b1[k] (the whole
// dword read as fp32, its high half b1's bf16 pattern or the one next to it);
// dwords 32..47 hold w2 as IEEE half, two units each (unit 2i in the low
// half); dword 48 holds b2 as fp32 (its bf16 value widened, exact); dwords
// 49..51 carry the expert's input scaling (key_lo, inv_span) and pos_span,
// read with the bias in one 16-byte load.  The lookup's mixed-precision
// multiply-adds read the half weights where they lie, so each hidden unit
// costs two instructions and the row 13 16-byte LDS reads.  A bf16 value
// converts to half exactly from 2^-14 up (half's normal range); the index
// build counts any weight outside it (fw_index_stats.weights_rounded).
constexpr uint32_t kInferStride = 104;
constexpr uint32_t kRowPairs = 0;     // pair dword of hidden unit 0 in a stage-2 row
constexpr uint32_t kRowOut = 32;      // dword of w2[0] (low half) and w2[1] (high half)
constexpr uint32_t kRowBias = 48;     // dword of b2
constexpr uint32_t kRowKeyLo = 49;    // ExpertMeta::key_lo
constexpr uint32_t kRowInvSpan = 50;  // ExpertMeta::inv_span
constexpr uint32_t kRowPosSpan = 51;  // ExpertMeta::pos_span
constexpr uint32_t kRowDwords = 52;   // stage-2 row stride (a 16-byte multiple)


// The per-lane lists are read with 32-bit buffer offsets: each list array is
// kept below kMaxListBytes, and kListPastEnd (above it) marks a lane with
// nothing to load.
constexpr uint64_t kMaxListBytes = 0x7FFF0000ull;
constexpr uint32_t kListPastEnd = 0x7FFFFFF0u;
static_assert(kListPastEnd > kMaxListBytes + 32, "past-the-end offset must be out of range");

// What the lookup reads of an expert record besides its row: position
// offset and error bound, one 8-byte load.
struct LdsExpert {
    int32_t pos_lo;
    uint32_t err;
};

// LDS stride of the expert rows, chosen so that lanes reading different
// experts spread over all LDS banks: a row of 52 dwords puts expert e at
// bank offset 52 e, which takes 8 values modulo 32 banks and 16 modulo 64
// (each 16-byte read covering 4 banks); the 8-byte records take 32.
static_assert(kRowDwords % 4 == 0 && kRowPosSpan < kRowDwords, "stage-2 row layout");

// Byte offsets of the lookup kernel's LDS image, every section 16-byte
// aligned: stage-1 weights (kInferStride fp32), expert records (LdsExpert
// each), expert rows (kRowDwords each), the
// port/protocol table, the source bucket table, and, with the boundary arrays
// in LDS (b_lds), B, Bs, off and soff.  The index build writes this image
// once per variant; the kernel copies it whole.
struct LdsLayout {
    size_t w1 = 0, meta, w2, pt, bk, b, bs, off, soff, bytes;
    __host__ __device__ static size_t up16(size_t x) { return (x + 15) & ~size_t(15); }
    __host__ __device__ LdsLayout(uint32_t E, uint32_t M, uint32_t Ms, uint32_t bs_bits,
                                  bool b_lds) {
        size_t o = up16(kInferStride * sizeof(float));
        meta = o;
        o = up16(o + size_t(E) * sizeof(LdsExpert));
        w2 = o;
        o = up16(o + size_t(E) * kRowDwords * sizeof(uint32_t));
        pt = o;
        o = up16(o + sizeof(PortTable));
        bk = o;
        o = up16(o + (bs_bits ? (size_t(2) << bs_bits) : 0));
        b = bs = off = soff = o;
        if (b_lds) {
            o = up16(o + size_t(M) * 4);
            bs = o;
            o = up16(o + size_t(Ms) * 4);
            off = o;
            o = up16(o + (size_t(M) + 1) * 4);
            soff = o;
            o = up16(o + (size_t(Ms) + 1) * 4);
        }
        bytes = o;
    }
};

// Everything the lookup kernel reads.
struct LookupArgs {
    const uint32_t* B;        // M boundaries
    uint32_t M;
    const float* w1;          // stage 1 in the inference layout (bf16 values, widened)
    const uint32_t* w2;       // stage-2 rows, E x kRowDwords
    const ExpertMeta* meta;   // E
    uint32_t E;
    const uint32_t* off;      // M + 1 per-interval list offsets
    const RuleRec* L;         // per-interval candidate records
    uint32_t nL;              // records in L
    const PortTable* pt;      // the first address-wildcard candidates (see PortTable)
    uint32_t pt_count;        // rules in the table (0: none)
    uint32_t pt_steps_s;      // forward steps after the high-byte table, per port field
    uint32_t pt_steps_d;
    ScanPlan G;               // the remaining address-wildcard candidates (grouped plan)
    const uint32_t* Bs;       // source intervals of the other destination-wildcard candidates
    uint32_t Ms;
    const uint16_t* bs_bucket; // interval holding the first address of each top-bits bucket
    uint32_t bs_bits;         // bucket bits (0: binary search over Bs instead)
    uint32_t bs_steps;        // forward steps after the bucket table
    const uint32_t* soff;     // Ms + 1 per-source-interval list offsets
    const RuleRec* S;         // per-source-interval candidate records
    uint32_t nS;              // records in S
    const uint4* image[2];    // LDS image per placement [boundaries in LDS]
    uint32_t use_net;         // 0: full binary search only
    unsigned long long* miss; // optional window-miss counter
};

// What the multi-chain kernels read of one ruleset: one per ruleset in device
// memory, written at load and rewritten when the learned index is built.
struct ChainView {
    const RuleRec* rules;   // the compiled list in rule order
    const uint2* pairs;     // destination (lo, w) per rule, padded by kPairPadding
    uint32_t n_rules;
    uint32_t dflt;          // default action
    uint32_t has_index;     // `la` describes a built learned index
    uint32_t lds_b;         // bytes of its LDS image with the boundary arrays (image[1])
    uint32_t lds_nob;       // bytes of its LDS image without them (image[0])
    uint32_t pad;
    ScanPlan plan;          // grouped scan plan (packet split)
    LookupArgs la;          // the learned lookup: network + error window, no miss counting
};

// The learned part of a ruleset's ChainView.
void index_chain_view(const LearnedIndex* ix, ChainView* v);

// ---- training kernels (rmi.hip)
hipError_t launch_fwd_bwd(const float* params, uint32_t H, const float* u, const float* t,
                          const uint32_t* ex, const float* inv_count, size_t n, size_t n_pad,
                          void* at, bool bf16, hipStream_t s);
hipError_t launch_grad_mfma(const uint16_t* at, const uint32_t* ex, size_t n_pad, uint32_t E,
                            float* partial, hipStream_t s);
uint32_t grad_mfma_chunks(size_t n_pad);
hipError_t launch_grad_reduce(const float* partial, uint32_t chunks, uint32_t E, uint32_t H,
                              float* grad, float* loss, hipStream_t s);
hipError_t launch_grad_fp32(const float* at, size_t n_pad, const uint32_t* seg, uint32_t E,
                            uint32_t H, float* grad, float* loss, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, size_t count, float lr,
                       float b1, float b2, float eps, float bc1, float bc2, hipStream_t s);
hipError_t launch_route(const float* w1, uint32_t E, const uint32_t* keys, size_t n,
                        uint32_t* expert, hipStream_t s);
hipError_t launch_err_bound(const LookupArgs& a, const uint32_t* keys, const int32_t* pos,
                            size_t n, uint32_t* err, hipStream_t s);
hipError_t launch_learned(const LookupArgs& a, PacketsDev pk, size_t n, int32_t* out_idx,
                          uint8_t* out_act, uint32_t dflt, const uint32_t* keys,
                          int32_t* out_interval, uint32_t packets_per_lane, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
size_t learned_lds_bytes(const LookupArgs& a, bool b_in_lds);

}  // namespace fw
