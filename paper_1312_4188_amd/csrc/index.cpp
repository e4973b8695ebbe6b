// Learned destination index: host-side build, GPU training driver, lookup and
// export entry points.
//
// Intervals: B = {0} with every rule's destination range start and every
// range end + 1 below 2^32, sorted and de-duplicated; interval j is
// [B[j], B[j+1]).  Every destination range is a union of whole intervals, so
// the rules whose destination covers interval j (its candidate list C_j, in
// rule order) are exactly the rules whose destination test a packet in j
// passes, and the first match over C_j is the first match overall.
//
// Storage splits C_j in two: the destination-wildcard rules, which belong to
// every C_j, form one shared list G; the rest form a per-interval list L_j.
// Both are cut short where no later entry can be a first match: G after its
// first rule that matches every packet (all five fields unspecified), L_j
// after its first rule that matches every packet of the interval (source,
// ports and protocol unspecified) and before any index past G's cut.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "index.h"
#include "lists.h"
#include "guard.h"

namespace fw {

struct LearnedIndex {
    uint32_t M = 0, E = 0, H = 0;
    uint32_t nG = 0;
    uint64_t nL = 0;
    uint32_t* d_B = nullptr;
    uint32_t* d_off = nullptr;
    RuleRec* d_L = nullptr;
    DevicePlan gplan;             // source-and-destination-wildcard candidates, grouped plan
    uint32_t Ms = 0;              // source intervals of the destination-wildcard candidates
    uint64_t nS = 0;
    uint32_t* d_Bs = nullptr;
    uint32_t* d_soff = nullptr;
    RuleRec* d_S = nullptr;
    std::vector<uint32_t> Bs, soff, S_idx, Gw_idx;
    PortTable pt{};               // the first address-wildcard candidates (host copy)
    // rules in the port table, its walk steps per port field; source bucket bits and steps
    uint32_t pt_shape[5] = {0, 0, 0, 0, 0};
    std::vector<uint16_t> bs_bucket;
    uint16_t* d_bs_bucket = nullptr;
    uint4* d_image[2] = {nullptr, nullptr};   // LDS images, see LdsLayout
    PortTable* d_pt = nullptr;
    float* d_w1 = nullptr;
    uint32_t* d_w2 = nullptr;
    ExpertMeta* d_meta = nullptr;
    std::vector<uint32_t> B, off, L_idx, G_idx, err;
    std::vector<float> weights;   // stage 1 then experts, bf16 values widened to float
    uint32_t weights_rounded = 0; // stage-2 weights IEEE half does not hold exactly
    uint64_t device_bytes = 0;
};

namespace {

// ---- small helpers

template <class T>
hipError_t dalloc(T** p, size_t count, uint64_t* total) {
    const size_t bytes = sizeof(T) * (count ? count : 1);
    *total += bytes;
    return hipMalloc(reinterpret_cast<void**>(p), bytes);
}

template <class T>
hipError_t upload(T* d, const std::vector<T>& h, hipStream_t s) {
    if (h.empty()) return hipSuccess;
    return hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s);
}

uint16_t to_bf16(float f) {  // round to nearest even; inputs are finite
    uint32_t b;
    std::memcpy(&b, &f, 4);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return uint16_t(b >> 16);
}

float from_bf16(uint16_t h) {
    const uint32_t b = uint32_t(h) << 16;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

// IEEE binary16 bits of f, rounded to nearest even.  A bf16 value (8
// significant bits) converts exactly when its magnitude is 0 or at least
// 2^-14, the smallest normal half; below that it is rounded to a multiple of
// 2^-24.
uint16_t to_f16(float f) {
    const _Float16 h = static_cast<_Float16>(f);
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}

float from_f16(uint16_t u) {
    _Float16 h;
    std::memcpy(&h, &u, 2);
    return static_cast<float>(h);
}

// splitmix64: a counter-based generator for the seeded weight initialisation.
struct SplitMix {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return double(next() >> 11) * 0x1.0p-53; }
    double normal() {
        const double u1 = uniform() + 1e-300, u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

// One 1 -> H -> 1 network on inputs in [0, 1]: ramps w1 * (u - c) with knots c
// spread over [0, 1], small random output weights.
void init_network(float* p, uint32_t H, SplitMix& rng) {
    for (uint32_t k = 0; k < H; ++k) {
        const double knot = (k + rng.uniform()) / H;
        const double slope = 1.0 + 0.1 * rng.normal();
        p[k] = float(slope);
        p[H + k] = float(-slope * knot);
        p[2 * H + k] = float(rng.normal() / std::sqrt(double(H)));
    }
    p[3 * H] = 0.0f;
}

// Fold each hidden unit's ReLU into a clamp to [0, 1].  Unit (w1, b1, w2)
// on inputs v in [0, 1] has pre-activation z = w1 v + b1 <= |w1| + |b1| < 2^k
// for every k from the one below up; scaling w1 and b1 by 2^-k and w2 by 2^k
// leaves w2 max(z, 0) unchanged, and since scaling by a power of two is exact
// in floating point (bf16 and fp32 share the exponent range), the fp32
// products and sums the lookup forms are bit for bit those of the unscaled
// unit; the scaled pre-activation is at most 1, so max(z, 0) equals
// clamp(z, 0, 1), which the hardware applies to the multiply-add for free.
// Among the first 24 such k, the smallest that `cost(w1', w2')` rates lowest
// is taken (the stage-2 rows store w1' and w2' as IEEE half, which holds only
// part of the fp32 range exactly).  A unit whose scaled values would not
// round-trip (far outside any trained range) is left as it is; the error
// bounds are measured with the lookup's own arithmetic either way.
// `row` is one network in 32-slot segments [w1][b1][w2].
template <class Get, class Put, class Cost>
void fold_relu(Get get, Put put, Cost cost) {
    for (uint32_t i = 0; i < 32; ++i) {
        const float a = get(i), b = get(32 + i), c = get(64 + i);
        const float m = std::fabs(a) + std::fabs(b);
        if (!(m > 0.0f) || !std::isfinite(m)) continue;
        int k0 = 0;
        std::frexp(m, &k0);                   // m < 2^k0
        int best = 0;
        uint32_t best_cost = ~0u;
        for (int k = k0; k < k0 + 24; ++k) {
            const float a2 = std::ldexp(a, -k), b2 = std::ldexp(b, -k), c2 = std::ldexp(c, k);
            const bool exact = std::ldexp(a2, k) == a && std::ldexp(b2, k) == b &&
                               std::ldexp(c2, -k) == c && std::isfinite(c2) &&
                               (a2 == 0.0f || std::isnormal(a2)) &&
                               (b2 == 0.0f || std::isnormal(b2)) &&
                               (c2 == 0.0f || std::isnormal(c2));
            if (!exact) continue;
            const uint32_t q = cost(a2, c2);
            if (q < best_cost) {
                best_cost = q;
                best = k;
            }
            if (q == 0) break;
        }
        if (best_cost == ~0u) continue;
        put(i, std::ldexp(a, -best));
        put(32 + i, std::ldexp(b, -best));
        put(64 + i, std::ldexp(c, best));
    }
}

// Whether IEEE half holds f exactly.
bool half_exact(float f) { return from_f16(to_f16(f)) == f; }

// Stage-2 weights of a unit that half would round: w2, and w1 unless w2 is
// zero (the unit then adds exactly nothing, whatever w1 is).
uint32_t half_rounding(float w1, float w2) {
    return uint32_t(!half_exact(w2)) + uint32_t(w2 != 0.0f && !half_exact(w1));
}

// Slot of parameter k of the training layout [w1 (H), b1 (H), w2 (H), b2] in
// the inference layout of 32-slot segments.
uint32_t infer_slot(uint32_t k, uint32_t H) {
    return k < 3 * H ? (k / H) * 32u + k % H : 96u;
}

// Device buffers of one training run (one stage).
struct Trainer {
    uint32_t E = 0, H = 0, P = 0;
    size_t n = 0, n_pad = 0;
    bool mfma = true;
    float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
    float *u = nullptr, *t = nullptr, *inv = nullptr, *partial = nullptr;
    uint32_t *ex = nullptr, *seg = nullptr;
    void* at = nullptr;
    uint64_t bytes = 0;

    hipError_t init(uint32_t E_, uint32_t H_, size_t n_, bool mfma_, hipStream_t s) {
        E = E_;
        H = H_;
        P = 3 * H + 1;
        n = n_;
        mfma = mfma_;
        n_pad = ((n + 511) / 512) * 512;
        if (n_pad == 0) n_pad = 512;
        const uint32_t E_pad = (E + 31u) & ~31u;
        hipError_t e;
        if ((e = dalloc(&params, size_t(E) * P, &bytes)) != hipSuccess) return e;
        if ((e = dalloc(&m, size_t(E) * P, &bytes)) != hipSuccess) return e;
        if ((e = dalloc(&v, size_t(E) * P, &bytes)) != hipSuccess) return e;
        if ((e = dalloc(&grad, size_t(E) * P, &bytes)) != hipSuccess) return e;
        if ((e = dalloc(&loss, E, &bytes)) != hipSuccess) return e;
        if ((e = dalloc(&u, n_pad, &bytes)) != hipSuccess) return e;
        if ((e = dalloc(&t, n_pad, &bytes)) != hipSuccess) return e;
        if ((e = dalloc(&inv, E, &bytes)) != hipSuccess) return e;
        if ((e = dalloc(&ex, n_pad, &bytes)) != hipSuccess) return e;
        if ((e = dalloc(&seg, size_t(E) + 1, &bytes)) != hipSuccess) return e;
        const size_t at_words = mfma ? size_t(kGradCols) * n_pad / 2 : size_t(kGradCols) * n_pad;
        uint32_t* atw = nullptr;
        if ((e = dalloc(&atw, at_words, &bytes)) != hipSuccess) return e;
        at = atw;
        if (mfma &&
            (e = dalloc(&partial, size_t(n_pad / 512) * E_pad * kGradCols, &bytes)) != hipSuccess)
            return e;
        // unused columns of the sample matrix and padded samples stay zero / no expert
        if ((e = launch_fill_u32(atw, at_words, 0u, s)) != hipSuccess) return e;
        if ((e = launch_fill_u32(ex, n_pad, kNoExpert, s)) != hipSuccess) return e;
        if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(m), size_t(E) * P, 0u, s)) != hipSuccess)
            return e;
        return launch_fill_u32(reinterpret_cast<uint32_t*>(v), size_t(E) * P, 0u, s);
    }

    // Samples must be sorted by network; counts give the per-network sizes.
    hipError_t load(const std::vector<float>& hu, const std::vector<float>& ht,
                    const std::vector<uint32_t>& hex, const std::vector<float>& hparams,
                    hipStream_t s) {
        std::vector<uint32_t> counts(E, 0);
        for (uint32_t e : hex) ++counts[e];
        std::vector<float> hinv(E);
        std::vector<uint32_t> hseg(E + 1, 0);
        for (uint32_t e = 0; e < E; ++e) {
            hinv[e] = counts[e] ? 1.0f / float(counts[e]) : 0.0f;
            hseg[e + 1] = hseg[e] + counts[e];
        }
        hipError_t e;
        if ((e = upload(u, hu, s)) != hipSuccess) return e;
        if ((e = upload(t, ht, s)) != hipSuccess) return e;
        if ((e = upload(ex, hex, s)) != hipSuccess) return e;
        if ((e = upload(inv, hinv, s)) != hipSuccess) return e;
        if ((e = upload(seg, hseg, s)) != hipSuccess) return e;
        if ((e = upload(params, hparams, s)) != hipSuccess) return e;
        return hipStreamSynchronize(s);   // host vectors are temporaries of the caller
    }

    hipError_t gradients(hipStream_t s) {
        hipError_t e = launch_fwd_bwd(params, H, u, t, ex, inv, n, n_pad, at, mfma, s);
        if (e != hipSuccess) return e;
        if (mfma) {
            e = launch_grad_mfma(static_cast<const uint16_t*>(at), ex, n_pad, E, partial, s);
            if (e != hipSuccess) return e;
            return launch_grad_reduce(partial, grad_mfma_chunks(n_pad), E, H, grad, loss, s);
        }
        return launch_grad_fp32(static_cast<const float*>(at), n_pad, seg, E, H, grad, loss, s);
    }

    hipError_t train(uint32_t steps, float lr0, hipStream_t s) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        for (uint32_t k = 1; k <= steps; ++k) {
            hipError_t e = gradients(s);
            if (e != hipSuccess) return e;
            // linear decay to a tenth of the initial rate
            const float lr = lr0 * (1.0f - 0.9f * float(k - 1) / float(steps));
            const float bc1 = float(1.0 - std::pow(0.9, double(k)));
            const float bc2 = float(1.0 - std::pow(0.999, double(k)));
            e = launch_adam(params, grad, m, v, size_t(E) * P, lr, b1, b2, eps, bc1, bc2, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }

    void release() {
        for (void* p : {static_cast<void*>(params), static_cast<void*>(m), static_cast<void*>(v),
                        static_cast<void*>(grad), static_cast<void*>(loss), static_cast<void*>(u),
                        static_cast<void*>(t), static_cast<void*>(inv), static_cast<void*>(ex),
                        static_cast<void*>(seg), at, static_cast<void*>(partial)})
            if (p) (void)hipFree(p);
        *this = Trainer{};
    }
};

void free_index_memory(LearnedIndex* ix) {
    free_plan(&ix->gplan);
    for (void* p : {static_cast<void*>(ix->d_B), static_cast<void*>(ix->d_off),
                    static_cast<void*>(ix->d_L), static_cast<void*>(ix->d_Bs),
                    static_cast<void*>(ix->d_soff), static_cast<void*>(ix->d_S),
                    static_cast<void*>(ix->d_w1), static_cast<void*>(ix->d_w2),
                    static_cast<void*>(ix->d_meta), static_cast<void*>(ix->d_pt), static_cast<void*>(ix->d_bs_bucket),
                    static_cast<void*>(ix->d_image[0]), static_cast<void*>(ix->d_image[1])})
        if (p) (void)hipFree(p);
}

LookupArgs args_of(const LearnedIndex* ix, uint32_t use_net) {
    LookupArgs a{};
    a.B = ix->d_B;
    a.M = ix->M;
    a.w1 = ix->d_w1;
    a.w2 = ix->d_w2;
    a.meta = ix->d_meta;
    a.E = ix->E;
    a.off = ix->d_off;
    a.L = ix->d_L;
    a.nL = uint32_t(ix->nL);
    a.nS = uint32_t(ix->nS);
    a.G = ix->gplan.plan;
    a.pt = ix->d_pt;
    a.pt_count = ix->pt_shape[0];
    a.pt_steps_s = ix->pt_shape[1];
    a.pt_steps_d = ix->pt_shape[2];
    a.bs_bucket = ix->d_bs_bucket;
    for (int b = 0; b < 2; ++b) a.image[b] = ix->d_image[b];
    a.bs_bits = ix->pt_shape[3];
    a.bs_steps = ix->pt_shape[4];
    a.Bs = ix->d_Bs;
    a.Ms = ix->Ms;
    a.soff = ix->d_soff;
    a.S = ix->d_S;
    a.use_net = use_net;
    a.miss = nullptr;
    return a;
}

// The lookup kernel's LDS image for one placement (see LdsLayout): w1 and
// w2 are the inference weights (w2 as stage-2 rows), meta holds the final
// error bounds.
std::vector<uint8_t> lds_image(const LearnedIndex* ix, const std::vector<float>& w1q,
                               const std::vector<ExpertMeta>& meta,
                               const std::vector<uint32_t>& w2r, bool b_lds) {
    const uint32_t E = ix->E;
    const LdsLayout L(E, ix->M, ix->Ms, ix->pt_shape[3], b_lds);
    std::vector<uint8_t> img(L.bytes, 0);
    auto put = [&](size_t at, const void* src, size_t bytes) {
        if (bytes) std::memcpy(img.data() + at, src, bytes);
    };
    put(L.w1, w1q.data(), kInferStride * sizeof(float));
    for (uint32_t e = 0; e < E; ++e) {
        const LdsExpert r{meta[e].pos_lo, meta[e].err};
        put(L.meta + size_t(e) * sizeof(LdsExpert), &r, sizeof r);
    }
    put(L.w2, w2r.data(), w2r.size() * 4);
    put(L.pt, &ix->pt, sizeof(PortTable));
    put(L.bk, ix->bs_bucket.data(), ix->bs_bucket.size() * 2);
    if (b_lds) {
        put(L.b, ix->B.data(), ix->B.size() * 4);
        put(L.bs, ix->Bs.data(), ix->Bs.size() * 4);
        put(L.off, ix->off.data(), ix->off.size() * 4);
        put(L.soff, ix->soff.data(), ix->soff.size() * 4);
    }
    return img;
}

// Pair dword of a stage-2 hidden unit: w1 as IEEE half in the low half (the
// lookup's mixed-precision multiply-add reads it there as an fp16 operand; the
// bf16 w1 converts exactly, see to_f16), and a high half chosen so that the
// whole dword read as fp32, which the lookup takes as the unit's bias, is the
// nearest such value to b1.  The low bits add less than one bf16 step to the
// magnitude of the high half's value, so the candidates are b1's own pattern
// and the one a step toward zero; the bias applied is then within half a bf16
// step of b1.
uint32_t pair_dword(uint16_t w1, uint16_t b1) {
    const float want = from_bf16(b1);
    auto as_float = [](uint32_t u) {
        float f;
        std::memcpy(&f, &u, 4);
        return f;
    };
    uint32_t best = (uint32_t(b1) << 16) | w1;
    if ((b1 & 0x7FFFu) != 0) {   // a step toward zero exists (b1 is not a zero)
        const uint32_t alt = (uint32_t(b1 - 1u) << 16) | w1;
        if (std::fabs(as_float(alt) - want) < std::fabs(as_float(best) - want)) best = alt;
    }
    return best;
}

// Stage-2 rows (see kRowDwords) from bf16 networks in 32-slot segments
// [w1][b1][w2][b2]: dword k = pair_dword(half w1[k], b1[k]); w2 as IEEE half,
// two units to a dword (even unit in the low half); b2 widened to fp32 (a bf16
// value is the top half of its fp32 pattern); the expert's key_lo, inv_span
// and pos_span beside the bias.  *rounded counts the weights half does not
// hold exactly (see half_rounding).
std::vector<uint32_t> stage2_rows(const std::vector<uint16_t>& seg, uint32_t E,
                                  const std::vector<ExpertMeta>& meta, uint32_t* rounded) {
    std::vector<uint32_t> out(size_t(E) * kRowDwords, 0);
    *rounded = 0;
    auto half = [](uint16_t bf) { return uint32_t(to_f16(from_bf16(bf))); };
    for (uint32_t e = 0; e < E; ++e) {
        const uint16_t* r = seg.data() + size_t(e) * kInferStride;
        uint32_t* o = out.data() + size_t(e) * kRowDwords;
        for (uint32_t k = 0; k < 32; ++k) {
            o[kRowPairs + k] = pair_dword(uint16_t(half(r[k])), r[32 + k]);
            *rounded += half_rounding(from_bf16(r[k]), from_bf16(r[64 + k]));
        }
        for (uint32_t k = 0; k < 16; ++k)
            o[kRowOut + k] = half(r[64 + 2 * k]) | (half(r[64 + 2 * k + 1]) << 16);
        o[kRowBias] = uint32_t(r[96]) << 16;
        o[kRowKeyLo] = meta[e].key_lo;
        std::memcpy(&o[kRowInvSpan], &meta[e].inv_span, 4);
        std::memcpy(&o[kRowPosSpan], &meta[e].pos_span, 4);
    }
    return out;
}

}  // namespace

void destroy_index(LearnedIndex* ix) {
    if (!ix) return;
    free_index_memory(ix);
    delete ix;
}

fw_status build_index(const fw_rule* rules, const RuleRec* recs, uint32_t n_rules,
                      const fw_index_opts& opts_in, fw_index_stats* stats, LearnedIndex** out) {
    (void)rules;
    *out = nullptr;
    fw_index_opts o = opts_in;
    if (o.experts == 0) o.experts = 64;
    if (o.hidden == 0) o.hidden = 32;
    if (o.epochs1 == 0) o.epochs1 = 1500;
    if (o.epochs2 == 0) o.epochs2 = 3000;
    if (o.lr == 0.0f) o.lr = 1e-2f;
    if (o.experts > kMaxExperts) return fail(FW_E_INVAL, "at most %u experts", kMaxExperts);
    if (o.hidden > kMaxHidden) return fail(FW_E_INVAL, "at most %u hidden units", kMaxHidden);
    if (!(o.lr > 0.0f) || !std::isfinite(o.lr)) return fail(FW_E_INVAL, "bad learning rate");
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    const auto t_start = std::chrono::steady_clock::now();

    LearnedIndex* ix = new LearnedIndex();
    // until the index is complete, any return or exception frees what it holds
    ScopeExit drop_ix([&] { destroy_index(ix); });
    std::vector<RuleRec> L, S, G;
    fw_status st = FW_OK;
    try {
        HostLists hl;
        if (!build_lists(recs, n_rules, &hl)) {
            st = fail(FW_E_NOMEM, "candidate lists exceed 2^32 entries");
        } else {
            ix->B = std::move(hl.B);
            ix->off = std::move(hl.off);
            ix->L_idx = std::move(hl.L_idx);
            ix->G_idx = std::move(hl.G_idx);
            ix->Bs = std::move(hl.Bs);
            ix->soff = std::move(hl.soff);
            ix->S_idx = std::move(hl.S_idx);
            ix->Gw_idx = std::move(hl.Gw_idx);
            L = std::move(hl.L);
            S = std::move(hl.S);
            ix->M = uint32_t(ix->B.size());
            ix->Ms = uint32_t(ix->Bs.size());
            ix->nL = ix->L_idx.size();
            ix->nS = ix->S_idx.size();
            ix->nG = uint32_t(ix->G_idx.size());
            build_port_table(hl.Gw, &ix->pt, &ix->pt_shape[0], &ix->pt_shape[1], &ix->pt_shape[2],
                             &G);
            build_bucket_table(ix->Bs, &ix->bs_bucket, &ix->pt_shape[3], &ix->pt_shape[4]);
        }
    } catch (const std::bad_alloc&) {
        st = fail(FW_E_NOMEM, "host allocation failed while building candidate lists");
    }
    if (st != FW_OK) return st;
    if (ix->nL * sizeof(RuleRec) > kMaxListBytes || ix->nS * sizeof(RuleRec) > kMaxListBytes)
        return fail(FW_E_NOMEM, "candidate lists exceed %llu bytes",
                    (unsigned long long)kMaxListBytes);
    const uint32_t M = ix->M, E = o.experts, H = o.hidden, P = 3 * H + 1;
    ix->E = E;
    ix->H = H;

    // device footprint of what the index keeps
    const uint64_t keep = uint64_t(M) * 4 + (uint64_t(M) + 1) * 4 + ix->nL * sizeof(RuleRec) +
                          uint64_t(ix->Ms) * 8 + 4 + ix->nS * sizeof(RuleRec) +
                          uint64_t(ix->nG ? ix->nG : 1) * sizeof(RuleRec) +
                          (uint64_t(ix->nG) + kPairPadding) * 8 + kGradCols * 4 +
                          uint64_t(E) * kRowDwords * 4 + uint64_t(E) * sizeof(ExpertMeta) + 8 +
                          sizeof(PortTable) + (uint64_t(1) << 12) * 2 +
                          LdsLayout(E, M, ix->Ms, ix->pt_shape[3], false).bytes +
                          LdsLayout(E, M, ix->Ms, ix->pt_shape[3], true).bytes;
    if (o.mem_budget && keep > o.mem_budget)
        return fail(FW_E_NOMEM, "learned index needs %llu bytes, budget is %llu",
                    (unsigned long long)keep, (unsigned long long)o.mem_budget);

    hipError_t e = hipSuccess;
    uint64_t bytes = 0;
    auto bail = [&](hipError_t err, const char* what) { return hip_fail(err, what); };
    if ((e = dalloc(&ix->d_B, M, &bytes)) != hipSuccess ||
        (e = dalloc(&ix->d_off, size_t(M) + 1, &bytes)) != hipSuccess ||
        (e = dalloc(&ix->d_L, ix->nL, &bytes)) != hipSuccess ||
        (e = dalloc(&ix->d_Bs, ix->Ms, &bytes)) != hipSuccess ||
        (e = dalloc(&ix->d_soff, size_t(ix->Ms) + 1, &bytes)) != hipSuccess ||
        (e = dalloc(&ix->d_S, ix->nS, &bytes)) != hipSuccess ||

        (e = dalloc(&ix->d_w1, kGradCols, &bytes)) != hipSuccess ||
        (e = dalloc(&ix->d_w2, size_t(E) * kRowDwords, &bytes)) != hipSuccess ||
        (e = dalloc(&ix->d_meta, E, &bytes)) != hipSuccess ||
        (e = dalloc(&ix->d_pt, 1, &bytes)) != hipSuccess ||
        (e = dalloc(&ix->d_bs_bucket, ix->bs_bucket.size(), &bytes)) != hipSuccess)
        return bail(e, "allocating the learned index");
    ix->device_bytes = bytes;
    if ((e = upload(ix->d_B, ix->B, s)) != hipSuccess ||
        (e = upload(ix->d_off, ix->off, s)) != hipSuccess ||
        (e = upload(ix->d_L, L, s)) != hipSuccess || (e = upload(ix->d_Bs, ix->Bs, s)) != hipSuccess ||
        (e = upload(ix->d_soff, ix->soff, s)) != hipSuccess ||
        (e = upload(ix->d_S, S, s)) != hipSuccess ||
        (e = upload(ix->d_bs_bucket, ix->bs_bucket, s)) != hipSuccess ||
        (e = hipMemcpyAsync(ix->d_pt, &ix->pt, sizeof(PortTable), hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess ||
        (e = make_plan(G.data(), uint32_t(G.size()), &ix->gplan)) != hipSuccess)
        return bail(e, "uploading the learned index");
    ix->device_bytes += ix->gplan.bytes;
    // the lookup scans this plan without address tests (its rules leave both
    // addresses unspecified, so it has port- and protocol-first groups only)
    for (uint32_t g = 0; g < ix->gplan.plan.n_groups; ++g)
        if (ix->gplan.plan.g[g].kind == kFirstDst || ix->gplan.plan.g[g].kind == kFirstSrc)
            return bail(hipErrorInvalidValue, "an address-first group in the wildcard plan");

    // ---- training samples: both ends of every interval, target = its position
    std::vector<uint32_t> keys;
    std::vector<int32_t> pos;
    keys.reserve(size_t(M) * 2);
    pos.reserve(size_t(M) * 2);
    for (uint32_t j = 0; j < M; ++j) {
        const uint32_t end = j + 1 < M ? ix->B[j + 1] - 1u : 0xFFFFFFFFu;
        keys.push_back(ix->B[j]);
        pos.push_back(int32_t(j));
        if (end != ix->B[j]) {
            keys.push_back(end);
            pos.push_back(int32_t(j));
        }
    }
    const size_t N = keys.size();
    uint32_t* d_keys = nullptr;
    int32_t* d_pos = nullptr;
    uint32_t* d_route = nullptr;
    uint32_t* d_err = nullptr;
    uint64_t scratch = 0;
    auto free_scratch = [&]() {
        for (void* p : {static_cast<void*>(d_keys), static_cast<void*>(d_pos),
                        static_cast<void*>(d_route), static_cast<void*>(d_err)})
            if (p) (void)hipFree(p);
        d_keys = nullptr;
        d_pos = nullptr;
        d_route = nullptr;
        d_err = nullptr;
    };
    ScopeExit drop_scratch([&] { free_scratch(); });   // freed early below on success
    if ((e = dalloc(&d_keys, N, &scratch)) != hipSuccess ||
        (e = dalloc(&d_pos, N, &scratch)) != hipSuccess ||
        (e = dalloc(&d_route, N, &scratch)) != hipSuccess ||
        (e = dalloc(&d_err, E, &scratch)) != hipSuccess)
        return bail(e, "allocating training buffers");
    auto fail_train = bail;
    if ((e = upload(d_keys, keys, s)) != hipSuccess || (e = upload(d_pos, pos, s)) != hipSuccess)
        return fail_train(e, "uploading training keys");

    SplitMix rng{0x5EEDull * 0x100000001B3ull ^ o.seed};
    float loss1 = 0.0f, loss2 = 0.0f;

    // ---- stage 1: one network, u = key / 2^32, target position / M
    std::vector<float> w1(P);
    init_network(w1.data(), H, rng);
    {
        Trainer tr;
        ScopeExit tr_release([&] { tr.release(); });
        if ((e = tr.init(1, H, N, o.use_mfma != 0, s)) != hipSuccess)
            return fail_train(e, "allocating stage-1 training");
        std::vector<float> hu(N), ht(N);
        std::vector<uint32_t> hex(N, 0);
        for (size_t k = 0; k < N; ++k) {
            hu[k] = float(keys[k]) * 0x1p-32f;
            ht[k] = float(pos[k]) / float(M);
        }
        e = tr.load(hu, ht, hex, w1, s);
        if (e == hipSuccess && o.train) e = tr.train(o.epochs1, o.lr, s);
        if (e == hipSuccess && o.train) e = tr.gradients(s);   // loss at the final weights
        if (e == hipSuccess)
            e = hipMemcpyAsync(w1.data(), tr.params, sizeof(float) * P, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && o.train)
            e = hipMemcpyAsync(&loss1, tr.loss, sizeof(float), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        tr.release();
        if (e != hipSuccess) return fail_train(e, "training stage 1");
    }
    // quantise to bf16; the lookup uses the widened bf16 values
    std::vector<float> w1q(kGradCols, 0.0f);   // inference layout, see kInferStride
    for (uint32_t k = 0; k < P; ++k) w1q[infer_slot(k, H)] = from_bf16(to_bf16(w1[k]));
    std::vector<float> w1_trained(w1q);        // exported as trained; the lookup gets the fold
    fold_relu([&](uint32_t k) { return w1q[k]; }, [&](uint32_t k, float v) { w1q[k] = v; },
              [](float, float) { return 0u; });   // stage 1 stays fp32
    if ((e = upload(ix->d_w1, w1q, s)) != hipSuccess)
        return fail_train(e, "uploading stage-1 weights");

    // ---- route every key with the quantised stage 1
    std::vector<uint32_t> route(N);
    if ((e = launch_route(ix->d_w1, E, d_keys, N, d_route, s)) != hipSuccess ||
        (e = hipMemcpyAsync(route.data(), d_route, sizeof(uint32_t) * N, hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail_train(e, "routing keys");

    // per-expert key and position ranges
    std::vector<ExpertMeta> meta(E);
    std::vector<uint32_t> klo(E, 0xFFFFFFFFu), khi(E, 0);
    std::vector<int32_t> plo(E, INT32_MAX), phi(E, -1);
    for (size_t k = 0; k < N; ++k) {
        const uint32_t ex = route[k];
        klo[ex] = std::min(klo[ex], keys[k]);
        khi[ex] = std::max(khi[ex], keys[k]);
        plo[ex] = std::min(plo[ex], pos[k]);
        phi[ex] = std::max(phi[ex], pos[k]);
    }
    for (uint32_t ex = 0; ex < E; ++ex) {
        ExpertMeta& m = meta[ex];
        std::memset(&m, 0, sizeof m);
        if (phi[ex] < 0) {   // no key routed here: predictions land on position 0
            m.key_lo = 0;
            m.inv_span = 0.0f;
            continue;
        }
        m.key_lo = klo[ex];
        m.inv_span = float(1.0 / (double(khi[ex]) - double(klo[ex]) + 1.0));
        m.pos_lo = plo[ex];
        m.pos_hi = phi[ex];
        m.pos_span = float(phi[ex] - plo[ex]);
    }

    // ---- stage 2: E networks, samples sorted by expert
    std::vector<size_t> order(N);
    std::iota(order.begin(), order.end(), size_t(0));
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return route[a] < route[b]; });
    std::vector<float> w2(size_t(E) * P);
    for (uint32_t ex = 0; ex < E; ++ex) init_network(w2.data() + size_t(ex) * P, H, rng);
    {
        Trainer tr;
        ScopeExit tr_release([&] { tr.release(); });
        if ((e = tr.init(E, H, N, o.use_mfma != 0, s)) != hipSuccess)
            return fail_train(e, "allocating stage-2 training");
        std::vector<float> hu(N), ht(N);
        std::vector<uint32_t> hex(N);
        for (size_t k = 0; k < N; ++k) {
            const size_t q = order[k];
            const uint32_t ex = route[q];
            const ExpertMeta& m = meta[ex];
            hex[k] = ex;
            hu[k] = keys[q] >= m.key_lo ? std::min(float(keys[q] - m.key_lo) * m.inv_span, 1.0f)
                                        : 0.0f;
            ht[k] = m.pos_span > 0.0f ? float(pos[q] - m.pos_lo) / m.pos_span : 0.0f;
        }
        e = tr.load(hu, ht, hex, w2, s);
        if (e == hipSuccess && o.train) e = tr.train(o.epochs2, o.lr, s);
        std::vector<float> l2(E, 0.0f);
        if (e == hipSuccess && o.train) e = tr.gradients(s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(w2.data(), tr.params, sizeof(float) * w2.size(),
                               hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && o.train)
            e = hipMemcpyAsync(l2.data(), tr.loss, sizeof(float) * E, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        tr.release();
        if (e != hipSuccess) return fail_train(e, "training stage 2");
        for (float x : l2) loss2 += x;
    }
    std::vector<uint16_t> w2q(size_t(E) * kInferStride, 0);
    ix->weights.assign(size_t(P) * (E + 1), 0.0f);
    for (uint32_t k = 0; k < P; ++k) ix->weights[k] = w1_trained[infer_slot(k, H)];
    for (uint32_t ex = 0; ex < E; ++ex) {
        for (uint32_t k = 0; k < P; ++k) {
            const uint16_t b = to_bf16(w2[size_t(ex) * P + k]);
            w2q[size_t(ex) * kInferStride + infer_slot(k, H)] = b;
            ix->weights[size_t(ex + 1) * P + k] = from_bf16(b);
        }
        uint16_t* row = w2q.data() + size_t(ex) * kInferStride;
        fold_relu([&](uint32_t k) { return from_bf16(row[k]); },
                  [&](uint32_t k, float v) { row[k] = to_bf16(v); },    // exact: v is bf16
                  half_rounding);
    }
    const std::vector<uint32_t> w2r = stage2_rows(w2q, E, meta, &ix->weights_rounded);
    if ((e = upload(ix->d_w2, w2r, s)) != hipSuccess ||
        (e = upload(ix->d_meta, meta, s)) != hipSuccess)
        return fail_train(e, "uploading stage-2 weights");

    // ---- error bounds with the inference arithmetic itself
    ix->err.assign(E, 0);
    if ((e = launch_fill_u32(d_err, E, 0u, s)) != hipSuccess ||
        (e = launch_err_bound(args_of(ix, 1), d_keys, d_pos, N, d_err, s)) != hipSuccess ||
        (e = hipMemcpyAsync(ix->err.data(), d_err, sizeof(uint32_t) * E, hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail_train(e, "measuring error bounds");
    if (o.zero_error_bounds) std::fill(ix->err.begin(), ix->err.end(), 0u);
    for (uint32_t ex = 0; ex < E; ++ex) meta[ex].err = ix->err[ex];
    if ((e = upload(ix->d_meta, meta, s)) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail_train(e, "uploading error bounds");
    // the kernel's LDS images, one per placement of the boundary arrays
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        const std::vector<uint8_t> img = lds_image(ix, w1q, meta, w2r, b != 0);
        uint8_t* d = nullptr;
        e = dalloc(&d, img.size(), &ix->device_bytes);
        ix->d_image[b] = reinterpret_cast<uint4*>(d);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d, img.data(), img.size(), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_train(e, "uploading the LDS images");
    free_scratch();

    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->n_boundaries = M;
        stats->n_global = ix->nG;
        stats->n_list_entries = ix->nL;
        uint32_t mx = 0;
        for (uint32_t j = 0; j < M; ++j) mx = std::max(mx, ix->off[j + 1] - ix->off[j]);
        stats->max_list = mx;
        uint32_t emax = 0;
        double esum = 0;
        for (uint32_t v : ix->err) {
            emax = std::max(emax, v);
            esum += v;
        }
        stats->err_max = emax;
        stats->err_mean = float(esum / E);
        stats->loss1 = loss1;
        stats->loss2 = loss2;
        stats->train_ms = float(std::chrono::duration<double, std::milli>(
                                    std::chrono::steady_clock::now() - t_start)
                                    .count());
        stats->weights_rounded = ix->weights_rounded;
        stats->device_bytes = ix->device_bytes;
    }
    drop_ix.dismiss();
    *out = ix;
    return FW_OK;
}

fw_status classify_learned(const LearnedIndex* ix, uint8_t default_action, PacketsDev pk,
                           size_t n, int32_t* out_idx, uint8_t* out_act, uint32_t lookup,
                           uint32_t packets_per_lane, hipStream_t stream,
                           uint64_t* window_misses) {
    if (lookup > 1) return fail(FW_E_INVAL, "lookup must be 0 or 1");
    LookupArgs a = args_of(ix, lookup == 0 ? 1u : 0u);
    hipError_t e = hipSuccess;
    // The miss count of this call only: a counter allocated on the stream for
    // it, so calls on other streams never share one.
    unsigned long long* cnt = nullptr;
    if (window_misses) {
        e = hipMallocAsync(reinterpret_cast<void**>(&cnt), 2 * sizeof(unsigned long long), stream);
        if (e == hipSuccess)
            e = launch_fill_u32(reinterpret_cast<uint32_t*>(cnt), 2, 0u, stream);
        if (e != hipSuccess) {
            if (cnt) (void)hipFreeAsync(cnt, stream);
            return hip_fail(e, "setting up the miss counter");
        }
        a.miss = cnt;
    }
    e = launch_learned(a, pk, n, out_idx, out_act, default_action, nullptr, nullptr,
                       packets_per_lane, stream);
    if (e != hipSuccess) {
        if (cnt) (void)hipFreeAsync(cnt, stream);
        return hip_fail(e, "learned lookup launch");
    }
    if (window_misses) {
        unsigned long long v = 0;
        e = hipMemcpyAsync(&v, cnt, sizeof v, hipMemcpyDeviceToHost, stream);
        const hipError_t e2 = hipFreeAsync(cnt, stream);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "reading the miss counter");
        *window_misses = v;
    }
    return FW_OK;
}

void index_chain_view(const LearnedIndex* ix, ChainView* v) {
    v->la = args_of(ix, 1u);
    v->has_index = 1u;
    v->lds_b = uint32_t(learned_lds_bytes(v->la, true));
    v->lds_nob = uint32_t(learned_lds_bytes(v->la, false));
}

fw_status index_lookup(const LearnedIndex* ix, const uint32_t* keys, size_t n,
                       int32_t* out_interval, uint32_t lookup, hipStream_t stream) {
    const LookupArgs a = args_of(ix, lookup == 0 ? 1u : 0u);
    const hipError_t e = launch_learned(a, PacketsDev{}, n, nullptr, nullptr, 0, keys,
                                        out_interval, 1, stream);
    if (e != hipSuccess) return hip_fail(e, "interval lookup launch");
    return FW_OK;
}

fw_status index_export(const LearnedIndex* ix, uint32_t what, void* host, size_t cap,
                       size_t* size) {
    const void* src = nullptr;
    size_t bytes = 0;
    switch (what) {
        case 0: src = ix->B.data(); bytes = ix->B.size() * 4; break;
        case 1: src = ix->off.data(); bytes = ix->off.size() * 4; break;
        case 2: src = ix->L_idx.data(); bytes = ix->L_idx.size() * 4; break;
        case 3: src = ix->G_idx.data(); bytes = ix->G_idx.size() * 4; break;
        case 4: src = ix->err.data(); bytes = ix->err.size() * 4; break;
        case 5: src = ix->weights.data(); bytes = ix->weights.size() * 4; break;
        case 6: src = ix->Bs.data(); bytes = ix->Bs.size() * 4; break;
        case 7: src = ix->soff.data(); bytes = ix->soff.size() * 4; break;
        case 8: src = ix->S_idx.data(); bytes = ix->S_idx.size() * 4; break;
        case 9: src = ix->Gw_idx.data(); bytes = ix->Gw_idx.size() * 4; break;
        case 10: src = &ix->pt; bytes = sizeof(PortTable); break;
        case 11: src = ix->pt_shape; bytes = sizeof ix->pt_shape; break;
        case 12: src = ix->bs_bucket.data(); bytes = ix->bs_bucket.size() * 2; break;
        default: return fail(FW_E_INVAL, "unknown export %u", what);
    }
    if (size) *size = bytes;
    if (host && cap && bytes) std::memcpy(host, src, std::min(cap, bytes));
    return FW_OK;
}

}  // namespace fw

using namespace fw;

extern "C" {

fw_status fw_rmi_gradients(uint32_t E, uint32_t H, const float* params, size_t n, const float* u,
                           const float* t, const uint32_t* expert, uint32_t use_mfma, float* grad,
                           float* loss) {
    return guarded([&]() -> fw_status {
        if (E == 0 || E > kMaxExperts) return fail(FW_E_INVAL, "E must be 1..%u", kMaxExperts);
        if (H == 0 || H > kMaxHidden) return fail(FW_E_INVAL, "H must be 1..%u", kMaxHidden);
        if (!params || !grad || (n && (!u || !t || !expert)))
            return fail(FW_E_INVAL, "NULL argument");
        if (n > (size_t(1) << 31)) return fail(FW_E_INVAL, "at most 2^31 samples");
        for (size_t k = 0; k < n; ++k)
            if (expert[k] >= E)
                return fail(FW_E_INVAL, "sample %zu: network index out of range", k);
        const uint32_t P = 3 * H + 1;
        std::vector<size_t> order(n);
        std::iota(order.begin(), order.end(), size_t(0));
        std::stable_sort(order.begin(), order.end(),
                         [&](size_t a, size_t b) { return expert[a] < expert[b]; });
        std::vector<float> hu(n), ht(n);
        std::vector<uint32_t> hex(n);
        for (size_t k = 0; k < n; ++k) {
            hu[k] = u[order[k]];
            ht[k] = t[order[k]];
            hex[k] = expert[order[k]];
        }
        std::vector<float> hp(params, params + size_t(E) * P);
        hipStream_t s = nullptr;
        Trainer tr;
        ScopeExit tr_release([&] { tr.release(); });
        hipError_t e = tr.init(E, H, n, use_mfma != 0, s);
        if (e == hipSuccess) e = tr.load(hu, ht, hex, hp, s);
        if (e == hipSuccess) e = tr.gradients(s);
        if (e == hipSuccess)
            e = hipMemcpy(grad, tr.grad, sizeof(float) * size_t(E) * P, hipMemcpyDeviceToHost);
        if (e == hipSuccess && loss)
            e = hipMemcpy(loss, tr.loss, sizeof(float) * E, hipMemcpyDeviceToHost);
        tr.release();
        if (e != hipSuccess) return hip_fail(e, "gradient kernels");
        return FW_OK;
    });
}

fw_status fw_rmi_adam_step(size_t count, float* params, const float* grad, float* m, float* v,
                           uint32_t step, float lr, float beta1, float beta2, float eps) {
    return guarded([&]() -> fw_status {
        if (!params || !grad || !m || !v) return fail(FW_E_INVAL, "NULL argument");
        if (step == 0) return fail(FW_E_INVAL, "step counts from 1");
        if (count > (size_t(1) << 31)) return fail(FW_E_INVAL, "at most 2^31 parameters");
        if (count == 0) return FW_OK;
        float* d = nullptr;
        hipError_t e = hipMalloc(&d, sizeof(float) * count * 4);
        if (e != hipSuccess) return hip_fail(e, "allocation");
        float *dp = d, *dg = d + count, *dm = d + 2 * count, *dv = d + 3 * count;
        e = hipMemcpy(dp, params, sizeof(float) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(dg, grad, sizeof(float) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(dm, m, sizeof(float) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(dv, v, sizeof(float) * count, hipMemcpyHostToDevice);
        const float bc1 = float(1.0 - std::pow(double(beta1), double(step)));
        const float bc2 = float(1.0 - std::pow(double(beta2), double(step)));
        if (e == hipSuccess)
            e = launch_adam(dp, dg, dm, dv, count, lr, beta1, beta2, eps, bc1, bc2, nullptr);
        if (e == hipSuccess)
            e = hipMemcpy(params, dp, sizeof(float) * count, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(m, dm, sizeof(float) * count, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(v, dv, sizeof(float) * count, hipMemcpyDeviceToHost);
        (void)hipFree(d);
        if (e != hipSuccess) return hip_fail(e, "Adam kernel");
        return FW_OK;
    });
}

}  // extern "C"
