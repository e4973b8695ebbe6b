// Learned destination index on gfx950: training kernels for the two-stage
// network, the shared inference routine, and the lookup + candidate-scan
// kernel.
//
// Every network maps one input to one output through H ReLU units:
//   f(u) = sum_k w2[k] * relu(w1[k] * u + b1[k]) + b2,
// parameters laid out [w1 (H), b1 (H), w2 (H), b2].  A stage of E such
// networks minimises the sum of each network's mean squared error over its
// own samples; Adam (Kingma and Ba) updates the fp32 master weights.
//
// Weight gradients are segmented sums over samples: for network e and
// parameter c, g[e][c] = sum over samples n of network e of A[n][c], where A
// holds each sample's per-parameter contributions.  With the one-hot
// expert-membership matrix S (S[n][e] = 1 when sample n trains e) this is the
// product S^T * A, which runs on the matrix cores as bf16 x bf16 -> fp32 MFMA
// (S is exact in bf16).  A plain fp32 reduction computes the same sums for
// checking.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "device_util.h"
#include "fw_internal.h"
#include "index.h"
#include "learned_core.h"
#include "scan_core.h"

namespace fw {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr uint32_t kChunk = 512;   // samples per MFMA work-group (32 steps of K = 16)

// Round to nearest even (inputs here are finite).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return uint16_t(b >> 16);
}

// ------------------------------------------------------------------ forward + backward
// One thread per sample: forward pass of the sample's network, dL/dy, and the
// sample's contribution to every parameter's gradient, written as column c of
// the transposed sample matrix AT[c][n]:
//   c in [0, H): dz_k * u      (w1)     c in [H, 2H): dz_k      (b1)
//   c in [2H, 3H): relu(z_k) d (w2)     c = 3H: d               (b2)
//   c = 3H + 1: (y - t)^2 / N_e (loss)
// with d = 2 (y - t) / N_e and dz_k = d * w2[k] * [z_k > 0].
template <bool BF16>
__global__ __launch_bounds__(256) void k_fwd_bwd(const float* __restrict__ params, uint32_t H,
                                                 const float* __restrict__ u,
                                                 const float* __restrict__ t,
                                                 const uint32_t* __restrict__ ex,
                                                 const float* __restrict__ inv_count, size_t n,
                                                 size_t n_pad, void* __restrict__ at_) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    auto put = [&](uint32_t c, float v) {
        if constexpr (BF16)
            static_cast<uint16_t*>(at_)[size_t(c) * n_pad + i] = f32_to_bf16(v);
        else
            static_cast<float*>(at_)[size_t(c) * n_pad + i] = v;
    };
    const uint32_t e = i < n ? ex[i] : kNoExpert;
    if (e == kNoExpert) {
        for (uint32_t c = 0; c < 3 * H + 2; ++c) put(c, 0.0f);
        return;
    }
    const uint32_t P = 3 * H + 1;
    const float* p = params + size_t(e) * P;
    const float x = u[i], target = t[i], inv = inv_count[e];
    float z[kMaxHidden];
    float y = p[3 * H];
#pragma unroll
    for (uint32_t k = 0; k < kMaxHidden; ++k) {
        if (k < H) {
            z[k] = fmaf(p[k], x, p[H + k]);
            y = fmaf(p[2 * H + k], fmaxf(z[k], 0.0f), y);
        }
    }
    const float r = y - target;
    const float d = 2.0f * r * inv;
#pragma unroll
    for (uint32_t k = 0; k < kMaxHidden; ++k) {
        if (k < H) {
            const float dz = z[k] > 0.0f ? d * p[2 * H + k] : 0.0f;
            put(k, dz * x);
            put(H + k, dz);
            put(2 * H + k, fmaxf(z[k], 0.0f) * d);
        }
    }
    put(3 * H, d);
    put(3 * H + 1, r * r * inv);
}

// ------------------------------------------------------------------ S^T * A on MFMA
// Grid (chunks, E_pad / 32); four waves, wave w computing output columns
// [32w, 32w + 32) of the 32 experts of its row tile over the chunk's kChunk
// samples.  v_mfma_f32_32x32x16_bf16: lane l supplies A-operand row l % 32,
// k = 8 (l / 32) + 0..7, and B-operand column l % 32 with the same k; it
// holds output rows 8 (r / 4) + 4 (l / 32) + r % 4 of column l % 32 in acc[r].
__global__ __launch_bounds__(256) void k_grad_mfma(const uint16_t* __restrict__ at,
                                                   const uint32_t* __restrict__ ex, size_t n_pad,
                                                   uint32_t E_pad, float* __restrict__ partial) {
    const uint32_t chunk = blockIdx.x, mtile = blockIdx.y;
    const uint32_t wave = wave_in_group(), lane = threadIdx.x & 63u;
    const uint32_t m = mtile * 32u + (lane & 31u);
    const uint32_t c = wave * 32u + (lane & 31u);
    const uint32_t kq = (lane >> 5) * 8u;
    f32x16 acc = {};
    const uint16_t* col = at + size_t(c) * n_pad;
    for (uint32_t ks = 0; ks < kChunk; ks += 16) {
        const size_t s0 = size_t(chunk) * kChunk + ks + kq;
        const uint4 e0 = *reinterpret_cast<const uint4*>(ex + s0);
        const uint4 e1 = *reinterpret_cast<const uint4*>(ex + s0 + 4);
        const unsigned short one = 0x3F80;  // 1.0 in bf16
        u16x8 a;
        a[0] = e0.x == m ? one : 0; a[1] = e0.y == m ? one : 0;
        a[2] = e0.z == m ? one : 0; a[3] = e0.w == m ? one : 0;
        a[4] = e1.x == m ? one : 0; a[5] = e1.y == m ? one : 0;
        a[6] = e1.z == m ? one : 0; a[7] = e1.w == m ? one : 0;
        const u16x8 b = *reinterpret_cast<const u16x8*>(col + s0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                      __builtin_bit_cast(bf16x8, b), acc, 0, 0,
                                                      0);
    }
    float* out = partial + size_t(chunk) * E_pad * kGradCols;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const uint32_t row = mtile * 32u + 8u * (r / 4) + 4u * (lane >> 5) + (r % 4);
        out[size_t(row) * kGradCols + c] = acc[r];
    }
}

// Sum the per-chunk partial products in chunk order (deterministic).
__global__ void k_grad_reduce(const float* __restrict__ partial, uint32_t chunks, uint32_t E,
                              uint32_t E_pad, uint32_t H, float* __restrict__ grad,
                              float* __restrict__ loss) {
    const uint32_t P = 3 * H + 1;
    const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= E * (P + 1)) return;
    const uint32_t e = o / (P + 1), c = o % (P + 1);
    float s = 0.0f;
    for (uint32_t k = 0; k < chunks; ++k) s += partial[(size_t(k) * E_pad + e) * kGradCols + c];
    if (c < P)
        grad[size_t(e) * P + c] = s;
    else if (loss)
        loss[e] = s;
}

// fp32 reference path: samples sorted by network, seg[e]..seg[e+1] belong to e;
// one thread per (network, column) sums its column in sample order.
__global__ void k_grad_fp32(const float* __restrict__ at, size_t n_pad,
                            const uint32_t* __restrict__ seg, uint32_t H,
                            float* __restrict__ grad, float* __restrict__ loss) {
    const uint32_t e = blockIdx.x, c = threadIdx.x;
    const uint32_t P = 3 * H + 1;
    if (c > P) return;
    float s = 0.0f;
    const float* col = at + size_t(c) * n_pad;
    for (uint32_t k = seg[e]; k < seg[e + 1]; ++k) s += col[k];
    if (c < P)
        grad[size_t(e) * P + c] = s;
    else if (loss)
        loss[e] = s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t count, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void k_fill(uint32_t* p, size_t n, uint32_t v) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_route(const float* __restrict__ w1, uint32_t E, const uint32_t* __restrict__ keys,
                        size_t n, uint32_t* __restrict__ out) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = route(w1, E, keys[i]);
}

// Per-expert maximum |predicted - true position| over the training keys.
__global__ void k_err_bound(LookupArgs a, const uint32_t* __restrict__ keys,
                            const int32_t* __restrict__ pos, size_t n, uint32_t* __restrict__ err) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t x = keys[i];
    const uint32_t e = route(a.w1, a.E, x);
    const int32_t p = position(a.w2 + size_t(e) * kRowDwords, a.meta[e].pos_lo, x);
    const int32_t d = p - pos[i];
    atomicMax(err + e, uint32_t(d < 0 ? -d : d));
}

// With one or two packets per lane, two work-groups per CU (the LDS footprint
// allows two): eight waves per SIMD, so at most 64 VGPRs.  Four packets per
// lane need more registers and run one work-group per CU.  Persistent: each
// wave strides over tiles of 64*K packets (see learned_tile).
template <bool B_LDS, int K, bool PLAN>
__global__ __launch_bounds__(kLearnedBlock, K >= 4 ? 4 : 8) void k_learned(LookupArgs a, PacketsDev pk, size_t n,
                                                           int32_t* __restrict__ out_idx,
                                                           uint8_t* __restrict__ out_act,
                                                           uint32_t dflt) {
    extern __shared__ __align__(16) unsigned char smem[];
    const IndexView v = stage_index<B_LDS>(a, smem);
    constexpr uint32_t kWaves = kLearnedBlock / 64;   // compile-time: keeps the loop scalar
    const size_t waves = size_t(gridDim.x) * kWaves;
    const size_t wave0 = size_t(blockIdx.x) * kWaves + wave_in_group();
    for (size_t base = wave0 * 64u * K; base < n; base += waves * 64u * K)
        learned_tile<K, PLAN>(a, v, pk, base, n, out_idx, out_act, dflt);
}

// Interval lookup only, one key per lane.
template <bool B_LDS>
__global__ __launch_bounds__(kLearnedBlock) void k_lookup(LookupArgs a,
                                                          const uint32_t* __restrict__ keys,
                                                          size_t n,
                                                          int32_t* __restrict__ out_interval) {
    extern __shared__ __align__(16) unsigned char smem[];
    const IndexView v = stage_index<B_LDS>(a, smem);
    constexpr uint32_t kWaves = kLearnedBlock / 64;   // compile-time: keeps the loop scalar
    const size_t waves = size_t(gridDim.x) * kWaves;
    const size_t wave0 = size_t(blockIdx.x) * kWaves + wave_in_group();
    for (size_t base = wave0 * 64u; base < n; base += waves * 64u) {
        const size_t i = base + (threadIdx.x & 63u);
        const bool valid = i < n;
        bool miss = false;
        const uint32_t x = valid ? keys[i] : 0u;
        const uint32_t j = locate(v.B, a.M, v.w2, v.meta, a.use_net,
                                                 a.use_net ? route(v.w1, a.E, x) : 0u, x, &miss);
        if (valid) out_interval[i] = int32_t(j);
    }
}

inline uint32_t blocks_for(size_t n, uint32_t per) { return uint32_t((n + per - 1) / per); }

struct LearnedLaunchCache {
    int device = -1;
    int cus = 0;
    int max_lds = 0;
};
thread_local LearnedLaunchCache g_cache;

// Resident work-groups per CU for (kernel, device, dynamic LDS bytes), and the
// largest dynamic LDS size granted to each kernel so far.  Queried once: a
// small batch's latency should not pay for occupancy queries on every call.
// The granted size only grows, so a launch never finds it lowered by another
// thread's smaller request.
std::mutex g_launch_mu;
std::map<std::tuple<const void*, int, size_t>, int> g_per_cu;
std::map<std::pair<const void*, int>, size_t> g_lds_granted;

template <class Kern>
hipError_t blocks_per_cu(Kern kern, size_t lds, int* per_cu) {
    const void* f = reinterpret_cast<const void*>(kern);
    std::lock_guard<std::mutex> lk(g_launch_mu);
    const auto key = std::make_tuple(f, g_cache.device, lds);
    const auto it = g_per_cu.find(key);
    if (it != g_per_cu.end()) {
        *per_cu = it->second;
        return hipSuccess;
    }
    size_t& granted = g_lds_granted[std::make_pair(f, g_cache.device)];
    if (lds > granted) {
        const hipError_t e =
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        granted = lds;
    }
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kern, kLearnedBlock,
                                                                      lds);
    if (e != hipSuccess) return e;
    g_per_cu[key] = *per_cu;
    return hipSuccess;
}

template <class Kern, class... Args>
hipError_t launch_persistent(Kern kern, size_t lds, size_t tiles, hipStream_t s, Args... args) {
    int per_cu = 0;
    const hipError_t e = blocks_per_cu(kern, lds, &per_cu);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const size_t want = (tiles + (kLearnedBlock / 64) - 1) / (kLearnedBlock / 64);
    size_t grid = size_t(per_cu) * size_t(g_cache.cus);
    if (grid > want) grid = want;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3(uint32_t(grid)), dim3(kLearnedBlock), lds, s, args...);
    return hipGetLastError();
}

}  // namespace

uint32_t grad_mfma_chunks(size_t n_pad) { return uint32_t(n_pad / kChunk); }

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fwd_bwd(const float* params, uint32_t H, const float* u, const float* t,
                          const uint32_t* ex, const float* inv_count, size_t n, size_t n_pad,
                          void* at, bool bf16, hipStream_t s) {
    if (bf16)
        hipLaunchKernelGGL(k_fwd_bwd<true>, dim3(blocks_for(n_pad, 256)), dim3(256), 0, s, params,
                           H, u, t, ex, inv_count, n, n_pad, at);
    else
        hipLaunchKernelGGL(k_fwd_bwd<false>, dim3(blocks_for(n_pad, 256)), dim3(256), 0, s,
                           params, H, u, t, ex, inv_count, n, n_pad, at);
    return hipGetLastError();
}

hipError_t launch_grad_mfma(const uint16_t* at, const uint32_t* ex, size_t n_pad, uint32_t E,
                            float* partial, hipStream_t s) {
    const uint32_t E_pad = (E + 31u) & ~31u;
    hipLaunchKernelGGL(k_grad_mfma, dim3(grad_mfma_chunks(n_pad), E_pad / 32u), dim3(256), 0, s,
                       at, ex, n_pad, E_pad, partial);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const float* partial, uint32_t chunks, uint32_t E, uint32_t H,
                              float* grad, float* loss, hipStream_t s) {
    const uint32_t E_pad = (E + 31u) & ~31u;
    const uint32_t total = E * (3 * H + 2);
    hipLaunchKernelGGL(k_grad_reduce, dim3(blocks_for(total, 256)), dim3(256), 0, s, partial,
                       chunks, E, E_pad, H, grad, loss);
    return hipGetLastError();
}

hipError_t launch_grad_fp32(const float* at, size_t n_pad, const uint32_t* seg, uint32_t E,
                            uint32_t H, float* grad, float* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_grad_fp32, dim3(E), dim3(kGradCols), 0, s, at, n_pad, seg, H, grad,
                       loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, size_t count, float lr,
                       float b1, float b2, float eps, float bc1, float bc2, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(count, 256)), dim3(256), 0, s, p, g, m, v, count,
                       lr, b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_route(const float* w1, uint32_t E, const uint32_t* keys, size_t n,
                        uint32_t* expert, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_route, dim3(blocks_for(n, 256)), dim3(256), 0, s, w1, E, keys, n, expert);
    return hipGetLastError();
}

hipError_t launch_err_bound(const LookupArgs& a, const uint32_t* keys, const int32_t* pos,
                            size_t n, uint32_t* err, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_err_bound, dim3(blocks_for(n, 256)), dim3(256), 0, s, a, keys, pos, n,
                       err);
    return hipGetLastError();
}

size_t learned_lds_bytes(const LookupArgs& a, bool b_in_lds) {
    return LdsLayout(a.E, a.M, a.Ms, a.bs_bits, b_in_lds).bytes;
}

hipError_t launch_learned(const LookupArgs& a, PacketsDev pk, size_t n, int32_t* out_idx,
                          uint8_t* out_act, uint32_t dflt, const uint32_t* keys,
                          int32_t* out_interval, uint32_t packets_per_lane, hipStream_t s) {
    if (n == 0) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (g_cache.device != dev) {
        e = hipDeviceGetAttribute(&g_cache.cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&g_cache.max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                      dev);
        if (e != hipSuccess) return e;
        g_cache.device = dev;
    }
    // One or two packets per lane keep two work-groups of 16 waves per CU, so
    // the staged index must stay within 80 KiB; four per lane run one
    // work-group per CU and may use up to 150 KiB.  The boundary arrays and
    // list offsets go to LDS when they fit (the binary searches probe them,
    // every packet reads its list bounds); the rest of the image always does
    // (past about 200 experts it outgrows 80 KiB, and one work-group per CU
    // runs).
    const uint32_t K = packets_per_lane ? packets_per_lane : kLearnedK;
    const size_t cap = std::min<size_t>(K >= 4 ? 150u * 1024u : 80u * 1024u,
                                        size_t(g_cache.max_lds));
    const bool b_lds = learned_lds_bytes(a, true) <= cap;
    const size_t lds = learned_lds_bytes(a, b_lds);
    if (keys) {
        const size_t tiles = (n + 63) / 64;
        return b_lds ? launch_persistent(k_lookup<true>, lds, tiles, s, a, keys, n, out_interval)
                     : launch_persistent(k_lookup<false>, lds, tiles, s, a, keys, n, out_interval);
    }
    const size_t tiles = (n + 64 * K - 1) / (64 * K);
    const bool plan = a.G.n_groups != 0;
#define FW_LEARNED(BL, KK, P) \
    launch_persistent(k_learned<BL, KK, P>, lds, tiles, s, a, pk, n, out_idx, out_act, dflt)
#define FW_LEARNED_K(BL, P) \
    (K == 1 ? FW_LEARNED(BL, 1, P) : K == 2 ? FW_LEARNED(BL, 2, P) : FW_LEARNED(BL, 4, P))
    if (b_lds) return plan ? FW_LEARNED_K(true, true) : FW_LEARNED_K(true, false);
    return plan ? FW_LEARNED_K(false, true) : FW_LEARNED_K(false, false);
#undef FW_LEARNED_K
#undef FW_LEARNED
}

}  // namespace fw
