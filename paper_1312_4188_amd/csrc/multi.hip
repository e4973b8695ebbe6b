// Many independent chains (rulesets, each with its own packet batch) in one
// persistent launch, with work-queue scheduling and an autotuner.
//
// Work items are tiles of one chain's packets.  Chains are ordered by an
// estimate of their cost (rules x packets, largest first) so the expensive
// items are handed out first; resident work-groups take items from a global
// counter until none are left, so uneven chains balance themselves.  Three
// rule placements (the paper's Section IV-A compares global, constant and
// shared memory for the rule table): records read through the scalar cache
// into SGPRs (each wave takes its own 64*K-packet items), the same records
// read by vector loads into VGPRs, or records staged into LDS tiles shared by
// the four waves of a work-group (items of 256*K packets).  The autotuner times the
// packets-per-lane x placement grid on the caller's own batches and caches
// the fastest choice per batch shape.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/fw.h"
#include "device_util.h"
#include "fw_internal.h"
#include "index.h"
#include "scan_core.h"

struct fw_ruleset;

namespace fw {

// Read-only view of a loaded ruleset (defined in api.cpp).
void ruleset_view(const fw_ruleset* rs, const RuleRec** rules, const uint2** pairs,
                  uint32_t* n_rules, uint8_t* default_action);

namespace {

struct ChainDesc {
    const RuleRec* rules;
    const uint2* pairs;
    const uint32_t* src;
    const uint32_t* dst;
    const uint16_t* sport;
    const uint16_t* dport;
    const uint8_t* proto;
    int32_t* out_idx;
    uint8_t* out_act;
    uint64_t n;
    uint32_t n_rules, dflt;
    uint32_t item_begin, pad;
};
static_assert(sizeof(ChainDesc) == 96, "descriptor layout");

constexpr uint32_t kDescPerChunk = 32;   // 3 KiB of kernel arguments per upload launch

// Scratch of fw_classify_multi_noalloc: the descriptor table of up to
// kNoAllocMaxChains chains, then the work-queue counter, in one static device
// array (each GPU the library runs on holds its own copy for the life of the
// process).  Host code never passes the array's name to a kernel: it takes
// the array's device address from hipGetSymbolAddress, once per device.
constexpr uint32_t kNoAllocMaxChains = 1024;
constexpr size_t kScratchTable = sizeof(ChainDesc) * kNoAllocMaxChains;
__device__ __align__(256) unsigned char scratch[kScratchTable + 256];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

struct DescChunk {
    ChainDesc d[kDescPerChunk];
};

__global__ void k_put_desc(DescChunk chunk, uint32_t count, ChainDesc* table, uint32_t at,
                           uint32_t* counter) {
    const uint32_t i = threadIdx.x;
    if (i < count) table[at + i] = chunk.d[i];
    if (at == 0 && i == 0) *counter = 0u;
}

__device__ __forceinline__ uint32_t chain_of(const ChainDesc* __restrict__ cd, uint32_t n_chains,
                                             uint32_t item) {
    uint32_t lo = 0, hi = n_chains - 1u;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1u) >> 1;
        if (cd[mid].item_begin <= item)
            lo = mid;
        else
            hi = mid - 1u;
    }
    return lo;
}

// Scalar placement: each wave takes 64*K-packet items on its own.
template <int K>
__global__ __launch_bounds__(256) void k_multi_scalar(const ChainDesc* __restrict__ cd,
                                                      uint32_t n_chains, uint32_t total_items,
                                                      uint32_t* __restrict__ counter) {
    const uint32_t lane = threadIdx.x & 63u;
    for (;;) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(counter, 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= total_items) break;
        const ChainDesc& c = cd[chain_of(cd, n_chains, item)];
        const size_t first = size_t(item - c.item_begin) * (64u * K);
        const PacketsDev pk{c.src, c.dst, c.sport, c.dport, c.proto};
        scan_wave<K>(c.pairs, c.rules, c.n_rules, pk, first, c.n, c.out_idx, c.out_act, c.dflt);
    }
}

// Vector placement: as the scalar placement, but every rule operand is read
// by vector loads (all lanes the same address) and held in VGPRs.
template <int K>
__global__ __launch_bounds__(256) void k_multi_vector(const ChainDesc* __restrict__ cd,
                                                      uint32_t n_chains, uint32_t total_items,
                                                      uint32_t* __restrict__ counter) {
    const uint32_t lane = threadIdx.x & 63u;
    for (;;) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(counter, 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= total_items) break;
        const ChainDesc& c = cd[chain_of(cd, n_chains, item)];
        const size_t first = size_t(item - c.item_begin) * (64u * K);
        const PacketsDev pk{c.src, c.dst, c.sport, c.dport, c.proto};
        WaveScan<K> w;
        w.init(pk, first, c.n, c.dflt);
        w.scan_vector(c.pairs, c.rules, c.n_rules);
        w.store(c.out_idx, c.out_act, c.n);
    }
}

// LDS placement: a work-group takes 256*K-packet items; rule tiles of TILE
// records are staged into LDS and scanned by all four waves, until every
// wave's packets have matched or the rules run out.
template <int K, int TILE>
__global__ __launch_bounds__(256) void k_multi_lds(const ChainDesc* __restrict__ cd,
                                                   uint32_t n_chains, uint32_t total_items,
                                                   uint32_t* __restrict__ counter) {
    __shared__ uint32_t s_item;
    __shared__ RuleRec s_rules[TILE];
    __shared__ uint2 s_pairs[TILE + kPairPadding];
    const uint32_t wave = wave_in_group();
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= total_items) break;
        const ChainDesc& c = cd[chain_of(cd, n_chains, item)];
        const size_t first = size_t(item - c.item_begin) * (256u * K) + size_t(wave) * 64u * K;
        const PacketsDev pk{c.src, c.dst, c.sport, c.dport, c.proto};
        WaveScan<K> w;
        const bool active = first < c.n;
        if (active) w.init(pk, first, c.n, c.dflt);
        int live = active && w.any_live();
        for (uint32_t r0 = 0; r0 < c.n_rules; r0 += TILE) {
            if (!__syncthreads_or(live)) break;
            const uint32_t cnt = min(uint32_t(TILE), c.n_rules - r0);
            const uint32_t* g = reinterpret_cast<const uint32_t*>(c.rules + r0);
            uint32_t* l = reinterpret_cast<uint32_t*>(s_rules);
            for (uint32_t k = threadIdx.x; k < cnt * 8u; k += blockDim.x) l[k] = g[k];
            for (uint32_t k = threadIdx.x; k < cnt; k += blockDim.x) s_pairs[k] = c.pairs[r0 + k];
            __syncthreads();
            if (live) live = w.template scan<FirstField::Dst>(s_pairs, s_rules, cnt, r0);
        }
        if (active) w.store(c.out_idx, c.out_act, c.n);
    }
}

struct Config {
    int K = 4;
    uint32_t tile = 0;     // LDS tile in rules; 0 = records read from global memory
    bool vector = false;   // with tile 0: vector loads instead of scalar loads
};

std::mutex g_tune_mu;
std::map<std::vector<uint64_t>, Config> g_tuned;

std::vector<uint64_t> shape_key(const fw_chain_batch* b, uint32_t n) {
    std::vector<uint64_t> key;
    key.reserve(2 * size_t(n));
    for (uint32_t c = 0; c < n; ++c) {
        key.push_back(fw_ruleset_size(b[c].rs));
        key.push_back(b[c].n);
    }
    return key;
}

template <class Kern>
hipError_t persistent_grid(Kern kern, uint32_t items, uint32_t* grid) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0);
    if (e != hipSuccess) return e;
    uint32_t g = uint32_t(std::max(1, per_cu) * std::max(1, cus));
    *grid = std::max(1u, std::min(g, items));
    return hipSuccess;
}

// One persistent launch over the batches.  The descriptor table and the work
// counter live in `scratch` when given (at least kScratchTable + 256 bytes,
// the table at its start and the counter at kScratchTable), else in memory
// allocated on the stream for this call and freed after it.
hipError_t run(const fw_chain_batch* b, uint32_t n_chains, Config cfg, hipStream_t s,
               void* scratch_mem = nullptr) {
    // order by estimated cost, largest first; skip empty batches
    std::vector<uint32_t> order;
    for (uint32_t c = 0; c < n_chains; ++c)
        if (b[c].n) order.push_back(c);
    if (order.empty()) return hipSuccess;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        return double(fw_ruleset_size(b[x].rs) + 1) * double(b[x].n) >
               double(fw_ruleset_size(b[y].rs) + 1) * double(b[y].n);
    });
    const uint64_t per_item = (cfg.tile ? 256u : 64u) * uint64_t(cfg.K);
    std::vector<ChainDesc> desc(order.size());
    uint64_t items = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        const fw_chain_batch& cb = b[order[k]];
        ChainDesc& d = desc[k];
        std::memset(&d, 0, sizeof d);
        uint8_t dflt = 0;
        ruleset_view(cb.rs, &d.rules, &d.pairs, &d.n_rules, &dflt);
        d.dflt = dflt;
        d.src = cb.pk.src_ip;
        d.dst = cb.pk.dst_ip;
        d.sport = cb.pk.src_port;
        d.dport = cb.pk.dst_port;
        d.proto = cb.pk.proto;
        d.out_idx = cb.out_rule_idx;
        d.out_act = cb.out_action;
        d.n = cb.n;
        d.item_begin = uint32_t(items);
        items += (cb.n + per_item - 1) / per_item;
    }
    if (items >= 0xFFFFFFFFull) return hipErrorInvalidValue;
    const uint32_t nc = uint32_t(desc.size());
    void* mem = scratch_mem;
    const size_t table_bytes = scratch_mem ? kScratchTable : sizeof(ChainDesc) * nc;
    if (scratch_mem && nc > kNoAllocMaxChains) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    if (!scratch_mem) e = hipMallocAsync(&mem, table_bytes + 256, s);
    if (e != hipSuccess) return e;
    ChainDesc* table = static_cast<ChainDesc*>(mem);
    uint32_t* counter = reinterpret_cast<uint32_t*>(static_cast<char*>(mem) + table_bytes);
    for (uint32_t at = 0; at < nc && e == hipSuccess; at += kDescPerChunk) {
        DescChunk ch{};
        const uint32_t cnt = std::min(kDescPerChunk, nc - at);
        std::memcpy(ch.d, desc.data() + at, sizeof(ChainDesc) * cnt);
        hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(kDescPerChunk), 0, s, ch, cnt, table, at,
                           counter);
        e = hipGetLastError();
    }
    uint32_t grid = 1;
    const uint32_t total = uint32_t(items);
#define FW_MULTI(KERN)                                                                   \
    do {                                                                                 \
        if (e == hipSuccess) e = persistent_grid(KERN, total, &grid);                    \
        if (e == hipSuccess) {                                                           \
            hipLaunchKernelGGL(KERN, dim3(grid), dim3(256), 0, s, table, nc, total, counter); \
            e = hipGetLastError();                                                       \
        }                                                                                \
    } while (0)
    if (cfg.tile == 0 && cfg.vector) {
        if (cfg.K == 1) FW_MULTI(k_multi_vector<1>);
        else if (cfg.K == 2) FW_MULTI(k_multi_vector<2>);
        else FW_MULTI(k_multi_vector<4>);
    } else if (cfg.tile == 0) {
        if (cfg.K == 1) FW_MULTI(k_multi_scalar<1>);
        else if (cfg.K == 2) FW_MULTI(k_multi_scalar<2>);
        else FW_MULTI(k_multi_scalar<4>);
    } else if (cfg.tile == 256) {
        if (cfg.K == 1) FW_MULTI((k_multi_lds<1, 256>));
        else if (cfg.K == 2) FW_MULTI((k_multi_lds<2, 256>));
        else FW_MULTI((k_multi_lds<4, 256>));
    } else {
        if (cfg.K == 1) FW_MULTI((k_multi_lds<1, 1024>));
        else if (cfg.K == 2) FW_MULTI((k_multi_lds<2, 1024>));
        else FW_MULTI((k_multi_lds<4, 1024>));
    }
#undef FW_MULTI
    if (scratch_mem) return e;
    const hipError_t e2 = hipFreeAsync(mem, s);
    return e != hipSuccess ? e : e2;
}

fw_status check_batches(const fw_chain_batch* b, uint32_t n) {
    if (!b && n) return fail(FW_E_INVAL, "batches is NULL");
    for (uint32_t c = 0; c < n; ++c) {
        if (!b[c].rs) return fail(FW_E_INVAL, "chain %u: ruleset is NULL", c);
        if (b[c].n == 0) continue;
        const fw_packets& p = b[c].pk;
        if (!p.src_ip || !p.dst_ip || !p.src_port || !p.dst_port || !p.proto ||
            !b[c].out_rule_idx || !b[c].out_action)
            return fail(FW_E_INVAL, "chain %u: NULL buffer", c);
        for (const void* q : {static_cast<const void*>(p.src_ip), static_cast<const void*>(p.dst_ip),
                              static_cast<const void*>(p.src_port),
                              static_cast<const void*>(p.dst_port),
                              static_cast<const void*>(p.proto),
                              static_cast<const void*>(b[c].out_rule_idx),
                              static_cast<const void*>(b[c].out_action)})
            if (reinterpret_cast<uintptr_t>(q) & 15u)
                return fail(FW_E_ALIGN, "chain %u: buffers must be 16-byte aligned", c);
    }
    return FW_OK;
}

fw_status resolve(const fw_chain_batch* b, uint32_t n, const fw_multi_opts& o, Config* cfg) {
    if (o.packets_per_lane != 0 && o.packets_per_lane != 1 && o.packets_per_lane != 2 &&
        o.packets_per_lane != 4)
        return fail(FW_E_INVAL, "packets_per_lane must be 0, 1, 2 or 4");
    if (o.placement > 3) return fail(FW_E_INVAL, "placement must be 0, 1, 2 or 3");
    if (o.rule_tile != 0 && o.rule_tile != 256 && o.rule_tile != 1024)
        return fail(FW_E_INVAL, "rule_tile must be 0, 256 or 1024");
    Config c;
    if (o.placement == 0 || o.packets_per_lane == 0) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(shape_key(b, n));
        if (it != g_tuned.end()) c = it->second;
    }
    if (o.packets_per_lane) c.K = int(o.packets_per_lane);
    if (o.placement == 1 || o.placement == 3) {
        c.tile = 0;
        c.vector = o.placement == 3;
    }
    if (o.placement == 2) {
        c.tile = o.rule_tile ? o.rule_tile : (c.tile ? c.tile : 1024u);
        c.vector = false;
    }
    *cfg = c;
    return FW_OK;
}

}  // namespace
}  // namespace fw

using namespace fw;

extern "C" {

fw_status fw_classify_multi(const fw_chain_batch* batches, uint32_t n_chains,
                            const fw_multi_opts* opts) {
    fw_multi_opts o{};
    if (opts) o = *opts;
    fw_status st = check_batches(batches, n_chains);
    if (st != FW_OK) return st;
    Config cfg;
    st = resolve(batches, n_chains, o, &cfg);
    if (st != FW_OK) return st;
    const hipError_t e = run(batches, n_chains, cfg, static_cast<hipStream_t>(o.stream));
    if (e != hipSuccess) return hip_fail(e, "multi-chain launch");
    return FW_OK;
}

fw_status fw_classify_multi_noalloc(const fw_chain_batch* batches, uint32_t n_chains,
                                    const fw_multi_opts* opts) {
    fw_multi_opts o{};
    if (opts) o = *opts;
    if (n_chains > kNoAllocMaxChains)
        return fail(FW_E_INVAL, "fw_classify_multi_noalloc takes at most %u chains (got %u)",
                    kNoAllocMaxChains, n_chains);
    fw_status st = check_batches(batches, n_chains);
    if (st != FW_OK) return st;
    Config cfg;
    st = resolve(batches, n_chains, o, &cfg);
    if (st != FW_OK) return st;
    void* mem = nullptr;
    hipError_t e = scratch_address(&mem);
    if (e != hipSuccess) return hip_fail(e, "looking up the scratch array");
    e = run(batches, n_chains, cfg, static_cast<hipStream_t>(o.stream), mem);
    if (e != hipSuccess) return hip_fail(e, "multi-chain launch (no allocation)");
    return FW_OK;
}

fw_status fw_autotune_multi(const fw_chain_batch* batches, uint32_t n_chains, void* stream,
                            fw_multi_opts* best, float* best_ms) {
    fw_status st = check_batches(batches, n_chains);
    if (st != FW_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t a = nullptr, z = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&z);
    Config win;
    float win_ms = -1.0f;
    const Config placements[] = {{4, 0u, false}, {4, 0u, true}, {4, 256u, false},
                                 {4, 1024u, false}};
    for (int K : {1, 2, 4}) {
        for (Config c : placements) {
            if (e != hipSuccess) break;
            c.K = K;
            e = run(batches, n_chains, c, s);   // warm-up
            float ms_best = -1.0f;
            for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
                e = hipEventRecord(a, s);
                if (e == hipSuccess) e = run(batches, n_chains, c, s);
                if (e == hipSuccess) e = hipEventRecord(z, s);
                if (e == hipSuccess) e = hipEventSynchronize(z);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, z);
                if (e == hipSuccess && (ms_best < 0 || ms < ms_best)) ms_best = ms;
            }
            if (e == hipSuccess && (win_ms < 0 || ms_best < win_ms)) {
                win_ms = ms_best;
                win = c;
            }
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (z) (void)hipEventDestroy(z);
    if (e != hipSuccess) return hip_fail(e, "autotuning");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[shape_key(batches, n_chains)] = win;
    }
    if (best) {
        std::memset(best, 0, sizeof *best);
        best->stream = stream;
        best->packets_per_lane = uint32_t(win.K);
        best->placement = win.tile ? 2u : (win.vector ? 3u : 1u);
        best->rule_tile = win.tile;
    }
    if (best_ms) *best_ms = win_ms;
    return FW_OK;
}

}  // extern "C"
