// Many independent chains (rulesets, each with its own packet batch) in one
// persistent launch, with work-queue scheduling and an autotuner.
//
// Work items are tiles of one chain's packets.  Chains are ordered by an
// estimate of their cost (rules x packets, largest first) so the expensive
// items are handed out first; resident work-groups take items from a global
// counter until none are left, so uneven chains balance themselves.
//
// The default placement classifies each chain the way fw_classify_ex does in
// mode AUTO on a large batch: through its learned index when one is built,
// else by the packet-split wave scan over its grouped plan.  Three more
// placements scan the plain rule list in rule order, as the paper's Section
// IV-A compares global, constant and shared memory for the rule table:
// records read through the scalar cache into SGPRs (each wave takes its own
// 64*K-packet items), the same records read by vector loads into VGPRs, or
// records staged into LDS tiles shared by the four waves of a work-group
// (items of 256*K packets).  The autotuner times the packets-per-lane x
// placement grid on the caller's own batches and caches the fastest choice
// per batch shape.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "../../include/fw.h"
#include "device_util.h"
#include "fw_internal.h"
#include "index.h"
#include "learned_core.h"
#include "multi.h"
#include "scan_core.h"
#include "guard.h"

struct fw_ruleset;

namespace fw {

// Read-only view of a loaded ruleset (defined in api.cpp): the device copy,
// and its host mirror in *host.
const ChainView* ruleset_chain_view(const fw_ruleset* rs, const ChainView** host);

static_assert(sizeof(ChainDesc) == 104, "descriptor layout");

namespace {

constexpr uint32_t kDescPerChunk = 32;   // 3.25 KiB of kernel arguments per upload launch

// Scratch of fw_classify_multi_noalloc: the work-queue counter, then the
// descriptor table of up to kMultiMaxChains chains (see kMultiScratchBytes),
// in one static device array (each GPU the library runs on holds its own copy
// for the life of the process).  Host code never passes the array's name to a
// kernel: it takes the array's device address from hipGetSymbolAddress, once
// per device.
__device__ __align__(256) unsigned char scratch[kMultiScratchBytes];

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

__device__ __forceinline__ PacketsDev packets_of(const ChainDesc& c) {
    return PacketsDev{c.src, c.dst, c.sport, c.dport, c.proto};
}

// Default placement: work-groups of 16 waves take items of 1024*K packets.  A
// chain with a learned index (and use_index set) goes through the learned
// lookup: the work-group stages that index's LDS image when its previous item
// was of another chain (B_LDS: the image with the boundary arrays, chosen per
// chain when it fits the LDS budget, as the single-chain kernel chooses per
// index; the launch's LDS is the largest image its chains use); the others
// through the grouped-plan wave scan,
// which needs no LDS.  Staging follows the two barriers of the item fetch, so
// no wave still reads the image it replaces.
// The two kinds of item as separate functions: each gets the kernel's whole
// register budget, where one inlined body holding both would spill.
template <int K, bool B_LDS>
__device__ __attribute__((noinline)) void auto_learned_item(const ChainDesc& c, size_t base,
                                                             unsigned char* smem, bool stage) {
    const ChainView& v = *c.view;
    const IndexView iv = stage ? stage_index<B_LDS>(v.la, smem) : index_view<B_LDS>(v.la, smem);
    if (base < c.n)
        learned_tile<K, true>(v.la, iv, packets_of(c), base, c.n, c.out_idx, c.out_act, v.dflt);
}

template <int K>
__device__ __attribute__((noinline)) void auto_scan_item(const ChainDesc& c, size_t base) {
    const ChainView& v = *c.view;
    WaveScan<K> w;
    w.init(packets_of(c), base, c.n, c.dflt);
    w.scan_plan(v.plan);
    w.store(c.out_idx, c.out_act, c.n);
}

template <int K>
__global__ __launch_bounds__(kLearnedBlock, K >= 4 ? 4 : 8) void k_multi_auto(
    const ChainDesc* __restrict__ cd, uint32_t n_chains, uint32_t total_items,
    uint32_t* __restrict__ counter, uint32_t use_index) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_item;
    const size_t wave_off = size_t(wave_in_group()) * 64u * K;
    const ChainView* staged = nullptr;   // whose image is in LDS (work-group uniform)
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= total_items) break;
        const ChainDesc& c = cd[chain_of(cd, n_chains, item)];
        const size_t base = size_t(item - c.item_begin) * (size_t(kLearnedBlock) * K) + wave_off;
        if (use_index && (c.index & kChainIndexed)) {
            if (c.index & kChainBoundariesInLds)
                auto_learned_item<K, true>(c, base, smem, staged != c.view);
            else
                auto_learned_item<K, false>(c, base, smem, staged != c.view);
            staged = c.view;
        } else if (base < c.n) {
            auto_scan_item<K>(c, base);
        }
    }
}

// The default placement when every chain of the launch has a learned index
// (and use_index is set): the same items and staging as k_multi_auto, with
// the learned tile inlined into the kernel (no scan item beside it, so no
// call and none of its register spills).  BL: every chain's boundary arrays
// in LDS (kBlAll), none (kBlNone), or chosen per chain (kBlMixed, both
// variants of the tile in one body).
constexpr int kBlNone = 0, kBlAll = 1, kBlMixed = 2;

template <int K, int BL>
__global__ __launch_bounds__(kLearnedBlock, K >= 4 ? 4 : 8) void k_multi_learned(
    const ChainDesc* __restrict__ cd, uint32_t n_chains, uint32_t total_items,
    uint32_t* __restrict__ counter) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_item;
    const size_t wave_off = size_t(wave_in_group()) * 64u * K;
    const ChainView* staged = nullptr;   // whose image is in LDS (work-group uniform)
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= total_items) break;
        const ChainDesc& c = cd[chain_of(cd, n_chains, item)];
        const size_t base = size_t(item - c.item_begin) * (size_t(kLearnedBlock) * K) + wave_off;
        const ChainView& v = *c.view;
        const bool stage = staged != c.view;
        staged = c.view;
        if (BL == kBlAll || (BL == kBlMixed && (c.index & kChainBoundariesInLds))) {
            const IndexView iv = stage ? stage_index<true>(v.la, smem) : index_view<true>(v.la, smem);
            if (base < c.n)
                learned_tile<K, true>(v.la, iv, packets_of(c), base, c.n, c.out_idx, c.out_act,
                                      v.dflt);
        } else {
            const IndexView iv =
                stage ? stage_index<false>(v.la, smem) : index_view<false>(v.la, smem);
            if (base < c.n)
                learned_tile<K, true>(v.la, iv, packets_of(c), base, c.n, c.out_idx, c.out_act,
                                      v.dflt);
        }
    }
}

// The default placement when no chain of the launch is looked up through a
// learned index: the same items with the grouped-plan wave scan inlined (no
// call, no LDS).
template <int K>
__global__ __launch_bounds__(kLearnedBlock, K >= 4 ? 4 : 8) void k_multi_scan(
    const ChainDesc* __restrict__ cd, uint32_t n_chains, uint32_t total_items,
    uint32_t* __restrict__ counter) {
    __shared__ uint32_t s_item;
    const size_t wave_off = size_t(wave_in_group()) * 64u * K;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= total_items) break;
        const ChainDesc& c = cd[chain_of(cd, n_chains, item)];
        const size_t base = size_t(item - c.item_begin) * (size_t(kLearnedBlock) * K) + wave_off;
        if (base < c.n) {
            WaveScan<K> w;
            w.init(packets_of(c), base, c.n, c.dflt);
            w.scan_plan(c.view->plan);
            w.store(c.out_idx, c.out_act, c.n);
        }
    }
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
        scan_wave<K>(c.pairs, c.rules, c.n_rules, packets_of(c), first, c.n, c.out_idx,
                     c.out_act, c.dflt);
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
        WaveScan<K> w;
        w.init(packets_of(c), first, c.n, c.dflt);
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
        WaveScan<K> w;
        const bool active = first < c.n;
        if (active) w.init(packets_of(c), first, c.n, c.dflt);
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

std::mutex g_tune_mu;
std::map<std::vector<uint64_t>, MultiConfig> g_tuned;

std::vector<uint64_t> shape_key(const fw_chain_batch* b, uint32_t n) {
    std::vector<uint64_t> key;
    key.reserve(2 * size_t(n));
    for (uint32_t c = 0; c < n; ++c) {
        key.push_back(fw_ruleset_size(b[c].rs));
        key.push_back(b[c].n);
    }
    return key;
}

// Resident work-groups per CU for (kernel, device, dynamic LDS), queried once
// per device and size: a serving loop's small launches should not pay for
// occupancy queries.
// The largest dynamic LDS size granted to each kernel so far only grows, so a
// launch never finds it lowered by a smaller request.
std::mutex g_occ_mu;
std::map<std::tuple<const void*, int, size_t>, int> g_occ;
std::map<std::pair<const void*, int>, size_t> g_granted;
std::map<int, int> g_cus;

template <class Kern>
hipError_t persistent_grid(Kern kern, uint32_t block, size_t lds, uint32_t items,
                           uint32_t* grid) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const void* f = reinterpret_cast<const void*>(kern);
    std::lock_guard<std::mutex> lk(g_occ_mu);
    auto cu = g_cus.find(dev);
    if (cu == g_cus.end()) {
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        cu = g_cus.emplace(dev, cus).first;
    }
    const auto key = std::make_tuple(f, dev, lds);
    auto it = g_occ.find(key);
    if (it == g_occ.end()) {
        size_t& granted = g_granted[std::make_pair(f, dev)];
        if (lds > granted) {   // above the default dynamic LDS limit the kernel must opt in
            e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
            if (e != hipSuccess) return e;
            granted = lds;
        }
        int per_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, int(block), lds);
        if (e != hipSuccess) return e;
        it = g_occ.emplace(key, per_cu).first;
    }
    if (it->second < 1) return hipErrorInvalidConfiguration;
    const uint32_t g = uint32_t(it->second * std::max(1, cu->second));
    *grid = std::max(1u, std::min(g, items));
    return hipSuccess;
}

// LDS budget of the learned lookup per packets-per-lane, as in the
// single-chain kernel: two work-groups per CU at one or two packets per lane.
uint32_t lds_cap_for(int K) { return K >= 4 ? 150u * 1024u : 80u * 1024u; }

}  // namespace

hipError_t multi_launch(const fw_chain_batch* b, uint32_t n_chains, MultiConfig cfg,
                        hipStream_t s, void* scratch_mem, void* host_staging) {
    // Order: rulesets by estimated cost (rules x their packets in this launch),
    // largest first, so the expensive items are handed out first; a ruleset's
    // entries side by side, largest first (a work-group then stages a learned
    // index once per run of its items); empty batches skipped.
    std::vector<uint32_t> order;
    std::map<const fw_ruleset*, double> share;
    for (uint32_t c = 0; c < n_chains; ++c) {
        if (!b[c].n) continue;
        order.push_back(c);
        share[b[c].rs] += double(b[c].n);
    }
    if (order.empty()) return hipSuccess;
    std::vector<double> cost(n_chains, 0.0);
    for (uint32_t c : order) cost[c] = double(fw_ruleset_size(b[c].rs) + 1) * share[b[c].rs];
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        if (cost[x] != cost[y]) return cost[x] > cost[y];
        if (b[x].rs != b[y].rs) return std::less<const fw_ruleset*>()(b[x].rs, b[y].rs);
        return b[x].n > b[y].n;
    });
    const uint64_t rows = cfg.placement == kPlaceAuto ? uint64_t(kLearnedBlock)
                          : cfg.placement == kPlaceLds ? 256u
                                                       : 64u;
    const uint64_t per_item = rows * uint64_t(cfg.K);
    const uint32_t nc = uint32_t(order.size());
    if (scratch_mem && nc > kMultiMaxChains) return hipErrorInvalidValue;
    std::vector<ChainDesc> local;
    ChainDesc* desc = nullptr;
    if (host_staging) {
        desc = reinterpret_cast<ChainDesc*>(static_cast<char*>(host_staging) + kMultiCounterBytes);
    } else {
        local.resize(nc);
        desc = local.data();
    }
    uint64_t items = 0;
    const uint32_t cap = lds_cap_for(cfg.K);
    size_t lds = 0;   // the largest learned image the launch's chains use
    bool all_learned = cfg.placement == kPlaceAuto && cfg.use_index;
    // chains looked up through their index (none unless the default placement
    // takes indexes), and those of them whose boundary arrays go to LDS
    uint32_t n_in_lds = 0, n_indexed = 0;
    for (uint32_t k = 0; k < nc; ++k) {
        const fw_chain_batch& cb = b[order[k]];
        ChainDesc& d = desc[k];
        std::memset(&d, 0, sizeof d);
        const ChainView* hv = nullptr;
        d.view = ruleset_chain_view(cb.rs, &hv);
        d.rules = hv->rules;
        d.pairs = hv->pairs;
        d.n_rules = hv->n_rules;
        d.dflt = hv->dflt;
        d.index = hv->has_index ? kChainIndexed : 0u;
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
        if (!hv->has_index) all_learned = false;
        if (cfg.placement == kPlaceAuto && cfg.use_index && hv->has_index) {
            const bool b_lds = hv->lds_b <= cap;
            if (b_lds) d.index |= kChainBoundariesInLds;
            n_in_lds += b_lds ? 1u : 0u;
            ++n_indexed;
            lds = std::max<size_t>(lds, b_lds ? hv->lds_b : hv->lds_nob);
        }
    }
    if (items >= 0xFFFFFFFFull) return hipErrorInvalidValue;
    void* mem = scratch_mem;
    hipError_t e = hipSuccess;
    if (!scratch_mem) e = hipMallocAsync(&mem, kMultiCounterBytes + sizeof(ChainDesc) * nc, s);
    if (e != hipSuccess) return e;
    // released on the stream below; this frees it when a step in between throws
    // (the occupancy cache allocates)
    ScopeExit release_on_throw([&] { (void)hipFreeAsync(mem, s); });
    if (scratch_mem) release_on_throw.dismiss();
    uint32_t* counter = static_cast<uint32_t*>(mem);
    ChainDesc* table = reinterpret_cast<ChainDesc*>(static_cast<char*>(mem) + kMultiCounterBytes);
    if (host_staging) {
        // the counter (cleared) and the table in one copy from page-locked memory
        std::memset(host_staging, 0, kMultiCounterBytes);
        e = hipMemcpyAsync(mem, host_staging, kMultiCounterBytes + sizeof(ChainDesc) * nc,
                           hipMemcpyHostToDevice, s);
    } else {
        for (uint32_t at = 0; at < nc && e == hipSuccess; at += kDescPerChunk) {
            DescChunk ch{};
            const uint32_t cnt = std::min(kDescPerChunk, nc - at);
            std::memcpy(ch.d, desc + at, sizeof(ChainDesc) * cnt);
            hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(kDescPerChunk), 0, s, ch, cnt, table,
                               at, counter);
            e = hipGetLastError();
        }
    }
    uint32_t grid = 1;
    const uint32_t total = uint32_t(items);
#define FW_MULTI(KERN)                                                                      \
    do {                                                                                    \
        if (e == hipSuccess) e = persistent_grid(KERN, 256, 0, total, &grid);               \
        if (e == hipSuccess) {                                                              \
            hipLaunchKernelGGL(KERN, dim3(grid), dim3(256), 0, s, table, nc, total, counter); \
            e = hipGetLastError();                                                          \
        }                                                                                   \
    } while (0)
#define FW_MULTI_LEARNED(KK, BL)                                                            \
    do {                                                                                    \
        if (e == hipSuccess)                                                                \
            e = persistent_grid(k_multi_learned<KK, BL>, kLearnedBlock, lds, total, &grid); \
        if (e == hipSuccess) {                                                              \
            hipLaunchKernelGGL((k_multi_learned<KK, BL>), dim3(grid), dim3(kLearnedBlock),  \
                               lds, s, table, nc, total, counter);                          \
            e = hipGetLastError();                                                          \
        }                                                                                   \
    } while (0)
#define FW_MULTI_AUTO(KK)                                                                   \
    do {                                                                                    \
        if (all_learned && n_in_lds == n_indexed) {                                         \
            FW_MULTI_LEARNED(KK, kBlAll);                                                   \
        } else if (all_learned && n_in_lds == 0) {                                          \
            FW_MULTI_LEARNED(KK, kBlNone);                                                  \
        } else if (all_learned) {                                                           \
            FW_MULTI_LEARNED(KK, kBlMixed);                                                 \
        } else if (n_indexed == 0) {                                                        \
            if (e == hipSuccess)                                                            \
                e = persistent_grid(k_multi_scan<KK>, kLearnedBlock, 0, total, &grid);      \
            if (e == hipSuccess) {                                                          \
                hipLaunchKernelGGL((k_multi_scan<KK>), dim3(grid), dim3(kLearnedBlock), 0,  \
                                   s, table, nc, total, counter);                           \
                e = hipGetLastError();                                                      \
            }                                                                               \
        } else {                                                                            \
            if (e == hipSuccess)                                                            \
                e = persistent_grid(k_multi_auto<KK>, kLearnedBlock, lds, total, &grid);    \
            if (e == hipSuccess) {                                                          \
                hipLaunchKernelGGL((k_multi_auto<KK>), dim3(grid), dim3(kLearnedBlock),     \
                                   lds, s, table, nc, total, counter,                       \
                                   uint32_t(cfg.use_index));                                \
                e = hipGetLastError();                                                      \
            }                                                                               \
        }                                                                                   \
    } while (0)
    switch (cfg.placement) {
        case kPlaceAuto:
            if (cfg.K == 1) FW_MULTI_AUTO(1);
            else if (cfg.K == 2) FW_MULTI_AUTO(2);
            else FW_MULTI_AUTO(4);
            break;
        case kPlaceVector:
            if (cfg.K == 1) FW_MULTI(k_multi_vector<1>);
            else if (cfg.K == 2) FW_MULTI(k_multi_vector<2>);
            else FW_MULTI(k_multi_vector<4>);
            break;
        case kPlaceScalar:
            if (cfg.K == 1) FW_MULTI(k_multi_scalar<1>);
            else if (cfg.K == 2) FW_MULTI(k_multi_scalar<2>);
            else FW_MULTI(k_multi_scalar<4>);
            break;
        default:
            if (cfg.tile == 256) {
                if (cfg.K == 1) FW_MULTI((k_multi_lds<1, 256>));
                else if (cfg.K == 2) FW_MULTI((k_multi_lds<2, 256>));
                else FW_MULTI((k_multi_lds<4, 256>));
            } else {
                if (cfg.K == 1) FW_MULTI((k_multi_lds<1, 1024>));
                else if (cfg.K == 2) FW_MULTI((k_multi_lds<2, 1024>));
                else FW_MULTI((k_multi_lds<4, 1024>));
            }
            break;
    }
#undef FW_MULTI_AUTO
#undef FW_MULTI_LEARNED
#undef FW_MULTI
    if (scratch_mem) return e;
    release_on_throw.dismiss();
    const hipError_t e2 = hipFreeAsync(mem, s);
    return e != hipSuccess ? e : e2;
}

fw_status check_multi_batches(const fw_chain_batch* b, uint32_t n) {
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

namespace {

fw_status resolve(const fw_chain_batch* b, uint32_t n, const fw_multi_opts& o, MultiConfig* cfg) {
    if (o.packets_per_lane != 0 && o.packets_per_lane != 1 && o.packets_per_lane != 2 &&
        o.packets_per_lane != 4)
        return fail(FW_E_INVAL, "packets_per_lane must be 0, 1, 2 or 4");
    if (o.placement > 4) return fail(FW_E_INVAL, "placement must be 0 to 4");
    if (o.rule_tile != 0 && o.rule_tile != 256 && o.rule_tile != 1024)
        return fail(FW_E_INVAL, "rule_tile must be 0, 256 or 1024");
    MultiConfig c;   // untuned default: grouped plan / learned index, 2 packets per lane
    if (o.placement == 0 || o.packets_per_lane == 0) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(shape_key(b, n));
        if (it != g_tuned.end()) c = it->second;
    }
    if (o.packets_per_lane) c.K = int(o.packets_per_lane);
    if (o.placement != 0) c.placement = o.placement;
    if (c.placement == kPlaceLds) c.tile = o.rule_tile ? o.rule_tile : (c.tile ? c.tile : 1024u);
    *cfg = c;
    return FW_OK;
}

}  // namespace
}  // namespace fw

using namespace fw;

extern "C" {

fw_status fw_classify_multi(const fw_chain_batch* batches, uint32_t n_chains,
                            const fw_multi_opts* opts) {
    return guarded([&]() -> fw_status {
        fw_multi_opts o{};
        if (opts) o = *opts;
        fw_status st = check_multi_batches(batches, n_chains);
        if (st != FW_OK) return st;
        MultiConfig cfg;
        st = resolve(batches, n_chains, o, &cfg);
        if (st != FW_OK) return st;
        const hipError_t e = multi_launch(batches, n_chains, cfg,
                                          static_cast<hipStream_t>(o.stream), nullptr, nullptr);
        if (e != hipSuccess) return hip_fail(e, "multi-chain launch");
        return FW_OK;
    });
}

fw_status fw_classify_multi_noalloc(const fw_chain_batch* batches, uint32_t n_chains,
                                    const fw_multi_opts* opts) {
    return guarded([&]() -> fw_status {
        fw_multi_opts o{};
        if (opts) o = *opts;
        if (n_chains > kMultiMaxChains)
            return fail(FW_E_INVAL, "fw_classify_multi_noalloc takes at most %u chains (got %u)",
                        kMultiMaxChains, n_chains);
        fw_status st = check_multi_batches(batches, n_chains);
        if (st != FW_OK) return st;
        MultiConfig cfg;
        st = resolve(batches, n_chains, o, &cfg);
        if (st != FW_OK) return st;
        void* mem = nullptr;
        hipError_t e = scratch_address(&mem);
        if (e != hipSuccess) return hip_fail(e, "looking up the scratch array");
        e = multi_launch(batches, n_chains, cfg, static_cast<hipStream_t>(o.stream), mem, nullptr);
        if (e != hipSuccess) return hip_fail(e, "multi-chain launch (no allocation)");
        return FW_OK;
    });
}

fw_status fw_autotune_multi(const fw_chain_batch* batches, uint32_t n_chains, void* stream,
                            fw_multi_opts* best, float* best_ms) {
    return guarded([&]() -> fw_status {
        fw_status st = check_multi_batches(batches, n_chains);
        if (st != FW_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        hipEvent_t a = nullptr, z = nullptr;
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&z);
        MultiConfig win;
        float win_ms = -1.0f;
        MultiConfig placements[5];
        placements[0].placement = kPlaceAuto;
        placements[1].placement = kPlaceScalar;
        placements[2].placement = kPlaceVector;
        placements[3].placement = kPlaceLds;
        placements[3].tile = 256;
        placements[4].placement = kPlaceLds;
        placements[4].tile = 1024;
        // the GPU reaches its steady clocks only after some tens of milliseconds of
        // sustained work: run the default configuration that long before timing any
        const auto t0 = std::chrono::steady_clock::now();
        while (e == hipSuccess &&
               std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(30)) {
            e = multi_launch(batches, n_chains, MultiConfig{}, s, nullptr, nullptr);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
        for (int K : {1, 2, 4}) {
            for (MultiConfig c : placements) {
                if (e != hipSuccess) break;
                c.K = K;
                e = multi_launch(batches, n_chains, c, s, nullptr, nullptr);   // warm-up
                float ms_best = -1.0f;
                for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
                    e = hipEventRecord(a, s);
                    if (e == hipSuccess)
                        e = multi_launch(batches, n_chains, c, s, nullptr, nullptr);
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
            best->placement = win.placement;
            best->rule_tile = win.tile;
        }
        if (best_ms) *best_ms = win_ms;
        return FW_OK;
    });
}

}  // extern "C"
