// Host construction of grouped scan plans (see ScanPlan).
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "fw_internal.h"
#include "lists.h"

namespace fw {
namespace {

uint2 first_pair(const RuleRec& q, uint32_t kind) {
    switch (kind) {
        case kFirstDst: return uint2{q.dst_lo, q.dst_w};
        case kFirstSrc: return uint2{q.src_lo, q.src_w};
        case kFirstPorts: return uint2{q.port_lo, q.port_w};
        default: return uint2{q.proto & 0xFFu, (q.proto >> 8) & 0xFFu};
    }
}

}  // namespace

hipError_t make_plan(const RuleRec* recs, uint32_t n, DevicePlan* out) {
    *out = DevicePlan{};
    PlanGroups pg;
    group_rules(recs, n, &pg);
    const auto& grp = pg.grp;
    ScanPlan plan{};
    plan.tail_idx = pg.tail_idx;
    plan.tail_act = pg.tail_act;
    // one allocation: per group, records then padded pairs, each section 256-B aligned
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t bytes = 0;
    for (auto& g : grp)
        if (!g.empty()) bytes += up(g.size() * sizeof(RuleRec)) + up((g.size() + kPairPadding) * 8);
    std::vector<unsigned char> host(bytes ? bytes : 32, 0);
    void* mem = nullptr;
    hipError_t e = hipMalloc(&mem, host.size());
    if (e != hipSuccess) return e;
    size_t off = 0;
    for (uint32_t k = 0; k < 4; ++k) {
        if (grp[k].empty()) continue;
        ScanGroup& sg = plan.g[plan.n_groups++];
        sg.kind = k;
        sg.count = uint32_t(grp[k].size());
        std::memcpy(host.data() + off, grp[k].data(), grp[k].size() * sizeof(RuleRec));
        sg.recs = reinterpret_cast<const RuleRec*>(static_cast<char*>(mem) + off);
        off += up(grp[k].size() * sizeof(RuleRec));
        for (size_t i = 0; i < grp[k].size(); ++i) {
            const uint2 p = first_pair(grp[k][i], k);
            std::memcpy(host.data() + off + i * 8, &p, 8);
        }
        sg.pairs = reinterpret_cast<const uint2*>(static_cast<char*>(mem) + off);
        off += up((grp[k].size() + kPairPadding) * 8);
    }
    e = hipMemcpy(mem, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return e;
    }
    out->mem = mem;
    out->plan = plan;
    out->bytes = host.size();
    return hipSuccess;
}

void free_plan(DevicePlan* p) {
    if (p->mem) (void)hipFree(p->mem);
    *p = DevicePlan{};
}

}  // namespace fw
