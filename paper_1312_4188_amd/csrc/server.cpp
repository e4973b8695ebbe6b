// Serving runtime: resident rulesets, continuous batching of arriving packet
// batches, admission by a memory budget.
//
// Each slot is one host thread with one HIP stream.  A slot that is free
// admits, in arrival order, every queued request that fits the slot's share
// of the budget (and the largest free block of the arena), up to max_group
// requests: a group.  The group is classified by one multi-chain launch with
// one entry per request (the chain's learned index where one is built, else
// its grouped scan plan), so per-request host work is a descriptor, not a
// launch.  Packets reach the GPU one of two ways:
//  - copy ingest: the group's small requests are packed into page-locked
//    staging and moved by one copy per packet field, the large ones by their
//    own copies straight from their buffers (each request at a 16-packet
//    boundary of the group's device block); the results come back the same
//    way;
//  - mapped ingest: the caller's buffers are page-locked host memory mapped
//    into the device's address space, and the kernel reads the packets and
//    writes the results in place over PCIe, with no copies at all.
// Groups on different slots overlap on the device; each request's result is
// the same as classifying it alone (classification is per packet).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <exception>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/fw.h"
#include "arena.h"
#include "index.h"
#include "multi.h"
#include "guard.h"

namespace fw {
extern thread_local std::string g_last_error;
const ChainView* ruleset_chain_view(const fw_ruleset* rs, const ChainView** host);

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t round256(size_t x) { return (x + 255) & ~size_t(255); }
size_t round16(size_t x) { return (x + 15) & ~size_t(15); }

// Byte offsets of a group of N packets (N a multiple of 16): the five packet
// arrays, then the two result arrays, each 256-byte aligned.  [0, in_bytes)
// is what goes in, [idx, bytes) what comes back.
struct GroupLayout {
    size_t src, dst, sp, dp, pr, idx, act, in_bytes, bytes;
    explicit GroupLayout(size_t N) {
        src = 0;
        dst = src + round256(4 * N);
        sp = dst + round256(4 * N);
        dp = sp + round256(2 * N);
        pr = dp + round256(2 * N);
        idx = pr + round256(N);
        in_bytes = idx;
        act = idx + round256(4 * N);
        bytes = act + round256(N);
    }
};

struct Request {
    uint64_t ticket = 0;
    uint32_t chain = 0;
    fw_host_packets pk{};
    size_t n = 0;
    int32_t* out_idx = nullptr;
    uint8_t* out_act = nullptr;
    fw_request_times times{};
    size_t at = 0;   // first packet inside its group (copy ingest)
    fw_status status = FW_OK;
    std::string error;
    bool done = false;
};

struct Group {
    std::vector<std::shared_ptr<Request>> reqs;
    size_t N = 0;               // packets, each request padded to 16
    size_t off = 0, bytes = 0;  // its block of the arena
};

}  // namespace
}  // namespace fw

struct fw_server {
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        void* d_desc = nullptr;   // descriptor table and counter of its launches
        void* h_desc = nullptr;   // page-locked staging of the same
        std::thread thread;
    };
    std::vector<fw_ruleset*> chains;
    fw_server_opts o{};
    int device = 0;
    char* d_arena = nullptr;   // copy ingest: packed groups on the device ...
    char* h_arena = nullptr;   // ... and their page-locked staging, at the same offsets
    std::unique_ptr<fw::Arena> arena;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<fw::Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<fw::Request>> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
};

namespace fw {
namespace {

constexpr uint32_t kMaxSlots = 16;

// Bytes a request of n packets adds to a group.
size_t request_bytes(size_t n) { return GroupLayout(round16(n)).bytes; }

// Under sv->mu: take queued requests, in arrival order, into a group that
// fits the slot's share of the budget, the arena's largest free block and the
// group caps (requests and packets: every request of a group completes when
// the group does, so the cap bounds what a request waits for beside its own
// work); the first request alone needs only the block.  Returns false (and
// takes nothing) when the first request does not fit yet.
bool admit(fw_server* sv, Group* g) {
    const size_t largest = sv->arena->largest();
    const size_t share = std::max<size_t>(sv->o.mem_budget / sv->o.slots, 1);
    size_t N = 0;
    uint32_t take = 0;
    for (const auto& r : sv->queue) {
        if (take >= sv->o.max_group) break;
        const size_t next = N + round16(r->n);
        const size_t bytes = GroupLayout(next).bytes;
        if (bytes > largest || (take > 0 && (bytes > share || next > sv->o.max_group_packets)))
            break;
        N = next;
        ++take;
    }
    if (take == 0) return false;
    g->N = N;
    g->bytes = GroupLayout(N).bytes;
    if (!sv->arena->alloc(g->bytes, &g->off)) return false;   // cannot happen: fits `largest`
    const double t = now_s();
    for (uint32_t k = 0; k < take; ++k) {
        auto r = sv->queue.front();
        sv->queue.pop_front();
        r->times.admit = t;
        g->reqs.push_back(std::move(r));
    }
    return true;
}

// Copy ingest moves a request of at least this many packets by its own
// copies straight between its buffers and the group's device block (seven
// copies; their fixed cost is below the host copying it twice); smaller ones
// are packed into staging and move with the group's few copies.
constexpr size_t kDirectCopyMin = 4096;

// Copy ingest: the small requests take the front of the group's block, packed
// into staging; the large ones follow.  Every request starts at a 16-packet
// boundary.  Returns the packets of the packed front.
size_t place(Group& g) {
    size_t at = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (auto& r : g.reqs)
            if ((r->n < kDirectCopyMin) == (pass == 0)) {
                r->at = at;
                at += round16(r->n);
            }
    size_t front = 0;
    for (const auto& r : g.reqs)
        if (r->n < kDirectCopyMin) front = std::max(front, r->at + round16(r->n));
    return front;
}

hipError_t copy_in(fw_server* sv, hipStream_t s, const Group& g, const GroupLayout& L,
                   size_t front) {
    char* h = sv->h_arena + g.off;
    char* d = sv->d_arena + g.off;
    hipError_t e = hipSuccess;
    const size_t offs[5] = {L.src, L.dst, L.sp, L.dp, L.pr};
    const size_t width[5] = {4, 4, 2, 2, 1};
    for (const auto& r : g.reqs) {
        const void* src[5] = {r->pk.src_ip, r->pk.dst_ip, r->pk.src_port, r->pk.dst_port,
                              r->pk.proto};
        for (int f = 0; f < 5 && e == hipSuccess; ++f) {
            const size_t at = offs[f] + width[f] * r->at, bytes = width[f] * r->n;
            if (r->n < kDirectCopyMin)
                std::memcpy(h + at, src[f], bytes);
            else
                e = hipMemcpyAsync(d + at, src[f], bytes, hipMemcpyHostToDevice, s);
        }
    }
    for (int f = 0; f < 5 && e == hipSuccess && front; ++f)
        e = hipMemcpyAsync(d + offs[f], h + offs[f], width[f] * front, hipMemcpyHostToDevice, s);
    return e;
}

hipError_t copy_out(fw_server* sv, hipStream_t s, const Group& g, const GroupLayout& L,
                    size_t front) {
    char* h = sv->h_arena + g.off;
    char* d = sv->d_arena + g.off;
    hipError_t e = hipSuccess;
    if (front) e = hipMemcpyAsync(h + L.idx, d + L.idx, 4 * front, hipMemcpyDeviceToHost, s);
    if (front && e == hipSuccess)
        e = hipMemcpyAsync(h + L.act, d + L.act, front, hipMemcpyDeviceToHost, s);
    for (const auto& r : g.reqs) {
        if (r->n < kDirectCopyMin || e != hipSuccess) continue;
        e = hipMemcpyAsync(r->out_idx, d + L.idx + 4 * r->at, 4 * r->n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->out_act, d + L.act + r->at, r->n, hipMemcpyDeviceToHost, s);
    }
    return e;
}

// After the group completed: hand out the packed front's results.
void unpack(fw_server* sv, const Group& g, const GroupLayout& L) {
    const char* h = sv->h_arena + g.off;
    for (const auto& r : g.reqs) {
        if (r->n >= kDirectCopyMin) continue;
        std::memcpy(r->out_idx, h + L.idx + 4 * r->at, 4 * r->n);
        std::memcpy(r->out_act, h + L.act + r->at, r->n);
    }
}

// Classify one group on a slot; returns once its results are in place.
fw_status run_group(fw_server* sv, fw_server::Slot& sl, Group& g) {
    const GroupLayout L(g.N);
    const bool mapped = sv->o.ingest == 1;
    std::vector<fw_chain_batch> b(g.reqs.size());
    hipError_t e = hipSuccess;
    size_t front = 0;
    if (mapped) {
        for (size_t k = 0; k < g.reqs.size(); ++k) {
            const Request& r = *g.reqs[k];
            b[k] = fw_chain_batch{sv->chains[r.chain],
                                  fw_packets{r.pk.src_ip, r.pk.dst_ip, r.pk.src_port,
                                             r.pk.dst_port, r.pk.proto},
                                  r.n, r.out_idx, r.out_act};
        }
    } else {
        front = place(g);
        e = copy_in(sv, sl.stream, g, L, front);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(sl.stream);
            return hip_fail(e, "copying a group's packets in");
        }
        char* d = sv->d_arena + g.off;
        for (size_t k = 0; k < g.reqs.size(); ++k) {
            const Request& r = *g.reqs[k];
            const size_t o = r.at;
            b[k] = fw_chain_batch{
                sv->chains[r.chain],
                fw_packets{reinterpret_cast<const uint32_t*>(d + L.src + 4 * o),
                           reinterpret_cast<const uint32_t*>(d + L.dst + 4 * o),
                           reinterpret_cast<const uint16_t*>(d + L.sp + 2 * o),
                           reinterpret_cast<const uint16_t*>(d + L.dp + 2 * o),
                           reinterpret_cast<const uint8_t*>(d + L.pr + o)},
                r.n, reinterpret_cast<int32_t*>(d + L.idx + 4 * o),
                reinterpret_cast<uint8_t*>(d + L.act + o)};
        }
    }
    MultiConfig cfg;
    cfg.placement = kPlaceAuto;
    cfg.use_index = sv->o.mode != FW_MODE_PACKET_SPLIT;
    cfg.K = g.N >= size_t(8192) * 64u * 2u ? 2 : 1;   // 8,192 waves or more at two per lane
    e = multi_launch(b.data(), uint32_t(b.size()), cfg, sl.stream, sl.d_desc, sl.h_desc);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(sl.stream);
        return hip_fail(e, "group launch");
    }
    if (!mapped) {
        e = copy_out(sv, sl.stream, g, L, front);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(sl.stream);
            return hip_fail(e, "copying a group's results out");
        }
    }
    e = hipEventRecord(sl.done, sl.stream);
    if (e == hipSuccess) e = hipEventSynchronize(sl.done);
    if (e != hipSuccess) return hip_fail(e, "group failed on the device");
    if (!mapped) unpack(sv, g, L);
    return FW_OK;
}

void slot_main(fw_server* sv, uint32_t k) {
    (void)hipSetDevice(sv->device);
    fw_server::Slot& sl = sv->slots[k];
    for (;;) {
        Group g;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] { return (sv->stop && sv->queue.empty()) || admit(sv, &g); });
            if (g.reqs.empty()) break;   // stopping, nothing left
        }
        fw_status st;
        try {   // host allocations inside may throw; a worker thread must not let them escape
            st = run_group(sv, sl, g);
        } catch (const std::exception&) {
            (void)hipStreamSynchronize(sl.stream);
            st = fail(FW_E_NOMEM, "host allocation failed while running a group");
        }
        const std::string err = st != FW_OK ? g_last_error : std::string();
        const double t = now_s();
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->arena->release(g.off, g.bytes);
        for (auto& r : g.reqs) {
            r->status = st;
            r->error = err;
            r->times.done = t;
            r->done = true;
        }
        sv->cv_done.notify_all();
        sv->cv_work.notify_all();   // freed memory may admit another slot's group
    }
}

void destroy_resources(fw_server* sv) {
    for (auto& sl : sv->slots) {
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.d_desc) (void)hipFree(sl.d_desc);
        if (sl.h_desc) (void)hipHostFree(sl.h_desc);
    }
    if (sv->d_arena) (void)hipFree(sv->d_arena);
    if (sv->h_arena) (void)hipHostFree(sv->h_arena);
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace
}  // namespace fw

using namespace fw;

extern "C" {

fw_status fw_server_create(fw_ruleset* const* chains, uint32_t n_chains, const fw_server_opts* opts,
                           fw_server** out) {
    return guarded([&]() -> fw_status {
        if (!out) return fail(FW_E_INVAL, "out is NULL");
        *out = nullptr;
        if (!chains || n_chains == 0) return fail(FW_E_INVAL, "no chains");
        for (uint32_t c = 0; c < n_chains; ++c)
            if (!chains[c]) return fail(FW_E_INVAL, "chain %u is NULL", c);
        fw_server_opts o{};
        if (opts) o = *opts;
        if (o.slots == 0) o.slots = 4;
        if (o.slots > kMaxSlots) return fail(FW_E_INVAL, "at most %u slots", kMaxSlots);
        if (o.max_group == 0) o.max_group = kMultiMaxChains;
        if (o.max_group_packets == 0) o.max_group_packets = uint64_t(1) << 20;
        if (o.max_group > kMultiMaxChains)
            return fail(FW_E_INVAL, "at most %u requests per group", kMultiMaxChains);
        if (o.mem_budget == 0) o.mem_budget = uint64_t(256) << 20;
        if (o.ingest > 1) return fail(FW_E_INVAL, "ingest must be 0 (copies) or 1 (mapped)");
        if (o.mode != FW_MODE_AUTO && o.mode != FW_MODE_PACKET_SPLIT && o.mode != FW_MODE_LEARNED)
            return fail(FW_E_INVAL,
                        "serving mode must be AUTO, PACKET_SPLIT or LEARNED (groups run as one "
                        "multi-chain launch)");
        if (o.mode == FW_MODE_LEARNED) {
            for (uint32_t c = 0; c < n_chains; ++c) {
                const ChainView* hv = nullptr;
                ruleset_chain_view(chains[c], &hv);
                if (!hv->has_index)
                    return fail(FW_E_NOINDEX, "chain %u has no learned index (mode LEARNED)", c);
            }
        }
        // owned here until every resource and worker is in place; a failure on
        // the way (a HIP error, or an exception guarded() turns into a status)
        // frees what was made
        std::unique_ptr<fw_server> own(new fw_server());
        fw_server* sv = own.get();
        sv->chains.assign(chains, chains + n_chains);
        sv->o = o;
        sv->arena = std::make_unique<Arena>(size_t(o.mem_budget));
        sv->slots.resize(o.slots);
        ScopeExit cleanup([sv] { destroy_resources(sv); });   // resources made so far
        hipError_t e = hipGetDevice(&sv->device);
        if (e == hipSuccess && o.ingest == 0)
            e = hipMalloc(reinterpret_cast<void**>(&sv->d_arena), o.mem_budget);
        if (e == hipSuccess && o.ingest == 0)
            e = hipHostMalloc(reinterpret_cast<void**>(&sv->h_arena), o.mem_budget,
                              hipHostMallocDefault);
        for (auto& sl : sv->slots) {
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
            if (e == hipSuccess) e = hipMalloc(&sl.d_desc, kMultiScratchBytes);
            if (e == hipSuccess)
                e = hipHostMalloc(&sl.h_desc, kMultiScratchBytes, hipHostMallocDefault);
        }
        if (e != hipSuccess) return hip_fail(e, "creating the server");
        try {
            for (uint32_t k = 0; k < o.slots; ++k)
                sv->slots[k].thread = std::thread(slot_main, sv, k);
        } catch (...) {   // stop and join the workers already started
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->stop = true;
                sv->cv_work.notify_all();
            }
            for (auto& sl : sv->slots)
                if (sl.thread.joinable()) sl.thread.join();
            throw;
        }
        cleanup.dismiss();
        *out = own.release();
        return FW_OK;
    });
}

fw_status fw_server_submit(fw_server* sv, uint32_t chain, const fw_host_packets* pk, size_t n,
                           int32_t* out_rule_idx, uint8_t* out_action, uint64_t* ticket) {
    return guarded([&]() -> fw_status {
        if (!sv || !ticket) return fail(FW_E_INVAL, "NULL server or ticket");
        if (chain >= sv->chains.size()) return fail(FW_E_INVAL, "chain %u out of range", chain);
        if (n > 0 && (!pk || !pk->src_ip || !pk->dst_ip || !pk->src_port || !pk->dst_port ||
                      !pk->proto || !out_rule_idx || !out_action))
            return fail(FW_E_INVAL, "NULL buffer");
        if (n > 0 && sv->o.ingest == 1 &&
            !(aligned16(pk->src_ip) && aligned16(pk->dst_ip) && aligned16(pk->src_port) &&
              aligned16(pk->dst_port) && aligned16(pk->proto) && aligned16(out_rule_idx) &&
              aligned16(out_action)))
            return fail(FW_E_ALIGN, "mapped ingest needs 16-byte aligned buffers");
        const size_t bytes = request_bytes(n);
        if (bytes > sv->o.mem_budget)
            return fail(FW_E_NOMEM, "request of %zu packets needs %zu bytes, budget %llu", n, bytes,
                        (unsigned long long)sv->o.mem_budget);
        auto r = std::make_shared<Request>();
        r->chain = chain;
        if (pk) r->pk = *pk;
        r->n = n;
        r->out_idx = out_rule_idx;
        r->out_act = out_action;
        r->times.submit = now_s();
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) return fail(FW_E_INVAL, "server is stopping");
        r->ticket = sv->next_ticket++;
        *ticket = r->ticket;
        sv->reqs[r->ticket] = r;
        if (n == 0) {
            r->times.admit = r->times.done = r->times.submit;
            r->done = true;
            return FW_OK;
        }
        sv->queue.push_back(r);
        sv->cv_work.notify_one();
        return FW_OK;
    });
}

fw_status fw_server_wait(fw_server* sv, uint64_t ticket, fw_request_times* times) {
    return guarded([&]() -> fw_status {
        if (!sv) return fail(FW_E_INVAL, "NULL server");
        std::unique_lock<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end())
            return fail(FW_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
        auto r = it->second;
        sv->cv_done.wait(lk, [&] { return r->done; });
        sv->reqs.erase(ticket);
        lk.unlock();
        if (times) *times = r->times;
        if (r->status != FW_OK) g_last_error = r->error;
        return r->status;
    });
}

fw_status fw_server_replay(fw_server* sv, uint32_t n_req, const double* arrival_s,
                           const uint32_t* chain, const size_t* offset, const size_t* n,
                           const fw_host_packets* pool, int32_t* out_idx, uint8_t* out_action,
                           fw_request_times* times) {
    return guarded([&]() -> fw_status {
        if (!sv) return fail(FW_E_INVAL, "NULL server");
        if (n_req == 0) return FW_OK;
        if (!arrival_s || !chain || !offset || !n || !pool || !out_idx || !out_action)
            return fail(FW_E_INVAL, "NULL argument");
        for (uint32_t k = 1; k < n_req; ++k)
            if (arrival_s[k] < arrival_s[k - 1])
                return fail(FW_E_INVAL, "arrivals must not decrease");
        std::vector<uint64_t> tickets(n_req, 0);
        const double t0 = now_s();
        fw_status st = FW_OK;
        uint32_t submitted = 0;
        for (uint32_t k = 0; k < n_req; ++k) {
            // sleep to within 200 us of the arrival, then spin for an exact submit time
            const double due = t0 + arrival_s[k], early = due - 2e-4;
            const double wait = early - now_s();
            if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
            while (now_s() < due) {
            }
            const size_t o = offset[k];
            const fw_host_packets pk{pool->src_ip + o, pool->dst_ip + o, pool->src_port + o,
                                     pool->dst_port + o, pool->proto + o};
            st = fw_server_submit(sv, chain[k], &pk, n[k], out_idx + o, out_action + o,
                                  &tickets[k]);
            if (st != FW_OK) break;
            ++submitted;
        }
        const std::string submit_error = st != FW_OK ? g_last_error : std::string();
        fw_status first_err = st;
        for (uint32_t k = 0; k < submitted; ++k) {
            fw_request_times t{};
            const fw_status w = fw_server_wait(sv, tickets[k], &t);
            if (w != FW_OK && first_err == FW_OK) first_err = w;
            t.submit = t0 + arrival_s[k];
            if (times) times[k] = t;
        }
        if (st != FW_OK) g_last_error = submit_error;
        return first_err;
    });
}

fw_status fw_server_destroy(fw_server* sv) {
    return guarded([&]() -> fw_status {
        if (!sv) return FW_OK;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stop = true;
            sv->cv_work.notify_all();
        }
        for (auto& sl : sv->slots)
            if (sl.thread.joinable()) sl.thread.join();
        hipError_t e = hipSuccess;
        for (auto& sl : sv->slots) {
            const hipError_t e2 = hipStreamSynchronize(sl.stream);
            if (e == hipSuccess) e = e2;
        }
        destroy_resources(sv);
        delete sv;
        if (e != hipSuccess) return hip_fail(e, "destroying the server");
        return FW_OK;
    });
}

}  // extern "C"
