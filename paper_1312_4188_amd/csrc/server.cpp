// Serving runtime: resident rulesets, continuous batching of arriving packet
// batches over several HIP streams, admission by a device-memory budget.
//
// Worker threads (four by default) own the device side, each an equal share
// of the slots.  A request waits in one FIFO queue until a worker has a
// slot (stream) free and the arena can hold its packets and results; it is
// then copied in, classified and copied out by that worker, and an event
// marks its completion.  Several workers issue the HIP calls of different
// requests in parallel (per-request host work is what bounds throughput for
// small requests).  Requests on different slots overlap on the device; each
// is classified exactly as it would be alone.  Copies run either on the
// request's slot stream, or (pipeline mode) on one shared upload stream and
// one shared download stream in admission order, with events ordering
// upload -> classification (slot stream) -> download.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/fw.h"
#include "index.h"

namespace fw {
extern thread_local std::string g_last_error;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t round256(size_t x) { return (x + 255) & ~size_t(255); }

// Device bytes of one request: five packet arrays and two result arrays, each 256-B aligned.
size_t request_bytes(size_t n) {
    return round256(4 * n) * 2 + round256(2 * n) * 2 + round256(n) + round256(4 * n) +
           round256(n);
}

// First-fit allocator over [0, size) with coalescing frees.
class Arena {
   public:
    explicit Arena(size_t size) { free_[0] = size; }
    bool alloc(size_t need, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                const size_t rest = it->second - need, at = it->first + need;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t size) {
        auto it = free_.emplace(off, size).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

   private:
    std::map<size_t, size_t> free_;
};

struct Request {
    uint64_t ticket = 0;
    uint32_t chain = 0;
    fw_host_packets pk{};
    size_t n = 0;
    int32_t* out_idx = nullptr;
    uint8_t* out_act = nullptr;
    fw_request_times times{};
    int slot = -1;
    size_t off = 0, bytes = 0;
    fw_status status = FW_OK;
    std::string error;
    bool done = false;
};

}  // namespace
}  // namespace fw

struct fw_server {
    std::vector<fw_ruleset*> chains;
    fw_server_opts o{};
    int device = 0;
    char* arena_base = nullptr;
    std::unique_ptr<fw::Arena> arena;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    hipStream_t up = nullptr, down = nullptr;        // pipeline mode: shared copy streams
    std::vector<hipEvent_t> ev_up, ev_comp;          // pipeline mode: per-slot stage events
    std::vector<std::shared_ptr<fw::Request>> slot_req;   // worker-owned
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<fw::Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<fw::Request>> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> workers;
};

namespace fw {
namespace {

fw_status launch_request(fw_server* sv, Request& r) {
    hipStream_t s = sv->streams[r.slot];
    char* base = sv->arena_base + r.off;
    const size_t n = r.n;
    auto* src = reinterpret_cast<uint32_t*>(base);
    auto* dst = reinterpret_cast<uint32_t*>(base + round256(4 * n));
    auto* sp = reinterpret_cast<uint16_t*>(base + round256(4 * n) * 2);
    auto* dp = reinterpret_cast<uint16_t*>(base + round256(4 * n) * 2 + round256(2 * n));
    auto* pr = reinterpret_cast<uint8_t*>(base + round256(4 * n) * 2 + round256(2 * n) * 2);
    auto* oi = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(pr) + round256(n));
    auto* oa = reinterpret_cast<uint8_t*>(reinterpret_cast<char*>(oi) + round256(4 * n));
    const bool pipe = sv->o.pipeline != 0;
    hipStream_t in = pipe ? sv->up : s, out = pipe ? sv->down : s;
    hipError_t e = hipMemcpyAsync(src, r.pk.src_ip, 4 * n, hipMemcpyHostToDevice, in);
    if (e == hipSuccess) e = hipMemcpyAsync(dst, r.pk.dst_ip, 4 * n, hipMemcpyHostToDevice, in);
    if (e == hipSuccess) e = hipMemcpyAsync(sp, r.pk.src_port, 2 * n, hipMemcpyHostToDevice, in);
    if (e == hipSuccess) e = hipMemcpyAsync(dp, r.pk.dst_port, 2 * n, hipMemcpyHostToDevice, in);
    if (e == hipSuccess) e = hipMemcpyAsync(pr, r.pk.proto, n, hipMemcpyHostToDevice, in);
    if (pipe && e == hipSuccess) e = hipEventRecord(sv->ev_up[r.slot], in);
    if (pipe && e == hipSuccess) e = hipStreamWaitEvent(s, sv->ev_up[r.slot], 0);
    if (e != hipSuccess) return hip_fail(e, "copying packets in");
    const fw_packets pk{src, dst, sp, dp, pr};
    fw_classify_opts co{};
    co.mode = sv->o.mode;
    co.partitions = sv->o.partitions;
    co.stream = s;
    const fw_status st = fw_classify_ex(sv->chains[r.chain], &pk, n, oi, oa, &co);
    if (st != FW_OK) return st;
    if (pipe) {
        e = hipEventRecord(sv->ev_comp[r.slot], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(out, sv->ev_comp[r.slot], 0);
        if (e != hipSuccess) return hip_fail(e, "ordering the copy out");
    }
    e = hipMemcpyAsync(r.out_idx, oi, 4 * n, hipMemcpyDeviceToHost, out);
    if (e == hipSuccess) e = hipMemcpyAsync(r.out_act, oa, n, hipMemcpyDeviceToHost, out);
    if (e == hipSuccess) e = hipEventRecord(sv->events[r.slot], out);
    if (e != hipSuccess) return hip_fail(e, "copying results out");
    return FW_OK;
}

// Worker owning slots [lo, hi).
void worker_main(fw_server* sv, uint32_t lo, uint32_t hi) {
    (void)hipSetDevice(sv->device);
    std::vector<int> free_slots;
    for (int k = int(hi) - 1; k >= int(lo); --k) free_slots.push_back(k);
    uint32_t mine = 0;   // requests in flight on this worker's slots
    for (;;) {
        std::vector<std::shared_ptr<Request>> admitted;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (mine == 0 && sv->queue.empty()) {
                if (sv->stop) break;
                sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
                continue;
            }
            // admit in arrival order while a slot is free and the memory fits
            while (!sv->queue.empty() && !free_slots.empty()) {
                auto& r = sv->queue.front();
                size_t off = 0;
                if (!sv->arena->alloc(r->bytes, &off)) break;
                r->off = off;
                r->slot = free_slots.back();
                free_slots.pop_back();
                r->times.admit = now_s();
                admitted.push_back(r);
                sv->queue.pop_front();
            }
        }
        bool progressed = !admitted.empty();
        for (auto& r : admitted) {
            sv->slot_req[r->slot] = r;
            r->status = launch_request(sv, *r);
            if (r->status != FW_OK) r->error = g_last_error;
            ++mine;
        }
        // completions
        std::vector<std::shared_ptr<Request>> finished;
        for (uint32_t k = lo; k < hi; ++k) {
            auto& r = sv->slot_req[k];
            if (!r) continue;
            bool complete = r->status != FW_OK;
            if (!complete) {
                const hipError_t q = hipEventQuery(sv->events[k]);
                if (q == hipSuccess) {
                    complete = true;
                } else if (q != hipErrorNotReady) {
                    r->status = hip_fail(q, "request failed on the device");
                    r->error = g_last_error;
                    complete = true;
                }
            }
            if (complete) {
                if (r->status != FW_OK) {
                    (void)hipStreamSynchronize(sv->streams[k]);
                    if (sv->o.pipeline) {
                        (void)hipStreamSynchronize(sv->up);
                        (void)hipStreamSynchronize(sv->down);
                    }
                }
                r->times.done = now_s();
                finished.push_back(r);
                free_slots.push_back(int(k));
                r.reset();
            }
        }
        if (!finished.empty()) {
            progressed = true;
            mine -= uint32_t(finished.size());
            std::lock_guard<std::mutex> lk(sv->mu);
            for (auto& r : finished) {
                sv->arena->release(r->off, r->bytes);
                r->done = true;
            }
            sv->cv_done.notify_all();
            sv->cv_work.notify_all();   // freed memory may admit another worker's request
        }
        if (!progressed) std::this_thread::yield();
    }
}

}  // namespace
}  // namespace fw

using namespace fw;

extern "C" {

fw_status fw_server_create(fw_ruleset* const* chains, uint32_t n_chains, const fw_server_opts* opts,
                           fw_server** out) {
    if (!out) return fail(FW_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!chains || n_chains == 0) return fail(FW_E_INVAL, "no chains");
    for (uint32_t c = 0; c < n_chains; ++c)
        if (!chains[c]) return fail(FW_E_INVAL, "chain %u is NULL", c);
    fw_server_opts o{};
    if (opts) o = *opts;
    if (o.slots == 0) o.slots = 8;
    if (o.slots > 64) return fail(FW_E_INVAL, "at most 64 slots");
    if (o.mem_budget == 0) o.mem_budget = uint64_t(256) << 20;
    if (o.mode > FW_MODE_HYBRID) return fail(FW_E_INVAL, "unknown mode %u", o.mode);
    if (o.pipeline > 1) return fail(FW_E_INVAL, "pipeline must be 0 or 1");
    if (o.workers > 16) return fail(FW_E_INVAL, "at most 16 workers");
    if (o.workers == 0) o.workers = 4;
    if (o.workers > o.slots) o.workers = o.slots;
    fw_server* sv = new (std::nothrow) fw_server();
    if (!sv) return fail(FW_E_NOMEM, "host allocation failed");
    sv->chains.assign(chains, chains + n_chains);
    sv->o = o;
    hipError_t e = hipGetDevice(&sv->device);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&sv->arena_base), o.mem_budget);
    if (e != hipSuccess) {
        delete sv;
        return hip_fail(e, "allocating the server arena");
    }
    sv->arena = std::make_unique<Arena>(size_t(o.mem_budget));
    sv->streams.assign(o.slots, nullptr);
    sv->events.assign(o.slots, nullptr);
    sv->slot_req.assign(o.slots, nullptr);
    sv->ev_up.assign(o.pipeline ? o.slots : 0, nullptr);
    sv->ev_comp.assign(o.pipeline ? o.slots : 0, nullptr);
    for (uint32_t k = 0; k < o.slots && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&sv->streams[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->events[k], hipEventDisableTiming);
        if (o.pipeline && e == hipSuccess)
            e = hipEventCreateWithFlags(&sv->ev_up[k], hipEventDisableTiming);
        if (o.pipeline && e == hipSuccess)
            e = hipEventCreateWithFlags(&sv->ev_comp[k], hipEventDisableTiming);
    }
    if (o.pipeline && e == hipSuccess) e = hipStreamCreateWithFlags(&sv->up, hipStreamNonBlocking);
    if (o.pipeline && e == hipSuccess)
        e = hipStreamCreateWithFlags(&sv->down, hipStreamNonBlocking);
    if (e != hipSuccess) {
        for (auto s : sv->streams)
            if (s) (void)hipStreamDestroy(s);
        for (auto s : {sv->up, sv->down})
            if (s) (void)hipStreamDestroy(s);
        for (auto& evs : {sv->events, sv->ev_up, sv->ev_comp})
            for (auto ev : evs)
                if (ev) (void)hipEventDestroy(ev);
        (void)hipFree(sv->arena_base);
        delete sv;
        return hip_fail(e, "creating server streams");
    }
    for (uint32_t w = 0; w < o.workers; ++w)
        sv->workers.emplace_back(worker_main, sv, w * o.slots / o.workers,
                                 (w + 1) * o.slots / o.workers);
    *out = sv;
    return FW_OK;
}

fw_status fw_server_submit(fw_server* sv, uint32_t chain, const fw_host_packets* pk, size_t n,
                           int32_t* out_rule_idx, uint8_t* out_action, uint64_t* ticket) {
    if (!sv || !ticket) return fail(FW_E_INVAL, "NULL server or ticket");
    if (chain >= sv->chains.size()) return fail(FW_E_INVAL, "chain %u out of range", chain);
    if (n > 0 && (!pk || !pk->src_ip || !pk->dst_ip || !pk->src_port || !pk->dst_port ||
                  !pk->proto || !out_rule_idx || !out_action))
        return fail(FW_E_INVAL, "NULL buffer");
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
    r->bytes = bytes;
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
    sv->cv_work.notify_all();
    return FW_OK;
}

fw_status fw_server_wait(fw_server* sv, uint64_t ticket, fw_request_times* times) {
    if (!sv) return fail(FW_E_INVAL, "NULL server");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return fail(FW_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
    auto r = it->second;
    sv->cv_done.wait(lk, [&] { return r->done; });
    sv->reqs.erase(ticket);
    lk.unlock();
    if (times) *times = r->times;
    if (r->status != FW_OK) g_last_error = r->error;
    return r->status;
}

fw_status fw_server_replay(fw_server* sv, uint32_t n_req, const double* arrival_s,
                           const uint32_t* chain, const size_t* offset, const size_t* n,
                           const fw_host_packets* pool, int32_t* out_idx, uint8_t* out_action,
                           fw_request_times* times) {
    if (!sv) return fail(FW_E_INVAL, "NULL server");
    if (n_req == 0) return FW_OK;
    if (!arrival_s || !chain || !offset || !n || !pool || !out_idx || !out_action)
        return fail(FW_E_INVAL, "NULL argument");
    for (uint32_t k = 1; k < n_req; ++k)
        if (arrival_s[k] < arrival_s[k - 1]) return fail(FW_E_INVAL, "arrivals must not decrease");
    std::vector<uint64_t> tickets(n_req, 0);
    const double t0 = now_s();
    fw_status st = FW_OK;
    uint32_t submitted = 0;
    for (uint32_t k = 0; k < n_req; ++k) {
        const double due = t0 + arrival_s[k];
        while (now_s() < due) {
        }
        const size_t o = offset[k];
        const fw_host_packets pk{pool->src_ip + o, pool->dst_ip + o, pool->src_port + o,
                                 pool->dst_port + o, pool->proto + o};
        st = fw_server_submit(sv, chain[k], &pk, n[k], out_idx + o, out_action + o, &tickets[k]);
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
}

fw_status fw_server_destroy(fw_server* sv) {
    if (!sv) return FW_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv_work.notify_all();
    }
    for (auto& t : sv->workers) t.join();
    hipError_t e = hipSuccess;
    for (auto s : sv->streams) {
        const hipError_t e2 = hipStreamDestroy(s);
        if (e == hipSuccess) e = e2;
    }
    for (auto s : {sv->up, sv->down}) {
        if (!s) continue;
        const hipError_t e2 = hipStreamDestroy(s);
        if (e == hipSuccess) e = e2;
    }
    for (auto& evs : {sv->events, sv->ev_up, sv->ev_comp})
        for (auto ev : evs) (void)hipEventDestroy(ev);
    const hipError_t e3 = hipFree(sv->arena_base);
    if (e == hipSuccess) e = e3;
    delete sv;
    if (e != hipSuccess) return hip_fail(e, "destroying the server");
    return FW_OK;
}

}  // extern "C"
