// Host-only parts of the library under the address and undefined-behaviour
// sanitizers: the arena allocator of the serving runtime, the candidate lists
// and lookup tables of the learned index, the grouping of a rule list into a
// scan plan, and the guard that keeps C++ exceptions from crossing the C
// interface.  Each is driven with seeded random inputs and edge cases
// and checked against a brute-force definition written here.  Exit status 0
// when every check passes.
#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <new>
#include <stdexcept>
#include <string>
#include <system_error>
#include <vector>

#include "../../paper_1312_4188_amd/csrc/arena.h"
#include "../../paper_1312_4188_amd/csrc/guard.h"
#include "../../paper_1312_4188_amd/csrc/lists.h"

// The library's fail() (which records the message for fw_last_error) lives
// with the HIP code; guarded() only needs its contract: record, return st.
static std::string g_last_message;
fw_status fw::fail(fw_status st, const char* fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_message = buf;
    return st;
}

using fw::RuleRec;

namespace {

int g_failures = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);            \
            std::fprintf(stderr, "\n");                   \
            if (++g_failures > 20) std::exit(1);          \
        }                                                 \
    } while (0)

struct Rng {   // splitmix64
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    uint32_t u32() { return uint32_t(next() >> 32); }
    uint32_t below(uint32_t n) { return uint32_t((next() >> 11) % n); }
};

void prefix(uint32_t base, uint32_t len, uint32_t* lo, uint32_t* w) {
    const uint32_t mask = len == 0 ? 0u : (0xFFFFFFFFu << (32u - len));
    *lo = base & mask;
    *w = ~mask;
}

// A random compiled rule: prefix lengths from {0, 8, 16, 24, 32} (or only
// the short ones with `wide`), ports 40% wildcard / 30% exact / 30% range,
// protocol 6, 17 or any.
RuleRec random_rule(Rng& g, uint32_t idx, bool wide) {
    static const uint32_t lens[5] = {0, 8, 16, 24, 32};
    RuleRec q{};
    prefix(g.u32(), wide ? lens[g.below(3)] : lens[g.below(5)], &q.src_lo, &q.src_w);
    prefix(g.u32(), wide ? lens[g.below(3)] : lens[g.below(5)], &q.dst_lo, &q.dst_w);
    uint32_t plo[2], pw[2];
    for (int f = 0; f < 2; ++f) {
        const uint32_t k = g.below(10), a = g.below(65536);
        if (k < 4) {
            plo[f] = 0;
            pw[f] = 65535;
        } else if (k < 7) {
            plo[f] = a;
            pw[f] = 0;
        } else {
            plo[f] = a;
            pw[f] = std::min<uint32_t>(g.below(4096), 65535 - a);
        }
    }
    q.port_lo = (plo[0] << 16) | plo[1];
    q.port_w = (pw[0] << 16) | pw[1];
    const uint32_t p = g.below(3);
    q.proto = (p == 0 ? 6u : p == 1 ? 17u : 0u) | ((p == 2 ? 255u : 0u) << 8) | (g.below(2) << 16);
    q.idx = idx;
    return q;
}

RuleRec catch_all(uint32_t idx) {
    RuleRec q{};
    q.src_w = q.dst_w = q.port_w = 0xFFFFFFFFu;
    q.proto = 255u << 8;
    q.idx = idx;
    return q;
}

bool in(uint32_t v, uint32_t lo, uint32_t w) { return v - lo <= w; }

bool matches(const RuleRec& q, uint32_t s, uint32_t d, uint32_t sp, uint32_t dp, uint32_t pr) {
    return in(s, q.src_lo, q.src_w) && in(d, q.dst_lo, q.dst_w) &&
           in(sp, q.port_lo >> 16, q.port_w >> 16) && in(dp, q.port_lo & 0xFFFFu, q.port_w & 0xFFFFu) &&
           in(pr, q.proto & 0xFFu, (q.proto >> 8) & 0xFFu);
}

uint32_t brute(const std::vector<RuleRec>& r, uint32_t s, uint32_t d, uint32_t sp, uint32_t dp,
               uint32_t pr) {
    for (const RuleRec& q : r)
        if (matches(q, s, d, sp, dp, pr)) return q.idx;
    return fw::kNoMatch;
}

uint32_t interval_of(const std::vector<uint32_t>& B, uint32_t x) {
    return uint32_t(std::upper_bound(B.begin(), B.end(), x) - B.begin()) - 1u;
}

// A packet: half inside a random rule's box, half uniform.
void packet(Rng& g, const std::vector<RuleRec>& r, uint32_t* s, uint32_t* d, uint32_t* sp,
            uint32_t* dp, uint32_t* pr) {
    if (!r.empty() && g.below(2)) {
        const RuleRec& q = r[g.below(uint32_t(r.size()))];
        *s = q.src_lo + uint32_t(uint64_t(g.u32()) % (uint64_t(q.src_w) + 1));
        *d = q.dst_lo + uint32_t(uint64_t(g.u32()) % (uint64_t(q.dst_w) + 1));
        *sp = (q.port_lo >> 16) + g.below((q.port_w >> 16) + 1);
        *dp = (q.port_lo & 0xFFFFu) + g.below((q.port_w & 0xFFFFu) + 1);
        *pr = (q.proto & 0xFFu) + g.below(((q.proto >> 8) & 0xFFu) + 1);
    } else {
        *s = g.u32();
        *d = g.u32();
        *sp = g.below(65536);
        *dp = g.below(65536);
        *pr = g.below(256);
    }
}

void check_lists(const std::vector<RuleRec>& rules, Rng& g, const char* what) {
    const uint32_t R = uint32_t(rules.size());
    fw::HostLists hl;
    CHECK(fw::build_lists(rules.data(), R, &hl), "%s: build_lists failed", what);
    CHECK(!hl.B.empty() && hl.B[0] == 0 && std::is_sorted(hl.B.begin(), hl.B.end()),
          "%s: boundaries", what);
    CHECK(hl.off.size() == hl.B.size() + 1 && hl.off.back() == hl.L_idx.size() &&
              hl.L.size() == hl.L_idx.size(),
          "%s: list offsets", what);
    CHECK(hl.soff.size() == hl.Bs.size() + 1 && hl.soff.back() == hl.S_idx.size(),
          "%s: source offsets", what);
    fw::PortTable pt;
    uint32_t count = 0, steps_s = 0, steps_d = 0;
    std::vector<RuleRec> rest;
    fw::build_port_table(hl.Gw, &pt, &count, &steps_s, &steps_d, &rest);
    CHECK(count <= fw::kPtRules && count + rest.size() == hl.Gw.size(), "%s: port table split",
          what);
    // the lookup scans the rules past the table without address tests: grouped,
    // they form port- and protocol-first groups only
    fw::PlanGroups rg;
    fw::group_rules(rest.data(), uint32_t(rest.size()), &rg);
    CHECK(rg.grp[fw::kFirstDst].empty() && rg.grp[fw::kFirstSrc].empty(),
          "%s: an address-first group past the port table", what);
    std::vector<uint16_t> bucket;
    uint32_t bits = 0, bsteps = 0;
    fw::build_bucket_table(hl.Bs, &bucket, &bits, &bsteps);
    CHECK(bits == 0 || (bucket.size() == (size_t(1) << bits) && bsteps <= 8), "%s: buckets", what);
    for (int t = 0; t < 20000; ++t) {
        uint32_t s, d, sp, dp, pr;
        packet(g, rules, &s, &d, &sp, &dp, &pr);
        const uint32_t want = brute(rules, s, d, sp, dp, pr);
        // first match over the lists: the destination interval's list, the source
        // interval's list of destination-wildcard rules, and the address-wildcard rules
        uint32_t best = fw::kNoMatch;
        const uint32_t j = interval_of(hl.B, d);
        for (uint32_t k = hl.off[j]; k < hl.off[j + 1]; ++k)
            if (matches(hl.L[k], s, d, sp, dp, pr)) best = std::min(best, hl.L[k].idx);
        if (!hl.Bs.empty()) {
            uint32_t i = interval_of(hl.Bs, s);
            if (bits) {   // the bucket walk lands on the same interval
                uint32_t w = bucket[s >> (32 - bits)];
                for (uint32_t k = 0; k < bsteps; ++k)
                    w += (w + 1 < hl.Bs.size() && hl.Bs[w + 1] <= s) ? 1u : 0u;
                CHECK(w == i, "%s: bucket walk %u != %u", what, w, i);
            }
            for (uint32_t k = hl.soff[i]; k < hl.soff[i + 1]; ++k)
                if (matches(hl.S[k], s, d, sp, dp, pr)) best = std::min(best, hl.S[k].idx);
        }
        // the port/protocol table's first rule, then the rest of the wildcard list
        uint32_t is = pt.bucket_s[sp >> 8], id = pt.bucket_d[dp >> 8];
        for (uint32_t k = 0; k < steps_s; ++k) is += pt.b_s[is + 1] <= sp ? 1u : 0u;
        for (uint32_t k = 0; k < steps_d; ++k) id += pt.b_d[id + 1] <= dp ? 1u : 0u;
        CHECK(is < fw::kPtMaxIv && id < fw::kPtMaxIv, "%s: port walk out of range", what);
        const uint64_t m = pt.mask_s[is] & pt.mask_d[id] & pt.mask_p[pr];
        const uint32_t e = pt.rule[m ? __builtin_ctzll(m) : fw::kPtRules];
        if (e != fw::kPtNone) best = std::min(best, e & 0xFFFFFFu);
        for (const RuleRec& q : rest)
            if (matches(q, s, d, sp, dp, pr)) best = std::min(best, q.idx);
        CHECK(best == want, "%s: packet %d first match %u, want %u", what, t, best, want);
    }
    // plan grouping: the rules before the first catch-all, each once, in order
    fw::PlanGroups pg;
    fw::group_rules(rules.data(), R, &pg);
    uint32_t cut = R;
    for (uint32_t r = 0; r < R; ++r)
        if (fw::is_catch_all(rules[r])) {
            cut = r;
            break;
        }
    CHECK(pg.tail_idx == (cut < R ? rules[cut].idx : fw::kNoMatch), "%s: plan tail", what);
    size_t total = 0;
    for (uint32_t k = 0; k < 4; ++k) {
        total += pg.grp[k].size();
        for (size_t i = 0; i < pg.grp[k].size(); ++i) {
            CHECK(fw::first_test(pg.grp[k][i]) == k, "%s: plan group kind", what);
            CHECK(i == 0 || pg.grp[k][i - 1].idx < pg.grp[k][i].idx, "%s: plan order", what);
        }
    }
    CHECK(total == cut, "%s: plan holds %zu of %u rules", what, total, cut);
}

void check_arena(Rng& g) {
    const size_t size = 4096;
    fw::Arena a(size);
    std::vector<int> owner(size, -1);
    std::vector<std::pair<size_t, size_t>> live;
    for (int op = 0; op < 20000; ++op) {
        if (live.empty() || g.below(3) != 0) {
            const size_t need = 1 + g.below(300);
            size_t off = 0;
            const size_t largest = a.largest();
            const bool ok = a.alloc(need, &off);
            CHECK(ok == (need <= largest), "arena: alloc(%zu) %d with largest %zu", need, ok,
                  largest);
            if (!ok) continue;
            CHECK(off + need <= size, "arena: block past the end");
            for (size_t b = off; b < off + need; ++b) {
                CHECK(owner[b] < 0, "arena: byte %zu handed out twice", b);
                owner[b] = op;
            }
            live.emplace_back(off, need);
        } else {
            const size_t k = g.below(uint32_t(live.size()));
            for (size_t b = live[k].first; b < live[k].first + live[k].second; ++b) owner[b] = -1;
            a.release(live[k].first, live[k].second);
            live.erase(live.begin() + long(k));
        }
        // the free blocks are exactly the unowned bytes, merged
        size_t prev_end = 0, free_bytes = 0;
        bool first = true;
        for (const auto& kv : a.blocks()) {
            CHECK(first || kv.first > prev_end, "arena: free blocks not merged or overlapping");
            for (size_t b = kv.first; b < kv.first + kv.second; ++b)
                CHECK(owner[b] < 0, "arena: byte %zu free and owned", b);
            prev_end = kv.first + kv.second;
            free_bytes += kv.second;
            first = false;
        }
        size_t unowned = 0;
        for (int o : owner) unowned += o < 0;
        CHECK(free_bytes == unowned, "arena: %zu free bytes, %zu unowned", free_bytes, unowned);
    }
    for (auto& l : live) a.release(l.first, l.second);
    CHECK(a.largest() == size && a.blocks().size() == 1, "arena: not whole after releasing all");
}

// guarded(): a body's own status passes through; any exception out of it
// becomes FW_E_NOMEM with a message, and nothing escapes.
void check_guard() {
    CHECK(fw::guarded([] { return FW_OK; }) == FW_OK, "guard: FW_OK not passed through");
    CHECK(fw::guarded([] { return FW_E_ALIGN; }) == FW_E_ALIGN, "guard: status not passed");
    g_last_message.clear();
    CHECK(fw::guarded([]() -> fw_status { throw std::bad_alloc(); }) == FW_E_NOMEM,
          "guard: bad_alloc");
    CHECK(g_last_message.find("host resources exhausted") != std::string::npos,
          "guard: no message for bad_alloc");
    CHECK(fw::guarded([]() -> fw_status {
              throw std::system_error(std::make_error_code(std::errc::resource_unavailable_try_again));
          }) == FW_E_NOMEM,
          "guard: system_error");
    CHECK(fw::guarded([]() -> fw_status { throw std::length_error("vector"); }) == FW_E_NOMEM,
          "guard: length_error");
    CHECK(fw::guarded([]() -> fw_status { throw 42; }) == FW_E_NOMEM, "guard: non-std exception");
    CHECK(fw::guarded([]() -> fw_status {
              std::vector<int> v(1000, 7);
              if (v[999] == 7) throw std::runtime_error("after allocating");
              return FW_OK;
          }) == FW_E_NOMEM,
          "guard: exception after allocations (their memory must be freed: ASan leak check)");
}

}  // namespace

int main() {
    Rng g{12345};
    check_guard();
    check_arena(g);
    struct Case {
        uint32_t R;
        bool wide;
        int catch_at;   // -1: none
    };
    const Case cases[] = {{0, false, -1},   {1, false, -1},  {1, false, 0},   {7, false, 3},
                          {64, false, -1},  {65, true, -1},  {300, false, -1}, {300, true, 150},
                          {2000, false, -1}, {2000, true, 1999}, {5000, false, 2500}};
    int k = 0;
    for (const Case& c : cases) {
        std::vector<RuleRec> rules;
        for (uint32_t r = 0; r < c.R; ++r) rules.push_back(random_rule(g, r, c.wide));
        if (c.catch_at >= 0) rules[size_t(c.catch_at)] = catch_all(uint32_t(c.catch_at));
        char what[64];
        std::snprintf(what, sizeof what, "case %d (R=%u)", k++, c.R);
        check_lists(rules, g, what);
    }
    // address-wildcard heavy: more than 64 such rules, so the table and the rest both serve
    std::vector<RuleRec> rules;
    for (uint32_t r = 0; r < 400; ++r) {
        RuleRec q = random_rule(g, r, false);
        if (g.below(2)) {   // both addresses unspecified
            q.src_lo = q.dst_lo = 0;
            q.src_w = q.dst_w = 0xFFFFFFFFu;
        }
        if (fw::is_catch_all(q)) q.proto = 6;   // keep the list going past it
        rules.push_back(q);
    }
    check_lists(rules, g, "address-wildcard heavy");
    if (g_failures) {
        std::fprintf(stderr, "%d check(s) failed\n", g_failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
