// Host-only construction of the learned index's candidate lists and lookup
// tables, and the grouping of a rule list into a scan plan.  No HIP: the
// tests build this file with the address and undefined-behaviour sanitizers.
//
// Intervals: B = {0} with every rule's destination range start and every
// range end + 1 below 2^32, sorted and de-duplicated; interval j is
// [B[j], B[j+1]).  Every destination range is a union of whole intervals, so
// the rules whose destination covers interval j (its candidate list C_j, in
// rule order) are exactly the rules whose destination test a packet in j
// passes, and the first match over C_j is the first match overall.
#include "lists.h"

#include <algorithm>
#include <cstring>

namespace fw {

bool full_match_all(const RuleRec& q) {
    return q.src_w == 0xFFFFFFFFu && q.dst_w == 0xFFFFFFFFu && q.port_lo == 0 &&
           q.port_w == 0xFFFFFFFFu && ((q.proto >> 8) & 0xFFu) == 255u;
}

bool full_match_in_interval(const RuleRec& q) {
    return q.src_w == 0xFFFFFFFFu && q.port_lo == 0 && q.port_w == 0xFFFFFFFFu &&
           ((q.proto >> 8) & 0xFFu) == 255u;
}

bool is_catch_all(const RuleRec& q) { return full_match_all(q); }

namespace {

// Elementary intervals of one address field over the rules `sel` (ascending
// indices into recs) and, per interval, the ascending list of those rules whose
// range for that field contains the whole interval, cut after the first rule
// that `full` says matches every packet of the interval.
template <class Range, class Full>
bool interval_lists(const RuleRec* recs, const std::vector<uint32_t>& sel, Range range, Full full,
                    std::vector<uint32_t>* B, std::vector<uint32_t>* off,
                    std::vector<uint32_t>* idx, std::vector<RuleRec>* out) {
    B->clear();
    B->reserve(sel.size() * 2 + 1);
    B->push_back(0u);
    for (uint32_t r : sel) {
        uint32_t lo, w;
        range(recs[r], &lo, &w);
        const uint64_t hi = uint64_t(lo) + w;
        B->push_back(lo);
        if (hi < 0xFFFFFFFFull) B->push_back(uint32_t(hi + 1));
    }
    std::sort(B->begin(), B->end());
    B->erase(std::unique(B->begin(), B->end()), B->end());
    const uint32_t M = uint32_t(B->size());
    std::vector<std::vector<uint32_t>> lists(M);
    std::vector<uint8_t> closed(M, 0);
    for (uint32_t r : sel) {
        uint32_t lo, w;
        range(recs[r], &lo, &w);
        const uint64_t hi = uint64_t(lo) + w;
        const uint32_t jlo = uint32_t(std::lower_bound(B->begin(), B->end(), lo) - B->begin());
        const uint32_t jhi =
            hi >= 0xFFFFFFFFull
                ? M - 1
                : uint32_t(std::lower_bound(B->begin(), B->end(), uint32_t(hi + 1)) - B->begin()) - 1;
        const bool f = full(recs[r]);
        for (uint32_t j = jlo; j <= jhi; ++j) {
            if (closed[j]) continue;
            lists[j].push_back(r);
            if (f) closed[j] = 1;
        }
    }
    off->assign(size_t(M) + 1, 0);
    uint64_t total = 0;
    for (uint32_t j = 0; j < M; ++j) {
        total += lists[j].size();
        if (total > 0xFFFFFFFFull) return false;   // offsets are 32-bit
        (*off)[j + 1] = uint32_t(total);
    }
    idx->clear();
    idx->reserve(total);
    out->clear();
    out->reserve(total);
    for (uint32_t j = 0; j < M; ++j)
        for (uint32_t r : lists[j]) {
            idx->push_back(r);
            out->push_back(recs[r]);
        }
    return true;
}

}  // namespace

// Port/protocol table (see PortTable) of the first kPtRules entries of the
// address-wildcard list `gw` that are not catch-alls; *rest receives the
// entries after them (ending with the catch-all, if any).  Ranges come from
// the packed records: sport = [port_lo >> 16, + port_w >> 16], dport the low
// halves, protocol (p - lo) <= w.
void build_port_table(const std::vector<RuleRec>& gw, PortTable* t, uint32_t* count,
                      uint32_t* steps_s, uint32_t* steps_d, std::vector<RuleRec>* rest) {
    std::memset(t, 0, sizeof *t);
    std::vector<RuleRec> tab;
    rest->clear();
    for (const RuleRec& q : gw) {
        if (tab.size() < kPtRules && !full_match_all(q))
            tab.push_back(q);
        else
            rest->push_back(q);
    }
    *count = uint32_t(tab.size());
    for (uint32_t r = 0; r < kPtRules + 4; ++r)
        t->rule[r] = r < tab.size() ? (tab[r].idx | (((tab[r].proto >> 16) & 0xFFu) << 24))
                                    : kPtNone;
    for (uint32_t p = 0; p < 256; ++p) {
        uint64_t m = 0;
        for (uint32_t r = 0; r < tab.size(); ++r) {
            const uint32_t lo = tab[r].proto & 0xFFu, w = (tab[r].proto >> 8) & 0xFFu;
            if (p - lo <= w) m |= uint64_t(1) << r;
        }
        t->mask_p[p] = m;
    }
    // one port field: boundaries, masks, high-byte table, longest walk
    auto field = [&](int shift, uint64_t* mask, uint32_t* b, uint8_t* bucket, uint32_t* steps) {
        std::vector<uint32_t> bs{0u};
        for (const RuleRec& q : tab) {
            const uint32_t lo = (q.port_lo >> shift) & 0xFFFFu, w = (q.port_w >> shift) & 0xFFFFu;
            bs.push_back(lo);
            if (lo + w < 0xFFFFu) bs.push_back(lo + w + 1u);
        }
        std::sort(bs.begin(), bs.end());
        bs.erase(std::unique(bs.begin(), bs.end()), bs.end());
        const uint32_t n = uint32_t(bs.size());   // <= 2 * kPtRules + 1
        for (uint32_t i = 0; i < kPtMaxIv + 2; ++i) b[i] = i < n ? bs[i] : 0x10000u;
        for (uint32_t i = 0; i < kPtMaxIv; ++i) {
            uint64_t m = 0;
            if (i < n)
                for (uint32_t r = 0; r < tab.size(); ++r) {
                    const uint32_t lo = (tab[r].port_lo >> shift) & 0xFFFFu;
                    const uint32_t w = (tab[r].port_w >> shift) & 0xFFFFu;
                    if (bs[i] - lo <= w) m |= uint64_t(1) << r;   // interval i inside the range
                }
            mask[i] = m;
        }
        uint32_t longest = 0;
        for (uint32_t h = 0; h < 256; ++h) {
            const uint32_t first = h << 8;
            const uint32_t i0 = uint32_t(std::upper_bound(bs.begin(), bs.end(), first) - bs.begin()) - 1u;
            const uint32_t i1 =
                uint32_t(std::upper_bound(bs.begin(), bs.end(), first + 255u) - bs.begin()) - 1u;
            bucket[h] = uint8_t(i0);
            longest = std::max(longest, i1 - i0);
        }
        *steps = longest;
    };
    field(16, t->mask_s, t->b_s, t->bucket_s, steps_s);
    field(0, t->mask_d, t->b_d, t->bucket_d, steps_d);
}

// Bucket table over the top `bits` bits of a 32-bit key for sorted interval
// starts B (B[0] = 0): entry h is the interval holding key h << (32 - bits),
// and `steps` forward steps from there reach the interval of any key of the
// bucket (the most starts inside one bucket).  Bits are chosen for about four
// buckets per interval, at most 12 (8 KiB of uint16); no table (bits = 0)
// when the intervals do not fit uint16 or some bucket would need more than 8
// steps, and the kernel then binary-searches B.
void build_bucket_table(const std::vector<uint32_t>& B, std::vector<uint16_t>* table,
                        uint32_t* bits, uint32_t* steps) {
    table->clear();
    *bits = 0;
    *steps = 0;
    const size_t M = B.size();
    if (M < 2 || M > 0xFFFFu) return;
    uint32_t b = 8;
    while (b < 12 && (size_t(1) << b) < 4 * M) ++b;
    const uint32_t shift = 32 - b;
    table->resize(size_t(1) << b);
    uint32_t longest = 0;
    for (uint64_t h = 0; h < (uint64_t(1) << b); ++h) {
        const uint32_t first = uint32_t(h << shift);
        const uint32_t last = uint32_t(((h + 1) << shift) - 1);
        const uint32_t i0 = uint32_t(std::upper_bound(B.begin(), B.end(), first) - B.begin()) - 1u;
        const uint32_t i1 = uint32_t(std::upper_bound(B.begin(), B.end(), last) - B.begin()) - 1u;
        (*table)[h] = uint16_t(i0);
        longest = std::max(longest, i1 - i0);
    }
    if (longest > 8) {
        table->clear();
        return;
    }
    *bits = b;
    *steps = longest;
}

// Destination intervals with their per-interval lists L_j (rules with a
// specified destination), the shared destination-wildcard candidates G cut
// at the first catch-all, and G split once more: rules of G with a specified
// source get source intervals and per-interval lists S_i (an address in
// source interval i passes exactly the source tests of the rules in S_i, by
// the same covering argument), and the rest of G (source and destination
// both unspecified, ending with the catch-all) is the wave-uniform list Gw.
bool build_lists(const RuleRec* recs, uint32_t n_rules, HostLists* ix) {
    uint32_t g_cut = 0xFFFFFFFFu;
    std::vector<uint32_t> dsel, ssel;
    *ix = HostLists{};
    std::vector<RuleRec>* Gw = &ix->Gw;
    for (uint32_t r = 0; r < n_rules; ++r) {
        const RuleRec& q = recs[r];
        if (q.dst_w != 0xFFFFFFFFu) {
            dsel.push_back(r);
            continue;
        }
        ix->G_idx.push_back(r);
        if (q.src_w != 0xFFFFFFFFu) {
            ssel.push_back(r);
        } else {
            ix->Gw_idx.push_back(r);
            Gw->push_back(q);
        }
        if (full_match_all(q)) {
            g_cut = r;
            break;
        }
    }
    // rules past the first catch-all are unreachable (dsel is ascending, so trim its tail)
    while (!dsel.empty() && dsel.back() > g_cut) dsel.pop_back();
    auto dst_range = [](const RuleRec& q, uint32_t* lo, uint32_t* w) {
        *lo = q.dst_lo;
        *w = q.dst_w;
    };
    auto src_range = [](const RuleRec& q, uint32_t* lo, uint32_t* w) {
        *lo = q.src_lo;
        *w = q.src_w;
    };
    if (!interval_lists(recs, dsel, dst_range, full_match_in_interval, &ix->B, &ix->off,
                        &ix->L_idx, &ix->L))
        return false;
    // a source-interval candidate (destination already unspecified) matches every
    // packet of its interval when ports and protocol are unspecified
    auto full_src = [](const RuleRec& q) {
        return q.port_lo == 0 && q.port_w == 0xFFFFFFFFu && ((q.proto >> 8) & 0xFFu) == 255u;
    };
    return interval_lists(recs, ssel, src_range, full_src, &ix->Bs, &ix->soff, &ix->S_idx,
                          &ix->S);
}

uint32_t first_test(const RuleRec& q) {
    if (q.dst_w != 0xFFFFFFFFu || q.src_w != 0xFFFFFFFFu)
        return q.dst_w <= q.src_w ? kFirstDst : kFirstSrc;
    if (!(q.port_lo == 0 && q.port_w == 0xFFFFFFFFu)) return kFirstPorts;
    return kFirstProto;
}

void group_rules(const RuleRec* recs, uint32_t n, PlanGroups* out) {
    for (auto& g : out->grp) g.clear();
    out->tail_idx = kNoMatch;
    out->tail_act = 0;
    for (uint32_t r = 0; r < n; ++r) {
        if (is_catch_all(recs[r])) {
            out->tail_idx = recs[r].idx;
            out->tail_act = (recs[r].proto >> 16) & 1u;
            break;
        }
        out->grp[first_test(recs[r])].push_back(recs[r]);
    }
}

}  // namespace fw
