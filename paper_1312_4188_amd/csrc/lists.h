// Host-only construction of the learned index's candidate lists and lookup
// tables, and of the grouped scan plan's rule groups (lists.cpp).  No HIP.
#pragma once

#include <cstdint>
#include <vector>

#include "host_types.h"

namespace fw {

// A rule that matches every packet (all five fields unspecified).
bool full_match_all(const RuleRec& q);
// A rule that matches every packet whose destination it covers (source,
// ports and protocol unspecified).
bool full_match_in_interval(const RuleRec& q);
bool is_catch_all(const RuleRec& q);

// The candidate lists of a rule list (compiled records in rule order).
struct HostLists {
    std::vector<uint32_t> B, off, L_idx;   // destination intervals and their lists
    std::vector<RuleRec> L;                // records of the per-interval lists
    std::vector<uint32_t> G_idx;           // destination-wildcard candidates, cut at the
                                           // first catch-all
    std::vector<uint32_t> Bs, soff, S_idx; // those with a specified source, by source interval
    std::vector<RuleRec> S;
    std::vector<uint32_t> Gw_idx;          // those with both addresses unspecified
    std::vector<RuleRec> Gw;
};

// Destination intervals with their per-interval lists L_j (rules with a
// specified destination), the shared destination-wildcard candidates G cut at
// the first catch-all, and G split once more: rules of G with a specified
// source get source intervals and per-interval lists S_i, the rest (both
// addresses unspecified, ending with the catch-all) is Gw.  False when a list
// array would need more than 2^32 entries.
bool build_lists(const RuleRec* recs, uint32_t n_rules, HostLists* out);

// Port/protocol table of the first kPtRules entries of `gw` that are not
// catch-alls; *rest receives the entries after them.
void build_port_table(const std::vector<RuleRec>& gw, PortTable* t, uint32_t* count,
                      uint32_t* steps_s, uint32_t* steps_d, std::vector<RuleRec>* rest);

// Bucket table over the top `bits` bits of a key for sorted interval starts
// B (bits 0: no table).
void build_bucket_table(const std::vector<uint32_t>& B, std::vector<uint16_t>* table,
                        uint32_t* bits, uint32_t* steps);

// The field a rule is tested on first: the narrower address prefix when
// either address is specified (destination on a tie), else the ports when
// either port range is, else the protocol.
uint32_t first_test(const RuleRec& q);

// A rule list cut at its first catch-all and split by first test, each group
// in rule order; the catch-all's index and action become the tail
// (tail_idx kNoMatch when there is none).
struct PlanGroups {
    std::vector<RuleRec> grp[4];
    uint32_t tail_idx = kNoMatch, tail_act = 0;
};
void group_rules(const RuleRec* recs, uint32_t n, PlanGroups* out);

}  // namespace fw
