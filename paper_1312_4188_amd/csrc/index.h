// Learned destination index: internal declarations.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fw.h"
#include "fw_internal.h"

namespace fw {

fw_status fail(fw_status st, const char* fmt, ...);
fw_status hip_fail(hipError_t e, const char* what);

struct LearnedIndex;

fw_status build_index(const fw_rule* rules, const RuleRec* recs, uint32_t n_rules,
                      const fw_index_opts& opts, fw_index_stats* stats, LearnedIndex** out);
void destroy_index(LearnedIndex* ix);
fw_status classify_learned(const LearnedIndex* ix, const RuleRec* rules, uint32_t n_rules,
                           uint8_t default_action, PacketsDev pk, size_t n, int32_t* out_idx,
                           uint8_t* out_act, uint32_t lookup, hipStream_t stream,
                           uint64_t* window_misses);
fw_status index_lookup(const LearnedIndex* ix, const uint32_t* keys, size_t n,
                       int32_t* out_interval, uint32_t lookup, hipStream_t stream);
fw_status index_export(const LearnedIndex* ix, uint32_t what, void* host, size_t cap,
                       size_t* size);

}  // namespace fw
