// The multi-chain launch as the library's other parts (the serving runtime)
// call it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fw.h"
#include "fw_internal.h"

namespace fw {

struct ChainView;

// One chain's batch as the multi-chain kernels read it (104 bytes).  The
// fields the scans use are copied from the ruleset's view, so a kernel reads
// them straight from the descriptor (scalar loads) rather than through
// `view`, a pointer read from memory that the kernel's own stores may alias.
struct ChainDesc {
    const ChainView* view;   // the ruleset (device copy)
    const RuleRec* rules;    // view->rules
    const uint2* pairs;      // view->pairs
    const uint32_t* src;
    const uint32_t* dst;
    const uint16_t* sport;
    const uint16_t* dport;
    const uint8_t* proto;
    int32_t* out_idx;
    uint8_t* out_act;
    uint64_t n;
    uint32_t n_rules, dflt;  // view->n_rules, view->dflt
    uint32_t item_begin;
    uint32_t index;          // kChainIndexed: view->has_index; kChainBoundariesInLds: this
                             // launch stages the index's image with its boundary arrays
};
constexpr uint32_t kChainIndexed = 1, kChainBoundariesInLds = 2;

// Placements (fw_multi_opts.placement): grouped plan and learned index, or
// the rule list in rule order through the scalar cache, LDS tiles or vector
// loads.
constexpr uint32_t kPlaceScalar = 1, kPlaceLds = 2, kPlaceVector = 3, kPlaceAuto = 4;

struct MultiConfig {
    int K = 2;                         // packets per lane
    uint32_t placement = kPlaceAuto;
    uint32_t tile = 0;                 // kPlaceLds: rules per LDS tile (256 or 1024)
    bool use_index = true;             // kPlaceAuto: take built learned indexes
};

// Scratch layout of one launch: the work-queue counter in the first
// kMultiCounterBytes, then the descriptor table.  A caller-provided scratch
// holds up to kMultiMaxChains descriptors.
constexpr uint32_t kMultiMaxChains = 1024;
constexpr size_t kMultiCounterBytes = 256;
constexpr size_t kMultiScratchBytes = kMultiCounterBytes + sizeof(ChainDesc) * kMultiMaxChains;

// One persistent launch over the batches (checked by check_multi_batches),
// asynchronous on `s`.  The counter and table go to `scratch_mem` when given
// (kMultiScratchBytes, at most kMultiMaxChains non-empty chains), else to
// memory allocated on the stream and freed after the launch.  With
// `host_staging` (page-locked host memory of kMultiScratchBytes, with
// scratch_mem; it must stay untouched until the stream passes the launch) the
// counter and table are written there and copied in one transfer; without it
// small kernels copy them from kernel arguments.
hipError_t multi_launch(const fw_chain_batch* b, uint32_t n_chains, MultiConfig cfg,
                        hipStream_t s, void* scratch_mem, void* host_staging);
fw_status check_multi_batches(const fw_chain_batch* b, uint32_t n);

}  // namespace fw
