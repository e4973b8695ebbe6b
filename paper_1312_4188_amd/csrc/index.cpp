// Learned destination index (work in progress: host build and kernels follow).
#include "index.h"

namespace fw {

struct LearnedIndex {};

fw_status build_index(const fw_rule*, const RuleRec*, uint32_t, const fw_index_opts&,
                      fw_index_stats*, LearnedIndex** out) {
    *out = nullptr;
    return fail(FW_E_INVAL, "learned index not available in this build");
}
void destroy_index(LearnedIndex* ix) { delete ix; }
fw_status classify_learned(const LearnedIndex*, const RuleRec*, uint32_t, uint8_t, PacketsDev,
                           size_t, int32_t*, uint8_t*, uint32_t, hipStream_t, uint64_t*) {
    return fail(FW_E_NOINDEX, "learned index not available in this build");
}
fw_status index_lookup(const LearnedIndex*, const uint32_t*, size_t, int32_t*, uint32_t,
                       hipStream_t) {
    return fail(FW_E_NOINDEX, "learned index not available in this build");
}
fw_status index_export(const LearnedIndex*, uint32_t, void*, size_t, size_t*) {
    return fail(FW_E_NOINDEX, "learned index not available in this build");
}

}  // namespace fw

extern "C" {
fw_status fw_rmi_gradients(uint32_t, uint32_t, const float*, size_t, const float*, const float*,
                           const uint32_t*, uint32_t, float*, float*) {
    return fw::fail(FW_E_INVAL, "not available in this build");
}
fw_status fw_rmi_adam_step(size_t, float*, const float*, float*, float*, uint32_t, float, float,
                           float, float) {
    return fw::fail(FW_E_INVAL, "not available in this build");
}
}
