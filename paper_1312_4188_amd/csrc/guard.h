// The C interface's entry points run their bodies through guarded(): a C++
// exception (a failed host allocation, a thread that cannot be started) would
// end the process if it crossed the extern "C" boundary, so it becomes the
// status FW_E_NOMEM instead.  Host-only.
#pragma once

#include <exception>
#include <new>

#include "../../include/fw.h"

namespace fw {

fw_status fail(fw_status st, const char* fmt, ...);

template <class F>
fw_status guarded(F&& body) noexcept {
    try {
        return body();
    } catch (const std::exception& e) {
        try {
            return fail(FW_E_NOMEM, "host resources exhausted: %s", e.what());
        } catch (...) {
            return FW_E_NOMEM;   // not even the message could be stored
        }
    } catch (...) {
        return FW_E_NOMEM;
    }
}

}  // namespace fw
