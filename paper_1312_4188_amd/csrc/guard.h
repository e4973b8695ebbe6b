// The C interface's entry points run their bodies through guarded(): a C++
// exception (a failed host allocation, a thread that cannot be started) would
// end the process if it crossed the extern "C" boundary, so it becomes the
// status FW_E_NOMEM instead.  Host-only.
#pragma once

#include <exception>
#include <new>
#include <utility>

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

// Undoes a partly built object when its scope ends by an early return or an
// exception, unless dismissed once the object is complete.
template <class F>
class ScopeExit {
   public:
    explicit ScopeExit(F f) : f_(std::move(f)) {}
    ScopeExit(const ScopeExit&) = delete;
    ScopeExit& operator=(const ScopeExit&) = delete;
    ~ScopeExit() {
        if (on_) f_();
    }
    void dismiss() { on_ = false; }

   private:
    F f_;
    bool on_ = true;
};

}  // namespace fw
