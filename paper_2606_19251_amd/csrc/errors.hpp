// Error reporting shared by every C entry point: a per-thread message and a wrapper that
// turns C++ exceptions into status codes so that none crosses the C interface.
#pragma once

#include <exception>
#include <new>
#include <string>

#include "amggnn.h"

namespace amgg {

std::string& last_error_slot();

inline int fail(int code, const std::string& msg) {
    last_error_slot() = msg;
    return code;
}

template <class F>
int guarded(F&& body) {
    try {
        last_error_slot().clear();
        return body();
    } catch (const std::bad_alloc&) {
        return fail(AMGG_EINVAL, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(AMGG_EINVAL, std::string("internal error: ") + e.what());
    } catch (...) {
        return fail(AMGG_EINVAL, "internal error");
    }
}

}  // namespace amgg
