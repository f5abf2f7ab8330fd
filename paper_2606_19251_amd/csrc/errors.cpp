#include "errors.hpp"

namespace amgg {

std::string& last_error_slot() {
    thread_local std::string msg;
    return msg;
}

}  // namespace amgg

extern "C" const char* amgg_last_error(void) { return amgg::last_error_slot().c_str(); }
