// Host-side pieces shared by the plan compiler (stl_compile.cpp, plain C++)
// and the launch layer (stl_api.cpp): the plan object and the thread-local
// error channel behind stl_last_error.
#pragma once

#include <stdint.h>

#include "../../include/stlmi.h"
#include "stl_plan.h"

struct stl_plan {
    stlmi::DevPlan dev;          // liveness-optimised forward slot map
    stlmi::DevPlan dev_trace;    // forward map with one slot per instruction (node trace output)
    int32_t n_nodes = 0;  // caller's nodes
    int32_t n_params = 0;
    int32_t D = 0;
    int32_t max_until_b = 0;
    int32_t has_until = 0;
};

namespace stlmi {
// sets the message stl_last_error returns and returns s
stl_status fail(stl_status s, const char* fmt, ...);
}  // namespace stlmi

// replaces the message stl_last_error returns (also used by mlp_kernels.hip)
void stlmi_set_error(const char* msg);
