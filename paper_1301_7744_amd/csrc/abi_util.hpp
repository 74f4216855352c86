// Helpers shared by the C ABI entry points (api.cpp, server.cpp).
#pragma once
#include <string>

#include "../../include/sttsm.h"
#include "plan.hpp"

namespace symt {

// Sets the calling thread's last-error message and returns code.
int fail(int code, const std::string &msg);
// Bytes per element of an sttsm_dtype, 0 if unknown.
int dtype_size(int dt);
// Validates a layout; *why says what is wrong.
bool layout_ok(const bcss_layout *L, std::string *why);
// Validates an sttsm problem (shapes, dtypes, precision) and fills its plan key.
int make_key(const bcss_layout *A, const bcss_layout *C, int32_t prec, PlanKey *key);

}  // namespace symt
