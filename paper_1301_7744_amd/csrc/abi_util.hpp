// Helpers shared by the C ABI entry points (api.cpp, server.cpp).
#pragma once
#include <hip/hip_runtime.h>

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
// Launches the X-panel kernels and levels 0..m-1-last_from_end of plan P on
// stream s; the last launched level writes `out`, the others the workspace w.
// tabs: null to use the plan's own device tables, else the device address of
// a copy of P->tab_blob (host-only plans).
int launch_levels(const Plan *P, const bcss_layout *A, const void *A_dev, const void *X_dev, int64_t rs_x,
                  int64_t cs_x, int last_from_end, void *out, char *w, const char *tabs, hipStream_t s);

}  // namespace symt
