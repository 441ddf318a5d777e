// Internal helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "ld.h"
#include "ld_plan.h"
#include "ld_program.h"

namespace ld {

void set_error(int code);

// true if the current HIP device is a gfx950; its index in *dev
bool device_ok(int* dev);

// Solve planned problems (all with status LD_OK) on the calling thread's
// buffers; s = nullptr uses the thread's own stream.  Synchronous.
bool run_plans_sync(const std::vector<const Plan*>& plans, const ItemShape& shape, int64_t* out, hipStream_t s);

int64_t run_plan_sync(const Plan& p);

// the public description of a plan
void info_from_plan(const Plan& p, ld_plan_info* info);

}  // namespace ld
