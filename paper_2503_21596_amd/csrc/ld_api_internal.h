// Internal helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ld_plan.h"

namespace ld {

void set_error(int code);

// blocks of 256 lanes for n_prefix prefixes (grid-stride beyond 2^16 blocks)
uint32_t grid_blocks(uint64_t n_prefix);

// enqueue the sweep kernel of one planned problem (result slot already reset)
bool launch_sweep(const Plan& p, const void* dev_blob, int64_t* dres, hipStream_t s);

// enqueue the result reset (where needed) and the sweep of one planned problem
bool launch_plan(const Plan& p, const void* dev_blob, int64_t* dres, hipStream_t s);

int64_t run_plan_sync(const Plan& p);

}  // namespace ld
