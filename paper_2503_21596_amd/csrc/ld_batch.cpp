// ld_norm_batch (see include/ld.h).
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "ld.h"
#include "ld_api_internal.h"
#include "ld_plan.h"

using namespace ld;

extern "C" int ld_norm_batch(const ld_problem* probs, int32_t count, int64_t* out, int32_t* status,
                             void* hip_stream)
{
    if (count < 0 || (count > 0 && (!probs || !out))) {
        set_error(LD_EINVAL);
        return LD_EINVAL;
    }
    int first = LD_OK;
    for (int32_t i = 0; i < count; ++i) {
        const ld_problem& q = probs[i];
        Plan p = make_plan(q.M, q.n, q.m, q.d, q.marginals, get_shape());
        out[i] = run_plan_sync(p);
        const int st = out[i] == INT64_MIN ? ld_last_error() : LD_OK;
        if (status) status[i] = st;
        if (st != LD_OK && first == LD_OK) first = st;
    }
    (void)hip_stream;
    if (first != LD_OK) set_error(first);
    return first;
}
