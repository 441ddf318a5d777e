// Batches: ld_norm_batch and the reusable batch handle (see include/ld.h).
//
// All problems of a batch are planned on host threads, packed into one device
// image and solved by one persistent queue launch per sweep-kernel shape, longest
// items first.  A batch handle keeps the image resident and replays the launch
// sequence from a captured HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "ld.h"
#include "ld_api_internal.h"
#include "ld_plan.h"
#include "ld_program.h"
#include "ld_tune.h"

using namespace ld;

namespace {

// Plan every problem with the batch sweep shape; per-problem status codes.
void plan_all(const ld_problem* probs, int32_t count, std::vector<Plan>& plans, std::vector<int32_t>& st)
{
    plans.assign(count, Plan{});
    st.assign(count, LD_OK);
    std::atomic<int32_t> next{0};
    auto work = [&]() {
        for (int32_t i; (i = next.fetch_add(1)) < count;) {
            const ld_problem& q = probs[i];
            plans[i] = make_plan(q.M, q.n, q.m, q.d, q.marginals, batch_shape_for(q.n, q.m, q.d));
            st[i] = plans[i].status;
        }
    };
    const int nt = std::max(1, std::min<int>((count + 63) / 64, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 1; t < std::min(nt, 16); ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
}

}  // namespace

struct ld_batch {
    std::vector<Plan> plans;
    std::vector<int32_t> status;
    std::vector<int32_t> index;   // problem i of the program -> position in the caller's batch
    Program prog;
    hipStream_t own = nullptr;
    void* dev = nullptr;
    int64_t* hres = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<hipStream_t> side;   // launches fan out over these inside the graph
    std::vector<hipEvent_t> fan_ev;
    float last_ms = 0.f;
};

namespace {

void release(ld_batch* b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->dev) (void)hipFree(b->dev);
    if (b->hres) (void)hipHostFree(b->hres);
    if (b->e0) (void)hipEventDestroy(b->e0);
    if (b->e1) (void)hipEventDestroy(b->e1);
    for (hipEvent_t e : b->fan_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t s : b->side)
        if (s) (void)hipStreamDestroy(s);
    if (b->own) (void)hipStreamDestroy(b->own);
    delete b;
}

}  // namespace

extern "C" {

int ld_plan_batch(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals, ld_plan_info* info)
{
    if (!info) return LD_EINVAL;
    Plan p = make_plan(M, n, m, d, marginals, batch_shape_for(n, m, d));
    info_from_plan(p, info);
    return p.status;
}

int ld_norm_batch(const ld_problem* probs, int32_t count, int64_t* out, int32_t* status, void* hip_stream)
{
    if (count < 0 || (count > 0 && (!probs || !out))) {
        set_error(LD_EINVAL);
        return LD_EINVAL;
    }
    if (count == 0) return LD_OK;
    std::vector<Plan> plans;
    std::vector<int32_t> st;
    plan_all(probs, count, plans, st);
    std::vector<const Plan*> ok_plans;
    std::vector<int32_t> where;
    int first = LD_OK;
    for (int32_t i = 0; i < count; ++i) {
        out[i] = INT64_MIN;
        if (st[i] == LD_OK) {
            ok_plans.push_back(&plans[i]);
            where.push_back(i);
        } else if (first == LD_OK) {
            first = st[i];
        }
    }
    if (!ok_plans.empty()) {
        std::vector<int64_t> vals(ok_plans.size());
        if (!run_plans_sync(ok_plans, batch_item_shape(), vals.data(), (hipStream_t)hip_stream)) {
            for (size_t k = 0; k < where.size(); ++k) st[where[k]] = LD_EHIP;
            if (first == LD_OK) first = LD_EHIP;
        } else {
            for (size_t k = 0; k < where.size(); ++k) out[where[k]] = vals[k];
        }
    }
    if (status) std::memcpy(status, st.data(), sizeof(int32_t) * (size_t)count);
    if (first != LD_OK) set_error(first);
    return first;
}

ld_batch* ld_batch_prepare(const ld_problem* probs, int32_t count, int32_t* status)
{
    if (count < 1 || !probs) {
        set_error(LD_EINVAL);
        return nullptr;
    }
    ld_batch* b = new ld_batch;
    plan_all(probs, count, b->plans, b->status);
    if (status) std::memcpy(status, b->status.data(), sizeof(int32_t) * (size_t)count);
    std::vector<const Plan*> ok_plans;
    for (int32_t i = 0; i < count; ++i)
        if (b->status[i] == LD_OK) {
            ok_plans.push_back(&b->plans[i]);
            b->index.push_back(i);
        }
    b->prog = build_program(ok_plans, batch_item_shape());
    bool ok = device_ok(nullptr);
    ok = ok && hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreate(&b->e0) == hipSuccess && hipEventCreate(&b->e1) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&b->hres, 8 * std::max<size_t>(ok_plans.size(), 1), hipHostMallocDefault) ==
                   hipSuccess;
    ok = ok && hipMalloc(&b->dev, b->prog.image.size()) == hipSuccess;
    if (ok) {
        patch_program(b->prog, b->dev);
        ok = hipMemcpy(b->dev, b->prog.image.data(), b->prog.image.size(), hipMemcpyHostToDevice) == hipSuccess;
    }
    // occupancy queries are not stream work: make them before the capture
    if (ok)
        for (const Launch& L : b->prog.launches) (void)capped_blocks(L.kernel, L.threads, L.lds);
    // capture reset + launches + result copy once; every run replays the graph
    const int n_side = batch_side_streams();
    for (int k = 0; ok && k < n_side; ++k) {
        hipStream_t s2 = nullptr;
        ok = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) == hipSuccess;
        if (ok) b->side.push_back(s2);
    }
    for (int k = 0; ok && k <= n_side && n_side > 0; ++k) {
        hipEvent_t e = nullptr;
        ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        if (ok) b->fan_ev.push_back(e);
    }
    ok = ok && hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        const bool enq = enqueue_program_fanned(b->prog, b->own, b->hres, b->side, b->fan_ev);
        ok = hipStreamEndCapture(b->own, &b->graph) == hipSuccess && enq;
    }
    ok = ok && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        release(b);
        set_error(LD_EHIP);
        return nullptr;
    }
    return b;
}

int ld_batch_run(ld_batch* b, void* hip_stream, int64_t* out)
{
    if (!b || !out) {
        set_error(LD_EINVAL);
        return LD_EINVAL;
    }
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : b->own;
    bool ok = hipEventRecord(b->e0, s) == hipSuccess;
    ok = ok && hipGraphLaunch(b->exec, s) == hipSuccess;
    ok = ok && hipEventRecord(b->e1, s) == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    ok = ok && hipEventElapsedTime(&b->last_ms, b->e0, b->e1) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        set_error(LD_EHIP);
        return LD_EHIP;
    }
    const int32_t count = (int32_t)b->plans.size();
    for (int32_t i = 0; i < count; ++i) out[i] = INT64_MIN;
    for (size_t k = 0; k < b->index.size(); ++k) out[b->index[k]] = b->hres[k];
    for (int k : b->prog.zero) out[b->index[k]] = 0;
    for (int32_t i = 0; i < count; ++i)
        if (b->status[i] != LD_OK) {
            set_error(b->status[i]);
            return b->status[i];
        }
    return LD_OK;
}

float ld_batch_last_ms(ld_batch* b) { return b ? b->last_ms : 0.f; }

void ld_batch_release(ld_batch* b) { release(b); }

}  // extern "C"
