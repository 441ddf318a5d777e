// C ABI: plain, range and introspection entry points (see include/ld.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "ld.h"
#include "ld_api_internal.h"
#include "ld_gray.h"
#include "ld_plan.h"
#include "ld_registry.h"

namespace ld {

thread_local int t_last_error = LD_OK;

void set_error(int code) { t_last_error = code; }

// ---------------------------------------------------------------------------
// per-thread device context: stream, device blob buffer, pinned staging, result

namespace {

struct Ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    void* dbuf = nullptr;
    size_t dcap = 0;
    void* hbuf = nullptr;
    size_t hcap = 0;
    int64_t* dres = nullptr;
    int64_t* hres = nullptr;
    ~Ctx()
    {
        // buffers are released at thread exit; errors here cannot be reported
        if (dbuf) (void)hipFree(dbuf);
        if (hbuf) (void)hipHostFree(hbuf);
        if (dres) (void)hipFree(dres);
        if (hres) (void)hipHostFree(hres);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

thread_local Ctx t_ctx;

bool ctx_ready(Ctx& c)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (c.device == dev && c.stream) return true;
    if (c.stream) return false;   // device switched mid-thread: not supported
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return false;
    if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess) return false;
    if (hipMalloc((void**)&c.dres, 64) != hipSuccess) return false;
    if (hipHostMalloc((void**)&c.hres, 64, hipHostMallocDefault) != hipSuccess) return false;
    c.device = dev;
    return true;
}

bool ensure(Ctx& c, size_t bytes)
{
    if (bytes <= c.dcap) return true;
    size_t cap = std::max<size_t>(bytes, 1 << 20);
    if (c.dbuf) (void)hipFree(c.dbuf);
    if (c.hbuf) (void)hipHostFree(c.hbuf);
    c.dbuf = c.hbuf = nullptr;
    c.dcap = c.hcap = 0;
    if (hipMalloc(&c.dbuf, cap) != hipSuccess) return false;
    if (hipHostMalloc(&c.hbuf, cap, hipHostMallocDefault) != hipSuccess) return false;
    c.dcap = c.hcap = cap;
    return true;
}

}  // namespace

uint32_t grid_blocks(uint64_t n_prefix)
{
    const uint64_t lanes = std::max<uint64_t>(n_prefix, 1);
    const uint64_t blocks = (lanes + 255) / 256;
    return (uint32_t)std::min<uint64_t>(blocks, 1u << 16);
}

bool launch_sweep(const Plan& p, const void* dev_blob, int64_t* dres, hipStream_t s)
{
    Desc D = make_desc(p, dev_blob, dres);
    void* args[] = {(void*)&D};
    if (p.wide) {
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(p.n_prefix, 1), 1u << 16);
        return hipLaunchKernel(p.kernel, dim3(blocks), dim3(64), args, p.lds, s) == hipSuccess;
    }
    return hipLaunchKernel(p.kernel, dim3(grid_blocks(p.n_prefix)), dim3(256), args, 0, s) == hipSuccess;
}

bool launch_plan(const Plan& p, const void* dev_blob, int64_t* dres, hipStream_t s)
{
    if (p.kind == PK_SUMABS) {
        const int32_t* dM = (const int32_t*)dev_blob;
        int64_t count = (int64_t)p.n * p.m;
        void* args[] = {(void*)&dM, (void*)&count, (void*)&dres};
        return hipLaunchKernel(kernel_sumabs(), dim3(1), dim3(256), args, 0, s) == hipSuccess;
    }
    int64_t cnt = 1, val = INT64_MIN;
    void* fargs[] = {(void*)&dres, (void*)&cnt, (void*)&val};
    if (hipLaunchKernel(kernel_fill(), dim3(1), dim3(256), fargs, 0, s) != hipSuccess) return false;
    return launch_sweep(p, dev_blob, dres, s);
}

// Run one planned problem synchronously on the calling thread's stream.
int64_t run_plan_sync(const Plan& p)
{
    if (p.status != LD_OK) {
        set_error(p.status);
        return INT64_MIN;
    }
    if (p.kind == PK_ZERO) return 0;
    Ctx& c = t_ctx;
    if (!ctx_ready(c) || !ensure(c, p.blob.size())) {
        set_error(LD_EHIP);
        return INT64_MIN;
    }
    std::memcpy(c.hbuf, p.blob.data(), p.blob.size());
    bool ok = hipMemcpyAsync(c.dbuf, c.hbuf, p.blob.size(), hipMemcpyHostToDevice, c.stream) == hipSuccess;
    ok = ok && launch_plan(p, c.dbuf, c.dres, c.stream);
    ok = ok && hipMemcpyAsync(c.hres, c.dres, 8, hipMemcpyDeviceToHost, c.stream) == hipSuccess;
    ok = ok && hipStreamSynchronize(c.stream) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        set_error(LD_EHIP);
        return INT64_MIN;
    }
    return *c.hres;
}

}  // namespace ld

using namespace ld;

struct ld_prepared {
    Plan plan;
    int device = -1;
    hipStream_t own = nullptr;
    void* dblob = nullptr;
    int64_t* dres = nullptr;
    int64_t* hres = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float last_ms = 0.f;
};

namespace {

void info_from_plan(const Plan& p, ld_plan_info* info)
{
    std::memset(info, 0, sizeof(*info));
    info->kind = p.kind;
    info->n = p.n;
    info->m = p.m;
    info->d = p.d;
    info->transposed = p.transposed;
    info->i64 = p.i64;
    info->mp = p.mp;
    info->R = p.R;
    info->C = p.C;
    info->P = p.P;
    info->P_tab = p.P_tab;
    info->n_prefix = p.n_prefix;
    info->words = p.words;
}

void release(ld_prepared* h)
{
    if (!h) return;
    if (h->dblob) (void)hipFree(h->dblob);
    if (h->dres) (void)hipFree(h->dres);
    if (h->hres) (void)hipHostFree(h->hres);
    if (h->e0) (void)hipEventDestroy(h->e0);
    if (h->e1) (void)hipEventDestroy(h->e1);
    if (h->own) (void)hipStreamDestroy(h->own);
    delete h;
}

}  // namespace

extern "C" {

ld_prepared* ld_prepare(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals)
{
    ld_prepared* h = new ld_prepared;
    h->plan = make_plan(M, n, m, d, marginals, get_shape());
    if (h->plan.status != LD_OK) {
        set_error(h->plan.status);
        delete h;
        return nullptr;
    }
    bool ok = hipGetDevice(&h->device) == hipSuccess;
    hipDeviceProp_t prop;
    ok = ok && hipGetDeviceProperties(&prop, h->device) == hipSuccess &&
         std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    ok = ok && hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreate(&h->e0) == hipSuccess && hipEventCreate(&h->e1) == hipSuccess;
    ok = ok && hipMalloc((void**)&h->dres, 64) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&h->hres, 64, hipHostMallocDefault) == hipSuccess;
    if (ok && !h->plan.blob.empty()) {
        ok = hipMalloc(&h->dblob, h->plan.blob.size()) == hipSuccess &&
             hipMemcpy(h->dblob, h->plan.blob.data(), h->plan.blob.size(), hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        release(h);
        set_error(LD_EHIP);
        return nullptr;
    }
    return h;
}

int ld_run(ld_prepared* h, void* hip_stream, int64_t* value)
{
    if (!h || !value) {
        set_error(LD_EINVAL);
        return LD_EINVAL;
    }
    if (h->plan.kind == PK_ZERO) {
        *value = 0;
        h->last_ms = 0.f;
        return LD_OK;
    }
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : h->own;
    bool ok = true;
    if (h->plan.kind == PK_SUMABS) {
        ok = hipEventRecord(h->e0, s) == hipSuccess && launch_plan(h->plan, h->dblob, h->dres, s) &&
             hipEventRecord(h->e1, s) == hipSuccess;
    } else {
        int64_t cnt = 1, val = INT64_MIN;
        void* fargs[] = {(void*)&h->dres, (void*)&cnt, (void*)&val};
        ok = hipLaunchKernel(kernel_fill(), dim3(1), dim3(256), fargs, 0, s) == hipSuccess;
        ok = ok && hipEventRecord(h->e0, s) == hipSuccess;
        ok = ok && launch_sweep(h->plan, h->dblob, h->dres, s);
        ok = ok && hipEventRecord(h->e1, s) == hipSuccess;
    }
    ok = ok && hipMemcpyAsync(h->hres, h->dres, 8, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    ok = ok && hipEventElapsedTime(&h->last_ms, h->e0, h->e1) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        set_error(LD_EHIP);
        return LD_EHIP;
    }
    *value = *h->hres;
    return LD_OK;
}

float ld_last_kernel_ms(ld_prepared* h) { return h ? h->last_ms : 0.f; }

int ld_prepared_plan(const ld_prepared* h, ld_plan_info* info)
{
    if (!h || !info) return LD_EINVAL;
    info_from_plan(h->plan, info);
    return LD_OK;
}

void ld_release(ld_prepared* h) { release(h); }

int64_t ld_norm(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals)
{
    Plan p = make_plan(M, n, m, d, marginals, get_shape());
    return run_plan_sync(p);
}

int64_t ld_norm_range(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals, int32_t q,
                      uint64_t prefix_begin, uint64_t prefix_end)
{
    Plan p = make_range_plan(M, n, m, d, marginals, q, prefix_begin, prefix_end);
    return run_plan_sync(p);
}

int ld_last_error(void) { return t_last_error; }

const char* ld_error_string(int code)
{
    switch (code) {
    case LD_OK: return "ok";
    case LD_EINVAL: return "invalid argument";
    case LD_EMARG_D: return "marginals are defined for d = 1 only";
    case LD_ETOOBIG: return "problem exceeds the supported search space or kernel shapes";
    case LD_EHIP: return "HIP runtime error or no gfx950 device";
    case LD_EBUSY: return "server busy";
    case LD_PENDING: return "result pending";
    case LD_ENOTFOUND: return "unknown ticket";
    default: return "unknown error code";
    }
}

int ld_plan(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals, ld_plan_info* info)
{
    if (!info) return LD_EINVAL;
    Plan p = make_plan(M, n, m, d, marginals, get_shape());
    info_from_plan(p, info);
    return p.status;
}

uint32_t ld_gray_digit(uint32_t d, uint32_t i, uint64_t j)
{
    if (d == 2) return brgc_digit(i, j);
    if (d < 2) return 0;
    return dgc_digit(d, i, j);
}

int32_t ld_gray_change(uint32_t d, uint64_t j, uint32_t* from, uint32_t* to)
{
    if (j == 0 || d < 2) return -1;
    if (d == 2) {
        const uint32_t i = brgc_changed(j);
        const uint32_t g = brgc_digit(i, j);
        if (from) *from = 1 - g;
        if (to) *to = g;
        return (int32_t)i;
    }
    uint32_t f = 0, t = 0;
    const uint32_t i = dgc_change_rt(d, j, &f, &t);
    if (from) *from = f;
    if (to) *to = t;
    return (int32_t)i;
}

void ld_set_sweep_shape(int32_t p_target, int32_t c_min, int32_t r_drop, int32_t dary_ptab)
{
    SweepShape s = get_shape();
    if (p_target > 0) s.p_target = std::min(p_target, 40);
    if (c_min > 0) s.c_min = std::min(c_min, 31);
    if (r_drop >= 0) s.r_drop = r_drop ? 1 : 0;
    if (dary_ptab > 0) s.dary_ptab = std::min(dary_ptab, 16);
    set_shape(s);
}

}  // extern "C"
