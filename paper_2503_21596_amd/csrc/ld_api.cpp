// C ABI: plain, range, prepared and introspection entry points (see include/ld.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ld.h"
#include "ld_api_internal.h"
#include "ld_gray.h"
#include "ld_plan.h"
#include "ld_program.h"
#include "ld_registry.h"
#include "ld_tune.h"

namespace ld {

thread_local int t_last_error = LD_OK;

void set_error(int code) { t_last_error = code; }

bool device_ok(int* dev_out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return false;
    if (dev_out) *dev_out = dev;
    return true;
}

// ---------------------------------------------------------------------------
// per-thread device context: stream, device image buffer, pinned staging, results

namespace {

struct Ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    std::vector<hipStream_t> side;   // launches of many-problem programs fan out over these
    std::vector<hipEvent_t> fan_ev;
    void* dbuf = nullptr;
    size_t dcap = 0;
    void* hbuf = nullptr;
    size_t hcap = 0;
    int64_t* hres = nullptr;
    size_t rcap = 0;
    ~Ctx()
    {
        // released at thread exit; errors here cannot be reported
        if (dbuf) (void)hipFree(dbuf);
        if (hbuf) (void)hipHostFree(hbuf);
        if (hres) (void)hipHostFree(hres);
        for (hipEvent_t e : fan_ev)
            if (e) (void)hipEventDestroy(e);
        for (hipStream_t s : side)
            if (s) (void)hipStreamDestroy(s);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

thread_local Ctx t_ctx;

bool ctx_ready(Ctx& c)
{
    int dev = 0;
    if (c.stream) return hipGetDevice(&dev) == hipSuccess && dev == c.device;
    if (!device_ok(&dev)) return false;
    if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess) return false;
    c.device = dev;
    return true;
}

bool ensure(Ctx& c, size_t bytes, size_t nres)
{
    if (bytes > c.dcap) {
        const size_t cap = std::max<size_t>(bytes, (size_t)1 << 20);
        if (c.dbuf) (void)hipFree(c.dbuf);
        if (c.hbuf) (void)hipHostFree(c.hbuf);
        c.dbuf = c.hbuf = nullptr;
        c.dcap = c.hcap = 0;
        if (hipMalloc(&c.dbuf, cap) != hipSuccess) return false;
        if (hipHostMalloc(&c.hbuf, cap, hipHostMallocDefault) != hipSuccess) return false;
        c.dcap = c.hcap = cap;
    }
    if (nres > c.rcap) {
        const size_t cap = std::max<size_t>(nres, 1024);
        if (c.hres) (void)hipHostFree(c.hres);
        c.hres = nullptr;
        c.rcap = 0;
        if (hipHostMalloc((void**)&c.hres, 8 * cap, hipHostMallocDefault) != hipSuccess) return false;
        c.rcap = cap;
    }
    return true;
}

}  // namespace

// Solve a set of planned problems synchronously on the calling thread's buffers.
// out[i] receives problem i's value; problems with value 0 need no search.
// the thread's side streams and fork/join events for fanned-out launches
bool ensure_side(Ctx& c, int n)
{
    while ((int)c.side.size() < n) {
        hipStream_t s2 = nullptr;
        if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess) return false;
        c.side.push_back(s2);
    }
    while ((int)c.fan_ev.size() < n + 1) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return false;
        c.fan_ev.push_back(e);
    }
    return true;
}

bool run_plans_sync(const std::vector<const Plan*>& plans, const ItemShape& shape, int64_t* out, hipStream_t s)
{
    Ctx& c = t_ctx;
    Program P = build_program(plans, shape);
    if (!ctx_ready(c) || !ensure(c, P.image.size(), P.n_probs)) return false;
    if (!s) s = c.stream;
    patch_program(P, c.dbuf);
    std::memcpy(c.hbuf, P.image.data(), P.image.size());
    // several kernel shapes: let their launches overlap on side streams
    const int n_side = P.launches.size() > 1 ? batch_side_streams() : 0;
    if (n_side > 0 && !ensure_side(c, n_side)) return false;
    const std::vector<hipStream_t> side(c.side.begin(), c.side.begin() + n_side);
    const std::vector<hipEvent_t> evs(c.fan_ev.begin(), c.fan_ev.begin() + (n_side > 0 ? n_side + 1 : 0));
    bool ok = hipMemcpyAsync(c.dbuf, c.hbuf, P.image.size(), hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && enqueue_program_fanned(P, s, c.hres, side, evs);
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return false;
    }
    std::memcpy(out, c.hres, 8 * (size_t)P.n_probs);
    for (int i : P.zero) out[i] = 0;
    return true;
}

int64_t run_plan_sync(const Plan& p)
{
    if (p.status != LD_OK) {
        set_error(p.status);
        return INT64_MIN;
    }
    if (p.kind == PK_ZERO) return 0;
    int64_t v = INT64_MIN;
    if (!run_plans_sync({&p}, plain_item_shape(), &v, nullptr)) {
        set_error(LD_EHIP);
        return INT64_MIN;
    }
    return v;
}

}  // namespace ld

using namespace ld;

struct ld_prepared {
    Plan plan;
    Program prog;
    int device = -1;
    hipStream_t own = nullptr;
    void* dev = nullptr;
    int64_t* hres = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float last_ms = 0.f;
};

namespace ld {

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
    if (!p.kernel) info->kernel = -1;
    else if (p.wide) info->kernel = 4;
    else if (p.mfma) info->kernel = 2;
    else if (p.pack16) info->kernel = 5;
    else if (p.i64) info->kernel = 3;
    else if (p.kind == PK_LD) info->kernel = p.kernel == kernel_dary32s(p.d, p.mp) ? 1 : 0;
    else info->kernel = p.kernel == kernel_bin32s(p.kind, p.mp, p.R) ? 1 : 0;
}

}  // namespace ld

namespace {

void release(ld_prepared* h)
{
    if (!h) return;
    if (h->dev) (void)hipFree(h->dev);
    if (h->hres) (void)hipHostFree(h->hres);
    if (h->e0) (void)hipEventDestroy(h->e0);
    if (h->e1) (void)hipEventDestroy(h->e1);
    if (h->own) (void)hipStreamDestroy(h->own);
    delete h;
}

}  // namespace

extern "C" {

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

ld_prepared* ld_prepare(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals)
{
    ld_prepared* h = new ld_prepared;
    h->plan = make_plan(M, n, m, d, marginals, get_shape());
    if (h->plan.status != LD_OK) {
        set_error(h->plan.status);
        delete h;
        return nullptr;
    }
    h->prog = build_program({&h->plan}, plain_item_shape());
    bool ok = device_ok(&h->device);
    ok = ok && hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreate(&h->e0) == hipSuccess && hipEventCreate(&h->e1) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&h->hres, 64, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMalloc(&h->dev, h->prog.image.size()) == hipSuccess;
    if (ok) {
        patch_program(h->prog, h->dev);
        ok = hipMemcpy(h->dev, h->prog.image.data(), h->prog.image.size(), hipMemcpyHostToDevice) == hipSuccess;
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
    bool ok = hipEventRecord(h->e0, s) == hipSuccess;
    ok = ok && enqueue_program(h->prog, s, nullptr);
    ok = ok && hipEventRecord(h->e1, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(h->hres, (uint8_t*)h->dev + h->prog.off_results, 8, hipMemcpyDeviceToHost, s) ==
                   hipSuccess;
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
    case LD_ECANCELED: return "request cancelled";
    case LD_ESCRATCH: return "problem image exceeds the static scratch array of ld_norm_noalloc";
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

void ld_set_sweep_shape(int32_t p_target, int32_t c_min, int32_t r_drop, int32_t dary_ptab, int32_t sgpr_r,
                        int32_t dary_sgpr)
{
    SweepShape s = get_shape();
    if (p_target > 0) s.p_target = std::min(p_target, 40);
    if (c_min > 0) s.c_min = std::min(c_min, 31);
    if (r_drop >= 0) s.r_drop = r_drop ? 1 : 0;
    if (dary_ptab > 0) s.dary_ptab = std::min(dary_ptab, 16);
    // an explicit variant replaces the tuned per-width choices of its kinds
    if (sgpr_r >= 0) {
        s.sgpr_r = (sgpr_r == VARIANT_MFMA || sgpr_r == VARIANT_PACK16) ? sgpr_r : std::min(sgpr_r, MAX_RS);
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 4; ++b) s.variant[c][b] = -1;
    }
    if (dary_sgpr >= 0) {
        s.dary_sgpr = dary_sgpr == VARIANT_PACK16 ? VARIANT_PACK16 : dary_sgpr ? 1 : 0;
        for (int c = 2; c < 4; ++c)
            for (int b = 0; b < 4; ++b) s.variant[c][b] = -1;
    }
    set_shape(s);
}

void ld_set_lane_fill(int32_t p_fill)
{
    if (p_fill < 0) return;
    SweepShape s = get_shape();
    s.p_fill = std::min(p_fill, 40);
    set_shape(s);
}

void ld_set_launch_waves(int32_t waves_per_simd)
{
    if (waves_per_simd >= 0) set_launch_waves(std::min(waves_per_simd, 32));
}

int ld_valu_probe(double target_ms, ld_valu_probe_result* out)
{
    if (!out || !(target_ms > 0)) {
        set_error(LD_EINVAL);
        return LD_EINVAL;
    }
    std::memset(out, 0, sizeof(*out));
    int dev = 0, wall_khz = 0;
    hipDeviceProp_t prop;
    if (!device_ok(&dev) || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0) {
        (void)hipGetLastError();
        set_error(LD_EHIP);
        return LD_EHIP;
    }
    // four blocks of four waves per CU: four waves per SIMD
    const uint32_t blocks = 4u * (uint32_t)prop.multiProcessorCount, threads = 256;
    const uint32_t waves = blocks * threads / 64;
    uint64_t* d_out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = hipMalloc((void**)&d_out, 24 * (size_t)waves) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    float ms = 0;
    uint32_t iters = 256;
    auto launch = [&](uint32_t it) {
        uint32_t seed = 12345u;
        void* args[] = {(void*)&it, (void*)&seed, (void*)&d_out};
        bool k = hipEventRecord(e0, s) == hipSuccess;
        k = k && hipLaunchKernel(kernel_valu_probe(), dim3(blocks), dim3(threads), args, 0, s) == hipSuccess;
        k = k && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        return k && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    };
    // a short launch sizes the measured one
    ok = ok && launch(iters);
    if (ok) {
        const double scale = target_ms / std::max(0.01, (double)ms);
        iters = (uint32_t)std::min(4.0e8, std::max(256.0, iters * scale));
        ok = launch(iters);
    }
    std::vector<uint64_t> h(3 * (size_t)waves);
    ok = ok && hipMemcpy(h.data(), d_out, 24 * (size_t)waves, hipMemcpyDeviceToHost) == hipSuccess;
    if (ok) {
        std::vector<double> clk;
        for (uint32_t w = 0; w < waves; ++w)
            if (h[3 * w + 1]) clk.push_back((double)h[3 * w] * wall_khz * 1e3 / (double)h[3 * w + 1]);
        std::sort(clk.begin(), clk.end());
        out->sclk_hz = clk.empty() ? 0.0 : clk[clk.size() / 2];
        out->sclk_max_hz = 1e3 * (double)prop.clockRate;
        out->seconds = ms * 1e-3;
        out->valu_lane_ops_per_s = (double)waves * iters * 64.0 * 64.0 / (ms * 1e-3);
        out->compute_units = prop.multiProcessorCount;
        out->waves = (int32_t)waves;
    }
    if (d_out) (void)hipFree(d_out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (!ok) {
        (void)hipGetLastError();
        set_error(LD_EHIP);
        return LD_EHIP;
    }
    return LD_OK;
}

}  // extern "C"
