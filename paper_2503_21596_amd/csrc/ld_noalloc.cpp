// ld_norm_noalloc: the plain solve of ld_norm on a fixed device-side scratch
// array instead of library-allocated device memory (see include/ld.h).
//
// The device image of the problem (tables, descriptor, queue head, result slot)
// lives in `scratch`, a file-scope __device__ array of LD_NOALLOC_SCRATCH_BYTES
// that every GPU the library runs on holds until the process ends.  In host code
// the array's name is only a host-side stand-in, so its device address is looked
// up once per device with hipGetSymbolAddress and every kernel argument and copy
// uses that address.  Nothing here calls hipMalloc, hipFree or hipHostMalloc.
#include <hip/hip_runtime.h>

#include <array>
#include <cstring>
#include <mutex>
#include <vector>

#include "ld.h"
#include "ld_api_internal.h"
#include "ld_plan.h"
#include "ld_program.h"

namespace {

static __device__ __align__(256) uint8_t scratch[LD_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;

struct DeviceScratch {
    std::mutex mu;          // calls on one device take turns: they share its array
    bool looked_up = false;
    uint8_t* ptr = nullptr; // device address of `scratch` on this device
};

std::array<DeviceScratch, MAX_DEVICES> g_scratch;

// device address of this device's array (current device set), or null on error
uint8_t* scratch_address(DeviceScratch& ds)
{
    if (!ds.looked_up) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        ds.ptr = (uint8_t*)p;
        ds.looked_up = true;
    }
    return ds.ptr;
}

}  // namespace

using namespace ld;

extern "C" int ld_norm_noalloc(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals,
                               int64_t* value, void* hip_stream)
{
    if (!value) {
        set_error(LD_EINVAL);
        return LD_EINVAL;
    }
    *value = INT64_MIN;
    Plan p = make_plan(M, n, m, d, marginals, get_shape());
    if (p.status != LD_OK) {
        set_error(p.status);
        return p.status;
    }
    if (p.kind == PK_ZERO) {
        *value = 0;
        return LD_OK;
    }
    Program P = build_program({&p}, plain_item_shape());
    if (P.image.size() > LD_NOALLOC_SCRATCH_BYTES) {
        set_error(LD_ESCRATCH);
        return LD_ESCRATCH;
    }
    int dev = 0;
    if (!device_ok(&dev) || dev < 0 || dev >= MAX_DEVICES) {
        set_error(LD_EHIP);
        return LD_EHIP;
    }
    DeviceScratch& ds = g_scratch[dev];
    std::lock_guard<std::mutex> g(ds.mu);
    uint8_t* base = scratch_address(ds);
    if (!base) {
        set_error(LD_EHIP);
        return LD_EHIP;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    patch_program(P, base);
    // the image is uploaded whole; enqueue_program resets the queue head and the
    // result slot with a kernel, so nothing left from an earlier call is read
    int64_t v = INT64_MIN;
    bool ok = hipMemcpyAsync(base, P.image.data(), P.image.size(), hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && enqueue_program(P, s, nullptr);
    ok = ok && hipMemcpyAsync(&v, base + P.off_results, sizeof v, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        set_error(LD_EHIP);
        return LD_EHIP;
    }
    *value = v;
    return LD_OK;
}
