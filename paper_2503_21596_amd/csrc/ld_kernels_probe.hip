// Clock and VALU-rate probe for the measurement of the int32 VALU roofline.
//
// Every wave issues a known number of v_sad_u32 (the scoring instruction of the
// sweeps, with one SGPR operand as there) in eight independent chains, and reads
// the shader-clock counter (s_memtime) and the constant-rate counter
// (s_memrealtime) around them.  The ratio of the two counter deltas gives the
// engine clock while the chip runs a VALU-bound load; the kernel time gives the
// VALU issue rate the chip sustains.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ld {

__global__ __launch_bounds__(256) void k_valu_probe(uint32_t iters, uint32_t seed, uint64_t* __restrict__ out)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    uint32_t a0 = seed + lane, a1 = a0 ^ 1u, a2 = a0 ^ 2u, a3 = a0 ^ 3u;
    uint32_t a4 = a0 ^ 4u, a5 = a0 ^ 5u, a6 = a0 ^ 6u, a7 = a0 ^ 7u;
    const uint32_t x = seed * 2654435761u + lane;
    const uint32_t y = __builtin_amdgcn_readfirstlane(seed ^ 0x9e3779b9u);
    const uint64_t c0 = __builtin_amdgcn_s_memtime();
    const uint64_t r0 = __builtin_amdgcn_s_memrealtime();
    for (uint32_t i = 0; i < iters; ++i) {
        // 64 v_sad_u32 per iteration, each chain advanced every eighth instruction
#define LD_SAD8 \
        "v_sad_u32 %0, %8, %9, %0\n" "v_sad_u32 %1, %8, %9, %1\n" "v_sad_u32 %2, %8, %9, %2\n" \
        "v_sad_u32 %3, %8, %9, %3\n" "v_sad_u32 %4, %8, %9, %4\n" "v_sad_u32 %5, %8, %9, %5\n" \
        "v_sad_u32 %6, %8, %9, %6\n" "v_sad_u32 %7, %8, %9, %7\n"
        asm volatile(LD_SAD8 LD_SAD8 LD_SAD8 LD_SAD8 LD_SAD8 LD_SAD8 LD_SAD8 LD_SAD8
                     : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                     : "v"(x), "s"(y));
#undef LD_SAD8
    }
    const uint64_t c1 = __builtin_amdgcn_s_memtime();
    const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
    const uint32_t sink = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
    if (lane == 0) {
        out[3 * wave + 0] = c1 - c0;
        out[3 * wave + 1] = r1 - r0;
        out[3 * wave + 2] = sink;
    }
}

const void* kernel_valu_probe() { return (const void*)&k_valu_probe; }

}  // namespace ld
