// d-ary sweep kernels (L_d, d >= 3), plus the small helper kernels.
#include <hip/hip_runtime.h>
#include <utility>

#include "ld_registry.h"
#include "ld_sweep.h"

namespace ld {

template <int MP, int DD>
__global__ __launch_bounds__(256) void k_dary32(Desc D)
{
    uint32_t best = 0;
    const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t rounds = (D.n_prefix + nth - 1) / nth;
    for (uint64_t j = 0; j < rounds; ++j) {
        uint64_t p = lane + j * nth;
        if (p >= D.n_prefix) p = D.n_prefix - 1;
        Dary32<MP, DD>::prefix(D, D.pfx_base + p, best);
    }
    publish(D.result, (int64_t)best);
}

template <int MP, int DD>
__global__ __launch_bounds__(256) void k_dary64(Desc D)
{
    int64_t best = INT64_MIN;
    const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t rounds = (D.n_prefix + nth - 1) / nth;
    for (uint64_t j = 0; j < rounds; ++j) {
        uint64_t p = lane + j * nth;
        if (p >= D.n_prefix) p = D.n_prefix - 1;
        Dary64<MP, DD>::prefix(D, D.pfx_base + p, best);
    }
    publish(D.result, best);
}

// Wide sweep (any column count / alphabet), one wave per block; dynamic LDS holds
// the state vectors and, for d-ary problems, the d message norms.
__global__ __launch_bounds__(64) void k_wide(Desc D)
{
    extern __shared__ int64_t lds[];
    int64_t best = INT64_MIN;
    for (uint64_t p = blockIdx.x; p < D.n_prefix; p += gridDim.x) {
        if (D.kind == KIND_LD) Wide::prefix_dary(D, D.pfx_base + p, lds, lds + (size_t)D.d * D.m, best);
        else Wide::prefix_bin(D, D.pfx_base + p, lds, best);
    }
    publish(D.result, best);
}

// sum_xy |M_xy| of an n x m int32 matrix: the value of L_d when d >= n (every
// row can take its own message, Eq. (L_o_norm)).  One block, int64 partials.
__global__ __launch_bounds__(256) void k_sumabs(const int32_t* __restrict__ M, int64_t count,
                                                int64_t* __restrict__ result)
{
    int64_t acc = 0;
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
        const int64_t v = M[i];
        acc += v < 0 ? -v : v;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ int64_t part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *result = part[0] + part[1] + part[2] + part[3];
}

// out[i] = value for i < count (result slots start at INT64_MIN before a max)
__global__ __launch_bounds__(256) void k_fill(int64_t* __restrict__ out, int64_t count, int64_t value)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = value;
}

namespace {

constexpr int NMPD = MAX_MP / 4;   // mp = 4, 8, ..., 64
const void* g_dary32[MAX_D + 1][NMPD] = {};
const void* g_dary64[MAX_D + 1][NMPD] = {};

template <int DD, int MP>
void reg_one()
{
    if constexpr (dary_fits(MP, DD)) {
        g_dary32[DD][MP / 4 - 1] = (const void*)&k_dary32<MP, DD>;
        if constexpr (MP % 8 == 0 && dary_fits(2 * MP, DD))
            g_dary64[DD][MP / 4 - 1] = (const void*)&k_dary64<MP, DD>;
    }
}

template <int DD, int... I>
void reg_d(std::integer_sequence<int, I...>)
{
    (reg_one<DD, 4 * (I + 1)>(), ...);
}

struct Init {
    Init()
    {
        reg_d<3>(std::make_integer_sequence<int, NMPD>{});
        reg_d<4>(std::make_integer_sequence<int, NMPD>{});
        reg_d<5>(std::make_integer_sequence<int, NMPD>{});
        reg_d<6>(std::make_integer_sequence<int, NMPD>{});
        reg_d<7>(std::make_integer_sequence<int, NMPD>{});
        reg_d<8>(std::make_integer_sequence<int, NMPD>{});
    }
} g_init;

}  // namespace

const void* kernel_dary32(int d, int mp)
{
    if (d < 3 || d > MAX_D || mp < 4 || mp > MAX_MP || (mp & 3)) return nullptr;
    return g_dary32[d][mp / 4 - 1];
}

const void* kernel_dary64(int d, int mp)
{
    if (d < 3 || d > MAX_D || mp < 8 || mp > MAX_MP || (mp & 7)) return nullptr;
    return g_dary64[d][mp / 4 - 1];
}

const void* kernel_sumabs() { return (const void*)&k_sumabs; }
const void* kernel_wide() { return (const void*)&k_wide; }
const void* kernel_fill() { return (const void*)&k_fill; }

const void* lookup_bin32_kind0(int mp, int R);
const void* lookup_bin32_kind1(int mp, int R);
const void* lookup_bin32_kind2(int mp, int R);
const void* lookup_bin64_kind0(int mp);
const void* lookup_bin64_kind1(int mp);
const void* lookup_bin64_kind2(int mp);

const void* kernel_bin32(int kind, int mp, int R)
{
    switch (kind) {
    case KIND_L1: return lookup_bin32_kind0(mp, R);
    case KIND_MARG: return lookup_bin32_kind1(mp, R);
    case KIND_L2: return lookup_bin32_kind2(mp, R);
    default: return nullptr;
    }
}

const void* kernel_bin64(int kind, int mp)
{
    switch (kind) {
    case KIND_L1: return lookup_bin64_kind0(mp);
    case KIND_MARG: return lookup_bin64_kind1(mp);
    case KIND_L2: return lookup_bin64_kind2(mp);
    default: return nullptr;
    }
}

}  // namespace ld
