// d-ary sweep kernels (L_d, d >= 3), plus the small helper kernels.
#include <hip/hip_runtime.h>
#include <utility>

#include "ld_registry.h"
#include "ld_program.h"
#include "ld_sweep_dary.h"

namespace ld {

// Persistent queue kernels (see k_bin32): one item = a range of prefixes of one
// problem, one lane per prefix.
template <int MP, int DD>
__global__ __launch_bounds__(256) void k_dary32(QArgs q)
{
    constexpr int R = dary_r(MP, DD);
    using K = Dary32<MP, DD, R>;
    const uint32_t lane = threadIdx.x & 63;
    uint32_t off[K::NO][MP];
    queue_priority(q);
    WaveBest wb;
    Item it;
    while (next_item(q, it)) {
        const Desc D = load_desc(q.descs + it.prob);
        if (wb.enter(it.prob, D.result)) K::load_offs(D, off);
        uint32_t best = 0;
        const uint32_t rounds = (it.count + 63) >> 6;
        for (uint32_t j = 0; j < rounds; ++j) {
            uint32_t i = lane + 64 * j;
            if (i >= it.count) i = it.count - 1;
            uint32_t pb = 0;
            K::prefix(D, D.pfx_base + it.p0 + i, off, pb);
            best = max(best, pb);
            if (D.rec) D.rec[it.p0 + i] = (int64_t)pb;
        }
        wb.add((int64_t)best);
        wb.item_end(q);
    }
    wb.flush();
}

template <int MP, int DD>
__global__ __launch_bounds__(256) void k_dary64(QArgs q)
{
    const uint32_t lane = threadIdx.x & 63;
    queue_priority(q);
    WaveBest wb;
    Item it;
    while (next_item(q, it)) {
        const Desc D = load_desc(q.descs + it.prob);
        wb.enter(it.prob, D.result);
        int64_t best = INT64_MIN;
        const uint32_t rounds = (it.count + 63) >> 6;
        for (uint32_t j = 0; j < rounds; ++j) {
            uint32_t i = lane + 64 * j;
            if (i >= it.count) i = it.count - 1;
            int64_t pb = INT64_MIN;
            Dary64<MP, DD>::prefix(D, D.pfx_base + it.p0 + i, pb);
            best = pb > best ? pb : best;
            if (D.rec) D.rec[it.p0 + i] = pb;
        }
        wb.add(best);
        wb.item_end(q);
    }
    wb.flush();
}

// Wide sweep (any column count / alphabet), one wave per block; each item's
// prefixes are swept one after another by the whole wave.  Dynamic LDS holds
// the state vectors and, for d-ary problems, the d message norms.
__global__ __launch_bounds__(64) void k_wide(QArgs q)
{
    extern __shared__ int64_t lds[];
    queue_priority(q);
    WaveBest wb;
    Item it;
    while (next_item(q, it)) {
        const Desc D = load_desc(q.descs + it.prob);
        wb.enter(it.prob, D.result);
        int64_t best = INT64_MIN;
        for (uint32_t i = 0; i < it.count; ++i) {
            const uint64_t v = D.pfx_base + it.p0 + i;
            int64_t pb = INT64_MIN;
            if (D.kind == KIND_LD) Wide::prefix_dary(D, v, lds, lds + (size_t)D.d * D.m, pb);
            else Wide::prefix_bin(D, v, lds, pb);
            best = pb > best ? pb : best;
            if (D.rec) D.rec[it.p0 + i] = pb;
        }
        wb.add(best);
        wb.item_end(q);
    }
    wb.flush();
}

// sum_xy |M_xy| of int32 matrices, one block per matrix: the value of L_d when
// d >= n (every row can take its own message, Eq. (L_o_norm)).  int64 partials.
__global__ __launch_bounds__(256) void k_sumabs_many(const SumItem* __restrict__ items, uint32_t n)
{
    __shared__ int64_t part[4];
    for (uint32_t b = blockIdx.x; b < n; b += gridDim.x) {
        const SumItem si = items[b];
        int64_t acc = 0;
        for (int64_t i = threadIdx.x; i < si.count; i += blockDim.x) {
            const int64_t v = si.M[i];
            acc += v < 0 ? -v : v;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) *si.result = part[0] + part[1] + part[2] + part[3];
        __syncthreads();
    }
}

// Start of a run: result slots to INT64_MIN (a max follows), queue heads to 0.
// A kernel rather than a memset so that captured graphs replay it correctly.
__global__ __launch_bounds__(256) void k_reset(int64_t* __restrict__ results, uint32_t n_results,
                                               uint32_t* __restrict__ heads, uint32_t n_heads)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_results; i += stride) results[i] = INT64_MIN;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_heads; i += stride) heads[i] = 0;
}

// dst[i] = src[i] for i < n, i = first, first + step, ...: up to four loads in
// flight per thread before its stores
__device__ __forceinline__ void copy16x4(const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n,
                                         uint64_t first, uint64_t step)
{
    for (uint64_t i = first; i < n; i += 4 * step) {
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i + k * step < n) v[k] = src[i + k * step];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i + k * step < n) dst[i + k * step] = v[k];
    }
}

// Server steps, one launch at raised wave priority (as express sweeps: a step
// shares each SIMD with the waves of a long bulk sweep).  Blocks [0, nops) each
// copy one newly admitted table or descriptor from the step buffer in host memory
// to its arena or descriptor slot; the blocks after them set the new problems'
// result slots to INT64_MIN and their unfinished-item counters to their item
// counts, and copy the rest of the step buffer (queue items with their zeroed
// heads, sum jobs) to device memory.  Host memory is microseconds away, so no
// thread waits on more than one load from it before its loads of data.
__global__ __launch_bounds__(256) void k_stage(StageArgs a)
{
    __builtin_amdgcn_s_setprio(3);
    if (blockIdx.x < a.nops) {
        const uint32_t b = blockIdx.x;
        const ScatterOp op = b < STAGE_INLINE ? a.iops[b] : a.ops[b];
        if ((((uintptr_t)op.src | (uintptr_t)op.dst | op.bytes) & 15) == 0)
            copy16x4((const uint4*)op.src, (uint4*)op.dst, op.bytes / 16, threadIdx.x, blockDim.x);
        else
            for (uint64_t i = threadIdx.x; i < op.bytes; i += blockDim.x) op.dst[i] = op.src[i];
        return;
    }
    const uint32_t nb = gridDim.x - a.nops;
    const uint32_t stride = nb * blockDim.x;
    const uint32_t tid = (blockIdx.x - a.nops) * blockDim.x + threadIdx.x;
    for (uint32_t i = tid; i < a.n_slots; i += stride) {
        const uint32_t slot = i < STAGE_INLINE ? a.islots[i] : a.slots[i];
        a.results[slot] = INT64_MIN;
        a.left[slot] = i < STAGE_INLINE ? a.icounts[i] : a.counts[i];
    }
    copy16x4(a.copy_src, a.copy_dst, a.copy_n16, tid, stride);
}

// Server steps: every result slot to host memory after the step's sweeps, at
// raised wave priority (as k_stage).
__global__ __launch_bounds__(256) void k_publish(const int64_t* __restrict__ results, int64_t* __restrict__ out,
                                                 uint32_t n)
{
    __builtin_amdgcn_s_setprio(3);
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = results[i];
    __threadfence_system();
}

// Locating a maximiser: *first = the smallest i < n with rec[i] == target (the
// caller sets *first to UINT64_MAX beforehand with k_set_u64).
__global__ __launch_bounds__(256) void k_first_equal(const int64_t* __restrict__ rec, uint64_t n, int64_t target,
                                                     unsigned long long* __restrict__ first)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (rec[i] == target) atomicMin(first, (unsigned long long)i);
}

__global__ __launch_bounds__(64) void k_set_u64(unsigned long long* __restrict__ p, unsigned long long v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// The other side of a binary strategy (Eq. LM2 is a max over a and b of a^T M b):
// out[i] = sign(sum_j A[i][j] v[j]) with ties to +1, for A = M (rows = 1) or M^T
// (rows = 0), M int32 n x m row-major, v in {-1, +1}.  fix0: out[0] = +1 (the
// marginal row or column of Eq. LMarg).
__global__ __launch_bounds__(256) void k_signs(const int32_t* __restrict__ M, int32_t n, int32_t m,
                                               const int32_t* __restrict__ v, int32_t rows, int32_t fix0,
                                               int32_t* __restrict__ out)
{
    const int32_t len = rows ? n : m, other = rows ? m : n;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) {
        int64_t acc = 0;
        for (int32_t j = 0; j < other; ++j) {
            const int64_t e = rows ? M[(size_t)i * m + j] : M[(size_t)j * m + i];
            acc += e * v[j];
        }
        out[i] = (fix0 && i == 0) ? 1 : (acc < 0 ? -1 : 1);
    }
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

const void* kernel_sumabs_many() { return (const void*)&k_sumabs_many; }
const void* kernel_wide() { return (const void*)&k_wide; }
const void* kernel_reset() { return (const void*)&k_reset; }
const void* kernel_stage() { return (const void*)&k_stage; }
const void* kernel_publish() { return (const void*)&k_publish; }
const void* kernel_first_equal() { return (const void*)&k_first_equal; }
const void* kernel_set_u64() { return (const void*)&k_set_u64; }
const void* kernel_signs() { return (const void*)&k_signs; }

const void* lookup_bin32_kind0(int mp, int R);
const void* lookup_bin32_kind1(int mp, int R);
const void* lookup_bin32_kind2(int mp, int R);
const void* lookup_bin32s_kind0(int mp, int R);
const void* lookup_bin32s_kind1(int mp, int R);
const void* lookup_bin32s_kind2(int mp, int R);
const void* lookup_bin16s_kind0(int words, int r);
const void* lookup_bin16s_kind2(int words, int r);
const void* lookup_mfma_kind0(int mp);
const void* lookup_mfma_kind1(int mp);
const void* lookup_mfma_kind2(int mp);
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

const void* kernel_bin32s(int kind, int mp, int R)
{
    switch (kind) {
    case KIND_L1: return lookup_bin32s_kind0(mp, R);
    case KIND_MARG: return lookup_bin32s_kind1(mp, R);
    case KIND_L2: return lookup_bin32s_kind2(mp, R);
    default: return nullptr;
    }
}

const void* kernel_bin16s(int kind, int words, int r)
{
    switch (kind) {
    case KIND_L1:
    case KIND_MARG: return lookup_bin16s_kind0(words, r);
    case KIND_L2: return lookup_bin16s_kind2(words, r);
    default: return nullptr;
    }
}

const void* kernel_mfma(int kind, int mp)
{
    switch (kind) {
    case KIND_L1: return lookup_mfma_kind0(mp);
    case KIND_MARG: return lookup_mfma_kind1(mp);
    case KIND_L2: return lookup_mfma_kind2(mp);
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
