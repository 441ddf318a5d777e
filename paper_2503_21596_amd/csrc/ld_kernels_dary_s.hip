// d-ary sweep kernels with the subset operands streamed through SGPRs (Dary32S),
// for d = 3, 4.  Compiled as LD_NPARTS compilation units (-DLD_PART=0 ..
// LD_NPARTS - 1), each instantiating every LD_NPARTS-th column count, so that the
// build runs them in parallel; part 0 holds the tables and the lookups.
#include <hip/hip_runtime.h>
#include <utility>

#include "ld_registry.h"
#include "ld_sweep_dary.h"

namespace ld {

// Waves per SIMD each instantiation is compiled for: the most whose register
// budget (512 / waves VGPRs) still holds the d state vectors, the subset scores and
// the temporaries of the Gray loop without spilling inside it (checked in the built
// code, see the ISA tests).  Left to itself the compiler spends the registers on
// scheduling freedom instead, and runs d = 3 at 36-40 columns and d = 4 at 28 with
// two waves, which leaves a quarter of the VALU issue slots idle.
constexpr int dary_s_waves(int mp, int d)
{
    if (d == 3) return mp <= 28 ? 4 : mp <= 40 ? 3 : 2;
    return mp <= 16 ? 4 : mp <= 28 ? 3 : 2;
}

// The same for the packed 16-bit kernels, by dword count W (two columns each):
// the d vectors of W dwords, the 2^R subset scores of each message and the
// temporaries.
constexpr int dary16_waves(int w, int d, int r)
{
    if (r == dary16_r(d)) return d == 3 ? (w <= 14 ? 3 : 2) : (w <= 12 ? 3 : 2);
    return d == 3 ? (w <= 20 ? 4 : 3) : (w <= 12 ? 4 : 3);
}

// Persistent queue kernel (see k_bin32): one item = a range of prefixes of one
// problem, one lane per prefix.  K is the sweep (Dary32S, plain or packed).
template <class K>
__device__ __forceinline__ void dary_s_queue(const QArgs& q)
{
    const uint32_t lane = threadIdx.x & 63;
    queue_priority(q);
    WaveBest wb;
    Item it;
    while (next_item(q, it)) {
        const Desc D = load_desc(q.descs + it.prob);
        wb.enter(it.prob, D.result);
        uint32_t best = 0;
        const uint32_t rounds = (it.count + 63) >> 6;
        for (uint32_t j = 0; j < rounds; ++j) {
            uint32_t i = lane + 64 * j;
            if (i >= it.count) i = it.count - 1;
            uint32_t pb = 0;
            K::prefix(D, D.pfx_base + it.p0 + i, pb);
            best = max(best, pb);
            if (D.rec) D.rec[it.p0 + i] = (int64_t)pb;
        }
        wb.add((int64_t)best);
        wb.item_end(q);
    }
    wb.flush();
}

template <int MP, int DD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(dary_s_waves(MP, DD)))) void k_dary32s(QArgs q)
{
    dary_s_queue<Dary32S<MP, DD, DARY_RS>>(q);
}

// At two waves per SIMD (d = 3, five low rows, more than 28 columns) enough
// registers are free to re-score both changed messages from one stream of operand
// loads; with three or four waves that would spill.
template <int W, int DD, int R>
constexpr bool dary16_paired()
{
    return DD == 3 && dary16_waves(W, DD, R) == 2;
}

template <int W, int DD, int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(dary16_waves(W, DD, R)))) void k_dary16s(QArgs q)
{
    dary_s_queue<Dary32S<W, DD, R, true, dary16_paired<W, DD, R>()>>(q);
}

#ifndef LD_PART
#define LD_PART 0
#define LD_NPARTS 1
#endif

constexpr int NMPD = MAX_MP / 4;   // mp = 4, 8, ..., 64
// zero before any part's registration runs (constant initialisation)
#if LD_PART == 0
const void* g_dary32s[MAX_D + 1][NMPD] = {};
const void* g_dary16s[2][MAX_D + 1][NMPD] = {};   // [larger R?][d][dword count 2, 4, ..., 32]
#else
extern const void* g_dary32s[MAX_D + 1][NMPD];
extern const void* g_dary16s[2][MAX_D + 1][NMPD];
#endif

namespace {

template <int DD, int MP>
void reg_one()
{
    if constexpr ((MP / 4 - 1) % LD_NPARTS == LD_PART) {
        if constexpr (dary_s_fits(MP, DD)) g_dary32s[DD][MP / 4 - 1] = (const void*)&k_dary32s<MP, DD>;
        if constexpr (dary16_fits(MP / 2, DD)) {
            g_dary16s[1][DD][MP / 4 - 1] = (const void*)&k_dary16s<MP / 2, DD, dary16_r(DD)>;
            g_dary16s[0][DD][MP / 4 - 1] = (const void*)&k_dary16s<MP / 2, DD, dary16_r_small(DD)>;
        }
    }
}

template <int DD, int... I>
void reg_mps(std::integer_sequence<int, I...>)
{
    (reg_one<DD, 4 * (I + 1)>(), ...);
}

struct Init {
    Init()
    {
        reg_mps<3>(std::make_integer_sequence<int, NMPD>{});
        reg_mps<4>(std::make_integer_sequence<int, NMPD>{});
    }
} g_init;

}  // namespace

#if LD_PART == 0
const void* kernel_dary32s(int d, int mp)
{
    if (d < 0 || d > MAX_D || mp < 4 || mp > MAX_MP || (mp & 3)) return nullptr;
    return g_dary32s[d][mp / 4 - 1];
}

const void* kernel_dary16s(int d, int words, int r)
{
    if (d < 0 || d > MAX_D || words < 2 || words > MAX_MP / 2 || (words & 1)) return nullptr;
    if (r != dary16_r(d) && r != dary16_r_small(d)) return nullptr;
    return g_dary16s[r == dary16_r(d) ? 1 : 0][d][words / 2 - 1];
}
#endif

}  // namespace ld
