// Binary-kind sweep kernels (L1, L_marg, L2) for one kind, selected by LD_KIND at
// compile time so the three kinds build as separate objects in parallel.
#include <hip/hip_runtime.h>
#include <utility>

#include "ld_registry.h"
#include "ld_sweep.h"

#ifndef LD_KIND
#error "LD_KIND must be 0 (L1), 1 (L_marg) or 2 (L2)"
#endif

namespace ld {

// Persistent queue kernel: each wave takes items (problem, prefix range); lane l
// of the wave takes prefixes p0 + l, p0 + l + 64, ... of the item.  Lanes past
// the item's end repeat its last prefix, which cannot change a maximum, so the
// wave stays converged.  The low-row operands are reloaded, and the running max
// published, only when the problem changes between consecutive items.
template <int MP, int KIND, int R>
__global__ __launch_bounds__(256) void k_bin32(QArgs q)
{
    using B = Bin32<MP, KIND, R>;
    const uint32_t lane = threadIdx.x & 63;
    uint32_t off[B::K][B::NW][MP];
    queue_priority(q);
    WaveBest wb;
    Item it;
    while (next_item(q, it)) {
        const Desc D = load_desc(q.descs + it.prob);
        if (wb.enter(it.prob, D.result)) B::load_offs(D, off);
        uint32_t best = B::best_init();
        const uint32_t rounds = (it.count + 63) >> 6;
        for (uint32_t j = 0; j < rounds; ++j) {
            uint32_t i = lane + 64 * j;
            if (i >= it.count) i = it.count - 1;
            uint32_t pb = B::best_init();
            B::prefix(D, D.pfx_base + it.p0 + i, off, pb);
            best = B::better(best, pb);
            if (D.rec) D.rec[it.p0 + i] = B::finish(pb);
        }
        wb.add(B::finish(best));
        wb.item_end(q);
    }
    wb.flush();
}

// Same queue loop with the low-row operands streamed through SGPRs (Bin32S).
template <int MP, int KIND, int R>
__global__ __launch_bounds__(256) void k_bin32s(QArgs q)
{
    using B = Bin32S<MP, KIND, R>;
    const uint32_t lane = threadIdx.x & 63;
    queue_priority(q);
    WaveBest wb;
    Item it;
    while (next_item(q, it)) {
        const Desc D = load_desc(q.descs + it.prob);
        wb.enter(it.prob, D.result);
        uint32_t best = B::best_init();
        const uint32_t rounds = (it.count + 63) >> 6;
        for (uint32_t j = 0; j < rounds; ++j) {
            uint32_t i = lane + 64 * j;
            if (i >= it.count) i = it.count - 1;
            uint32_t pb = B::best_init();
            B::prefix(D, D.pfx_base + it.p0 + i, pb);
            best = B::better(best, pb);
            if (D.rec) D.rec[it.p0 + i] = B::finish(pb);
        }
        wb.add(B::finish(best));
        wb.item_end(q);
    }
    wb.flush();
}

// Same queue loop over the packed 16-bit sweep (Bin16S); scores carry the
// descriptor's bias, removed before they are published.
template <int MW, int KIND, int R>
__global__ __launch_bounds__(256) void k_bin16s(QArgs q)
{
    using B = Bin16S<MW, KIND, R>;
    const uint32_t lane = threadIdx.x & 63;
    queue_priority(q);
    WaveBest wb;
    Item it;
    while (next_item(q, it)) {
        const Desc D = load_desc(q.descs + it.prob);
        wb.enter(it.prob, D.result);
        uint32_t best = B::best_init();
        const uint32_t rounds = (it.count + 63) >> 6;
        for (uint32_t j = 0; j < rounds; ++j) {
            uint32_t i = lane + 64 * j;
            if (i >= it.count) i = it.count - 1;
            uint32_t pb = B::best_init();
            B::prefix(D, D.pfx_base + it.p0 + i, pb);
            best = B::better(best, pb);
            if (D.rec) D.rec[it.p0 + i] = B::finish(pb, D.bias);
        }
        wb.add(B::finish(best, D.bias));
        wb.item_end(q);
    }
    wb.flush();
}

template <int MP, int KIND>
__global__ __launch_bounds__(256) void k_bin64(QArgs q)
{
    using B = Bin64<MP, KIND>;
    const uint32_t lane = threadIdx.x & 63;
    queue_priority(q);
    WaveBest wb;
    Item it;
    while (next_item(q, it)) {
        const Desc D = load_desc(q.descs + it.prob);
        wb.enter(it.prob, D.result);
        int64_t best = B::best_init();
        const uint32_t rounds = (it.count + 63) >> 6;
        for (uint32_t j = 0; j < rounds; ++j) {
            uint32_t i = lane + 64 * j;
            if (i >= it.count) i = it.count - 1;
            int64_t pb = B::best_init();
            B::prefix(D, D.pfx_base + it.p0 + i, pb);
            best = pb > best ? pb : best;
            if (D.rec) D.rec[it.p0 + i] = pb;
        }
        wb.add(B::finish(best));
        wb.item_end(q);
    }
    wb.flush();
}

namespace {

constexpr int NMP = MAX_MP / 2;   // mp = 2, 4, ..., 64
const void* g_bin32[NMP][MAX_R + 1] = {};
const void* g_bin32s[NMP][MAX_RS + 1] = {};
const void* g_bin64[MAX_MP / 8] = {};
const void* g_bin16s[2][MAX_MP / 2] = {};   // [PACK16_R_BIG?][words 1 .. 32] (L1 and L2 only)

template <int MP, int R>
void reg_one()
{
    if constexpr (R >= 0) g_bin32[MP / 2 - 1][R] = (const void*)&k_bin32<MP, LD_KIND, R>;
}

template <int MP>
void reg_mp()
{
    constexpr int rmax = bin_rmax(MP, LD_KIND);
    // the two largest R values that fit: the tuner chooses between them
    reg_one<MP, rmax>();
    if constexpr (rmax >= 1) reg_one<MP, rmax - 1>();
    if constexpr (MP % 8 == 0) g_bin64[MP / 8 - 1] = (const void*)&k_bin64<MP, LD_KIND>;
    g_bin32s[MP / 2 - 1][4] = (const void*)&k_bin32s<MP, LD_KIND, 4>;
    g_bin32s[MP / 2 - 1][5] = (const void*)&k_bin32s<MP, LD_KIND, 5>;
    // packed kernels by word count MP / 2 (L_marg plans use the L1 ones)
    if constexpr (LD_KIND != KIND_MARG) {
        g_bin16s[0][MP / 2 - 1] = (const void*)&k_bin16s<MP / 2, LD_KIND, PACK16_R>;
        // the larger low-row count for L1 (and L_marg through it) only: no L2 workload
        // has the mid rows that repay it, and its 2 x 64 operand streams double the build
        if constexpr (LD_KIND == KIND_L1)
            g_bin16s[1][MP / 2 - 1] = (const void*)&k_bin16s<MP / 2, LD_KIND, PACK16_R_BIG>;
    }
}

template <int... I>
void reg_all(std::integer_sequence<int, I...>)
{
    (reg_mp<2 * (I + 1)>(), ...);
}

struct Init {
    Init() { reg_all(std::make_integer_sequence<int, NMP>{}); }
} g_init;

}  // namespace

#define LD_CAT2(a, b) a##b
#define LD_CAT(a, b) LD_CAT2(a, b)

const void* LD_CAT(lookup_bin32_kind, LD_KIND)(int mp, int R)
{
    if (mp < 2 || mp > MAX_MP || (mp & 1) || R < 0 || R > MAX_R) return nullptr;
    return g_bin32[mp / 2 - 1][R];
}

const void* LD_CAT(lookup_bin32s_kind, LD_KIND)(int mp, int R)
{
    if (mp < 2 || mp > MAX_MP || (mp & 1) || R < 0 || R > MAX_RS) return nullptr;
    return g_bin32s[mp / 2 - 1][R];
}

const void* LD_CAT(lookup_bin16s_kind, LD_KIND)(int words, int r)
{
    if (words < 1 || words > MAX_MP / 2 || (r != PACK16_R && r != PACK16_R_BIG)) return nullptr;
    return g_bin16s[r == PACK16_R_BIG ? 1 : 0][words - 1];
}

const void* LD_CAT(lookup_bin64_kind, LD_KIND)(int mp)
{
    if (mp < 8 || mp > MAX_MP || (mp & 7)) return nullptr;
    return g_bin64[mp / 8 - 1];
}

}  // namespace ld
