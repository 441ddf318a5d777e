// Binary-kind sweep kernels whose Gray-code state update runs on the matrix cores
// (int8 MFMA), for one kind selected by LD_KIND at compile time.
//
// The scores of a word need one |.|-accumulate per column on the VALU whatever
// produces the column sums, so the matrix cores can take over only the state
// update.  Here a wave keeps the column sums of every low-row pattern of two
// prefixes in MFMA accumulator tiles, and each Gray step (Sec. 2.1.2: one mid row
// k flips, adding +-delta_k to every column sum) is one v_mfma_i32_32x32x16_i8
// per tile: A holds the mid rows' deltas as int8, B is the step's sign in the
// slot of row k, and the accumulator adds the product to every pattern column.
//
// Register layout of v_mfma_i32_32x32x16_i8 (wave64):
//   A: lane l holds tile row l % 32 and reduction slots 8 (l / 32) + b, b < 8
//   B: lane l holds tile column l % 32 and the same reduction slots
//   D: lane l holds tile column l % 32 and rows 8 (e / 4) + 4 (l / 32) + e % 4,
//      e < 16
// The tile rows are assigned so that element e of tile t is matrix column
// y = 16 t + e in both lane halves, and lane half h sweeps prefix h of the pair:
// each lane holds every column of one word (prefix, low pattern = l % 32), so a
// score is a chain of v_sad_u32 over the lane's own registers, with no cross-lane
// step.  A tile row i therefore stands for column 16 t + 4 (i / 8) + i % 4 of
// prefix (i / 4) % 2, and its A row is that column of the mid-row deltas.
//
// Accumulators hold true value + 2^31 (wrapping int32 arithmetic, exact while
// sum |M| < 2^31, as in the VALU kernels; the matrix cores wrap int32 sums the
// same way); |true value| is one v_sad_u32 against 2^31.  The tables are those of
// the SGPR-operand kernel with R = 5 (row stride RS), read here per lane.
#include <hip/hip_runtime.h>
#include <utility>

#include "ld_registry.h"
#include "ld_sweep.h"

#ifndef LD_KIND
#error "LD_KIND must be 0 (L1), 1 (L_marg) or 2 (L2)"
#endif

namespace ld {

typedef int32_t i32x16 __attribute__((ext_vector_type(16)));

template <int MP, int KIND>
struct BinMfma {
    static constexpr int NT = (MP + 15) / 16;   // accumulator tiles (16 columns each)
    static constexpr int RS = (MP + 15) & ~15;  // table row stride, dwords
    static constexpr int NW = 32;               // low patterns (R = 5): the tile columns
    static constexpr uint32_t BIAS = 0x80000000u;

    __device__ static constexpr uint32_t best_init() { return KIND == KIND_MARG ? BIAS : 0u; }

    __device__ static __forceinline__ uint32_t better(uint32_t a, uint32_t b)
    {
        if constexpr (KIND == KIND_MARG) return (uint32_t)max((int32_t)a, (int32_t)b);
        else return max(a, b);
    }

    __device__ static __forceinline__ uint32_t better3(uint32_t a, uint32_t b, uint32_t c)
    {
        if constexpr (KIND == KIND_MARG) return (uint32_t)max((int32_t)a, max((int32_t)b, (int32_t)c));
        else return max(a, max(b, c));
    }

    // A Gray step changes a column sum by +-delta; the int8 operands carry delta / SC
    // and the step operand +-SC.  For L1 and L_marg every delta is twice a matrix
    // entry (a sign flips from -1 to +1), for L2 it is the entry itself.  The
    // planner admits a problem only when every delta / SC fits in int8.
    static constexpr uint32_t SC = KIND == KIND_L2 ? 1u : 2u;

    // A operand of tile t: reduction slot 8 h + b (lane half h, byte b) carries
    // mid row 8 h + b, so C <= 16
    __device__ static __forceinline__ int64_t mid_operand(const Desc& D, int t, uint32_t lane)
    {
        const int32_t* mid = (const int32_t*)D.mid;
        const uint32_t i = lane & 31, h = lane >> 5;
        const int y = 16 * t + 4 * (int)(i / 8) + (int)(i % 4);
        uint64_t a = 0;
        for (int b = 0; b < 8; ++b) {
            const int k = 8 * (int)h + b;
            const bool in = k < D.C && y < MP;
            const int32_t v = mid[in ? (size_t)(2 * k) * RS + y : 0] / (int32_t)SC;
            a |= (uint64_t)(uint8_t)(int8_t)(in ? v : 0) << (8 * b);
        }
        return (int64_t)a;
    }

    // The scores read the accumulators from inline assembly, which the compiler's
    // hazard tracking does not cover: it inserts the wait states an MFMA result
    // needs before an ordinary VALU read, but not before an asm read.  Every MFMA
    // result therefore passes through this statement, whose 24 wait states cover
    // the longest XDL write-to-VALU-read requirement; the scores depend on its
    // output, so they cannot be scheduled above it.
    __device__ static __forceinline__ void settle(i32x16& x)
    {
        asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" : "+v"(x));
    }

    // B operand of a step that sets mid row k to digit g (0 -> 1 adds delta,
    // 1 -> 0 subtracts it): +-SC in slot k, i.e. byte k % 8 of the lanes of half
    // k / 8.  The byte value and the lane masks are computed on the scalar unit;
    // the VALU broadcasts the value once and masks it into each dword.
    __device__ static __forceinline__ int64_t step_operand(uint32_t k, uint32_t g)
    {
        const uint32_t val = (g ? SC : 256u - SC) << (8 * (k & 3));
        const uint64_t half = (k >> 3) ? 0xffffffff00000000ull : 0x00000000ffffffffull;
        const uint64_t mlo = (k & 4) ? 0 : half, mhi = (k & 4) ? half : 0;
        uint32_t v, lo, hi;
        asm("v_mov_b32 %0, %3\n\t"
            "v_cndmask_b32_e64 %1, 0, %0, %4\n\t"
            "v_cndmask_b32_e64 %2, 0, %0, %5\n\t"
            "s_nop 1"   // VALU write -> MFMA read of the same VGPR
            : "=&v"(v), "=&v"(lo), "=v"(hi)
            : "s"(val), "s"(mlo), "s"(mhi));
        return (int64_t)(((uint64_t)hi << 32) | lo);
    }

    // Score the word held in acc (one word per lane, three independent chains of
    // v_sad_u32 against 2^31, or c_y + 2^31, from an SGPR) and apply step tn to
    // acc.  Each tile's MFMA is issued as soon as the tile has been read, so the
    // next word's first tile is ready by the time its scoring starts.
    __device__ static __forceinline__ uint32_t score_step(i32x16 (&acc)[NT], const int64_t (&a)[NT],
                                                         const uint32_t (&tot)[MP], uint32_t tn)
    {
        const uint32_t k = brgc_changed(tn);
        const int64_t b = step_operand(k, brgc_digit(k, tn));
        uint32_t c[3] = {0, 0, 0};
        static_for<NT>([&](auto t) {
            constexpr int T = t;
            static_for<16>([&](auto e) {
                constexpr int E = e, y = 16 * T + E;
                if constexpr (y < MP) {
                    const uint32_t x = (uint32_t)acc[T][E];
                    uint32_t& s = c[y % 3];
                    if constexpr (KIND == KIND_MARG && y == 0) {
                        s += x - BIAS;   // the linear column, signed
                    } else if constexpr (KIND == KIND_L2) {
                        s = sad_u32_s(x, BIAS, s);     // |g_y|
                        s = sad_u32_s(x, tot[y], s);   // |c_y - g_y|
                    } else {
                        s = sad_u32_s(x, BIAS, s);
                    }
                }
            });
            acc[T] = __builtin_amdgcn_mfma_i32_32x32x16_i8(a[T], b, acc[T], 0, 0, 0);
            settle(acc[T]);
        });
        return c[0] + c[1] + c[2];
    }

    // Sweep the prefix pair (v0 in lane half 0, v1 in half 1): all 2^C words of
    // the mid rows, each with every low pattern.  Returns the lane's best score.
    __device__ static __forceinline__ uint32_t pair(const Desc& D, uint64_t v, const int64_t (&a)[NT],
                                                    const uint32_t (&tot)[MP], uint32_t lane)
    {
        cptr<uint32_t> base = as_const<uint32_t>(D.base);
        cptr<int32_t> hid = as_const<int32_t>(D.hid);
        const uint32_t* offs = (const uint32_t*)D.offs;
        const uint32_t w = lane & 31;
        uint32_t s[MP];
        static_for<MP>([&](auto y) { s[y] = base[y]; });
        for (int r = 0; r < D.P; ++r) {
            const uint32_t mask = 0u - (uint32_t)((v >> r) & 1u);
            static_for<MP>([&](auto y) { s[y] += mask & (uint32_t)hid[r * RS + y]; });
        }
        i32x16 acc[NT];
        static_for<NT>([&](auto t) {
            static_for<16>([&](auto e) {
                constexpr int T = t, E = e, y = 16 * T + E;
                // column y of word (prefix, low pattern w); pad rows hold 2^31 (zero)
                if constexpr (y < MP) acc[T][E] = (int32_t)(s[y] - offs[w * RS + y] + BIAS);
                else acc[T][E] = (int32_t)BIAS;
            });
        });
        // The walk, two words per round so that one max3 takes both scores (the
        // planner gives this kernel C >= 1, so the word count is even).  After the
        // last word the step applied is step 1 again: dead, but always valid.
        uint32_t best = best_init();
        const uint32_t nsteps = 1u << D.C;
        for (uint32_t t = 1; t < nsteps; t += 2) {
            const uint32_t sa = score_step(acc, a, tot, t);
            const uint32_t sb = score_step(acc, a, tot, t + 1 < nsteps ? t + 1 : 1);
            best = better3(best, sa, sb);
        }
        return best;
    }

    __device__ static __forceinline__ int64_t finish(uint32_t best)
    {
        if constexpr (KIND == KIND_MARG) return (int64_t)(int32_t)best;
        else return (int64_t)best;
    }
};

// maximum over the 32 lanes of one wave half
__device__ __forceinline__ int64_t half_max(int64_t v)
{
#pragma unroll
    for (int off = 16; off >= 1; off >>= 1) {
        const int64_t o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Persistent queue kernel: a wave takes items (problem, prefix range) and sweeps
// their prefixes two at a time (one per lane half).  With an odd count the last
// pair repeats the last prefix, which cannot change a maximum.
template <int MP, int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_mfma8(QArgs q)
{
    using B = BinMfma<MP, KIND>;
    const uint32_t lane = threadIdx.x & 63;
    queue_priority(q);
    WaveBest wb;
    Item it;
    while (next_item(q, it)) {
        const Desc D = load_desc(q.descs + it.prob);
        wb.enter(it.prob, D.result);
        int64_t a[B::NT];
        static_for<B::NT>([&](auto t) { a[t] = B::mid_operand(D, t, lane); });
        // L2: the second term of column y is |(c_y + 2^31) - acc| (c = column
        // totals), read from the difference of the two operand tables of pattern 0
        uint32_t tot[MP];
        if constexpr (KIND == KIND_L2) {
            cptr<uint32_t> o = as_const<uint32_t>(D.offs);
            static_for<MP>([&](auto y) { tot[y] = o[B::NW * B::RS + y] - o[y] + B::BIAS; });
        } else {
            static_for<MP>([&](auto y) { tot[y] = 0; });
        }
        uint32_t best = B::best_init();
        for (uint32_t j = 0; j < it.count; j += 2) {
            uint32_t i = j + (lane >> 5);
            if (i >= it.count) i = it.count - 1;
            const uint32_t pb = B::pair(D, D.pfx_base + it.p0 + i, a, tot, lane);
            best = B::better(best, pb);
            if (D.rec) {
                const int64_t r = half_max(B::finish(pb));
                D.rec[it.p0 + i] = r;
            }
        }
        wb.add(B::finish(best));
        wb.item_end(q);
    }
    wb.flush();
}

namespace {

constexpr int NMP = MAX_MP / 2;   // mp = 2, 4, ..., 64
const void* g_mfma[NMP] = {};

template <int... I>
void reg_all(std::integer_sequence<int, I...>)
{
    ((g_mfma[I] = (const void*)&k_mfma8<2 * (I + 1), LD_KIND>), ...);
}

struct Init {
    Init() { reg_all(std::make_integer_sequence<int, NMP>{}); }
} g_init;

}  // namespace

#define LD_CAT2(a, b) a##b
#define LD_CAT(a, b) LD_CAT2(a, b)

const void* LD_CAT(lookup_mfma_kind, LD_KIND)(int mp)
{
    if (mp < 2 || mp > MAX_MP || (mp & 1)) return nullptr;
    return g_mfma[mp / 2 - 1];
}

}  // namespace ld
