// Register-resident Gray-code sweeps for gfx950 (CDNA4, wave64).
//
// One lane owns one sub-cube of the assignment space: a fixed prefix on the high
// rows, a Gray-code walk over the mid rows (arXiv:2503.21596 Sec. 2.1.2 for the
// binary code, Sec. 2.3.2 for the d-ary one) and, for the binary kinds, every
// pattern of the R low rows scored against the same state.  Because every lane of
// the grid walks the same mid-row code from the same start, the changed row and
// its direction are wave-uniform at each step (the group property the paper proves
// in its Appendix on group-uniform changes), so the row index lives in SGPRs and the
// row itself is read with scalar loads.
//
// Column sums of the int32 path are kept offset-binary (true value + 2^31, as
// uint32).  With B = sum |M_xy| < 2^31 every partial sum lies in (-2^31, 2^31), so
// the wrapped additions are exact and a term |s + o| of a score is one
// v_sad_u32 (|a - b| + c on unsigned operands) against a precomputed operand.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "ld_gray.h"
#include "ld_types.h"

namespace ld {

// Pointer into the constant address space: uniform loads through it become
// scalar (SMEM) loads.  The tables are read-only for the lifetime of a launch.
template <class T>
using cptr = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ cptr<T> as_const(const void* p)
{
    return (cptr<T>)(uintptr_t)p;
}

__device__ __forceinline__ uint32_t sad_u32(uint32_t a, uint32_t b, uint32_t acc)
{
    uint32_t r;
    asm("v_sad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(acc));
    return r;
}

// A value the compiler must keep in a VGPR: the low-row operands are the same
// in every lane, but read from SGPRs they would not fit (and would spill through
// v_writelane / v_readlane), so they are copied once into VGPRs.
__device__ __forceinline__ uint32_t in_vgpr(uint32_t x)
{
    uint32_t r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// v_sad_u32 with the operand b taken from an SGPR
__device__ __forceinline__ uint32_t sad_u32_s(uint32_t a, uint32_t b, uint32_t acc)
{
    uint32_t r;
    asm("v_sad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(acc));
    return r;
}

// v_sad_u16 with the operand b taken from an SGPR.  On gfx950 it adds the absolute
// differences of both 16-bit halves, taken as unsigned values, to a 32-bit
// accumulator: |a[15:0] - b[15:0]| + |a[31:16] - b[31:16]| + acc.
__device__ __forceinline__ uint32_t sad_u16_s(uint32_t a, uint32_t b, uint32_t acc)
{
    uint32_t r;
    asm("v_sad_u16 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(acc));
    return r;
}

// Compile-time loop: f(integral_constant<int, i>) for i = 0 .. N-1, so that
// offsets derived from i can be immediates of a load.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}

template <int N, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));

constexpr int ipow_c(int b, int e) { return e == 0 ? 1 : b * ipow_c(b, e - 1); }

// Four 8-dword scalar loads at base + O0 .. O3 (wave-uniform base in SGPRs),
// complete on return.  Scalar loads may return out of order, so one wait for all
// of them closes the statement; keeping the wait inside the statement means no
// instruction can touch the destination SGPRs while a load is still in flight.
// The destinations are early-clobber ("=&s"): a later load of the statement still
// reads `base`, so no destination may share its registers (a first load landing
// on the base pair would redirect the ones after it).
template <int O0, int O1, int O2, int O3>
__device__ __forceinline__ void sload_4x8(uint64_t base, u32x8& x0, u32x8& x1, u32x8& x2, u32x8& x3)
{
    asm volatile("s_load_dwordx8 %0, %4, %5\n\t"
                 "s_load_dwordx8 %1, %4, %6\n\t"
                 "s_load_dwordx8 %2, %4, %7\n\t"
                 "s_load_dwordx8 %3, %4, %8\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&s"(x0), "=&s"(x1), "=&s"(x2), "=&s"(x3)
                 : "s"(base), "n"(O0), "n"(O1), "n"(O2), "n"(O3));
}

template <int O0, int O1>
__device__ __forceinline__ void sload_2x8(uint64_t base, u32x8& x0, u32x8& x1)
{
    asm volatile("s_load_dwordx8 %0, %2, %3\n\t"
                 "s_load_dwordx8 %1, %2, %4\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&s"(x0), "=&s"(x1)
                 : "s"(base), "n"(O0), "n"(O1));
}

template <int O0>
__device__ __forceinline__ void sload_1x8(uint64_t base, u32x8& x0)
{
    asm volatile("s_load_dwordx8 %0, %1, %2\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&s"(x0)
                 : "s"(base), "n"(O0));
}

// ---------------------------------------------------------------------------
// binary kinds, int32 (offset-binary) path

template <int MP, int KIND, int R>
struct Bin32 {
    static constexpr int NW = 1 << R;
    static constexpr int K = (KIND == KIND_L2) ? 2 : 1;
    // one stored row of deltas, padded to a multiple of 16 dwords so the whole
    // row is fetched with s_load_dwordx16
    static constexpr int RS = (MP + 15) & ~15;

    // best starts at the smallest score of its kind (0, or INT32_MIN for L_marg)
    __device__ static constexpr uint32_t best_init() { return KIND == KIND_MARG ? 0x80000000u : 0u; }

    __device__ static __forceinline__ uint32_t better(uint32_t a, uint32_t b)
    {
        if constexpr (KIND == KIND_MARG) return (uint32_t)max((int32_t)a, (int32_t)b);
        else return max(a, b);
    }

    __device__ static __forceinline__ void load_offs(const Desc& D, uint32_t (&off)[K][NW][MP])
    {
        cptr<uint32_t> o = as_const<uint32_t>(D.offs);
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int w = 0; w < NW; ++w)
#pragma unroll
                for (int y = 0; y < MP; ++y) off[k][w][y] = in_vgpr(o[(k * NW + w) * RS + y]);
    }

    __device__ static __forceinline__ void score(const uint32_t (&s)[MP], const uint32_t (&off)[K][NW][MP],
                                                 uint32_t& best)
    {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            if constexpr (KIND == KIND_L1) {
                uint32_t acc = 0;
#pragma unroll
                for (int y = 0; y < MP; ++y) acc = sad_u32(s[y], off[0][w][y], acc);
                best = max(best, acc);
            } else if constexpr (KIND == KIND_MARG) {
                uint32_t acc = s[0] - off[0][w][0];   // the linear column, signed
#pragma unroll
                for (int y = 1; y < MP; ++y) acc = sad_u32(s[y], off[0][w][y], acc);
                best = (uint32_t)max((int32_t)best, (int32_t)acc);
            } else {
                uint32_t acc = 0;
#pragma unroll
                for (int y = 0; y < MP; ++y) {
                    acc = sad_u32(s[y], off[0][w][y], acc);
                    acc = sad_u32(s[y], off[1][w][y], acc);
                }
                best = max(best, acc);
            }
        }
    }

    // Sweep one prefix value v: start state, then the Gray walk over 2^C words of
    // the mid rows, scoring NW low patterns at each word.
    __device__ static __forceinline__ void prefix(const Desc& D, uint64_t v, const uint32_t (&off)[K][NW][MP],
                                                  uint32_t& best)
    {
        cptr<uint32_t> base = as_const<uint32_t>(D.base);
        cptr<int32_t> hid = as_const<int32_t>(D.hid);
        uint32_t s[MP];
#pragma unroll
        for (int y = 0; y < MP; ++y) s[y] = base[y];
        for (int h = 0; h < D.P; ++h) {
            const uint32_t mask = 0u - (uint32_t)((v >> h) & 1u);
#pragma unroll
            for (int y = 0; y < MP; ++y) s[y] += mask & (uint32_t)hid[h * RS + y];
        }
        // The row for the next word is fetched (scalar loads) in the same block
        // as the scoring of the current word, so its latency hides behind the
        // v_sad chain.  After the last word the update is dead but harmless.
        const uint32_t nsteps = 1u << D.C;
        for (uint32_t t = 0; t < nsteps; ++t) {
            const uint32_t tn = (t + 1 < nsteps) ? t + 1 : 1;   // always a valid step
            const uint32_t k = brgc_changed(tn);
            const uint32_t g = brgc_digit(k, tn);                // new value of digit k
            const uint64_t addr = __builtin_amdgcn_readfirstlane(
                                      (uint32_t)((2 * k + (1 - g)) * (RS * 4)))
                                  + (uint64_t)(uintptr_t)D.mid;
            cptr<int32_t> row = (cptr<int32_t>)__builtin_assume_aligned((const int32_t*)addr, 64);
            int32_t nx[RS];
#pragma unroll
            for (int y = 0; y < RS; ++y) nx[y] = row[y];
            score(s, off, best);
#pragma unroll
            for (int y = 0; y < MP; ++y) s[y] += (uint32_t)nx[y];
        }
    }

    __device__ static __forceinline__ int64_t finish(uint32_t best)
    {
        if constexpr (KIND == KIND_MARG) return (int64_t)(int32_t)best;
        else return (int64_t)best;
    }
};

// ---------------------------------------------------------------------------
// binary kinds, int32 path, low-row operands streamed through SGPRs
//
// The low-row operands are the same in every lane, so instead of holding copies
// in VGPRs (which caps R at 2 for m = 42) they are read with scalar loads straight
// into SGPRs and consumed as the scalar operand of v_sad_u32.  Only the state vector
// lives in VGPRs, so R is free: a state is scored for 2^R words and its row update
// costs 1/2^R of the scoring.  The small register footprint also allows seven
// waves per SIMD, which hides the scalar-load latency.
//
// Operand streams are consumed four at a time (four independent accumulators) so
// that dependent v_sad_u32 instructions are four apart.  Stream order: for L1 and
// L_marg stream w is pattern w; for L2 the streams of patterns w and w + 1 are
// (w, +M part), (w, total - M part), (w + 1, ...), (w + 1, ...).
template <int MP, int KIND, int R>
struct Bin32S {
    static constexpr int NW = 1 << R;
    static constexpr int K = (KIND == KIND_L2) ? 2 : 1;
    static constexpr int RS = (MP + 15) & ~15;   // row stride of every table, dwords
    static constexpr int N8 = (MP + 7) / 8;      // 8-column chunks of a row
    static_assert(R >= 2, "four operand streams per group");

    __device__ static constexpr uint32_t best_init() { return KIND == KIND_MARG ? 0x80000000u : 0u; }

    __device__ static __forceinline__ uint32_t better(uint32_t a, uint32_t b)
    {
        if constexpr (KIND == KIND_MARG) return (uint32_t)max((int32_t)a, (int32_t)b);
        else return max(a, b);
    }

    template <int S0, int S1, int S2, int S3, int C8>
    __device__ static __forceinline__ void chunk4(const uint32_t (&s)[MP], uint64_t ob, uint32_t (&a)[4])
    {
        u32x8 o0, o1, o2, o3;
        sload_4x8<(S0 * RS + 8 * C8) * 4, (S1 * RS + 8 * C8) * 4, (S2 * RS + 8 * C8) * 4,
                  (S3 * RS + 8 * C8) * 4>(ob, o0, o1, o2, o3);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            constexpr int y0 = 8 * C8;
            if (y0 + j >= MP) continue;
            if (KIND == KIND_MARG && y0 + j == 0) {
                // the linear column: s_0 - o_0 is the signed value itself
                a[0] = s[0] - o0[0];
                a[1] = s[0] - o1[0];
                a[2] = s[0] - o2[0];
                a[3] = s[0] - o3[0];
                continue;
            }
            const uint32_t x = s[y0 + j];
            a[0] = sad_u32_s(x, o0[j], a[0]);
            a[1] = sad_u32_s(x, o1[j], a[1]);
            a[2] = sad_u32_s(x, o2[j], a[2]);
            a[3] = sad_u32_s(x, o3[j], a[3]);
        }
    }

    __device__ static __forceinline__ void score(const uint32_t (&s)[MP], uint64_t ob, uint32_t& best)
    {
        if constexpr (KIND == KIND_L2) {
            static_for<NW / 2>([&](auto h) {
                constexpr int w = 2 * h;
                uint32_t a[4] = {0, 0, 0, 0};
                static_for<N8>([&](auto c) { chunk4<w, NW + w, w + 1, NW + w + 1, c>(s, ob, a); });
                best = max(best, max(a[0] + a[1], a[2] + a[3]));
            });
        } else {
            static_for<NW / 4>([&](auto g) {
                constexpr int w = 4 * g;
                uint32_t a[4] = {0, 0, 0, 0};
                static_for<N8>([&](auto c) { chunk4<w, w + 1, w + 2, w + 3, c>(s, ob, a); });
                if constexpr (KIND == KIND_MARG)
                    best = (uint32_t)max(max((int32_t)best, max((int32_t)a[0], (int32_t)a[1])),
                                         max((int32_t)a[2], (int32_t)a[3]));
                else
                    best = max(max(best, max(a[0], a[1])), max(a[2], a[3]));
            });
        }
    }

    // s += the row at `row` (RS dwords, wave-uniform address)
    __device__ static __forceinline__ void add_row(uint32_t (&s)[MP], uint64_t row)
    {
        static_for<(N8 + 3) / 4>([&](auto q) {
            constexpr int c0 = 4 * q;
            constexpr int n = (N8 - c0) < 4 ? (N8 - c0) : 4;
            u32x8 r[4];
            if constexpr (n == 4)
                sload_4x8<32 * c0, 32 * (c0 + 1), 32 * (c0 + 2), 32 * (c0 + 3)>(row, r[0], r[1], r[2], r[3]);
            else if constexpr (n == 3) {
                sload_2x8<32 * c0, 32 * (c0 + 1)>(row, r[0], r[1]);
                sload_1x8<32 * (c0 + 2)>(row, r[2]);
            } else if constexpr (n == 2)
                sload_2x8<32 * c0, 32 * (c0 + 1)>(row, r[0], r[1]);
            else
                sload_1x8<32 * c0>(row, r[0]);
#pragma unroll
            for (int i = 0; i < n; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if (8 * (c0 + i) + j < MP) s[8 * (c0 + i) + j] += r[i][j];
        });
    }

    // Sweep one prefix value v: start state, then the Gray walk over 2^C words of
    // the mid rows, scoring the 2^R low patterns at each word.
    __device__ static __forceinline__ void prefix(const Desc& D, uint64_t v, uint32_t& best)
    {
        cptr<uint32_t> base = as_const<uint32_t>(D.base);
        cptr<int32_t> hid = as_const<int32_t>(D.hid);
        uint32_t s[MP];
#pragma unroll
        for (int y = 0; y < MP; ++y) s[y] = base[y];
        for (int h = 0; h < D.P; ++h) {
            const uint32_t mask = 0u - (uint32_t)((v >> h) & 1u);
#pragma unroll
            for (int y = 0; y < MP; ++y) s[y] += mask & (uint32_t)hid[h * RS + y];
        }
        const uint64_t ob = (uint64_t)(uintptr_t)D.offs;
        const uint64_t mb = (uint64_t)(uintptr_t)D.mid;
        const uint32_t nsteps = 1u << D.C;
        for (uint32_t t = 0;;) {
            score(s, ob, best);
            if (++t == nsteps) break;
            const uint32_t k = brgc_changed(t);
            const uint32_t g = brgc_digit(k, t);   // new value of digit k
            add_row(s, mb + __builtin_amdgcn_readfirstlane((uint32_t)((2 * k + (1 - g)) * (RS * 4))));
        }
    }

    __device__ static __forceinline__ int64_t finish(uint32_t best)
    {
        if constexpr (KIND == KIND_MARG) return (int64_t)(int32_t)best;
        else return (int64_t)best;
    }
};

// ---------------------------------------------------------------------------
// binary kinds, int32 path, two columns per register (packed 16-bit), low-row
// operands streamed through SGPRs
//
// When every column has sum_x |M_xy| <= 2^15 - 1, every column sum and every
// low-row operand fits 16 bits offset by 2^15, so one dword holds two columns
// (column 2j in the low half).  One v_sad_u16 then scores two columns of a word,
// which halves the scoring instructions of Bin32S.  A row update stays one 32-bit
// add per dword: the stored delta is d_2j + 2^16 d_2j+1 modulo 2^32, and since both
// new halves lie in [0, 2^16) no carry crosses between them.
// L_marg runs through the L1 instantiation: its linear column 0 is stored with an
// offset h >= half its bound, so the term |x + 2h| equals x + 2h for every
// reachable x; the descriptor's bias (2h) is subtracted from the maximum.
template <int MW, int KIND, int R>
struct Bin16S {
    static constexpr int NW = 1 << R;
    static constexpr int K = (KIND == KIND_L2) ? 2 : 1;
    static constexpr int RS = (MW + 15) & ~15;   // row stride of every table, dwords
    static constexpr int N8 = (MW + 7) / 8;      // 8-dword chunks of a row
    static_assert(R >= 2, "four operand streams per group");
    static_assert(KIND == KIND_L1 || KIND == KIND_L2, "L_marg runs as L1 with a bias");

    __device__ static constexpr uint32_t best_init() { return 0u; }
    __device__ static __forceinline__ uint32_t better(uint32_t a, uint32_t b) { return max(a, b); }

    template <int S0, int S1, int S2, int S3, int C8>
    __device__ static __forceinline__ void chunk4(const uint32_t (&s)[MW], uint64_t ob, uint32_t (&a)[4])
    {
        u32x8 o0, o1, o2, o3;
        sload_4x8<(S0 * RS + 8 * C8) * 4, (S1 * RS + 8 * C8) * 4, (S2 * RS + 8 * C8) * 4,
                  (S3 * RS + 8 * C8) * 4>(ob, o0, o1, o2, o3);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            constexpr int y0 = 8 * C8;
            if (y0 + j >= MW) continue;
            const uint32_t x = s[y0 + j];
            a[0] = sad_u16_s(x, o0[j], a[0]);
            a[1] = sad_u16_s(x, o1[j], a[1]);
            a[2] = sad_u16_s(x, o2[j], a[2]);
            a[3] = sad_u16_s(x, o3[j], a[3]);
        }
    }

    __device__ static __forceinline__ void score(const uint32_t (&s)[MW], uint64_t ob, uint32_t& best)
    {
        if constexpr (KIND == KIND_L2) {
            // each accumulator runs through both message sides of its pattern, so the
            // two halves of the score need no add
            static_for<NW / 4>([&](auto g) {
                constexpr int w = 4 * g;
                uint32_t a[4] = {0, 0, 0, 0};
                static_for<N8>([&](auto c) { chunk4<w, w + 1, w + 2, w + 3, c>(s, ob, a); });
                static_for<N8>([&](auto c) { chunk4<NW + w, NW + w + 1, NW + w + 2, NW + w + 3, c>(s, ob, a); });
                best = max(max(best, a[0]), a[1]);   // two v_max3 per four patterns
                best = max(max(best, a[2]), a[3]);
            });
        } else {
            static_for<NW / 4>([&](auto g) {
                constexpr int w = 4 * g;
                uint32_t a[4] = {0, 0, 0, 0};
                static_for<N8>([&](auto c) { chunk4<w, w + 1, w + 2, w + 3, c>(s, ob, a); });
                best = max(max(best, a[0]), a[1]);   // two v_max3 per four patterns
                best = max(max(best, a[2]), a[3]);
            });
        }
    }

    // s += the row at `row` (RS dwords, wave-uniform address)
    __device__ static __forceinline__ void add_row(uint32_t (&s)[MW], uint64_t row)
    {
        static_for<(N8 + 3) / 4>([&](auto q) {
            constexpr int c0 = 4 * q;
            constexpr int n = (N8 - c0) < 4 ? (N8 - c0) : 4;
            u32x8 r[4];
            if constexpr (n == 4)
                sload_4x8<32 * c0, 32 * (c0 + 1), 32 * (c0 + 2), 32 * (c0 + 3)>(row, r[0], r[1], r[2], r[3]);
            else if constexpr (n == 3) {
                sload_2x8<32 * c0, 32 * (c0 + 1)>(row, r[0], r[1]);
                sload_1x8<32 * (c0 + 2)>(row, r[2]);
            } else if constexpr (n == 2)
                sload_2x8<32 * c0, 32 * (c0 + 1)>(row, r[0], r[1]);
            else
                sload_1x8<32 * c0>(row, r[0]);
#pragma unroll
            for (int i = 0; i < n; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if (8 * (c0 + i) + j < MW) s[8 * (c0 + i) + j] += r[i][j];
        });
    }

    // Sweep one prefix value v: start state, then the Gray walk over 2^C words of
    // the mid rows, scoring the 2^R low patterns at each word.
    __device__ static __forceinline__ void prefix(const Desc& D, uint64_t v, uint32_t& best)
    {
        cptr<uint32_t> base = as_const<uint32_t>(D.base);
        cptr<uint32_t> hid = as_const<uint32_t>(D.hid);
        uint32_t s[MW];
#pragma unroll
        for (int y = 0; y < MW; ++y) s[y] = base[y];
        for (int h = 0; h < D.P; ++h) {
            const uint32_t mask = 0u - (uint32_t)((v >> h) & 1u);
#pragma unroll
            for (int y = 0; y < MW; ++y) s[y] += mask & hid[h * RS + y];
        }
        const uint64_t ob = (uint64_t)(uintptr_t)D.offs;
        const uint64_t mb = (uint64_t)(uintptr_t)D.mid;
        const uint32_t nsteps = 1u << D.C;
        for (uint32_t t = 0;;) {
            score(s, ob, best);
            if (++t == nsteps) break;
            const uint32_t k = brgc_changed(t);
            const uint32_t g = brgc_digit(k, t);   // new value of digit k
            add_row(s, mb + __builtin_amdgcn_readfirstlane((uint32_t)((2 * k + (1 - g)) * (RS * 4))));
        }
    }

    __device__ static __forceinline__ int64_t finish(uint32_t best, int32_t bias) { return (int64_t)best - bias; }
};

// ---------------------------------------------------------------------------
// binary kinds, int64 path (sum |M_xy| >= 2^31); no low-row patterns

template <int MP, int KIND>
struct Bin64 {
    __device__ static constexpr int64_t best_init() { return INT64_MIN; }

    __device__ static __forceinline__ int64_t score(const int64_t (&s)[MP], cptr<int64_t> cc)
    {
        int64_t acc;
        if constexpr (KIND == KIND_L1) {
            acc = 0;
#pragma unroll
            for (int y = 0; y < MP; ++y) acc += s[y] < 0 ? -s[y] : s[y];
        } else if constexpr (KIND == KIND_MARG) {
            acc = s[0];
#pragma unroll
            for (int y = 1; y < MP; ++y) acc += s[y] < 0 ? -s[y] : s[y];
        } else {
            acc = 0;
#pragma unroll
            for (int y = 0; y < MP; ++y) {
                const int64_t u = s[y], w = cc[y] - s[y];
                acc += (u < 0 ? -u : u) + (w < 0 ? -w : w);
            }
        }
        return acc;
    }

    __device__ static __forceinline__ void prefix(const Desc& D, uint64_t v, int64_t& best)
    {
        cptr<int64_t> base = as_const<int64_t>(D.base);
        cptr<int64_t> hid = as_const<int64_t>(D.hid);
        cptr<int64_t> mid = as_const<int64_t>(D.mid);
        cptr<int64_t> cc = as_const<int64_t>(D.offs);   // column totals (L2)
        int64_t s[MP];
#pragma unroll
        for (int y = 0; y < MP; ++y) s[y] = base[y];
        for (int h = 0; h < D.P; ++h) {
            const int64_t mask = -(int64_t)((v >> h) & 1u);
#pragma unroll
            for (int y = 0; y < MP; ++y) s[y] += mask & hid[h * MP + y];
        }
        const uint64_t nsteps = 1ull << D.C;
        for (uint64_t t = 0;;) {
            const int64_t sc = score(s, cc);
            best = sc > best ? sc : best;
            if (++t == nsteps) break;
            const uint32_t k = brgc_changed(t);
            const uint32_t g = brgc_digit(k, t);
            cptr<int64_t> row = mid + (2 * k + (1 - g)) * MP;
#pragma unroll
            for (int y = 0; y < MP; ++y) s[y] += row[y];
        }
    }

    __device__ static __forceinline__ int64_t finish(int64_t best) { return best; }
};

// ---------------------------------------------------------------------------
// work queue

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }


// The descriptor is the same for the whole wave: read it with scalar loads so its
// fields, and every loop bound derived from them, live in SGPRs.
__device__ __forceinline__ Desc load_desc(const Desc* p)
{
    static_assert(sizeof(Desc) % 4 == 0, "descriptor must be a whole number of dwords");
    cptr<uint32_t> src = as_const<uint32_t>(p);
    uint32_t w[sizeof(Desc) / 4];
#pragma unroll
    for (int i = 0; i < (int)(sizeof(Desc) / 4); ++i) w[i] = src[i];
    Desc D;
    __builtin_memcpy(&D, w, sizeof(Desc));
    return D;
}

// Next item for this wave; false once the queue is exhausted, which every wave
// reaches, so the grid always drains.  Items are popped through the shared head
// (dynamic balancing: XCDs run at slightly different clocks, and a static split
// measured 6 % slower on a 3 s sweep); the planner sizes items so that pops stay
// rare next to the work, since atomics on one address serialize across XCDs.
// Implicit items (q.items == nullptr: one problem, equal items) are computed from
// their index.  A pop is executed by every lane (lane 0 adds 1, the others 0) so
// that no lane-0-only branch precedes the readfirstlane that broadcasts lane 0's
// old value: after such a branch the compiler may re-enter the loop with lane 0
// inactive, and readfirstlane would then read another lane's stale value.
__device__ __forceinline__ bool next_item(const QArgs& q, Item& it)
{
    const uint32_t add = (threadIdx.x & 63) == 0 ? 1u : 0u;
    const uint32_t i = uni(atomicAdd(q.head, add));
    if (i >= q.n_items) return false;
    if (q.items == nullptr) {
        it.prob = q.prob;
        it.p0 = (uint64_t)i * q.per;
        const uint64_t left = q.n_prefix - it.p0;
        it.count = (uint32_t)(left < q.per ? left : q.per);
        return true;
    }
    cptr<uint32_t> w = as_const<uint32_t>(q.items) + 4 * (size_t)i;
    it.prob = w[0];
    it.count = w[1];
    it.p0 = (uint64_t)w[2] | ((uint64_t)w[3] << 32);
    return true;
}

// ---------------------------------------------------------------------------
// wave-level max and the per-problem result

__device__ __forceinline__ int64_t wave_max(int64_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int64_t o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// The wave max is the same in every lane, so every lane issues the atomic max
// (no lane-0-only branch; see next_item).  Kernels call this once per run of
// consecutive items of one problem, not per item: atomics on one address from
// every XCD serialize, and one per item dominated small items.
__device__ __forceinline__ void publish(int64_t* result, int64_t v)
{
    v = wave_max(v);
    // through a global (not generic) pointer, so that the compiler issues the
    // wave-uniform max from a single lane rather than one atomic per lane
    typedef __attribute__((address_space(1))) int64_t gint64;
    __hip_atomic_fetch_max((gint64*)(uintptr_t)result, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Serving: count one finished item of problem `prob` (its maximum already
// published); the wave that finishes the last item reads the problem's value and
// reports it to the host through q.done.  The decrement is issued from one lane
// (lane 0 adds -1, the others 0) and its old value broadcast, as for queue pops.
__device__ __forceinline__ void item_done(const QArgs& q, uint32_t prob, int64_t* result)
{
    typedef __attribute__((address_space(1))) uint32_t gu32;
    typedef __attribute__((address_space(1))) int64_t gi64;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t add = (threadIdx.x & 63) == 0 ? 0xffffffffu : 0u;
    const uint32_t old =
        uni(__hip_atomic_fetch_add((gu32*)(uintptr_t)(q.left + prob), add, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT));
    if (old == 1) {
        const int64_t v = __hip_atomic_load((gi64*)(uintptr_t)result, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        DoneRec* d = q.done + prob;
        __hip_atomic_store(&d->value, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&d->flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Serving's express launches (q.done set) raise their waves' issue priority: they
// share each SIMD with the waves of a long bulk launch, and at equal priority a
// small request would be issued only its share of one wave among many.
__device__ __forceinline__ void queue_priority(const QArgs& q)
{
    if (q.done != nullptr) __builtin_amdgcn_s_setprio(3);
}

// Per-wave running maximum over consecutive items of one problem.
struct WaveBest {
    int64_t best = INT64_MIN;
    int64_t* result = nullptr;
    uint32_t prob = 0xffffffffu;
    // true when `prob` starts a new run (the previous run has been published)
    __device__ __forceinline__ bool enter(uint32_t prob_, int64_t* result_)
    {
        if (prob_ == prob) return false;
        flush();
        prob = prob_;
        result = result_;
        best = INT64_MIN;
        return true;
    }
    __device__ __forceinline__ void add(int64_t v) { best = v > best ? v : best; }
    __device__ __forceinline__ void flush()
    {
        if (prob != 0xffffffffu) publish(result, best);
    }
    // after an item: with completion tracking (serving), publish now and count the
    // item; otherwise keep accumulating until the problem changes
    __device__ __forceinline__ void item_end(const QArgs& q)
    {
        if (q.left == nullptr) return;
        const uint32_t p = prob;
        flush();
        prob = 0xffffffffu;
        item_done(q, p, result);
    }
};

}  // namespace ld
