// Host-side table of the sweep kernel instantiations.
//
// Every instantiation is fixed at compile time by its padded column count MP and
// (binary kinds) the number of low rows R scored per state, or (d-ary) the
// alphabet size d, so that the column-sum vectors live entirely in VGPRs.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace ld {

// VGPR budget for the register-resident state of one lane: the state vector(s)
// plus the low-row operands must fit in 224 registers so that two waves fit on a
// SIMD (512 VGPRs per lane slot) with room for temporaries.
constexpr int VGPR_STATE_BUDGET = 224;
constexpr int MAX_R = 3;
constexpr int MAX_RS = 5;   // low rows of the SGPR-operand binary kernels (R = 4, 5 built)

constexpr int bin_k(int kind) { return kind == 2 ? 2 : 1; }

// largest R <= MAX_R with (1 + K * 2^R) * mp <= budget, or -1 if even R = 0 fails
constexpr int bin_rmax(int mp, int kind)
{
    for (int r = MAX_R; r >= 0; --r)
        if ((1 + bin_k(kind) * (1 << r)) * mp <= VGPR_STATE_BUDGET) return r;
    return -1;
}

// d-ary: d vectors of mp columns
constexpr bool dary_fits(int mp, int d) { return d * mp <= 192; }

// SGPR-operand d-ary kernels: R = 3 low rows, built for d = 3, 4 while the d
// message vectors take at most 160 VGPRs
constexpr int DARY_RS = 3;
constexpr bool dary_s_fits(int mp, int d) { return (d == 3 || d == 4) && d * mp <= 160; }

// packed 16-bit d-ary kernels (two columns per dword, VARIANT_PACK16), d = 3, 4,
// while the d message vectors take at most 96 VGPRs; by dword count (mp / 2).
// Low rows per state: 5 for d = 3 (243 words), 4 for d = 4 (256 words).  A mid
// step re-scores the 2^R subsets of the two messages it changes, so one more low
// row halves that work per word (d = 3: 6.9 instructions per word against 9.9
// with R = 4; d = 4: 5.2 against 8.1 with R = 3), at the price of the registers
// for twice the subset scores: three waves per SIMD instead of four up to 28
// (d = 3) or 24 (d = 4) columns, two beyond.  Measured 18-28 % faster at every
// size that fills the device.  A smaller problem has a third as many states, and
// so lanes, at the larger R: below half a wave per SIMD its plan takes the kernel
// with one low row fewer (dary16_r_small).
constexpr int dary16_r(int d) { return d == 3 ? 5 : 4; }
constexpr int dary16_r_small(int d) { return dary16_r(d) - 1; }
constexpr bool dary16_fits(int words, int d) { return (d == 3 || d == 4) && d * words <= 96; }

// d-ary low rows scored per state: the largest R <= 2 whose 2^R - 1 subset
// operands fit beside the d state vectors, (d + 2^R - 1) * mp <= 200
constexpr int dary_r(int mp, int d)
{
    for (int r = 2; r >= 1; --r)
        if ((d + (1 << r) - 1) * mp <= 200) return r;
    return 0;
}

// lookups; return nullptr when no instantiation exists
const void* kernel_bin32(int kind, int mp, int R);
const void* kernel_bin32s(int kind, int mp, int R);
// packed 16-bit kernel (two columns per dword; L1 and, through it, L_marg, and L2),
// by dword count; PACK16_R low rows, or (L1 and L_marg) PACK16_R_BIG for a plain
// call of a large problem (one row update per 64 words instead of 32; with its operands it holds
// four waves per SIMD instead of five, which only problems with many mid rows per
// lane repay: 42 x 42 L1 1.267 -> 1.244 s, but 36 x 36 L1 17.8 -> 18.1 ms and the
// batch and served workloads slower)
constexpr int PACK16_R = 5;
constexpr int PACK16_R_BIG = 6;
constexpr int VARIANT_PACK16 = 16;   // binary variant value selecting kernel_bin16s
constexpr int64_t PACK16_BOUND = 32767;   // largest sum_x |M_xy| of a column it takes
const void* kernel_bin16s(int kind, int words, int r);
// int8-MFMA state-update kernel (binary kinds, int32, R = 5, C <= 16)
const void* kernel_mfma(int kind, int mp);
constexpr int MFMA_MAX_C = 16;
constexpr int VARIANT_MFMA = 8;   // binary variant value selecting kernel_mfma
const void* kernel_bin64(int kind, int mp);
const void* kernel_dary32(int d, int mp);
const void* kernel_dary32s(int d, int mp);   // SGPR-operand d-ary kernel (DARY_RS low rows)
// packed 16-bit d-ary kernel with r = dary16_r(d) or dary16_r_small(d) low rows
const void* kernel_dary16s(int d, int words, int r);
const void* kernel_dary64(int d, int mp);
const void* kernel_sumabs_many();
const void* kernel_wide();
const void* kernel_reset();
const void* kernel_stage();     // k_stage(StageArgs): server step staging
const void* kernel_publish();   // k_publish(results, out, n): server step results to host memory
const void* kernel_first_equal();
const void* kernel_set_u64();
const void* kernel_signs();
const void* kernel_valu_probe();   // clock and VALU-rate probe (ld_valu_probe)
constexpr size_t WIDE_LDS_MAX = 64 * 1024;   // bytes of state per wave

// padded column count used for a problem with m columns
inline int pad_bin32(int m) { return (m + 1) & ~1; }
inline int pad_bin64(int m) { return (m + 7) & ~7; }
inline int pad_dary(int m) { return (m + 3) & ~3; }

}  // namespace ld
