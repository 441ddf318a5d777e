// Gray-code arithmetic shared by the sweep kernels and the host planner.
//
// Binary reflected Gray code (BRGC), arXiv:2503.21596 Sec. 2.1.2:
//   digit i of word j        G_{i,j} = floor((j + 2^i) / 2^(i+1)) mod 2   (Eq. Hamming_equation)
//   digit changed at word j  the i with j / 2^i odd, i.e. the number of
//                            trailing zero bits of j                         (Eq. Hamming_equation_change)
// d-ary reflected Gray code, Sec. 2.3.2:
//   S = (0, 1, ..., d-1, d-1, ..., 1, 0)                                    (Eq. N_ary_G2)
//   I_{i,j} = floor(j / d^i) mod 2d,  G_{i,j} = S[I_{i,j}]                  (Eqs. N_ary_G1, N_ary_G3)
//   digit changed at word j  min{ i : floor(j / d^i) mod d != 0 }          (Eq. d_aryGrayChange_1)
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define LD_HD __host__ __device__ __forceinline__
#else
#define LD_HD inline
#endif

namespace ld {

LD_HD uint32_t brgc_digit(uint32_t i, uint64_t j)
{
    return (uint32_t)(((j + (1ull << i)) >> (i + 1)) & 1ull);
}

LD_HD uint32_t brgc_changed(uint64_t j)
{
    return (uint32_t)__builtin_ctzll(j);
}

// S[x] of Eq. N_ary_G2 for x in [0, 2d)
LD_HD uint32_t dgc_reflect(uint32_t x, uint32_t d)
{
    return x < d ? x : 2u * d - 1u - x;
}

LD_HD uint32_t dgc_digit(uint32_t d, uint32_t i, uint64_t j)
{
    uint64_t q = j;
    for (uint32_t k = 0; k < i; ++k) q /= d;
    return dgc_reflect((uint32_t)(q % (2u * d)), d);
}

// For word j >= 1 of the d-ary reflected Gray code: the changed digit and its
// old and new values.  Because d^i divides j, floor((j-1)/d^i) = floor(j/d^i) - 1,
// so the old value is S[(q - 1) mod 2d] with q = j / d^i.
template <uint32_t D>
LD_HD uint32_t dgc_change(uint32_t j, uint32_t* from, uint32_t* to)
{
    uint32_t i = 0, q = j;
    while (q % D == 0u) { q /= D; ++i; }
    *to = dgc_reflect(q % (2u * D), D);
    *from = dgc_reflect((q - 1u) % (2u * D), D);
    return i;
}

LD_HD uint32_t dgc_change_rt(uint32_t d, uint64_t j, uint32_t* from, uint32_t* to)
{
    uint32_t i = 0;
    uint64_t q = j;
    while (q % d == 0u) { q /= d; ++i; }
    *to = dgc_reflect((uint32_t)(q % (2u * d)), d);
    *from = dgc_reflect((uint32_t)((q - 1u) % (2u * d)), d);
    return i;
}

}  // namespace ld
