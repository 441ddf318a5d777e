// Problem descriptor shared by the host planner and the sweep kernels.
#pragma once
#include <stdint.h>

namespace ld {

// Which score a sweep evaluates (arXiv:2503.21596):
//   KIND_L1   Eq. (LM2)      sum_y |(aM)_y|, a in {+-1}^n
//   KIND_MARG Eq. (LMarg)    (aM)_0 + sum_{y>=1} |(aM)_y|, a_0 = +1
//   KIND_L2   Eq. (L_o_norm) at d = 2, evaluated on the sum g of the rows sent
//             as message 0: |g_y| + |c_y - g_y| per column, c = column totals
//   KIND_LD   Eq. (L_o_norm) at d >= 3 with one column-sum vector per message
enum Kind : int32_t { KIND_L1 = 0, KIND_MARG = 1, KIND_L2 = 2, KIND_LD = 3, KIND_SUMABS = 4 };

constexpr int MAX_MP = 64;      // widest column count held in registers
constexpr int MAX_D = 8;        // widest message alphabet with a register-resident kernel

// One problem as the kernels see it.  The row roles are fixed by the planner:
//
//  binary (L1, L_marg, L2): state s = column sums of the current sign vector,
//    int32 path: stored offset-binary (s + 2^31, unsigned), int64 path: plain.
//    base[MP]            state with the fixed row at +1, every mid row at Gray
//                        digit 0 and every high row at prefix bit 0
//    hid[P][MP]          change of the state when high row h has prefix bit 1
//    mid[C][2][MP]       change when mid row k flips 0 -> 1 ([k][0]) or 1 -> 0 ([k][1])
//    offs[K][2^R][MP]    per low-row pattern w: the value o with |s - o| equal to
//                        the column term of the word (s, w); K = 2 for L2
//                        (the two terms |g| and |c - g|), else 1
//    packed 16-bit int32 path: the same tables with two columns per dword (column
//    2j in bits 0..15, 2j+1 in bits 16..31), states and operands offset by 2^15,
//    and each stored delta the integer d_2j + 2^16 d_2j+1 modulo 2^32, so that one
//    32-bit add moves both columns; it needs sum_x |M_xy| <= 2^15 - 1 per column
//  d-ary (d >= 3): state g_k = column sums of the rows sent as message k
//    base[MP]            group-0 start: every mid row is at Gray digit 0
//    hid[P_tab+P][MP]    the prefix rows (restricted-growth table rows, then
//                        plain base-d rows)
//    mid[C][MP]          the Gray-swept rows
//    tab[]               restricted-growth prefixes, 4 bits per digit
//
// A lane processes prefix values v = pfx_base + p for p in [0, n_prefix): for the
// binary kinds bit h of v is the sign bit of high row h; for d-ary v is split as
// v = t * d^P + f with t indexing tab (when P_tab > 0) and f giving base-d digits.
struct Desc {
    int32_t kind;
    int32_t m;          // real columns
    int32_t mp;         // padded columns (pad columns contribute 0)
    int32_t d;
    int32_t i64;        // 1: int64 state, 0: offset-binary uint32 state
    int32_t R, C, P;    // low / mid / high row counts
    int32_t P_tab;      // d-ary restricted-growth prefix rows
    int32_t inst;       // kernel instantiation index
    int32_t bias;       // packed 16-bit kernels: constant added to every score (the
                        // linear column of L_marg is scored as |x + bias|, x >= -bias)
    uint64_t pfx_base;
    uint64_t n_prefix;
    uint64_t dpow_free; // d^P (d-ary)
    const void* base;
    const void* hid;
    const void* mid;
    const void* offs;
    const uint64_t* tab;
    int64_t* result;
    int64_t* rec;       // if not null: rec[v - pfx_base] = best of prefix v (locating a maximiser)
};

// One unit of a device work queue: prefixes [p0, p0 + count) of problem `prob`.
struct Item {
    uint32_t prob;
    uint32_t count;
    uint64_t p0;
};

// Arguments of every sweep kernel: waves pop items through the atomic counter
// `head` until it passes n_items.  With items == nullptr the items are implicit:
// item i covers prefixes [i * per, min((i + 1) * per, n_prefix)) of problem
// `prob` (one problem swept evenly, nothing to build or upload).
// Completion record of one problem in host-mapped memory (serving): the wave that
// finishes a problem's last item writes the value, then sets flag.
struct DoneRec {
    int64_t value;
    uint32_t flag;
    uint32_t pad;
};

struct QArgs {
    const Desc* descs;
    const Item* items;
    uint32_t n_items;
    uint32_t prob;
    uint32_t* head;
    uint64_t per;
    uint64_t n_prefix;
    // serving only (null otherwise): left[p] counts problem p's unfinished items;
    // each item publishes its maximum and decrements it, and the last one reports
    // the value in done[p]
    uint32_t* left;
    DoneRec* done;
};

}  // namespace ld
