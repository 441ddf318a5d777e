// Host planner: validation, value-preserving preprocessing, the row roles of the
// sweep and the device tables of one problem.
#pragma once
#include <stdint.h>
#include <utility>
#include <vector>

#include "ld_types.h"

namespace ld {

enum PlanKind : int32_t { PK_L1 = 0, PK_MARG = 1, PK_L2 = 2, PK_LD = 3, PK_SUMABS = 4, PK_ZERO = 5 };

// (input index, sign) pairs folded into one row or column by preprocessing
using Members = std::vector<std::pair<int, int>>;

struct SweepShape {
    int p_target = 20;   // at most this many high rows (2^20 lanes) for a binary problem
    int p_min = 19;      // at least this many, when the problem has them
    int c_goal = 12;     // between the two: aim for 2^c_goal words per prefix
    int c_min = 4;       // least mid rows per lane when the problem allows it ...
    int p_fill = 16;     // ... and still keeps 2^p_fill prefixes (lanes); 0: c_min always
    int r_drop = 0;      // 1: one low row fewer than the register budget allows
    int dary_ptab = 8;   // restricted-growth prefix rows for d >= 3
    int dary_cwords = 4096;  // target d^C words per lane for d >= 3
    int c_target = 0;        // > 0: binary prefixes of 2^c_target words (mid + low rows), the
                             // rest of the rows become prefix rows (batch planning)
    int dary_lanes = 1 << 19;  // d >= 3: move mid rows into the prefix until this many
                               // lanes exist (0: keep dary_cwords words per lane)
    int sgpr_r = 16;           // int32 binary kinds: low rows of the SGPR-operand kernel
                               // (4 or 5); 0 selects the VGPR-operand kernel; 8 the kernel
                               // whose state update runs on the matrix cores (int8 MFMA,
                               // R = 5) where the problem's operands fit it; 16 the packed
                               // 16-bit kernel (R = 5) where every column bound fits it
    int dary_sgpr = 16;        // d-ary int32 problems (d = 3, 4): 16 the packed 16-bit kernel where
                               // every column bound fits it, 1 the SGPR-operand kernel where built,
                               // 0 the VGPR-operand kernel
    // tuned kernel variant per (kind class, padded-width bucket); -1 = the setting
    // above.  Classes: 0 L1 / L_marg, 1 L2, 2 L_3, 3 L_4; buckets: mp in (16b, 16b + 16].
    // Binary classes hold sgpr_r (0, 4, 5, 8, 16), d-ary classes dary_sgpr (0, 1, 16).
    int variant[4][4] = {{-1, -1, -1, -1}, {-1, -1, -1, -1}, {-1, -1, -1, -1}, {-1, -1, -1, -1}};
    int merge = 1;             // 1: merge proportional rows / columns and (d >= 2) uniform-
                               // sign columns before planning (exact reductions)
    int pfx_cap = 0;           // > 0 (batch planning): at most about 2^pfx_cap prefixes per
                               // problem; larger problems get more words per prefix instead
    int big_r_c = 11;          // plain calls of the packed binary kernel: at least this many mid
                               // rows at PACK16_R switch it to PACK16_R_BIG low rows (0: never)
};

struct Plan {
    int status = 0;            // LD_OK or an error code
    int kind = PK_ZERO;
    int n = 0, m = 0, d = 1;   // after preprocessing
    int transposed = 0;
    int i64 = 0;
    int mp = 0;
    int R = 0, C = 0, P = 0, P_tab = 0;
    uint64_t n_prefix = 0;
    uint64_t pfx_base = 0;
    uint64_t dpow_free = 1;
    double lanes_est = 0;   // d-ary plans while shaping: the lane count of the shape
    double words = 0;
    std::vector<int32_t> M;    // preprocessed matrix, n x m
    // per row / column of M: the input rows / columns (input columns / rows when
    // transposed) folded into it by preprocessing, each with the sign it enters with
    std::vector<Members> row_members, col_members;
    // device tables, laid out in one blob; offsets in bytes, each 256-aligned
    std::vector<uint8_t> blob;
    size_t off_base = 0, off_hid = 0, off_mid = 0, off_offs = 0, off_tab = 0;
    const void* kernel = nullptr;  // sweep kernel, null for PK_ZERO / PK_SUMABS
    int record = 0;                // 1: the sweep also stores every prefix's maximum
    int wide = 0;                  // 1: the wide (LDS-state, one wave per prefix) kernel
    int mfma = 0;                  // 1: the int8-MFMA kernel (one wave sweeps two prefixes)
    int pack16 = 0;                // 1: the packed 16-bit kernel (two columns per dword)
    int32_t bias = 0;              // packed L_marg: constant in every score (Desc::bias)
    size_t lds = 0;                // dynamic LDS bytes of the wide kernel
};

// prefixes one wave sweeps at a time: `lanes` for the register kernels (one per
// lane), two for the MFMA kernel (one per lane half), one for the wide kernel
inline uint64_t wave_prefixes(const Plan& p, uint64_t lanes) { return p.wide ? 1 : p.mfma ? 2 : lanes; }

// class and bucket of SweepShape::variant for a problem (class -1: none)
int variant_class(int kind, int d);
inline int variant_bucket(int mp) { return mp <= 16 ? 0 : mp <= 32 ? 1 : mp <= 48 ? 2 : 3; }

SweepShape get_shape();
void set_shape(const SweepShape& s);

// Full problem as ld_norm sees it.
Plan make_plan(const int32_t* M, int n, int m, int d, int marginals, const SweepShape& shape);

// Prefix-range problem as ld_norm_range sees it (no preprocessing).
Plan make_range_plan(const int32_t* M, int n, int m, int d, int marginals, int q,
                     uint64_t pfx_begin, uint64_t pfx_end);

// Fill the pointer fields of a descriptor for a blob placed at device address dev.
Desc make_desc(const Plan& p, const void* dev_blob, int64_t* result);

}  // namespace ld
