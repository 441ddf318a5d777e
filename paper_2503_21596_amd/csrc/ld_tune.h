// Tuned sweep shapes for batches and plain calls.
#pragma once
#include "ld_plan.h"
#include "ld_program.h"

namespace ld {

struct Tuning {
    int bin_c_target = 8;         // batch, binary kinds: mid + low rows per prefix (2^c words)
    int dary_cwords = 729;        // batch, d >= 3: words per prefix (d^C <= this)
    double item_words = 1 << 16;  // batch: words per queue item
    int batch_pfx_cap = 0;        // batch: at most about 2^this prefixes per problem (0: no cap)
    int plain_p_target = 20;      // plain calls: at most 2^this lanes for a binary problem
    int plain_p_min = 19;         // plain calls: at least 2^this lanes when the problem has them
    int plain_c_goal = 12;        // plain calls: aim for 2^this words per prefix
    int plain_r_drop = 0;         // plain calls: one low row fewer than the register budget allows
    int sgpr_r = 16;              // int32 binary kinds: 16 the packed 16-bit kernel where it fits, else
                                  // low rows of the SGPR-operand kernel (4, 5; 0: VGPR kernel)
    int dary_variant = 16;        // int32 d = 3, 4: 16 packed where it fits, 1 SGPR operands, 0 VGPR
    int plain_dary_lanes = 1 << 19;  // plain calls, d >= 3: trade mid rows for prefix rows until
                                     // this many lanes exist
    int plain_big_r_c = 11;          // plain calls: mid rows at which the packed binary kernel
                                     // takes one more low row (0: never)
    int batch_side_streams = 3;      // batches: launches fan out over this many extra streams
                                     // (inside the captured graph for batch handles; 0: one
                                     // chain of launches)
    // kernel variant per (kind class, width bucket), as SweepShape::variant (-1: the above)
    int variant[4][4] = {{-1, -1, -1, -1}, {-1, -1, -1, -1}, {-1, -1, -1, -1}, {-1, -1, -1, -1}};
};

Tuning get_tuning();
void set_tuning(const Tuning& t);

// sweep shape of one problem inside a batch
SweepShape batch_shape_for(int n, int m, int d);

// queue-item shape of a batch
ItemShape batch_item_shape();

// extra streams a batch's launches fan out over
int batch_side_streams();

}  // namespace ld
