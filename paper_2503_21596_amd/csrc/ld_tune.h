// Tuned sweep shapes for batches and plain calls.
#pragma once
#include "ld_plan.h"
#include "ld_program.h"

namespace ld {

struct Tuning {
    int bin_c_target = 10;        // batch, binary kinds: mid + low rows per prefix (2^c words)
    int dary_cwords = 2187;       // batch, d >= 3: words per prefix (d^C <= this)
    double item_words = 1 << 18;  // batch: words per queue item
    int plain_p_target = 20;      // plain calls: high rows of a large binary problem
    int plain_r_drop = 0;         // plain calls: one low row fewer than the register budget allows
};

Tuning get_tuning();
void set_tuning(const Tuning& t);

// sweep shape of one problem inside a batch
SweepShape batch_shape_for(int n, int m, int d);

// queue-item shape of a batch
ItemShape batch_item_shape();

}  // namespace ld
