// A Program is everything needed to solve a set of planned problems on the GPU:
// one device image (tables, descriptors, queue items, queue heads, result slots)
// and the list of kernel launches over it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "ld_plan.h"
#include "ld_types.h"

namespace ld {

// one problem of k_sumabs_many: sum |M| of `count` int32 entries into *result
struct SumItem {
    const int32_t* M;
    int64_t count;
    int64_t* result;
};

struct Launch {
    const void* kernel = nullptr;
    uint32_t threads = 256;
    uint32_t blocks = 1;
    size_t lds = 0;
    size_t off_items = 0;     // byte offset of this launch's items in the image
    uint32_t n_items = 0;
    uint32_t head = 0;        // index of this launch's queue head
    double cost = 0;          // estimated VALU work, for ordering
    bool implicit = false;    // items computed on the device (one problem)
    uint32_t prob = 0;        // implicit items: the problem
    uint64_t per = 0;         // implicit items: prefixes per item
    uint64_t n_prefix = 0;    // implicit items: prefixes of the problem
};

struct Program {
    std::vector<uint8_t> image;              // host copy of the device image
    size_t off_descs = 0, off_items = 0, off_heads = 0, off_results = 0, off_sums = 0;
    uint32_t n_probs = 0, n_heads = 0, n_sums = 0;
    std::vector<size_t> blob_off;            // per problem, byte offset of its tables
    std::vector<size_t> rec_off;             // per problem, byte offset of its per-prefix
                                             // maxima (0: not recorded, see Plan::record)
    std::vector<Launch> launches;
    std::vector<int> zero;                   // problems whose value is 0 without a search
    void* dev = nullptr;                     // device address the image was patched for
};

struct ItemShape {
    uint32_t lanes_per_item = 64;   // prefixes per item for the register kernels
    double item_words = 0;          // if > 0: grow items up to about this many words
    uint32_t max_items = 1u << 20;  // per problem
    uint32_t min_items = 0;         // keep at least this many items per problem when it has that
                                    // many wave-sized pieces (single problems, server requests)
    // a launch shared by several problems: grow the items until the launch holds at
    // most about this many (pops on the one queue head serialize, tens of ns each)
    uint32_t max_launch_items = 1u << 16;
};

// queue items of a single-problem launch: about 2^22 words each (pops stay rare
// next to the work), at least two per resident wave (the SGPR-operand kernels
// hold seven waves per SIMD: 7168 on 256 CUs)
inline ItemShape plain_item_shape()
{
    ItemShape s;
    s.item_words = (double)(1u << 22);
    s.min_items = 16384;
    return s;
}

// Prefixes per queue item of a problem cut with shape `sh` (all items but the last
// hold that many; the last holds the rest).
uint64_t item_prefixes(const Plan& p, const ItemShape& sh);
// Estimated cost of an item of `count` prefixes: lane-level VALU instructions of one
// lane of the wave that sweeps it.
double item_cost(const Plan& p, uint64_t count);
// Split one problem's prefix space into queue items (tagged with problem index
// `prob`), each with its estimated VALU cost, in prefix order.  `wide` items are
// swept by one wave prefix after prefix; register-kernel items put one prefix on
// each lane.
void split_items(const Plan& p, uint32_t prob, const ItemShape& sh, std::vector<std::pair<double, Item>>& out);

// estimated VALU operations per word of a planned problem
double word_cost(const Plan& p);

// copy jobs of k_stage: bytes from src to dst, both device-visible
struct ScatterOp {
    const uint8_t* src;
    uint8_t* dst;
    uint64_t bytes;
};

// One server step's staging (k_stage): pointers into the step buffer in host
// memory (device view) and into device memory.  The first STAGE_INLINE copy jobs
// and new slots travel in the arguments themselves, one host-memory round trip
// fewer for a step that admits a few requests.
constexpr uint32_t STAGE_INLINE = 4;
struct StageArgs {
    const ScatterOp* ops;       // host: copy jobs (tables and descriptors of new problems)
    uint32_t nops;
    uint32_t n_slots;           // new problems
    const uint32_t* slots;      // host: their result slots
    const uint32_t* counts;     // host: their item counts
    int64_t* results;           // device: result slots
    uint32_t* left;             // device: unfinished-item counters
    const uint4* copy_src;      // host: queue items, heads and sum jobs of the step
    uint4* copy_dst;            // device: where the step's launches read them
    uint64_t copy_n16;          // 16-byte units
    ScatterOp iops[STAGE_INLINE];          // ops[0 .. STAGE_INLINE)
    uint32_t islots[STAGE_INLINE], icounts[STAGE_INLINE];
};

// Build the image and launches for the given plans (all with status LD_OK).
Program build_program(const std::vector<const Plan*>& plans, const ItemShape& shape);

// Write device pointers into the image for a device buffer at `dev`.
void patch_program(Program& prog, void* dev);

// Enqueue: reset of heads and results, every launch, and the copy of the results
// to host_results (pinned, n_probs int64).  Nothing here allocates.
bool enqueue_program(const Program& prog, hipStream_t s, int64_t* host_results);
// The same with the launches spread over the side streams (fork after the reset,
// join before the copy); evs holds side.size() + 1 events.  Also valid under
// stream capture, where the forks and joins become graph edges.
bool enqueue_program_fanned(const Program& prog, hipStream_t s, int64_t* host_results,
                            const std::vector<hipStream_t>& side, const std::vector<hipEvent_t>& evs);

// Blocks per launch that fill the device once for a kernel (occupancy x CUs).
uint32_t resident_blocks(const void* kernel, uint32_t threads, size_t lds);
// The same, capped at the waves per SIMD set by set_launch_waves (plain and batch
// launches; the server sizes its own launches).
uint32_t capped_blocks(const void* kernel, uint32_t threads, size_t lds);
void set_launch_waves(int waves_per_simd);   // 0: as many as occupancy allows
uint32_t device_cus();                       // compute units of the current device

}  // namespace ld
