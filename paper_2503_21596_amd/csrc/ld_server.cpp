// Request server: continuous batching of L_d solves on one GPU (see include/ld.h).
//
// Submitting threads plan their request and queue it.  One scheduler thread owns
// the device.  Each scheduler step:
//   1. retires finished steps: a request whose items have all run is complete,
//      and its value is read from the result copy of the step that ran its last
//      items;
//   2. admits queued requests while a result slot and arena bytes are free;
//   3. picks items, smallest remaining work first, up to about step_ms of
//      device work;
//   4. enqueues: one staging kernel that reads the step buffer (new tables,
//      descriptors, items) from pinned host memory, puts tables and descriptors
//      in place and resets the new result slots; one persistent queue launch per
//      kernel shape; and a kernel that writes every result slot to pinned host
//      memory.  The staging and result kernels raise their waves' priority, as
//      express launches do, since a step shares the SIMDs with a long bulk
//      sweep; runtime copies (kernels too) could not.
// One bulk step and up to two express steps are in flight, so a request that
// arrives while others run is swept in the next step.  Result slots keep partial
// maxima between steps.  A bulk request completes when the step with its last
// items retires; an express request as soon as its last item ends (that wave
// reports the value in a host-mapped record, without waiting for the rest of its
// step).
//
// There are two lanes, each with its own stream and steps: bulk and express.  A
// request of less than about a millisecond of work goes to the express lane,
// whose launches take at most one block per CU while bulk work runs, with their
// waves at raised issue priority; bulk launches leave one block per CU free (always
// when their kernel fits five or more per CU, else while there is express work and
// it fits three), so express work starts at once instead of queueing behind bulk
// steps, and runs at close to the speed of an idle SIMD.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ld.h"
#include "ld_api_internal.h"
#include "ld_plan.h"
#include "ld_program.h"
#include "ld_registry.h"
#include "ld_tune.h"

using namespace ld;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Sustained VALU rate used to size steps (lane-instructions/s: about 95 % of 256
// CUs x 64 lanes x 2.37 GHz); only step lengths and the express threshold depend on
// it.  Item costs (split_items) count the instructions of one lane of the wave that
// runs the item, so an item occupies the device for about cost x 64 lane-instructions.
constexpr double STEP_OPS_PER_S = 3.6e13;
constexpr double COST_UNITS_PER_S = STEP_OPS_PER_S / 64.0;

// An idle scheduler polls for new requests this long before it sleeps: longer than
// the gaps of a few hundred requests per second, so that such a stream never waits
// for a thread wake-up.  It keeps one host thread busy meanwhile.
constexpr double IDLE_SPIN_S = 0.05;

constexpr size_t TIMINGS_KEPT = (size_t)1 << 20;   // per-request timing records kept

// least queue items of a request that has that many 64-lane pieces: about one per
// resident wave of a sweep kernel (4 to 6 per SIMD on 1024 SIMDs)
constexpr uint32_t SERVE_MIN_ITEMS = 4096;

struct Request {
    uint64_t ticket = 0;
    Plan plan;
    double t_submit = 0, t_done = 0, t_issue = 0, t_queued = 0;
    int status = LD_PENDING;
    int64_t value = 0;
    // scheduling state
    int slot = -1;
    size_t arena_off = 0, arena_size = 0;
    bool tracked = false;            // completes through its host-mapped record
    // queue items, implicit: item k holds prefixes [k per, min((k + 1) per, n_prefix)),
    // all but the last one the same length, so issuing them in order is longest first
    uint32_t n_items = 0;
    uint64_t per = 0;
    double cost_full = 0, cost_last = 0;
    uint32_t next = 0;               // first item not yet issued
    double remaining = 0;            // estimated cost of the items not yet issued
    uint32_t outstanding = 0;        // issued items, plus the admission, whose step has not retired
    bool canceled = false;
    bool is_sum = false;
    int lane = 0;                    // 0 bulk, 1 express
};

// first-fit allocator over [0, size)
struct Arena {
    std::map<size_t, size_t> free_;   // offset -> bytes
    explicit Arena(size_t size = 0) { if (size) free_[0] = size; }
    bool alloc(size_t bytes, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Step {
    hipEvent_t ev = nullptr;
    bool busy = false;
    uint8_t* host = nullptr;      // step buffer, pinned host memory the device reads directly
    uint8_t* host_dev = nullptr;  // its device view
    uint8_t* dev = nullptr;       // device copy of its items, heads and sum jobs
    int64_t* hres = nullptr;      // every result slot after the step (pinned, written by k_publish)
    int64_t* hres_dev = nullptr;  // its device view
    std::vector<std::pair<Request*, uint32_t>> issued;   // request, items in this step
};

struct Lane {
    hipStream_t stream = nullptr;
    Step steps[2];
    int next_step = 0;
    std::deque<Request*> pending;   // submitted, not admitted (FIFO)
};

constexpr int BULK = 0, EXPRESS = 1;

}  // namespace

struct ld_server {
    ld_server_config cfg{};
    int device = 0;
    int cus = 0;                      // compute units of the device
    double express_cost = 0;          // request cost (item-cost units) below which it is express
    // bulk steps in flight: one.  A request arriving behind bulk work then waits for
    // one step, not two (the gap between steps costs less: on the served traces
    // mean latency fell by about a seventh, p99 unchanged)
    int bulk_depth = 1;
    double idle_spin_s = IDLE_SPIN_S;   // how long an idle scheduler polls for arrivals (config)
    uint8_t* arena_dev = nullptr;
    Desc* d_descs = nullptr;
    int64_t* d_results = nullptr;
    uint32_t* d_left = nullptr;      // per slot: items of the request not yet finished
    DoneRec* done_host = nullptr;    // per slot: completion record (host-mapped)
    DoneRec* done_dev = nullptr;     // the same memory as the kernels address it
    size_t step_bytes = 0;
    Lane lanes[2];
    Arena arena;
    std::vector<int> free_slots;
    std::vector<Request*> slots;

    std::mutex mu;
    // API calls waiting for mu.  While steps are in flight the scheduler polls in a
    // loop and takes mu on every pass; the mutex is not fair, so a call could wait
    // milliseconds for it.  The scheduler lets waiting calls go first.
    std::atomic<int> api_waiting{0};
    std::condition_variable cv;       // scheduler wake-up
    // submissions so far and the stop request, readable without mu: an idle
    // scheduler watches them for a while before it sleeps on cv
    std::atomic<uint64_t> arrivals{0};
    std::atomic<bool> stopping{false};
    std::condition_variable done_cv;  // request completion
    std::unordered_map<uint64_t, Request*> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool failed = false;
    std::thread worker;

    uint64_t st_submitted = 0, st_completed = 0, st_rejected = 0, st_launches = 0, st_items = 0;
    std::vector<double> latencies_ms;
    std::deque<ld_request_timing> timings;   // completed requests, oldest first (bounded)
    double wait_sum_ms = 0, plan_sum_ms = 0, run_sum_ms = 0;
    uint64_t wait_n = 0, plan_n = 0, run_n = 0;

    ~ld_server()
    {
        for (auto& ln : lanes) {
            for (auto& s : ln.steps) {
                if (s.ev) (void)hipEventDestroy(s.ev);
                if (s.host) (void)hipHostFree(s.host);
                if (s.dev) (void)hipFree(s.dev);
                if (s.hres) (void)hipHostFree(s.hres);
            }
            if (ln.stream) (void)hipStreamDestroy(ln.stream);
        }
        if (arena_dev) (void)hipFree(arena_dev);
        if (d_descs) (void)hipFree(d_descs);
        if (d_results) (void)hipFree(d_results);
        if (d_left) (void)hipFree(d_left);
        if (done_host) (void)hipHostFree(done_host);
        for (auto& kv : all) delete kv.second;
    }
};

namespace {

// mu for an API call: announced, so that the scheduler steps aside (scheduler_lock)
struct ApiLock {
    std::unique_lock<std::mutex> lk;
    explicit ApiLock(ld_server* S) : lk(S->mu, std::defer_lock)
    {
        S->api_waiting.fetch_add(1, std::memory_order_relaxed);
        lk.lock();
        S->api_waiting.fetch_sub(1, std::memory_order_relaxed);
    }
};

// mu for the scheduler thread, after any API call waiting for it (bounded, so that
// a stream of calls cannot hold the scheduler off)
std::unique_lock<std::mutex> scheduler_lock(ld_server* S)
{
    for (int k = 0; k < 256 && S->api_waiting.load(std::memory_order_relaxed) > 0; ++k) std::this_thread::yield();
    return std::unique_lock<std::mutex>(S->mu);
}

// complete a request (mu held)
void finish(ld_server* S, Request* r, int status, int64_t value)
{
    r->status = status;
    r->value = value;
    r->t_done = now_s();
    if (status == LD_OK) {
        S->st_completed++;
        S->latencies_ms.push_back(1e3 * (r->t_done - r->t_submit));
        if (r->t_issue > 0) {
            S->run_sum_ms += 1e3 * (r->t_done - r->t_issue);
            S->run_n++;
        }
        ld_request_timing t{};
        t.ticket = r->ticket;
        t.lane = r->lane;
        t.items = (int32_t)r->n_items;
        t.words = r->plan.words;
        t.plan_ms = 1e3 * (r->t_queued - r->t_submit);
        const double issued = r->t_issue > 0 ? r->t_issue : r->t_done;
        t.wait_ms = 1e3 * (issued - r->t_queued);
        t.run_ms = 1e3 * (r->t_done - issued);
        S->timings.push_back(t);
        if (S->timings.size() > TIMINGS_KEPT) S->timings.pop_front();
    }
    r->plan = Plan{};   // keep only the outcome
    S->done_cv.notify_all();
}

void release_slot(ld_server* S, Request* r)
{
    if (r->slot >= 0) {
        S->slots[r->slot] = nullptr;
        S->free_slots.push_back(r->slot);
        r->slot = -1;
    }
    if (r->arena_size) {
        S->arena.release(r->arena_off, r->arena_size);
        r->arena_size = 0;
    }
}

// Retire the oldest busy step of a lane if it has finished.
bool retire(ld_server* S, Lane& L)
{
    for (int k = 0; k < 2; ++k) {
        Step& st = L.steps[(L.next_step + k) % 2];
        if (!st.busy) continue;
        {
            const hipError_t q = hipEventQuery(st.ev);
            if (q == hipErrorNotReady) return true;
            if (q != hipSuccess) return false;
        }
        auto g = scheduler_lock(S);
        for (auto& [r, n] : st.issued) {
            r->outstanding -= n;
            // (a request that completed through its record has no items left)
            if (r->outstanding == 0 && r->next >= r->n_items && r->slot >= 0) {
                const int slot = r->slot;
                const int64_t v = st.hres[slot];
                release_slot(S, r);
                if (r->status == LD_PENDING) finish(S, r, r->canceled ? LD_ECANCELED : LD_OK, v);
            }
        }
        st.issued.clear();
        st.busy = false;
        return true;
    }
    return true;
}

int busy_steps(const Lane& L) { return (int)L.steps[0].busy + (int)L.steps[1].busy; }

// Build and enqueue one step of lane `li`.  Returns false on a HIP error.
bool issue_step(ld_server* S, int li, bool* issued_any)
{
    *issued_any = false;
    Lane& L = S->lanes[li];
    Step& st = L.steps[L.next_step];
    if (st.busy) return true;
    const int max_slots = S->cfg.max_inflight_problems;
    std::vector<Request*> admitted;
    std::vector<std::pair<Request*, std::vector<Item>>> picks;
    bool express_active = false;
    {
        auto g = scheduler_lock(S);
        // 2. admission by slot and arena space (FIFO; a request too big for the
        // free arena waits and holds back the ones behind it)
        while (!L.pending.empty() && !S->free_slots.empty()) {
            Request* r = L.pending.front();
            const size_t bytes = align256(std::max<size_t>(r->plan.blob.size(), 256));
            size_t off;
            if (!S->arena.alloc(bytes, &off)) break;
            L.pending.pop_front();
            r->arena_off = off;
            r->arena_size = bytes;
            r->slot = S->free_slots.back();
            S->free_slots.pop_back();
            S->slots[r->slot] = r;
            // the admitting step writes the slot's descriptor, tables and counters:
            // hold the slot until that step retires, even if it runs none of the
            // request's items (a cancel meanwhile must not hand the slot on)
            r->outstanding += 1;
            admitted.push_back(r);
        }
        // 3. items: smallest remaining work first, up to the step budget
        std::vector<Request*> live;
        for (Request* r : S->slots)
            if (r && r->lane == li && r->next < r->n_items) live.push_back(r);
        std::sort(live.begin(), live.end(), [](Request* a, Request* b) { return a->remaining < b->remaining; });
        // a long bulk queue (saturation) gets steps twice as long: fewer steps, less
        // per-step overhead; the express lane keeps small requests responsive
        double budget = COST_UNITS_PER_S * S->cfg.step_ms * 1e-3;
        if (li == BULK && live.size() > 16) budget *= 2;
        // bulk launches leave room for express work only while there is some
        express_active = busy_steps(S->lanes[EXPRESS]) > 0 || !S->lanes[EXPRESS].pending.empty();
        for (Request* r : S->slots)
            if (r && r->lane == EXPRESS && r->status == LD_PENDING) express_active = true;
        double used = 0;
        size_t n_items = 0;
        for (Request* r : live) {
            if (used >= budget || n_items >= (size_t)S->cfg.max_items_per_launch) break;
            std::vector<Item> take;
            while (r->next < r->n_items && (take.empty() || used < budget) &&
                   n_items < (size_t)S->cfg.max_items_per_launch) {
                Item it;
                it.prob = (uint32_t)r->slot;
                it.p0 = (uint64_t)r->next * r->per;
                it.count = (uint32_t)std::min<uint64_t>(r->per, r->plan.n_prefix - it.p0);
                const double c = r->next + 1 == r->n_items ? r->cost_last : r->cost_full;
                used += c;
                r->remaining -= c;
                ++r->next;
                take.push_back(it);
                ++n_items;
            }
            if (!take.empty()) {
                if (r->t_issue == 0) {
                    r->t_issue = now_s();
                    S->wait_sum_ms += 1e3 * (r->t_issue - r->t_submit);
                    S->wait_n++;
                }
                r->outstanding += (uint32_t)take.size();
                picks.push_back({r, std::move(take)});
            }
        }
        // sum-|M| requests run once, in the step that admits them
        for (Request* r : admitted)
            if (r->is_sum) {
                r->outstanding += 1;
                picks.push_back({r, {}});
            }
    }
    if (admitted.empty() && picks.empty()) return true;

    // layout of the step buffer: scatter ops, new tables, new descriptors, reset
    // slots, items (grouped by kernel), sum items
    std::map<std::pair<const void*, size_t>, std::vector<Item>> groups;
    std::map<std::pair<const void*, size_t>, size_t> group_lds;
    std::vector<SumItem> sums;
    for (auto& [r, items] : picks) {
        if (r->is_sum) {
            SumItem si;
            si.M = (const int32_t*)(S->arena_dev + r->arena_off);
            si.count = (int64_t)r->plan.n * r->plan.m;
            si.result = S->d_results + r->slot;
            sums.push_back(si);
            continue;
        }
        auto key = std::make_pair(r->plan.kernel, (size_t)(r->plan.wide ? 1 : 0));
        auto& v = groups[key];
        v.insert(v.end(), items.begin(), items.end());
        group_lds[key] = std::max(group_lds[key], r->plan.lds);
    }
    size_t off = 0;
    const size_t off_ops = off;
    off = align256(off + sizeof(ScatterOp) * 2 * admitted.size());
    std::vector<size_t> blob_at(admitted.size()), desc_at(admitted.size());
    for (size_t k = 0; k < admitted.size(); ++k) {
        blob_at[k] = off;
        off = align256(off + admitted[k]->plan.blob.size());
    }
    for (size_t k = 0; k < admitted.size(); ++k) {
        desc_at[k] = off;
        off = align256(off + sizeof(Desc));
    }
    const size_t off_slots = off;
    off = align256(off + 4 * admitted.size());
    const size_t off_counts = off;
    off = align256(off + 4 * admitted.size());
    // from here on the buffer is copied to device memory by k_stage (the launches
    // pop its items and count on its heads); the part above is read in place
    const size_t off_copy = off;
    std::vector<std::pair<size_t, size_t>> gpos;   // items offset, count per group
    for (auto& g : groups) {
        gpos.push_back({off, g.second.size()});
        off = align256(off + sizeof(Item) * g.second.size());
    }
    const size_t off_heads = off;
    off = align256(off + 4 * std::max<size_t>(groups.size(), 1));
    const size_t off_sums = off;
    off = align256(off + sizeof(SumItem) * sums.size());
    if (off > S->step_bytes) {
        // cannot happen with the admission limits below; refuse rather than overflow
        return false;
    }

    uint8_t* H = st.host;
    uint8_t* HD = st.host_dev;
    uint8_t* D = st.dev;
    std::vector<ScatterOp> ops;
    for (size_t k = 0; k < admitted.size(); ++k) {
        Request* r = admitted[k];
        std::memcpy(H + blob_at[k], r->plan.blob.data(), r->plan.blob.size());
        ops.push_back({HD + blob_at[k], S->arena_dev + r->arena_off, (uint64_t)r->plan.blob.size()});
        const Desc d = make_desc(r->plan, S->arena_dev + r->arena_off, S->d_results + r->slot);
        std::memcpy(H + desc_at[k], &d, sizeof(Desc));
        ops.push_back({HD + desc_at[k], (uint8_t*)(S->d_descs + r->slot), (uint64_t)sizeof(Desc)});
        const uint32_t slot = (uint32_t)r->slot;
        std::memcpy(H + off_slots + 4 * k, &slot, 4);
        const uint32_t count = r->is_sum ? 0u : r->n_items;
        std::memcpy(H + off_counts + 4 * k, &count, 4);
        // the completion record starts clear (nothing can write it: the slot was free)
        __atomic_store_n(&S->done_host[slot].flag, 0u, __ATOMIC_RELEASE);
        r->tracked = !r->is_sum && r->lane == EXPRESS;
    }
    if (!ops.empty()) std::memcpy(H + off_ops, ops.data(), sizeof(ScatterOp) * ops.size());
    size_t gi = 0;
    for (auto& g : groups) {
        std::memcpy(H + gpos[gi].first, g.second.data(), sizeof(Item) * g.second.size());
        ++gi;
    }
    std::memset(H + off_heads, 0, 4 * std::max<size_t>(groups.size(), 1));
    if (!sums.empty()) std::memcpy(H + off_sums, sums.data(), sizeof(SumItem) * sums.size());

    // 4. enqueue: staging (reads the step buffer in host memory), the queue
    // launches, the sum jobs, the results to host memory
    hipStream_t s = L.stream;
    uint32_t* dheads = (uint32_t*)(D + off_heads);
    bool ok;
    {
        StageArgs a{};
        a.ops = (const ScatterOp*)(HD + off_ops);
        a.nops = (uint32_t)ops.size();
        a.n_slots = (uint32_t)admitted.size();
        a.slots = (const uint32_t*)(HD + off_slots);
        a.counts = (const uint32_t*)(HD + off_counts);
        a.results = S->d_results;
        a.left = S->d_left;
        a.copy_src = (const uint4*)(HD + off_copy);
        a.copy_dst = (uint4*)(D + off_copy);
        a.copy_n16 = (off - off_copy) / 16;
        for (uint32_t k = 0; k < STAGE_INLINE && k < a.nops; ++k) a.iops[k] = ops[k];
        for (uint32_t k = 0; k < STAGE_INLINE && k < a.n_slots; ++k) {
            a.islots[k] = (uint32_t)admitted[k]->slot;
            a.icounts[k] = admitted[k]->is_sum ? 0u : admitted[k]->n_items;
        }
        // one block per copy job, then blocks for the slots and the rest of the buffer
        const uint64_t rest = std::min<uint64_t>(
            512, std::max<uint64_t>({(a.copy_n16 + 1023) / 1024, ((uint64_t)a.n_slots + 255) / 256, 1}));
        void* args[] = {(void*)&a};
        ok = hipLaunchKernel(kernel_stage(), dim3((uint32_t)(a.nops + rest)), dim3(256), args, 0, s) == hipSuccess;
    }
    gi = 0;
    size_t n_items = 0;
    for (auto& g : groups) {
        QArgs q{};   // explicit items (several problems per launch)
        q.descs = S->d_descs;
        if (li == EXPRESS) {
            // small requests report their value as soon as their last item ends.
            // (Not for bulk work: its many items would all count down one counter,
            // and atomics on one address from every XCD serialize.)
            q.left = S->d_left;
            q.done = S->done_dev;
        }
        q.items = (const Item*)(D + gpos[gi].first);
        q.n_items = (uint32_t)gpos[gi].second;
        q.head = dheads + gi;
        const uint32_t threads = g.first.second ? 64 : 256;
        const size_t lds = group_lds[g.first];
        const uint32_t want = (q.n_items + threads / 64 - 1) / (threads / 64);
        const uint32_t resident = resident_blocks(g.first.first, threads, lds);
        const uint32_t per_cu = S->cus > 0 ? resident / (uint32_t)S->cus : 0;
        uint32_t cap = resident;
        // express work takes one block per CU (at raised wave priority) while bulk
        // steps run, the whole device otherwise.  Bulk work leaves room for it:
        // always when its kernel fits five or more per CU (a wave fewer per SIMD
        // does not slow a VALU-bound sweep there, and an express request then never
        // waits for a bulk step to drain), else while express work exists.  The room
        // is one block per CU, and a bulk launch takes at most five per CU: bulk L2
        // launches of six per CU (kernels rated at seven) held back express
        // dispatches until the bulk launch drained, milliseconds later, while five
        // per CU never did.
        if (li == EXPRESS) {
            if (busy_steps(S->lanes[BULK]) > 0) cap = std::min<uint32_t>(resident, std::max(S->cus, 1));
        } else if (per_cu >= 5 || (per_cu >= 3 && express_active)) {
            cap = std::min<uint32_t>(resident - (uint32_t)S->cus, 5u * (uint32_t)S->cus);
        }
        const uint32_t blocks = std::max<uint32_t>(1, std::min(want, cap));
        void* args[] = {(void*)&q};
        ok = ok && hipLaunchKernel(g.first.first, dim3(blocks), dim3(threads), args, lds, s) == hipSuccess;
        n_items += q.n_items;
        ++gi;
    }
    if (ok && !sums.empty()) {
        const SumItem* ds = (const SumItem*)(D + off_sums);
        uint32_t n = (uint32_t)sums.size();
        void* args[] = {(void*)&ds, (void*)&n};
        ok = hipLaunchKernel(kernel_sumabs_many(), dim3(std::min<uint32_t>(n, 1024)), dim3(256), args, 0, s) ==
             hipSuccess;
    }
    {
        const int64_t* res = S->d_results;
        int64_t* out = st.hres_dev;
        uint32_t n = (uint32_t)max_slots;
        void* args[] = {(void*)&res, (void*)&out, (void*)&n};
        ok = ok && hipLaunchKernel(kernel_publish(), dim3((n + 255) / 256), dim3(256), args, 0, s) == hipSuccess;
    }
    ok = ok && hipEventRecord(st.ev, s) == hipSuccess;
    {
        auto g = scheduler_lock(S);
        for (auto& [r, items] : picks) st.issued.push_back({r, r->is_sum ? 1u : (uint32_t)items.size()});
        for (Request* r : admitted) st.issued.push_back({r, 1u});   // the admission hold
        S->st_launches += groups.size() + (sums.empty() ? 0 : 1);
        S->st_items += n_items;
    }
    st.busy = true;
    L.next_step = 1 - L.next_step;
    *issued_any = true;
    return ok;
}

// Requests whose last item has ended report through their host-mapped record;
// complete them without waiting for the rest of their step (mu held).  Their slot
// is released when the step retires.
void poll_done(ld_server* S)
{
    for (Request* r : S->slots) {
        if (!r || !r->tracked || r->status != LD_PENDING) continue;
        const DoneRec& d = S->done_host[r->slot];
        if (__atomic_load_n(&d.flag, __ATOMIC_ACQUIRE) == 0) continue;
        const int64_t v = __atomic_load_n(&d.value, __ATOMIC_RELAXED);
        finish(S, r, r->canceled ? LD_ECANCELED : LD_OK, v);
    }
}

void scheduler(ld_server* S)
{
    (void)hipSetDevice(S->device);
    auto busy_all = [&]() { return busy_steps(S->lanes[BULK]) + busy_steps(S->lanes[EXPRESS]); };
    for (;;) {
        bool have_work[2];
        int bulk_depth = S->bulk_depth;
        {
            std::unique_lock<std::mutex> lk = scheduler_lock(S);
            auto work_left = [&](int li) {
                if (!S->lanes[li].pending.empty() && !S->free_slots.empty()) return true;
                for (Request* r : S->slots)
                    if (r && r->lane == li && r->next < r->n_items) return true;
                return false;
            };
            auto any_work = [&]() { return work_left(BULK) || work_left(EXPRESS); };
            poll_done(S);
            if (busy_all() == 0) {
                if (!S->stop && !any_work() && S->idle_spin_s > 0) {
                    // Idle.  A thread woken from a condition variable starts tens to
                    // hundreds of microseconds later, which a small request would pay
                    // on top of its own run time; so watch the arrival count first and
                    // sleep only after idle_spin_s without one.
                    const uint64_t seen = S->arrivals.load(std::memory_order_acquire);
                    lk.unlock();
                    const double t0 = now_s();
                    while (S->arrivals.load(std::memory_order_acquire) == seen &&
                           !S->stopping.load(std::memory_order_acquire) && now_s() - t0 < S->idle_spin_s)
                        std::this_thread::yield();
                    lk.lock();
                }
                S->cv.wait(lk, [&]() { return S->stop || any_work(); });
                if (S->stop && !any_work()) return;
            }
            have_work[BULK] = work_left(BULK);
            have_work[EXPRESS] = work_left(EXPRESS);
            // a long bulk queue (saturation) keeps a second bulk step queued behind
            // the running one, so that the device never waits for the host
            size_t bulk_live = S->lanes[BULK].pending.size();
            for (Request* r : S->slots)
                if (r && r->lane == BULK && r->next < r->n_items) ++bulk_live;
            bulk_depth = bulk_live > 16 ? 2 : S->bulk_depth;
        }
        bool ok = true, issued = false;
        for (int li : {EXPRESS, BULK}) {
            Lane& L = S->lanes[li];
            ok = ok && retire(S, L);
            bool one = false;
            if (ok && have_work[li] && busy_steps(L) < (li == BULK ? bulk_depth : 2)) ok = issue_step(S, li, &one);
            issued = issued || one;
        }
        if (!ok) break;
        if (!issued && busy_all() > 0) {
            // steps in flight and nothing to add: poll again at once for finished
            // requests and steps (the device writes completion records to host
            // memory; a timed wait would add the timer's slack to every latency)
            std::this_thread::yield();
        }
    }
    // a HIP failure: fail everything still open
    std::lock_guard<std::mutex> g(S->mu);
    S->failed = true;
    for (auto& kv : S->all)
        if (kv.second->status == LD_PENDING) finish(S, kv.second, LD_EHIP, INT64_MIN);
}

}  // namespace

extern "C" {

ld_server* ld_server_create(const ld_server_config* cfg_in)
{
    ld_server_config cfg{};
    if (cfg_in) cfg = *cfg_in;
    if (!cfg.arena_bytes) cfg.arena_bytes = (uint64_t)256 << 20;
    if (cfg.max_inflight_problems <= 0) cfg.max_inflight_problems = 1024;
    if (cfg.max_items_per_launch <= 0) cfg.max_items_per_launch = 65536;
    if (cfg.words_per_item <= 0) cfg.words_per_item = (double)(1 << 17);
    if (cfg.step_ms <= 0) cfg.step_ms = 4.0;
    if (cfg.express_ms == 0) cfg.express_ms = 1.0;
    if (cfg.max_queued <= 0) cfg.max_queued = 65536;
    if (cfg.idle_spin_ms == 0) cfg.idle_spin_ms = 1e3 * IDLE_SPIN_S;
    if (cfg.min_items == 0) cfg.min_items = (int32_t)SERVE_MIN_ITEMS;
    ld_server* S = new ld_server;
    S->cfg = cfg;
    S->express_cost = COST_UNITS_PER_S * cfg.express_ms * 1e-3;
    S->idle_spin_s = std::max(0.0, cfg.idle_spin_ms * 1e-3);
    S->device = cfg.device;
    int count = 0;
    bool ok = hipGetDeviceCount(&count) == hipSuccess && cfg.device >= 0 && cfg.device < count &&
              hipSetDevice(cfg.device) == hipSuccess && device_ok(nullptr);
    {
        hipDeviceProp_t prop;
        ok = ok && hipGetDeviceProperties(&prop, cfg.device) == hipSuccess;
        if (ok) S->cus = prop.multiProcessorCount;
    }
    // The lanes' streams must run on different hardware queues, or express
    // launches would wait behind bulk ones in one in-order queue.  A process has
    // few hardware queues (4 by default) and streams beyond that share them, so
    // plain streams created after others (a batch's graph, prepared handles) can
    // land on the same queue.  A stream with a CU mask gets a queue of its own;
    // the mask here enables every CU.
    if (ok) {
        std::vector<uint32_t> mask((size_t)(S->cus + 31) / 32, 0xffffffffu);
        if (S->cus % 32) mask.back() = (1u << (S->cus % 32)) - 1;
        for (auto& ln : S->lanes) {
            if (hipExtStreamCreateWithCUMask(&ln.stream, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
                ln.stream = nullptr;
                ok = hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) == hipSuccess;
            }
            if (!ok) break;
        }
    }
    ok = ok && hipMalloc((void**)&S->arena_dev, cfg.arena_bytes) == hipSuccess;
    ok = ok && hipMalloc((void**)&S->d_descs, sizeof(Desc) * cfg.max_inflight_problems) == hipSuccess;
    ok = ok && hipMalloc((void**)&S->d_results, 8 * (size_t)cfg.max_inflight_problems) == hipSuccess;
    ok = ok && hipMalloc((void**)&S->d_left, 4 * (size_t)cfg.max_inflight_problems) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&S->done_host, sizeof(DoneRec) * cfg.max_inflight_problems,
                             hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess;
    ok = ok && hipHostGetDevicePointer((void**)&S->done_dev, S->done_host, 0) == hipSuccess;
    if (ok) std::memset(S->done_host, 0, sizeof(DoneRec) * cfg.max_inflight_problems);
    // a step uploads at most every slot's tables and descriptors plus its items
    S->step_bytes = align256(sizeof(ScatterOp) * 2 * cfg.max_inflight_problems) + cfg.arena_bytes +
                    align256(256 + sizeof(Desc)) * (size_t)cfg.max_inflight_problems +
                    align256(4 * (size_t)cfg.max_inflight_problems) +
                    align256(sizeof(Item) * (size_t)cfg.max_items_per_launch) + 256 * 64 +
                    align256(sizeof(SumItem) * (size_t)cfg.max_inflight_problems) + (1 << 16);
    for (auto& ln : S->lanes)
    for (auto& st : ln.steps) {
        ok = ok && hipEventCreateWithFlags(&st.ev, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipHostMalloc((void**)&st.host, S->step_bytes, hipHostMallocMapped | hipHostMallocCoherent) ==
                       hipSuccess;
        ok = ok && hipHostGetDevicePointer((void**)&st.host_dev, st.host, 0) == hipSuccess;
        ok = ok && hipMalloc((void**)&st.dev, S->step_bytes) == hipSuccess;
        ok = ok && hipHostMalloc((void**)&st.hres, 8 * (size_t)cfg.max_inflight_problems,
                                 hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess;
        ok = ok && hipHostGetDevicePointer((void**)&st.hres_dev, st.hres, 0) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        delete S;
        set_error(LD_EHIP);
        return nullptr;
    }
    // first use of a stream sets up its hardware queue (milliseconds): do it now,
    // not in the first request's latency
    for (auto& ln : S->lanes) {
        unsigned long long* dummy = (unsigned long long*)ln.steps[0].dev;   // step_bytes >= 64 KiB
        unsigned long long v = 0;
        void* args[] = {(void*)&dummy, (void*)&v};
        ok = ok && hipLaunchKernel(kernel_set_u64(), dim3(1), dim3(64), args, 0, ln.stream) == hipSuccess;
        ok = ok && hipStreamSynchronize(ln.stream) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        delete S;
        set_error(LD_EHIP);
        return nullptr;
    }
    S->arena = Arena(cfg.arena_bytes);
    S->slots.assign(cfg.max_inflight_problems, nullptr);
    for (int i = cfg.max_inflight_problems - 1; i >= 0; --i) S->free_slots.push_back(i);
    S->worker = std::thread(scheduler, S);
    return S;
}

int ld_server_submit(ld_server* S, const ld_problem* p, uint64_t* ticket)
{
    if (!S || !p || !ticket) {
        set_error(LD_EINVAL);
        return LD_EINVAL;
    }
    Request* r = new Request;
    r->t_submit = now_s();
    // Requests mostly run a few at a time, so a large one must fill the device by
    // itself (a batch shape would cap its lanes); and its queue items must be short,
    // so that a step of step_ms still holds a few items per resident wave and a
    // request arriving meanwhile waits at most about two steps.  Hence the plain
    // shape with more, shorter lanes: 2^22 lanes at most, about 2^11 words each.
    SweepShape sh = get_shape();
    sh.p_target = std::max(sh.p_target, 22);
    sh.p_min = std::max(sh.p_min, 18);
    sh.c_goal = std::min(sh.c_goal, 11);
    r->plan = make_plan(p->M, p->n, p->m, p->d, p->marginals, sh);
    if (r->plan.status == LD_OK && r->plan.kind != PK_ZERO) {
        if (r->plan.kind == PK_SUMABS) {
            r->is_sum = true;
        } else {
            ItemShape ish;
            ish.item_words = S->cfg.words_per_item;
            ish.max_items = 1u << 16;
            // a small request's items spread over the device (one per resident wave or
            // so) instead of a few waves each sweeping many prefixes
            ish.min_items = (uint32_t)std::max(0, S->cfg.min_items);
            // the items stay implicit (a large request has up to 2^16 of them, and
            // this runs on the submitting thread)
            r->per = item_prefixes(r->plan, ish);
            r->n_items = (uint32_t)((r->plan.n_prefix + r->per - 1) / r->per);
            if (r->n_items > 0) {
                r->cost_full = item_cost(r->plan, r->per);
                r->cost_last = item_cost(r->plan, r->plan.n_prefix - (uint64_t)(r->n_items - 1) * r->per);
                r->remaining = r->cost_full * (r->n_items - 1) + r->cost_last;
            }
        }
        if (align256(r->plan.blob.size()) > S->cfg.arena_bytes) r->plan.status = LD_ETOOBIG;
        r->lane = (S->cfg.express_ms > 0 && (r->is_sum || r->remaining < S->express_cost)) ? EXPRESS : BULK;
    }
    r->t_queued = now_s();
    ApiLock g(S);
    if (S->failed) {
        delete r;
        set_error(LD_EHIP);
        return LD_EHIP;
    }
    if (r->plan.status == LD_OK && r->plan.kind != PK_ZERO &&
        (int)(S->lanes[BULK].pending.size() + S->lanes[EXPRESS].pending.size()) >= S->cfg.max_queued) {
        delete r;
        S->st_rejected++;
        set_error(LD_EBUSY);
        return LD_EBUSY;
    }
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->all[r->ticket] = r;
    S->st_submitted++;
    if (r->plan.status != LD_OK) {
        const int st = r->plan.status;
        finish(S, r, st, INT64_MIN);
        set_error(st);
        return st;
    }
    if (r->plan.kind == PK_ZERO) {
        finish(S, r, LD_OK, 0);
        return LD_OK;
    }
    S->plan_sum_ms += 1e3 * (r->t_queued - r->t_submit);
    S->plan_n++;
    S->lanes[r->lane].pending.push_back(r);
    S->arrivals.fetch_add(1, std::memory_order_release);
    S->cv.notify_one();
    return LD_OK;
}

int ld_server_poll(ld_server* S, uint64_t ticket, int64_t* value)
{
    if (!S) return LD_EINVAL;
    ApiLock g(S);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return LD_ENOTFOUND;
    if (it->second->status == LD_PENDING) return LD_PENDING;
    if (value && it->second->status == LD_OK) *value = it->second->value;
    return it->second->status;
}

int ld_server_wait(ld_server* S, uint64_t ticket, int64_t* value)
{
    if (!S) return LD_EINVAL;
    ApiLock g(S);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return LD_ENOTFOUND;
    Request* r = it->second;
    S->done_cv.wait(g.lk, [&]() { return r->status != LD_PENDING; });
    if (value && r->status == LD_OK) *value = r->value;
    return r->status;
}

int ld_server_cancel(ld_server* S, uint64_t ticket)
{
    if (!S) return LD_EINVAL;
    ApiLock g(S);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return LD_ENOTFOUND;
    Request* r = it->second;
    if (r->status != LD_PENDING) return r->status;
    auto& pend = S->lanes[r->lane].pending;
    auto q = std::find(pend.begin(), pend.end(), r);
    if (q != pend.end()) {
        pend.erase(q);
        finish(S, r, LD_ECANCELED, INT64_MIN);
        return LD_OK;
    }
    // in flight: drop the items not yet issued; it completes when its issued
    // items have retired
    r->canceled = true;
    r->remaining = 0;
    r->next = r->n_items;
    if (r->outstanding == 0) {
        release_slot(S, r);
        finish(S, r, LD_ECANCELED, INT64_MIN);
    }
    return LD_OK;
}

void ld_server_stats(ld_server* S, ld_stats* out)
{
    if (!S || !out) return;
    ApiLock g(S);
    std::memset(out, 0, sizeof(*out));
    out->submitted = S->st_submitted;
    out->completed = S->st_completed;
    out->rejected = S->st_rejected;
    out->launches = S->st_launches;
    out->items = S->st_items;
    out->queued = (int32_t)(S->lanes[BULK].pending.size() + S->lanes[EXPRESS].pending.size());
    for (Request* r : S->slots)
        if (r) out->inflight++;
    if (!S->latencies_ms.empty()) {
        std::vector<double> v = S->latencies_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) { return v[std::min(v.size() - 1, (size_t)(q * (v.size() - 1) + 0.5))]; };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        double s = 0;
        for (double x : v) s += x;
        out->mean_ms = s / v.size();
    }
    if (S->wait_n) out->mean_wait_ms = S->wait_sum_ms / (double)S->wait_n;
    if (S->plan_n) out->mean_plan_ms = S->plan_sum_ms / (double)S->plan_n;
    if (S->run_n) out->mean_run_ms = S->run_sum_ms / (double)S->run_n;
}

int32_t ld_server_timings(ld_server* S, ld_request_timing* out, int32_t max)
{
    if (!S) return -1;
    ApiLock g(S);
    int32_t n = 0;
    for (const ld_request_timing& t : S->timings) {
        if (n >= max || !out) break;
        out[n++] = t;
    }
    return n;
}

void ld_server_destroy(ld_server* S)
{
    if (!S) return;
    {
        ApiLock g(S);
        // queued requests are cancelled; in-flight ones finish their issued items
        for (auto& ln : S->lanes)
            while (!ln.pending.empty()) {
                Request* r = ln.pending.front();
                ln.pending.pop_front();
                finish(S, r, LD_ECANCELED, INT64_MIN);
            }
        for (Request* r : S->slots) {
            if (!r) continue;
            r->canceled = true;
            r->next = r->n_items;
            r->remaining = 0;
            if (r->outstanding == 0) {   // admitted, nothing issued: done now
                release_slot(S, r);
                finish(S, r, LD_ECANCELED, INT64_MIN);
            }
        }
        S->stop = true;
        S->stopping.store(true, std::memory_order_release);
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (auto& ln : S->lanes)
        if (ln.stream) (void)hipStreamSynchronize(ln.stream);
    delete S;
}

}  // extern "C"
