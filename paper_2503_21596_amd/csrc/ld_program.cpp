// Program builder and launcher (see ld_program.h).
#include "ld_program.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <atomic>
#include <mutex>
#include <utility>

#include "ld.h"
#include "ld_registry.h"

namespace ld {

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// descriptors and sum items as built: their pointers hold byte offsets into the
// image until patch_program rebases them on a device address
struct Rel {
    std::vector<Desc> descs;
    std::vector<SumItem> sums;
};

}  // namespace

// VALU work of one word, for ordering items longest first (the exact constant
// does not matter, only that it grows with the columns and the messages).
double word_cost(const Plan& p)
{
    // lane-level VALU instructions per word of the kernel the plan runs (measured
    // counts: 22.4 for the packed 42-column L1 sweep, 44.1 for the 32-bit one, 9.95
    // for the packed d = 3 sweep at 40 columns; the int64 and LDS kernels take about
    // three instructions per 32-bit one)
    const double W = p.pack16 ? p.mp / 2.0 : (double)p.mp;   // dwords per row
    const double R = (double)p.R;
    switch (p.kind) {
    case PK_L1:
    case PK_MARG:
    case PK_L2: {
        const double sides = p.kind == PK_L2 ? 2.0 : 1.0;
        if (p.i64 || p.wide) return 3.0 * (sides * p.m + 1.0);
        const double c = sides * W + W / std::ldexp(1.0, p.R) + 0.75;
        return p.mfma ? 1.12 * c : c;
    }
    case PK_LD: {
        if (p.i64 || p.wide) return 3.0 * (4.0 * p.m + p.d);
        const double blk = std::pow((double)p.d, R);            // words per state
        return (2.0 * std::ldexp(1.0, p.R) * W + blk * (p.d + 1.0)) / blk;
    }
    default: return 1.0;
    }
}

uint64_t item_prefixes(const Plan& p, const ItemShape& sh)
{
    const bool wide = p.wide != 0;
    const double wpp = p.words / (double)std::max<uint64_t>(p.n_prefix, 1);   // words per prefix
    uint64_t per;
    if (wide) {
        per = 1;
        if (sh.item_words > 0) per = (uint64_t)std::max(1.0, std::floor(sh.item_words / 64.0 / wpp));
    } else if (p.mfma) {
        per = 2;
        if (sh.item_words > 0) per = 2 * (uint64_t)std::max(1.0, std::floor(sh.item_words / wpp / 2));
    } else {
        per = sh.lanes_per_item;
        if (sh.item_words > 0) {
            const double want = std::floor(sh.item_words / wpp / sh.lanes_per_item);
            per = (uint64_t)sh.lanes_per_item * (uint64_t)std::max(1.0, want);
        }
    }
    if (sh.min_items > 0) {
        // at least min_items items when the problem has that many wave-sized pieces,
        // so that a small problem spreads over the device instead of a few waves
        const uint64_t unit = wide ? 1 : p.mfma ? 2 : sh.lanes_per_item;
        const uint64_t kmax = std::max<uint64_t>(1, p.n_prefix / (unit * sh.min_items));
        per = std::min<uint64_t>(per, unit * kmax);
    }
    per = std::max<uint64_t>(per, (p.n_prefix + sh.max_items - 1) / sh.max_items);
    return std::min<uint64_t>(per, 0xffffffffull);
}

double item_cost(const Plan& p, uint64_t count)
{
    const double wpp = p.words / (double)std::max<uint64_t>(p.n_prefix, 1);
    // a register-kernel wave covers 64 prefixes per round, each lane one word of
    // them per step; an MFMA-kernel wave covers two prefixes, 64 words per step
    const double rounds = p.wide ? (double)count : p.mfma ? std::ceil(count / 2.0) / 32.0 : std::ceil(count / 64.0);
    return rounds * wpp * word_cost(p);
}

void split_items(const Plan& p, uint32_t prob, const ItemShape& sh, std::vector<std::pair<double, Item>>& out)
{
    const uint64_t per = item_prefixes(p, sh);
    const double full = item_cost(p, per);
    if (out.empty()) out.reserve((size_t)((p.n_prefix + per - 1) / per));
    for (uint64_t p0 = 0; p0 < p.n_prefix; p0 += per) {
        Item it;
        it.prob = prob;
        it.count = (uint32_t)std::min<uint64_t>(per, p.n_prefix - p0);
        it.p0 = p0;
        out.push_back({it.count == per ? full : item_cost(p, it.count), it});
    }
}

Program build_program(const std::vector<const Plan*>& plans, const ItemShape& sh)
{
    Program P;
    const uint32_t n = (uint32_t)plans.size();
    P.n_probs = n;
    P.blob_off.assign(n, 0);
    size_t off = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const Plan& p = *plans[i];
        if (p.kind == PK_ZERO) {
            P.zero.push_back((int)i);
            continue;
        }
        P.blob_off[i] = off;
        off = align256(off + p.blob.size());
    }
    P.off_descs = off;
    off = align256(off + (size_t)n * sizeof(Desc));

    // group the problems by sweep kernel; the sum-|M| problems go to one launch
    std::map<std::pair<const void*, size_t>, std::vector<uint32_t>> groups;
    std::vector<uint32_t> sums;
    for (uint32_t i = 0; i < n; ++i) {
        const Plan& p = *plans[i];
        if (p.kind == PK_ZERO) continue;
        if (p.kind == PK_SUMABS) {
            sums.push_back(i);
            continue;
        }
        groups[{p.kernel, p.wide ? (size_t)1 : (size_t)0}].push_back(i);
    }

    // items: per problem, ranges of prefixes; per group, longest first
    std::vector<std::pair<Launch, std::vector<Item>>> launches;
    uint32_t heads = 0;
    for (auto& g : groups) {
        Launch L;
        L.kernel = g.first.first;
        if (g.second.size() == 1 && n == 1) {
            // a single problem: equal items, computed on the device from their index
            const Plan& p = *plans[g.second[0]];
            L.threads = g.first.second != 0 ? 64 : 256;
            L.lds = p.lds;
            L.implicit = true;
            L.prob = g.second[0];
            // items of about item_words words (one lane per prefix), but at least
            // min_items of them when the problem has that many lane-sized pieces
            const double wpp = p.words / (double)std::max<uint64_t>(p.n_prefix, 1);
            const uint64_t lanes = wave_prefixes(p, sh.lanes_per_item);
            uint64_t k = 1;
            if (sh.item_words > 0) k = (uint64_t)std::max(1.0, std::floor(sh.item_words / (wpp * lanes)));
            const uint64_t kmax = std::max<uint64_t>(1, p.n_prefix / (lanes * std::max<uint32_t>(sh.min_items, 1)));
            uint64_t per = lanes * std::min(k, kmax);
            per = std::max<uint64_t>(per, (p.n_prefix + sh.max_items - 1) / sh.max_items);
            L.per = per;
            L.n_prefix = p.n_prefix;
            L.n_items = (uint32_t)((p.n_prefix + per - 1) / per);
            L.head = heads++;
            L.cost = p.words * word_cost(p);
            launches.push_back({L, {}});
            continue;
        }
        L.threads = g.first.second != 0 ? 64 : 256;
        ItemShape gsh = sh;
        if (sh.max_launch_items > 0 && sh.item_words > 0) {
            double words = 0;
            for (uint32_t i : g.second) words += (double)plans[i]->words;
            gsh.item_words = std::max(sh.item_words, words / sh.max_launch_items);
        }
        std::vector<std::pair<double, Item>> its;
        for (uint32_t i : g.second) {
            L.lds = std::max(L.lds, plans[i]->lds);
            split_items(*plans[i], i, gsh, its);
        }
        std::stable_sort(its.begin(), its.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
        std::vector<Item> items;
        items.reserve(its.size());
        for (auto& c : its) {
            L.cost += c.first;
            items.push_back(c.second);
        }
        L.n_items = (uint32_t)items.size();
        L.head = heads++;
        launches.push_back({L, std::move(items)});
    }
    std::stable_sort(launches.begin(), launches.end(),
                     [](const auto& a, const auto& b) { return a.first.cost > b.first.cost; });

    P.off_items = off;
    size_t ioff = 0;
    for (auto& l : launches) {
        l.first.off_items = P.off_items + ioff;
        ioff += l.second.size() * sizeof(Item);
    }
    off = align256(off + ioff);
    P.n_heads = heads;
    P.off_heads = off;
    off = align256(off + 4 * (size_t)std::max<uint32_t>(heads, 1));
    P.off_results = off;
    off = align256(off + 8 * (size_t)std::max<uint32_t>(n, 1));
    P.n_sums = (uint32_t)sums.size();
    P.off_sums = off;
    off = align256(off + sizeof(SumItem) * (size_t)std::max<uint32_t>(P.n_sums, 1));
    P.rec_off.assign(n, 0);
    for (uint32_t i = 0; i < n; ++i)
        if (plans[i]->record && plans[i]->kernel && plans[i]->kind != PK_ZERO) {
            P.rec_off[i] = off;
            off = align256(off + 8 * (size_t)plans[i]->n_prefix);
        }

    P.image.assign(off, 0);
    Rel rel;
    rel.descs.resize(n);
    for (uint32_t i = 0; i < n; ++i) {
        const Plan& p = *plans[i];
        if (p.kind == PK_ZERO) continue;
        std::memcpy(P.image.data() + P.blob_off[i], p.blob.data(), p.blob.size());
        // pointers as byte offsets into the image (rebased by patch_program)
        Desc D = make_desc(p, (const void*)(uintptr_t)P.blob_off[i],
                           (int64_t*)(uintptr_t)(P.off_results + 8 * (size_t)i));
        D.rec = (int64_t*)(uintptr_t)P.rec_off[i];
        rel.descs[i] = D;
    }
    for (auto& l : launches) {
        std::memcpy(P.image.data() + l.first.off_items, l.second.data(), l.second.size() * sizeof(Item));
        P.launches.push_back(l.first);
    }
    for (uint32_t i = 0; i < n; ++i) {
        const int64_t v = INT64_MIN;
        std::memcpy(P.image.data() + P.off_results + 8 * (size_t)i, &v, 8);
    }
    for (uint32_t j = 0; j < P.n_sums; ++j) {
        const uint32_t i = sums[j];
        SumItem si;
        si.M = (const int32_t*)(uintptr_t)P.blob_off[i];
        si.count = (int64_t)plans[i]->n * plans[i]->m;
        si.result = (int64_t*)(uintptr_t)(P.off_results + 8 * (size_t)i);
        rel.sums.push_back(si);
    }
    // relative descriptors are kept with the image bytes themselves: patching
    // adds the device base to the stored offsets
    for (uint32_t i = 0; i < n; ++i)
        std::memcpy(P.image.data() + P.off_descs + i * sizeof(Desc), &rel.descs[i], sizeof(Desc));
    for (uint32_t j = 0; j < P.n_sums; ++j)
        std::memcpy(P.image.data() + P.off_sums + j * sizeof(SumItem), &rel.sums[j], sizeof(SumItem));
    return P;
}

void patch_program(Program& P, void* dev)
{
    const uintptr_t old = (uintptr_t)P.dev;
    const uintptr_t nb = (uintptr_t)dev;
    auto fix = [&](auto& ptr) { ptr = (std::remove_reference_t<decltype(ptr)>)((uintptr_t)ptr - old + nb); };
    for (uint32_t i = 0; i < P.n_probs; ++i) {
        Desc D;
        std::memcpy(&D, P.image.data() + P.off_descs + i * sizeof(Desc), sizeof(Desc));
        if (D.result) {   // unused slots (problems with value 0) stay all-zero
            fix(D.base);
            fix(D.hid);
            fix(D.mid);
            fix(D.offs);
            fix(D.tab);
            fix(D.result);
            if (D.rec) fix(D.rec);
        }
        std::memcpy(P.image.data() + P.off_descs + i * sizeof(Desc), &D, sizeof(Desc));
    }
    for (uint32_t j = 0; j < P.n_sums; ++j) {
        SumItem si;
        std::memcpy(&si, P.image.data() + P.off_sums + j * sizeof(SumItem), sizeof(SumItem));
        fix(si.M);
        fix(si.result);
        std::memcpy(P.image.data() + P.off_sums + j * sizeof(SumItem), &si, sizeof(SumItem));
    }
    P.dev = dev;
}

namespace {
std::atomic<int> g_launch_waves{0};   // waves per SIMD of plain and batch launches; 0: occupancy
}  // namespace

void set_launch_waves(int waves_per_simd) { g_launch_waves.store(std::max(0, waves_per_simd)); }

uint32_t capped_blocks(const void* kernel, uint32_t threads, size_t lds)
{
    const uint32_t full = resident_blocks(kernel, threads, lds);
    const int w = g_launch_waves.load();
    if (w <= 0) return full;
    // blocks of threads / 64 waves; four SIMDs per CU
    const uint32_t cus = std::max<uint32_t>(1, device_cus());
    const uint32_t cap = std::max<uint32_t>(1, (uint32_t)w * 4 * cus / std::max<uint32_t>(1, threads / 64));
    return std::min(full, cap);
}

uint32_t device_cus()
{
    static std::atomic<uint32_t> cus{0};
    uint32_t c = cus.load();
    if (c) return c;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        c = (uint32_t)prop.multiProcessorCount;
    cus.store(c);
    return c;
}

uint32_t resident_blocks(const void* kernel, uint32_t threads, size_t lds)
{
    static std::mutex mu;
    static std::map<std::pair<const void*, size_t>, uint32_t> cache;
    std::lock_guard<std::mutex> g(mu);
    auto key = std::make_pair(kernel, lds);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    uint32_t blocks = 1024;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, (int)threads, lds) == hipSuccess &&
        per_cu > 0)
        blocks = (uint32_t)per_cu * (uint32_t)prop.multiProcessorCount;
    cache[key] = blocks;
    return blocks;
}

bool enqueue_program(const Program& P, hipStream_t s, int64_t* host_results)
{
    return enqueue_program_fanned(P, s, host_results, {}, {});
}

bool enqueue_program_fanned(const Program& P, hipStream_t s, int64_t* host_results,
                            const std::vector<hipStream_t>& side, const std::vector<hipEvent_t>& evs)
{
    uint8_t* dev = (uint8_t*)P.dev;
    int64_t* results = (int64_t*)(dev + P.off_results);
    uint32_t* heads = (uint32_t*)(dev + P.off_heads);
    uint32_t nr = P.n_probs, nh = P.n_heads;
    {
        const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(64, (std::max(nr, nh) + 255) / 256));
        void* args[] = {(void*)&results, (void*)&nr, (void*)&heads, (void*)&nh};
        if (hipLaunchKernel(kernel_reset(), dim3(blocks), dim3(256), args, 0, s) != hipSuccess) return false;
    }
    // Fan the launches out over the side streams: each waits for the reset, takes
    // launches greedily by estimated work (most work first), and the main stream
    // waits for all of them before the result copy.  Launches of different kernel
    // shapes share no queue head and no problem, so they may overlap; one that
    // drains its queue leaves its CUs to the others instead of to nothing.
    const bool fan = !side.empty() && evs.size() >= side.size() + 1 && P.launches.size() > 1;
    std::vector<hipStream_t> lanes{s};
    if (fan) {
        if (hipEventRecord(evs[0], s) != hipSuccess) return false;
        for (size_t k = 0; k < side.size(); ++k) {
            if (hipStreamWaitEvent(side[k], evs[0], 0) != hipSuccess) return false;
            lanes.push_back(side[k]);
        }
    }
    std::vector<double> load(lanes.size(), 0.0);
    for (const Launch& L : P.launches) {
        const size_t li = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
        load[li] += L.cost;
        hipStream_t ls = lanes[li];
        QArgs q{};
        q.descs = (const Desc*)(dev + P.off_descs);
        q.items = L.implicit ? nullptr : (const Item*)(dev + L.off_items);
        q.n_items = L.n_items;
        q.head = heads + L.head;
        q.prob = L.prob;
        q.per = L.per;
        q.n_prefix = L.n_prefix;
        const uint32_t waves_per_block = L.threads / 64;
        const uint32_t want = (L.n_items + waves_per_block - 1) / waves_per_block;
        const uint32_t blocks = std::max<uint32_t>(1, std::min(want, capped_blocks(L.kernel, L.threads, L.lds)));
        void* args[] = {(void*)&q};
        if (hipLaunchKernel(L.kernel, dim3(blocks), dim3(L.threads), args, L.lds, ls) != hipSuccess) return false;
    }
    if (fan)
        for (size_t k = 0; k < side.size(); ++k) {
            if (hipEventRecord(evs[k + 1], side[k]) != hipSuccess) return false;
            if (hipStreamWaitEvent(s, evs[k + 1], 0) != hipSuccess) return false;
        }
    if (P.n_sums) {
        const SumItem* items = (const SumItem*)(dev + P.off_sums);
        uint32_t ns = P.n_sums;
        void* args[] = {(void*)&items, (void*)&ns};
        const uint32_t blocks = std::min<uint32_t>(ns, 1024);
        if (hipLaunchKernel(kernel_sumabs_many(), dim3(blocks), dim3(256), args, 0, s) != hipSuccess) return false;
    }
    if (host_results && nr)
        if (hipMemcpyAsync(host_results, results, 8 * (size_t)nr, hipMemcpyDeviceToHost, s) != hipSuccess)
            return false;
    return true;
}

}  // namespace ld
