// Autotuner: picks the sweep and queue shapes by timing candidates on a small
// calibration set on the device at hand, then applies them to every later plan.
// The paper found no general rule for its launch shapes and recommends timing a
// smaller matrix first and reusing the result for larger ones (Sec. 4); this is
// that procedure, automated.
#include "ld_tune.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ld.h"
#include "ld_api_internal.h"
#include "ld_registry.h"

namespace ld {

namespace {

std::mutex g_mu;
Tuning g_tuning;

// SplitMix64, for the calibration matrices only
struct Rng {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    int uniform(int lo, int hi) { return lo + (int)(next() % (uint64_t)(hi - lo + 1)); }
};

struct Cal {
    std::vector<std::vector<int32_t>> mats;
    std::vector<ld_problem> probs;
};

// a mixed set with the size law of the batch workload (n in [12, 28], m in
// [8, 40], d in {1, 2, 3} with n <= 20 for d = 3, a fifth with marginals), fewer
// problems so that one candidate times in tens of milliseconds
Cal calibration_batch(int count, uint64_t seed)
{
    Cal c;
    Rng r{seed};
    c.mats.resize(count);
    for (int i = 0; i < count; ++i) {
        int d = r.uniform(1, 3);
        const int marg = r.uniform(0, 4) == 0 ? 1 : 0;
        if (marg) d = 1;
        const int n = d == 3 ? r.uniform(12, 20) : r.uniform(12, 28);
        const int m = r.uniform(8, 40);
        auto& M = c.mats[i];
        M.resize((size_t)n * m);
        for (auto& v : M) v = r.uniform(-1000, 1000);
        c.probs.push_back({M.data(), n, m, d, marg});
    }
    return c;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// best-of-three wall time of one batch with the current tuning
double time_batch(const Cal& c)
{
    std::vector<int64_t> out(c.probs.size());
    double best = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
        const double t0 = now_s();
        if (ld_norm_batch(c.probs.data(), (int32_t)c.probs.size(), out.data(), nullptr, nullptr) != LD_OK) return 1e30;
        best = std::min(best, now_s() - t0);
    }
    return best;
}

double time_plain(const std::vector<int32_t>& M, int n, int m, int d = 1)
{
    double best = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
        const double t0 = now_s();
        if (ld_norm(M.data(), n, m, d, 0) == INT64_MIN) return 1e30;
        best = std::min(best, now_s() - t0);
    }
    return best;
}

const char* const CLASS_NAME[4] = {"l1", "l2", "d3", "d4"};

bool write_tuning(const char* path, const Tuning& t, const std::string& notes)
{
    FILE* f = std::fopen(path, "w");
    if (!f) return false;
    std::fprintf(f, "{\n");
    for (int c = 0; c < 4; ++c)
        for (int b = 0; b < 4; ++b)
            std::fprintf(f, "  \"variant_%s_%d\": %d,\n", CLASS_NAME[c], b, t.variant[c][b]);
    std::fprintf(f,
                 "  \"bin_c_target\": %d,\n  \"dary_cwords\": %d,\n  \"item_words\": %.0f,\n"
                 "  \"batch_pfx_cap\": %d,\n  \"plain_p_target\": %d,\n  \"plain_c_goal\": %d,\n"
                 "  \"plain_r_drop\": %d,\n  \"sgpr_r\": %d,\n  \"dary_variant\": %d,\n"
                 "  \"plain_p_min\": %d,\n  \"plain_dary_lanes\": %d,\n  \"plain_big_r_c\": %d,\n"
                 "  \"batch_side_streams\": %d,\n  \"measured\": [%s]\n}\n",
                 t.bin_c_target, t.dary_cwords, t.item_words, t.batch_pfx_cap, t.plain_p_target, t.plain_c_goal,
                 t.plain_r_drop, t.sgpr_r, t.dary_variant, t.plain_p_min, t.plain_dary_lanes, t.plain_big_r_c,
                 t.batch_side_streams, notes.c_str());
    std::fclose(f);
    return true;
}

bool read_key(const std::string& text, const char* key, double* v)
{
    const std::string k = std::string("\"") + key + "\"";
    const size_t at = text.find(k);
    if (at == std::string::npos) return false;
    const size_t colon = text.find(':', at + k.size());
    if (colon == std::string::npos) return false;
    return std::sscanf(text.c_str() + colon + 1, "%lf", v) == 1;
}

}  // namespace

Tuning get_tuning()
{
    std::lock_guard<std::mutex> g(g_mu);
    return g_tuning;
}

void set_tuning(const Tuning& t)
{
    {
        std::lock_guard<std::mutex> g(g_mu);
        g_tuning = t;
    }
    SweepShape s = get_shape();
    s.p_target = t.plain_p_target;
    s.p_min = std::min(t.plain_p_min, t.plain_p_target);
    s.c_goal = t.plain_c_goal;
    s.r_drop = t.plain_r_drop;
    s.sgpr_r = t.sgpr_r;
    s.dary_sgpr = t.dary_variant;
    s.dary_lanes = t.plain_dary_lanes;
    s.big_r_c = t.plain_big_r_c;
    std::memcpy(s.variant, t.variant, sizeof s.variant);
    set_shape(s);
}

SweepShape batch_shape_for(int n, int m, int d)
{
    (void)n;
    (void)m;
    const Tuning t = get_tuning();
    SweepShape s = get_shape();
    s.c_target = t.bin_c_target;
    s.dary_cwords = t.dary_cwords;
    s.dary_lanes = 0;   // many problems share the device: keep the tuned words per lane
    s.pfx_cap = t.batch_pfx_cap;
    (void)d;
    return s;
}

int batch_side_streams() { return std::max(0, std::min(7, get_tuning().batch_side_streams)); }

ItemShape batch_item_shape()
{
    ItemShape s;
    s.lanes_per_item = 64;
    s.item_words = get_tuning().item_words;
    s.max_items = 4096;   // per problem: large problems get larger items
    return s;
}

}  // namespace ld

using namespace ld;

extern "C" {

int ld_autotune(const char* path, double budget_seconds)
{
    if (!device_ok(nullptr)) {
        set_error(LD_EHIP);
        return LD_EHIP;
    }
    const double t_end = now_s() + std::max(1.0, budget_seconds);
    const Tuning start = get_tuning();
    Tuning best = start;
    std::string notes;
    char buf[160];

    // batch shape: words per prefix (binary and d-ary), prefixes per problem and
    // words per queue item
    const Cal cal = calibration_batch(1024, 0x5eed);
    double best_t = 1e30;
    for (int c : {8, 10, 12})
        for (int cap : {0, 16})
            for (double w : {65536.0, 262144.0}) {
                if (now_s() > t_end) break;
                Tuning t = best;
                t.bin_c_target = c;
                t.dary_cwords = c <= 8 ? 729 : c <= 10 ? 2187 : 6561;
                t.batch_pfx_cap = cap;
                t.item_words = w;
                set_tuning(t);
                const double dt = time_batch(cal);
                std::snprintf(buf, sizeof buf,
                              "%s{\"batch_c\": %d, \"pfx_cap\": %d, \"item_words\": %.0f, \"ms\": %.3f}",
                              notes.empty() ? "" : ", ", c, cap, w, 1e3 * dt);
                notes += buf;
                if (dt < best_t) {
                    best_t = dt;
                    best = t;
                }
            }
    set_tuning(best);

    // batch launches fanned out over side streams (the launches of different kernel
    // shapes overlap, so one that drains its queue leaves its CUs to the others)
    for (int k : {0, 1, 3}) {
        if (now_s() > t_end) break;
        Tuning t = best;
        t.batch_side_streams = k;
        set_tuning(t);
        const double dt = time_batch(cal);
        std::snprintf(buf, sizeof buf, ", {\"batch_side_streams\": %d, \"ms\": %.3f}", k, 1e3 * dt);
        notes += buf;
        if (dt < best_t) {
            best_t = dt;
            best = t;
        }
    }
    set_tuning(best);

    // plain calls: kernel variant (low rows of the SGPR-operand kernel, or the
    // VGPR-operand kernel), lane range and words per prefix, timed on a 40 x 40
    // and a 35 x 42 L1 problem and a 31 x 31 L2 problem.  The first has rows
    // enough that the upper lane bound decides its shape, and few enough queue
    // items per wave at the lower bounds that the end of the launch shows, as it
    // does for larger problems (a 38 x 38 problem preferred 2^20 lanes, which cost
    // a 42 x 42 one 3.5 %); in the last the least lane count binds (with too few
    // lanes it runs at half speed, which the two large ones cannot show).  Each
    // time counts relative to the same problem under the starting table, so the
    // millisecond problem weighs as much as the large ones.
    {
        Rng r{0xca1};
        std::vector<int32_t> A((size_t)40 * 40), B((size_t)35 * 42), C((size_t)31 * 31);
        for (auto& v : A) v = r.uniform(-100, 100);
        for (auto& v : B) v = r.uniform(-100, 100);
        for (auto& v : C) v = r.uniform(-100, 100);
        set_tuning(best);
        const double ra = time_plain(A, 40, 40), rb = time_plain(B, 35, 42), rc = time_plain(C, 31, 31, 2);
        double bt = 1e30;
        Tuning bp = best;
        for (int sr : {VARIANT_PACK16, 5, 4, 0})
            for (int pm : {16, 18, 19})
                for (int p : {20, 22})
                    for (int c : {12, 14}) {
                        if (now_s() > t_end) break;
                        Tuning t = best;
                        t.sgpr_r = sr;
                        t.plain_p_min = pm;
                        t.plain_p_target = p;
                        t.plain_c_goal = c;
                        set_tuning(t);
                        const double ta = time_plain(A, 40, 40), tb = time_plain(B, 35, 42),
                                     tc = time_plain(C, 31, 31, 2);
                        const double dt = ta / ra + tb / rb + tc / rc;
                        std::snprintf(buf, sizeof buf,
                                      ", {\"sgpr_r\": %d, \"p_min\": %d, \"plain_p\": %d, \"c_goal\": %d, \"ms\": [%.3f, "
                                      "%.3f, %.3f], \"score\": %.4f}",
                                      sr, pm, p, c, 1e3 * ta, 1e3 * tb, 1e3 * tc, dt);
                        notes += buf;
                        if (dt < bt) {
                            bt = dt;
                            bp = t;
                        }
                    }
        best = bp;
    }
    set_tuning(best);

    // plain calls, d >= 3: lane count, timed on an L_3 problem of 24 x 32 and an
    // L_4 problem of 20 x 24 (sum of the two times; both large enough that their
    // plans can trade mid rows up to the largest candidate, where the end of the
    // launch, a fraction of one item per wave, stops mattering)
    {
        Rng r{0xd3a};
        std::vector<int32_t> A((size_t)24 * 32), B((size_t)20 * 24);
        for (auto& v : A) v = r.uniform(-100, 100);
        for (auto& v : B) v = r.uniform(-100, 100);
        double bt = 1e30;
        Tuning bp = best;
        for (int lanes : {1 << 18, 1 << 19, 1 << 20, 1 << 21}) {
            if (now_s() > t_end) break;
            Tuning t = best;
            t.plain_dary_lanes = lanes;
            set_tuning(t);
            const double dt = time_plain(A, 24, 32, 3) + time_plain(B, 20, 24, 4);
            std::snprintf(buf, sizeof buf, ", {\"dary_lanes\": %d, \"ms\": %.3f}", lanes, 1e3 * dt);
            notes += buf;
            if (dt < bt) {
                bt = dt;
                bp = t;
            }
        }
        best = bp;
    }
    set_tuning(best);

    // kernel variant per kind class and width bucket (binary: packed 16-bit kernel,
    // SGPR-operand kernel with 5 or 4 low rows, VGPR-operand kernel, int8-MFMA
    // kernel; d-ary: packed 16-bit, SGPR- or VGPR-operand kernel), timed on one
    // problem each of
    // a few milliseconds (L1 with 33 rows, L2 with 32, L_3 with 22, L_4 with 19;
    // width 16b + 14, or square for the narrowest L1 bucket so that the planner
    // does not transpose it)
    {
        Rng r{0x7a2};
        const int rows[4] = {33, 32, 22, 19};
        const int dval[4] = {1, 2, 3, 4};
        for (int c = 0; c < 4 && now_s() < t_end; ++c)
            for (int b = 0; b < 4 && now_s() < t_end; ++b) {
                const int m = 16 * b + 14;
                const int n = (c == 0) ? std::min(rows[c], m) : rows[c];
                std::vector<int32_t> M((size_t)n * m);
                for (auto& x : M) x = r.uniform(-100, 100);
                std::vector<int> options =
                    c < 2 ? std::vector<int>{VARIANT_PACK16, 5, 4, 0, VARIANT_MFMA}
                          : std::vector<int>{VARIANT_PACK16, 1, 0};
                double bt = 1e30, t_default = 1e30;
                int pick = -1;
                std::vector<std::pair<const void*, double>> timed;   // kernel the option plans, its time
                for (int o : options) {
                    Tuning t = best;
                    t.variant[c][b] = o;
                    set_tuning(t);
                    // an option whose plan runs a kernel already timed (it does not fit
                    // this width, say) takes that time instead of another run
                    const void* k = make_plan(M.data(), n, m, dval[c], 0, get_shape()).kernel;
                    double dt = 1e30;
                    bool seen = false;
                    for (auto& kt : timed)
                        if (kt.first == k) {
                            dt = kt.second;
                            seen = true;
                        }
                    for (int rep = 0; rep < 3 && !seen; ++rep) {
                        const double t0 = now_s();
                        if (ld_norm(M.data(), n, m, dval[c], 0) == INT64_MIN) {
                            dt = 1e30;
                            break;
                        }
                        dt = std::min(dt, now_s() - t0);
                    }
                    if (!seen) timed.push_back({k, dt});
                    std::snprintf(buf, sizeof buf, ", {\"class\": \"%s\", \"bucket\": %d, \"variant\": %d, \"ms\": %.4f}",
                                  CLASS_NAME[c], b, o, 1e3 * dt);
                    notes += buf;
                    if (o == options[0]) t_default = dt;
                    if (dt < bt) {
                        bt = dt;
                        pick = o;
                    }
                }
                // the default (packed) kernel stays unless another is clearly faster:
                // ties of a few per cent are noise, not a reason to switch kernels
                best.variant[c][b] = bt < 0.97 * t_default ? pick : options[0];
            }
    }
    set_tuning(best);
    if (path && *path && !write_tuning(path, best, notes)) {
        set_error(LD_EINVAL);
        return LD_EINVAL;
    }
    return LD_OK;
}

int ld_load_tuning(const char* path)
{
    FILE* f = path ? std::fopen(path, "r") : nullptr;
    if (!f) {
        set_error(LD_EINVAL);
        return LD_EINVAL;
    }
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
    std::fclose(f);
    Tuning t = get_tuning();
    double v;
    if (read_key(text, "bin_c_target", &v)) t.bin_c_target = std::max(0, std::min(40, (int)v));
    if (read_key(text, "dary_cwords", &v)) t.dary_cwords = std::max(1, (int)v);
    if (read_key(text, "item_words", &v)) t.item_words = std::max(1.0, v);
    if (read_key(text, "batch_pfx_cap", &v)) t.batch_pfx_cap = std::max(0, std::min(40, (int)v));
    if (read_key(text, "plain_p_target", &v)) t.plain_p_target = std::max(0, std::min(40, (int)v));
    if (read_key(text, "plain_p_min", &v)) t.plain_p_min = std::max(0, std::min(40, (int)v));
    if (read_key(text, "plain_c_goal", &v)) t.plain_c_goal = std::max(0, std::min(40, (int)v));
    if (read_key(text, "plain_r_drop", &v)) t.plain_r_drop = v != 0;
    if (read_key(text, "sgpr_r", &v))
        t.sgpr_r = (v == 4 || v == 5 || v == VARIANT_MFMA || v == VARIANT_PACK16) ? (int)v : 0;
    if (read_key(text, "dary_variant", &v))
        t.dary_variant = v == VARIANT_PACK16 ? VARIANT_PACK16 : v != 0 ? 1 : 0;
    if (read_key(text, "batch_side_streams", &v)) t.batch_side_streams = std::max(0, std::min(7, (int)v));
    if (read_key(text, "plain_dary_lanes", &v)) t.plain_dary_lanes = (int)std::max(0.0, std::min(v, 1073741824.0));
    if (read_key(text, "plain_big_r_c", &v)) t.plain_big_r_c = (int)std::max(0.0, std::min(v, 31.0));
    for (int c = 0; c < 4; ++c)
        for (int b = 0; b < 4; ++b) {
            char key[32];
            std::snprintf(key, sizeof key, "variant_%s_%d", CLASS_NAME[c], b);
            if (read_key(text, key, &v)) t.variant[c][b] = (int)v;
        }
    set_tuning(t);
    return LD_OK;
}

}  // extern "C"
