// Long solves that survive interruption: the prefix space of the plain plan is
// swept in chunks, and after every chunk the best value so far and the next prefix
// are saved to a state file (written to a temporary file, then renamed over the
// old one, so a crash leaves either the old or the new state).  A later call with
// the same problem and the same plan continues from the saved prefix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>

#include "ld.h"
#include "ld_api_internal.h"
#include "ld_plan.h"
#include "ld_program.h"

namespace ld {

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// FNV-1a over the problem and the plan shape: prefixes mean something only for
// the plan they were numbered in
uint64_t fingerprint(const int32_t* M, int n, int m, int d, int marg, const Plan& p)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* data, size_t bytes) {
        const uint8_t* b = (const uint8_t*)data;
        for (size_t i = 0; i < bytes; ++i) h = (h ^ b[i]) * 1099511628211ull;
    };
    const int32_t head[11] = {n, m, d, marg, p.kind, p.mp, p.R, p.C, p.P, p.P_tab, p.i64};
    mix(head, sizeof head);
    mix(&p.n_prefix, 8);
    mix(M, 4 * (size_t)n * m);
    return h;
}

struct State {
    uint64_t fp = 0, next = 0, total = 0;
    int64_t best = INT64_MIN;
};

bool load_state(const char* path, State* s)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    unsigned long long fp = 0, next = 0, total = 0;
    long long best = 0;
    const int got = std::fscanf(f, "ld_norm_resumable 1\nfingerprint %llx\nnext %llu\ntotal %llu\nbest %lld\n", &fp,
                                &next, &total, &best);
    std::fclose(f);
    if (got != 4) return false;
    s->fp = fp;
    s->next = next;
    s->total = total;
    s->best = best;
    return true;
}

bool save_state(const char* path, const State& s)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    const bool ok = std::fprintf(f, "ld_norm_resumable 1\nfingerprint %016llx\nnext %llu\ntotal %llu\nbest %lld\n",
                                 (unsigned long long)s.fp, (unsigned long long)s.next, (unsigned long long)s.total,
                                 (long long)s.best) > 0;
    const bool closed = std::fclose(f) == 0;
    return ok && closed && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

}  // namespace ld

using namespace ld;

extern "C" int ld_norm_resumable(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals,
                                 const char* state_path, double chunk_seconds, double max_seconds, int64_t* value)
{
    if (!state_path || !*state_path || !value || !(chunk_seconds > 0) || !(max_seconds > 0)) {
        set_error(LD_EINVAL);
        return LD_EINVAL;
    }
    Plan p = make_plan(M, n, m, d, marginals, get_shape());
    if (p.status != LD_OK) {
        set_error(p.status);
        return p.status;
    }
    if (p.kind == PK_ZERO || p.kind == PK_SUMABS) {   // no search: one call
        const int64_t v = run_plan_sync(p);
        if (v == INT64_MIN) return ld_last_error();
        *value = v;
        return LD_OK;
    }
    State st;
    const uint64_t fp = fingerprint(M, n, m, d, marginals, p);
    if (!load_state(state_path, &st) || st.fp != fp || st.total != p.n_prefix || st.next > p.n_prefix) {
        st = State{};   // another problem, another plan, or no state yet: start over
        st.fp = fp;
        st.total = p.n_prefix;
    }
    const double t_end = now_s() + max_seconds;
    const double words_per_prefix = p.words / (double)p.n_prefix;
    uint64_t chunk = std::max<uint64_t>(1, p.n_prefix / 256);   // first chunk: a probe
    while (st.next < st.total) {
        const uint64_t cnt = std::min<uint64_t>(chunk, st.total - st.next);
        Plan c = p;
        c.pfx_base = st.next;
        c.n_prefix = cnt;
        c.words = words_per_prefix * (double)cnt;
        const double t0 = now_s();
        const int64_t v = run_plan_sync(c);
        if (v == INT64_MIN) return ld_last_error();
        const double dt = now_s() - t0;
        st.best = std::max(st.best, v);
        st.next += cnt;
        if (!save_state(state_path, st)) {
            set_error(LD_EINVAL);
            return LD_EINVAL;
        }
        // next chunk: about chunk_seconds of work at the rate just measured
        const double per = dt / (double)cnt;
        chunk = (uint64_t)std::max(1.0, std::min((double)p.n_prefix, chunk_seconds / std::max(per, 1e-12)));
        if (st.next < st.total && now_s() >= t_end) {
            set_error(LD_PENDING);
            return LD_PENDING;
        }
    }
    *value = st.best;
    return LD_OK;
}
