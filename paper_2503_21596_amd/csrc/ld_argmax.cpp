// A maximising assignment (the strategy) together with the value.
//
// The value pass is the ordinary sweep with one extra store per prefix: the best
// score of every prefix (lane sub-cube).  The first prefix whose best equals the
// value is found on the device; its rows are then fixed and the rest of the rows
// are resolved by prefix-range sweeps that each fix up to 12 more rows (again the
// first sub-range reaching the value wins), until every row is fixed.  The sweep
// loops themselves are unchanged, and the refinement sweeps cover one lane's
// sub-cube, so the cost over the value pass is small.
//
// The planner may drop zero rows and columns and transpose L1 / L_marg problems
// (Sec. 2.2: both values are transpose invariant); the assignment is mapped back
// to the caller's rows, and for d = 1 the other side (the column signs of the
// bilinear form a^T M b, or the row signs when the planner transposed) is
// computed on the device as the sign of the matching matrix-vector product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ld.h"
#include "ld_api_internal.h"
#include "ld_plan.h"
#include "ld_program.h"
#include "ld_registry.h"

namespace ld {

namespace {

struct Session {
    hipStream_t s = nullptr;
    std::vector<void*> dev;
    std::vector<void*> host;
    ~Session()
    {
        // errors while releasing cannot be reported
        if (s) (void)hipStreamSynchronize(s);
        for (void* p : dev) (void)hipFree(p);
        for (void* p : host) (void)hipHostFree(p);
        if (s) (void)hipStreamDestroy(s);
    }
    void* dalloc(size_t bytes)
    {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) return nullptr;
        dev.push_back(p);
        return p;
    }
    void* halloc(size_t bytes)
    {
        void* p = nullptr;
        if (hipHostMalloc(&p, std::max<size_t>(bytes, 64), hipHostMallocDefault) != hipSuccess) return nullptr;
        host.push_back(p);
        return p;
    }
};

// One recorded sweep of plan p: its value and the first prefix (relative to the
// plan's range) whose best equals `target`, or the value itself when target is
// INT64_MIN.  Returns false on a device error.
bool sweep_locate(Session& S, Plan p, int64_t target, int64_t* value, uint64_t* first)
{
    p.record = 1;
    Program P = build_program({&p}, plain_item_shape());
    uint8_t* dev = (uint8_t*)S.dalloc(P.image.size() + 256);
    int64_t* hv = (int64_t*)S.halloc(64);
    if (!dev || !hv) return false;
    patch_program(P, dev);
    unsigned long long* dfirst = (unsigned long long*)(dev + P.image.size());
    bool ok = hipMemcpyAsync(dev, P.image.data(), P.image.size(), hipMemcpyHostToDevice, S.s) == hipSuccess;
    ok = ok && enqueue_program(P, S.s, nullptr);
    ok = ok && hipMemcpyAsync(hv, dev + P.off_results, 8, hipMemcpyDeviceToHost, S.s) == hipSuccess;
    ok = ok && hipStreamSynchronize(S.s) == hipSuccess;
    if (!ok) return false;
    *value = hv[0];
    const int64_t want = target == INT64_MIN ? hv[0] : target;
    const int64_t* rec = (const int64_t*)(dev + P.rec_off[0]);
    uint64_t n = p.n_prefix;
    unsigned long long init = ~0ull;
    {
        void* args[] = {(void*)&dfirst, (void*)&init};
        ok = hipLaunchKernel(kernel_set_u64(), dim3(1), dim3(64), args, 0, S.s) == hipSuccess;
    }
    {
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(1024, (n + 255) / 256);
        int64_t t = want;
        void* args[] = {(void*)&rec, (void*)&n, (void*)&t, (void*)&dfirst};
        ok = ok && hipLaunchKernel(kernel_first_equal(), dim3(std::max<uint32_t>(blocks, 1)), dim3(256), args, 0,
                                   S.s) == hipSuccess;
    }
    ok = ok && hipMemcpyAsync(hv + 1, dfirst, 8, hipMemcpyDeviceToHost, S.s) == hipSuccess;
    ok = ok && hipStreamSynchronize(S.s) == hipSuccess;
    if (!ok) return false;
    *first = (uint64_t)hv[1];
    return true;
}

uint64_t ipow(uint64_t b, int e)
{
    uint64_t r = 1;
    while (e-- > 0) r *= b;
    return r;
}

// Resolve the rows of B (n x m, row 0 fixed) that the prefix-range plans leave
// free: on entry the last q rows are fixed by prefix `pfx` (digit h <-> row
// n - q + h, base `radix`); on return q = n - 1 and pfx holds every row.
int refine(Session& S, const std::vector<int32_t>& B, int n, int m, int d, int marg, int64_t value, int& q,
           uint64_t& pfx)
{
    const int radix = d == 1 ? 2 : d;
    int kmax = 0;
    while (ipow(radix, kmax + 1) <= 4096) ++kmax;
    while (q < n - 1) {
        const int k = std::min(kmax, n - 1 - q);
        const uint64_t span = ipow(radix, k);
        Plan r = make_range_plan(B.data(), n, m, d, marg, q + k, pfx * span, (pfx + 1) * span);
        if (r.status != LD_OK) return r.status;
        int64_t v = 0;
        uint64_t f = 0;
        if (!sweep_locate(S, r, value, &v, &f)) return LD_EHIP;
        if (v != value || f >= span) return LD_EHIP;   // the range must reach the value
        pfx = pfx * span + f;
        q += k;
    }
    return LD_OK;
}

}  // namespace

}  // namespace ld

using namespace ld;

extern "C" int ld_argmax(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals, int64_t* value,
                         int32_t* assignment, int32_t* col_assignment)
{
    if (!value || !assignment) {
        set_error(LD_EINVAL);
        return LD_EINVAL;
    }
    Plan p = make_plan(M, n, m, d, marginals, get_shape());
    if (p.status != LD_OK) {
        set_error(p.status);
        return p.status;
    }
    const bool binary = d == 1;
    // default for rows the planner dropped (all zero): any choice attains the value
    for (int x = 0; x < n; ++x) assignment[x] = binary ? 1 : 0;
    if (binary && col_assignment)
        for (int y = 0; y < m; ++y) col_assignment[y] = 1;
    if (p.kind == PK_ZERO) {
        *value = 0;
        return LD_OK;
    }
    if (!device_ok(nullptr)) {
        set_error(LD_EHIP);
        return LD_EHIP;
    }
    Session S;
    if (hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking) != hipSuccess) {
        set_error(LD_EHIP);
        return LD_EHIP;
    }
    const int nA = p.n, mA = p.m;
    std::vector<int32_t> a(nA, 0);   // per row of the planner's matrix: sign or message

    if (p.kind == PK_SUMABS) {
        // d >= rows: every row its own message (Eq. L_o_norm reaches sum |M_xy|)
        int64_t v = 0;
        if (!run_plans_sync({&p}, plain_item_shape(), &v, S.s)) {
            set_error(LD_EHIP);
            return LD_EHIP;
        }
        *value = v;
        for (int x = 0; x < nA; ++x)
            for (auto mb : p.row_members[x]) assignment[mb.first] = x;
        return LD_OK;
    }

    int64_t V = 0;
    uint64_t vstar = 0;
    if (!sweep_locate(S, p, INT64_MIN, &V, &vstar) || vstar >= p.n_prefix) {
        set_error(LD_EHIP);
        return LD_EHIP;
    }
    *value = V;
    const int marg = p.kind == PK_MARG ? 1 : 0;
    int rc = LD_OK;
    if (p.kind != PK_LD) {
        // binary: prefix bit h is row nA - P + h of the planner's matrix (its high
        // rows come last), so the plan's prefix is a range-plan prefix as it stands
        const int dd = p.kind == PK_L2 ? 2 : 1;
        int q = p.P;
        uint64_t pfx = vstar;
        rc = refine(S, p.M, nA, mA, dd, marg, V, q, pfx);
        if (rc == LD_OK)
            for (int x = 1; x < nA; ++x) {
                const int bit = (int)((pfx >> (x - 1)) & 1u);
                a[x] = p.kind == PK_L2 ? bit : (bit ? 1 : -1);
            }
        a[0] = p.kind == PK_L2 ? 0 : 1;
    } else {
        // d-ary: the prefix rows come first (restricted-growth digits, then plain
        // base-d digits); move them behind the mid and low rows for the range plans
        const int nh = p.P_tab + p.P;
        std::vector<int> digit(nh, 0);
        const uint64_t t = vstar / p.dpow_free;
        uint64_t fr = vstar - t * p.dpow_free;
        uint64_t code = 0;
        std::memcpy(&code, p.blob.data() + p.off_tab + 8 * t, 8);
        for (int h = 0; h < nh; ++h) {
            if (h < p.P_tab) {
                digit[h] = (int)((code >> (4 * h)) & 15u);
            } else {
                digit[h] = (int)(fr % (uint64_t)p.d);
                fr /= (uint64_t)p.d;
            }
        }
        // B rows: A row 0, the free rows (A rows nh ..), then A rows 1 .. nh-1
        std::vector<int> from;   // B row -> A row
        from.push_back(0);
        for (int x = nh; x < nA; ++x) from.push_back(x);
        for (int x = 1; x < nh; ++x) from.push_back(x);
        std::vector<int32_t> B((size_t)nA * mA);
        for (int i = 0; i < nA; ++i)
            std::memcpy(B.data() + (size_t)i * mA, p.M.data() + (size_t)from[i] * mA, 4 * (size_t)mA);
        int q = nh - 1;
        uint64_t pfx = 0;
        for (int h = nh - 1; h >= 1; --h) pfx = pfx * (uint64_t)p.d + (uint64_t)digit[h];
        rc = refine(S, B, nA, mA, p.d, 0, V, q, pfx);
        if (rc == LD_OK) {
            a[0] = digit.empty() ? 0 : digit[0];
            for (int i = 1; i < nA; ++i) {
                a[from[i]] = (int)(pfx % (uint64_t)p.d);
                pfx /= (uint64_t)p.d;
            }
        }
    }
    if (rc != LD_OK) {
        set_error(rc);
        return rc;
    }

    if (!binary) {
        // merged rows (positive multiples only, for d >= 2) share the row's message
        for (int x = 0; x < nA; ++x)
            for (auto mb : p.row_members[x]) assignment[mb.first] = a[x];
        return LD_OK;
    }
    // d = 1: the enumerated side maps back through the preprocessing; the other
    // side is the sign of the matching product with the caller's matrix
    std::vector<int32_t> side(p.transposed ? m : n, 1);
    // a row merged with sign s takes s times the row's sign (rule A1)
    for (int x = 0; x < nA; ++x)
        for (auto mb : p.row_members[x]) side[mb.first] = mb.second * a[x];
    std::vector<int32_t> other;
    {
        const int len_other = p.transposed ? n : m;
        int32_t* dM = (int32_t*)S.dalloc(4 * (size_t)n * m);
        int32_t* dv = (int32_t*)S.dalloc(4 * side.size());
        int32_t* dout = (int32_t*)S.dalloc(4 * (size_t)len_other);
        int32_t* hout = (int32_t*)S.halloc(4 * (size_t)len_other);
        if (!dM || !dv || !dout || !hout) {
            set_error(LD_EHIP);
            return LD_EHIP;
        }
        bool ok = hipMemcpyAsync(dM, M, 4 * (size_t)n * m, hipMemcpyHostToDevice, S.s) == hipSuccess;
        ok = ok && hipMemcpyAsync(dv, side.data(), 4 * side.size(), hipMemcpyHostToDevice, S.s) == hipSuccess;
        int32_t nn = n, mm = m, rows = p.transposed ? 1 : 0, fix0 = marginals ? 1 : 0;
        void* args[] = {(void*)&dM, (void*)&nn, (void*)&mm, (void*)&dv, (void*)&rows, (void*)&fix0, (void*)&dout};
        const uint32_t blocks = (uint32_t)std::max(1, std::min(64, (len_other + 255) / 256));
        ok = ok && hipLaunchKernel(kernel_signs(), dim3(blocks), dim3(256), args, 0, S.s) == hipSuccess;
        ok = ok && hipMemcpyAsync(hout, dout, 4 * (size_t)len_other, hipMemcpyDeviceToHost, S.s) == hipSuccess;
        ok = ok && hipStreamSynchronize(S.s) == hipSuccess;
        if (!ok) {
            set_error(LD_EHIP);
            return LD_EHIP;
        }
        other.assign(hout, hout + len_other);
    }
    const std::vector<int32_t>& rows_side = p.transposed ? other : side;
    const std::vector<int32_t>& cols_side = p.transposed ? side : other;
    for (int x = 0; x < n; ++x) assignment[x] = rows_side[x];
    if (marginals) assignment[0] = 1;
    if (col_assignment)
        for (int y = 0; y < m; ++y) col_assignment[y] = cols_side[y];
    return LD_OK;
}
