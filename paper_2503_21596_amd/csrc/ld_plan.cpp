// Host planner (see ld_plan.h).
#include "ld_plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "ld.h"
#include "ld_registry.h"

namespace ld {

namespace {

std::mutex g_shape_mu;
SweepShape g_shape;

struct Mat {
    int n = 0, m = 0;
    std::vector<int32_t> a;
    // input rows / columns folded into each row / column, with the sign they enter with
    // (preprocessing only; a merge appends the members of the row it absorbs)
    std::vector<Members> ri, ci;
    int32_t at(int x, int y) const { return a[(size_t)x * m + y]; }
};

Mat transpose(const Mat& A)
{
    Mat T;
    T.n = A.m;
    T.m = A.n;
    T.a.resize(A.a.size());
    for (int x = 0; x < A.n; ++x)
        for (int y = 0; y < A.m; ++y) T.a[(size_t)y * T.m + x] = A.at(x, y);
    T.ri = A.ci;
    T.ci = A.ri;
    return T;
}

bool row_zero(const Mat& A, int x)
{
    for (int y = 0; y < A.m; ++y)
        if (A.at(x, y)) return false;
    return true;
}

bool col_zero(const Mat& A, int y)
{
    for (int x = 0; x < A.n; ++x)
        if (A.at(x, y)) return false;
    return true;
}

// Drop all-zero rows and columns; rows / columns with index 0 are kept when
// keep0 is set (the marginal row and column of Eq. (LMarg)).
Mat drop_zeros(const Mat& A, bool keep0)
{
    std::vector<int> rows, cols;
    for (int x = 0; x < A.n; ++x)
        if ((keep0 && x == 0) || !row_zero(A, x)) rows.push_back(x);
    for (int y = 0; y < A.m; ++y)
        if ((keep0 && y == 0) || !col_zero(A, y)) cols.push_back(y);
    Mat B;
    B.n = (int)rows.size();
    B.m = (int)cols.size();
    B.a.resize((size_t)B.n * B.m);
    for (int i = 0; i < B.n; ++i)
        for (int j = 0; j < B.m; ++j) B.a[(size_t)i * B.m + j] = A.at(rows[i], cols[j]);
    for (int x : rows) B.ri.push_back(A.ri[x]);
    for (int y : cols) B.ci.push_back(A.ci[y]);
    return B;
}

Mat drop_first_row_col(const Mat& A)
{
    Mat B;
    B.n = A.n - 1;
    B.m = A.m - 1;
    B.a.resize((size_t)std::max(0, B.n) * std::max(0, B.m));
    for (int x = 1; x < A.n; ++x)
        for (int y = 1; y < A.m; ++y) B.a[(size_t)(x - 1) * B.m + (y - 1)] = A.at(x, y);
    B.ri.assign(A.ri.begin() + std::min<size_t>(1, A.ri.size()), A.ri.end());
    B.ci.assign(A.ci.begin() + std::min<size_t>(1, A.ci.size()), A.ci.end());
    return B;
}

// --- exact reductions (Sec. 2.1.1, Sec. 2.2, Sec. 2.3.1; Appendices A and B) ---

// v = c u for some c != 0 (both rows nonzero): returns sign(c), else 0
int proportional(const int32_t* u, const int32_t* v, int len, int stride)
{
    int k = 0;
    while (k < len && u[(size_t)k * stride] == 0) ++k;
    if (k == len || v[(size_t)k * stride] == 0) return 0;
    const int64_t uk = u[(size_t)k * stride], vk = v[(size_t)k * stride];
    for (int y = 0; y < len; ++y)
        if ((int64_t)v[(size_t)y * stride] * uk != (int64_t)u[(size_t)y * stride] * vk) return 0;
    return ((uk < 0) == (vk < 0)) ? 1 : -1;
}

bool fits_i32(int64_t v) { return v >= INT32_MIN && v <= INT32_MAX; }

// Merge proportional rows (rows = true) or columns: the pair is replaced by the
// first plus sign(c) times the second, i.e. (1 + |c|) times the first.  A merge
// needs `allow(sign)` (rule A1: any sign for d = 1; A2: any sign for columns when
// d >= 2; A3: c > 0 only for rows when d >= 2); index 0 is left alone when keep0
// (the marginal row / column of Eq. LMarg).  Merges that would overflow int32 are
// skipped.  Returns true if anything merged.
template <class Allow>
bool merge_proportional(Mat& A, bool rows, bool keep0, Allow allow)
{
    const int cnt = rows ? A.n : A.m, len = rows ? A.m : A.n;
    const int stride = rows ? 1 : A.m;   // step between the entries of one row / column
    auto line = [&](int i) { return A.a.data() + (rows ? (size_t)i * A.m : (size_t)i); };
    std::vector<char> gone(cnt, 0);
    bool any = false;
    for (int i = keep0 ? 1 : 0; i < cnt; ++i) {
        if (gone[i]) continue;
        for (int j = i + 1; j < cnt; ++j) {
            if (gone[j]) continue;
            const int sg = proportional(line(i), line(j), len, stride);
            if (sg == 0 || !allow(sg)) continue;
            bool ok = true;
            for (int t = 0; t < len && ok; ++t)
                ok = fits_i32((int64_t)line(i)[(size_t)t * stride] + sg * (int64_t)line(j)[(size_t)t * stride]);
            if (!ok) continue;
            for (int t = 0; t < len; ++t) line(i)[(size_t)t * stride] += sg * line(j)[(size_t)t * stride];
            auto& to = rows ? A.ri[i] : A.ci[i];
            for (auto mb : (rows ? A.ri[j] : A.ci[j])) to.push_back({mb.first, mb.second * sg});
            gone[j] = 1;
            any = true;
        }
    }
    if (!any) return false;
    // compact: drop the absorbed rows / columns
    std::vector<int> keep;
    for (int i = 0; i < cnt; ++i)
        if (!gone[i]) keep.push_back(i);
    Mat B;
    B.n = rows ? (int)keep.size() : A.n;
    B.m = rows ? A.m : (int)keep.size();
    B.a.resize((size_t)B.n * B.m);
    for (int x = 0; x < B.n; ++x)
        for (int y = 0; y < B.m; ++y) B.a[(size_t)x * B.m + y] = rows ? A.at(keep[x], y) : A.at(x, keep[y]);
    B.ri = A.ri;
    B.ci = A.ci;
    if (rows) {
        B.ri.clear();
        for (int i : keep) B.ri.push_back(A.ri[i]);
    } else {
        B.ci.clear();
        for (int i : keep) B.ci.push_back(A.ci[i]);
    }
    A = std::move(B);
    return true;
}

// d >= 2 (Appendix A): columns whose entries all share one sign (zeros allowed)
// merge into one column of |M_xy1| + |M_xy2| + ...  Skipped on int32 overflow.
bool merge_uniform_columns(Mat& A)
{
    std::vector<int> uni;
    for (int y = 0; y < A.m; ++y) {
        bool pos = true, neg = true;
        for (int x = 0; x < A.n; ++x) {
            pos = pos && A.at(x, y) >= 0;
            neg = neg && A.at(x, y) <= 0;
        }
        if (pos || neg) uni.push_back(y);
    }
    if (uni.size() < 2) return false;
    std::vector<int64_t> col(A.n, 0);
    for (int x = 0; x < A.n; ++x) {
        for (int y : uni) col[x] += std::abs((int64_t)A.at(x, y));
        if (!fits_i32(col[x])) return false;
    }
    const int y0 = uni[0];
    for (int x = 0; x < A.n; ++x) A.a[(size_t)x * A.m + y0] = (int32_t)col[x];
    for (size_t k = 1; k < uni.size(); ++k)
        for (auto mb : A.ci[uni[k]]) A.ci[y0].push_back(mb);
    std::vector<int> keep;
    for (int y = 0; y < A.m; ++y)
        if (y == y0 || std::find(uni.begin(), uni.end(), y) == uni.end()) keep.push_back(y);
    Mat B;
    B.n = A.n;
    B.m = (int)keep.size();
    B.a.resize((size_t)B.n * B.m);
    for (int x = 0; x < B.n; ++x)
        for (int j = 0; j < B.m; ++j) B.a[(size_t)x * B.m + j] = A.at(x, keep[j]);
    B.ri = A.ri;
    for (int y : keep) B.ci.push_back(A.ci[y]);
    A = std::move(B);
    return true;
}

// All merges for one kind, repeated until none applies.
void reduce(Mat& A, int d, bool marg)
{
    for (bool again = true; again;) {
        again = false;
        if (d == 1) {
            auto any = [](int) { return true; };
            again |= merge_proportional(A, true, marg, any);
            again |= merge_proportional(A, false, marg, any);
        } else {
            again |= merge_proportional(A, true, false, [](int sg) { return sg > 0; });
            again |= merge_proportional(A, false, false, [](int) { return true; });
            again |= merge_uniform_columns(A);
        }
    }
}

int64_t sum_abs(const Mat& A)
{
    int64_t s = 0;
    for (int32_t v : A.a) s += v < 0 ? -(int64_t)v : (int64_t)v;
    return s;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

template <class T>
void put(std::vector<uint8_t>& blob, size_t off, size_t idx, T v)
{
    std::memcpy(blob.data() + off + sizeof(T) * idx, &v, sizeof(T));
}

constexpr int64_t BIAS = (int64_t)1 << 31;
constexpr uint64_t WORD_LIMIT = (uint64_t)1 << 62;
constexpr double RGS_TRADE_MAX = 4096;   // restricted-growth strings a lane trade may grow the table to

// Binary tables.  Row roles in A: row 0 fixed (a_0 = +1, or message 0 for L2),
// rows 1..R low, then C mid rows, then P high rows.  A digit is the bit of the
// Gray word / prefix / low pattern:
//   L1 / L_marg: digit 1 -> a = +1 (contributes +M_x), digit 0 -> a = -1 (-M_x)
//   L2: the digit is the message; the state is the sum of the rows sent as
//       message 0 (the fixed row and every digit-0 row)
void build_binary(Plan& p, const Mat& A)
{
    const bool l2 = (p.kind == PK_L2);
    const int m = A.m, mp = p.mp, R = p.R, C = p.C, P = p.P;
    const int NW = 1 << R;
    auto v0 = [&](int x, int y) -> int64_t { return l2 ? (int64_t)A.at(x, y) : -(int64_t)A.at(x, y); };
    auto v1 = [&](int x, int y) -> int64_t { return l2 ? 0 : (int64_t)A.at(x, y); };
    const int mid0 = 1 + R, high0 = 1 + R + C;

    std::vector<int64_t> base(mp, 0), total(mp, 0);
    for (int y = 0; y < m; ++y) {
        int64_t b = A.at(0, y);
        for (int x = mid0; x < high0 + P; ++x) b += v0(x, y);
        base[y] = b;
        for (int x = 0; x < A.n; ++x) total[y] += A.at(x, y);
    }
    auto delta = [&](int x, int y) -> int64_t { return y < m ? v1(x, y) - v0(x, y) : 0; };

    if (!p.i64 && p.pack16) {
        // two columns per dword: halves offset by 2^15; a delta dword is
        // d_lo + 2^16 d_hi modulo 2^32; L_marg's column 0 carries the offset h
        // (state + h, operand - h) so that its term is x + 2h = x + bias
        const int MW = mp / 2;
        const int RS = (MW + 15) & ~15;
        const int K = l2 ? 2 : 1;
        const int64_t h = p.bias / 2, H = 1 << 15;
        auto half = [](int64_t v) { return (uint32_t)((uint64_t)v & 0xffffu); };
        auto pack = [&](int64_t lo, int64_t hi) { return half(lo) | (half(hi) << 16); };
        auto dpack = [](int64_t lo, int64_t hi) { return (uint32_t)(uint64_t)(lo + hi * 65536); };
        p.off_base = 0;
        p.off_hid = align256(p.off_base + 4 * (size_t)MW);
        p.off_mid = align256(p.off_hid + 4 * (size_t)std::max(P, 1) * RS);
        p.off_offs = align256(p.off_mid + 4 * (size_t)std::max(C, 1) * 2 * RS);
        p.off_tab = align256(p.off_offs + 4 * (size_t)K * NW * RS);
        p.blob.assign(p.off_tab, 0);
        for (int j = 0; j < MW; ++j)
            put<uint32_t>(p.blob, p.off_base, j, pack(base[2 * j] + H + (j == 0 ? h : 0), base[2 * j + 1] + H));
        for (int hh = 0; hh < P; ++hh)
            for (int j = 0; j < MW; ++j)
                put<uint32_t>(p.blob, p.off_hid, (size_t)hh * RS + j,
                              dpack(delta(high0 + hh, 2 * j), delta(high0 + hh, 2 * j + 1)));
        for (int k = 0; k < C; ++k)
            for (int j = 0; j < MW; ++j) {
                const int64_t a = delta(mid0 + k, 2 * j), b = delta(mid0 + k, 2 * j + 1);
                put<uint32_t>(p.blob, p.off_mid, (size_t)(2 * k) * RS + j, dpack(a, b));
                put<uint32_t>(p.blob, p.off_mid, (size_t)(2 * k + 1) * RS + j, dpack(-a, -b));
            }
        for (int w = 0; w < NW; ++w) {
            std::vector<int64_t> low(mp, 0);
            for (int y = 0; y < m; ++y)
                for (int i = 0; i < R; ++i) low[y] += ((w >> i) & 1) ? v1(1 + i, y) : v0(1 + i, y);
            for (int j = 0; j < MW; ++j) {
                put<uint32_t>(p.blob, p.off_offs, (size_t)w * RS + j,
                              pack(H - low[2 * j] - (j == 0 ? h : 0), H - low[2 * j + 1]));
                if (l2)
                    put<uint32_t>(p.blob, p.off_offs, (size_t)(NW + w) * RS + j,
                                  pack(H + total[2 * j] - low[2 * j], H + total[2 * j + 1] - low[2 * j + 1]));
            }
        }
    } else if (!p.i64) {
        const int RS = (mp + 15) & ~15;
        const int K = l2 ? 2 : 1;
        p.off_base = 0;
        p.off_hid = align256(p.off_base + 4 * (size_t)mp);
        p.off_mid = align256(p.off_hid + 4 * (size_t)std::max(P, 1) * RS);
        p.off_offs = align256(p.off_mid + 4 * (size_t)std::max(C, 1) * 2 * RS);
        p.off_tab = align256(p.off_offs + 4 * (size_t)K * NW * RS);
        p.blob.assign(p.off_tab, 0);
        for (int y = 0; y < mp; ++y) put<uint32_t>(p.blob, p.off_base, y, (uint32_t)(base[y] + BIAS));
        for (int h = 0; h < P; ++h)
            for (int y = 0; y < mp; ++y)
                put<int32_t>(p.blob, p.off_hid, (size_t)h * RS + y, (int32_t)(uint32_t)delta(high0 + h, y));
        for (int k = 0; k < C; ++k)
            for (int y = 0; y < mp; ++y) {
                const int64_t dv = delta(mid0 + k, y);
                put<int32_t>(p.blob, p.off_mid, (size_t)(2 * k) * RS + y, (int32_t)(uint32_t)dv);
                put<int32_t>(p.blob, p.off_mid, (size_t)(2 * k + 1) * RS + y, (int32_t)(uint32_t)(-dv));
            }
        for (int w = 0; w < NW; ++w)
            for (int y = 0; y < mp; ++y) {
                int64_t low = 0;
                if (y < m)
                    for (int i = 0; i < R; ++i) low += ((w >> i) & 1) ? v1(1 + i, y) : v0(1 + i, y);
                // |s - o| with s = true + 2^31 must equal |true + low| (and for L2
                // the second operand gives |total - (true + low)|)
                put<uint32_t>(p.blob, p.off_offs, (size_t)w * RS + y, (uint32_t)(BIAS - low));
                if (l2)
                    put<uint32_t>(p.blob, p.off_offs, (size_t)(NW + w) * RS + y,
                                  (uint32_t)(BIAS + total[y] - low));
            }
    } else {
        p.off_base = 0;
        p.off_hid = align256(p.off_base + 8 * (size_t)mp);
        p.off_mid = align256(p.off_hid + 8 * (size_t)std::max(P, 1) * mp);
        p.off_offs = align256(p.off_mid + 8 * (size_t)std::max(C, 1) * 2 * mp);
        p.off_tab = align256(p.off_offs + 8 * (size_t)mp);
        p.blob.assign(p.off_tab, 0);
        for (int y = 0; y < mp; ++y) put<int64_t>(p.blob, p.off_base, y, base[y]);
        for (int h = 0; h < P; ++h)
            for (int y = 0; y < mp; ++y) put<int64_t>(p.blob, p.off_hid, (size_t)h * mp + y, delta(high0 + h, y));
        for (int k = 0; k < C; ++k)
            for (int y = 0; y < mp; ++y) {
                put<int64_t>(p.blob, p.off_mid, (size_t)(2 * k) * mp + y, delta(mid0 + k, y));
                put<int64_t>(p.blob, p.off_mid, (size_t)(2 * k + 1) * mp + y, -delta(mid0 + k, y));
            }
        for (int y = 0; y < mp; ++y) put<int64_t>(p.blob, p.off_offs, y, total[y]);
    }
}

// d-ary tables.  Row roles in A: P_tab prefix rows covered by tab[], then P
// plain prefix rows, then C mid rows, then R low rows; `fixed0`: row 0 comes
// first and is fixed at message 0 (range plans).  The low rows are not part of
// any state vector: offs[S] = 2^31 - (sum of the low rows in subset S) lets the
// kernel score every message choice of the low rows against the same state.
void build_dary(Plan& p, const Mat& A, const std::vector<uint64_t>& tab, bool fixed0)
{
    const int m = A.m, mp = p.mp, C = p.C, R = p.R;
    const int nh = p.P_tab + p.P;
    const int h0 = fixed0 ? 1 : 0;          // first prefix row
    const int mid0 = h0 + nh;
    const int low0 = mid0 + C;
    const int NS = 1 << R;
    const size_t es = p.i64 ? 8 : 4;
    // dwords per row: mp, or mp / 2 in the packed form (two columns per dword,
    // halves offset by 2^15, row entries d_2j + 2^16 d_2j+1 modulo 2^32)
    const int W = p.pack16 ? mp / 2 : mp;
    const int64_t H = 1 << 15;
    auto col = [&](int x, int y) -> int64_t { return y < m ? A.at(x, y) : 0; };
    auto half = [](int64_t v) { return (uint32_t)((uint64_t)v & 0xffffu); };
    p.off_base = 0;
    p.off_hid = align256(es * (size_t)W);
    p.off_mid = align256(p.off_hid + es * (size_t)std::max(nh, 1) * W);
    p.off_offs = align256(p.off_mid + es * (size_t)std::max(C, 1) * W);
    const int RS = (W + 15) & ~15;   // subset-operand row stride (scalar loads of 8 dwords)
    p.off_tab = align256(p.off_offs + 4 * (size_t)NS * RS);
    const size_t end = align256(p.off_tab + 8 * std::max<size_t>(tab.size(), 1));
    p.blob.assign(end, 0);
    std::vector<int64_t> base(mp, 0);
    for (int y = 0; y < m; ++y) {
        if (fixed0) base[y] += A.at(0, y);
        for (int c = 0; c < C; ++c) base[y] += A.at(mid0 + c, y);
    }
    for (int j = 0; j < W; ++j) {
        if (p.pack16) put<uint32_t>(p.blob, p.off_base, j, half(base[2 * j] + H) | (half(base[2 * j + 1] + H) << 16));
        else if (p.i64) put<int64_t>(p.blob, p.off_base, j, base[j]);
        else put<uint32_t>(p.blob, p.off_base, j, (uint32_t)(base[j] + BIAS));
    }
    auto row = [&](size_t off, int slot, int x) {
        for (int j = 0; j < W; ++j) {
            const size_t at = (size_t)slot * W + j;
            if (p.pack16) put<uint32_t>(p.blob, off, at, (uint32_t)(uint64_t)(col(x, 2 * j) + 65536 * col(x, 2 * j + 1)));
            else if (p.i64) put<int64_t>(p.blob, off, at, col(x, j));
            else put<int32_t>(p.blob, off, at, (int32_t)col(x, j));
        }
    };
    for (int h = 0; h < nh; ++h) row(p.off_hid, h, h0 + h);
    for (int c = 0; c < C; ++c) row(p.off_mid, c, mid0 + c);
    for (int sub = 0; sub < NS; ++sub) {
        std::vector<int64_t> low(mp, 0);
        for (int y = 0; y < m; ++y)
            for (int i = 0; i < R; ++i)
                if ((sub >> i) & 1) low[y] += A.at(low0 + i, y);
        for (int j = 0; j < W; ++j) {
            const uint32_t o = p.pack16 ? (half(H - low[2 * j]) | (half(H - low[2 * j + 1]) << 16))
                                        : (uint32_t)(BIAS - low[j]);
            put<uint32_t>(p.blob, p.off_offs, (size_t)sub * RS + j, o);
        }
    }
    for (size_t i = 0; i < tab.size(); ++i) put<uint64_t>(p.blob, p.off_tab, i, tab[i]);
}

// All restricted-growth strings of length L over {0..d-1}: s_0 = 0 and each
// s_i at most one above the largest earlier digit.  Every assignment of rows to
// messages can be relabelled (a permutation of the messages, which keeps the
// witness value of Eq. (L_o_norm)) so that its first L digits form such a string.
void rgs(int L, int d, std::vector<uint64_t>& out)
{
    if (L <= 0) {
        out.push_back(0);
        return;
    }
    struct Frame { int i, mx; uint64_t code; };
    std::vector<Frame> st;
    st.push_back({1, 0, 0});
    while (!st.empty()) {
        Frame f = st.back();
        st.pop_back();
        if (f.i == L) {
            out.push_back(f.code);
            continue;
        }
        const int top = std::min(f.mx + 1, d - 1);
        for (int v = top; v >= 0; --v)
            st.push_back({f.i + 1, std::max(f.mx, v), f.code | ((uint64_t)v << (4 * f.i))});
    }
}

// number of restricted-growth strings of length L with at most d distinct digits
// (sum over k <= d of the Stirling numbers of the second kind S(L, k))
double rgs_count(int L, int d)
{
    std::vector<double> S(d + 1, 0.0);   // S[k] for the current length
    S[0] = 1.0;                          // length 0
    for (int n = 1; n <= L; ++n) {
        for (int k = std::min(n, d); k >= 1; --k) S[k] = k * S[k] + S[k - 1];
        S[0] = 0.0;                      // no non-empty string has zero distinct digits
    }
    double t = 0;
    for (int k = 1; k <= d; ++k) t += S[k];
    return L == 0 ? 1.0 : t;
}

uint64_t upow(uint64_t b, int e, bool* overflow)
{
    uint64_t r = 1;
    for (int i = 0; i < e; ++i) {
        if (r > WORD_LIMIT / b) *overflow = true;
        r *= b;
    }
    return r;
}

void choose_binary_shape(Plan& p, const SweepShape& sh, int F)
{
    // F free rows beyond the R low rows
    const int Fp = F - p.R;
    int P, C;
    if (sh.c_target > 0) {
        C = std::min(Fp, std::max(0, sh.c_target - p.R));
        P = Fp - C;
        if (sh.pfx_cap > 0 && P > sh.pfx_cap) {
            P = sh.pfx_cap;
            C = Fp - P;
        }
    } else {
        // enough lanes to fill the device, enough words per lane to amortise its
        // start: 2^c_goal words per prefix, 2^p_min .. 2^p_target prefixes
        P = F - sh.c_goal;
        P = std::max(P, std::min(Fp, sh.p_min));
        P = std::min(P, std::min(Fp, sh.p_target));
        P = std::max(P, 0);
        C = Fp - P;
        if (C < sh.c_min) {
            // mid rows amortise a lane's start, but a small problem takes lanes
            // first: it keeps at least 2^p_fill of them (one wave per SIMD at
            // 2^16), and only rows beyond those become mid rows, up to c_min
            int want = sh.c_min;
            if (sh.p_fill > 0) want = std::min(want, Fp - sh.p_fill);
            C = std::min(Fp, std::max(C, want));
            P = Fp - C;
        }
    }
    if (C > 31) {
        C = 31;
        P = Fp - 31;
    }
    p.C = C;
    p.P = P;
    p.n_prefix = (uint64_t)1 << P;
}

// The wide kernel: int64 tables with row stride m, state in LDS.
bool use_wide(Plan& p, int states)
{
    p.wide = 1;
    p.i64 = 1;
    p.mp = p.m;
    p.lds = 8 * ((size_t)states * p.m + (size_t)states);
    p.kernel = kernel_wide();
    return p.lds <= WIDE_LDS_MAX;
}

// int32 binary kernel: the SGPR-operand kernel with sh.sgpr_r low rows when it
// exists for this width, else the VGPR-operand kernel with as many low rows as
// its register budget allows
// d-ary variant for a problem: 0 VGPR operands, 1 SGPR operands, 16 packed 16-bit
int dary_variant(const SweepShape& sh, int d, int mp)
{
    const int cls = variant_class(PK_LD, d);
    const int tuned = cls >= 0 ? sh.variant[cls][variant_bucket(mp)] : -1;
    return tuned >= 0 ? tuned : sh.dary_sgpr;
}

int bin_variant(const Plan& p, const SweepShape& sh)
{
    const int cls = variant_class(p.kind, p.d);
    const int tuned = cls >= 0 ? sh.variant[cls][variant_bucket(p.mp)] : -1;
    return tuned >= 0 ? tuned : sh.sgpr_r;
}

// The packed 16-bit kernel needs every column sum and operand to fit 16 bits offset
// by 2^15: sum_x |M_xy| <= 2^15 - 1 for every column, and for L_marg's linear
// column 0 also its offset h = ceil(B_0 / 2) on top (B_0 + h <= 2^15 - 1).  On
// success p.bias = 2h (L_marg) or 0.
bool pack16_fits(Plan& p, const Mat& A)
{
    for (int y = 0; y < A.m; ++y) {
        int64_t b = 0;
        for (int x = 0; x < A.n; ++x) b += std::abs((int64_t)A.at(x, y));
        const int64_t h = (p.kind == PK_MARG && y == 0) ? (b + 1) / 2 : 0;
        if (b + h > PACK16_BOUND) return false;
        if (p.kind == PK_MARG && y == 0) p.bias = (int32_t)(2 * h);
    }
    return true;
}

// (the MFMA variant plans as the SGPR-operand kernel with R = 5, whose tables it
// shares; use_mfma switches the kernel once the tables are built)
void pick_bin32(Plan& p, const SweepShape& sh, Mat const& A)
{
    int sr = bin_variant(p, sh);
    if (sr == VARIANT_PACK16) {
        p.bias = 0;
        const void* k =
            pack16_fits(p, A) ? kernel_bin16s(p.kind == PK_L2 ? KIND_L2 : KIND_L1, p.mp / 2, PACK16_R) : nullptr;
        if (k) {
            p.kernel = k;
            p.pack16 = 1;
            p.R = PACK16_R;
            return;
        }
        p.bias = 0;
        sr = 5;
    }
    if (sr == VARIANT_MFMA) sr = 5;
    p.kernel = sr > 0 ? kernel_bin32s(p.kind, p.mp, sr) : nullptr;
    if (p.kernel) {
        p.R = sr;
        return;
    }
    p.R = std::max(0, bin_rmax(p.mp, p.kind) - (sh.r_drop ? 1 : 0));
    p.kernel = kernel_bin32(p.kind, p.mp, p.R);
}

// d-ary register kernel of a plan (p.mp set, p.i64 known): the packed 16-bit
// kernel where the variant asks for it and every column bound fits, else the
// SGPR-operand kernel, else the VGPR-operand or int64 one, else the wide kernel.
// `rows` is the number of rows the sweep can give low rows (range plans pad with
// zero rows and pass a large value).  Sets p.kernel, p.R and p.pack16; false if no
// kernel holds the problem.
bool pick_dary(Plan& p, const SweepShape& sh, const Mat& A, int rows)
{
    const int d = p.d;
    p.kernel = nullptr;
    p.pack16 = 0;
    p.bias = 0;
    if (A.m <= MAX_MP && d <= MAX_D && !p.i64) {
        const int v = dary_variant(sh, d, p.mp);
        if (v == VARIANT_PACK16 && rows >= 1 + dary16_r_small(d) && pack16_fits(p, A)) {
            // the larger R where the rows allow (make_plan may step back to the
            // smaller one when a single problem has too few lanes at it)
            const int r = rows >= 1 + dary16_r(d) ? dary16_r(d) : dary16_r_small(d);
            p.kernel = kernel_dary16s(d, p.mp / 2, r);
            if (p.kernel) {
                p.pack16 = 1;
                p.R = r;
                return true;
            }
        }
        if (v != 0 && rows >= 1 + DARY_RS) {
            p.kernel = kernel_dary32s(d, p.mp);
            if (p.kernel) {
                p.R = DARY_RS;
                return true;
            }
        }
    }
    if (A.m <= MAX_MP && d <= MAX_D) p.kernel = p.i64 ? kernel_dary64(d, p.mp) : kernel_dary32(d, p.mp);
    if (!p.kernel && !use_wide(p, d)) return false;
    // the register kernel scores R low rows per state; the others walk every row
    p.R = (!p.wide && !p.i64) ? dary_r(p.mp, d) : 0;
    return true;
}

// Switch an int32 binary plan built for R = 5 to the int8-MFMA kernel when its
// operands fit: 1 <= C <= 16 mid rows, and every mid-row delta divided by the
// step scale (2 for L1 and L_marg, whose deltas are twice an entry; 1 for L2)
// lies in [-128, 127].  Values are the same either way.
void use_mfma(Plan& p)
{
    if (p.i64 || p.wide || p.R != 5 || p.C < 1 || p.C > MFMA_MAX_C) return;
    if (p.kind != PK_L1 && p.kind != PK_MARG && p.kind != PK_L2) return;
    const void* k = kernel_mfma(p.kind == PK_L1 ? KIND_L1 : p.kind == PK_MARG ? KIND_MARG : KIND_L2, p.mp);
    if (!k) return;
    const int sc = p.kind == PK_L2 ? 1 : 2;
    const int RS = (p.mp + 15) & ~15;
    for (int kk = 0; kk < p.C; ++kk)
        for (int y = 0; y < p.mp; ++y) {
            int32_t v;
            std::memcpy(&v, p.blob.data() + p.off_mid + 4 * ((size_t)(2 * kk) * RS + y), 4);
            if (v % sc != 0 || v / sc < -128 || v / sc > 127) return;
        }
    p.kernel = k;
    p.mfma = 1;
}

Plan finish_binary(Plan p, Mat A, const SweepShape& sh)
{
    // A: row 0 fixed; p.kind set; p.i64 set
    if (A.n - 1 > 62) {
        p.status = LD_ETOOBIG;
        return p;
    }
    p.mp = p.i64 ? pad_bin64(A.m) : pad_bin32(A.m);
    p.kernel = nullptr;
    if (A.m <= MAX_MP && p.mp <= MAX_MP) {
        if (p.i64) {
            p.R = 0;
            p.kernel = kernel_bin64(p.kind, p.mp);
        } else {
            pick_bin32(p, sh, A);
        }
    }
    if (!p.kernel) {
        p.R = 0;
        if (!use_wide(p, 1)) {
            p.status = LD_ETOOBIG;
            return p;
        }
    }
    // too few free rows for R low patterns: append all-zero rows (they change no
    // column sum, so the maximum is unchanged; only words are repeated)
    while (A.n - 1 < p.R) {
        A.a.resize((size_t)(A.n + 1) * A.m, 0);
        A.n += 1;
    }
    choose_binary_shape(p, sh, A.n - 1);
    // a plain call of a large problem (many mid rows per lane) takes the packed
    // kernel with one more low row: the same prefixes, one mid row fewer
    if (p.pack16 && sh.c_target == 0 && sh.big_r_c > 0 && p.C >= sh.big_r_c) {
        if (const void* k = kernel_bin16s(p.kind == PK_L2 ? KIND_L2 : KIND_L1, p.mp / 2, PACK16_R_BIG)) {
            p.kernel = k;
            p.R = PACK16_R_BIG;
            choose_binary_shape(p, sh, A.n - 1);
        }
    }
    if (p.wide && p.C > 40) {
        p.status = LD_ETOOBIG;
        return p;
    }
    p.words = (double)((uint64_t)1 << (A.n - 1));
    build_binary(p, A);
    if (!p.wide && !p.i64 && bin_variant(p, sh) == VARIANT_MFMA) use_mfma(p);
    return p;
}

// Prefix, mid and low rows of a d-ary plan whose kernel and R are chosen: sets
// p.P_tab, p.C, p.P and p.lanes_est (the lane count).
void shape_dary(Plan& p, const SweepShape& sh, const Mat& A)
{
    const int d = p.d;
    // restricted-growth prefixes hold 4 bits per digit; for d > 16 only the first
    // row is fixed (message 0), which is the paper's fix-one-entry reduction
    p.P_tab = d <= 16 ? std::min(A.n - p.R, std::max(1, std::min(16, sh.dary_ptab))) : 1;
    while (p.P_tab > 1 && rgs_count(p.P_tab, d) > (double)(1 << 20)) --p.P_tab;
    const int rest = A.n - p.P_tab - p.R;
    int C = 0;
    {
        uint64_t w = 1;
        while (C < rest && w * (uint64_t)d <= (uint64_t)std::max(1, sh.dary_cwords)) {
            w *= d;
            ++C;
        }
    }
    int P = rest - C;
    // batch planning: a large problem takes more words per prefix, not more prefixes
    if (sh.pfx_cap > 0)
        while (P > 0 && rgs_count(p.P_tab, d) * std::pow((double)d, P) > std::ldexp(1.0, sh.pfx_cap)) {
            --P;
            ++C;
        }
    // a single problem should fill the device: trade mid rows for prefix rows
    // (more lanes, fewer words each).  Up to 2^17 lanes (two waves per SIMD) the
    // trade goes on down to two mid rows; beyond that, up to dary_lanes, only while
    // each lane keeps about 2^12 words, since a lane's start costs about as much as
    // scoring a few hundred words
    if (sh.dary_lanes > 0) {
        auto lanes = [&](int pt, int pf) { return rgs_count(pt, d) * std::pow((double)d, pf); };
        auto trade = [&]() {
            // a longer restricted-growth prefix removes no more words once the table
            // holds a few thousand strings (the relabelling factor is then d! already),
            // but the host builds and uploads the table on every plan
            if (d <= 16 && p.P_tab < 16 && P == 0 && rgs_count(p.P_tab + 1, d) <= (double)RGS_TRADE_MAX)
                ++p.P_tab;
            else
                ++P;
            --C;
        };
        const double fill = std::min((double)sh.dary_lanes, (double)(1 << 17));
        while (C > 2 && lanes(p.P_tab, P) < fill) trade();
        int c_floor = 2;
        while (std::pow((double)d, c_floor + p.R) < 4096.0) ++c_floor;
        while (C > c_floor && lanes(p.P_tab, P) < (double)sh.dary_lanes) trade();
    }
    // the register kernels count a lane's d^C Gray words in 32 bits: move mid rows
    // back into the prefix until d^C < 2^32 (the batch prefix cap above can push C
    // past that; values do not depend on the split)
    while (C > 0 && std::pow((double)d, C) > 4294967295.0) {
        --C;
        ++P;
    }
    p.C = C;
    p.P = P;
    p.lanes_est = rgs_count(p.P_tab, d) * std::pow((double)d, P);
}

}  // namespace

int variant_class(int kind, int d)
{
    switch (kind) {
    case PK_L1:
    case PK_MARG: return 0;
    case PK_L2: return 1;
    case PK_LD: return d == 3 ? 2 : d == 4 ? 3 : -1;
    default: return -1;
    }
}

SweepShape get_shape()
{
    std::lock_guard<std::mutex> g(g_shape_mu);
    return g_shape;
}

void set_shape(const SweepShape& s)
{
    std::lock_guard<std::mutex> g(g_shape_mu);
    g_shape = s;
}

Plan make_plan(const int32_t* M, int n, int m, int d, int marginals, const SweepShape& sh)
{
    Plan p;
    if (!M || n < 1 || m < 1 || d < 1 || (marginals != 0 && marginals != 1)) {
        p.status = LD_EINVAL;
        return p;
    }
    if (marginals && d >= 2) {
        p.status = LD_EMARG_D;
        return p;
    }
    Mat A;
    A.n = n;
    A.m = m;
    A.a.assign(M, M + (size_t)n * m);
    for (int x = 0; x < n; ++x) A.ri.push_back({{x, 1}});
    for (int y = 0; y < m; ++y) A.ci.push_back({{y, 1}});
    p.d = d;

    if (d == 1 && marginals) {
        A = drop_zeros(A, true);
        if (row_zero(A, 0) && col_zero(A, 0)) {
            // no marginals at all: L_marg is L1 of the correlation block (Sec. 2.2)
            A = drop_first_row_col(A);
            A = drop_zeros(A, false);
            p.kind = PK_L1;
        } else {
            p.kind = PK_MARG;
        }
    } else {
        A = drop_zeros(A, false);
        p.kind = d == 1 ? PK_L1 : (d == 2 ? PK_L2 : PK_LD);
    }
    if (sh.merge && A.n > 0 && A.m > 0) reduce(A, d, p.kind == PK_MARG);
    if (A.n == 0 || A.m == 0) {
        p.kind = PK_ZERO;
        p.n = p.m = 0;
        return p;
    }
    if ((p.kind == PK_L1 || p.kind == PK_MARG) && A.n > A.m) {
        A = transpose(A);   // L1(M) = L1(M^T); L_marg too (row 0 <-> column 0)
        p.transposed = 1;
    }
    if (p.kind == PK_L2 || p.kind == PK_LD) {
        if (d >= A.n) {
            p.kind = PK_SUMABS;   // every row can take its own message
        }
    }
    p.n = A.n;
    p.m = A.m;
    p.d = std::min(d, A.n);
    p.row_members = A.ri;
    p.col_members = A.ci;
    const int64_t B = sum_abs(A);
    p.i64 = B > (int64_t)0x7fffffff ? 1 : 0;

    if (p.kind == PK_SUMABS) {
        p.M = A.a;
        p.blob.resize(align256(4 * A.a.size()));
        std::memcpy(p.blob.data(), A.a.data(), 4 * A.a.size());
        p.words = 1;
        return p;
    }
    if (p.kind != PK_LD) {
        p.M = A.a;
        return finish_binary(p, A, sh);
    }

    // d >= 3, d < n
    p.mp = pad_dary(A.m);
    if (!pick_dary(p, sh, A, A.n)) {
        p.status = LD_ETOOBIG;
        return p;
    }
    shape_dary(p, sh, A);
    // a single problem should fill the device: when the packed kernel's larger R
    // leaves fewer lanes than half a wave per SIMD (or than dary_lanes asks), its
    // kernel with one low row fewer has d times as many states to spread.  (Measured:
    // 16 x 32 L_3 has 3281 lanes at R = 5, 68.6 us, and 9843 at R = 4, 41 us; 16 x 32
    // L_4 has 44720 lanes at R = 4, 83 us, and 178880 at R = 3, 96 us.)
    const double fill = std::min((double)sh.dary_lanes, (double)(1 << 15));
    if (p.pack16 && sh.dary_lanes > 0 && p.R == dary16_r(d) && p.lanes_est < fill &&
        A.n >= 1 + dary16_r_small(d)) {
        if (const void* k = kernel_dary16s(d, p.mp / 2, dary16_r_small(d))) {
            p.kernel = k;
            p.R = dary16_r_small(d);
            shape_dary(p, sh, A);
        }
    }
    if (p.status != LD_OK) return p;
    std::vector<uint64_t> tab;
    rgs(p.P_tab, d, tab);
    bool of = false;
    p.dpow_free = upow(d, p.P, &of);
    const uint64_t cw = upow(d, p.C, &of);
    if (of || (double)tab.size() * (double)p.dpow_free * (double)cw * std::pow((double)d, p.R) >
                  (double)WORD_LIMIT) {
        p.status = LD_ETOOBIG;
        return p;
    }
    p.n_prefix = (uint64_t)tab.size() * p.dpow_free;
    p.words = (double)p.n_prefix * (double)cw * std::pow((double)d, p.R);
    p.M = A.a;
    build_dary(p, A, tab, false);
    return p;
}


Plan make_range_plan(const int32_t* M, int n, int m, int d, int marginals, int q,
                     uint64_t pfx_begin, uint64_t pfx_end)
{
    Plan p;
    if (!M || n < 1 || m < 1 || d < 1 || (marginals != 0 && marginals != 1) || q < 0 || q > n - 1 ||
        pfx_begin >= pfx_end) {
        p.status = LD_EINVAL;
        return p;
    }
    if (marginals && d >= 2) {
        p.status = LD_EMARG_D;
        return p;
    }
    const int radix = d == 1 ? 2 : d;
    bool of = false;
    const uint64_t npfx = upow(radix, q, &of);
    if (of || pfx_end > npfx) {
        p.status = of ? LD_ETOOBIG : LD_EINVAL;
        return p;
    }
    Mat A;
    A.n = n;
    A.m = m;
    A.a.assign(M, M + (size_t)n * m);
    p.n = n;
    p.m = m;
    p.d = d;
    p.kind = d == 1 ? (marginals ? PK_MARG : PK_L1) : (d == 2 ? PK_L2 : PK_LD);
    p.i64 = sum_abs(A) > (int64_t)0x7fffffff ? 1 : 0;
    p.pfx_base = pfx_begin;
    p.n_prefix = pfx_end - pfx_begin;
    p.M = A.a;
    const int free_rows = n - 1 - q;   // rows 1 .. n-q-1

    if (p.kind != PK_LD) {
        p.mp = p.i64 ? pad_bin64(m) : pad_bin32(m);
        p.R = 0;
        p.kernel = nullptr;
        if (m <= MAX_MP && p.mp <= MAX_MP) {
            if (p.i64)
                p.kernel = kernel_bin64(p.kind, p.mp);
            else
                pick_bin32(p, get_shape(), A);
        }
        if (!p.kernel) {
            p.R = 0;
            if (!use_wide(p, 1)) {
                p.status = LD_ETOOBIG;
                return p;
            }
        }
        // rows: 0 fixed, then R low + C mid taken from rows 1..n-q-1 (padded with
        // zero rows when there are fewer than R), then the q prefix rows in order
        Mat B;
        const int lowmid = std::max(free_rows, p.R);
        B.n = 1 + lowmid + q;
        B.m = m;
        B.a.assign((size_t)B.n * m, 0);
        for (int y = 0; y < m; ++y) B.a[y] = A.at(0, y);
        for (int x = 1; x <= free_rows; ++x)
            for (int y = 0; y < m; ++y) B.a[(size_t)x * m + y] = A.at(x, y);
        for (int i = 0; i < q; ++i)
            for (int y = 0; y < m; ++y) B.a[(size_t)(1 + lowmid + i) * m + y] = A.at(n - q + i, y);
        p.C = lowmid - p.R;
        p.P = q;
        if (p.C > 31) {
            p.status = LD_ETOOBIG;
            return p;
        }
        p.words = (double)p.n_prefix * (double)((uint64_t)1 << lowmid);
        build_binary(p, B);
        if (!p.wide && !p.i64 && bin_variant(p, get_shape()) == VARIANT_MFMA) use_mfma(p);
        return p;
    }

    // d >= 3: row 0 fixed at message 0; rows 1..n-q-1 mid; the last q rows prefix
    p.mp = pad_dary(m);
    if (!pick_dary(p, get_shape(), A, 1 << 20)) {
        p.status = LD_ETOOBIG;
        return p;
    }
    // rows 1..n-q-1 give the C mid rows and the R low rows (zero rows pad them when
    // there are fewer than R: a zero row changes no message sum)
    const int lowmid = std::max(free_rows, p.R);
    const uint64_t cw = upow(d, lowmid - p.R, &of);
    if (of || cw > 0xffffffffull) {
        p.status = LD_ETOOBIG;
        return p;
    }
    p.P_tab = 0;
    p.P = q;
    p.C = lowmid - p.R;
    p.dpow_free = npfx;
    p.words = (double)p.n_prefix * (double)cw * std::pow((double)d, p.R);
    // B: row 0, then the q prefix rows, then the mid and low rows
    Mat B;
    B.n = 1 + q + lowmid;
    B.m = m;
    B.a.assign((size_t)B.n * m, 0);
    for (int y = 0; y < m; ++y) B.a[y] = A.at(0, y);
    for (int i = 0; i < q; ++i)
        for (int y = 0; y < m; ++y) B.a[(size_t)(1 + i) * m + y] = A.at(n - q + i, y);
    for (int c = 0; c < free_rows; ++c)
        for (int y = 0; y < m; ++y) B.a[(size_t)(1 + q + c) * m + y] = A.at(1 + c, y);
    build_dary(p, B, {}, true);
    return p;
}

Desc make_desc(const Plan& p, const void* dev_blob, int64_t* result)
{
    Desc D{};
    D.kind = p.kind == PK_L1 ? KIND_L1 : p.kind == PK_MARG ? KIND_MARG : p.kind == PK_L2 ? KIND_L2 : KIND_LD;
    D.m = p.m;
    D.mp = p.mp;
    D.d = p.d;
    D.i64 = p.i64;
    D.R = p.R;
    D.C = p.C;
    D.P = p.P;
    D.P_tab = p.P_tab;
    D.bias = p.bias;
    D.pfx_base = p.pfx_base;
    D.n_prefix = p.n_prefix;
    D.dpow_free = p.dpow_free;
    const uint8_t* b = (const uint8_t*)dev_blob;
    D.base = b + p.off_base;
    D.hid = b + p.off_hid;
    D.mid = b + p.off_mid;
    D.offs = b + p.off_offs;
    D.tab = (const uint64_t*)(b + p.off_tab);
    D.result = result;
    return D;
}

}  // namespace ld
