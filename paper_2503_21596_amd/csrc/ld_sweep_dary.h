// d-ary (L_d, d >= 3) register sweeps and the wide (LDS-state) sweep for gfx950.
// The shared pieces (offset-binary state, v_sad_u32, scalar-load helpers, queue
// items and result publishing) are in ld_sweep.h.
#pragma once
#include "ld_sweep.h"

namespace ld {

// ---------------------------------------------------------------------------
// d-ary kind (d >= 3): one column-sum vector per message, updated by the two-slot
// rule of Eq. (update2); only the two touched message norms are recomputed.

// The R low rows are not walked: for every message k the lane keeps
// X[k][S] = || g_k + (sum of the low rows in subset S) ||_1 for every subset S of
// the low rows (S = 0 is the plain norm).  A word of the block fixes the messages
// w of the low rows; its score is T + sum over the messages k that receive low
// rows of (X[k][S_k(w)] - X[k][0]), T = sum_k X[k][0].  A mid step changes two
// messages, so only their 2^R entries are recomputed, and the best of the d^R
// words of the block is a small max over message choices.
template <int MP, int DD, int R>
struct Dary32 {
    static constexpr int NS = 1 << R;   // subsets of the low rows
    static constexpr int RS = (MP + 15) & ~15;   // row stride of the subset operands

    __device__ static __forceinline__ uint32_t norm(const uint32_t (&g)[MP], const uint32_t (&o)[MP])
    {
        uint32_t acc = 0;
#pragma unroll
        for (int y = 0; y < MP; ++y) acc = sad_u32(g[y], o[y], acc);
        return acc;
    }

    __device__ static __forceinline__ void add_row(uint32_t (&g)[MP], uint32_t mask, cptr<int32_t> row)
    {
#pragma unroll
        for (int y = 0; y < MP; ++y) g[y] += mask & (uint32_t)row[y];
    }

    // operand of subset S >= 1: 2^31 - (sum of the low rows in S), so that
    // |g - o| = |true g + low sum|; the empty subset uses the single bias 2^31
    static constexpr int NO = NS > 1 ? NS - 1 : 1;
    __device__ static __forceinline__ void load_offs(const Desc& D, uint32_t (&off)[NO][MP])
    {
        cptr<uint32_t> o = as_const<uint32_t>(D.offs);
#pragma unroll
        for (int s = 1; s < NS; ++s)
#pragma unroll
            for (int y = 0; y < MP; ++y) off[s - 1][y] = in_vgpr(o[s * RS + y]);
    }

    __device__ static __forceinline__ uint32_t norm0(const uint32_t (&g)[MP], uint32_t bias)
    {
        uint32_t acc = 0;
#pragma unroll
        for (int y = 0; y < MP; ++y) acc = sad_u32(g[y], bias, acc);
        return acc;
    }

    __device__ static __forceinline__ void refresh(const uint32_t (&g)[MP], const uint32_t (&off)[NO][MP],
                                                   uint32_t bias, uint32_t (&X)[NS])
    {
        X[0] = norm0(g, bias);
#pragma unroll
        for (int s = 1; s < NS; ++s) X[s] = norm(g, off[s - 1]);
    }

    // best score of the d^R words of the block
    __device__ static __forceinline__ uint32_t block(const uint32_t (&X)[DD][NS])
    {
        uint32_t T = 0;
#pragma unroll
        for (int k = 0; k < DD; ++k) T += X[k][0];
        if constexpr (R == 0) {
            return T;
        } else if constexpr (R == 1) {
            int32_t b = (int32_t)(X[0][1] - X[0][0]);
#pragma unroll
            for (int k = 1; k < DD; ++k) b = max(b, (int32_t)(X[k][1] - X[k][0]));
            return T + (uint32_t)b;
        } else {
            // both low rows on one message k: X[k][3]; on two messages k != l:
            // X[k][1] - X[k][0] + X[l][2] - X[l][0]
            int32_t b = (int32_t)(X[0][3] - X[0][0]);
#pragma unroll
            for (int k = 1; k < DD; ++k) b = max(b, (int32_t)(X[k][3] - X[k][0]));
#pragma unroll
            for (int k = 0; k < DD; ++k)
#pragma unroll
                for (int l = 0; l < DD; ++l)
                    if (k != l)
                        b = max(b, (int32_t)(X[k][1] - X[k][0]) + (int32_t)(X[l][2] - X[l][0]));
            return T + (uint32_t)b;
        }
    }

    __device__ static __forceinline__ void prefix(const Desc& D, uint64_t v, const uint32_t (&off)[NO][MP],
                                                  uint32_t& best)
    {
        cptr<uint32_t> base = as_const<uint32_t>(D.base);
        cptr<int32_t> hid = as_const<int32_t>(D.hid);
        cptr<int32_t> mid = as_const<int32_t>(D.mid);
        const uint32_t bias = in_vgpr(0x80000000u);   // one register, not a constant per use
        uint32_t g[DD][MP];
#pragma unroll
        for (int y = 0; y < MP; ++y) g[0][y] = base[y];
#pragma unroll
        for (int k = 1; k < DD; ++k)
#pragma unroll
            for (int y = 0; y < MP; ++y) g[k][y] = 0x80000000u;

        uint64_t code = 0, fr = v;
        if (D.P_tab > 0) {
            const uint64_t t = v / D.dpow_free;
            fr = v - t * D.dpow_free;
            code = D.tab[t];
        }
        const int nh = D.P_tab + D.P;
        for (int h = 0; h < nh; ++h) {
            uint32_t digit;
            if (h < D.P_tab) {
                digit = (uint32_t)(code >> (4 * h)) & 15u;
            } else {
                digit = (uint32_t)(fr % DD);
                fr /= DD;
            }
            cptr<int32_t> row = hid + h * MP;
#pragma unroll
            for (int k = 0; k < DD; ++k) add_row(g[k], digit == (uint32_t)k ? 0xffffffffu : 0u, row);
        }
        uint32_t X[DD][NS];
#pragma unroll
        for (int k = 0; k < DD; ++k) refresh(g[k], off, bias, X[k]);
        best = max(best, block(X));

        uint32_t nsteps = 1;
        for (int c = 0; c < D.C; ++c) nsteps *= DD;
        for (uint32_t t = 1; t < nsteps; ++t) {
            uint32_t from, to;
            const uint32_t i = dgc_change<DD>(t, &from, &to);
            cptr<int32_t> row = mid + i * MP;
#pragma unroll
            for (int k = 0; k < DD; ++k) {
                if ((uint32_t)k == from) {
#pragma unroll
                    for (int y = 0; y < MP; ++y) g[k][y] -= (uint32_t)row[y];
                    refresh(g[k], off, bias, X[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < DD; ++k) {
                if ((uint32_t)k == to) {
#pragma unroll
                    for (int y = 0; y < MP; ++y) g[k][y] += (uint32_t)row[y];
                    refresh(g[k], off, bias, X[k]);
                }
            }
            best = max(best, block(X));
        }
    }
};

// ---------------------------------------------------------------------------
// d-ary int32 path with the subset operands streamed through SGPRs (as Bin32S):
// only the d message vectors live in VGPRs, so three low rows fit (d^3 words per
// mid step instead of d^2) for d = 3, 4.  X[k][S] = |g_k + sum of low rows in S|_1
// for every subset S; a mid step recomputes the 2^R norms of the two messages it
// touches, and the best of the block's d^R words is the maximum over every
// assignment of the low rows to messages of sum_k X[k][rows sent to k].
//
// PK = true is the packed 16-bit form (as Bin16S): MP counts dwords of two columns
// each (column 2j in bits 0..15), states and operands offset by 2^15 per half, row
// entries stored as d_2j + 2^16 d_2j+1 modulo 2^32, and one v_sad_u16 scores both
// columns of a dword.  It needs sum_x |M_xy| <= 2^15 - 1 for every column: then
// every per-message column sum, with or without low rows added, lies in
// (-2^15, 2^15), so no half ever carries into the other.
template <int MP, int DD, int R, bool PK = false, bool PAIRED = false>
struct Dary32S {
    static constexpr int NS = 1 << R;
    static constexpr int RS = (MP + 15) & ~15;
    static constexpr int N8 = (MP + 7) / 8;
    static constexpr uint32_t ZERO = PK ? 0x80008000u : 0x80000000u;   // an empty message's state
    static_assert(NS % 4 == 0, "four subset streams per group");

    __device__ static __forceinline__ uint32_t sad(uint32_t x, uint32_t o, uint32_t acc)
    {
        if constexpr (PK)
            return sad_u16_s(x, o, acc);
        else
            return sad_u32_s(x, o, acc);
    }

    // X[s] = sum_y |g_y - o_s,y| for the NS subset operands (o_0 = 2^31)
    __device__ static __forceinline__ void refresh(const uint32_t (&g)[MP], uint64_t ob, uint32_t (&X)[NS])
    {
        static_for<NS / 4>([&](auto q) {
            constexpr int s0 = 4 * q;
            uint32_t a[4] = {0, 0, 0, 0};
            static_for<N8>([&](auto c) {
                u32x8 o0, o1, o2, o3;
                sload_4x8<(s0 * RS + 8 * c) * 4, ((s0 + 1) * RS + 8 * c) * 4, ((s0 + 2) * RS + 8 * c) * 4,
                          ((s0 + 3) * RS + 8 * c) * 4>(ob, o0, o1, o2, o3);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    constexpr int y0 = 8 * c;
                    if (y0 + j >= MP) continue;
                    const uint32_t x = g[y0 + j];
                    a[0] = sad(x, o0[j], a[0]);
                    a[1] = sad(x, o1[j], a[1]);
                    a[2] = sad(x, o2[j], a[2]);
                    a[3] = sad(x, o3[j], a[3]);
                }
            });
            X[s0] = a[0];
            X[s0 + 1] = a[1];
            X[s0 + 2] = a[2];
            X[s0 + 3] = a[3];
        });
    }

    // refresh of messages KA and KB together: each statement of operand loads serves
    // both (half the scalar loads and waits of two refresh calls)
    template <int KA, int KB>
    __device__ static __forceinline__ void refresh_pair(const uint32_t (&g)[DD][MP], uint64_t ob,
                                                        uint32_t (&X)[DD][NS])
    {
        static_for<NS / 4>([&](auto q) {
            constexpr int s0 = 4 * q;
            uint32_t a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
            static_for<N8>([&](auto c) {
                u32x8 o0, o1, o2, o3;
                sload_4x8<(s0 * RS + 8 * c) * 4, ((s0 + 1) * RS + 8 * c) * 4, ((s0 + 2) * RS + 8 * c) * 4,
                          ((s0 + 3) * RS + 8 * c) * 4>(ob, o0, o1, o2, o3);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    constexpr int y0 = 8 * c;
                    if (y0 + j >= MP) continue;
                    const uint32_t x = g[KA][y0 + j], z = g[KB][y0 + j];
                    a[0] = sad(x, o0[j], a[0]);
                    a[1] = sad(x, o1[j], a[1]);
                    a[2] = sad(x, o2[j], a[2]);
                    a[3] = sad(x, o3[j], a[3]);
                    b[0] = sad(z, o0[j], b[0]);
                    b[1] = sad(z, o1[j], b[1]);
                    b[2] = sad(z, o2[j], b[2]);
                    b[3] = sad(z, o3[j], b[3]);
                }
            });
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                X[KA][s0 + i] = a[i];
                X[KB][s0 + i] = b[i];
            }
        });
    }

    // best score of the d^R words of the block: every assignment of the R low rows
    // to messages, as the subsets S_k of rows sent to each message k
    __device__ static __forceinline__ uint32_t block(const uint32_t (&X)[DD][NS])
    {
        uint32_t b = 0;
        static_for<ipow_c(DD, R)>([&](auto code) {
            uint32_t sum = 0;
            static_for<DD>([&](auto k) { sum += X[k][subset_of<code, k>()]; });
            b = max(b, sum);
        });
        return b;
    }

    // the low rows (bit j = low row j) that assignment `code` (base-DD digits)
    // sends to message k
    template <int CODE, int K>
    __device__ static constexpr int subset_of()
    {
        int s = 0, c = CODE;
        for (int j = 0; j < R; ++j) {
            if (c % DD == K) s |= 1 << j;
            c /= DD;
        }
        return s;
    }

    __device__ static __forceinline__ void prefix(const Desc& D, uint64_t v, uint32_t& best)
    {
        cptr<uint32_t> base = as_const<uint32_t>(D.base);
        cptr<int32_t> hid = as_const<int32_t>(D.hid);
        cptr<int32_t> mid = as_const<int32_t>(D.mid);
        const uint64_t ob = (uint64_t)(uintptr_t)D.offs;
        uint32_t g[DD][MP];
#pragma unroll
        for (int y = 0; y < MP; ++y) g[0][y] = base[y];
#pragma unroll
        for (int k = 1; k < DD; ++k)
#pragma unroll
            for (int y = 0; y < MP; ++y) g[k][y] = ZERO;

        uint64_t code = 0, fr = v;
        if (D.P_tab > 0) {
            const uint64_t t = v / D.dpow_free;
            fr = v - t * D.dpow_free;
            code = D.tab[t];
        }
        const int nh = D.P_tab + D.P;
        for (int h = 0; h < nh; ++h) {
            uint32_t digit;
            if (h < D.P_tab) {
                digit = (uint32_t)(code >> (4 * h)) & 15u;
            } else {
                digit = (uint32_t)(fr % DD);
                fr /= DD;
            }
            cptr<int32_t> row = hid + h * MP;
#pragma unroll
            for (int k = 0; k < DD; ++k) {
                const uint32_t mask = digit == (uint32_t)k ? 0xffffffffu : 0u;
#pragma unroll
                for (int y = 0; y < MP; ++y) g[k][y] += mask & (uint32_t)row[y];
            }
        }
        uint32_t X[DD][NS];
#pragma unroll
        for (int k = 0; k < DD; ++k) refresh(g[k], ob, X[k]);
        best = max(best, block(X));

        uint32_t nsteps = 1;
        for (int c = 0; c < D.C; ++c) nsteps *= DD;
        for (uint32_t t = 1; t < nsteps; ++t) {
            uint32_t from, to;
            const uint32_t i = dgc_change<DD>(t, &from, &to);
            cptr<int32_t> row = mid + i * MP;
            // PAIRED (d = 3 only): the reflected code moves a digit by one, so the two
            // changed messages are {0, 1} (from + to = 1) or {1, 2} (from + to = 3),
            // re-scored together
            static_assert(!PAIRED || DD == 3, "pairs by from + to need d = 3");
#pragma unroll
            for (int k = 0; k < DD; ++k) {
                if ((uint32_t)k == from) {
#pragma unroll
                    for (int y = 0; y < MP; ++y) g[k][y] -= (uint32_t)row[y];
                    if constexpr (!PAIRED) refresh(g[k], ob, X[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < DD; ++k) {
                if ((uint32_t)k == to) {
#pragma unroll
                    for (int y = 0; y < MP; ++y) g[k][y] += (uint32_t)row[y];
                    if constexpr (!PAIRED) refresh(g[k], ob, X[k]);
                }
            }
            if constexpr (PAIRED) {
                if (from + to == 1u)
                    refresh_pair<0, 1>(g, ob, X);
                else
                    refresh_pair<1, 2>(g, ob, X);
            }
            best = max(best, block(X));
        }
    }
};

template <int MP, int DD>
struct Dary64 {
    __device__ static __forceinline__ int64_t norm(const int64_t (&g)[MP])
    {
        int64_t acc = 0;
#pragma unroll
        for (int y = 0; y < MP; ++y) acc += g[y] < 0 ? -g[y] : g[y];
        return acc;
    }

    __device__ static __forceinline__ void prefix(const Desc& D, uint64_t v, int64_t& best)
    {
        cptr<int64_t> base = as_const<int64_t>(D.base);
        cptr<int64_t> hid = as_const<int64_t>(D.hid);
        cptr<int64_t> mid = as_const<int64_t>(D.mid);
        int64_t g[DD][MP];
#pragma unroll
        for (int y = 0; y < MP; ++y) g[0][y] = base[y];
#pragma unroll
        for (int k = 1; k < DD; ++k)
#pragma unroll
            for (int y = 0; y < MP; ++y) g[k][y] = 0;
        uint64_t code = 0, fr = v;
        if (D.P_tab > 0) {
            const uint64_t t = v / D.dpow_free;
            fr = v - t * D.dpow_free;
            code = D.tab[t];
        }
        const int nh = D.P_tab + D.P;
        for (int h = 0; h < nh; ++h) {
            uint32_t digit;
            if (h < D.P_tab) {
                digit = (uint32_t)(code >> (4 * h)) & 15u;
            } else {
                digit = (uint32_t)(fr % DD);
                fr /= DD;
            }
            cptr<int64_t> row = hid + h * MP;
#pragma unroll
            for (int k = 0; k < DD; ++k) {
                const int64_t mask = digit == (uint32_t)k ? -1 : 0;
#pragma unroll
                for (int y = 0; y < MP; ++y) g[k][y] += mask & row[y];
            }
        }
        int64_t N[DD];
#pragma unroll
        for (int k = 0; k < DD; ++k) N[k] = norm(g[k]);
        int64_t total = 0;
#pragma unroll
        for (int k = 0; k < DD; ++k) total += N[k];
        best = total > best ? total : best;
        uint32_t nsteps = 1;
        for (int c = 0; c < D.C; ++c) nsteps *= DD;
        for (uint32_t t = 1; t < nsteps; ++t) {
            uint32_t from, to;
            const uint32_t i = dgc_change<DD>(t, &from, &to);
            cptr<int64_t> row = mid + i * MP;
#pragma unroll
            for (int k = 0; k < DD; ++k) {
                if ((uint32_t)k == from) {
#pragma unroll
                    for (int y = 0; y < MP; ++y) g[k][y] -= row[y];
                    N[k] = norm(g[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < DD; ++k) {
                if ((uint32_t)k == to) {
#pragma unroll
                    for (int y = 0; y < MP; ++y) g[k][y] += row[y];
                    N[k] = norm(g[k]);
                }
            }
            total = 0;
#pragma unroll
            for (int k = 0; k < DD; ++k) total += N[k];
            best = total > best ? total : best;
        }
    }
};


// ---------------------------------------------------------------------------
// Wide sweep: any column count and alphabet.  One wave owns one prefix at a
// time; lane l holds columns l, l + 64, ... of every state vector in LDS (the
// entries are private to their lane, so no barrier is needed) and the score of a
// word is a wave-wide sum.  int64 throughout.  Tables use the int64 layouts with
// the row stride equal to the real column count.

__device__ __forceinline__ int64_t wave_sum(int64_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int64_t iabs64(int64_t v) { return v < 0 ? -v : v; }

struct Wide {
    // binary kinds: one state vector s
    __device__ static int64_t score_bin(const Desc& D, const int64_t* s, const int64_t* tot)
    {
        const int lane = threadIdx.x & 63;
        int64_t acc = 0;
        for (int y = lane; y < D.m; y += 64) {
            if (D.kind == KIND_L1) acc += iabs64(s[y]);
            else if (D.kind == KIND_MARG) acc += (y == 0) ? s[0] : iabs64(s[y]);
            else acc += iabs64(s[y]) + iabs64(tot[y] - s[y]);
        }
        return wave_sum(acc);
    }

    __device__ static int64_t norm(const Desc& D, const int64_t* g)
    {
        const int lane = threadIdx.x & 63;
        int64_t acc = 0;
        for (int y = lane; y < D.m; y += 64) acc += iabs64(g[y]);
        return wave_sum(acc);
    }

    __device__ static void prefix_bin(const Desc& D, uint64_t v, int64_t* s, int64_t& best)
    {
        const int lane = threadIdx.x & 63, m = D.m;
        const int64_t* base = (const int64_t*)D.base;
        const int64_t* hid = (const int64_t*)D.hid;
        const int64_t* mid = (const int64_t*)D.mid;
        const int64_t* tot = (const int64_t*)D.offs;
        for (int y = lane; y < m; y += 64) {
            int64_t a = base[y];
            for (int h = 0; h < D.P; ++h)
                if ((v >> h) & 1u) a += hid[(size_t)h * m + y];
            s[y] = a;
        }
        int64_t sc = score_bin(D, s, tot);
        best = sc > best ? sc : best;
        const uint64_t nsteps = 1ull << D.C;
        for (uint64_t t = 1; t < nsteps; ++t) {
            const uint32_t k = brgc_changed(t);
            const uint32_t g = brgc_digit(k, t);
            const int64_t* row = mid + (size_t)(2 * k + (1 - g)) * m;
            for (int y = lane; y < m; y += 64) s[y] += row[y];
            sc = score_bin(D, s, tot);
            best = sc > best ? sc : best;
        }
    }

    // d-ary: D.d state vectors g_k = LDS[k*m ...]
    __device__ static void prefix_dary(const Desc& D, uint64_t v, int64_t* g, int64_t* N, int64_t& best)
    {
        const int lane = threadIdx.x & 63, m = D.m, K = D.d;
        const int64_t* base = (const int64_t*)D.base;
        const int64_t* hid = (const int64_t*)D.hid;
        const int64_t* mid = (const int64_t*)D.mid;
        for (int y = lane; y < m; y += 64) {
            g[y] = base[y];
            for (int k = 1; k < K; ++k) g[(size_t)k * m + y] = 0;
        }
        uint64_t code = 0, fr = v;
        if (D.P_tab > 0) {
            const uint64_t t = v / D.dpow_free;
            fr = v - t * D.dpow_free;
            code = D.tab[t];
        }
        const int nh = D.P_tab + D.P;
        for (int h = 0; h < nh; ++h) {
            uint32_t digit;
            if (h < D.P_tab) {
                digit = (uint32_t)(code >> (4 * h)) & 15u;
            } else {
                digit = (uint32_t)(fr % (uint64_t)K);
                fr /= (uint64_t)K;
            }
            const int64_t* row = hid + (size_t)h * m;
            for (int y = lane; y < m; y += 64) g[(size_t)digit * m + y] += row[y];
        }
        int64_t total = 0;
        for (int k = 0; k < K; ++k) {
            N[k] = norm(D, g + (size_t)k * m);
            total += N[k];
        }
        best = total > best ? total : best;
        uint64_t nsteps = 1;
        for (int c = 0; c < D.C; ++c) nsteps *= (uint64_t)K;
        for (uint64_t t = 1; t < nsteps; ++t) {
            uint32_t from, to;
            const uint32_t i = dgc_change_rt((uint32_t)K, t, &from, &to);
            const int64_t* row = mid + (size_t)i * m;
            int64_t* gf = g + (size_t)from * m;
            int64_t* gt = g + (size_t)to * m;
            for (int y = lane; y < m; y += 64) {
                gf[y] -= row[y];
                gt[y] += row[y];
            }
            const int64_t nf = norm(D, gf), nt = norm(D, gt);
            total += (nf - N[from]) + (nt - N[to]);
            N[from] = nf;
            N[to] = nt;
            best = total > best ? total : best;
        }
    }
};

}  // namespace ld
