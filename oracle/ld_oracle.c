/*
 * CPU oracle for the L_d norms of an integer matrix -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  It shares no code with the GPU library: it enumerates
 * every assignment by plain binary / base-d counting (no Gray code, no incremental
 * state) and evaluates each definition from scratch in int64.
 *
 * Definitions followed (Marton, Bene, Divianszky, Drotos, arXiv:2503.21596):
 *   L1     -- Eq. (LM2):  max over a in {+-1}^n of sum_y |sum_x a_x M_xy|
 *   L_marg -- Eq. (LMarg): a_1 fixed to +1, column 1 enters linearly,
 *             the other columns in absolute value.
 *   L_d    -- Eqs. (L_o_norm), (ma): max over a in {0..d-1}^n of
 *             sum_k sum_y |sum_{x: a_x = k} M_xy|.
 * Symmetry reductions used (Sec. 2.1.2 for L1, Sec. 2.3.2 for L_d):
 *   L1 is unchanged under a -> -a, so row 0 is fixed to +1;
 *   L_marg fixes row 0 to +1 by its own definition;
 *   L_d is unchanged under relabelling of the messages, so row 0 is fixed to 0
 *   (oracle_ld), or only one assignment per relabelling class is scored
 *   (oracle_ld_classes, for alphabets too large for d^(n-1) assignments).
 * The *_all variants fix nothing and enumerate all 2^n / d^n assignments; tests
 * use them to pin the symmetry reductions.
 *
 * Matrices are int32, row-major, M[x*m + y].  Every sum is int64.
 * An empty matrix (n == 0 or m == 0) has value 0.
 *
 * Parity status of every function is pinned by tests/test_oracle_pins.py
 * (printed values of the worked example, closed forms, brute force over both
 * parties, invariances); oracle_l1_split and oracle_ld_split are pinned by
 * agreement with oracle_l1 / oracle_lmarg / oracle_ld on inputs small enough for
 * both and large enough that several tiles of both tables, and ragged thread
 * ranges, are visited; oracle_ld_classes by agreement with oracle_ld and
 * oracle_ld_all, and its class count by the Stirling numbers of the second kind.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#include "ld_oracle.h"

static int64_t iabs64(int64_t v) { return v < 0 ? -v : v; }

/* ------------------------------------------------------------------ */
/* thread pool helper: split [0, total) into nthreads contiguous ranges */

typedef struct {
    const int32_t* M;
    int n, m, d, marg;
    int q;             /* range mode: number of trailing prefix rows (0 = none) */
    uint64_t pfx;      /* range mode: the prefix value of the trailing rows     */
    uint64_t lo, hi;   /* counter range handled by this thread                  */
    int fix;           /* 1: row 0 fixed (+1 for binary, 0 for d-ary)          */
    int64_t best;
} job_t;

/* Binary score of one sign vector given by `a` (values +1/-1), Eq. (LM2) or
 * Eq. (LMarg). */
static int64_t score_binary(const int32_t* M, int n, int m, const int8_t* a, int marg)
{
    int64_t total = 0;
    for (int y = 0; y < m; ++y) {
        int64_t s = 0;
        for (int x = 0; x < n; ++x) s += (int64_t)a[x] * (int64_t)M[(size_t)x * m + y];
        if (marg && y == 0) total += s;
        else total += iabs64(s);
    }
    return total;
}

/* d-ary score of one assignment `a` (values 0..d-1), Eqs. (L_o_norm), (ma). */
static int64_t score_dary(const int32_t* M, int n, int m, int d, const int8_t* a)
{
    int64_t total = 0;
    for (int k = 0; k < d; ++k) {
        for (int y = 0; y < m; ++y) {
            int64_t g = 0;
            for (int x = 0; x < n; ++x)
                if (a[x] == k) g += M[(size_t)x * m + y];
            total += iabs64(g);
        }
    }
    return total;
}

/* Decode counter value `c` into raw digits (0..radix-1) of the free rows
 * [first, n - q); the trailing q rows receive the digits of `pfx`. */
static void decode(int8_t* digit, int n, int radix, int first, int q, uint64_t pfx, uint64_t c)
{
    for (int x = first; x < n - q; ++x) {
        digit[x] = (int8_t)(c % (uint64_t)radix);
        c /= (uint64_t)radix;
    }
    for (int i = 0; i < q; ++i) {
        digit[n - q + i] = (int8_t)(pfx % (uint64_t)radix);
        pfx /= (uint64_t)radix;
    }
}

static void* worker(void* arg)
{
    job_t* j = (job_t*)arg;
    int8_t digit[256], a[256];
    const int binary = (j->d == 1);
    const int radix = binary ? 2 : j->d;
    const int first = j->fix ? 1 : 0;
    /* the fixed row: digit 1 (a = +1) for the binary problems, message 0 for L_d */
    if (j->fix) digit[0] = (int8_t)(binary ? 1 : 0);
    int64_t best = INT64_MIN;
    for (uint64_t c = j->lo; c < j->hi; ++c) {
        decode(digit, j->n, radix, first, j->q, j->pfx, c);
        int64_t v;
        if (binary) {
            for (int x = 0; x < j->n; ++x) a[x] = (int8_t)(digit[x] ? 1 : -1);
            v = score_binary(j->M, j->n, j->m, a, j->marg);
        } else {
            v = score_dary(j->M, j->n, j->m, j->d, digit);
        }
        if (v > best) best = v;
    }
    j->best = best;
    return NULL;
}

static uint64_t ipow(uint64_t b, int e)
{
    uint64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

/* Run the enumeration over `count` counter values split across threads. */
static int64_t run_jobs(const int32_t* M, int n, int m, int d, int marg, int fix,
                        int q, uint64_t pfx, uint64_t count, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((uint64_t)nthreads > count) nthreads = (int)(count ? count : 1);
    job_t jobs[256];
    pthread_t th[256];
    uint64_t per = count / (uint64_t)nthreads, rem = count % (uint64_t)nthreads, at = 0;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t len = per + ((uint64_t)t < rem ? 1 : 0);
        jobs[t] = (job_t){M, n, m, d, marg, q, pfx, at, at + len, fix, INT64_MIN};
        at += len;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, worker, &jobs[t]);
    worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    int64_t best = INT64_MIN;
    for (int t = 0; t < nthreads; ++t)
        if (jobs[t].best > best) best = jobs[t].best;
    return best;
}

/* ------------------------------------------------------------------ */
/* public entry points                                                 */

int64_t oracle_l1(const int32_t* M, int n, int m, int nthreads)
{
    if (n <= 0 || m <= 0) return 0;
    if (n > 64) return INT64_MIN;
    return run_jobs(M, n, m, 1, 0, 1, 0, 0, (uint64_t)1 << (n - 1), nthreads);
}

int64_t oracle_l1_all(const int32_t* M, int n, int m, int nthreads)
{
    if (n <= 0 || m <= 0) return 0;
    if (n > 63) return INT64_MIN;
    return run_jobs(M, n, m, 1, 0, 0, 0, 0, (uint64_t)1 << n, nthreads);
}

int64_t oracle_lmarg(const int32_t* M, int n, int m, int nthreads)
{
    if (n <= 0 || m <= 0) return 0;
    if (n > 64) return INT64_MIN;
    return run_jobs(M, n, m, 1, 1, 1, 0, 0, (uint64_t)1 << (n - 1), nthreads);
}

int64_t oracle_ld(const int32_t* M, int n, int m, int d, int nthreads)
{
    if (n <= 0 || m <= 0) return 0;
    if (d < 2) return INT64_MIN;
    return run_jobs(M, n, m, d, 0, 1, 0, 0, ipow((uint64_t)d, n - 1), nthreads);
}

int64_t oracle_ld_all(const int32_t* M, int n, int m, int d, int nthreads)
{
    if (n <= 0 || m <= 0) return 0;
    if (d < 2) return INT64_MIN;
    return run_jobs(M, n, m, d, 0, 0, 0, 0, ipow((uint64_t)d, n), nthreads);
}

/* Max over the assignments whose trailing q rows carry a prefix value in
 * [pfx_begin, pfx_end): for d == 1 bit i of the prefix set to 1 means
 * a_{n-q+i} = +1 (0 means -1); for d >= 2 digit i (base d) of the prefix is
 * a_{n-q+i}.  Row 0 is fixed as in the full functions and rows 1 .. n-q-1 are
 * free.  Returns INT64_MIN for an empty prefix range. */
int64_t oracle_range(const int32_t* M, int n, int m, int d, int marg, int q,
                     uint64_t pfx_begin, uint64_t pfx_end, int nthreads)
{
    if (n <= 0 || m <= 0) return 0;
    if (q < 0 || q > n - 1) return INT64_MIN;
    int radix = (d == 1) ? 2 : d;
    uint64_t inner = ipow((uint64_t)radix, n - 1 - q);
    int64_t best = INT64_MIN;
    for (uint64_t p = pfx_begin; p < pfx_end; ++p) {
        int64_t v = run_jobs(M, n, m, d, marg, 1, q, p, inner, nthreads);
        if (v > best) best = v;
    }
    return best;
}

/* ------------------------------------------------------------------ */
/* Split-table direct enumeration for large binary problems.
 *
 * Still evaluates Eq. (LM2) / Eq. (LMarg) for every sign vector with row 0
 * fixed to +1: the free rows 1..n-1 are split into a lower half A and an upper
 * half B, the partial column sums of each half are tabulated for every sign
 * pattern of that half (row 0 included in A's table), and the column sums of a
 * full sign vector are formed as TA[p] + TB[q] for every pair (p, q) before the
 * score is taken.  Sums are int64 throughout.                               */

typedef struct {
    const int64_t* TA; const int64_t* TB;
    uint64_t na, nb_lo, nb_hi;
    int m, marg;
    int64_t best;
} split_job_t;

/* Every pair (p, q) is scored exactly once.  The pairs are visited tile by tile
 * (TILE_Q values of q against TILE_P values of p) so that the rows of both
 * tables in use stay in cache; the order of a maximum does not matter. */
#define TILE_P 512
#define TILE_Q 64

static void* split_worker(void* arg)
{
    split_job_t* j = (split_job_t*)arg;
    const int m = j->m;
    int64_t best = INT64_MIN;
    for (uint64_t q0 = j->nb_lo; q0 < j->nb_hi; q0 += TILE_Q) {
        const uint64_t q1 = q0 + TILE_Q < j->nb_hi ? q0 + TILE_Q : j->nb_hi;
        for (uint64_t p0 = 0; p0 < j->na; p0 += TILE_P) {
            const uint64_t p1 = p0 + TILE_P < j->na ? p0 + TILE_P : j->na;
            for (uint64_t q = q0; q < q1; ++q) {
                const int64_t* tb = j->TB + q * (uint64_t)m;
                for (uint64_t p = p0; p < p1; ++p) {
                    const int64_t* ta = j->TA + p * (uint64_t)m;
                    int64_t total = 0;
                    if (j->marg) {
                        total = ta[0] + tb[0];
                        for (int y = 1; y < m; ++y) total += iabs64(ta[y] + tb[y]);
                    } else {
                        for (int y = 0; y < m; ++y) total += iabs64(ta[y] + tb[y]);
                    }
                    if (total > best) best = total;
                }
            }
        }
    }
    j->best = best;
    return NULL;
}

/* Tabulate sum over rows r0..r0+k-1 of sign(bit)*M_r for every k-bit pattern,
 * plus `extra` (row 0 with +1 when non-NULL). */
static void tabulate(int64_t* T, const int32_t* M, int m, int r0, int k, const int32_t* extra)
{
    uint64_t cnt = (uint64_t)1 << k;
    for (uint64_t p = 0; p < cnt; ++p) {
        int64_t* t = T + p * (uint64_t)m;
        for (int y = 0; y < m; ++y) t[y] = extra ? extra[y] : 0;
        for (int i = 0; i < k; ++i) {
            const int32_t* row = M + (size_t)(r0 + i) * m;
            int sgn = ((p >> i) & 1u) ? 1 : -1;
            for (int y = 0; y < m; ++y) t[y] += (int64_t)sgn * row[y];
        }
    }
}

int64_t oracle_l1_split(const int32_t* M, int n, int m, int marg, int nthreads)
{
    if (n <= 0 || m <= 0) return 0;
    if (n > 64 || n < 2) return marg ? oracle_lmarg(M, n, m, nthreads) : oracle_l1(M, n, m, nthreads);
    int f = n - 1;            /* free rows 1..n-1 */
    int ka = f / 2, kb = f - ka;
    uint64_t na = (uint64_t)1 << ka, nb = (uint64_t)1 << kb;
    int64_t* TA = (int64_t*)malloc(na * (uint64_t)m * sizeof(int64_t));
    int64_t* TB = (int64_t*)malloc(nb * (uint64_t)m * sizeof(int64_t));
    if (!TA || !TB) { free(TA); free(TB); return INT64_MIN; }
    tabulate(TA, M, m, 1, ka, M /* row 0 with +1 */);
    tabulate(TB, M, m, 1 + ka, kb, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((uint64_t)nthreads > nb) nthreads = (int)nb;
    split_job_t jobs[256];
    pthread_t th[256];
    uint64_t per = nb / (uint64_t)nthreads, rem = nb % (uint64_t)nthreads, at = 0;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t len = per + ((uint64_t)t < rem ? 1 : 0);
        jobs[t] = (split_job_t){TA, TB, na, at, at + len, m, marg, INT64_MIN};
        at += len;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, split_worker, &jobs[t]);
    split_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    int64_t best = INT64_MIN;
    for (int t = 0; t < nthreads; ++t)
        if (jobs[t].best > best) best = jobs[t].best;
    free(TA); free(TB);
    return best;
}

/* ------------------------------------------------------------------ */
/* L_d over one assignment per relabelling class.
 *
 * Eq. (L_o_norm) is unchanged when the d messages are permuted, so every
 * assignment has the value of the one whose messages appear in first-use order:
 * a_0 = 0 and each a_x at most one above max(a_0 .. a_{x-1}) (a restricted-growth
 * string).  These strings are walked in lexicographic order; string number c is
 * scored by thread c mod nthreads, each with the plain per-assignment score. */

/* next restricted-growth string after a[0..n-1] with digits below d; 0 when a is
 * the last one */
static int rgs_next(int8_t* a, int n, int d)
{
    for (int i = n - 1; i >= 1; --i) {
        int mx = 0;
        for (int k = 0; k < i; ++k)
            if (a[k] > mx) mx = a[k];
        const int top = mx + 1 < d - 1 ? mx + 1 : d - 1;
        if (a[i] < top) {
            ++a[i];
            for (int k = i + 1; k < n; ++k) a[k] = 0;
            return 1;
        }
    }
    return 0;
}

typedef struct {
    const int32_t* M;
    int n, m, d, t, nthreads;
    int64_t best;
    uint64_t count;
} cls_job_t;

static void* cls_worker(void* arg)
{
    cls_job_t* j = (cls_job_t*)arg;
    int8_t a[256];
    memset(a, 0, sizeof a);
    int64_t best = INT64_MIN;
    uint64_t c = 0, mine = 0;
    do {
        if (c % (uint64_t)j->nthreads == (uint64_t)j->t) {
            const int64_t v = j->M ? score_dary(j->M, j->n, j->m, j->d, a) : 0;
            if (v > best) best = v;
            ++mine;
        }
        ++c;
    } while (rgs_next(a, j->n, j->d));
    j->best = best;
    j->count = mine;
    return NULL;
}

static int64_t run_classes(const int32_t* M, int n, int m, int d, int nthreads, uint64_t* count)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    cls_job_t jobs[256];
    pthread_t th[256];
    for (int t = 0; t < nthreads; ++t) jobs[t] = (cls_job_t){M, n, m, d, t, nthreads, INT64_MIN, 0};
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, cls_worker, &jobs[t]);
    cls_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    int64_t best = INT64_MIN;
    uint64_t total = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (jobs[t].best > best) best = jobs[t].best;
        total += jobs[t].count;
    }
    if (count) *count = total;
    return best;
}

int64_t oracle_ld_classes(const int32_t* M, int n, int m, int d, int nthreads)
{
    if (n <= 0 || m <= 0) return 0;
    if (d < 2 || n > 256) return INT64_MIN;
    return run_classes(M, n, m, d, nthreads, NULL);
}

/* number of restricted-growth strings of length n with digits below d, counted by
 * the same walk (the number of relabelling classes) */
uint64_t oracle_rgs_count(int n, int d)
{
    if (n <= 0 || d < 1 || n > 256) return 0;
    uint64_t cnt = 0;
    run_classes(NULL, n, 1, d, 1, &cnt);
    return cnt;
}

/* ------------------------------------------------------------------ */
/* Split-table direct enumeration for L_d, d >= 2 (Eqs. (L_o_norm), (ma)).
 *
 * Still evaluates the definition for every assignment with row 0 fixed to
 * message 0: the free rows 1..n-1 are split into a lower half A and an upper
 * half B.  For every assignment p of A's rows (a base-d counter) the table
 * TA[p][k][y] holds the column sums of the rows sent to message k, row 0
 * included; TB[q][k][y] holds the same for B's rows.  The per-message column
 * sums of the full assignment (p, q) are TA[p][k][y] + TB[q][k][y], and its
 * value is the sum over k and y of their absolute values.  int64 throughout. */

typedef struct {
    const int64_t* TA; const int64_t* TB;
    uint64_t na, nb_lo, nb_hi;
    int w;             /* d * m entries per table row */
    int64_t best;
} ldsplit_job_t;

static void* ldsplit_worker(void* arg)
{
    ldsplit_job_t* j = (ldsplit_job_t*)arg;
    const int w = j->w;
    int64_t best = INT64_MIN;
    for (uint64_t q0 = j->nb_lo; q0 < j->nb_hi; q0 += TILE_Q) {
        const uint64_t q1 = q0 + TILE_Q < j->nb_hi ? q0 + TILE_Q : j->nb_hi;
        for (uint64_t p0 = 0; p0 < j->na; p0 += TILE_P) {
            const uint64_t p1 = p0 + TILE_P < j->na ? p0 + TILE_P : j->na;
            for (uint64_t q = q0; q < q1; ++q) {
                const int64_t* tb = j->TB + q * (uint64_t)w;
                for (uint64_t p = p0; p < p1; ++p) {
                    const int64_t* ta = j->TA + p * (uint64_t)w;
                    int64_t total = 0;
                    for (int e = 0; e < w; ++e) total += iabs64(ta[e] + tb[e]);
                    if (total > best) best = total;
                }
            }
        }
    }
    j->best = best;
    return NULL;
}

/* Tabulate, for every assignment of rows r0..r0+k-1 to messages (digit i of the
 * base-d counter p is the message of row r0+i), the per-message column sums
 * T[p][msg][y]; with with_row0 set, row 0 is added to message 0. */
static void tabulate_dary(int64_t* T, const int32_t* M, int m, int d, int r0, int k, int with_row0)
{
    const uint64_t cnt = ipow((uint64_t)d, k);
    const int w = d * m;
    for (uint64_t p = 0; p < cnt; ++p) {
        int64_t* t = T + p * (uint64_t)w;
        for (int e = 0; e < w; ++e) t[e] = 0;
        if (with_row0)
            for (int y = 0; y < m; ++y) t[y] += M[y];
        uint64_t c = p;
        for (int i = 0; i < k; ++i) {
            const int msg = (int)(c % (uint64_t)d);
            c /= (uint64_t)d;
            const int32_t* row = M + (size_t)(r0 + i) * m;
            for (int y = 0; y < m; ++y) t[(size_t)msg * m + y] += row[y];
        }
    }
}

int64_t oracle_ld_split(const int32_t* M, int n, int m, int d, int nthreads)
{
    if (n <= 0 || m <= 0) return 0;
    if (d < 2) return INT64_MIN;
    const int f = n - 1;      /* free rows 1..n-1 */
    const int ka = f / 2, kb = f - ka;
    const uint64_t na = ipow((uint64_t)d, ka), nb = ipow((uint64_t)d, kb);
    const int w = d * m;
    int64_t* TA = (int64_t*)malloc(na * (uint64_t)w * sizeof(int64_t));
    int64_t* TB = (int64_t*)malloc(nb * (uint64_t)w * sizeof(int64_t));
    if (!TA || !TB) { free(TA); free(TB); return INT64_MIN; }
    tabulate_dary(TA, M, m, d, 1, ka, 1);
    tabulate_dary(TB, M, m, d, 1 + ka, kb, 0);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((uint64_t)nthreads > nb) nthreads = (int)nb;
    ldsplit_job_t jobs[256];
    pthread_t th[256];
    uint64_t per = nb / (uint64_t)nthreads, rem = nb % (uint64_t)nthreads, at = 0;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t len = per + ((uint64_t)t < rem ? 1 : 0);
        jobs[t] = (ldsplit_job_t){TA, TB, na, at, at + len, w, INT64_MIN};
        at += len;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, ldsplit_worker, &jobs[t]);
    ldsplit_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    int64_t best = INT64_MIN;
    for (int t = 0; t < nthreads; ++t)
        if (jobs[t].best > best) best = jobs[t].best;
    free(TA); free(TB);
    return best;
}

/* Value of one given assignment: Eq. (LM2)/(LMarg) when d == 1 (a_x = +-1),
 * Eq. (L_o_norm) when d >= 2 (a_x in 0..d-1).  Used to test attainment. */
int64_t oracle_value_of(const int32_t* M, int n, int m, int d, int marg, const int8_t* a)
{
    if (n <= 0 || m <= 0) return 0;
    if (d == 1) return score_binary(M, n, m, a, marg);
    return score_dary(M, n, m, d, a);
}
