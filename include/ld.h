/*
 * ld.h -- C ABI of the MI355X (gfx950) L_d-norm library.
 *
 * The library computes, by exhaustive Gray-code search on the GPU, the quantities
 * defined in Marton, Bene, Divianszky, Drotos, arXiv:2503.21596:
 *
 *   d = 1, marginals = 0   L1(M)     = max_{a in {+-1}^n} sum_y |sum_x a_x M_xy|
 *                          the local bound of a correlation Bell expression, Eq. (LM2)
 *   d = 1, marginals = 1   L_marg(M) = max_{a_0 = +1, a_x = +-1}
 *                          ( sum_x a_x M_x0 + sum_{y>=1} |sum_x a_x M_xy| ),  Eq. (LMarg)
 *                          (row 0 and column 0 carry the marginal coefficients)
 *   d >= 2                 L_d(M)    = max_{a in {0..d-1}^n} sum_k sum_y |sum_{x: a_x=k} M_xy|
 *                          the classical d-dimensional bound of a prepare-and-measure
 *                          witness, Eqs. (L_o_norm), (ma).  d = 1 never means this
 *                          formula (the paper notes Eq. (LM2) is not its d = 1 case).
 *
 * Matrices: int32, row-major, M[x*m + y] (x = row, y = column), host memory owned by
 * the caller, read during the call only (the library copies what it needs).  The
 * paper requires integer entries; convert real coefficients before calling.
 *
 * Values are exact int64.  |value| <= sum |M_xy| < 2^63, so INT64_MIN is never a
 * value and marks an error; ld_last_error() then gives the code.  L_marg may be
 * negative (M = [[-5]] gives -5), so no negative number can serve as an error code.
 *
 * Thread safety: every entry point may be called from several host threads at
 * once; each thread uses its own HIP stream and device buffers.
 */
#ifndef LD_H
#define LD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes (0 = success) */
#define LD_OK 0
#define LD_EINVAL 1      /* null M, n < 1, m < 1, d < 1, marginals not 0/1, bad range   */
#define LD_EMARG_D 2     /* marginals with d >= 2: the paper defines them for L1 only   */
#define LD_ETOOBIG 3     /* search space over 2^62 words after symmetry removal, or a
                            shape no register-resident kernel covers (see ld_plan)       */
#define LD_EHIP 4        /* HIP runtime error or no usable gfx950 device                */
#define LD_EBUSY 5       /* server: arena or queue full, retry later                     */
#define LD_PENDING 6     /* server: result not ready yet                                  */
#define LD_ENOTFOUND 7   /* server: unknown ticket                                        */
#define LD_ECANCELED 8   /* server: request cancelled before it completed                 */
#define LD_ESCRATCH 9    /* ld_norm_noalloc: the problem's device image exceeds the static
                            scratch array (LD_NOALLOC_SCRATCH_BYTES)                      */

/* ld_norm -- L1 / L_marg / L_d of one matrix (definitions above).
 * Preprocessing keeps the value exactly: all-zero rows and columns are dropped
 * (Sec. 2.1.1, 2.2, 2.3.1), L1 and L_marg are computed on the transpose when
 * n > m (Sec. 2.1.1; for L_marg the marginal row and column swap roles), and
 * for d >= 2 with d >= (remaining rows) the value is sum |M_xy|.
 * Synchronous: returns after the result is on the host.
 * Returns the value, or INT64_MIN with ld_last_error() set. */
int64_t ld_norm(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals);

/* ld_norm_noalloc -- ld_norm for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same planning, kernels and value as ld_norm.  The problem's device
 * image (tables, descriptor, queue head, result slot) is placed in a static
 * device array of LD_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds
 * from load until the process ends; the call makes no hipMalloc, hipFree or
 * hipHostMalloc.  A problem whose image exceeds the array (far beyond the
 * register-kernel shapes: the wide kernel's int64 tables of about a million
 * entries) fails with LD_ESCRATCH before anything is launched.
 * M: host, row-major n x m, read during the call.  value: host pointer receiving
 * the result (INT64_MIN on error).  hip_stream: a hipStream_t, or NULL for the
 * null stream; the call returns after the result is on the host.  Every call on a
 * GPU uses that GPU's one array and overwrites it (the queue head and result slot
 * are reset by a kernel each call); calls in one process take turns on a lock per
 * device, so they do not overlap.  Returns LD_OK or an error code, also in
 * ld_last_error(). */
#define LD_NOALLOC_SCRATCH_BYTES (1u << 20)
int ld_norm_noalloc(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals, int64_t* value,
                    void* hip_stream);

/* One problem of a batch. */
typedef struct {
    const int32_t* M;     /* host, row-major n x m, caller-owned */
    int32_t n, m, d, marginals;
} ld_problem;

/* ld_norm_batch -- many independent problems, same values as ld_norm each.
 * The problems are planned on host threads, packed into one device image and
 * swept by persistent work-queue launches (one per kernel shape) whose waves pull
 * (problem, prefix range) items, longest first, until the queue is empty.
 * out[i] receives problem i's value, or INT64_MIN on error; status (nullable)
 * receives each problem's error code.  hip_stream: a hipStream_t, or NULL for
 * the library's own stream; with a caller stream the call still returns after
 * the results are in out[].  Returns LD_OK, or the first error code met. */
int ld_norm_batch(const ld_problem* probs, int32_t count, int64_t* out, int32_t* status,
                  void* hip_stream);

/* Reusable batch: ld_batch_prepare plans and uploads the problems once (the
 * matrices are not retained) and captures the reset, the queue launches and the
 * result copy in a HIP graph; ld_batch_run replays it on hip_stream (NULL: the
 * handle's stream), waits, and writes count values to out (INT64_MIN and an
 * error return for problems that failed to plan).  ld_batch_last_ms: device time
 * of the last run (HIP events around the graph).  One thread at a time per handle. */
typedef struct ld_batch ld_batch;
ld_batch* ld_batch_prepare(const ld_problem* probs, int32_t count, int32_t* status);
int ld_batch_run(ld_batch* b, void* hip_stream, int64_t* out);
float ld_batch_last_ms(ld_batch* b);
void ld_batch_release(ld_batch* b);

/* ld_norm_range -- the maximum over part of the search space, for spot checks
 * at full size.  No preprocessing.  Row 0 is fixed (a_0 = +1 for d = 1, message
 * 0 for d >= 2), the last q rows are set by a prefix value p in
 * [prefix_begin, prefix_end): for d = 1 bit i of p is 1 when a_{n-q+i} = +1; for
 * d >= 2 digit i (base d) of p is the message of row n-q+i.  Rows 1 .. n-q-1
 * are free.  Returns INT64_MIN on error (empty range: LD_EINVAL). */
int64_t ld_norm_range(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals,
                      int32_t q, uint64_t prefix_begin, uint64_t prefix_end);

/* ld_norm_resumable -- a long solve that survives interruption (a multi-hour
 * d = 3 problem, a preemptible job).  The search space of ld_norm's plan is swept
 * in chunks of about chunk_seconds; after every chunk the best value so far and
 * the next prefix are written to state_path (a text file, replaced atomically
 * through state_path + ".tmp").  If state_path holds the state of the same matrix,
 * kind and plan, the sweep continues where it stopped; any other content is
 * overwritten and the sweep starts over.  Returns LD_OK with *value once the whole
 * space has been swept (the value equals ld_norm's), or LD_PENDING when
 * max_seconds have passed (the state is saved: call again to continue), or an
 * error code (LD_EINVAL also when the state file cannot be written). */
int ld_norm_resumable(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals,
                      const char* state_path, double chunk_seconds, double max_seconds, int64_t* value);

/* ld_argmax -- the value together with one assignment that reaches it (the
 * strategy the paper's program reports next to the value, Sec. 2.1.3).
 * assignment (n entries, caller-owned): d = 1: a_x in {-1, +1} for every row
 * (a_0 = +1 with marginals, Eq. (LMarg)); d >= 2: the message of every row in
 * {0 .. d-1} (Eq. (L_o_norm)).  col_assignment (m entries, nullable, d = 1 only):
 * column signs b_y with a^T M b = value (b_0 = +1 with marginals).  Among
 * several maximisers the one returned is unspecified; it always attains *value.
 * Cost: the sweep of ld_norm plus one store per prefix and a few small
 * refinement sweeps.  Returns LD_OK or an error code (as ld_norm's). */
int ld_argmax(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals, int64_t* value,
              int32_t* assignment, int32_t* col_assignment);

/* How a problem is laid out for the sweep.  kind: 0 L1, 1 L_marg, 2 L2, 3 L_d
 * (d >= 3), 4 sum|M| (d >= rows), 5 constant zero (empty after preprocessing). */
typedef struct {
    int32_t kind;
    int32_t n, m, d;      /* after preprocessing */
    int32_t transposed;
    int32_t i64;          /* 1: int64 path (sum |M_xy| >= 2^31) */
    int32_t mp;           /* padded column count of the kernel instantiation */
    int32_t R, C, P;      /* low (patterns per state), mid (Gray), high (prefix) rows */
    int32_t P_tab;        /* d-ary rows covered by restricted-growth prefixes */
    uint64_t n_prefix;    /* prefixes, i.e. lane-sized work units */
    double words;         /* assignments scored */
    int32_t kernel;       /* sweep kernel: 0 VGPR operands, 1 SGPR operands, 2 int8-MFMA
                             state update, 3 int64, 4 wide (LDS state), 5 packed 16-bit
                             (two columns per register), -1 none */
    int32_t reserved;
} ld_plan_info;

/* ---------------------------------------------------------------------------
 * Prepared problems: plan once, keep the tables resident in HBM, run many times.
 * ld_prepare plans M as ld_norm does and copies its tables to the current
 * device (synchronously); M is not retained.  Returns NULL on error.
 * ld_run enqueues the sweep on hip_stream (a hipStream_t, or NULL for a stream
 * owned by the handle), copies the 8-byte result back and waits for it.
 * The sweep kernel is bracketed by two HIP events on that stream;
 * ld_last_kernel_ms gives the time between them for the last ld_run.
 * A handle is used by one thread at a time; ld_release frees it. */
typedef struct ld_prepared ld_prepared;
ld_prepared* ld_prepare(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals);
int ld_run(ld_prepared* h, void* hip_stream, int64_t* value);
float ld_last_kernel_ms(ld_prepared* h);
int ld_prepared_plan(const ld_prepared* h, ld_plan_info* info);
void ld_release(ld_prepared* h);

/* Error code of the calling thread's last failed call, and its text. */
int ld_last_error(void);
const char* ld_error_string(int code);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of L_d solves on one GPU.
 *
 * A scheduler thread owns the device.  Requests are admitted while the arena
 * (device bytes for their tables) and the in-flight slots allow; each admitted
 * problem's tables are uploaded once and its prefix space is cut into queue
 * items.  The scheduler issues short steps -- queue launches over items chosen
 * smallest-remaining-work first, about step_ms of device work each, at most two
 * steps in flight -- so a request that arrives while others run joins at the next
 * step.  Partial maxima stay in device result slots between steps; a request is
 * complete when all its items have run.  Values equal ld_norm's. */
typedef struct {
    uint64_t arena_bytes;           /* device bytes for problem tables (0: 256 MiB)        */
    int32_t max_inflight_problems;  /* result slots (0: 1024)                              */
    int32_t max_items_per_launch;   /* cap on one step's items (0: 65536)                  */
    double words_per_item;          /* queue-item size (0: 2^17 words)                      */
    double step_ms;                 /* device work per bulk step (0: 4 ms)                  */
    int32_t max_queued;             /* submitted but not admitted; beyond: LD_EBUSY (0: 65536) */
    int32_t device;                 /* HIP device index                                     */
    double express_ms;              /* requests below this estimated device time take the
                                       express lane (0: 1 ms; negative: no express lane)    */
    double idle_spin_ms;            /* an idle scheduler polls for arrivals this long before
                                       it sleeps, keeping one host thread busy (0: 50 ms;
                                       negative: it sleeps at once)                          */
    int32_t min_items;              /* a request with that many 64-lane pieces is cut into at
                                       least this many queue items, so that a small request
                                       spreads over the device (0: 4096; negative: no floor,
                                       items of words_per_item only)                          */
} ld_server_config;

typedef struct {
    uint64_t submitted, completed, rejected, launches, items;
    int32_t inflight, queued;
    double p50_ms, p99_ms, mean_ms;  /* latency: submit -> completion seen by the scheduler */
    double mean_wait_ms;             /* mean of submit -> first step issued                  */
    double mean_plan_ms;             /* mean of submit -> queued (planning, submitting thread) */
    double mean_run_ms;              /* mean of first step issued -> completion               */
} ld_stats;

typedef struct ld_server ld_server;
/* NULL on error (ld_last_error). cfg may be NULL for the defaults. */
ld_server* ld_server_create(const ld_server_config* cfg);
/* Copies M; plans on the calling thread.  *ticket identifies the request.  Returns
 * LD_OK, LD_EBUSY (queue full; nothing stored), or a planning error (the ticket
 * then completes at once with that error). */
int ld_server_submit(ld_server* s, const ld_problem* p, uint64_t* ticket);
/* LD_PENDING until the request completes; then its status (LD_OK: *value set).
 * A completed ticket can be read any number of times until the server is destroyed. */
int ld_server_poll(ld_server* s, uint64_t ticket, int64_t* value);
int ld_server_wait(ld_server* s, uint64_t ticket, int64_t* value);
/* Cancel a queued or in-flight request (its remaining items are dropped). */
int ld_server_cancel(ld_server* s, uint64_t ticket);
void ld_server_stats(ld_server* s, ld_stats* out);
/* Per-request latency split of completed requests (status LD_OK), oldest first:
 * where a request's time went between submission and completion. */
typedef struct {
    uint64_t ticket;
    int32_t lane;      /* 0 bulk, 1 express                                           */
    int32_t items;     /* queue items the request was cut into                        */
    double words;      /* assignments its sweep scores                                 */
    double plan_ms;    /* submit -> queued: planning on the submitting thread          */
    double wait_ms;    /* queued -> first step with its items issued                   */
    double run_ms;     /* that step issued -> completion seen by the scheduler         */
} ld_request_timing;
/* Copies the timings of the first `max` completed requests (at most the last 2^20 are
 * kept) to out; returns how many it wrote, or -1 for a null server. */
int32_t ld_server_timings(ld_server* s, ld_request_timing* out, int32_t max);
/* Drains in-flight steps, stops the scheduler, frees the device memory. */
void ld_server_destroy(ld_server* s);

/* ---------------------------------------------------------------------------
 * Introspection (host only, never touches the GPU). */


/* Plan a problem as ld_norm would.  Returns LD_OK or an error code. */
int ld_plan(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals,
            ld_plan_info* info);

/* Plan a problem as ld_norm_batch and ld_batch_prepare plan each member (the
 * batch sweep shape: tuned words per prefix and prefix cap per problem).
 * Returns LD_OK or an error code. */
int ld_plan_batch(const int32_t* M, int32_t n, int32_t m, int32_t d, int32_t marginals,
                  ld_plan_info* info);

/* Gray-code digits as the kernels compute them (Sec. 2.1.2, 2.3.2).
 * ld_gray_digit: digit i of word j of the d-ary reflected Gray code (d = 2: the
 * binary reflected code, Eq. (Hamming_equation)).
 * ld_gray_change: for word j >= 1, the digit that differs from word j - 1
 * (Eqs. (Hamming_equation_change), (d_aryGrayChange_1)) and its old / new value. */
uint32_t ld_gray_digit(uint32_t d, uint32_t i, uint64_t j);
int32_t ld_gray_change(uint32_t d, uint64_t j, uint32_t* from, uint32_t* to);

/* Sweep shape used for new plans (0 = keep, and -1 = keep for r_drop and sgpr_r).
 * p_target: high rows (lanes = 2^p_target) for large binary problems; c_min: least
 * mid rows per lane; r_drop: 1 to score one low row fewer per state than the
 * register budget of the VGPR-operand kernel allows; dary_ptab: rows covered by
 * restricted-growth prefixes (<= 16); sgpr_r: low rows scored per state by the
 * int32 binary kernel that reads its low-row operands from SGPRs (4 or 5), 0
 * for the kernel that holds them in VGPRs, 8 for the kernel whose Gray-code
 * state update runs on the matrix cores (int8 MFMA, 5 low rows; used where every
 * mid-row delta fits int8 and there are 1 to 16 mid rows, else the SGPR kernel
 * with 5 low rows runs), or 16 for the kernel that holds two columns per register
 * as 16-bit halves (5 low rows; used where every column has sum_x |M_xy| <= 32767,
 * and for L_marg column 0 at most 21844, else the SGPR kernel with 5 low rows
 * runs); dary_sgpr: 1 for the d-ary kernel with
 * SGPR operands (d = 3, 4, three low rows) where it is built, 0 for the VGPR one,
 * 16 for the packed 16-bit d-ary kernel (two columns per register; five low rows
 * for d = 3, four for d = 4, one fewer for a single problem that would have under
 * 2^15 lanes at that count; used under the same column bound as the binary one,
 * else the SGPR-operand kernel runs).  The compiled defaults are 16 for both.
 * An explicit sgpr_r or dary_sgpr also replaces the autotuner's per-width choices
 * for those kinds.  Values never depend on the shape. */
void ld_set_sweep_shape(int32_t p_target, int32_t c_min, int32_t r_drop, int32_t dary_ptab, int32_t sgpr_r,
                        int32_t dary_sgpr);

/* Lane floor of small binary problems for new plans: a problem with few free rows
 * keeps at least 2^p_fill prefixes (lanes) before rows become mid rows (up to the
 * c_min of ld_set_sweep_shape); p_fill = 0 turns the floor off, so such problems
 * take c_min mid rows whenever they have them.  The default is 16 (one wave per
 * SIMD).  Negative values are ignored.  Values never depend on it. */
void ld_set_lane_fill(int32_t p_fill);

/* Resident waves per SIMD of the sweep launches of plain and batch calls made from
 * now on (the paper's total-thread-count question, Sec. 4): the persistent queue
 * kernels launch at most waves_per_simd x 4 x CUs waves.  0 (the default) launches
 * as many as the kernel's occupancy allows; negative values are ignored.  Batches
 * prepared earlier keep the launches they captured.  Values never depend on it. */
void ld_set_launch_waves(int32_t waves_per_simd);

/* Autotuner.  The paper found no general rule for the launch shape and advises
 * timing a smaller matrix first (Sec. 4).  ld_autotune times candidate shapes on
 * the current device -- words per prefix and per queue item for batches, lane
 * count and low rows for plain calls -- within about budget_seconds, applies the
 * fastest, and writes them as JSON to path (NULL: do not write).
 * ld_load_tuning applies a file written by ld_autotune.  Shapes change speed only,
 * never values. */
int ld_autotune(const char* path, double budget_seconds);
int ld_load_tuning(const char* path);

/* Measurement aid for the int32 VALU roofline (not part of the search).  Runs a
 * kernel on the current device in which every wave issues a known number of
 * v_sad_u32 (the scoring instruction of the sweeps) in independent chains, four
 * waves per SIMD, for about target_ms, and reports:
 *   sclk_hz              engine clock under that load: the shader-clock counter
 *                        (s_memtime) against the constant-rate counter
 *                        (s_memrealtime, hipDeviceAttributeWallClockRate), median
 *                        over waves;
 *   sclk_max_hz          hipDeviceProp_t::clockRate (the rated peak clock);
 *   valu_lane_ops_per_s  lane-instructions issued per second over the launch
 *                        (kernel time from HIP events);
 *   compute_units, waves, seconds.
 * Returns 0, LD_EINVAL (null out, target_ms <= 0) or LD_EHIP (no gfx950 device,
 * or a HIP error).  Allocates and frees a small device buffer and a stream. */
typedef struct {
    double sclk_hz;
    double sclk_max_hz;
    double valu_lane_ops_per_s;
    double seconds;
    int32_t compute_units;
    int32_t waves;
} ld_valu_probe_result;
int ld_valu_probe(double target_ms, ld_valu_probe_result* out);

#ifdef __cplusplus
}
#endif

#endif /* LD_H */
