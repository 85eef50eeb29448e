/*
 * credit.h -- C ABI of the MI355X (gfx950) wide reduction-reuse row-kernel library.
 *
 * The operators are members of the reduction-reuse class of the CREDIT paper
 * (Sec. III-B, Eq. (1)): each row of width N is reduced to a few scalar
 * statistics r, then every element is reused to write a full-size output
 * y_i = h(x_i, r).  Three kernel variants exist for every operator:
 *
 *   CREDIT_TWO_PASS      the global-reread baseline (Sec. IV-A): one workgroup
 *                        streams the row once for the statistics and again to
 *                        write the output.
 *   CREDIT_ROW_RESIDENT  one workgroup keeps its whole row in registers (the
 *                        one-CTA staged baseline of Sec. IV-A) and writes the
 *                        output without a second global read.
 *   CREDIT_SPLIT_ROW     the row is split into k slices held by k co-resident
 *                        workgroups (Eq. (2)); each reduces its slice, the k
 *                        partial statistics are exchanged through device memory
 *                        (the L2 / Infinity Cache stands in for the cluster's
 *                        distributed shared memory of Sec. III-C, Eq. (5)), and
 *                        every workgroup applies h to its own retained slice.
 *
 * A plan (variant, k) is chosen per shape by the profitability model of
 * Sec. III-D (Eq. (7)-(9), with MI355X terms), by a learned selector, by
 * exhaustive timing, or given by the caller.
 *
 * Conventions shared by every entry point:
 *   - Device pointers are plain HIP device addresses; the caller owns all
 *     tensors and the workspace.  Nothing in an operator call allocates.
 *   - Matrices are row-major [M, ld] with unit inner stride; ld >= N is given
 *     in ELEMENTS.  Rows of any alignment use the same 16-byte accesses;
 *     aligned rows holding whole vectors take an unmasked row loop.
 *   - I/O dtypes: CREDIT_F32 (float), CREDIT_BF16 (raw 16-bit bfloat16),
 *     CREDIT_FP8_E4M3 (raw uint8 OCP e4m3fn).  FP8 tensors carry one FP32
 *     scale per row: value = decode(code) * scale[row].  FP8 inputs read their
 *     scales; FP8 outputs write theirs (scale = row amax / 448, or 1 for an
 *     all-zero row) and the codes are rounded to nearest even and saturated to
 *     +-448.  All arithmetic is FP32.  gamma, beta, dgamma, dbeta, mean and
 *     rstd are FP32 vectors in every dtype.
 *   - Calls are asynchronous on `stream`.  M == 0 is a no-op.  N == 0, ld < N,
 *     a NULL required pointer, or a workspace smaller than
 *     credit_workspace_size() returns CREDIT_ERR_INVALID_ARG /
 *     CREDIT_ERR_WORKSPACE.  An explicit plan that is illegal for the shape
 *     returns CREDIT_ERR_UNSUPPORTED; plans are never silently changed.
 *   - The workspace must be zero-filled before its first use; the library
 *     keeps it valid across calls.  Two calls that may run concurrently must
 *     not share a workspace.
 *   - Operator calls never allocate device memory and never time kernels.
 *     With plan == NULL they run the plan cached for the shape (credit_select
 *     fills the cache with the configured selector's choice, timing kernels
 *     where that selector times), else the learned network's first legal
 *     choice, computed on the handle's stream in buffers allocated when the
 *     model was set (the fixed rule without a model).
 *   - Operator calls may be recorded into a HIP graph (stream capture) and
 *     replayed: a recorded split-row launch is preceded by a one-thread kernel
 *     that advances a device-side exchange epoch, so every replay is a new
 *     epoch.  A plan == NULL call on a shape with no cached plan, made while
 *     its stream is capturing, takes the fixed rule (host arithmetic only) and
 *     caches nothing; operator calls record no memset nodes.
 *   - A split-row launch assumes its workgroups can all be resident at once:
 *     its grid is the occupancy bound times the CU count.  The library orders
 *     its own such launches on a device one after another, whatever their
 *     streams (outside graph capture).  Other kernels that wait on one another
 *     (other libraries', other processes') running at the same time can keep
 *     members of a row group from starting; the bounded exchange wait then
 *     ends the launch and credit_check_errors() returns CREDIT_ERR_TIMEOUT (the
 *     output is not valid).  CREDIT_OPT_MAX_GROUPS caps the row groups to
 *     leave room for such work; two-pass and resident plans have no such
 *     requirement.
 *   - No C++ exception crosses this interface and nothing aborts.
 */
#ifndef CREDIT_H
#define CREDIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The enumerations are int-sized in both languages.  Compiled as C++ they
 * take int as their fixed underlying type, so any int a caller passes (ctypes
 * passes plain ints) is a value of the type, and an out-of-range one is
 * rejected with CREDIT_ERR_INVALID_ARG rather than being undefined. */
#ifdef __cplusplus
#define CREDIT_ENUM enum : int
#else
#define CREDIT_ENUM enum
#endif

typedef CREDIT_ENUM {
    CREDIT_OK = 0,
    CREDIT_ERR_INVALID_ARG = 1,
    CREDIT_ERR_UNSUPPORTED = 2, /* plan illegal for this shape / dtype        */
    CREDIT_ERR_WORKSPACE = 3,   /* workspace missing or too small              */
    CREDIT_ERR_HIP = 4,         /* a HIP runtime call failed                   */
    CREDIT_ERR_TIMEOUT = 5,     /* a split-row exchange wait hit its bound     */
    CREDIT_ERR_MODEL = 6        /* selector model missing, corrupt or foreign  */
} credit_status_t;

typedef CREDIT_ENUM { CREDIT_F32 = 0, CREDIT_BF16 = 1, CREDIT_FP8_E4M3 = 2 } credit_dtype_t;
/* Operators.  The first three exist in both directions; the others are the
 * remaining reduction-reuse workloads of the paper's evaluation suite
 * (Sec. IV-A) and exist in one direction each: SOFTMAX_LOGITS, PEARSON and
 * WVAR backward only, the two QUANT operators and LAYERNORM_FP8_OUT forward
 * only.  Where a call
 * names an (operator, direction) pair, any other pair is CREDIT_ERR_INVALID_ARG. */
typedef CREDIT_ENUM {
    CREDIT_SOFTMAX = 0,
    CREDIT_LAYERNORM = 1,
    CREDIT_RMSNORM = 2,
    CREDIT_SOFTMAX_LOGITS = 3, /* softmax backward taking the logits x (y is rebuilt in the row) */
    CREDIT_QUANT_INT8 = 4,     /* row-wise int8 quantisation (codes + per-row scale)             */
    CREDIT_QUANT_FP8 = 5,      /* row-wise e4m3 quantisation (codes + per-row scale)             */
    CREDIT_PEARSON = 6,        /* Pearson correlation of two rows                                */
    CREDIT_WVAR = 7,           /* weighted variance of a row                                     */
    CREDIT_LAYERNORM_FP8_OUT = 8 /* LayerNorm forward fused with row-wise e4m3 quantisation      */
} credit_op_t;
typedef CREDIT_ENUM { CREDIT_FWD = 0, CREDIT_BWD = 1 } credit_dir_t;
typedef CREDIT_ENUM { CREDIT_TWO_PASS = 0, CREDIT_ROW_RESIDENT = 1, CREDIT_SPLIT_ROW = 2 } credit_variant_t;
typedef CREDIT_ENUM {
    CREDIT_SEL_LEARNED = 0,    /* MLP over shape features; falls back to ANALYTIC   */
    CREDIT_SEL_ANALYTIC = 1,   /* Eq. (9) with one timing of the baseline (Eq. (7)) */
    CREDIT_SEL_EXHAUSTIVE = 2, /* time every legal plan, keep the fastest           */
    CREDIT_SEL_FIXED = 3,      /* resident if it fits, else smallest legal k, else two-pass */
    CREDIT_SEL_PEAK = 4,       /* Eq. (9) with the baseline priced at calibrated copy bandwidth */
    CREDIT_SEL_LEARNED_TIMED = 5 /* the MLP's two best legal plans, each timed once (cold,
                                    median of 7), the faster kept; falls back to ANALYTIC */
} credit_selector_t;

/* variant and split factor; k == 1 for CREDIT_TWO_PASS and CREDIT_ROW_RESIDENT,
 * k in {2, 4, 8, 16, 32} for CREDIT_SPLIT_ROW. */
typedef struct {
    int32_t variant;
    int32_t k;
} credit_plan_t;

typedef struct credit_handle_s *credit_handle_t;

/* Human-readable name of a status code (static storage). */
const char *credit_status_string(credit_status_t s);

/* Library version string (static storage). */
const char *credit_version(void);

/* Creates a handle bound to HIP device `device`: reads its properties, sizes
 * the persistent grids, allocates the handle's small device-side error flag.
 * The handle owns the plan cache, the selector model and timing buffers.
 * Environment read here: CREDIT_SELECTOR (learned | analytic | exhaustive |
 * fixed | peak) sets the selector; CREDIT_FORCE_PLAN (two_pass | resident |
 * split:<k>) is used by calls with plan == NULL wherever it is legal for the
 * shape (elsewhere the selector decides); CREDIT_SPIN_LIMIT sets the split-row
 * wait bound; CREDIT_CHECKED=1 makes every operator call wait for its launches
 * and return CREDIT_ERR_TIMEOUT itself when an exchange wait expired (calls on
 * a capturing stream are not waited on); CREDIT_LOG (stderr or a file path,
 * appended) writes one JSON line per operator call: operator, dtype, M, N,
 * plan, whether the caller gave it, the selector, launch geometry and status.
 * Unrecognised values are ignored. */
credit_status_t credit_create(int device, credit_handle_t *h);
credit_status_t credit_destroy(credit_handle_t h);

/* Selector of credit_select (and so of the plans cached for operator calls
 * with plan == NULL). */
credit_status_t credit_set_selector(credit_handle_t h, credit_selector_t s);

/* Bytes of workspace an operator call needs for (op, dir, dtype, M, N) under
 * `plan` (NULL: the largest over the plans legal for the shape, enough for
 * whatever plan a call with plan == NULL runs; nothing is selected or timed).
 * The size covers split-row exchange slots (M * stages * k * q * 8 bytes) and,
 * for normalisation backward, per-row-group dgamma/dbeta column partials. */
credit_status_t credit_workspace_size(credit_handle_t h, credit_op_t op, credit_dir_t dir,
                                      credit_dtype_t dt, int64_t M, int64_t N,
                                      const credit_plan_t *plan, size_t *bytes);

/* Whether `plan` is legal for the shape: the slice of ceil(N/k) elements must
 * fit the kernel's capacity (the capacity rule of Eq. (3)): 32 16-byte vectors
 * per thread of registers at most (fewer for the backward operators), and for
 * the FP32 / BF16 softmax, LayerNorm and RMSNorm forward up to 16 or 36 more
 * per thread in LDS (64 KiB or 144 KiB per workgroup); and, for
 * k > 1, the k workgroups of a row must be co-resident.  Returns CREDIT_OK or
 * CREDIT_ERR_UNSUPPORTED. */
credit_status_t credit_plan_legal(credit_handle_t h, credit_op_t op, credit_dir_t dir,
                                  credit_dtype_t dt, int64_t M, int64_t N,
                                  const credit_plan_t *plan);

/* Picks a plan for the shape with the handle's selector (Sec. III-D) and
 * caches it for operator calls with plan == NULL.  Selectors that time kernels
 * allocate the handle's timing buffers here (inputs of the shape and a
 * 512 MiB cache-flush buffer).  predicted_us (nullable) receives the model's
 * predicted time where the selector has one, else -1. */
credit_status_t credit_select(credit_handle_t h, credit_op_t op, credit_dir_t dir,
                              credit_dtype_t dt, int64_t M, int64_t N, credit_plan_t *out,
                              float *predicted_us);

/* ---------------------------------------------------------------- operators */

/* Row softmax: y = exp(x - max x) / sum exp(x - max x).  Entries of -inf
 * (masks, FP32 / BF16) give 0; a row with no finite entry is 0/0 and gives
 * NaN, like the plain definition. */
credit_status_t credit_softmax_fwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                                   const void *x, int64_t ldx, const float *x_scale, void *y,
                                   int64_t ldy, float *y_scale, const credit_plan_t *plan,
                                   void *ws, size_t ws_bytes, void *stream);

/* Softmax backward from the forward output: dx = y * (dy - sum(dy * y)). */
credit_status_t credit_softmax_bwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                                   const void *y, int64_t ldy, const float *y_scale,
                                   const void *dy, int64_t lddy, const float *dy_scale, void *dx,
                                   int64_t lddx, float *dx_scale, const credit_plan_t *plan,
                                   void *ws, size_t ws_bytes, void *stream);

/* LayerNorm: mean and biased variance per row, rstd = 1/sqrt(var + eps),
 * y = (x - mean) * rstd * gamma + beta.  mean / rstd outputs are nullable. */
credit_status_t credit_layernorm_fwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                                     const void *x, int64_t ldx, const float *x_scale,
                                     const float *gamma, const float *beta, float eps, void *y,
                                     int64_t ldy, float *y_scale, float *mean, float *rstd,
                                     const credit_plan_t *plan, void *ws, size_t ws_bytes,
                                     void *stream);

/* The same LayerNorm forward without a workspace argument and without any
 * allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * split-row exchange slots live in a library-owned scratch array of
 * credit_noalloc_scratch_bytes() (16 MiB) per device, set up when the handle
 * is created and kept until the process ends; a plan needing more
 * (M * 3 * k * 2 * 8 + 256 bytes for LayerNorm) returns CREDIT_ERR_WORKSPACE.
 * plan == NULL takes the cached plan of the shape, else the fixed rule (no
 * device work besides the operator's own kernels).  Every call on a device
 * shares that device's scratch: calls that may overlap on one device (two
 * streams, two threads) race and must be serialised by the caller.  `stream`
 * must belong to the handle's device. */
credit_status_t credit_layernorm_fwd_noalloc(credit_handle_t h, int64_t M, int64_t N,
                                             credit_dtype_t dt, const void *x, int64_t ldx,
                                             const float *x_scale, const float *gamma,
                                             const float *beta, float eps, void *y, int64_t ldy,
                                             float *y_scale, float *mean, float *rstd,
                                             const credit_plan_t *plan, void *stream);
size_t credit_noalloc_scratch_bytes(void);

/* LayerNorm backward: xhat = (x - mean) * rstd, g = dy * gamma,
 * dx = rstd * (g - mean(g) - xhat * mean(g * xhat)),
 * dgamma = sum over rows of dy * xhat, dbeta = sum over rows of dy.
 * mean and rstd are the forward's saved statistics; pass both NULL to have
 * them recomputed from x in the same pass (one more reduction stage).
 * dgamma / dbeta are overwritten (not accumulated); either may be NULL. */
credit_status_t credit_layernorm_bwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                                     const void *x, int64_t ldx, const float *x_scale,
                                     const void *dy, int64_t lddy, const float *dy_scale,
                                     const float *gamma, const float *mean, const float *rstd,
                                     float eps, void *dx, int64_t lddx, float *dx_scale,
                                     float *dgamma, float *dbeta, const credit_plan_t *plan,
                                     void *ws, size_t ws_bytes, void *stream);

/* RMSNorm: rstd = 1/sqrt(mean(x^2) + eps), y = x * rstd * gamma.  rstd nullable. */
credit_status_t credit_rmsnorm_fwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                                   const void *x, int64_t ldx, const float *x_scale,
                                   const float *gamma, float eps, void *y, int64_t ldy,
                                   float *y_scale, float *rstd, const credit_plan_t *plan,
                                   void *ws, size_t ws_bytes, void *stream);

/* RMSNorm backward: xhat = x * rstd, g = dy * gamma,
 * dx = rstd * (g - xhat * mean(g * xhat)), dgamma = sum over rows of dy * xhat.
 * rstd NULL: recomputed from x.  dgamma nullable. */
credit_status_t credit_rmsnorm_bwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                                   const void *x, int64_t ldx, const float *x_scale,
                                   const void *dy, int64_t lddy, const float *dy_scale,
                                   const float *gamma, const float *rstd, float eps, void *dx,
                                   int64_t lddx, float *dx_scale, float *dgamma,
                                   const credit_plan_t *plan, void *ws, size_t ws_bytes,
                                   void *stream);

/* Softmax backward from the logits (the softmax-logits workload, Sec. IV-A):
 * y = softmax(x) is recomputed inside the row from the resident x, then
 * dx = y * (dy - sum(dy * y)).  One statistics stage carries (max, sum of
 * exponentials, sum of dy times the exponentials); FP8 output adds its amax
 * stage.  All three dtypes; x, dy and dx share `dt` (FP8 scales as above). */
credit_status_t credit_softmax_logits_bwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                                          const void *x, int64_t ldx, const float *x_scale,
                                          const void *dy, int64_t lddy, const float *dy_scale,
                                          void *dx, int64_t lddx, float *dx_scale,
                                          const credit_plan_t *plan, void *ws, size_t ws_bytes,
                                          void *stream);

/* Row-wise quantisation (the int8-quantisation workload, Sec. IV-A):
 * amax = max |x| over the row, q_scale[row] = amax / Q (1 for an all-zero
 * row), codes from v = x * (Q / amax) computed in FP32 (Q / amax rounded to
 * FP32 first).  op = CREDIT_QUANT_INT8: Q = 127, code = round-half-even(v)
 * clamped to [-127, 127], stored as int8.  op = CREDIT_QUANT_FP8: Q = 448,
 * code = OCP e4m3fn RNE of v saturated to +-448, stored as uint8.
 * x is CREDIT_F32 or CREDIT_BF16 (`dt`); q is [M, ldq] bytes. */
credit_status_t credit_quantize_rows(credit_handle_t h, credit_op_t op, int64_t M, int64_t N,
                                     credit_dtype_t dt, const void *x, int64_t ldx, void *q,
                                     int64_t ldq, float *q_scale, const credit_plan_t *plan,
                                     void *ws, size_t ws_bytes, void *stream);

/* LayerNorm forward fused with row-wise e4m3 quantisation of its output (the
 * quantisation workload of Sec. IV-A fed by a LayerNorm): y as in
 * credit_layernorm_fwd is computed in FP32 from an FP32 / BF16 row (`dt`),
 * then one more statistics stage takes amax |y|, q_scale[row] = amax / 448
 * (1 for an all-zero row) and the codes are e4m3 RNE of y * (448 / amax)
 * saturated to +-448, stored as uint8 in q [M, ldq].  mean / rstd nullable. */
credit_status_t credit_layernorm_fwd_fp8_out(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                                             const void *x, int64_t ldx, const float *gamma,
                                             const float *beta, float eps, void *q, int64_t ldq,
                                             float *q_scale, float *mean, float *rstd,
                                             const credit_plan_t *plan, void *ws, size_t ws_bytes,
                                             void *stream);

/* Pearson-correlation backward (Sec. IV-A): per row, with xc = x - mean(x),
 * yc = y - mean(y), Sxx = sum xc^2, Syy = sum yc^2, Sxy = sum xc yc and
 * r = Sxy / sqrt(Sxx Syy), given the upstream gradient dr[row]:
 *   dx = dr * (yc / sqrt(Sxx Syy) - r * xc / Sxx),
 *   dy = dr * (xc / sqrt(Sxx Syy) - r * yc / Syy).
 * One stage of five co-moment statistics.  A row with Sxx or Syy == 0 gives
 * non-finite outputs (r is undefined there).  CREDIT_F32 or CREDIT_BF16;
 * dr is FP32 [M]. */
credit_status_t credit_pearson_bwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                                   const void *x, int64_t ldx, const void *y, int64_t ldy,
                                   const float *dr, void *dx, int64_t lddx, void *dy, int64_t lddy,
                                   const credit_plan_t *plan, void *ws, size_t ws_bytes,
                                   void *stream);

/* Weighted-variance backward (Sec. IV-A): per row, W = sum w,
 * mu = sum w x / W, v = sum w (x - mu)^2 / W, given the upstream gradient
 * dv[row]:  dx = dv * 2 w (x - mu) / W,  dw = dv * ((x - mu)^2 - v) / W.
 * One stage of three statistics (W, mu, sum w (x - mu)^2).  A row with
 * W == 0 gives non-finite outputs.  CREDIT_F32 or CREDIT_BF16; dv is FP32 [M]. */
credit_status_t credit_wvar_bwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                                const void *x, int64_t ldx, const void *w, int64_t ldw,
                                const float *dv, void *dx, int64_t lddx, void *dw, int64_t lddw,
                                const credit_plan_t *plan, void *ws, size_t ws_bytes, void *stream);

/* Elementwise FP32 -> dtype encode of an [M, N] matrix with optional per-row
 * output scale (FP8: code = RNE_sat(x / scale[row])); and the inverse decode.
 * Contiguous rows (ld == N). */
credit_status_t credit_encode(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                              const float *x, const float *row_scale, void *out, void *stream);
credit_status_t credit_decode(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                              const void *in, const float *row_scale, float *out, void *stream);

/* Status of work already issued: synchronises `stream`, reports a sticky HIP
 * error or a split-row exchange timeout (then clears the timeout flag). */
credit_status_t credit_check_errors(credit_handle_t h, void *stream);

/* ------------------------------------------------------- timing and models */

/* Times `plan` on (op, dir, dtype, M, N) with library-owned buffers:
 * `reps` runs (0: 15), each preceded by a 512 MiB cache flush when `flush` is
 * nonzero, bracketed by HIP events; writes the median in microseconds.
 * Follows the median-of-15 protocol of Sec. III-A. */
credit_status_t credit_time_plan(credit_handle_t h, credit_op_t op, credit_dir_t dir,
                                 credit_dtype_t dt, int64_t M, int64_t N,
                                 const credit_plan_t *plan, int reps, int flush,
                                 float *median_us);

/* The same timing with the spread of the runs: median, minimum, 90th
 * percentile (nearest rank) and median absolute deviation, in microseconds.
 * The exhaustive selector counts plans within max(1%, 2 MAD) of the fastest
 * median as equally fast and keeps the one that moves fewer bytes (row-
 * resident, then split plans by increasing k, then two-pass). */
typedef struct {
    float median_us, min_us, p90_us, mad_us;
    int32_t runs;
} credit_timing_t;
credit_status_t credit_time_plan_stats(credit_handle_t h, credit_op_t op, credit_dir_t dir,
                                       credit_dtype_t dt, int64_t M, int64_t N,
                                       const credit_plan_t *plan, int reps, int flush,
                                       credit_timing_t *out);

/* Times the work-free control kernel of Sec. III-D for a split factor k at
 * (op, dir, dtype, M, N): the same persistent grid, split factor, occupancy
 * and exchange waits as the split-row kernel, no row data.  k == 1 gives the
 * one-workgroup control.  Median of `reps` runs in microseconds. */
credit_status_t credit_time_control(credit_handle_t h, credit_op_t op, credit_dir_t dir,
                                    credit_dtype_t dt, int64_t M, int64_t N, int32_t k,
                                    int reps, float *median_us);

/* Times a plain device copy of `bytes` bytes (read + write) and returns the
 * achieved GB/s (median of `reps`); the practical HBM ceiling used to price
 * traffic in the CREDIT_SEL_PEAK model. */
credit_status_t credit_copy_bandwidth(credit_handle_t h, size_t bytes, int reps, float *gbps);

/* Evaluates the analytic model of Sec. III-D for every plan of the shape with
 * caller-supplied measurements (no GPU work):
 *   t_base_us    the measured baseline time T_B (Eq. (7))
 *   t_ctrl_us    control-kernel excess T_ctrl for k = 2,4,8,16,32 (5 entries)
 * out_delta_us receives Delta T for k = 2,4,8,16,32 (Eq. (9)); illegal plans
 * get -INFINITY.  Host-only: callable without a GPU for a handle created on
 * a device, and with h == NULL using MI355X defaults. */
credit_status_t credit_model_delta(credit_handle_t h, credit_op_t op, credit_dir_t dir,
                                   credit_dtype_t dt, int64_t M, int64_t N, float t_base_us,
                                   const float *t_ctrl_us, float *out_delta_us);

/* Byte accounting of an operator per element (static analysis of Eq. (4)):
 * baseline (two-pass) bytes b_B, staged bytes, eliminated reread b_reread,
 * retained bytes b_keep, stages L and statistics per stage q (up to 4). */
typedef struct {
    float b_base;
    float b_staged;
    float b_reread;
    float b_keep;
    int32_t stages;
    int32_t q[4];
} credit_workload_t;
credit_status_t credit_workload_info(credit_op_t op, credit_dir_t dir, credit_dtype_t dt,
                                     int recompute_stats, credit_workload_t *out);

/* MI355X primitive costs (the analogue of the paper's primitive table,
 * Sec. III-A, Table II), each the median of `reps` launches (0: 15) of a
 * microbenchmark kernel.  Latencies in nanoseconds (from the 100 MHz
 * real-time counter); rates in bytes per shader-clock cycle for one
 * workgroup of 256 threads on one CU; clock_mhz is the s_memtime rate seen
 * over the probes.  A handoff is one agent-scope store by one workgroup seen
 * by a polling agent-scope load in another (the exchange's access path); the
 * workgroup pairs are hardware ids (0, 8) and (0, 1), whose XCDs are
 * reported.  exchange_ns[i] is one exchange round (q = 1) of a row group of
 * k = 2, 4, 8, 16, 32 workgroups.  Allocates its own buffers. */
typedef struct {
    float clock_mhz;
    float lds_load_ns;          /* dependent LDS load                             */
    float l2_load_ns;           /* dependent agent-scope load, L2 hit             */
    float handoff_same_xcd_ns;  /* one-way handoff between two workgroups, 1 XCD  */
    float handoff_cross_xcd_ns; /* ... on two XCDs                                */
    float barrier_ns;           /* one 256-thread workgroup barrier               */
    float exchange_ns[5];
    float lds_read_bpc, lds_write_bpc, l2_read_bpc, global_write_bpc;
    int32_t xcd_same[2], xcd_cross[2];
    int32_t errors;             /* bounded waits that gave up (0 expected)        */
} credit_primitives_t;
/* A successful run without errors also calibrates the handle's analytic model
 * (Eq. (8)): the measured clock replaces the 2.4 GHz peak, one workgroup's
 * global store rate the slot-store rate, and one workgroup's LDS read rate
 * prices the replay of slices held in LDS. */
credit_status_t credit_probe_primitives(credit_handle_t h, int reps, credit_primitives_t *out);

/* ------------------------------------------------------------ learned model
 * A 12 -> 64 -> 64 -> CREDIT_NUM_PLANS ReLU network over standardized shape
 * features predicts the fastest plan; trained on the GPU by the library's
 * own kernels from timings it collects. */
#define CREDIT_NUM_FEATURES 12
#define CREDIT_NUM_PLANS 7 /* two-pass, resident, split k = 2, 4, 8, 16, 32 */
#define CREDIT_MLP_HIDDEN 64

/* Plan of class c in [0, CREDIT_NUM_PLANS). */
credit_status_t credit_plan_of_class(int32_t c, credit_plan_t *out);

/* The 12 raw (unstandardized) features of a shape: is-softmax, is-LayerNorm
 * (RMSNorm: both 0), is-backward, log2 of the element bytes (2, 1, 0 for
 * FP32, BF16, FP8), log2 M, log2 N, aligned rows (1 when N * e is a multiple
 * of 16 bytes, so rows of ld = N from an aligned base hold whole aligned
 * vectors, else 0), and for each split class k = 2, 4, 8, 16, 32
 * log2(W_k * fill_k): fill_k is how full the slice keeps the bucket it runs
 * in (the slice's 16-byte vectors over 256 * the smallest vectors-per-thread
 * bucket of the operator holding them, register buckets first, then LDS
 * buckets where the operator has them) and W_k = ceil(M / row groups) the
 * waves of row groups (Eq. (8)) of the plan's host-only geometry (as
 * credit_plan_geometry with h == NULL reports it); -1 when the plan is
 * illegal (the slice exceeds the capacity of Eq. (3)).  Defined
 * for the softmax, LayerNorm and RMSNorm operators (the learned selector's
 * domain; the other operators are planned by the analytic model):
 * CREDIT_ERR_UNSUPPORTED else. */
credit_status_t credit_features(credit_op_t op, credit_dir_t dir, credit_dtype_t dt, int64_t M,
                                int64_t N, float *feat12);

/* Number of FP32 parameters of the network (W1, b1, W2, b2, W3, b3 in that
 * order, weights row-major [out][in]). */
int64_t credit_mlp_num_params(void);

/* Sets / gets the parameters and the feature standardization (mu, sd: 12 each). */
credit_status_t credit_mlp_set(credit_handle_t h, const float *params, const float *mu,
                               const float *sd);
credit_status_t credit_mlp_get(credit_handle_t h, float *params, float *mu, float *sd);

/* Loss and gradient at the current parameters on the GPU, without updating:
 * masked soft-target cross-entropy averaged over n samples.  feats are raw;
 * targets [n][C] sum to 1 over legal plans; mask [n][C] is 1 for legal. */
credit_status_t credit_mlp_grad(credit_handle_t h, const float *feats, const float *targets,
                                const uint8_t *mask, int64_t n, float *loss, float *grad);

/* Full-batch Adam training on the GPU (beta1 0.9, beta2 0.999, eps 1e-8) for
 * `epochs` steps from a seeded He initialisation (seed != 0) or from the
 * current parameters (seed == 0).  The standardization is computed from the
 * given features when seed != 0.  The handle keeps the Adam moments and step
 * count: seed == 0 continues from them (they are zero after a seeded start,
 * credit_mlp_set, or loading a model saved without them), so training split
 * over calls, or resumed from a saved model, takes the same steps as one call. */
credit_status_t credit_mlp_train(credit_handle_t h, const float *feats, const float *targets,
                                 const uint8_t *mask, int64_t n, int epochs, float lr,
                                 uint64_t seed, float *final_loss);

/* Logits [n][C] for raw features, computed on the GPU. */
credit_status_t credit_mlp_predict(credit_handle_t h, const float *feats, int64_t n,
                                   float *logits);

/* Saves / loads the network with a header (format version, arch, CU count,
 * feature schema, the library that wrote it, the plan classes in order), the
 * standardization, the parameters and the Adam moments and step count (the
 * training checkpoint; files of format 1, without them, load with zero
 * moments); a foreign or corrupt file returns CREDIT_ERR_MODEL and leaves the
 * handle without a model.  Values are written with 9 significant digits, so a
 * saved and reloaded network is bit-identical. */
credit_status_t credit_save_model(credit_handle_t h, const char *path);
credit_status_t credit_load_model(credit_handle_t h, const char *path);

/* ------------------------------------------------------------- diagnostics */

/* Handle options. */
typedef CREDIT_ENUM {
    CREDIT_OPT_SPIN_LIMIT = 0,  /* poll iterations before an exchange wait gives up */
    CREDIT_OPT_TEST_DROP_PUBLISH = 1, /* test only: member 1 of each row group skips
                                         publishing its partials (forces the timeout
                                         path of CREDIT_ERR_TIMEOUT) */
    CREDIT_OPT_MAX_GROUPS = 2,  /* cap on concurrent row groups (0: occupancy bound) */
    CREDIT_OPT_TEST_SKEW = 3,   /* test only: before each exchange, member c of a row
                                   group waits (c * 7 + row) % 13 microseconds, so the
                                   members publish out of step (Sec. III-C) */
    CREDIT_OPT_ROWS = 4         /* rows per workgroup of LayerNorm / RMSNorm forward
                                   resident and split plans: 0 = the library's rule,
                                   1 = one row at a time, 2 or 4 = that many rows at
                                   once where the slice has at most 8 vectors per
                                   thread (each gamma / beta vector loaded once per
                                   2 or 4 rows, one exchange round per row block);
                                   other values return CREDIT_ERR_INVALID_ARG */
} credit_option_t;
credit_status_t credit_set_option(credit_handle_t h, credit_option_t opt, int64_t value);

/* Sets the next exchange epoch (process-wide); epochs are 32-bit and never 0.
 * Used to exercise epoch wrap-around. */
credit_status_t credit_set_epoch(uint32_t next_epoch);

/* Launch geometry the library would use for a plan: grid size (workgroups),
 * threads per workgroup, per-thread vector count, co-resident workgroups per
 * CU, rows per workgroup.  Every output pointer is nullable.  Host-only. */
credit_status_t credit_plan_geometry(credit_handle_t h, credit_op_t op, credit_dir_t dir,
                                     credit_dtype_t dt, int64_t M, int64_t N,
                                     const credit_plan_t *plan, int32_t *grid, int32_t *block,
                                     int32_t *vpt, int32_t *per_cu, int32_t *rows);

/* Resources of the row-resident / split-row kernel instance of (op, dir, dt)
 * that holds `vpt` 16-byte vectors per thread per tensor (vpt in
 * {1, 2, 4, 8, 12, 16, 24, 32}, up to the operator's register capacity, and
 * 48 and 68 for the FP32 / BF16 forward operators with LDS slices) and
 * `rows` rows per workgroup (1; 2 or 4 for the multi-row LayerNorm / RMSNorm
 * forward with vpt <= 8):
 * registers per lane, private (scratch) bytes per lane, workgroups per CU by
 * the occupancy query and by the library's register model, and, for an
 * instance that uses private memory, the workgroups per CU its co-residency
 * probe verified when the handle was created (-1: no private memory, not
 * probed; 0: no split plan of it is run).  Split plans of a probed instance
 * never exceed the verified count (Sec. III-C: every member must be live for
 * the exchange to complete).  Returns CREDIT_ERR_UNSUPPORTED for a vpt the
 * operator does not instantiate.  With h == NULL only model_per_cu is filled
 * (the others are -1) and no device is touched.  Host-only. */
typedef struct {
    int32_t registers;
    int32_t private_bytes;
    int32_t per_cu;
    int32_t model_per_cu;
    int32_t coresident_per_cu;
} credit_instance_t;
credit_status_t credit_instance_info(credit_handle_t h, credit_op_t op, credit_dir_t dir,
                                     credit_dtype_t dt, int32_t vpt, int32_t rows,
                                     credit_instance_t *out);

#ifdef __cplusplus
}
#endif
#endif /* CREDIT_H */
