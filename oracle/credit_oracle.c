/*
 * credit_oracle.c -- FP64 CPU oracle for the wide reduction-reuse row operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  It is used by tests/, by the smoke check and by the
 * benchmark's CPU-baseline leg, and by nothing else.  It shares no code,
 * header, table or constant with the GPU path.
 *
 * Every operator is written as its plain definition in double precision.  The
 * method under test (the reduction-reuse class of the CREDIT paper, Sec. III-B,
 * Eq. (1)) reaches these definitions exactly up to rounding order: each row is
 * reduced to a few scalar statistics r, then every element is reused to
 * produce y_i = h(x_i, r).  The oracle does no slicing, no blocking and no
 * fusion: it reduces a whole row with a compensated (Neumaier) sum and then
 * applies h.  Rows are independent, so rows are spread over OpenMP threads;
 * that changes nothing in any row's arithmetic.
 *
 * Inputs are already-decoded double arrays (row-major, contiguous, M x N).
 * The low-precision codecs below (bfloat16, OCP FP8 e4m3fn) are provided so
 * the tests can decode exactly what the GPU consumed and can locate the
 * rounding grid of a reference value.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- helpers */

/* Neumaier-compensated sum of n doubles spaced by `stride`. */
static double csum(const double *v, int64_t n, int64_t stride)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double a = v[i * stride];
        double t = s + a;
        if (fabs(s) >= fabs(a))
            c += (s - t) + a;
        else
            c += (a - t) + s;
        s = t;
    }
    return s + c;
}

/* Compensated accumulator used where the summand is formed on the fly. */
typedef struct { double s, c; } acc_t;
static inline void acc_add(acc_t *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}
static inline double acc_get(const acc_t *a) { return a->s + a->c; }

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

double oracle_sum(const double *v, int64_t n) { return csum(v, n, 1); }

/* ------------------------------------------------------------- the codecs */

/* bfloat16: 1 sign, 8 exponent, 7 fraction bits; the upper half of an IEEE
 * binary32.  Decoding is exact. */
void oracle_decode_bf16(const uint16_t *in, double *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t u = (uint32_t)in[i] << 16;
        float f;
        memcpy(&f, &u, 4);
        out[i] = (double)f;
    }
}

/* Round a double to the nearest bfloat16, ties to even, directly from the
 * double value (no intermediate binary32 rounding).  Overflow gives +-inf,
 * NaN gives the canonical quiet NaN 0x7FC0. */
static uint16_t bf16_from_double(double d)
{
    if (isnan(d)) return 0x7FC0;
    uint16_t sign = signbit(d) ? 0x8000 : 0;
    double a = fabs(d);
    if (a == 0.0) return sign;
    if (isinf(a)) return sign | 0x7F80;
    int e;
    frexp(a, &e);           /* a = f * 2^e, f in [0.5, 1)  => floor(log2 a) = e-1 */
    int lg = e - 1;
    if (lg < -126) lg = -126;               /* subnormal range keeps a fixed spacing */
    double ulp = ldexp(1.0, lg - 7);        /* 8 significant bits */
    double r = rint(a / ulp);               /* default mode: nearest, ties to even */
    double v = r * ulp;
    if (v >= ldexp(1.0, 128)) return sign | 0x7F80;
    float f = (float)v;                     /* exact: v lies on the bfloat16 grid */
    uint32_t u;
    memcpy(&u, &f, 4);
    return sign | (uint16_t)(u >> 16);
}

void oracle_encode_bf16(const double *in, uint16_t *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) out[i] = bf16_from_double(in[i]);
}

/* OCP FP8 e4m3fn: 1 sign, 4 exponent (bias 7), 3 fraction bits; no infinity;
 * S.1111.111 is NaN; largest finite 448; smallest subnormal 2^-9. */
static double e4m3_value(uint8_t b)
{
    int s = b >> 7, E = (b >> 3) & 0xF, F = b & 7;
    double v;
    if (E == 15 && F == 7) return NAN;
    if (E == 0)
        v = ldexp((double)F, -9);
    else
        v = ldexp(1.0 + F / 8.0, E - 7);
    return s ? -v : v;
}

void oracle_decode_e4m3(const uint8_t *in, double *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) out[i] = e4m3_value(in[i]);
}

/* Round a double to e4m3fn, ties to even, saturating to +-448 (values whose
 * rounded magnitude would exceed 448 become 448).  NaN maps to 0x7F. */
static uint8_t e4m3_from_double(double d)
{
    if (isnan(d)) return 0x7F;
    uint8_t sign = signbit(d) ? 0x80 : 0;
    double a = fabs(d);
    if (a == 0.0) return sign;
    if (a >= 448.0) return sign | 0x7E;
    int e;
    frexp(a, &e);
    int lg = e - 1;
    if (lg < -6) lg = -6;                   /* below 2^-6 the spacing is 2^-9 */
    double ulp = ldexp(1.0, lg - 3);        /* 4 significant bits */
    double v = rint(a / ulp) * ulp;
    if (v > 448.0) v = 448.0;
    if (v == 0.0) return sign;
    if (v < ldexp(1.0, -6))                 /* subnormal: v = F * 2^-9 */
        return sign | (uint8_t)(v * 512.0);
    frexp(v, &e);
    int E = (e - 1) + 7;
    int F = (int)(ldexp(v, -(e - 1)) * 8.0 - 8.0);
    return sign | (uint8_t)((E << 3) | F);
}

void oracle_encode_e4m3(const double *in, uint8_t *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) out[i] = e4m3_from_double(in[i]);
}

/* The same two encoders applied to binary32 inputs (each converted to double
 * exactly), spread over threads: for sweeps over every FP32 bit pattern. */
void oracle_encode_bf16_f32(const float *in, uint16_t *out, int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = bf16_from_double((double)in[i]);
}

void oracle_encode_e4m3_f32(const float *in, uint8_t *out, int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = e4m3_from_double((double)in[i]);
}

/* Spacing of the e4m3 grid at magnitude v (the size of one step). */
double oracle_e4m3_step(double v)
{
    double a = fabs(v);
    if (a < ldexp(1.0, -6)) return ldexp(1.0, -9);
    int e;
    frexp(a, &e);
    return ldexp(1.0, (e - 1) - 3);
}

/* ---------------------------------------------------------------- softmax */

/* y_i = exp(x_i - max_j x_j) / sum_j exp(x_j - max_j x_j), per row.
 * Statistics: r = (max, sum of shifted exponentials); h = exp(x - max) / sum. */
void oracle_softmax_fwd(int64_t M, int64_t N, const double *x, double *y)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        const double *xr = x + m * N;
        double *yr = y + m * N;
        double mx = -INFINITY;
        for (int64_t i = 0; i < N; ++i)
            if (xr[i] > mx) mx = xr[i];
        acc_t s = {0, 0};
        for (int64_t i = 0; i < N; ++i) acc_add(&s, exp(xr[i] - mx));
        double sum = acc_get(&s);
        for (int64_t i = 0; i < N; ++i) yr[i] = exp(xr[i] - mx) / sum;
    }
}

/* dx_i = y_i * (dy_i - sum_j dy_j y_j), per row, for the given y. */
void oracle_softmax_bwd(int64_t M, int64_t N, const double *y, const double *dy, double *dx)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        const double *yr = y + m * N, *gr = dy + m * N;
        double *dr = dx + m * N;
        acc_t c = {0, 0};
        for (int64_t i = 0; i < N; ++i) acc_add(&c, gr[i] * yr[i]);
        double cs = acc_get(&c);
        for (int64_t i = 0; i < N; ++i) dr[i] = yr[i] * (gr[i] - cs);
    }
}

/* --------------------------------------------------------------- LayerNorm */

/* mu = mean(x); var = mean((x - mu)^2) (biased); rstd = 1/sqrt(var + eps);
 * y = (x - mu) * rstd * gamma + beta.  mean/rstd outputs may be NULL. */
void oracle_layernorm_fwd(int64_t M, int64_t N, const double *x, const double *gamma,
                          const double *beta, double eps, double *y, double *mean, double *rstd)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        const double *xr = x + m * N;
        double *yr = y + m * N;
        double mu = csum(xr, N, 1) / (double)N;
        acc_t v = {0, 0};
        for (int64_t i = 0; i < N; ++i) acc_add(&v, (xr[i] - mu) * (xr[i] - mu));
        double var = acc_get(&v) / (double)N;
        double rs = 1.0 / sqrt(var + eps);
        for (int64_t i = 0; i < N; ++i) yr[i] = (xr[i] - mu) * rs * gamma[i] + beta[i];
        if (mean) mean[m] = mu;
        if (rstd) rstd[m] = rs;
    }
}

/* Column sums dgamma_j = sum_m a[m, j] * b[m, j] (b == NULL: sum_m a[m, j]),
 * where a and b are M x N; compensated per column. */
static void column_sums(int64_t M, int64_t N, const double *a, const double *b, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        acc_t s = {0, 0};
        for (int64_t m = 0; m < M; ++m)
            acc_add(&s, b ? a[m * N + j] * b[m * N + j] : a[m * N + j]);
        out[j] = acc_get(&s);
    }
}

/* LayerNorm backward with statistics recomputed from x in FP64:
 * xhat = (x - mu) * rstd; g = dy * gamma;
 * dx = rstd * (g - mean(g) - xhat * mean(g * xhat));
 * dgamma_j = sum_m dy * xhat; dbeta_j = sum_m dy.  `xhat_ws` is M x N scratch. */
void oracle_layernorm_bwd(int64_t M, int64_t N, const double *x, const double *dy,
                          const double *gamma, double eps, double *dx, double *dgamma,
                          double *dbeta, double *xhat_ws)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        const double *xr = x + m * N, *gr = dy + m * N;
        double *dr = dx + m * N, *hr = xhat_ws + m * N;
        double mu = csum(xr, N, 1) / (double)N;
        acc_t v = {0, 0};
        for (int64_t i = 0; i < N; ++i) acc_add(&v, (xr[i] - mu) * (xr[i] - mu));
        double rs = 1.0 / sqrt(acc_get(&v) / (double)N + eps);
        acc_t c1 = {0, 0}, c2 = {0, 0};
        for (int64_t i = 0; i < N; ++i) {
            hr[i] = (xr[i] - mu) * rs;
            double g = gr[i] * gamma[i];
            acc_add(&c1, g);
            acc_add(&c2, g * hr[i]);
        }
        double m1 = acc_get(&c1) / (double)N, m2 = acc_get(&c2) / (double)N;
        for (int64_t i = 0; i < N; ++i) dr[i] = rs * (gr[i] * gamma[i] - m1 - hr[i] * m2);
    }
    if (dgamma) column_sums(M, N, dy, xhat_ws, dgamma);
    if (dbeta) column_sums(M, N, dy, NULL, dbeta);
}

/* ----------------------------------------------------------------- RMSNorm */

/* rstd = 1/sqrt(mean(x^2) + eps); y = x * rstd * gamma.  rstd may be NULL. */
void oracle_rmsnorm_fwd(int64_t M, int64_t N, const double *x, const double *gamma,
                        double eps, double *y, double *rstd)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        const double *xr = x + m * N;
        double *yr = y + m * N;
        acc_t s = {0, 0};
        for (int64_t i = 0; i < N; ++i) acc_add(&s, xr[i] * xr[i]);
        double rs = 1.0 / sqrt(acc_get(&s) / (double)N + eps);
        for (int64_t i = 0; i < N; ++i) yr[i] = xr[i] * rs * gamma[i];
        if (rstd) rstd[m] = rs;
    }
}

/* RMSNorm backward, statistics recomputed in FP64:
 * xhat = x * rstd; g = dy * gamma; dx = rstd * (g - xhat * mean(g * xhat));
 * dgamma_j = sum_m dy * xhat.  `xhat_ws` is M x N scratch. */
void oracle_rmsnorm_bwd(int64_t M, int64_t N, const double *x, const double *dy,
                        const double *gamma, double eps, double *dx, double *dgamma,
                        double *xhat_ws)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        const double *xr = x + m * N, *gr = dy + m * N;
        double *dr = dx + m * N, *hr = xhat_ws + m * N;
        acc_t s = {0, 0};
        for (int64_t i = 0; i < N; ++i) acc_add(&s, xr[i] * xr[i]);
        double rs = 1.0 / sqrt(acc_get(&s) / (double)N + eps);
        acc_t c = {0, 0};
        for (int64_t i = 0; i < N; ++i) {
            hr[i] = xr[i] * rs;
            acc_add(&c, gr[i] * gamma[i] * hr[i]);
        }
        double mc = acc_get(&c) / (double)N;
        for (int64_t i = 0; i < N; ++i) dr[i] = rs * (gr[i] * gamma[i] - hr[i] * mc);
    }
    if (dgamma) column_sums(M, N, dy, xhat_ws, dgamma);
}

/* ------------------------------------------- the other evaluation workloads */

/* Softmax backward taking the logits (the softmax-logits workload): y is the
 * softmax of x as defined above, then dx_i = y_i * (dy_i - sum_j dy_j y_j). */
void oracle_softmax_logits_bwd(int64_t M, int64_t N, const double *x, const double *dy, double *dx)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        const double *xr = x + m * N, *gr = dy + m * N;
        double *dr = dx + m * N;
        double mx = -INFINITY;
        for (int64_t i = 0; i < N; ++i)
            if (xr[i] > mx) mx = xr[i];
        acc_t s = {0, 0};
        for (int64_t i = 0; i < N; ++i) acc_add(&s, exp(xr[i] - mx));
        const double sum = acc_get(&s);
        acc_t c = {0, 0};
        for (int64_t i = 0; i < N; ++i) acc_add(&c, gr[i] * (exp(xr[i] - mx) / sum));
        const double cs = acc_get(&c);
        for (int64_t i = 0; i < N; ++i) dr[i] = exp(xr[i] - mx) / sum * (gr[i] - cs);
    }
}

/* Row-wise quantisation (the int8-quantisation workload of Sec. IV-A).  Per
 * row: amax = max |x| (exact), and each code is the nearest point of the code
 * grid to the real number x * Q / amax, ties to the even code; the row scale is
 * amax / Q rounded once to FP32.  An all-zero row has scale 1 and codes 0.
 * fmt 0 (int8, Q = 127): the grid is the integers -127..127, stored two's
 * complement.  fmt 1 (e4m3, Q = 448): the grid is the finite e4m3fn values
 * (|x| <= amax keeps x * Q / amax inside +-448, so nothing saturates).
 *
 * The decisions are exact: x and amax are binary32 numbers (24-bit
 * significands), Q is a 7- or 9-bit integer, and every grid point or midpoint
 * g has at most 9 significant bits, so both sides of the comparison
 * x * Q <=> g * amax are exact products in binary64.  Nothing here evaluates
 * x * Q / amax in floating point to take a decision.
 * x holds FP32 values (BF16 inputs are exact in FP32). */

/* Sorted non-negative e4m3 magnitudes: codes 0x00..0x7E are increasing. */
static double e4m3_mag[127];
static void e4m3_mag_init(void)
{
    for (int c = 0; c < 127; ++c) e4m3_mag[c] = e4m3_value((uint8_t)c);
}

/* int8 code of x * Q / amax (amax > 0). */
static int8_t int8_code_exact(double x, double Q, double amax)
{
    const double xq = x * Q;                /* exact */
    /* f = floor(x * Q / amax): start from a nearby integer, then step until
     * f * amax <= xq < (f + 1) * amax holds exactly */
    double f = floor(xq / amax);
    while (f * amax > xq) f -= 1.0;
    while ((f + 1.0) * amax <= xq) f += 1.0;
    /* nearest of f, f + 1: compare 2 xq with (2f + 1) amax, both exact */
    const double lhs = 2.0 * xq, mid = (2.0 * f + 1.0) * amax;
    double c;
    if (lhs < mid)
        c = f;
    else if (lhs > mid)
        c = f + 1.0;
    else
        c = fmod(f, 2.0) == 0.0 ? f : f + 1.0;   /* tie: the even integer */
    if (c > 127.0) c = 127.0;
    if (c < -127.0) c = -127.0;
    return (int8_t)c;
}

/* e4m3 code of x * Q / amax (amax > 0). */
static uint8_t e4m3_code_exact(double x, double Q, double amax)
{
    const uint8_t sign = signbit(x) ? 0x80 : 0;
    const double aq = fabs(x) * Q;          /* exact */
    /* largest grid magnitude g[lo] with g[lo] * amax <= aq (binary search) */
    int lo = 0, hi = 126;
    while (lo < hi) {
        const int m = (lo + hi + 1) / 2;
        if (e4m3_mag[m] * amax <= aq) lo = m; else hi = m - 1;
    }
    int c = lo;
    if (lo < 126) {
        /* nearest of g[lo], g[lo + 1]: compare 2 aq with (g[lo] + g[lo + 1]) amax */
        const double lhs = 2.0 * aq, mid = (e4m3_mag[lo] + e4m3_mag[lo + 1]) * amax;
        if (lhs > mid || (lhs == mid && (lo & 1))) c = lo + 1;   /* tie: even code */
    }
    return sign | (uint8_t)c;
}

void oracle_quantize_rows(int64_t M, int64_t N, const float *x, int fmt, uint8_t *codes, float *scale)
{
    const float Qf = fmt == 0 ? 127.0f : 448.0f;
    e4m3_mag_init();
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        const float *xr = x + m * N;
        uint8_t *cr = codes + m * N;
        float amax = 0.0f;
        for (int64_t i = 0; i < N; ++i) {
            float a = fabsf(xr[i]);
            if (a > amax) amax = a;
        }
        volatile float sc = amax > 0.0f ? amax / Qf : 1.0f;   /* one correctly rounded FP32 division */
        scale[m] = sc;
        for (int64_t i = 0; i < N; ++i) {
            if (amax == 0.0f)
                cr[i] = fmt == 0 ? 0 : (signbit(xr[i]) ? 0x80 : 0);
            else if (fmt == 0)
                cr[i] = (uint8_t)int8_code_exact((double)xr[i], (double)Qf, (double)amax);
            else
                cr[i] = e4m3_code_exact((double)xr[i], (double)Qf, (double)amax);
        }
    }
}

/* The same codes taken with FP32 arithmetic instead: inv = Q / amax and
 * v = x * inv, each rounded to FP32, then v rounded to the grid.  This is not
 * the definition; the tests use it only to count where the two disagree. */
void oracle_quantize_rows_fp32_product(int64_t M, int64_t N, const float *x, int fmt, uint8_t *codes)
{
    const float Q = fmt == 0 ? 127.0f : 448.0f;
    for (int64_t m = 0; m < M; ++m) {
        const float *xr = x + m * N;
        float amax = 0.0f;
        for (int64_t i = 0; i < N; ++i)
            if (fabsf(xr[i]) > amax) amax = fabsf(xr[i]);
        volatile float inv = amax > 0.0f ? Q / amax : 1.0f;
        for (int64_t i = 0; i < N; ++i) {
            volatile float v = xr[i] * inv;
            if (fmt == 0) {
                float r = rintf(v);
                if (r > 127.0f) r = 127.0f;
                if (r < -127.0f) r = -127.0f;
                codes[m * N + i] = (uint8_t)(int8_t)r;
            } else {
                codes[m * N + i] = e4m3_from_double((double)v);
            }
        }
    }
}

/* Pearson-correlation backward.  Per row: xc = x - mean(x), yc = y - mean(y),
 * Sxx = sum xc^2, Syy = sum yc^2, Sxy = sum xc yc, r = Sxy / sqrt(Sxx Syy);
 * dr/dx_i = yc_i / sqrt(Sxx Syy) - r xc_i / Sxx (the terms through the means
 * vanish because sum yc = 0), symmetrically for y; scaled by dr[m]. */
void oracle_pearson_bwd(int64_t M, int64_t N, const double *x, const double *y, const double *dr,
                        double *dx, double *dy)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        const double *xr = x + m * N, *yr = y + m * N;
        const double mx = csum(xr, N, 1) / (double)N, my = csum(yr, N, 1) / (double)N;
        acc_t sxx = {0, 0}, syy = {0, 0}, sxy = {0, 0};
        for (int64_t i = 0; i < N; ++i) {
            const double a = xr[i] - mx, b = yr[i] - my;
            acc_add(&sxx, a * a);
            acc_add(&syy, b * b);
            acc_add(&sxy, a * b);
        }
        const double Sxx = acc_get(&sxx), Syy = acc_get(&syy), Sxy = acc_get(&sxy);
        const double den = sqrt(Sxx * Syy), r = Sxy / den;
        for (int64_t i = 0; i < N; ++i) {
            const double a = xr[i] - mx, b = yr[i] - my;
            dx[m * N + i] = dr[m] * (b / den - r * a / Sxx);
            dy[m * N + i] = dr[m] * (a / den - r * b / Syy);
        }
    }
}

/* Weighted-variance backward.  Per row: W = sum w, mu = sum w x / W,
 * v = sum w (x - mu)^2 / W; dv/dx_i = 2 w_i (x_i - mu) / W and
 * dv/dw_i = ((x_i - mu)^2 - v) / W (the terms through mu vanish because
 * sum w (x - mu) = 0); scaled by dv[m]. */
void oracle_wvar_bwd(int64_t M, int64_t N, const double *x, const double *w, const double *dv,
                     double *dx, double *dw)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        const double *xr = x + m * N, *wr = w + m * N;
        acc_t sw = {0, 0}, swx = {0, 0};
        for (int64_t i = 0; i < N; ++i) {
            acc_add(&sw, wr[i]);
            acc_add(&swx, wr[i] * xr[i]);
        }
        const double W = acc_get(&sw), mu = acc_get(&swx) / W;
        acc_t s2 = {0, 0};
        for (int64_t i = 0; i < N; ++i) acc_add(&s2, wr[i] * (xr[i] - mu) * (xr[i] - mu));
        const double v = acc_get(&s2) / W;
        for (int64_t i = 0; i < N; ++i) {
            const double d = xr[i] - mu;
            dx[m * N + i] = dv[m] * 2.0 * wr[i] * d / W;
            dw[m * N + i] = dv[m] * (d * d - v) / W;
        }
    }
}
