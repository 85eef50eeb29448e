/* Calls every entry point of the CPU oracle on small, exactly sized heap
 * buffers, so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * catches any out-of-bounds access or undefined operation in it.  Exits 0 when
 * every call returns and the results are finite where they must be. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_num_threads(void);
double oracle_sum(const double *v, int64_t n);
void oracle_decode_bf16(const uint16_t *in, double *out, int64_t n);
void oracle_encode_bf16(const double *in, uint16_t *out, int64_t n);
void oracle_decode_e4m3(const uint8_t *in, double *out, int64_t n);
void oracle_encode_e4m3(const double *in, uint8_t *out, int64_t n);
double oracle_e4m3_step(double v);
void oracle_softmax_fwd(int64_t M, int64_t N, const double *x, double *y);
void oracle_softmax_bwd(int64_t M, int64_t N, const double *y, const double *dy, double *dx);
void oracle_layernorm_fwd(int64_t M, int64_t N, const double *x, const double *gamma, const double *beta,
                          double eps, double *y, double *mean, double *rstd);
void oracle_layernorm_bwd(int64_t M, int64_t N, const double *x, const double *dy, const double *gamma, double eps,
                          double *dx, double *dgamma, double *dbeta, double *xhat_ws);
void oracle_rmsnorm_fwd(int64_t M, int64_t N, const double *x, const double *gamma, double eps, double *y,
                        double *rstd);
void oracle_rmsnorm_bwd(int64_t M, int64_t N, const double *x, const double *dy, const double *gamma, double eps,
                        double *dx, double *dgamma, double *xhat_ws);
void oracle_softmax_logits_bwd(int64_t M, int64_t N, const double *x, const double *dy, double *dx);
void oracle_quantize_rows(int64_t M, int64_t N, const float *x, int fmt, uint8_t *codes, float *scale);
void oracle_pearson_bwd(int64_t M, int64_t N, const double *x, const double *y, const double *dr, double *dx,
                        double *dy);
void oracle_wvar_bwd(int64_t M, int64_t N, const double *x, const double *w, const double *dv, double *dx,
                     double *dw);

static double *vec(int64_t n, unsigned seed, double lo, double hi)
{
    double *v = malloc(sizeof(double) * (size_t)n);
    unsigned s = seed * 2654435761u + 1u;
    for (int64_t i = 0; i < n; ++i) {
        s = s * 1664525u + 1013904223u;
        v[i] = lo + (hi - lo) * (double)(s >> 8) / 16777216.0;
    }
    return v;
}

static int finite_all(const double *v, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

int main(void)
{
    int bad = 0;
    const int64_t M = 3, N = 7, MN = M * N;
    double *x = vec(MN, 1, -3, 3), *dy = vec(MN, 2, -1, 1), *w = vec(MN, 3, 0.1, 1), *g = vec(N, 4, 0.5, 1.5);
    double *b = vec(N, 5, -0.1, 0.1), *rv = vec(M, 6, -1, 1);
    double *y = malloc(sizeof(double) * MN), *dx = malloc(sizeof(double) * MN), *d2 = malloc(sizeof(double) * MN);
    double *ws = malloc(sizeof(double) * MN), *mean = malloc(sizeof(double) * M), *rstd = malloc(sizeof(double) * M);
    double *dg = malloc(sizeof(double) * N), *db = malloc(sizeof(double) * N);
    bad |= oracle_num_threads() < 1;
    bad |= !isfinite(oracle_sum(x, MN));
    uint16_t *bits = malloc(sizeof(uint16_t) * 65536);
    double *dec = malloc(sizeof(double) * 65536);
    for (int i = 0; i < 65536; ++i) bits[i] = (uint16_t)i;
    oracle_decode_bf16(bits, dec, 65536);
    oracle_encode_bf16(x, bits, MN);
    uint8_t *codes = malloc(256);
    for (int i = 0; i < 256; ++i) codes[i] = (uint8_t)i;
    oracle_decode_e4m3(codes, dec, 256);
    oracle_encode_e4m3(x, codes, MN);
    bad |= !(oracle_e4m3_step(1.0) > 0);
    oracle_softmax_fwd(M, N, x, y);
    bad |= !finite_all(y, MN);
    oracle_softmax_bwd(M, N, y, dy, dx);
    oracle_softmax_logits_bwd(M, N, x, dy, d2);
    bad |= !finite_all(dx, MN) || !finite_all(d2, MN);
    oracle_layernorm_fwd(M, N, x, g, b, 1e-5, y, mean, rstd);
    oracle_layernorm_bwd(M, N, x, dy, g, 1e-5, dx, dg, db, ws);
    bad |= !finite_all(y, MN) || !finite_all(dx, MN) || !finite_all(dg, N) || !finite_all(db, N);
    oracle_rmsnorm_fwd(M, N, x, g, 1e-5, y, rstd);
    oracle_rmsnorm_bwd(M, N, x, dy, g, 1e-5, dx, dg, ws);
    bad |= !finite_all(y, MN) || !finite_all(dx, MN);
    float *xf = malloc(sizeof(float) * MN), *sc = malloc(sizeof(float) * M);
    uint8_t *q = malloc((size_t)MN);
    for (int64_t i = 0; i < MN; ++i) xf[i] = (float)x[i];
    oracle_quantize_rows(M, N, xf, 0, q, sc);
    oracle_quantize_rows(M, N, xf, 1, q, sc);
    oracle_pearson_bwd(M, N, x, dy, rv, dx, d2);
    bad |= !finite_all(dx, MN) || !finite_all(d2, MN);
    oracle_wvar_bwd(M, N, x, w, rv, dx, d2);
    bad |= !finite_all(dx, MN) || !finite_all(d2, MN);
    free(x); free(dy); free(w); free(g); free(b); free(rv); free(y); free(dx); free(d2); free(ws);
    free(mean); free(rstd); free(dg); free(db); free(bits); free(dec); free(codes); free(xf); free(sc); free(q);
    printf(bad ? "oracle sanitize: FAILED\n" : "oracle sanitize: ok\n");
    return bad;
}
