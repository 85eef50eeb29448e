// mlp.hip -- kernels of the learned plan selector: a 12 -> 64 -> 64 -> C
// ReLU network over standardized shape features, trained full-batch with a
// masked soft-target cross-entropy and Adam.  All reductions run in a fixed
// order (no atomics), so training is deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace credit {

// z[s][f] = (raw[s][f] - mu[f]) / sd[f]
__global__ __launch_bounds__(256) void k_mlp_standardize(const float *raw, const float *mu, const float *sd, float *z,
                                                         int64_t n, int nf) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n * nf) return;
    const int f = (int)(i % nf);
    z[i] = (raw[i] - mu[f]) / sd[f];
}

// out[s][o] = act(b[o] + sum_i W[o][i] * in[s][i]), act = ReLU when relu != 0
__global__ __launch_bounds__(256) void k_mlp_dense(const float *in, const float *W, const float *b, float *out,
                                                   int64_t n, int I, int O, int relu) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * O) return;
    const int64_t s = t / O;
    const int o = (int)(t % O);
    float acc = b[o];
    const float *w = W + (int64_t)o * I;
    const float *x = in + s * I;
    for (int i = 0; i < I; ++i) acc = fmaf(w[i], x[i], acc);
    out[t] = relu ? fmaxf(acc, 0.f) : acc;
}

// Per sample: p = softmax of the logits over legal classes; loss_s =
// -sum_c t_c log p_c; dlogits = (p - t) / n on legal classes, 0 elsewhere.
__global__ __launch_bounds__(256) void k_mlp_xent(const float *logits, const float *targets, const uint8_t *mask,
                                                  float *dlogits, float *loss, int64_t n, int C) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const float *l = logits + s * C;
    const float *t = targets + s * C;
    const uint8_t *m = mask + s * C;
    float mx = -INFINITY;
    for (int c = 0; c < C; ++c)
        if (m[c]) mx = fmaxf(mx, l[c]);
    float z = 0.f;
    for (int c = 0; c < C; ++c)
        if (m[c]) z += expf(l[c] - mx);
    const float lz = logf(z);
    float ls = 0.f;
    const float inv_n = 1.f / (float)n;
    for (int c = 0; c < C; ++c) {
        float g = 0.f;
        if (m[c]) {
            const float lp = l[c] - mx - lz;
            ls -= t[c] * lp;
            g = (expf(lp) - t[c]) * inv_n;
        }
        dlogits[s * C + c] = g;
    }
    loss[s] = ls;
}

// Sum of n per-sample losses divided by n (one workgroup, fixed order).
__global__ __launch_bounds__(256) void k_mlp_mean(const float *v, int64_t n, float *out) {
    __shared__ float part[256];
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += v[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int i = 0; i < 256; ++i) t += part[i];
        out[0] = t / (float)n;
    }
}

// dW[o][i] = sum_s dout[s][o] * in[s][i]; db[o] = sum_s dout[s][o]
// (one thread per weight; thread i == I of row o computes db[o]).
__global__ __launch_bounds__(256) void k_mlp_dense_bwd_w(const float *dout, const float *in, float *dW, float *db,
                                                         int64_t n, int I, int O) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)O * (I + 1)) return;
    const int o = (int)(t / (I + 1));
    const int i = (int)(t % (I + 1));
    float acc = 0.f;
    if (i < I) {
        for (int64_t s = 0; s < n; ++s) acc = fmaf(dout[s * O + o], in[s * I + i], acc);
        dW[(int64_t)o * I + i] = acc;
    } else {
        for (int64_t s = 0; s < n; ++s) acc += dout[s * O + o];
        db[o] = acc;
    }
}

// din[s][i] = [act[s][i] > 0] * sum_o dout[s][o] * W[o][i]  (ReLU backward)
__global__ __launch_bounds__(256) void k_mlp_dense_bwd_in(const float *dout, const float *W, const float *act,
                                                          float *din, int64_t n, int I, int O) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * I) return;
    const int64_t s = t / I;
    const int i = (int)(t % I);
    float acc = 0.f;
    for (int o = 0; o < O; ++o) acc = fmaf(dout[s * O + o], W[(int64_t)o * I + i], acc);
    din[t] = act[t] > 0.f ? acc : 0.f;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
__global__ __launch_bounds__(256) void k_mlp_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                                                  float b1, float b2, float eps, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

const void *mlp_kernel(int which) {
    switch (which) {
    case 0: return (const void *)&k_mlp_standardize;
    case 1: return (const void *)&k_mlp_dense;
    case 2: return (const void *)&k_mlp_xent;
    case 3: return (const void *)&k_mlp_mean;
    case 4: return (const void *)&k_mlp_dense_bwd_w;
    case 5: return (const void *)&k_mlp_dense_bwd_in;
    case 6: return (const void *)&k_mlp_adam;
    }
    return nullptr;
}

}  // namespace credit
