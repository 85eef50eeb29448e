// twopass.h -- the global-reread baseline (Sec. IV-A, the multi-pass kernel
// whose reread traffic N * b_reread appears in Eq. (4)).
//
// One workgroup per row (persistent over rows).  Each statistics stage
// streams the row from global memory in batches of U 128-bit vectors per
// thread; the output pass streams it again and writes.  Nothing is retained
// between passes, so a reread is served by L2 / Infinity Cache when the row
// is still there and by HBM otherwise.  Normalisation backward computes dx
// here; dgamma / dbeta come from k_colstats + k_colreduce.
#pragma once
#include "device.h"
#include "resident.h"

namespace credit {

// EPV FP32 parameters of the vector at column `col` with nv valid elements.
template <int DT>
__device__ __forceinline__ void load_params_n(const float *p, int64_t col, int nv, bool aligned, float *out) {
    constexpr int EPV = Io<DT>::EPV;
    if (nv == EPV && aligned) {
#pragma unroll
        for (int i = 0; i < EPV; i += 4) {
            float4 v = *(const float4 *)(p + col + i);
            out[i] = v.x; out[i + 1] = v.y; out[i + 2] = v.z; out[i + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < EPV; ++i) out[i] = i < nv ? p[col + i] : 0.f;
    }
}

// One vector of a row: full vectors use a 128-bit load through an
// under-aligned type (any row alignment), the trailing partial vector goes
// element by element; vectors past the end read as zero.
template <int DT, bool NT>
__device__ __forceinline__ u32x4 row_vec(const char *row, int64_t v, int nv) {
    constexpr int EPV = Io<DT>::EPV, B = Io<DT>::BYTES;
    if (nv == EPV) {
        const u32x4_u *p = (const u32x4_u *)(row + v * EPV * B);
        if constexpr (NT)
            return __builtin_nontemporal_load(p);
        else
            return *p;
    }
    return load_vec<DT, false>(row, v * EPV, nv, false);
}

template <int DT, int BLOCK, int U, bool NT, class F>
__device__ __forceinline__ void stream_row(const char *r0, const char *r1, int64_t N, bool, bool, F f) {
    constexpr int EPV = Io<DT>::EPV;
    const int64_t nvec = (N + EPV - 1) / EPV;
    for (int64_t v0 = threadIdx.x; v0 < nvec; v0 += (int64_t)BLOCK * U) {
        u32x4 d0[U], d1[U];
        int nv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t v = v0 + (int64_t)u * BLOCK;
            int64_t r = N - v * EPV;
            nv[u] = r <= 0 ? 0 : (r >= EPV ? EPV : (int)r);
            d0[u] = row_vec<DT, NT>(r0, v, nv[u]);
            if (r1) d1[u] = row_vec<DT, NT>(r1, v, nv[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) f(v0 + (int64_t)u * BLOCK, d0[u], r1 ? d1[u] : d0[u], nv[u]);
    }
}

// Stores one vector of a row (full: one under-aligned 128-bit store).
template <int DT>
__device__ __forceinline__ void row_store(char *row, int64_t v, int nv, u32x4 x) {
    constexpr int EPV = Io<DT>::EPV, B = Io<DT>::BYTES;
    if (nv == EPV)
        __builtin_nontemporal_store(x, (u32x4_u *)(row + v * EPV * B));
    else
        store_vec<DT>(row, v * EPV, nv, false, x);
}

// Stores the EPV one-byte codes of vector v of a row (nv valid).
template <int EPV>
__device__ __forceinline__ void code_store(char *row, int64_t v, int nv, const unsigned *w) {
    char *p = row + v * EPV;
    if (nv == EPV) {
        if constexpr (EPV == 4) {
            __builtin_nontemporal_store(w[0], (u32_u *)p);
        } else if constexpr (EPV == 8) {
            u32x2 x = {w[0], w[1]};
            __builtin_nontemporal_store(x, (u32x2_u *)p);
        } else {
            u32x4 x = {w[0], w[1], w[2], w[3]};
            __builtin_nontemporal_store(x, (u32x4_u *)p);
        }
        return;
    }
    for (int i = 0; i < nv; ++i) p[i] = (char)((w[i / 4] >> (8 * (i % 4))) & 0xffu);
}

template <int OP, int DT, int BLOCK, int U>
__global__ __launch_bounds__(BLOCK) void k_twopass(RowArgs a) {
    constexpr int EPV = Io<DT>::EPV, B = Io<DT>::BYTES, NW = BLOCK / 64;
    constexpr bool FP8 = DT == DT_FP8;
    constexpr bool TWO = OpTraits<OP>::TWO;
    __shared__ float red[2 * NW * 6];  // up to six statistics per reduction
    int parity = 0;
    const int64_t N = a.N;
    const float invN = 1.f / (float)N;
    const bool al0 = a.flags & F_ALIGN0, al1 = a.flags & F_ALIGN1, alp = a.flags & F_ALIGNP;

    for (int64_t row = blockIdx.x; row < a.M; row += gridDim.x) {
        const char *r0 = (const char *)a.in0 + row * a.ld0 * B;
        const char *r1 = TWO ? (const char *)a.in1 + row * a.ld1 * B : nullptr;
        char *orow = (char *)a.out + row * a.ldo * (byte_out(OP) ? 1 : B);
        char *orow1 = two_out(OP) ? (char *)a.out1 + row * a.ldo1 * B : nullptr;
        const bool writer = threadIdx.x == 0;

        if constexpr (OP == OP_SOFTMAX_FWD) {
            const float K = (FP8 ? a.s0[row] : 1.f) * kLog2e;
            float st[2] = {-INFINITY, 0.f};  // online base-2 (c, s)
            stream_row<DT, BLOCK, U, false>(r0, nullptr, N, al0, al1, [&](int64_t, u32x4 v, u32x4, int nv) {
                float q[EPV];
                decode<DT>(v, q, 1.f);
                float bm = -INFINITY;
#pragma unroll
                for (int i = 0; i < EPV; ++i)
                    if (i < nv) bm = fmaxf(bm, q[i]);
                if (bm == -INFINITY) return;
                const float cb = bm * K;
                if (cb > st[0]) {
                    st[1] = st[0] == -INFINITY ? 0.f : st[1] * fast_exp2(st[0] - cb);
                    st[0] = cb;
                }
#pragma unroll
                for (int i = 0; i < EPV; ++i)
                    if (i < nv) st[1] += fast_exp2(fmaf(q[i], K, -st[0]));
            });
            block_reduce<NW, 2>(st, MergeSoftmax(), red, parity);
            const float cmax = st[0], inv_s = 1.f / st[1];
            const float omul = FP8 ? kFp8Max : inv_s;
            const float csh = kExpShift - cmax, omuls = omul * kExpUnshift;
            if (FP8 && writer) a.so[row] = inv_s / kFp8Max;
            stream_row<DT, BLOCK, U, true>(r0, nullptr, N, al0, al1, [&](int64_t v, u32x4 d, u32x4, int nv) {
                if (nv == 0) return;
                float q[EPV], y[EPV];
                decode<DT>(d, q, 1.f);
#pragma unroll
                for (int i = 0; i < EPV; ++i) y[i] = fast_exp2(fmaf(q[i], K, csh)) * omuls;
                row_store<DT>(orow, v, nv, encode<DT>(y, 1.f));
            });
        } else if constexpr (OP == OP_LN_FWD || OP == OP_RMS_FWD || OP == OP_LN_BWD || OP == OP_RMS_BWD ||
                             OP == OP_LNQ_FWD) {
            constexpr bool LN = OP == OP_LN_FWD || OP == OP_LN_BWD || OP == OP_LNQ_FWD;
            constexpr bool QO = OP == OP_LNQ_FWD;  // e4m3 codes out from an FP32 / BF16 row
            constexpr bool BWD = OP == OP_LN_BWD || OP == OP_RMS_BWD;
            const float xs = FP8 ? a.s0[row] : 1.f;
            const float gs = (FP8 && BWD) ? a.s1[row] : 1.f;
            float mean = 0.f, rstd = 0.f;
            if (!BWD || (a.flags & F_RECOMPUTE)) {
                if constexpr (LN) {
                    // Chan merge of exact per-vector (count, mean, M2), the
                    // means taken relative to the row's first element K so
                    // that the merged means are deviations of the size of the
                    // row's spread; mean = K + the merged deviation
                    const float K = row_first<DT>(r0) * xs;
                    float st[3] = {0.f, 0.f, 0.f};
                    stream_row<DT, BLOCK, U, false>(r0, nullptr, N, al0, al1, [&](int64_t, u32x4 v, u32x4, int nv) {
                        if (nv == 0) return;
                        float x[EPV];
                        decode<DT>(v, x, xs);
                        float s = 0.f;
#pragma unroll
                        for (int i = 0; i < EPV; ++i) s += i < nv ? x[i] - K : 0.f;
                        const float n = (float)nv, m = s / n;
                        float m2 = 0.f;
#pragma unroll
                        for (int i = 0; i < EPV; ++i) {
                            float d = (x[i] - K) - m;
                            if (i < nv) m2 = fmaf(d, d, m2);
                        }
                        chan_merge(st[0], st[1], st[2], n, m, m2);
                    });
                    block_reduce<NW, 3>(st, MergeChan(), red, parity);
                    mean = K + st[1];
                    rstd = rsqrtf(st[2] * invN + a.eps);
                } else {
                    float st[1] = {0.f};
                    // each vector is summed on its own, then added: a thread's
                    // running sum takes N/(threads*EPV) additions instead of
                    // N/threads (rows of millions of elements)
                    stream_row<DT, BLOCK, U, false>(r0, nullptr, N, al0, al1, [&](int64_t, u32x4 v, u32x4, int) {
                        float x[EPV];
                        decode<DT>(v, x, xs);
                        float sv = 0.f;
#pragma unroll
                        for (int i = 0; i < EPV; ++i) sv = fmaf(x[i], x[i], sv);
                        st[0] += sv;
                    });
                    block_reduce<NW, 1>(st, MergeSum(), red, parity);
                    rstd = rsqrtf(st[0] * invN + a.eps);
                }
                if (writer) {
                    if (a.mean_out) a.mean_out[row] = mean;
                    if (a.rstd_out) a.rstd_out[row] = rstd;
                }
            } else {
                if constexpr (LN) mean = a.mean_in[row];
                rstd = a.rstd_in[row];
            }
            float c1 = 0.f, c2 = 0.f;
            if constexpr (BWD) {
                float st[2] = {0.f, 0.f};
                stream_row<DT, BLOCK, U, false>(r0, r1, N, al0, al1, [&](int64_t v, u32x4 dxv, u32x4 dyv, int nv) {
                    float x[EPV], dy[EPV], gm[EPV];
                    decode<DT>(dxv, x, xs);
                    decode<DT>(dyv, dy, gs);
                    load_params_n<DT>(a.gamma, v * EPV, nv, alp, gm);
                    float sg = 0.f, sgx = 0.f;  // per vector, then added
#pragma unroll
                    for (int i = 0; i < EPV; ++i) {
                        float xh = (x[i] - mean) * rstd;
                        float g = dy[i] * gm[i];
                        sg += g;
                        sgx = fmaf(g, xh, sgx);
                    }
                    st[0] += sg;
                    st[1] += sgx;
                });
                block_reduce<NW, 2>(st, MergeSum(), red, parity);
                c1 = LN ? st[0] * invN : 0.f;
                c2 = st[1] * invN;
            }
            auto apply = [&](int64_t v, u32x4 d0v, u32x4 d1v, int nv, float *y) {
                float x[EPV], gm[EPV];
                decode<DT>(d0v, x, xs);
                load_params_n<DT>(a.gamma, v * EPV, nv, alp, gm);
                if constexpr (BWD) {
                    float dy[EPV];
                    decode<DT>(d1v, dy, gs);
#pragma unroll
                    for (int i = 0; i < EPV; ++i) {
                        float xh = (x[i] - mean) * rstd;
                        y[i] = rstd * (dy[i] * gm[i] - c1 - xh * c2);
                    }
                } else if constexpr (LN) {
                    float bb[EPV];
                    load_params_n<DT>(a.beta, v * EPV, nv, alp, bb);
#pragma unroll
                    for (int i = 0; i < EPV; ++i) y[i] = fmaf((x[i] - mean) * rstd, gm[i], bb[i]);
                } else {
#pragma unroll
                    for (int i = 0; i < EPV; ++i) y[i] = x[i] * rstd * gm[i];
                }
            };
            float oinv = 1.f;
            if constexpr (FP8 || QO) {
                float am[1] = {0.f};
                stream_row<DT, BLOCK, U, false>(r0, r1, N, al0, al1, [&](int64_t v, u32x4 d0v, u32x4 d1v, int nv) {
                    float y[EPV];
                    apply(v, d0v, d1v, nv, y);
#pragma unroll
                    for (int i = 0; i < EPV; ++i)
                        if (i < nv) am[0] = fmaxf(am[0], fabsf(y[i]));
                });
                block_reduce<NW, 1>(am, MergeMax(), red, parity);
                oinv = am[0] > 0.f ? kFp8Max / am[0] : 1.f;
                if (writer) a.so[row] = am[0] > 0.f ? am[0] / kFp8Max : 1.f;
            }
            stream_row<DT, BLOCK, U, true>(r0, r1, N, al0, al1, [&](int64_t v, u32x4 d0v, u32x4 d1v, int nv) {
                if (nv == 0) return;
                float y[EPV];
                apply(v, d0v, d1v, nv, y);
                if constexpr (QO) {
                    unsigned w[EPV / 4];
                    quant_codes<false, EPV>(y, oinv, w);
                    code_store<EPV>(orow, v, nv, w);
                } else {
                    row_store<DT>(orow, v, nv, encode<DT>(y, oinv));
                }
            });
        } else if constexpr (OP == OP_SOFTMAX_BWD) {
            const float ys = FP8 ? a.s0[row] : 1.f, gs = FP8 ? a.s1[row] : 1.f;
            float st[1] = {0.f};
            stream_row<DT, BLOCK, U, false>(r0, r1, N, al0, al1, [&](int64_t, u32x4 yv, u32x4 gv, int) {
                float y[EPV], g[EPV];
                decode<DT>(yv, y, ys);
                decode<DT>(gv, g, gs);
                float sv = 0.f;  // per vector, then added
#pragma unroll
                for (int i = 0; i < EPV; ++i) sv = fmaf(g[i], y[i], sv);
                st[0] += sv;
            });
            block_reduce<NW, 1>(st, MergeSum(), red, parity);
            const float cs = st[0];
            float oinv = 1.f;
            if constexpr (FP8) {
                float am[1] = {0.f};
                stream_row<DT, BLOCK, U, false>(r0, r1, N, al0, al1, [&](int64_t, u32x4 yv, u32x4 gv, int) {
                    float y[EPV], g[EPV];
                    decode<DT>(yv, y, ys);
                    decode<DT>(gv, g, gs);
#pragma unroll
                    for (int i = 0; i < EPV; ++i) am[0] = fmaxf(am[0], fabsf(y[i] * (g[i] - cs)));
                });
                block_reduce<NW, 1>(am, MergeMax(), red, parity);
                oinv = am[0] > 0.f ? kFp8Max / am[0] : 1.f;
                if (writer) a.so[row] = am[0] > 0.f ? am[0] / kFp8Max : 1.f;
            }
            stream_row<DT, BLOCK, U, true>(r0, r1, N, al0, al1, [&](int64_t v, u32x4 yv, u32x4 gv, int nv) {
                if (nv == 0) return;
                float y[EPV], g[EPV], dx[EPV];
                decode<DT>(yv, y, ys);
                decode<DT>(gv, g, gs);
#pragma unroll
                for (int i = 0; i < EPV; ++i) dx[i] = y[i] * (g[i] - cs);
                row_store<DT>(orow, v, nv, encode<DT>(dx, oinv));
            });
        } else if constexpr (OP == OP_SMXL_BWD) {
            // pass 1 streams x and dy with online (c, s, t); the output pass
            // streams them again
            const float K = (FP8 ? a.s0[row] : 1.f) * kLog2e, gs = FP8 ? a.s1[row] : 1.f;
            float st[3] = {-INFINITY, 0.f, 0.f};
            stream_row<DT, BLOCK, U, false>(r0, r1, N, al0, al1, [&](int64_t, u32x4 xv, u32x4 gv, int nv) {
                float q[EPV], g[EPV];
                decode<DT>(xv, q, 1.f);
                decode<DT>(gv, g, gs);
                float bm = -INFINITY;
#pragma unroll
                for (int i = 0; i < EPV; ++i)
                    if (i < nv) bm = fmaxf(bm, q[i]);
                if (bm == -INFINITY) return;
                const float cb = bm * K;
                if (cb > st[0]) {
                    const float f = st[0] == -INFINITY ? 0.f : fast_exp2(st[0] - cb);
                    st[1] *= f;
                    st[2] *= f;
                    st[0] = cb;
                }
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    if (i < nv) {
                        const float e = fast_exp2(fmaf(q[i], K, -st[0]));
                        st[1] += e;
                        st[2] = fmaf(e, g[i], st[2]);
                    }
                }
            });
            block_reduce<NW, 3>(st, MergeSoftmax3(), red, parity);
            const float cmax = st[0], inv_s = 1.f / st[1], cdot = st[2] * inv_s;
            const float csh = kExpShift - cmax, invs_s = inv_s * kExpUnshift;
            auto h = [&](u32x4 xv, u32x4 gv, float *dx) {
                float q[EPV], g[EPV];
                decode<DT>(xv, q, 1.f);
                decode<DT>(gv, g, gs);
#pragma unroll
                for (int i = 0; i < EPV; ++i) dx[i] = fast_exp2(fmaf(q[i], K, csh)) * invs_s * (g[i] - cdot);
            };
            float oinv = 1.f;
            if constexpr (FP8) {
                float am[1] = {0.f};
                stream_row<DT, BLOCK, U, false>(r0, r1, N, al0, al1, [&](int64_t, u32x4 xv, u32x4 gv, int nv) {
                    float dx[EPV];
                    h(xv, gv, dx);
#pragma unroll
                    for (int i = 0; i < EPV; ++i)
                        if (i < nv) am[0] = fmaxf(am[0], fabsf(dx[i]));
                });
                block_reduce<NW, 1>(am, MergeMax(), red, parity);
                oinv = am[0] > 0.f ? kFp8Max / am[0] : 1.f;
                if (writer) a.so[row] = am[0] > 0.f ? am[0] / kFp8Max : 1.f;
            }
            stream_row<DT, BLOCK, U, true>(r0, r1, N, al0, al1, [&](int64_t v, u32x4 xv, u32x4 gv, int nv) {
                if (nv == 0) return;
                float dx[EPV];
                h(xv, gv, dx);
                row_store<DT>(orow, v, nv, encode<DT>(dx, oinv));
            });
        } else if constexpr (is_quant(OP)) {
            constexpr bool I8 = OP == OP_QUANT_I8;
            float am[1] = {0.f};
            stream_row<DT, BLOCK, U, false>(r0, nullptr, N, al0, al1, [&](int64_t, u32x4 xv, u32x4, int) {
                float q[EPV];
                decode<DT>(xv, q, 1.f);
#pragma unroll
                for (int i = 0; i < EPV; ++i) am[0] = fmaxf(am[0], fabsf(q[i]));  // invalid elements read 0
            });
            block_reduce<NW, 1>(am, MergeMax(), red, parity);
            const float qm = I8 ? 127.f : kFp8Max;
            const float amx = am[0];
            float qsc = 1.f, inv = 1.f;  // an all-zero row: every code is 0
            if (amx > 0.f) quant_row_factors(amx, qm, qsc, inv);
            if (writer) a.so[row] = amx > 0.f ? amx / qm : 1.f;
            stream_row<DT, BLOCK, U, true>(r0, nullptr, N, al0, al1, [&](int64_t v, u32x4 xv, u32x4, int nv) {
                if (nv == 0) return;
                float q[EPV];
                decode<DT>(xv, q, 1.f);
                unsigned w[EPV / 4];
                quant_codes_exact<I8, EPV>(q, qsc, inv, amx > 0.f ? amx : 1.f, w);
                code_store<EPV>(orow, v, nv, w);
            });
        } else if constexpr (OP == OP_PEARSON_BWD) {
            // pass 1: exact per-vector co-moments, merged pairwise
            float st[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            stream_row<DT, BLOCK, U, false>(r0, r1, N, al0, al1, [&](int64_t, u32x4 xv, u32x4 yv, int nv) {
                if (nv == 0) return;
                float x[EPV], y[EPV];
                decode<DT>(xv, x, 1.f);
                decode<DT>(yv, y, 1.f);
                float sx = 0.f, sy = 0.f;
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    sx += x[i];
                    sy += y[i];
                }
                const float n = (float)nv, mx = sx / n, my = sy / n;
                float cxx = 0.f, cyy = 0.f, cxy = 0.f;
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    if (i < nv) {
                        const float dx = x[i] - mx, dy = y[i] - my;
                        cxx = fmaf(dx, dx, cxx);
                        cyy = fmaf(dy, dy, cyy);
                        cxy = fmaf(dx, dy, cxy);
                    }
                }
                co_merge(st, n, mx, my, cxx, cyy, cxy);
            });
            block_reduce<NW, 6>(st, MergeCo(), red, parity);
            const float mx = st[1], my = st[2];
            const float ix = rsqrtf(st[3]), iy = rsqrtf(st[4]);
            const float dr = a.rowg[row];
            const float r = st[5] * ix * iy;
            const float ca = dr * ix * iy, cbx = dr * r / st[3], cby = dr * r / st[4];
            stream_row<DT, BLOCK, U, true>(r0, r1, N, al0, al1, [&](int64_t v, u32x4 xv, u32x4 yv, int nv) {
                if (nv == 0) return;
                float x[EPV], y[EPV], gx[EPV], gy[EPV];
                decode<DT>(xv, x, 1.f);
                decode<DT>(yv, y, 1.f);
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    const float xc = x[i] - mx, yc = y[i] - my;
                    gx[i] = fmaf(ca, yc, -cbx * xc);
                    gy[i] = fmaf(ca, xc, -cby * yc);
                }
                row_store<DT>(orow, v, nv, encode<DT>(gx, 1.f));
                row_store<DT>(orow1, v, nv, encode<DT>(gy, 1.f));
            });
        } else if constexpr (OP == OP_WVAR_BWD) {
            // pass 1: exact per-vector weighted (W, mean, M2), Chan-merged
            float st[3] = {0.f, 0.f, 0.f};
            stream_row<DT, BLOCK, U, false>(r0, r1, N, al0, al1, [&](int64_t, u32x4 xv, u32x4 wv, int nv) {
                if (nv == 0) return;
                float x[EPV], w[EPV];
                decode<DT>(xv, x, 1.f);
                decode<DT>(wv, w, 1.f);
                float sw = 0.f, swx = 0.f;
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    sw += w[i];
                    swx = fmaf(w[i], x[i], swx);
                }
                if (sw == 0.f) return;
                const float m = swx / sw;
                float m2 = 0.f;
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    const float d = x[i] - m;
                    m2 = fmaf(w[i] * d, d, m2);
                }
                chan_merge(st[0], st[1], st[2], sw, m, m2);
            });
            block_reduce<NW, 3>(st, MergeChan(), red, parity);
            const float W = st[0], mu = st[1], var = st[2] / W;
            const float f = a.rowg[row] / W, f2 = 2.f * f;
            stream_row<DT, BLOCK, U, true>(r0, r1, N, al0, al1, [&](int64_t v, u32x4 xv, u32x4 wv, int nv) {
                if (nv == 0) return;
                float x[EPV], w[EPV], gx[EPV], gw[EPV];
                decode<DT>(xv, x, 1.f);
                decode<DT>(wv, w, 1.f);
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    const float d = x[i] - mu;
                    gx[i] = f2 * w[i] * d;
                    gw[i] = f * fmaf(d, d, -var);
                }
                row_store<DT>(orow, v, nv, encode<DT>(gx, 1.f));
                row_store<DT>(orow1, v, nv, encode<DT>(gw, 1.f));
            });
        }
    }
}

// dgamma / dbeta partials for the two-pass normalisation backward: block
// (bx, by) covers 256 column vectors and the rows [by*M/RB, (by+1)*M/RB);
// partial[by][p][col] = sum over those rows of dy*xhat (p = 0) and dy (p = 1).
template <int DT, bool LN>
__global__ __launch_bounds__(256) void k_colstats(RowArgs a, int rowblocks) {
    constexpr int EPV = Io<DT>::EPV, B = Io<DT>::BYTES, NCP = LN ? 2 : 1;
    constexpr bool FP8 = DT == DT_FP8;
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t col = v * EPV;
    const int64_t r = a.N - col;
    const int nv = r <= 0 ? 0 : (r >= EPV ? EPV : (int)r);
    if (nv == 0) return;
    const int64_t rb = blockIdx.y;
    const int64_t m0 = rb * a.M / rowblocks, m1 = (rb + 1) * a.M / rowblocks;
    const bool al0 = a.flags & F_ALIGN0, al1 = a.flags & F_ALIGN1;
    float ag[EPV], ab[EPV];
#pragma unroll
    for (int i = 0; i < EPV; ++i) ag[i] = ab[i] = 0.f;
    for (int64_t m = m0; m < m1; ++m) {
        const float xs = FP8 ? a.s0[m] : 1.f, gs = FP8 ? a.s1[m] : 1.f;
        const float mean = LN ? a.mean_in[m] : 0.f, rstd = a.rstd_in[m];
        float x[EPV], dy[EPV];
        decode<DT>(load_vec<DT, true>((const char *)a.in0 + m * a.ld0 * B, col, nv, al0), x, xs);
        decode<DT>(load_vec<DT, true>((const char *)a.in1 + m * a.ld1 * B, col, nv, al1), dy, gs);
#pragma unroll
        for (int i = 0; i < EPV; ++i) {
            ag[i] = fmaf(dy[i], (x[i] - mean) * rstd, ag[i]);
            ab[i] += dy[i];
        }
    }
    float *dst = a.colpart + rb * NCP * a.N;
#pragma unroll
    for (int i = 0; i < EPV; ++i) {
        if (i < nv) {
            dst[col + i] = ag[i];
            if (LN) dst[a.N + col + i] = ab[i];
        }
    }
}

}  // namespace credit
