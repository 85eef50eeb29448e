// multirow.h -- the LayerNorm / RMSNorm forward with R rows per workgroup.
//
// The row-resident / split-row kernel (resident.h) handles one row of its
// row group at a time, so every row re-reads the FP32 gamma (and beta) of its
// slice -- 8 bytes per element against 1-2 bytes of FP8 / BF16 data -- and
// pays one exchange round per statistics stage.  Here a workgroup holds the
// same slice (the same columns) of R consecutive rows at once: each parameter
// vector is loaded once per R rows, and each exchange round carries the
// statistics of all R rows (Eq. (5) with q = R x the per-row statistics).
// The row arithmetic is the one of resident.h: LayerNorm moments about a
// per-thread shift, merged with Chan's update on means taken relative to the
// row's first element; RMSNorm sums of squares; FP8 output through a per-row
// amax stage, after which the quantising pass recomputes y from the resident
// x, gamma and beta (no y is kept across the stage).
#pragma once
#include "resident.h"

namespace credit {

// Waves per SIMD the register allocation must allow: R x VPT retained
// vectors, the working registers of the statistics and output passes (FP8
// decodes 16 values per vector) and 2 x R per-row factors.
template <int OP, int DT, int VPT, int R> constexpr int multirow_waves() {
    constexpr int data = R * VPT * 4;
    constexpr int work = 80 + (DT == DT_FP8 ? (OP == OP_LN_FWD ? 64 : 32) : 0) + 4 * R;
    constexpr int w = 512 / (data + work);
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// Chan merge of R (count, mean, M2) tuples laid out [R][3].
template <int R> struct MergeChanR {
    __device__ __forceinline__ void operator()(float (&a)[3 * R], const float (&b)[3 * R]) const {
#pragma unroll
        for (int i = 0; i < R; ++i) chan_merge(a[3 * i], a[3 * i + 1], a[3 * i + 2], b[3 * i], b[3 * i + 1], b[3 * i + 2]);
    }
};
template <int R> struct MergeMaxR {
    __device__ __forceinline__ void operator()(float (&a)[R], const float (&b)[R]) const {
#pragma unroll
        for (int i = 0; i < R; ++i) a[i] = fmaxf(a[i], b[i]);
    }
};

template <int OP, int DT, int VPT, int R, bool AL, bool FULLS>
__device__ __forceinline__ void rows_loop(const RowArgs &a, int c, int grp, const Slice &sl, float *red, float *xb) {
    constexpr int EPV = Io<DT>::EPV, B = Io<DT>::BYTES;
    constexpr bool FP8 = DT == DT_FP8;
    constexpr bool LN = OP == OP_LN_FWD;
    constexpr int Q = LN ? 2 : 1;  // exchanged statistics per row
    static_assert(OP == OP_LN_FWD || OP == OP_RMS_FWD, "norm forward only");
    int parity = 0;
    const int tid = threadIdx.x;
    const float invN = 1.f / (float)a.N;
    auto ok_of = [&](int j) -> bool { return FULLS || (int64_t)(j * kBlock + tid) < sl.nfv; };
    const bool tail = !FULLS && sl.tail_n > 0 && tid == sl.owner;
    const int tn = sl.tail_n;
    const int64_t tcol = sl.c0 + sl.nfv * EPV;
    float held = 0.f;
    if (FULLS) {
        held = (float)(VPT * EPV);
    } else {
        for (int j = 0; j < VPT; ++j) held += ok_of(j) ? (float)EPV : 0.f;
        if (tail) held += (float)tn;
    }
    const int64_t nblk = (a.M + R - 1) / R;
    for (int64_t blk = grp; blk < nblk; blk += a.groups) {
        const int64_t row0 = blk * R;
        const int nr = (int)(a.M - row0 < R ? a.M - row0 : R);  // rows of this block (uniform)
        uint32_t toff = (uint32_t)tid * 16u, poff = (uint32_t)tid * (EPV * 4u);
        asm volatile("" : "+v"(toff));
        asm volatile("" : "+v"(poff));
        auto doff = [&](int j) -> uint32_t { return (FULLS || ok_of(j)) ? toff + (uint32_t)j * (kBlock * 16u) : 0u; };
        auto pofs = [&](int j) -> uint32_t {
            return (FULLS || ok_of(j)) ? poff + (uint32_t)j * (kBlock * EPV * 4u) : 0u;
        };
        const char *rb[R];
        char *ob[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int64_t row = i < nr ? row0 + i : row0;  // absent rows alias the first (never stored)
            rb[i] = (const char *)a.in0 + row * a.ld0 * B;
            ob[i] = (char *)a.out + row * a.ldo * B;
        }
        u32x4 d[R][VPT];
        if (FULLS || sl.nfv > 0) {
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < VPT; ++j) d[i][j] = vload_nt<AL>(rb[i] + sl.c0 * B, doff(j));
        } else {
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < VPT; ++j) d[i][j] = u32x4{0u, 0u, 0u, 0u};
        }
        u32x4 t[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            t[i] = u32x4{0u, 0u, 0u, 0u};
            if (tail) t[i] = load_vec<DT, false>(rb[i], tcol, tn, false);
        }
        auto fresh = [&]() {
#pragma unroll
            for (int i = 0; i < R; ++i) opaque<VPT>(d[i]);
        };
        if constexpr (!FULLS) {
            fresh();
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < VPT; ++j) d[i][j] = ok_of(j) ? d[i][j] : u32x4{0u, 0u, 0u, 0u};
        }
        float xs[R];
#pragma unroll
        for (int i = 0; i < R; ++i) xs[i] = FP8 ? a.s0[i < nr ? row0 + i : row0] : 1.f;

        // ---- statistics of the R rows, one exchange round for all of them
        float mean_q[R], amul[R];
        if constexpr (LN) {
            float st[3 * R], K[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                K[i] = row_first<DT>(rb[i]);
                float q0[EPV], qt[EPV];
                decode<DT>(d[i][0], q0, 1.f);
                decode<DT>(t[i], qt, 1.f);
                const float Kt = (FULLS || ok_of(0)) ? q0[0] : (tail ? qt[0] : K[i]);
                float s1 = 0.f, s2 = 0.f;
                fresh();
#pragma unroll
                for (int j = 0; j < VPT; ++j) {
                    float q[EPV];
                    decode<DT>(d[i][j], q, 1.f);
                    const bool ok = ok_of(j);
#pragma unroll
                    for (int e = 0; e < EPV; ++e) {
                        const float dd = ok ? q[e] - Kt : 0.f;
                        s1 += dd;
                        s2 = fmaf(dd, dd, s2);
                    }
                    keep_order(s1, s2);
                }
                if (tail) {
                    float q[EPV];
                    decode<DT>(t[i], q, 1.f);
#pragma unroll
                    for (int e = 0; e < EPV; ++e) {
                        const float dd = e < tn ? q[e] - Kt : 0.f;
                        s1 += dd;
                        s2 = fmaf(dd, dd, s2);
                    }
                }
                st[3 * i] = held;
                st[3 * i + 1] = 0.f;
                st[3 * i + 2] = 0.f;
                if (held > 0.f) {
                    const float m = s1 / held;
                    st[3 * i + 1] = (Kt - K[i]) + m;
                    st[3 * i + 2] = fmaxf(s2 - s1 * m, 0.f);
                }
            }
            block_reduce<4, 3 * R>(st, MergeChanR<R>(), red, parity);
            if (a.k > 1) {
                float mine[2 * R];
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    mine[2 * i] = st[3 * i + 1];
                    mine[2 * i + 1] = st[3 * i + 2];
                }
                exchange<2 * R>(a, blk, 0, c, mine, xb);
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    float n = 0.f, mean = 0.f, m2 = 0.f;
                    for (int m = 0; m < a.k; ++m) {
                        const int64_t lo = (int64_t)m * a.chunk;
                        const int64_t cnt = a.N - lo < a.chunk ? a.N - lo : a.chunk;
                        chan_merge(n, mean, m2, cnt > 0 ? (float)cnt : 0.f, xb[2 * R * m + 2 * i],
                                   xb[2 * R * m + 2 * i + 1]);
                    }
                    st[3 * i + 1] = mean;
                    st[3 * i + 2] = m2;
                }
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
                mean_q[i] = K[i] + st[3 * i + 1];
                const float rstd = rsqrtf(xs[i] * xs[i] * (st[3 * i + 2] * invN) + a.eps);
                amul[i] = xs[i] * rstd;
                if (c == 0 && tid == 0 && i < nr) {
                    if (a.mean_out) a.mean_out[row0 + i] = xs[i] * mean_q[i];
                    if (a.rstd_out) a.rstd_out[row0 + i] = rstd;
                }
            }
        } else {
            float st[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                float s = 0.f;
                fresh();
#pragma unroll
                for (int j = 0; j < VPT; ++j) {
                    float q[EPV];
                    decode<DT>(d[i][j], q, 1.f);
#pragma unroll
                    for (int e = 0; e < EPV; ++e) s = fmaf(q[e], q[e], s);
                    keep_order(s);
                }
                if (tail) {
                    float q[EPV];
                    decode<DT>(t[i], q, 1.f);
#pragma unroll
                    for (int e = 0; e < EPV; ++e) s = fmaf(q[e], q[e], s);
                }
                st[i] = s;
            }
            block_reduce<4, R>(st, MergeSum(), red, parity);
            if (a.k > 1) {
                exchange<R>(a, blk, 0, c, st, xb);
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    float s = xb[i];
                    for (int m = 1; m < a.k; ++m) s += xb[R * m + i];
                    st[i] = s;
                }
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
                mean_q[i] = 0.f;
                const float rstd = rsqrtf(xs[i] * xs[i] * (st[i] * invN) + a.eps);
                amul[i] = xs[i] * rstd;
                if (c == 0 && tid == 0 && i < nr) {
                    if (a.mean_out) a.mean_out[row0 + i] = 0.f;
                    if (a.rstd_out) a.rstd_out[row0 + i] = rstd;
                }
            }
        }
        auto h = [&](int i, const float *q, const float *g, const float *bb, float *y) {
#pragma unroll
            for (int e = 0; e < EPV; ++e) {
                if constexpr (LN)
                    y[e] = fmaf((q[e] - mean_q[i]) * amul[i], g[e], bb[e]);
                else
                    y[e] = q[e] * amul[i] * g[e];
            }
        };
        // a pass over the slots: each parameter vector is loaded once for the
        // R rows; with store == false it only takes the rows' amax
        float oinv[R];
#pragma unroll
        for (int i = 0; i < R; ++i) oinv[i] = 1.f;
        auto pass = [&](bool store, float (&amax)[R]) {
            fresh();
            const float *gp = a.gamma, *bp = a.beta;
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                __builtin_amdgcn_sched_barrier(0);
                float g[EPV], bb[LN ? EPV : 1];
                if (FULLS || sl.nfv > 0) {  // a slice of no full vector reads no parameter vector
                    load_params_v<DT, AL>(gp + sl.c0, pofs(j), g);
                    if constexpr (LN) load_params_v<DT, AL>(bp + sl.c0, pofs(j), bb);
                } else {
#pragma unroll
                    for (int e = 0; e < EPV; ++e) g[e] = bb[LN ? e : 0] = 0.f;
                }
                const bool ok = ok_of(j);
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    float q[EPV], y[EPV];
                    decode<DT>(d[i][j], q, 1.f);
                    h(i, q, g, LN ? bb : g, y);
                    if (store) {
                        if ((FULLS || ok) && i < nr)
                            vstore_nt<AL>(ob[i] + sl.c0 * B, toff + (uint32_t)j * (kBlock * 16u),
                                          encode<DT>(y, oinv[i]));
                    } else {
#pragma unroll
                        for (int e = 0; e < EPV; ++e) amax[i] = fmaxf(amax[i], ok ? fabsf(y[e]) : 0.f);
                    }
                }
            }
            if (tail) {
                float g[EPV], bb[EPV];
                load_params_tail<DT>(a.gamma, tcol, tn, g);
                if constexpr (LN) load_params_tail<DT>(a.beta, tcol, tn, bb);
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    float q[EPV], y[EPV];
                    decode<DT>(t[i], q, 1.f);
                    h(i, q, g, bb, y);
                    if (store) {
                        if (i < nr) store_vec<DT>(ob[i], tcol, tn, false, encode<DT>(y, oinv[i]));
                    } else {
#pragma unroll
                        for (int e = 0; e < EPV; ++e) amax[i] = fmaxf(amax[i], e < tn ? fabsf(y[e]) : 0.f);
                    }
                }
            }
        };
        if constexpr (FP8) {
            float am[R];
#pragma unroll
            for (int i = 0; i < R; ++i) am[i] = 0.f;
            pass(false, am);
            block_reduce<4, R>(am, MergeMaxR<R>(), red, parity);
            if (a.k > 1) {
                exchange<R>(a, blk, 1, c, am, xb);
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    float v = xb[i];
                    for (int m = 1; m < a.k; ++m) v = fmaxf(v, xb[R * m + i]);
                    am[i] = v;
                }
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
                oinv[i] = am[i] > 0.f ? kFp8Max / am[i] : 1.f;
                if (c == 0 && tid == 0 && i < nr) a.so[row0 + i] = am[i] > 0.f ? am[i] / kFp8Max : 1.f;
            }
        }
        float unused[R];
        pass(true, unused);
    }
}

template <int OP, int DT, int VPT, int R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(multirow_waves<OP, DT, VPT, R>())))
void k_multirow(RowArgs a) {
    constexpr int EPV = Io<DT>::EPV;
    if (a.flags & F_PROBE) {
        coresidency_probe(a);
        return;
    }
    if (a.epoch == 0u && a.epoch_ptr)
        a.epoch = __hip_atomic_load(a.epoch_ptr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __shared__ float red[2 * 4 * 3 * R];
    __shared__ float xb[kMaxK * 2 * R];
    int c, grp;
    member_of(a, blockIdx.x, c, grp);
    Slice sl;
    sl.c0 = (int64_t)c * a.chunk;
    const int64_t rem = a.N - sl.c0;
    sl.nval = rem <= 0 ? 0 : (rem < a.chunk ? rem : a.chunk);
    sl.nfv = sl.nval / EPV;
    sl.tail_n = (int)(sl.nval - sl.nfv * EPV);
    sl.owner = (int)(sl.nfv % kBlock);
    constexpr int AL_ALL = F_ALIGN0 | F_ALIGNO | F_ALIGNP;
    const bool al = (a.flags & AL_ALL) == AL_ALL;
    if (al && sl.nval == (int64_t)VPT * kBlock * EPV)
        rows_loop<OP, DT, VPT, R, true, true>(a, c, grp, sl, red, xb);
    else
        rows_loop<OP, DT, VPT, R, false, false>(a, c, grp, sl, red, xb);
}

}  // namespace credit
