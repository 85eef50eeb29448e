// device.h -- gfx950 device building blocks shared by the row kernels:
// I/O codecs, 128-bit row-slice loads and stores, wave64 / workgroup
// reductions, and the split-row partial exchange.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kargs.h"

namespace credit {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kFp8Max = 448.0f;
constexpr float kLog2Fp8Max = 8.807354922057604f;  // log2(448)
constexpr int kBlock = kBlockThreads;  // one wave per SIMD

template <int DT> struct Io;
template <> struct Io<DT_F32> { static constexpr int EPV = 4, BYTES = 4; };
template <> struct Io<DT_BF16> { static constexpr int EPV = 8, BYTES = 2; };
template <> struct Io<DT_FP8> { static constexpr int EPV = 16, BYTES = 1; };

__device__ __forceinline__ float fast_exp2(float v) { return __builtin_amdgcn_exp2f(v); }
// The hardware exp2 flushes results below 2^-126 to zero.  Output passes that
// evaluate their exponential there (BF16 softmax, backward from the logits,
// two-pass) take 2^(v + kExpShift) and fold 2^-kExpShift into their per-row
// factor, so those outputs down to 2^-158 keep their denormal value (v <= 0
// there, so the shifted exponential cannot overflow; the factor's product is
// exact).  The FP32 softmax forward (register slots) and the FP8 one on
// slices of up to 64 values per thread reuse the sum pass's unshifted
// exponentials about each thread's own maximum instead: an output whose
// exponential lies below 2^-126 of that maximum is 0, an absolute error
// under 1.2e-38 (FP32) or far below an e4m3 step (FP8).
constexpr float kExpShift = 32.f;
constexpr float kExpUnshift = 0x1p-32f;

// ------------------------------------------------------------------ codecs
// Decode one 16-byte vector into EPV floats; FP8 codes are multiplied by the
// row scale (OCP e4m3fn through the gfx950 hardware conversion).
template <int DT> __device__ __forceinline__ void decode(const u32x4 v, float *f, float scale);

template <> __device__ __forceinline__ void decode<DT_F32>(const u32x4 v, float *f, float) {
#pragma unroll
    for (int i = 0; i < 4; ++i) f[i] = __uint_as_float(v[i]);
}
template <> __device__ __forceinline__ void decode<DT_BF16>(const u32x4 v, float *f, float) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = __uint_as_float(v[i] << 16);
        f[2 * i + 1] = __uint_as_float(v[i] & 0xffff0000u);
    }
}
template <> __device__ __forceinline__ void decode<DT_FP8>(const u32x4 v, float *f, float scale) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)v[i], false);
        f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)v[i], true);
        f[4 * i + 0] = lo.x * scale;
        f[4 * i + 1] = lo.y * scale;
        f[4 * i + 2] = hi.x * scale;
        f[4 * i + 3] = hi.y * scale;
    }
}

__device__ __forceinline__ unsigned bf16_bits(float x) {
    __bf16 b = (__bf16)x;  // v_cvt_pk_bf16_f32: round to nearest even
    return (unsigned)__builtin_bit_cast(unsigned short, b);
}

// Encode EPV floats into one 16-byte vector.  FP8: code = RNE(f * inv_scale),
// clamped to the finite range first so it saturates at +-448.
template <int DT> __device__ __forceinline__ u32x4 encode(const float *f, float inv_scale);

template <> __device__ __forceinline__ u32x4 encode<DT_F32>(const float *f, float) {
    u32x4 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = __float_as_uint(f[i]);
    return v;
}
template <> __device__ __forceinline__ u32x4 encode<DT_BF16>(const float *f, float) {
    u32x4 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = bf16_bits(f[2 * i]) | (bf16_bits(f[2 * i + 1]) << 16);
    return v;
}
__device__ __forceinline__ float sat448(float x) { return __builtin_amdgcn_fmed3f(x, -kFp8Max, kFp8Max); }
template <> __device__ __forceinline__ u32x4 encode<DT_FP8>(const float *f, float inv_scale) {
    u32x4 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int w = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(f[4 * i] * inv_scale),
                                                sat448(f[4 * i + 1] * inv_scale), 0, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(f[4 * i + 2] * inv_scale),
                                            sat448(f[4 * i + 3] * inv_scale), w, true);
        v[i] = (unsigned)w;
    }
    return v;
}

// One-byte codes of EPV FP32 values scaled by inv (packed little-endian into
// EPV / 4 words): int8 rounds f * inv half to even and clamps to [-127, 127];
// e4m3 rounds to nearest even with saturation to +-448.  Used for outputs
// computed in FP32 (the LayerNorm -> e4m3 forward), whose accuracy is judged
// against the FP64 result; the row-quantisation operator takes its codes
// from quant_codes_exact below.
template <bool I8, int EPV> __device__ __forceinline__ void quant_codes(const float *f, float inv, unsigned *w) {
#pragma unroll
    for (int i = 0; i < EPV / 4; ++i) {
        if constexpr (I8) {
            unsigned word = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const float v = __builtin_rintf(__builtin_amdgcn_fmed3f(f[4 * i + b] * inv, -127.f, 127.f));
                word |= ((unsigned)(int)v & 0xffu) << (8 * b);
            }
            w[i] = word;
        } else {
            int word = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(f[4 * i] * inv), sat448(f[4 * i + 1] * inv), 0, false);
            word = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(f[4 * i + 2] * inv), sat448(f[4 * i + 3] * inv), word, true);
            w[i] = (unsigned)word;
        }
    }
}

// Row-quantisation codes by their definition: the grid point nearest to
// x * Q / amax, ties to the even code (Q = 127: the integers -127..127; Q = 448:
// the finite e4m3 values).  `inv` is Q / (amax * sc) rounded to FP32 and `sc`
// a power of two that keeps that reciprocal finite (2^64 when amax < 2^-100,
// else 1), so v = (x * sc) * inv is x * Q / amax within 2^-23 |v|.  Rounding v
// therefore gives the exact code except where x * Q / amax lies within a few
// FP32 units of a decision boundary (a half-integer, or the midpoint of two
// adjacent e4m3 values).  Those elements are decided exactly: x * Q and
// b * amax, for a boundary b with at most 9 significant bits, are exact FP64
// products, and so is their comparison.  amax > 0.
__device__ __forceinline__ float fp8_byte_value(unsigned code) {
    return __builtin_amdgcn_cvt_f32_fp8((int)code, 0);
}
// The exact code of one element whose FP32 estimate lies near a boundary:
// byte b (int8 two's complement or e4m3) is the rounding of the estimate,
// at most one grid step from the exact code; aq = |x| Q (exact in FP64).
__device__ __forceinline__ unsigned exact_code_fix(bool i8, float x, unsigned b, float amax) {
    const double aq = (double)__builtin_fabsf(x) * (double)(i8 ? 127.f : kFp8Max);
    if (i8) {
        // magnitude m of the code, the grid points m - 1, m, m + 1 of |x| Q / amax
        const int c = (int)(signed char)(unsigned char)b;
        int m = c < 0 ? -c : c;
        const double up = (double)(2 * m + 1) * (double)amax * 0.5;
        const double dn = (double)(2 * m - 1) * (double)amax * 0.5;
        if (aq > up || (aq == up && (m & 1))) ++m;
        else if (m > 0 && (aq < dn || (aq == dn && (m & 1)))) --m;
        m = m > 127 ? 127 : m;
        const int code = x < 0.f ? -m : m;
        return (unsigned)code & 0xffu;
    }
    unsigned mc = b & 0x7fu;
    const float g = fp8_byte_value(mc);
    if (mc < 0x7eu) {
        const double up = (double)((g + fp8_byte_value(mc + 1u)) * 0.5f) * (double)amax;
        if (aq > up || (aq == up && (mc & 1u))) return (b & 0x80u) | (mc + 1u);
    }
    if (mc > 0u) {
        const double dn = (double)((g + fp8_byte_value(mc - 1u)) * 0.5f) * (double)amax;
        if (aq < dn || (aq == dn && (mc & 1u))) return (b & 0x80u) | (mc - 1u);
    }
    return b;
}
template <bool I8, int EPV>
__device__ __forceinline__ void quant_codes_exact(const float *f, float sc, float inv, float amax, unsigned *w) {
    float v[EPV];
#pragma unroll
    for (int i = 0; i < EPV; ++i) v[i] = (f[i] * sc) * inv;
    unsigned nm = 0;  // elements whose estimate lies near a decision boundary
    if constexpr (I8) {
#pragma unroll
        for (int i = 0; i < EPV / 4; ++i) w[i] = 0u;
#pragma unroll
        for (int i = 0; i < EPV; ++i) {
            const float c = __builtin_rintf(__builtin_amdgcn_fmed3f(v[i], -127.f, 127.f));
            // |v - x Q / amax| <= 127 * 2^-23 < 2^-16
            nm |= (__builtin_fabsf(v[i] - c) > 0.5f - 0x1p-14f ? 1u : 0u) << i;
            w[i / 4] |= ((unsigned)(int)c & 0xffu) << (8 * (i % 4));
        }
    } else {
#pragma unroll
        for (int i = 0; i < EPV / 4; ++i) {
            int word = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(v[4 * i]), sat448(v[4 * i + 1]), 0, false);
            word = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(v[4 * i + 2]), sat448(v[4 * i + 3]), word, true);
            w[i] = (unsigned)word;
        }
#pragma unroll
        for (int i = 0; i < EPV; ++i) {
            const float a = __builtin_fabsf(v[i]);
            // normal e4m3 range: a midpoint has FP32 fraction bits 19..0 equal
            // to 0x80000 and v is within 2 FP32 units of x Q / amax; subnormal
            // range: midpoints at (j + 1/2) 2^-9
            const unsigned low = __float_as_uint(a) & 0xfffffu;
            const float t = a * 512.f;
            const bool near = a >= 0x1p-6f ? low - 0x7fffcu <= 8u
                                           : __builtin_fabsf(t - __builtin_floorf(t) - 0.5f) < 0x1p-12f;
            nm |= (near ? 1u : 0u) << i;
        }
    }
    while (nm) {  // rare: one element at a time
        const int i = __builtin_ctz(nm);
        nm &= nm - 1u;
        // element i and its code word by selects over values the compiler
        // cannot regroup into an array (a lane-varying index into a register
        // array would place the array in private memory)
        float x = 0.f;
        unsigned word = 0u;
#pragma unroll
        for (int k = 0; k < EPV; ++k) {
            float fk = f[k];
            asm volatile("" : "+v"(fk));
            x = i == k ? fk : x;
        }
#pragma unroll
        for (int k = 0; k < EPV / 4; ++k) {
            unsigned wk = w[k];
            asm volatile("" : "+v"(wk));
            word = (i >> 2) == k ? wk : word;
        }
        const int sh = 8 * (i & 3);
        const unsigned nb = exact_code_fix(I8, x, (word >> sh) & 0xffu, amax);
        const unsigned nw = (word & ~(0xffu << sh)) | (nb << sh);
#pragma unroll
        for (int k = 0; k < EPV / 4; ++k) w[k] = (i >> 2) == k ? nw : w[k];
    }
}
// Per-row factors of quant_codes_exact: the power-of-two pre-scale and the
// FP32 reciprocal Q / (amax * sc).  amax > 0.
__device__ __forceinline__ void quant_row_factors(float amax, float Q, float &sc, float &inv) {
    sc = amax < 0x1p-100f ? 0x1p64f : 1.f;
    inv = Q / (amax * sc);
}

// ------------------------------------------------------------ loads/stores
// Vector at element e of a row starting at byte pointer `row`; nv in [0, EPV]
// elements are valid.  Full vectors of aligned rows use one 128-bit access;
// partial vectors and misaligned rows go element by element.  Invalid
// elements read as code 0 (value 0).
template <int DT, bool NT>
__device__ __forceinline__ u32x4 load_vec(const char *row, int64_t e, int nv, bool aligned) {
    constexpr int EPV = Io<DT>::EPV, B = Io<DT>::BYTES;
    const char *p = row + e * B;
    if (nv == EPV && aligned) {
        if constexpr (NT)
            return __builtin_nontemporal_load((const u32x4 *)p);
        else
            return *(const u32x4 *)p;
    }
    u32x4 v = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < EPV; ++i) {
        if (i < nv) {
            unsigned bits;
            if constexpr (B == 4)
                bits = *(const unsigned *)(p + 4 * i);
            else if constexpr (B == 2)
                bits = *(const unsigned short *)(p + 2 * i);
            else
                bits = *(const unsigned char *)(p + i);
            constexpr int PER = 4 / B;  // elements per 32-bit word
            v[i / PER] |= bits << (8 * B * (i % PER));
        }
    }
    return v;
}

// The first element of a row, decoded with scale 1: the common shift of a
// row's moment sums (every workgroup of a row group reads the same element).
template <int DT> __device__ __forceinline__ float row_first(const char *row) {
    float f[Io<DT>::EPV];
    decode<DT>(load_vec<DT, false>(row, 0, 1, false), f, 1.f);
    return f[0];
}

template <int DT>
__device__ __forceinline__ void store_vec(char *row, int64_t e, int nv, bool aligned, u32x4 v) {
    constexpr int EPV = Io<DT>::EPV, B = Io<DT>::BYTES;
    char *p = row + e * B;
    if (nv == EPV && aligned) {
        __builtin_nontemporal_store(v, (u32x4 *)p);
        return;
    }
#pragma unroll
    for (int i = 0; i < EPV; ++i) {
        if (i < nv) {
            constexpr int PER = 4 / B;
            unsigned bits = v[i / PER] >> (8 * B * (i % PER));
            if constexpr (B == 4)
                *(unsigned *)(p + 4 * i) = bits;
            else if constexpr (B == 2)
                *(unsigned short *)(p + 2 * i) = (unsigned short)bits;
            else
                *(unsigned char *)(p + i) = (unsigned char)bits;
        }
    }
}

// Hides the contents of retained data registers from the optimiser between
// passes over them, so each pass decodes the packed data again instead of the
// compiler keeping every decoded FP32 value of the first pass alive.  Emits no
// instruction.
template <int V> __device__ __forceinline__ void opaque(u32x4 (&d)[V]) {
#pragma unroll
    for (int j = 0; j < V; ++j) asm volatile("" : "+v"(d[j]));
}

// Orders a pass over the retained slots: the accumulators are made opaque
// after each slot, so the scheduler cannot decode later slots ahead of earlier
// ones and keep all of their decoded values live at once (which spilled the
// two-input kernels).  Emits no instruction.
__device__ __forceinline__ void keep1(float &v) { asm volatile("" : "+v"(v)); }
template <class... T> __device__ __forceinline__ void keep_order(T &...v) {
    int unused[] = {(keep1(v), 0)...};
    (void)unused;
}

// -------------------------------------------------------- wave64 reduction
// Partner value across lanes (lane ^ m) inside each 32-lane half: DPP quad
// permutes for m = 1, 2 and ds_swizzle bit-mode xor for m = 4, 8, 16.
template <int MASK> __device__ __forceinline__ float xor_lane(float v) {
    int i = __float_as_int(v);
    if constexpr (MASK == 1)
        return __int_as_float(__builtin_amdgcn_mov_dpp(i, 0xB1, 0xF, 0xF, false));  // [1,0,3,2]
    else if constexpr (MASK == 2)
        return __int_as_float(__builtin_amdgcn_mov_dpp(i, 0x4E, 0xF, 0xF, false));  // [2,3,0,1]
    else
        return __int_as_float(__builtin_amdgcn_ds_swizzle(i, 0x1F | (MASK << 10)));
}

// Butterfly over the 32 lanes of each half, then lanes 0 and 32 merged in
// that order; every lane returns the same (wave-uniform) tuple.
template <int NV, class Merge>
__device__ __forceinline__ void wave_reduce(float (&v)[NV], Merge merge) {
    float o[NV];
#define CREDIT_XSTEP(M)                                  \
    _Pragma("unroll") for (int i = 0; i < NV; ++i) o[i] = xor_lane<M>(v[i]); \
    merge(v, o);
    CREDIT_XSTEP(1)
    CREDIT_XSTEP(2)
    CREDIT_XSTEP(4)
    CREDIT_XSTEP(8)
    CREDIT_XSTEP(16)
#undef CREDIT_XSTEP
    float hi[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        hi[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[i]), 32));
        v[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[i]), 0));
    }
    merge(v, hi);
}

// Workgroup reduction over NW waves.  `red` is LDS scratch of [2][NW][NV]
// floats used alternately (parity flips each call), so one barrier per call
// suffices.  Waves are merged in order 0..NW-1: the result is uniform.
template <int NW, int NV, class Merge>
__device__ __forceinline__ void block_reduce(float (&v)[NV], Merge merge, float *red, int &parity) {
    wave_reduce<NV>(v, merge);
    const int wave = threadIdx.x >> 6;
    float *buf = red + parity * (NW * NV);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) buf[wave * NV + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = buf[i];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
        float t[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) t[i] = buf[w * NV + i];
        merge(v, t);
    }
    parity ^= 1;
}

// ------------------------------------------------------------- merges
struct MergeSum {
    template <int NV> __device__ __forceinline__ void operator()(float (&a)[NV], const float (&b)[NV]) const {
#pragma unroll
        for (int i = 0; i < NV; ++i) a[i] += b[i];
    }
};
struct MergeMax {
    __device__ __forceinline__ void operator()(float (&a)[1], const float (&b)[1]) const { a[0] = fmaxf(a[0], b[0]); }
};
// Online softmax statistics in the base-2 domain: (c, s) with c = max of
// x*log2(e) and s = sum of 2^(x*log2(e) - c).  Empty partials have c = -inf.
struct MergeSoftmax {
    __device__ __forceinline__ void operator()(float (&a)[2], const float (&b)[2]) const {
        float c = fmaxf(a[0], b[0]);
        float sa = a[0] == -INFINITY ? 0.f : a[1] * fast_exp2(a[0] - c);
        float sb = b[0] == -INFINITY ? 0.f : b[1] * fast_exp2(b[0] - c);
        a[0] = c;
        a[1] = sa + sb;
    }
};
// Chan et al. pairwise combination of (count, mean, M2).  The weight
// nb / (n + nb) goes through the hardware reciprocal (1 ulp) rather than a
// correctly rounded division: its scale / fixup sequence ran on every merge
// of every row (the wave and workgroup levels plus the k members of a split
// row), and a 1-ulp weight moves the mean by 1 ulp of the means' difference.
__device__ __forceinline__ void chan_merge(float &n, float &mean, float &m2, float nb, float meanb, float m2b) {
    float nn = n + nb;
    if (nb == 0.f) return;
    if (n == 0.f) { n = nb; mean = meanb; m2 = m2b; return; }
    float d = meanb - mean;
    float wb = nb * __builtin_amdgcn_rcpf(nn);
    mean = mean + d * wb;
    m2 = m2 + m2b + d * d * n * wb;
    n = nn;
}
struct MergeChan {
    __device__ __forceinline__ void operator()(float (&a)[3], const float (&b)[3]) const {
        chan_merge(a[0], a[1], a[2], b[0], b[1], b[2]);
    }
};

// Online softmax statistics with a weighted sum riding along: (c, s, t) with
// s = sum 2^(q - c) and t = sum g * 2^(q - c); both sums rescale together.
struct MergeSoftmax3 {
    __device__ __forceinline__ void operator()(float (&a)[3], const float (&b)[3]) const {
        float c = fmaxf(a[0], b[0]);
        float fa = a[0] == -INFINITY ? 0.f : fast_exp2(a[0] - c);
        float fb = b[0] == -INFINITY ? 0.f : fast_exp2(b[0] - c);
        a[0] = c;
        a[1] = a[1] * fa + b[1] * fb;
        a[2] = a[2] * fa + b[2] * fb;
    }
};
// Pairwise combination of bivariate co-moments (count, mean_x, mean_y, Cxx,
// Cyy, Cxy): Chan's update applied to the cross term as well.
__device__ __forceinline__ void co_merge(float (&a)[6], float nb, float mxb, float myb, float cxxb, float cyyb,
                                         float cxyb) {
    if (nb == 0.f) return;
    if (a[0] == 0.f) {
        a[0] = nb; a[1] = mxb; a[2] = myb; a[3] = cxxb; a[4] = cyyb; a[5] = cxyb;
        return;
    }
    const float n = a[0] + nb, dx = mxb - a[1], dy = myb - a[2];
    const float wb = nb * __builtin_amdgcn_rcpf(n), f = a[0] * wb;  // as in chan_merge
    a[1] = a[1] + dx * wb;
    a[2] = a[2] + dy * wb;
    a[3] = a[3] + cxxb + dx * dx * f;
    a[4] = a[4] + cyyb + dy * dy * f;
    a[5] = a[5] + cxyb + dx * dy * f;
    a[0] = n;
}
struct MergeCo {
    __device__ __forceinline__ void operator()(float (&a)[6], const float (&b)[6]) const {
        co_merge(a, b[0], b[1], b[2], b[3], b[4], b[5]);
    }
};

// ------------------------------------------------- workgroup -> (member, group)
// Hardware workgroup ids are dealt round-robin to the 8 XCDs (id % 8), each
// with its own L2.  With F_XCD, an XCD hosts only some member indices c, i.e.
// the same column slices for every row group it runs, so the gamma / beta
// columns it reads (N bytes per XCD) stay in its L2 across rows.  Row groups
// are spread over XCDs instead; the exchange does not care, because its
// agent-scope slot accesses are served at the memory side either way.
__device__ __forceinline__ void member_of(const RowArgs &a, int bid, int &c, int &grp) {
    if (a.flags & F_XCD) {
        const int x = bid & 7, idx = bid >> 3;
        if (a.k >= 8) {
            const int per = a.k >> 3;
            c = x + 8 * (idx % per);
            grp = idx / per;
        } else {
            const int per = 8 / a.k;
            c = x % a.k;
            grp = idx * per + x / a.k;
        }
    } else {
        c = bid % a.k;
        grp = bid / a.k;
    }
}

// ---------------------------------------------------- co-residency probe
// Launched in place of the row work (F_PROBE) at a split-row grid: every
// workgroup announces itself on a counter, then waits (bounded) until the
// counter holds the whole grid; a workgroup that gives up counts a miss.  No
// miss means every workgroup of the grid was resident at the same time, with
// the kernel's own register, LDS and private-memory demand.  Counter words:
// errflag[96] (arrivals) and errflag[97] (misses), zeroed by the host.
__device__ __forceinline__ void coresidency_probe(const RowArgs &a) {
    if (threadIdx.x == 0) {
        unsigned *arrived = a.errflag + 96, *missed = a.errflag + 97;
        __hip_atomic_fetch_add(arrived, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while (__hip_atomic_load(arrived, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x) {
            if (++spins > a.spin_limit) {
                __hip_atomic_fetch_add(missed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
}

// --------------------------------------------------- split-row exchange
// Slot word: high 32 bits = launch epoch, low 32 bits = FP32 partial.  Each
// word is written with one agent-scope atomic store and polled with
// agent-scope atomic loads, so a reader that sees the current epoch also sees
// the value that came with it; no fence and no counter reset are needed.
__device__ __forceinline__ unsigned long long *slot_ptr(const RowArgs &a, int64_t row, int stage, int c, int j) {
    return a.slots + (((row * kMaxStages + stage) * (int64_t)a.k + c) * a.qs + j);
}

// Publishes this workgroup's q partials for (row, stage) and gathers all k*q
// partials of the row group into LDS `xb` (member-major).  Returns after a
// barrier, with xb valid for every thread.  A bounded wait: after
// a.spin_limit polls (or once another workgroup of this launch has reported a
// timeout) the wait gives up, raises the error flag and proceeds.
template <int Q>
__device__ __forceinline__ void exchange(const RowArgs &a, int64_t row, int stage, int c,
                                         const float (&mine)[Q], float *xb) {
    const int tid = threadIdx.x;
    const int kq = a.k * Q;
    if (a.flags & F_TEST_SKEW) {
        // test only: member c of row `row` publishes about (c * 7 + row) % 13
        // microseconds late, so members reach the exchange out of step
        // (the real-time counter runs at 100 MHz)
        const uint64_t ticks = (uint64_t)((c * 7 + row) % 13) * 100u;
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while (__builtin_amdgcn_s_memrealtime() - t0 < ticks) __builtin_amdgcn_s_sleep(8);
        __syncthreads();
    }
    if (tid < Q) {
        bool drop = (a.flags & F_TEST_DROP_PUBLISH) && c == 1;
        if (!drop) {
            unsigned long long w = ((unsigned long long)a.epoch << 32) | __float_as_uint(mine[tid]);
            __hip_atomic_store(slot_ptr(a, row, stage, c, tid), w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (tid < 64) {
        // wave 0 polls the k * Q slots, P per lane (P = 1 unless k * Q > 64)
        constexpr int P = (kMaxK * Q + 63) / 64;
        const int lane = tid;
        bool ok[P];
        unsigned long long w[P];
        unsigned long long *p[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int s = lane + 64 * i;
            ok[i] = s >= kq;
            w[i] = 0;
            p[i] = ok[i] ? nullptr : slot_ptr(a, row, stage, s / Q, s % Q);
        }
        unsigned spins = 0;
        while (true) {
            bool all = true;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                if (!ok[i]) {
                    w[i] = __hip_atomic_load(p[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok[i] = (unsigned)(w[i] >> 32) == a.epoch;
                }
                all = all && ok[i];
            }
            if (__all(all)) break;
            // The flag holds the epoch of the launch that timed out, so a stale
            // flag from an earlier launch never cuts this launch's waits short.
            // It is one word for the whole launch: read every 32 polls only, so
            // hundreds of waiting workgroups do not keep one line hot (2% of
            // the FP32 LayerNorm forward at N = 524288).
            if (++spins > a.spin_limit ||
                ((spins & 31u) == 0u &&
                 __hip_atomic_load(a.errflag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == a.epoch)) {
                if (lane == 0)
                    __hip_atomic_store(a.errflag, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int s = lane + 64 * i;
            if (s < kq) xb[s] = ok[i] ? __uint_as_float((unsigned)w[i]) : 0.f;
        }
    }
    __syncthreads();
}

}  // namespace credit
