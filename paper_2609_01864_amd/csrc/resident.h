// resident.h -- the row-resident (k == 1) and split-row (k > 1) kernels.
//
// A workgroup of 256 threads (one wave per SIMD) owns a slice of `chunk`
// elements of a row (Eq. (2): the slices I_c of the k members of a row group
// partition the row).  It loads the slice once with 128-bit loads and keeps it
// in registers in the packed I/O format (the staged copy of Fig. 2b, held in
// VGPRs instead of shared memory), reduces it thread -> wave -> workgroup, and,
// when k > 1, exchanges the q partials of every stage with the other members
// (replicated gather: every member reads all k slots and combines them in the
// fixed order c = 0..k-1, so all members reconstruct bit-identical statistics,
// Eq. (5)).  It then applies h to its own retained slice and writes it.  The
// workgroup is persistent: row group `grp` processes rows grp, grp + groups, ...
//
// Slot j of thread t holds vector j * 256 + t of the slice (rotated by the row
// group for the operators that read gamma / beta, see sv below).  Two row loops
// exist, chosen once per workgroup (the choice is uniform, and both contain
// workgroup barriers):
//   AL && FULLS   every slot of every thread is a full, 16-byte aligned vector:
//                 straight-line 128-bit loads and stores, no masks;
//   !AL, !FULLS   any alignment and length: 128-bit accesses through
//                 under-aligned pointer types; slots past the last full vector
//                 re-read the slice's first vector and are zeroed / masked; the
//                 trailing partial vector (< 16 bytes) is handled element-wise
//                 by the thread that owns it.
#pragma once
#include "device.h"

namespace credit {

template <int OP> struct OpTraits {
    static constexpr bool TWO = two_in(OP);    // two resident input tensors
    static constexpr bool TWOO = two_out(OP);  // two output tensors
    static constexpr bool QUANT = is_quant(OP);  // row quantisation
    static constexpr bool BOUT = byte_out(OP);   // one-byte codes out
    static constexpr int NCP = OP == OP_LN_BWD ? 2 : (OP == OP_RMS_BWD ? 1 : 0);  // column partials
};

// FP32 registers per thread that hold the normalised row y of a norm forward
// with FP8 output between its amax stage and its quantize pass (0: y is
// recomputed from x, gamma and beta instead).
template <int OP, int DT, int VPT> constexpr int yc_regs() {
    constexpr bool f8o = (DT == DT_FP8 && (OP == OP_LN_FWD || OP == OP_RMS_FWD)) || OP == OP_LNQ_FWD;
    return f8o && VPT * Io<DT>::EPV <= kYcMax ? VPT * Io<DT>::EPV : 0;
}

// FP32 registers per thread that hold an FP8 softmax row's decoded values,
// then their exponentials, across the three passes of the forward (0: the
// packed row is decoded and exponentiated again in the output pass).  Up to
// kEcMax values: beyond that the registers cost more occupancy than the
// saved decode and exponential gain.
template <int OP, int DT, int VPT> constexpr int ec_regs() {
    return OP == OP_SOFTMAX_FWD && DT == DT_FP8 && VPT * Io<DT>::EPV <= kEcMax ? VPT * Io<DT>::EPV : 0;
}

// FP32 registers per thread that hold g = dy * gamma of a BF16 LayerNorm /
// RMSNorm backward between its statistics and output passes (slices of up to
// two vectors; 0 otherwise: FP32 keeps g in place of dy, wider BF16 slices
// reload gamma).
template <int OP, int DT, int VPT> constexpr int gk_regs() {
    return (OP == OP_LN_BWD || OP == OP_RMS_BWD) && DT == DT_BF16 && VPT <= 2 ? VPT * Io<DT>::EPV : 0;
}

// Waves per SIMD the register allocation must allow (each workgroup is one
// wave per SIMD, so this is also the workgroups per CU): the retained data,
// the FP32 column partials, a kept y and the working registers within
// 512 / W VGPRs.
template <int OP, int DT, int VPT> constexpr int resident_waves() {
    constexpr int data = VPT * 4 * (OpTraits<OP>::TWO ? 2 : 1) + OpTraits<OP>::NCP * VPT * Io<DT>::EPV +
                         yc_regs<OP, DT, VPT>() + ec_regs<OP, DT, VPT>() + gk_regs<OP, DT, VPT>();
    constexpr int work = 64 + (DT == DT_FP8 || OP == OP_LNQ_FWD ? 32 : 0) +
                         (OP == OP_SOFTMAX_FWD || OP == OP_SOFTMAX_BWD ? 0 : 16);
    static_assert(OP < OP_COUNT, "operator");
    constexpr int w = 512 / (data + work);
    constexpr int ov = wave_override(OP, DT, VPT);
    return ov ? ov : (w < 1 ? 1 : (w > 8 ? 8 : w));
}

// Slots are addressed as (uniform base pointer, 32-bit per-thread byte
// offset), so the compiler emits SGPR-base + VGPR-offset instructions and keeps
// no 64-bit address per slot alive across passes.  AL: 16-byte aligned
// pointer types; otherwise the same 128-bit accesses through 1-byte aligned
// types (gfx950 runs in unaligned-access mode), so rows of any alignment keep
// vector loads and stores.
typedef u32x4 u32x4_u __attribute__((aligned(1)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef f32x4 f32x4_u __attribute__((aligned(1)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef u32x2 u32x2_u __attribute__((aligned(1)));
typedef unsigned u32_u __attribute__((aligned(1)));

#ifndef CREDIT_LOAD_NT
#define CREDIT_LOAD_NT 1
#endif
#ifndef CREDIT_STORE_NT
#define CREDIT_STORE_NT 1
#endif
template <bool AL> __device__ __forceinline__ u32x4 vload_nt(const char *base, uint32_t off) {
    if constexpr (!CREDIT_LOAD_NT)
        return AL ? *(const u32x4 *)(base + off) : *(const u32x4_u *)(base + off);
    if constexpr (AL)
        return __builtin_nontemporal_load((const u32x4 *)(base + off));
    else
        return __builtin_nontemporal_load((const u32x4_u *)(base + off));
}
template <bool AL> __device__ __forceinline__ void vstore_nt(char *base, uint32_t off, u32x4 v) {
    if constexpr (!CREDIT_STORE_NT) {
        if constexpr (AL) *(u32x4 *)(base + off) = v;
        else *(u32x4_u *)(base + off) = v;
        return;
    }
    if constexpr (AL)
        __builtin_nontemporal_store(v, (u32x4 *)(base + off));
    else
        __builtin_nontemporal_store(v, (u32x4_u *)(base + off));
}

// NB (4, 8 or 16) bytes of quantisation codes at base + off.
template <int NB, bool AL> __device__ __forceinline__ void bstore_nt(char *base, uint32_t off, const unsigned *w) {
    char *p = base + off;
    if constexpr (NB == 4) {
        if constexpr (AL) __builtin_nontemporal_store(w[0], (unsigned *)p);
        else __builtin_nontemporal_store(w[0], (u32_u *)p);
    } else if constexpr (NB == 8) {
        u32x2 v = {w[0], w[1]};
        if constexpr (AL) __builtin_nontemporal_store(v, (u32x2 *)p);
        else __builtin_nontemporal_store(v, (u32x2_u *)p);
    } else {
        u32x4 v = {w[0], w[1], w[2], w[3]};
        vstore_nt<AL>(base, off, v);
    }
}

// EPV FP32 parameters (gamma / beta) of one vector slot.
template <int DT, bool AL>
__device__ __forceinline__ void load_params_v(const float *base, uint32_t off, float *out) {
    constexpr int EPV = Io<DT>::EPV;
    const char *p = (const char *)base + off;
#pragma unroll
    for (int i = 0; i < EPV; i += 4) {
        f32x4 v = AL ? *(const f32x4 *)(p + 4 * i) : *(const f32x4_u *)(p + 4 * i);
        out[i] = v.x; out[i + 1] = v.y; out[i + 2] = v.z; out[i + 3] = v.w;
    }
}

// Parameters of the trailing partial vector (n valid elements, n < EPV).
template <int DT>
__device__ __forceinline__ void load_params_tail(const float *p, int64_t col, int n, float *out) {
#pragma unroll
    for (int i = 0; i < Io<DT>::EPV; ++i) out[i] = i < n ? p[col + i] : 0.f;
}

// Combines the k exchanged partials of a stage in member order.
template <int Q, class Merge>
__device__ __forceinline__ void combine_members(float (&v)[Q], const float *xb, int k, Merge merge) {
#pragma unroll
    for (int j = 0; j < Q; ++j) v[j] = xb[j];
    for (int c = 1; c < k; ++c) {
        float t[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j) t[j] = xb[c * Q + j];
        merge(v, t);
    }
}

// Reduces a per-thread tuple over the workgroup and, for k > 1, over the row
// group.  Sum- and max-type statistics.
template <int Q, class Merge>
__device__ __forceinline__ void row_reduce(float (&v)[Q], Merge merge, const RowArgs &a, int64_t row,
                                           int stage, int c, float *red, float *xb, int &parity) {
    block_reduce<4, Q>(v, merge, red, parity);
    if (a.k > 1) {
        exchange<Q>(a, row, stage, c, v, xb);
        combine_members<Q>(v, xb, a.k, merge);
    }
}

// Chan statistics (n, mean, M2) over the workgroup and the row group.  The
// exchange carries (mean, M2); each member's count follows from its slice.
__device__ __forceinline__ void row_reduce_chan(float (&v)[3], const RowArgs &a, int64_t row, int stage,
                                                int c, float *red, float *xb, int &parity) {
    block_reduce<4, 3>(v, MergeChan(), red, parity);
    if (a.k > 1) {
        float mine[2] = {v[1], v[2]};
        exchange<2>(a, row, stage, c, mine, xb);
        float n = 0.f, mean = 0.f, m2 = 0.f;
        for (int m = 0; m < a.k; ++m) {
            int64_t lo = (int64_t)m * a.chunk;
            int64_t cnt = a.N - lo < a.chunk ? a.N - lo : a.chunk;
            float nm = cnt > 0 ? (float)cnt : 0.f;
            chan_merge(n, mean, m2, nm, xb[2 * m], xb[2 * m + 1]);
        }
        v[0] = n; v[1] = mean; v[2] = m2;
    }
}

// Bivariate co-moments (n, mean_x, mean_y, Cxx, Cyy, Cxy) over the workgroup
// and the row group; the exchange carries the five moments, each member's
// count follows from its slice.
__device__ __forceinline__ void row_reduce_co(float (&v)[6], const RowArgs &a, int64_t row, int stage, int c,
                                              float *red, float *xb, int &parity) {
    block_reduce<4, 6>(v, MergeCo(), red, parity);
    if (a.k > 1) {
        float mine[5] = {v[1], v[2], v[3], v[4], v[5]};
        exchange<5>(a, row, stage, c, mine, xb);
        float t[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int m = 0; m < a.k; ++m) {
            int64_t lo = (int64_t)m * a.chunk;
            int64_t cnt = a.N - lo < a.chunk ? a.N - lo : a.chunk;
            const float *p = xb + 5 * m;
            co_merge(t, cnt > 0 ? (float)cnt : 0.f, p[0], p[1], p[2], p[3], p[4]);
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] = t[i];
    }
}

// Geometry of a workgroup's slice.
struct Slice {
    int64_t c0;    // first column
    int64_t nval;  // valid elements
    int64_t nfv;   // full vectors
    int tail_n;    // elements of the trailing partial vector (0: none)
    int owner;     // thread that holds it
};

// Slots of the slice held in LDS beyond the VPT register slots (the overflow
// of Eq. (3)'s capacity into LDS): L vectors per thread, stored [L][256] so
// that each wave writes and reads only its own 64-vector rows.
template <int L> struct LdsSlice { u32x4 v[L][kBlock]; };
template <> struct LdsSlice<0> { u32x4 v[1][1]; };

template <int OP, int DT, int VPT, bool AL, bool FULLS, int L>
__device__ __forceinline__ void row_loop(const RowArgs &a, int c, int grp, const Slice &sl, float *red, float *xb,
                                         u32x4 *lds) {
    static_assert(L == 0 || OP == OP_SOFTMAX_FWD || OP == OP_LN_FWD || OP == OP_RMS_FWD,
                  "LDS slots exist for the single-input forward operators");
    using T = OpTraits<OP>;
    constexpr int EPV = Io<DT>::EPV, B = Io<DT>::BYTES, NCP = T::NCP;
    constexpr int OB = T::BOUT ? 1 : B;  // output element bytes
    constexpr bool FP8 = DT == DT_FP8;
    // slots per batch of parameter loads: 16 FP32 parameter registers in flight
    constexpr int GBW = 16 / EPV / (OP == OP_LN_FWD || OP == OP_LNQ_FWD ? 2 : 1);
    constexpr int GB = GBW < 1 ? 1 : (VPT < GBW ? VPT : GBW);
    int parity = 0;
    const int tid = threadIdx.x;
    const float invN = 1.f / (float)a.N;
    // Slot j holds vector sv(j) * 256 + tid of the slice.  Operators that
    // read gamma / beta rotate the slot order by the row group (fixed for the
    // workgroup, so column partials stay per slot across rows): the
    // workgroups sharing an XCD then stream the same parameter columns at
    // different moments instead of in lockstep (1.5-2% on FP32 LayerNorm
    // forward; FP8 rows, whose slices are short, measured 1% slower).
    constexpr bool ROT = DT != DT_FP8 && (OP == OP_LN_FWD || OP == OP_RMS_FWD || OP == OP_LNQ_FWD ||
                                          OP == OP_LN_BWD || OP == OP_RMS_BWD);
    const int rot = ROT ? grp % VPT : 0;
    auto sv = [&](int j) -> int {
        if (j >= VPT) return j;  // LDS slots keep their order
        const int r = j + rot;
        return r >= VPT ? r - VPT : r;
    };
    auto ok_of = [&](int j) -> bool { return FULLS || (int64_t)(sv(j) * kBlock + tid) < sl.nfv; };
    auto col_of = [&](int j) -> int64_t { return sl.c0 + (int64_t)(sv(j) * kBlock + tid) * EPV; };
    const bool tail = !FULLS && sl.tail_n > 0 && tid == sl.owner;
    const int tn = sl.tail_n;
    const int64_t tcol = sl.c0 + sl.nfv * EPV;
    // elements this thread holds (for the Chan counts)
    float held = 0.f;
    if (FULLS) {
        held = (float)((VPT + L) * EPV);
    } else {
        for (int j = 0; j < VPT + L; ++j) held += ok_of(j) ? (float)EPV : 0.f;
        if (tail) held += (float)tn;
    }

    float cp[NCP ? NCP : 1][NCP ? VPT * EPV : 1];
    float cpt[NCP ? NCP : 1][NCP ? EPV : 1];
    if constexpr (NCP) {
#pragma unroll
        for (int p = 0; p < NCP; ++p) {
#pragma unroll
            for (int i = 0; i < VPT * EPV; ++i) cp[p][i] = 0.f;
#pragma unroll
            for (int i = 0; i < EPV; ++i) cpt[p][i] = 0.f;
        }
    }

    for (int64_t row = grp; row < a.M; row += a.groups) {
        const char *r0 = (const char *)a.in0 + row * a.ld0 * B;
        const char *r1 = T::TWO ? (const char *)a.in1 + row * a.ld1 * B : nullptr;
        char *orow = (char *)a.out + row * a.ldo * OB;
        char *orow1 = T::TWOO ? (char *)a.out1 + row * a.ldo1 * B : nullptr;
        const bool writer = c == 0 && tid == 0;
        // Uniform bases of this row's slice and per-thread byte offsets that are
        // made opaque each row, so slot addresses are formed next to their use
        // instead of being hoisted out of the row loop as 64-bit registers.
        const char *b0 = r0 + sl.c0 * B;
        const char *b1 = T::TWO ? r1 + sl.c0 * B : nullptr;
        char *bo = orow + sl.c0 * OB;
        char *bo1 = T::TWOO ? orow1 + sl.c0 * B : nullptr;
        uint32_t toff = (uint32_t)tid * 16u, poff = (uint32_t)tid * (EPV * 4u);
        asm volatile("" : "+v"(toff));
        asm volatile("" : "+v"(poff));
        uint32_t qoff = (uint32_t)tid * (uint32_t)EPV;  // codes: EPV bytes per slot
        if constexpr (T::BOUT) asm volatile("" : "+v"(qoff));
        // masked slots re-read the slice's first vector (only when nfv >= 1);
        // their data is zeroed before use and their stores are skipped
        auto doff = [&](int j) -> uint32_t {
            return (FULLS || ok_of(j)) ? toff + (uint32_t)sv(j) * (kBlock * 16u) : 0u;
        };
        auto pofs = [&](int j) -> uint32_t {
            return (FULLS || ok_of(j)) ? poff + (uint32_t)sv(j) * (kBlock * EPV * 4u) : 0u;
        };
        auto ST = [&](int j, u32x4 v) {
            if (FULLS || ok_of(j)) vstore_nt<AL>(bo, toff + (uint32_t)sv(j) * (kBlock * 16u), v);
        };
        auto ST1 = [&](int j, u32x4 v) {
            if (FULLS || ok_of(j)) vstore_nt<AL>(bo1, toff + (uint32_t)sv(j) * (kBlock * 16u), v);
        };
        auto QST = [&](int j, const unsigned *w) {
            if (FULLS || ok_of(j)) bstore_nt<EPV, AL>(bo, qoff + (uint32_t)sv(j) * (uint32_t)(kBlock * EPV), w);
        };
        // a slice without full vectors (only a trailing partial one, or none)
        // has every slot masked and reads no parameter vector: sl.c0 may lie
        // at or past N there
        auto PAR = [&](const float *p, int j, float *out) {
            if (FULLS || sl.nfv > 0) {
                load_params_v<DT, AL>(p + sl.c0, pofs(j), out);
            } else {
#pragma unroll
                for (int i = 0; i < EPV; ++i) out[i] = 0.f;
            }
        };
        u32x4 d0[VPT];
        u32x4 d1[T::TWO ? VPT : 1];
        if (FULLS || sl.nfv > 0) {  // uniform: a slice without full vectors issues no vector load
#pragma unroll
            for (int j = 0; j < VPT; ++j) d0[j] = vload_nt<AL>(b0, doff(j));
            if constexpr (T::TWO) {
#pragma unroll
                for (int j = 0; j < VPT; ++j) d1[j] = vload_nt<AL>(b1, doff(j));
            }
        } else {
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                d0[j] = u32x4{0u, 0u, 0u, 0u};
                if constexpr (T::TWO) d1[j] = u32x4{0u, 0u, 0u, 0u};
            }
        }
        if constexpr (L > 0) {
            // the LDS slots: direct global -> LDS loads (16 bytes per lane, the
            // wave's 64 lanes land in its own row of the slot), in flight with
            // the register loads; the same masked-slot addressing.  Like the
            // register slots they carry the non-temporal hint (cache policy 2):
            // x is read once, and a cached stream would evict the parameter
            // vectors that every row rereads from L2
            if (FULLS || sl.nfv > 0) {
                const int wave = tid >> 6;
#pragma unroll
                for (int l = 0; l < L; ++l)
                    __builtin_amdgcn_global_load_lds((const void *)(b0 + doff(VPT + l)),
                                                     (__attribute__((address_space(3))) void *)(lds + l * kBlock + wave * 64),
                                                     16, 0, 2);
            }
        }
        // LDS slot l (slot VPT + l of the slice), zero where masked; valid
        // once lds_ready() has run in this row
        auto LD = [&](int l) -> u32x4 {
            const u32x4 v = lds[l * kBlock + tid];
            return (FULLS || ok_of(VPT + l)) ? v : u32x4{0u, 0u, 0u, 0u};
        };
        auto lds_ready = [&]() {
            if constexpr (L > 0) __builtin_amdgcn_s_waitcnt(0);
        };
        u32x4 t0 = {0u, 0u, 0u, 0u}, t1 = {0u, 0u, 0u, 0u};
        if (tail) {
            t0 = load_vec<DT, false>(r0, tcol, tn, false);
            if constexpr (T::TWO) t1 = load_vec<DT, false>(r1, tcol, tn, false);
        }
        // Called at the start of every pass over the retained slice.
        auto fresh = [&]() {
            opaque<VPT>(d0);
            if constexpr (T::TWO) opaque<VPT>(d1);
        };
        if constexpr (!FULLS) {
            fresh();  // all loads are in flight; wait for them once here
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                const bool ok = ok_of(j);
                d0[j] = ok ? d0[j] : u32x4{0u, 0u, 0u, 0u};
                if constexpr (T::TWO) d1[j] = ok ? d1[j] : u32x4{0u, 0u, 0u, 0u};
            }
        }

        if constexpr (OP == OP_SOFTMAX_FWD) {
            // Base-2 statistics: K = scale * log2(e); c = max(q * K); s = sum 2^(q*K - c).
            const float K = (FP8 ? a.s0[row] : 1.f) * kLog2e;
            // EC: the slice is decoded once into ec, which then holds
            // e = 2^(q*K - ct) about the thread's own maximum ct; the output is
            // e * 2^(ct - c) * omul, one multiply per element instead of a
            // second decode and exponential.  ECI: an FP32 slice is its own
            // decoded form, so e overwrites it in place (no extra registers).
            constexpr bool EC = ec_regs<OP, DT, VPT>() > 0;
            constexpr bool ECI = DT == DT_F32;
            float ec[EC ? VPT * EPV : 1];
            static_assert(!(EC && L > 0), "kept exponentials cover register slots only");
            float qmax = -INFINITY;
            fresh();
            lds_ready();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float q[EPV];
                decode<DT>(d0[j], q, 1.f);
                const bool ok = ok_of(j);
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    qmax = fmaxf(qmax, ok ? q[i] : -INFINITY);
                    if constexpr (EC) ec[j * EPV + i] = q[i];
                }
                keep_order(qmax);
            }
#pragma unroll
            for (int l = 0; l < L; ++l) {
                float q[EPV];
                decode<DT>(LD(l), q, 1.f);
                const bool ok = ok_of(VPT + l);
#pragma unroll
                for (int i = 0; i < EPV; ++i) qmax = fmaxf(qmax, ok ? q[i] : -INFINITY);
                keep_order(qmax);
            }
            if (tail) {
                float q[EPV];
                decode<DT>(t0, q, 1.f);
                for (int i = 0; i < tn; ++i) qmax = fmaxf(qmax, q[i]);
            }
            float st[2] = {qmax == -INFINITY ? -INFINITY : qmax * K, 0.f};
            const float ct = qmax == -INFINITY ? 0.f : st[0];
            fresh();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float q[EPV], ev[EPV];
                if constexpr (!EC) decode<DT>(d0[j], q, 1.f);
                const bool ok = ok_of(j);
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    ev[i] = fast_exp2(fmaf(EC ? ec[j * EPV + i] : q[i], K, -ct));
                    if constexpr (EC) ec[j * EPV + i] = ev[i];
                    st[1] += ok ? ev[i] : 0.f;
                }
                if constexpr (ECI)
                    d0[j] = u32x4{__float_as_uint(ev[0]), __float_as_uint(ev[1]), __float_as_uint(ev[2]),
                                  __float_as_uint(ev[3])};
                keep_order(st[1]);
            }
#pragma unroll
            for (int l = 0; l < L; ++l) {  // LDS slots: the exponentials are not kept
                float q[EPV];
                decode<DT>(LD(l), q, 1.f);
                const bool ok = ok_of(VPT + l);
#pragma unroll
                for (int i = 0; i < EPV; ++i) st[1] += ok ? fast_exp2(fmaf(q[i], K, -ct)) : 0.f;
                keep_order(st[1]);
            }
            if (tail) {
                float q[EPV];
                decode<DT>(t0, q, 1.f);
                for (int i = 0; i < tn; ++i) st[1] += fast_exp2(fmaf(q[i], K, -ct));
            }
            row_reduce<2>(st, MergeSoftmax(), a, row, 0, c, red, xb, parity);
            const float cmax = st[0];
            const float inv_s = 1.f / st[1];
            // FP8 output: the largest output is 2^0 * inv_s, so amax = inv_s and the
            // code of element i is 448 * 2^(q*K - c) (no second statistics stage).
            const float omul = FP8 ? kFp8Max : inv_s;
            const float csh = kExpShift - cmax, omuls = omul * kExpUnshift;
            if (FP8 && writer) a.so[row] = inv_s / kFp8Max;
            if constexpr (EC || ECI) {
                // ct <= cmax, so the exponent is at most 32 for a thread with a
                // finite element.  A thread whose elements are all -inf (masked)
                // has ct = 0 and exponentials of 0; with the row maximum far
                // below zero its unclamped factor 2^(32 - cmax) would overflow
                // and 0 * inf would store NaN.  The clamp keeps it finite.
                const float f = fast_exp2(fminf(ct + csh, 64.f)) * omuls;
#pragma unroll
                for (int j = 0; j < VPT; ++j) {
                    float y[EPV];
                    if constexpr (EC) {
#pragma unroll
                        for (int i = 0; i < EPV; ++i) y[i] = ec[j * EPV + i] * f;
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i) y[i] = __uint_as_float(d0[j][i]) * f;
                    }
                    ST(j, encode<DT>(y, 1.f));
                }
            } else {
                // FP8: 448 * 2^(q K - c) is taken as one exponential, 2^(q K + log2 448 - c),
                // saving a multiply per element (outputs below 2^-126 of the largest
                // are 0 either way, far below the smallest e4m3 code)
                const float cs8 = kLog2Fp8Max - cmax;
                fresh();
#pragma unroll
                for (int j = 0; j < VPT; ++j) {
                    float q[EPV], y[EPV];
                    decode<DT>(d0[j], q, 1.f);
#pragma unroll
                    for (int i = 0; i < EPV; ++i)
                        y[i] = FP8 ? fast_exp2(fmaf(q[i], K, cs8)) : fast_exp2(fmaf(q[i], K, csh)) * omuls;
                    ST(j, encode<DT>(y, 1.f));
                }
            }
#pragma unroll
            for (int l = 0; l < L; ++l) {
                float q[EPV], y[EPV];
                decode<DT>(LD(l), q, 1.f);
#pragma unroll
                for (int i = 0; i < EPV; ++i) y[i] = fast_exp2(fmaf(q[i], K, csh)) * omuls;
                ST(VPT + l, encode<DT>(y, 1.f));
            }
            if (tail) {
                float q[EPV], y[EPV];
                decode<DT>(t0, q, 1.f);
#pragma unroll
                for (int i = 0; i < EPV; ++i) y[i] = fast_exp2(fmaf(q[i], K, csh)) * omuls;
                store_vec<DT>(orow, tcol, tn, false, encode<DT>(y, 1.f));
            }
        } else if constexpr (OP == OP_LN_FWD || OP == OP_RMS_FWD || OP == OP_LNQ_FWD) {
            constexpr bool LN = OP != OP_RMS_FWD;
            constexpr bool QO = OP == OP_LNQ_FWD;  // e4m3 codes out from an FP32 / BF16 row
            constexpr bool F8O = FP8 || QO;        // FP8 output: one more (amax) stage
            // Statistics on the decoded codes q (x = xs * q for FP8, q = x
            // otherwise), so the per-row scale is applied once per row, not per
            // element: mean_x = xs mean_q, var_x = xs^2 var_q, y uses xs * rstd.
            const float xs = FP8 ? a.s0[row] : 1.f;
            float mean_q = 0.f, amul;
            if constexpr (LN) {
                // one pass of moments about a per-thread shift Kt (its first
                // held value), turned into (count, mean, M2) with the mean taken
                // relative to the row's first element K (common to every
                // member) and Chan-merged: the merged means are deviations of
                // the size of the row's spread, not of its offset, so their
                // roundings stay small; the mean is K + the merged deviation
                const float K = row_first<DT>(r0);
                float Kt = 0.f;
                {
                    float q[EPV];
                    decode<DT>(d0[0], q, 1.f);
                    float qt[EPV];
                    decode<DT>(t0, qt, 1.f);
                    Kt = (FULLS || ok_of(0)) ? q[0] : (tail ? qt[0] : K);
                }
                float s1 = 0.f, s2 = 0.f;
                fresh();
                lds_ready();
#pragma unroll
                for (int j = 0; j < VPT + L; ++j) {
                    float q[EPV];
                    decode<DT>(j < VPT ? d0[j < VPT ? j : 0] : LD(j < VPT ? 0 : j - VPT), q, 1.f);
                    const bool ok = ok_of(j);
#pragma unroll
                    for (int i = 0; i < EPV; ++i) {
                        float d = ok ? q[i] - Kt : 0.f;
                        s1 += d;
                        s2 = fmaf(d, d, s2);
                    }
                    keep_order(s1, s2);
                }
                if (tail) {
                    float q[EPV];
                    decode<DT>(t0, q, 1.f);
                    for (int i = 0; i < tn; ++i) {
                        float d = q[i] - Kt;
                        s1 += d;
                        s2 = fmaf(d, d, s2);
                    }
                }
                float st[3] = {held, 0.f, 0.f};
                if (held > 0.f) {
                    const float m = s1 / held;
                    st[1] = (Kt - K) + m;
                    st[2] = fmaxf(s2 - s1 * m, 0.f);
                }
                row_reduce_chan(st, a, row, 0, c, red, xb, parity);
                mean_q = K + st[1];
                const float rstd = rsqrtf(xs * xs * (st[2] * invN) + a.eps);
                amul = xs * rstd;
                if (writer) {
                    if (a.mean_out) a.mean_out[row] = xs * mean_q;
                    if (a.rstd_out) a.rstd_out[row] = rstd;
                }
            } else {
                float st[1] = {0.f};
                fresh();
                lds_ready();
#pragma unroll
                for (int j = 0; j < VPT + L; ++j) {
                    float q[EPV];
                    decode<DT>(j < VPT ? d0[j < VPT ? j : 0] : LD(j < VPT ? 0 : j - VPT), q, 1.f);
#pragma unroll
                    for (int i = 0; i < EPV; ++i) st[0] = fmaf(q[i], q[i], st[0]);
                    keep_order(st[0]);
                }
                if (tail) {
                    float q[EPV];
                    decode<DT>(t0, q, 1.f);
#pragma unroll
                    for (int i = 0; i < EPV; ++i) st[0] = fmaf(q[i], q[i], st[0]);
                }
                row_reduce<1>(st, MergeSum(), a, row, 0, c, red, xb, parity);
                const float rstd = rsqrtf(xs * xs * (st[0] * invN) + a.eps);
                amul = xs * rstd;
                if (writer) {
                    if (a.mean_out) a.mean_out[row] = 0.f;
                    if (a.rstd_out) a.rstd_out[row] = rstd;
                }
            }
            auto h = [&](const float *q, const float *g, const float *bb, float *y) {
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    if constexpr (LN)
                        y[i] = fmaf((q[i] - mean_q) * amul, g[i], bb[i]);
                    else
                        y[i] = q[i] * amul * g[i];
                }
            };
            // FP8 output keeps y in registers between the amax stage and the
            // quantize pass when the slice holds at most kYcMax values per
            // thread: gamma / beta are then read once instead of twice
            constexpr bool YC = yc_regs<OP, DT, VPT>() > 0;
            float yc[YC ? VPT * EPV : 1], yct[YC ? EPV : 1];
            // the trailing partial vector of the output
            auto store_out_tail = [&](const float *y, float oinv) {
                if constexpr (QO) {
                    unsigned w[EPV / 4];
                    quant_codes<false, EPV>(y, oinv, w);
                    for (int i = 0; i < tn; ++i) orow[tcol + i] = (char)((w[i / 4] >> (8 * (i % 4))) & 0xffu);
                } else {
                    store_vec<DT>(orow, tcol, tn, false, encode<DT>(y, oinv));
                }
            };
            // output pass over the slots in batches of GB: the parameter loads of
            // a batch are issued together; store == false only measures amax
            auto out_pass = [&](bool store, float oinv, float &amax) {
                fresh();
#pragma unroll
                for (int jb = 0; jb < VPT + L; jb += GB) {
                    // keep the scheduler from hoisting every batch's parameter
                    // loads to the top (that would hold VPT slots of gamma/beta)
                    __builtin_amdgcn_sched_barrier(0);
                    float g[GB][EPV], bb[GB][LN ? EPV : 1];
#pragma unroll
                    for (int u = 0; u < GB; ++u) {
                        PAR(a.gamma, jb + u, g[u]);
                        if constexpr (LN) PAR(a.beta, jb + u, bb[u]);
                    }
#pragma unroll
                    for (int u = 0; u < GB; ++u) {
                        const int j = jb + u;
                        float q[EPV], y[EPV];
                        decode<DT>(j < VPT ? d0[j < VPT ? j : 0] : LD(j < VPT ? 0 : j - VPT), q, 1.f);
                        h(q, g[u], LN ? bb[u] : g[u], y);
                        if (store) {
                            if constexpr (QO) {
                                unsigned w[EPV / 4];
                                quant_codes<false, EPV>(y, oinv, w);
                                QST(j, w);
                            } else {
                                ST(j, encode<DT>(y, oinv));
                            }
                        } else {
                            const bool ok = ok_of(j);
#pragma unroll
                            for (int i = 0; i < EPV; ++i) {
                                amax = fmaxf(amax, ok ? fabsf(y[i]) : 0.f);
                                if constexpr (YC) yc[j * EPV + i] = y[i];
                            }
                            keep_order(amax);
                        }
                    }
                }
                if (tail) {
                    float q[EPV], y[EPV], g[EPV], bb[EPV];
                    decode<DT>(t0, q, 1.f);
                    load_params_tail<DT>(a.gamma, tcol, tn, g);
                    if constexpr (LN) load_params_tail<DT>(a.beta, tcol, tn, bb);
                    h(q, g, bb, y);
                    if (store) {
                        store_out_tail(y, oinv);
                    } else {
                        for (int i = 0; i < tn; ++i) amax = fmaxf(amax, fabsf(y[i]));
                        if constexpr (YC) {
#pragma unroll
                            for (int i = 0; i < EPV; ++i) yct[i] = y[i];
                        }
                    }
                }
            };
            float oinv = 1.f;
            if constexpr (F8O) {
                float am[1] = {0.f};
                out_pass(false, 1.f, am[0]);
                row_reduce<1>(am, MergeMax(), a, row, 1, c, red, xb, parity);
                oinv = am[0] > 0.f ? kFp8Max / am[0] : 1.f;
                if (writer) a.so[row] = am[0] > 0.f ? am[0] / kFp8Max : 1.f;
            }
            if constexpr (YC) {
#pragma unroll
                for (int j = 0; j < VPT; ++j) {
                    if constexpr (QO) {
                        unsigned w[EPV / 4];
                        quant_codes<false, EPV>(&yc[j * EPV], oinv, w);
                        QST(j, w);
                    } else {
                        ST(j, encode<DT>(&yc[j * EPV], oinv));
                    }
                }
                if (tail) store_out_tail(yct, oinv);
            } else {
                float unused = 0.f;
                out_pass(true, oinv, unused);
            }
        } else if constexpr (OP == OP_SOFTMAX_BWD) {
            const float ys = FP8 ? a.s0[row] : 1.f, gs = FP8 ? a.s1[row] : 1.f;
            float st[1] = {0.f};
            fresh();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float y[EPV], g[EPV];
                decode<DT>(d0[j], y, ys);
                decode<DT>(d1[j], g, gs);
#pragma unroll
                for (int i = 0; i < EPV; ++i) st[0] = fmaf(g[i], y[i], st[0]);
                keep_order(st[0]);
            }
            if (tail) {
                float y[EPV], g[EPV];
                decode<DT>(t0, y, ys);
                decode<DT>(t1, g, gs);
#pragma unroll
                for (int i = 0; i < EPV; ++i) st[0] = fmaf(g[i], y[i], st[0]);
            }
            row_reduce<1>(st, MergeSum(), a, row, 0, c, red, xb, parity);
            const float cs = st[0];
            auto h = [&](u32x4 yv, u32x4 gv, float *dx) {
                float y[EPV], g[EPV];
                decode<DT>(yv, y, ys);
                decode<DT>(gv, g, gs);
#pragma unroll
                for (int i = 0; i < EPV; ++i) dx[i] = y[i] * (g[i] - cs);
            };
            float oinv = 1.f;
            if constexpr (FP8) {
                float am[1] = {0.f};
                fresh();
#pragma unroll
                for (int j = 0; j < VPT; ++j) {
                    float dx[EPV];
                    h(d0[j], d1[j], dx);
#pragma unroll
                    for (int i = 0; i < EPV; ++i) am[0] = fmaxf(am[0], fabsf(dx[i]));  // masked: y = 0
                }
                if (tail) {
                    float dx[EPV];
                    h(t0, t1, dx);
#pragma unroll
                    for (int i = 0; i < EPV; ++i) am[0] = fmaxf(am[0], fabsf(dx[i]));
                }
                row_reduce<1>(am, MergeMax(), a, row, 1, c, red, xb, parity);
                oinv = am[0] > 0.f ? kFp8Max / am[0] : 1.f;
                if (writer) a.so[row] = am[0] > 0.f ? am[0] / kFp8Max : 1.f;
            }
            fresh();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float dx[EPV];
                h(d0[j], d1[j], dx);
                ST(j, encode<DT>(dx, oinv));
            }
            if (tail) {
                float dx[EPV];
                h(t0, t1, dx);
                store_vec<DT>(orow, tcol, tn, false, encode<DT>(dx, oinv));
            }
        } else if constexpr (OP == OP_LN_BWD || OP == OP_RMS_BWD) {
            constexpr bool LN = OP == OP_LN_BWD;
            const float xs = FP8 ? a.s0[row] : 1.f, gs = FP8 ? a.s1[row] : 1.f;
            float mean = 0.f, rstd;
            if (a.flags & F_RECOMPUTE) {
                if constexpr (LN) {
                    // moments about a per-thread shift, means relative to the
                    // row's first element, Chan-merged (as in the forward)
                    const float K = row_first<DT>(r0) * xs;
                    float Kt = 0.f;
                    {
                        float x[EPV], xt[EPV];
                        decode<DT>(d0[0], x, xs);
                        decode<DT>(t0, xt, xs);
                        Kt = (FULLS || ok_of(0)) ? x[0] : (tail ? xt[0] : K);
                    }
                    float s1 = 0.f, s2 = 0.f;
                    fresh();
#pragma unroll
                    for (int j = 0; j < VPT; ++j) {
                        float x[EPV];
                        decode<DT>(d0[j], x, xs);
                        const bool ok = ok_of(j);
#pragma unroll
                        for (int i = 0; i < EPV; ++i) {
                            float d = ok ? x[i] - Kt : 0.f;
                            s1 += d;
                            s2 = fmaf(d, d, s2);
                        }
                        keep_order(s1, s2);
                    }
                    if (tail) {
                        float x[EPV];
                        decode<DT>(t0, x, xs);
                        for (int i = 0; i < tn; ++i) {
                            float d = x[i] - Kt;
                            s1 += d;
                            s2 = fmaf(d, d, s2);
                        }
                    }
                    float st[3] = {held, 0.f, 0.f};
                    if (held > 0.f) {
                        const float m = s1 / held;
                        st[1] = (Kt - K) + m;
                        st[2] = fmaxf(s2 - s1 * m, 0.f);
                    }
                    row_reduce_chan(st, a, row, 2, c, red, xb, parity);
                    mean = K + st[1];
                    rstd = rsqrtf(st[2] * invN + a.eps);
                } else {
                    float st[1] = {0.f};
                    fresh();
#pragma unroll
                    for (int j = 0; j < VPT; ++j) {
                        float x[EPV];
                        decode<DT>(d0[j], x, xs);
#pragma unroll
                        for (int i = 0; i < EPV; ++i) st[0] = fmaf(x[i], x[i], st[0]);
                        keep_order(st[0]);
                    }
                    if (tail) {
                        float x[EPV];
                        decode<DT>(t0, x, xs);
#pragma unroll
                        for (int i = 0; i < EPV; ++i) st[0] = fmaf(x[i], x[i], st[0]);
                    }
                    row_reduce<1>(st, MergeSum(), a, row, 2, c, red, xb, parity);
                    rstd = rsqrtf(st[0] * invN + a.eps);
                }
            } else {
                if constexpr (LN) mean = a.mean_in[row];
                rstd = a.rstd_in[row];
            }
            // stage: (sum g, sum g*xhat) for LayerNorm, (sum g*xhat) for RMSNorm;
            // masked slots have dy = 0, hence g = 0
            constexpr int Q = LN ? 2 : 1;
            float st[Q];
#pragma unroll
            for (int t = 0; t < Q; ++t) st[t] = 0.f;
            auto acc = [&](const float *x, const float *dy, const float *gm) {
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    float xh = (x[i] - mean) * rstd;
                    float g = dy[i] * gm[i];
                    if constexpr (LN) {
                        st[0] += g;
                        st[1] = fmaf(g, xh, st[1]);
                    } else {
                        st[0] = fmaf(g, xh, st[0]);
                    }
                }
            };
            // GI: the statistics pass also adds the column partials and keeps
            // g = dy * gamma, so the output pass reads no gamma and needs no
            // second product.  FP32 overwrites the resident dy with g; BF16
            // slices of up to two vectors keep g in registers of their own
            // (gk_regs; larger slices would lose a workgroup per CU).
            constexpr bool GK = gk_regs<OP, DT, VPT>() > 0;
            constexpr bool GI = DT == DT_F32 || GK;
            float gk[GK ? VPT * EPV : 1];
            fresh();
#pragma unroll
            for (int jb = 0; jb < VPT; jb += GB) {
                __builtin_amdgcn_sched_barrier(0);
                float gm[GB][EPV];
#pragma unroll
                for (int u = 0; u < GB; ++u) PAR(a.gamma, jb + u, gm[u]);
#pragma unroll
                for (int u = 0; u < GB; ++u) {
                    const int j = jb + u;
                    float x[EPV], dy[EPV];
                    decode<DT>(d0[j], x, xs);
                    decode<DT>(d1[j], dy, gs);
                    if constexpr (GI) {
                        float g[EPV];
#pragma unroll
                        for (int i = 0; i < EPV; ++i) {  // masked slots: x = dy = 0, adding 0
                            float xh = (x[i] - mean) * rstd;
                            g[i] = dy[i] * gm[u][i];
                            if constexpr (LN) {
                                st[0] += g[i];
                                st[1] = fmaf(g[i], xh, st[1]);
                            } else {
                                st[0] = fmaf(g[i], xh, st[0]);
                            }
                            cp[0][j * EPV + i] = fmaf(dy[i], xh, cp[0][j * EPV + i]);
                            if constexpr (LN) cp[NCP - 1][j * EPV + i] += dy[i];
                        }
                        if constexpr (GK) {
#pragma unroll
                            for (int i = 0; i < EPV; ++i) gk[j * EPV + i] = g[i];
                        } else {
                            d1[j] = u32x4{__float_as_uint(g[0]), __float_as_uint(g[1]), __float_as_uint(g[2]),
                                          __float_as_uint(g[3])};
                        }
                    } else {
                        acc(x, dy, gm[u]);
                    }
                    if constexpr (LN) keep_order(st[0], st[LN ? 1 : 0]);
                    else keep_order(st[0]);
                }
            }
            if (tail) {
                float x[EPV], dy[EPV], gm[EPV];
                decode<DT>(t0, x, xs);
                decode<DT>(t1, dy, gs);
                load_params_tail<DT>(a.gamma, tcol, tn, gm);
                acc(x, dy, gm);
            }
            row_reduce<Q>(st, MergeSum(), a, row, 0, c, red, xb, parity);
            const float c1 = LN ? st[0] * invN : 0.f;
            const float c2 = (LN ? st[1] : st[0]) * invN;
            auto hh = [&](const float *x, const float *dy, const float *gm, float *dx) {
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    float xh = (x[i] - mean) * rstd;
                    dx[i] = rstd * (dy[i] * gm[i] - c1 - xh * c2);
                }
            };
            auto out_pass = [&](bool store, float oinv, float &amax) {
                fresh();
                if constexpr (GI) {
#pragma unroll
                    for (int j = 0; j < VPT; ++j) {
                        float x[EPV], dx[EPV];
                        decode<DT>(d0[j], x, xs);
#pragma unroll
                        for (int i = 0; i < EPV; ++i) {
                            float xh = (x[i] - mean) * rstd;
                            float gv;
                            if constexpr (GK) gv = gk[j * EPV + i];
                            else gv = __uint_as_float(d1[j][i]);
                            dx[i] = rstd * (gv - c1 - xh * c2);
                        }
                        ST(j, encode<DT>(dx, oinv));
                    }
                }
#pragma unroll
                for (int jb = 0; jb < (GI ? 0 : VPT); jb += GB) {
                    __builtin_amdgcn_sched_barrier(0);
                    float gm[GB][EPV];
#pragma unroll
                    for (int u = 0; u < GB; ++u)
                        PAR(a.gamma, jb + u, gm[u]);
#pragma unroll
                    for (int u = 0; u < GB; ++u) {
                        const int j = jb + u;
                        float x[EPV], dy[EPV], dx[EPV];
                        decode<DT>(d0[j], x, xs);
                        decode<DT>(d1[j], dy, gs);
                        hh(x, dy, gm[u], dx);
                        const bool ok = ok_of(j);
                        if (store) {
#pragma unroll
                            for (int i = 0; i < EPV; ++i) {  // masked slots add dy = 0
                                float xh = (x[i] - mean) * rstd;
                                cp[0][j * EPV + i] = fmaf(dy[i], xh, cp[0][j * EPV + i]);
                                if constexpr (LN) cp[NCP - 1][j * EPV + i] += dy[i];
                            }
                            ST(j, encode<DT>(dx, oinv));
                        } else {
#pragma unroll
                            for (int i = 0; i < EPV; ++i) amax = fmaxf(amax, ok ? fabsf(dx[i]) : 0.f);
                        }
                    }
                }
                if (tail) {
                    float x[EPV], dy[EPV], gm[EPV], dx[EPV];
                    decode<DT>(t0, x, xs);
                    decode<DT>(t1, dy, gs);
                    load_params_tail<DT>(a.gamma, tcol, tn, gm);
                    hh(x, dy, gm, dx);
                    if (store) {
#pragma unroll
                        for (int i = 0; i < EPV; ++i) {
                            float xh = (x[i] - mean) * rstd;
                            cpt[0][i] = fmaf(dy[i], xh, cpt[0][i]);
                            if constexpr (LN) cpt[NCP - 1][i] += dy[i];
                        }
                        store_vec<DT>(orow, tcol, tn, false, encode<DT>(dx, oinv));
                    } else {
                        for (int i = 0; i < tn; ++i) amax = fmaxf(amax, fabsf(dx[i]));
                    }
                }
            };
            float oinv = 1.f;
            if constexpr (FP8) {
                float am[1] = {0.f};
                out_pass(false, 1.f, am[0]);
                row_reduce<1>(am, MergeMax(), a, row, 1, c, red, xb, parity);
                oinv = am[0] > 0.f ? kFp8Max / am[0] : 1.f;
                if (writer) a.so[row] = am[0] > 0.f ? am[0] / kFp8Max : 1.f;
            }
            float unused = 0.f;
            out_pass(true, oinv, unused);
        } else if constexpr (OP == OP_SMXL_BWD) {
            // Softmax backward from the logits: y = softmax(x) is rebuilt from the
            // resident x.  One stage carries (c, s, t): c = max of x*log2(e),
            // s = sum 2^(xK - c), t = sum dy 2^(xK - c), so sum dy*y = t / s.
            const float K = (FP8 ? a.s0[row] : 1.f) * kLog2e;
            const float gs = FP8 ? a.s1[row] : 1.f;
            float qmax = -INFINITY;
            fresh();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float q[EPV];
                decode<DT>(d0[j], q, 1.f);
                const bool ok = ok_of(j);
#pragma unroll
                for (int i = 0; i < EPV; ++i) qmax = fmaxf(qmax, ok ? q[i] : -INFINITY);
            }
            if (tail) {
                float q[EPV];
                decode<DT>(t0, q, 1.f);
                for (int i = 0; i < tn; ++i) qmax = fmaxf(qmax, q[i]);
            }
            float st[3] = {qmax == -INFINITY ? -INFINITY : qmax * K, 0.f, 0.f};
            const float ct = qmax == -INFINITY ? 0.f : st[0];
            fresh();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float q[EPV], g[EPV];
                decode<DT>(d0[j], q, 1.f);
                decode<DT>(d1[j], g, gs);
                const bool ok = ok_of(j);
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    const float e = ok ? fast_exp2(fmaf(q[i], K, -ct)) : 0.f;
                    st[1] += e;
                    st[2] = fmaf(e, g[i], st[2]);
                }
                keep_order(st[1], st[2]);
            }
            if (tail) {
                float q[EPV], g[EPV];
                decode<DT>(t0, q, 1.f);
                decode<DT>(t1, g, gs);
                for (int i = 0; i < tn; ++i) {
                    const float e = fast_exp2(fmaf(q[i], K, -ct));
                    st[1] += e;
                    st[2] = fmaf(e, g[i], st[2]);
                }
            }
            row_reduce<3>(st, MergeSoftmax3(), a, row, 0, c, red, xb, parity);
            const float cmax = st[0], inv_s = 1.f / st[1];
            const float cdot = st[2] * inv_s;
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
                fresh();
#pragma unroll
                for (int j = 0; j < VPT; ++j) {
                    float dx[EPV];
                    h(d0[j], d1[j], dx);
                    const bool ok = ok_of(j);
#pragma unroll
                    for (int i = 0; i < EPV; ++i) am[0] = fmaxf(am[0], ok ? fabsf(dx[i]) : 0.f);
                }
                if (tail) {
                    float dx[EPV];
                    h(t0, t1, dx);
                    for (int i = 0; i < tn; ++i) am[0] = fmaxf(am[0], fabsf(dx[i]));
                }
                row_reduce<1>(am, MergeMax(), a, row, 1, c, red, xb, parity);
                oinv = am[0] > 0.f ? kFp8Max / am[0] : 1.f;
                if (writer) a.so[row] = am[0] > 0.f ? am[0] / kFp8Max : 1.f;
            }
            fresh();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float dx[EPV];
                h(d0[j], d1[j], dx);
                ST(j, encode<DT>(dx, oinv));
            }
            if (tail) {
                float dx[EPV];
                h(t0, t1, dx);
                store_vec<DT>(orow, tcol, tn, false, encode<DT>(dx, oinv));
            }
        } else if constexpr (T::QUANT) {
            // Row-wise quantisation: amax stage, then the code nearest to
            // x * qmax / amax (decided exactly, ties to even) with the row scale
            // amax / qmax (1 for an all-zero row).
            constexpr bool I8 = OP == OP_QUANT_I8;
            float am[1] = {0.f};
            fresh();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float q[EPV];
                decode<DT>(d0[j], q, 1.f);
#pragma unroll
                for (int i = 0; i < EPV; ++i) am[0] = fmaxf(am[0], fabsf(q[i]));  // masked slots are 0
                keep_order(am[0]);
            }
            if (tail) {
                float q[EPV];
                decode<DT>(t0, q, 1.f);
                for (int i = 0; i < tn; ++i) am[0] = fmaxf(am[0], fabsf(q[i]));
            }
            row_reduce<1>(am, MergeMax(), a, row, 0, c, red, xb, parity);
            const float qm = I8 ? 127.f : kFp8Max;
            const float amx = am[0];
            float qsc = 1.f, inv = 1.f;  // an all-zero row: every code is 0
            if (amx > 0.f) quant_row_factors(amx, qm, qsc, inv);
            if (writer) a.so[row] = amx > 0.f ? amx / qm : 1.f;
            fresh();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float q[EPV];
                decode<DT>(d0[j], q, 1.f);
                unsigned w[EPV / 4];
                quant_codes_exact<I8, EPV>(q, qsc, inv, amx > 0.f ? amx : 1.f, w);
                QST(j, w);
            }
            if (tail) {
                float q[EPV];
                decode<DT>(t0, q, 1.f);
                unsigned w[EPV / 4];
                quant_codes_exact<I8, EPV>(q, qsc, inv, amx > 0.f ? amx : 1.f, w);
                for (int i = 0; i < tn; ++i) orow[tcol + i] = (char)((w[i / 4] >> (8 * (i % 4))) & 0xffu);
            }
        } else if constexpr (OP == OP_PEARSON_BWD) {
            // Pearson correlation r of the rows x and y: one stage of bivariate
            // co-moments (one pass of sums about a per-thread shift), then
            // dx = dr (yc / sqrt(Cxx Cyy) - r xc / Cxx) and symmetrically dy.
            float Kx = 0.f, Ky = 0.f;
            {
                float x[EPV], y[EPV], xt[EPV], yt[EPV];
                decode<DT>(d0[0], x, 1.f);
                decode<DT>(d1[0], y, 1.f);
                decode<DT>(t0, xt, 1.f);
                decode<DT>(t1, yt, 1.f);
                const bool first = FULLS || ok_of(0);
                Kx = first ? x[0] : (tail ? xt[0] : 0.f);
                Ky = first ? y[0] : (tail ? yt[0] : 0.f);
            }
            float sx = 0.f, sy = 0.f, sxx = 0.f, syy = 0.f, sxy = 0.f;
            auto acc = [&](const float *x, const float *y, int n, bool ok) {
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    const bool v = ok && i < n;
                    const float dx = v ? x[i] - Kx : 0.f, dy = v ? y[i] - Ky : 0.f;
                    sx += dx;
                    sy += dy;
                    sxx = fmaf(dx, dx, sxx);
                    syy = fmaf(dy, dy, syy);
                    sxy = fmaf(dx, dy, sxy);
                }
            };
            fresh();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float x[EPV], y[EPV];
                decode<DT>(d0[j], x, 1.f);
                decode<DT>(d1[j], y, 1.f);
                acc(x, y, EPV, ok_of(j));
                keep_order(sx, sy, sxx, syy, sxy);
            }
            if (tail) {
                float x[EPV], y[EPV];
                decode<DT>(t0, x, 1.f);
                decode<DT>(t1, y, 1.f);
                acc(x, y, tn, true);
            }
            float st[6] = {held, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (held > 0.f) {
                const float mx = sx / held, my = sy / held;
                st[1] = Kx + mx;
                st[2] = Ky + my;
                st[3] = fmaxf(sxx - sx * mx, 0.f);
                st[4] = fmaxf(syy - sy * my, 0.f);
                st[5] = sxy - sx * my;
            }
            row_reduce_co(st, a, row, 0, c, red, xb, parity);
            const float mx = st[1], my = st[2];
            const float ix = rsqrtf(st[3]), iy = rsqrtf(st[4]);
            const float dr = a.rowg[row];
            const float r = st[5] * ix * iy;
            const float ca = dr * ix * iy, cbx = dr * r / st[3], cby = dr * r / st[4];
            auto h = [&](u32x4 xv, u32x4 yv, float *gx, float *gy) {
                float x[EPV], y[EPV];
                decode<DT>(xv, x, 1.f);
                decode<DT>(yv, y, 1.f);
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    const float xc = x[i] - mx, yc = y[i] - my;
                    gx[i] = fmaf(ca, yc, -cbx * xc);
                    gy[i] = fmaf(ca, xc, -cby * yc);
                }
            };
            fresh();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float gx[EPV], gy[EPV];
                h(d0[j], d1[j], gx, gy);
                ST(j, encode<DT>(gx, 1.f));
                ST1(j, encode<DT>(gy, 1.f));
            }
            if (tail) {
                float gx[EPV], gy[EPV];
                h(t0, t1, gx, gy);
                store_vec<DT>(orow, tcol, tn, false, encode<DT>(gx, 1.f));
                store_vec<DT>(orow1, tcol, tn, false, encode<DT>(gy, 1.f));
            }
        } else if constexpr (OP == OP_WVAR_BWD) {
            // Weighted variance v = sum w (x - mu)^2 / W, mu = sum w x / W,
            // W = sum w: one stage of weighted (W, mean, M2) (one pass of sums
            // about a per-thread shift, Chan-merged with W as the count), then
            // dx = dv 2 w (x - mu) / W and dw = dv ((x - mu)^2 - v) / W.
            float K = 0.f;
            {
                float x[EPV], xt[EPV];
                decode<DT>(d0[0], x, 1.f);
                decode<DT>(t0, xt, 1.f);
                K = (FULLS || ok_of(0)) ? x[0] : (tail ? xt[0] : 0.f);
            }
            float sw = 0.f, swd = 0.f, swdd = 0.f;
            auto acc = [&](const float *x, const float *w, int n) {
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    const float wi = i < n ? w[i] : 0.f;  // masked slots hold w = 0
                    const float d = x[i] - K, wd = wi * d;
                    sw += wi;
                    swd += wd;
                    swdd = fmaf(wd, d, swdd);
                }
            };
            fresh();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float x[EPV], w[EPV];
                decode<DT>(d0[j], x, 1.f);
                decode<DT>(d1[j], w, 1.f);
                acc(x, w, EPV);
                keep_order(sw, swd, swdd);
            }
            if (tail) {
                float x[EPV], w[EPV];
                decode<DT>(t0, x, 1.f);
                decode<DT>(t1, w, 1.f);
                acc(x, w, tn);
            }
            float st[3] = {sw, 0.f, 0.f};
            if (sw != 0.f) {
                const float m = swd / sw;
                st[1] = K + m;
                st[2] = fmaxf(swdd - swd * m, 0.f);
            }
            row_reduce<3>(st, MergeChan(), a, row, 0, c, red, xb, parity);
            const float W = st[0], mu = st[1], var = st[2] / W;
            const float f = a.rowg[row] / W, f2 = 2.f * f;
            auto h = [&](u32x4 xv, u32x4 wv, float *gx, float *gw) {
                float x[EPV], w[EPV];
                decode<DT>(xv, x, 1.f);
                decode<DT>(wv, w, 1.f);
#pragma unroll
                for (int i = 0; i < EPV; ++i) {
                    const float d = x[i] - mu;
                    gx[i] = f2 * w[i] * d;
                    gw[i] = f * fmaf(d, d, -var);
                }
            };
            fresh();
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                float gx[EPV], gw[EPV];
                h(d0[j], d1[j], gx, gw);
                ST(j, encode<DT>(gx, 1.f));
                ST1(j, encode<DT>(gw, 1.f));
            }
            if (tail) {
                float gx[EPV], gw[EPV];
                h(t0, t1, gx, gw);
                store_vec<DT>(orow, tcol, tn, false, encode<DT>(gx, 1.f));
                store_vec<DT>(orow1, tcol, tn, false, encode<DT>(gw, 1.f));
            }
        }
    }

    if constexpr (NCP) {
        for (int p = 0; p < NCP; ++p) {
            float *dst = a.colpart + ((int64_t)grp * NCP + p) * a.N;
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                if (!ok_of(j)) continue;
                const int64_t col = col_of(j);
#pragma unroll
                for (int i = 0; i < EPV; ++i) dst[col + i] = cp[p][j * EPV + i];
            }
            if (tail)
                for (int i = 0; i < tn; ++i) dst[tcol + i] = cpt[p][i];
        }
    }
}

template <int OP, int DT, int VPT, int L = 0>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(resident_waves<OP, DT, VPT>())))
void k_resident(RowArgs a) {
    constexpr int EPV = Io<DT>::EPV;
    if (a.flags & F_PROBE) {
        coresidency_probe(a);
        return;
    }
    // a launch recorded in a graph takes its epoch from device memory, bumped
    // by the kernel launched before it on every replay
    if (a.epoch == 0u && a.epoch_ptr)
        a.epoch = __hip_atomic_load(a.epoch_ptr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __shared__ float red[2 * 4 * 6];  // up to six statistics per reduction
    __shared__ float xb[kMaxK * kMaxQ];
    __shared__ LdsSlice<L> ls;
    int c, grp;
    member_of(a, blockIdx.x, c, grp);
    Slice sl;
    sl.c0 = (int64_t)c * a.chunk;
    const int64_t rem = a.N - sl.c0;
    sl.nval = rem <= 0 ? 0 : (rem < a.chunk ? rem : a.chunk);
    sl.nfv = sl.nval / EPV;
    sl.tail_n = (int)(sl.nval - sl.nfv * EPV);
    sl.owner = (int)(sl.nfv % kBlock);
    constexpr int AL_ALL = F_ALIGN0 | F_ALIGNO | F_ALIGNP | (OpTraits<OP>::TWO ? F_ALIGN1 : 0) |
                           (OpTraits<OP>::TWOO ? F_ALIGNO1 : 0);
    const bool al = (a.flags & AL_ALL) == AL_ALL;
    if (al && sl.nval == (int64_t)(VPT + L) * kBlock * EPV)
        row_loop<OP, DT, VPT, true, true, L>(a, c, grp, sl, red, xb, &ls.v[0][0]);
    else
        row_loop<OP, DT, VPT, false, false, L>(a, c, grp, sl, red, xb, &ls.v[0][0]);
}

}  // namespace credit
