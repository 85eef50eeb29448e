// kargs.h -- kernel argument block and enumerations shared by the host
// library and the gfx950 kernels.
#pragma once
#include <stdint.h>

namespace credit {

enum KOp {
    OP_SOFTMAX_FWD = 0, OP_LN_FWD = 1, OP_RMS_FWD = 2, OP_SOFTMAX_BWD = 3, OP_LN_BWD = 4, OP_RMS_BWD = 5,
    // the other reduction-reuse workloads of the evaluation suite (Sec. IV-A)
    OP_SMXL_BWD = 6,     // softmax backward from the logits (y recomputed in the row)
    OP_QUANT_I8 = 7,     // row-wise int8 quantisation, scale = amax / 127
    OP_QUANT_F8 = 8,     // row-wise e4m3 quantisation, scale = amax / 448
    OP_PEARSON_BWD = 9,  // Pearson-correlation backward (x, y, dr -> dx, dy)
    OP_WVAR_BWD = 10,    // weighted-variance backward (x, w, dv -> dx, dw)
    OP_LNQ_FWD = 11,     // LayerNorm forward writing e4m3 codes + row scales from FP32 / BF16 input
    OP_COUNT = 12
};
enum KDt { DT_F32 = 0, DT_BF16 = 1, DT_FP8 = 2 };

constexpr int kMaxStages = 3;  // statistics stages per row (recompute, main, amax)
constexpr int kMaxQ = 5;       // statistics per stage (Pearson co-moments)
constexpr int kMaxK = 32;      // largest split factor
constexpr int kBlockThreads = 256;  // threads per row-resident / split-row workgroup
constexpr int kYcMax = 128;   // most FP32 y values per thread kept across an FP8-output amax stage
constexpr int kEcMax = 64;    // most FP32 exponentials per thread kept by the FP8 softmax forward

enum KFlags {
    F_ALIGN0 = 1,              // rows of in0 start 16-byte aligned
    F_ALIGN1 = 2,              // rows of in1 start 16-byte aligned
    F_ALIGNO = 4,              // rows of out start 16-byte aligned
    F_XCD = 8,                 // XCD-aware member mapping (grid % 8 == 0)
    F_RECOMPUTE = 16,          // norm backward: recompute mean/rstd from x
    F_TEST_DROP_PUBLISH = 32,  // test only: member 1 never publishes
    F_ALIGNP = 64,             // gamma / beta 16-byte aligned
    F_ALIGNO1 = 128,           // rows of out1 start 16-byte aligned
    F_PROBE = 256,             // co-residency probe: no row work (see coresidency_probe)
    F_TEST_SKEW = 512,         // test only: members publish after a member- and row-dependent delay
};

// Statistics exchanged per stage (slot stride of the exchange workspace).
constexpr int q_of(int op) {
    return op == OP_PEARSON_BWD ? 5 : (op == OP_SMXL_BWD || op == OP_WVAR_BWD) ? 3 : 2;
}
// Operators with two resident input tensors / two output tensors.
constexpr bool two_in(int op) {
    return (op >= OP_SOFTMAX_BWD && op <= OP_SMXL_BWD) || op == OP_PEARSON_BWD || op == OP_WVAR_BWD;
}
constexpr bool two_out(int op) { return op == OP_PEARSON_BWD || op == OP_WVAR_BWD; }
constexpr bool is_quant(int op) { return op == OP_QUANT_I8 || op == OP_QUANT_F8; }
constexpr bool byte_out(int op) { return is_quant(op) || op == OP_LNQ_FWD; }  // one-byte codes out

// Register-resident slice sizes: vectors (16 bytes) per thread per tensor.
constexpr int kVpts[] = {1, 2, 4, 8, 12, 16, 24, 32};
constexpr int kNumVpts = 8;
// Slices beyond the register file: 32 vectors per thread in registers plus
// L = vpt - 32 in LDS (4 KiB per vector x 256 threads): 48 (64 KiB of LDS,
// two workgroups per CU) and 68 (144 KiB: one workgroup per CU, whose LDS also
// holds the reduction and exchange buffers; slots in multiples of 4).  Built for
// the single-input forward operators with FP32 / BF16 rows, whose register
// slices end at 32 vectors.
constexpr int kLdsVpts[] = {48, 68};
constexpr int kRegVptMax = 32;
constexpr bool lds_capable(int op, int dt) {
    return (op == OP_SOFTMAX_FWD || op == OP_LN_FWD || op == OP_RMS_FWD) && (dt == DT_F32 || dt == DT_BF16);
}
// LDS vectors per thread of a slice bucket (0: registers only).
constexpr int lds_vpt(int vpt) { return vpt > kRegVptMax ? vpt - kRegVptMax : 0; }
// Rows per workgroup of the multi-row LayerNorm / RMSNorm forward: a
// workgroup holds the same slice of R rows at once (R x VPT vectors per
// thread), so each gamma / beta vector is loaded once per R rows and one
// exchange round carries the statistics of all R rows.  Built for slices of
// up to kMrVptMax vectors per thread.
constexpr int kMrRows[] = {2, 4};
constexpr int kMrVptMax = 8;
constexpr bool multirow_capable(int op) { return op == OP_LN_FWD || op == OP_RMS_FWD; }
// Instances built: FP8 rows decode 16 values per vector, so FP8 holds at most
// 8 vectors per thread over its R rows (beyond that the registers spill).
constexpr bool multirow_fits(int dt, int vpt, int rows) {
    return vpt <= kMrVptMax && (dt != DT_FP8 || vpt * rows <= 8);
}
// Largest instantiated vectors-per-thread for (op, dtype): bounded by the
// register file (data of one or two tensors, plus FP32 dgamma/dbeta column
// partials for normalisation backward).
constexpr int max_vpt(int op, int dt) {
    return (op <= OP_RMS_FWD || op == OP_QUANT_I8 || op == OP_QUANT_F8 || op == OP_LNQ_FWD) ? (dt == DT_FP8 ? 16 : 32)
         : (op == OP_SOFTMAX_BWD || op == OP_SMXL_BWD || op == OP_PEARSON_BWD || op == OP_WVAR_BWD) ? 16
         : op == OP_LN_BWD ? (dt == DT_F32 ? 8 : dt == DT_BF16 ? 4 : 2)
         : (dt == DT_F32 ? 8 : dt == DT_BF16 ? 8 : 4);
}

// Measured exceptions to the register model below: LayerNorm backward
// instances that run faster on MI355X with one more co-resident workgroup per
// CU than fit their registers (the compiler spills a little): BF16 with 4
// vectors per thread 14% faster at 3, FP8 with 2 vectors 17% faster at 3, FP32
// with 4 vectors 6% faster at 4 (M = 2048, N = 131072).  For every other
// instance measured, more workgroups with heavier spilling, or fewer without
// spilling, was slower.
constexpr int wave_override(int op, int dt, int vpt) {
    return op != OP_LN_BWD ? 0
         : (dt == DT_BF16 && vpt == 4) ? 3
         : (dt == DT_FP8 && vpt == 2) ? 3
         : (dt == DT_F32 && vpt == 4) ? 4 : 0;
}

struct RowArgs {
    const void *in0;   // x (forward, norm backward) or y (softmax backward)
    const void *in1;   // dy (backward); y (Pearson); w (weighted variance)
    void *out;         // y (forward), dx (backward) or the codes (quantisation)
    void *out1;        // second output: dy (Pearson), dw (weighted variance)
    int64_t ld0, ld1, ldo, ldo1;
    const float *rowg; // per-row upstream gradient dr / dv (Pearson, weighted variance)
    const float *s0, *s1;  // FP8 per-row input scales
    float *so;             // FP8 per-row output scales
    const float *gamma, *beta;
    const float *mean_in, *rstd_in;  // saved statistics (norm backward)
    float *mean_out, *rstd_out;      // statistics outputs (forward; two-pass recompute)
    float *colpart;                  // [groups][ncp][N] dgamma/dbeta partials
    unsigned long long *slots;       // split-row exchange slots
    unsigned *errflag;               // exchange-timeout flag (holds the epoch)
    int64_t M, N;
    int64_t chunk;     // elements per slice (multiple of the vector width)
    int k;             // split factor
    int qs;            // slot stride: statistics per stage of this operator
    int groups;        // concurrent row groups = grid / k
    unsigned epoch;    // exchange epoch of this launch (never 0); 0: read it from epoch_ptr
    const unsigned *epoch_ptr;  // device-side epoch (launches captured into a graph)
    unsigned spin_limit;
    float eps;
    int flags;
};

}  // namespace credit
