// kargs.h -- kernel argument block and enumerations shared by the host
// library and the gfx950 kernels.
#pragma once
#include <stdint.h>

namespace credit {

enum KOp { OP_SOFTMAX_FWD = 0, OP_LN_FWD = 1, OP_RMS_FWD = 2, OP_SOFTMAX_BWD = 3, OP_LN_BWD = 4, OP_RMS_BWD = 5 };
enum KDt { DT_F32 = 0, DT_BF16 = 1, DT_FP8 = 2 };

constexpr int kMaxStages = 3;  // statistics stages per row (recompute, main, amax)
constexpr int kMaxQ = 2;       // statistics per stage
constexpr int kMaxK = 32;      // largest split factor
constexpr int kBlockThreads = 256;  // threads per row-resident / split-row workgroup

enum KFlags {
    F_ALIGN0 = 1,              // rows of in0 start 16-byte aligned
    F_ALIGN1 = 2,              // rows of in1 start 16-byte aligned
    F_ALIGNO = 4,              // rows of out start 16-byte aligned
    F_XCD = 8,                 // XCD-aware member mapping (grid % 8 == 0)
    F_RECOMPUTE = 16,          // norm backward: recompute mean/rstd from x
    F_TEST_DROP_PUBLISH = 32,  // test only: member 1 never publishes
    F_ALIGNP = 64,             // gamma / beta 16-byte aligned
};

// Register-resident slice sizes: vectors (16 bytes) per thread per tensor.
constexpr int kVpts[] = {1, 2, 4, 8, 12, 16, 24, 32};
constexpr int kNumVpts = 8;
// Largest instantiated vectors-per-thread for (op, dtype): bounded by the
// register file (data of one or two tensors, plus FP32 dgamma/dbeta column
// partials for normalisation backward).
constexpr int max_vpt(int op, int dt) {
    return op <= OP_RMS_FWD ? (dt == DT_FP8 ? 16 : 32)
         : op == OP_SOFTMAX_BWD ? 16
         : op == OP_LN_BWD ? (dt == DT_F32 ? 8 : dt == DT_BF16 ? 4 : 2)
         : (dt == DT_F32 ? 8 : dt == DT_BF16 ? 8 : 4);
}

struct RowArgs {
    const void *in0;   // x (forward, norm backward) or y (softmax backward)
    const void *in1;   // dy (backward)
    void *out;         // y (forward) or dx (backward)
    int64_t ld0, ld1, ldo;
    const float *s0, *s1;  // FP8 per-row input scales
    float *so;             // FP8 per-row output scales
    const float *gamma, *beta;
    const float *mean_in, *rstd_in;  // saved statistics (norm backward)
    float *mean_out, *rstd_out;      // statistics outputs (forward; two-pass recompute)
    float *colpart;                  // [groups][ncp][N] dgamma/dbeta partials
    unsigned long long *slots;       // split-row exchange slots
    unsigned *errflag;               // exchange-timeout flag (holds the epoch)
    const void *safe;                // 16 readable bytes (target of masked-off vector loads)
    int64_t M, N;
    int64_t chunk;     // elements per slice (multiple of the vector width)
    int k;             // split factor
    int groups;        // concurrent row groups = grid / k
    unsigned epoch;    // exchange epoch of this launch (never 0)
    unsigned spin_limit;
    float eps;
    int flags;
};

}  // namespace credit
