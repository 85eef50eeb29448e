// Kernel instantiations for OP_LN_FWD: the register-resident / split-row kernel
// for every (dtype, vectors-per-thread) within the register budget (FP8 rows in
// inst_ln_fwd_fp8.hip, built with the default instruction schedule), and the
// two-pass kernel for 256- and 1024-thread workgroups (FP8 at 1024 threads
// keeps 2 vectors in flight per thread: its decoded values then fit the 128
// registers a 1024-thread workgroup allows, without spilling).
#include "resident.h"
#include "twopass.h"

namespace credit {

#define CREDIT_R(DT, V) \
    if (max_vpt(OP_LN_FWD, DT) >= V && dt == DT && vpt == V) return (const void *)&k_resident<OP_LN_FWD, (max_vpt(OP_LN_FWD, DT) >= V ? DT : DT_F32), (max_vpt(OP_LN_FWD, DT) >= V ? V : 1)>;
#define CREDIT_RV(DT) \
    CREDIT_R(DT, 1) CREDIT_R(DT, 2) CREDIT_R(DT, 4) CREDIT_R(DT, 8) \
    CREDIT_R(DT, 12) CREDIT_R(DT, 16) CREDIT_R(DT, 24) CREDIT_R(DT, 32)

// slices beyond the register file: 32 vectors in registers, the rest in LDS
#define CREDIT_RL(DT, V) \
    if (dt == DT && vpt == V) return (const void *)&k_resident<OP_LN_FWD, DT, kRegVptMax, V - kRegVptMax>;

const void *resident_kernel_ln_fwd_fp8(int vpt);  // inst_ln_fwd_fp8.hip (default schedule)

const void *resident_kernel_ln_fwd(int dt, int vpt) {
    CREDIT_RV(DT_F32)
    CREDIT_RV(DT_BF16)
    if (dt == DT_FP8) return resident_kernel_ln_fwd_fp8(vpt);
    CREDIT_RL(DT_F32, 48) CREDIT_RL(DT_F32, 68)
    CREDIT_RL(DT_BF16, 48) CREDIT_RL(DT_BF16, 68)
    return nullptr;
}

const void *twopass_kernel_ln_fwd(int dt, int block) {
    if (block == 256) {
        if (dt == DT_F32) return (const void *)&k_twopass<OP_LN_FWD, DT_F32, 256, 4>;
        if (dt == DT_BF16) return (const void *)&k_twopass<OP_LN_FWD, DT_BF16, 256, 4>;
        if (dt == DT_FP8) return (const void *)&k_twopass<OP_LN_FWD, DT_FP8, 256, 4>;
    } else if (block == 1024) {
        if (dt == DT_F32) return (const void *)&k_twopass<OP_LN_FWD, DT_F32, 1024, 4>;
        if (dt == DT_BF16) return (const void *)&k_twopass<OP_LN_FWD, DT_BF16, 1024, 4>;
        if (dt == DT_FP8) return (const void *)&k_twopass<OP_LN_FWD, DT_FP8, 1024, 2>;
    }
    return nullptr;
}

}  // namespace credit
