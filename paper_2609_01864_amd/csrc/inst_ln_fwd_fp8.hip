// Kernel instantiations for OP_LN_FWD with FP8 rows: the register-resident /
// split-row kernel for every vectors-per-thread within the register budget.
// Kept apart from the FP32 / BF16 instances so that it builds with the default
// instruction schedule (1-2% faster for these than the ILP-maximising one).
#include "resident.h"

namespace credit {

#define CREDIT_R8(V) \
    if (max_vpt(OP_LN_FWD, DT_FP8) >= V && vpt == V) \
        return (const void *)&k_resident<OP_LN_FWD, DT_FP8, (max_vpt(OP_LN_FWD, DT_FP8) >= V ? V : 1)>;

const void *resident_kernel_ln_fwd_fp8(int vpt) {
    CREDIT_R8(1) CREDIT_R8(2) CREDIT_R8(4) CREDIT_R8(8)
    CREDIT_R8(12) CREDIT_R8(16) CREDIT_R8(24) CREDIT_R8(32)
    return nullptr;
}

}  // namespace credit
