// Kernel instantiations for OP_RMS_FWD with FP8 rows: the register-resident /
// split-row kernel for every vectors-per-thread within the register budget.
// Kept apart from the FP32 / BF16 instances so that it builds with the default
// instruction schedule (with the ILP-maximising one the 12- and 16-vector
// slices spill to private memory).
#include "resident.h"

namespace credit {

#define CREDIT_R8(V) \
    if (max_vpt(OP_RMS_FWD, DT_FP8) >= V && vpt == V) \
        return (const void *)&k_resident<OP_RMS_FWD, DT_FP8, (max_vpt(OP_RMS_FWD, DT_FP8) >= V ? V : 1)>;

const void *resident_kernel_rms_fwd_fp8(int vpt) {
    CREDIT_R8(1) CREDIT_R8(2) CREDIT_R8(4) CREDIT_R8(8)
    CREDIT_R8(12) CREDIT_R8(16) CREDIT_R8(24) CREDIT_R8(32)
    return nullptr;
}

}  // namespace credit
