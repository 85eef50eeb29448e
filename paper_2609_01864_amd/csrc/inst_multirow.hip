// Kernel instantiations of the multi-row LayerNorm / RMSNorm forward: every
// (operator, dtype, vectors-per-thread, rows per workgroup) that multirow_fits.
#include "multirow.h"

namespace credit {

#define CREDIT_M(OP, DT, V, R) \
    if (multirow_fits(DT, V, R) && op == OP && dt == DT && vpt == V && rows == R) \
        return (const void *)&k_multirow<OP, DT, (multirow_fits(DT, V, R) ? V : 1), R>;
#define CREDIT_MV(OP, DT, R) CREDIT_M(OP, DT, 1, R) CREDIT_M(OP, DT, 2, R) CREDIT_M(OP, DT, 4, R) CREDIT_M(OP, DT, 8, R)
#define CREDIT_MD(OP, R) CREDIT_MV(OP, DT_F32, R) CREDIT_MV(OP, DT_BF16, R) CREDIT_MV(OP, DT_FP8, R)

const void *multirow_kernel(int op, int dt, int vpt, int rows) {
    CREDIT_MD(OP_LN_FWD, 2) CREDIT_MD(OP_LN_FWD, 4)
    CREDIT_MD(OP_RMS_FWD, 2) CREDIT_MD(OP_RMS_FWD, 4)
    return nullptr;
}

}  // namespace credit
