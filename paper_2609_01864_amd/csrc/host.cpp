// host.cpp -- the C ABI of libcredit: validation, plan resolution (legality,
// persistent-grid geometry, workspace layout), launches, timing, the plan
// selectors of Sec. III-D and the learned selector's training driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/credit.h"
#include "kargs.h"

namespace credit {
const void *resident_kernel_softmax_fwd(int, int);
const void *resident_kernel_ln_fwd(int, int);
const void *multirow_kernel(int, int, int, int);
const void *resident_kernel_rms_fwd(int, int);
const void *resident_kernel_softmax_bwd(int, int);
const void *resident_kernel_ln_bwd(int, int);
const void *resident_kernel_rms_bwd(int, int);
const void *twopass_kernel_softmax_fwd(int, int);
const void *twopass_kernel_ln_fwd(int, int);
const void *twopass_kernel_rms_fwd(int, int);
const void *twopass_kernel_softmax_bwd(int, int);
const void *twopass_kernel_ln_bwd(int, int);
const void *twopass_kernel_rms_bwd(int, int);
const void *resident_kernel_smxl_bwd(int, int);
const void *resident_kernel_quant_i8(int, int);
const void *resident_kernel_quant_f8(int, int);
const void *resident_kernel_pearson_bwd(int, int);
const void *resident_kernel_wvar_bwd(int, int);
const void *twopass_kernel_smxl_bwd(int, int);
const void *twopass_kernel_quant_i8(int, int);
const void *twopass_kernel_quant_f8(int, int);
const void *twopass_kernel_pearson_bwd(int, int);
const void *twopass_kernel_wvar_bwd(int, int);
const void *resident_kernel_lnq_fwd(int, int);
const void *twopass_kernel_lnq_fwd(int, int);
const void *colreduce_kernel();
const void *colreduce1_kernel();
const void *colstats_kernel(int, bool);
const void *control_kernel();
const void *zero_kernel();
const void *epoch_bump_kernel();
const void *flush_kernel();
const void *fill_kernel();
const void *copy_kernel();
const void *encode_kernel(int);
const void *decode_kernel(int);
const void *mlp_kernel(int);
const void *probe_kernel(int);
}  // namespace credit

using namespace credit;

namespace {

constexpr int kSplitKs[5] = {2, 4, 8, 16, 32};
constexpr size_t kFlushBytes = (size_t)512 << 20;
constexpr double kClockHz = 2.4e9;      // MI355X peak engine clock
constexpr double kSlotBytes = 8.0;      // one exchange slot word
constexpr double kSlotRate = 64.0;      // slot-store issue rate, bytes per cycle per CU
constexpr int kDefaultCUs = 256;
constexpr int kLdsBytes = 163840;
constexpr int kMlpParams = CREDIT_NUM_FEATURES * CREDIT_MLP_HIDDEN + CREDIT_MLP_HIDDEN +
                           CREDIT_MLP_HIDDEN * CREDIT_MLP_HIDDEN + CREDIT_MLP_HIDDEN +
                           CREDIT_NUM_PLANS * CREDIT_MLP_HIDDEN + CREDIT_NUM_PLANS;

std::atomic<uint32_t> g_epoch{1};
// Host-chosen exchange epochs keep the top bit clear (graph-recorded launches
// use device-side epochs with it set) and are never 0.
uint32_t next_epoch() {
    uint32_t e = g_epoch.fetch_add(1) & 0x7fffffffu;
    while (e == 0) e = g_epoch.fetch_add(1) & 0x7fffffffu;
    return e;
}

// Public (operator, direction) -> kernel operator; -1 for a pair that does
// not exist (e.g. a forward of the backward-only workloads).
int kop(int op, int dir) {
    if (dir != CREDIT_FWD && dir != CREDIT_BWD) return -1;
    if (op >= CREDIT_SOFTMAX && op <= CREDIT_RMSNORM) return op + 3 * dir;
    if (op == CREDIT_SOFTMAX_LOGITS && dir == CREDIT_BWD) return OP_SMXL_BWD;
    if (op == CREDIT_QUANT_INT8 && dir == CREDIT_FWD) return OP_QUANT_I8;
    if (op == CREDIT_QUANT_FP8 && dir == CREDIT_FWD) return OP_QUANT_F8;
    if (op == CREDIT_PEARSON && dir == CREDIT_BWD) return OP_PEARSON_BWD;
    if (op == CREDIT_WVAR && dir == CREDIT_BWD) return OP_WVAR_BWD;
    if (op == CREDIT_LAYERNORM_FP8_OUT && dir == CREDIT_FWD) return OP_LNQ_FWD;
    return -1;
}
// I/O dtypes an operator is built for: quantisation reads FP32 / BF16 and
// writes codes; Pearson and weighted variance take FP32 / BF16.
bool dt_ok(int k_op, int dt) {
    if (dt < CREDIT_F32 || dt > CREDIT_FP8_E4M3) return false;
    if (is_quant(k_op) || k_op == OP_PEARSON_BWD || k_op == OP_WVAR_BWD || k_op == OP_LNQ_FWD)
        return dt != CREDIT_FP8_E4M3;
    return k_op >= 0 && k_op < OP_COUNT;
}
bool core_op(int k_op) { return k_op >= OP_SOFTMAX_FWD && k_op <= OP_RMS_BWD; }
int dt_bytes(int dt) { return dt == CREDIT_F32 ? 4 : dt == CREDIT_BF16 ? 2 : 1; }
int dt_epv(int dt) { return 16 / dt_bytes(dt); }
int ncp_of(int k_op) { return k_op == OP_LN_BWD ? 2 : k_op == OP_RMS_BWD ? 1 : 0; }
bool two_inputs(int k_op) { return two_in(k_op); }
int out_bytes(int k_op, int dt) { return byte_out(k_op) ? 1 : dt_bytes(dt); }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Every slice bucket: register-only, then registers plus LDS.
constexpr int kAllVpts[] = {1, 2, 4, 8, 12, 16, 24, 32, 48, 68};
bool instance_exists(int k_op, int dt, int vpt) {
    for (int v : kVpts)
        if (v == vpt) return vpt <= max_vpt(k_op, dt);
    for (int v : kLdsVpts)
        if (v == vpt) return lds_capable(k_op, dt);
    return false;
}

const void *resident_fn(int k_op, int dt, int vpt) {
    switch (k_op) {
    case OP_SOFTMAX_FWD: return resident_kernel_softmax_fwd(dt, vpt);
    case OP_LN_FWD: return resident_kernel_ln_fwd(dt, vpt);
    case OP_RMS_FWD: return resident_kernel_rms_fwd(dt, vpt);
    case OP_SOFTMAX_BWD: return resident_kernel_softmax_bwd(dt, vpt);
    case OP_LN_BWD: return resident_kernel_ln_bwd(dt, vpt);
    case OP_RMS_BWD: return resident_kernel_rms_bwd(dt, vpt);
    case OP_SMXL_BWD: return resident_kernel_smxl_bwd(dt, vpt);
    case OP_QUANT_I8: return resident_kernel_quant_i8(dt, vpt);
    case OP_QUANT_F8: return resident_kernel_quant_f8(dt, vpt);
    case OP_PEARSON_BWD: return resident_kernel_pearson_bwd(dt, vpt);
    case OP_WVAR_BWD: return resident_kernel_wvar_bwd(dt, vpt);
    case OP_LNQ_FWD: return resident_kernel_lnq_fwd(dt, vpt);
    }
    return nullptr;
}
// The row-resident / split-row instance of (op, dtype, vectors per thread)
// that holds `rows` rows per workgroup (1: the single-row kernel).
const void *instance_fn(int k_op, int dt, int vpt, int rows) {
    if (rows <= 1) return resident_fn(k_op, dt, vpt);
    if (!multirow_capable(k_op) || !multirow_fits(dt, vpt, rows)) return nullptr;
    return multirow_kernel(k_op, dt, vpt, rows);
}
bool multirow_exists(int k_op, int dt, int vpt, int rows) {
    bool r = false;
    for (int x : kMrRows) r |= x == rows;
    return r && multirow_capable(k_op) && instance_exists(k_op, dt, vpt) && multirow_fits(dt, vpt, rows);
}
const void *twopass_fn(int k_op, int dt, int block) {
    switch (k_op) {
    case OP_SOFTMAX_FWD: return twopass_kernel_softmax_fwd(dt, block);
    case OP_LN_FWD: return twopass_kernel_ln_fwd(dt, block);
    case OP_RMS_FWD: return twopass_kernel_rms_fwd(dt, block);
    case OP_SOFTMAX_BWD: return twopass_kernel_softmax_bwd(dt, block);
    case OP_LN_BWD: return twopass_kernel_ln_bwd(dt, block);
    case OP_RMS_BWD: return twopass_kernel_rms_bwd(dt, block);
    case OP_SMXL_BWD: return twopass_kernel_smxl_bwd(dt, block);
    case OP_QUANT_I8: return twopass_kernel_quant_i8(dt, block);
    case OP_QUANT_F8: return twopass_kernel_quant_f8(dt, block);
    case OP_PEARSON_BWD: return twopass_kernel_pearson_bwd(dt, block);
    case OP_WVAR_BWD: return twopass_kernel_wvar_bwd(dt, block);
    case OP_LNQ_FWD: return twopass_kernel_lnq_fwd(dt, block);
    }
    return nullptr;
}

// Host copy of the kernels' register model: waves per SIMD a resident kernel
// is compiled for (used when no device is available to ask).
int model_waves(int k_op, int dt, int vpt) {
    if (vpt > kRegVptMax) {  // registers of a 32-vector slice; LDS of the rest
        const int lds = lds_vpt(vpt) * kBlockThreads * 16 + 1024;
        return std::max(1, std::min(model_waves(k_op, dt, kRegVptMax), kLdsBytes / lds));
    }
    int data = vpt * 4 * (two_inputs(k_op) ? 2 : 1) + ncp_of(k_op) * vpt * dt_epv(dt);
    const bool f8o = (dt == CREDIT_FP8_E4M3 && (k_op == OP_LN_FWD || k_op == OP_RMS_FWD)) || k_op == OP_LNQ_FWD;
    if (f8o && vpt * dt_epv(dt) <= kYcMax) data += vpt * dt_epv(dt);  // y kept across the amax stage
    if (k_op == OP_SOFTMAX_FWD && dt == CREDIT_FP8_E4M3 && vpt * dt_epv(dt) <= kEcMax)
        data += vpt * dt_epv(dt);  // decoded values, then exponentials, kept across the passes
    if ((k_op == OP_LN_BWD || k_op == OP_RMS_BWD) && dt == CREDIT_BF16 && vpt <= 2)
        data += vpt * dt_epv(dt);  // g = dy * gamma kept between the passes
    int work = 64 + (dt == CREDIT_FP8_E4M3 || k_op == OP_LNQ_FWD ? 32 : 0) +
               (k_op == OP_SOFTMAX_FWD || k_op == OP_SOFTMAX_BWD ? 0 : 16);
    int w = 512 / (data + work);
    if (int ov = wave_override(k_op, dt, vpt)) return ov;
    return std::max(1, std::min(8, w));
}
// The same for the multi-row forward kernel (rows > 1).
int model_waves(int k_op, int dt, int vpt, int rows) {
    if (rows <= 1) return model_waves(k_op, dt, vpt);
    const int data = rows * vpt * 4;
    const int work = 80 + (dt == CREDIT_FP8_E4M3 ? (k_op == OP_LN_FWD ? 64 : 32) : 0) + 4 * rows;
    return std::max(1, std::min(8, 512 / (data + work)));
}

// Number of exchange stages of a row (for the control kernel and the model).
int stages_of(int k_op, int dt, bool recompute) {
    int L = 1;
    if ((dt == CREDIT_FP8_E4M3 && k_op != OP_SOFTMAX_FWD && !is_quant(k_op)) || k_op == OP_LNQ_FWD) L += 1;
    if (recompute && (k_op == OP_LN_BWD || k_op == OP_RMS_BWD)) L += 1;
    return L;
}

struct Launch {
    int variant = 0, k = 1;
    const void *fn = nullptr;
    int grid = 0, block = 0, vpt = 0, groups = 0, per_cu = 0;
    int rows = 1;  // rows per workgroup (multi-row norm forward when > 1)
    size_t shmem = 0;
    int64_t chunk = 0;
    bool xcd = false;
    int parts = 0, rowblocks = 0;  // dgamma/dbeta partial rows
    int slices = 0;                // first-level column-reduction slices (0: one level)
    size_t off_slots = 0, off_colpart = 0, off_stats = 0, off_colsum = 0, ws_bytes = 0;
};

}  // namespace

// Device scratch of the allocation-free entry point
// (credit_layernorm_fwd_noalloc): split-row exchange slots in place of a
// caller's workspace.  One copy per device, kept until the process ends and
// shared by every call on that device.  Host code never hands `scratch`
// itself to a kernel: each handle takes the array's address on its device
// with hipGetSymbolAddress when it is created.
constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct credit_handle_s {
    int device = 0;
    char *scratch_dev = nullptr;  // this device's copy of `scratch`
    int cus = kDefaultCUs;
    std::string arch;
    hipStream_t stream = nullptr;  // timing stream
    unsigned *errflag = nullptr;
    credit_selector_t selector = CREDIT_SEL_FIXED;
    bool selector_set = false;
    bool force_set = false;  // CREDIT_FORCE_PLAN: used for plan == NULL where legal
    credit_plan_t force_plan{CREDIT_TWO_PASS, 1};
    int64_t spin_limit = 1 << 22;
    bool drop_publish = false;
    bool skew = false;  // test only: members publish out of step
    // device calibration of the analytic model (the MI355X analogue of the
    // paper's primitive table), filled by credit_probe_primitives; until then
    // the peak clock and nominal rates
    struct {
        bool probed = false;
        double clock_hz = kClockHz;
        double slot_bpc = kSlotRate;     // bytes per cycle of one workgroup's stores
        double lds_read_bpc = kSlotRate;  // bytes per cycle of one workgroup's LDS reads
    } cal;
    int64_t max_groups = 0;
    int rows_opt = 0;  // rows per workgroup of norm-forward plans (0: the library's rule)
    // CREDIT_CHECKED: every operator call waits for its launches and reports
    // an expired exchange wait itself; CREDIT_LOG: one JSON line per call
    bool checked = false;
    FILE *log = nullptr;
    bool log_owned = false;
    // private memory (bytes per lane) of the row-resident / split-row
    // instances, and for those that use it the workgroups per CU verified
    // co-resident at handle creation (0: none)
    std::map<const void *, size_t> scratch;
    std::map<const void *, int> coresident;
    std::recursive_mutex lock;
    std::map<const void *, int> occ_cache;
    std::map<std::tuple<int, int, int, int64_t, int64_t, int>, credit_plan_t> plan_cache;
    // timing arena
    char *arena = nullptr;
    size_t arena_bytes = 0;
    char *flushbuf = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    float copy_gbps = 0.f;
    std::tuple<int, int, int64_t, int64_t> prepared{-1, -1, -1, -1};  // inputs currently filled
    // learned selector; `inf` holds the network and one row of activations on
    // the device, allocated when a model is set, so that picking a plan in an
    // operator call allocates nothing
    bool has_model = false;
    float *inf = nullptr;
    std::vector<float> params = std::vector<float>(kMlpParams, 0.f);
    float mu[CREDIT_NUM_FEATURES] = {0};
    float sd[CREDIT_NUM_FEATURES] = {0};
    // Adam state of the training that produced `params`: first and second
    // moments and the steps taken (0: none, the moments are zero), kept so
    // that training resumes, also from a saved model
    std::vector<float> adam_m = std::vector<float>(kMlpParams, 0.f);
    std::vector<float> adam_v = std::vector<float>(kMlpParams, 0.f);
    int64_t adam_t = 0;
};

namespace {

int occupancy(credit_handle_t h, const void *fn, int block, size_t shmem) {
    if (!h) return -1;
    auto it = h->occ_cache.find(fn);
    if (it != h->occ_cache.end() && shmem == 0) return it->second;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, block, shmem) != hipSuccess) return 0;
    if (shmem == 0) h->occ_cache[fn] = n;
    return n;
}

// The dgamma / dbeta partial rows are summed in two levels when there are
// many: slices of kColPer partial rows each in parallel, then the slices, so
// the reduction has parallelism over rows as well as columns (fixed order).
constexpr int kColPer = 16;
size_t colsum_layout(Launch &L, int ncp, int64_t N, size_t off) {
    L.slices = L.parts > 2 * kColPer ? (L.parts + kColPer - 1) / kColPer : 0;
    if (!L.slices) return off;
    L.off_colsum = off;
    return align256(off + (size_t)L.slices * ncp * N * 4);
}

// Rows per workgroup of a resident / split plan (Launch::rows): the option
// when set, else the library's rule, from back-to-back timings on MI355X
// (M = 1024..16384): two rows per workgroup where one exchange round per two
// rows pays -- RMSNorm (every dtype) and BF16 LayerNorm at k >= 16 (RMSNorm
// FP32 N = 131072 at k = 16: 199 -> 188 us, BF16 N = 262144 at k = 32:
// 1206 -> 871 us) -- and for row-resident plans with enough rows to fill every
// row-group slot twice over (FP32 LayerNorm 16384 x 4096: 106 -> 99 us).
// Elsewhere one row: with fewer rows than slots two-row blocks leave
// workgroups idle, and FP32 / FP8 LayerNorm at k = 16 lost 3% / 16% (FP8
// keeps no normalised row across its amax stage here, so it reads gamma and
// beta twice per row block).
int rows_for(credit_handle_t h, int k_op, int dt, int vpt, int64_t M, int k, int64_t slots1) {
    int want = h ? h->rows_opt : 0;
    if (want == 0) {
        want = 1;
        if (k >= 16 && (k_op == OP_RMS_FWD || (k_op == OP_LN_FWD && dt == CREDIT_BF16))) want = 2;
        if (k == 1 && dt != CREDIT_FP8_E4M3 && M >= 2 * slots1) want = 2;
    }
    if (want <= 1 || M < 2 || !multirow_exists(k_op, dt, vpt, want)) return 1;
    return want;
}

// Resolves a plan into launch geometry and workspace layout.  Returns
// CREDIT_ERR_UNSUPPORTED when the plan is illegal for the shape.
credit_status_t resolve(credit_handle_t h, int k_op, int dt, int64_t M, int64_t N, credit_plan_t plan,
                        bool recompute, Launch &L) {
    L = Launch();
    L.variant = plan.variant;
    const int epv = dt_epv(dt);
    const int64_t nvec = (N + epv - 1) / epv;
    const int cus = h ? h->cus : kDefaultCUs;
    const int ncp = ncp_of(k_op);
    if (plan.variant == CREDIT_TWO_PASS) {
        if (plan.k != 1) return CREDIT_ERR_UNSUPPORTED;
        L.k = 1;
        L.block = nvec >= 4096 ? 1024 : 256;
        L.fn = twopass_fn(k_op, dt, L.block);
        if (!L.fn) return CREDIT_ERR_UNSUPPORTED;
        int occ = h ? occupancy(h, L.fn, L.block, 0) : std::max(1, 2048 / L.block);
        if (occ <= 0) return CREDIT_ERR_HIP;
        L.per_cu = occ;
        L.grid = (int)std::min<int64_t>(M, (int64_t)occ * cus);
        L.groups = L.grid;
        size_t off = 256;  // error/reserved header
        if (ncp) {
            int64_t colblocks = (nvec + 255) / 256;
            L.rowblocks = (int)std::max<int64_t>(1, std::min<int64_t>(M, (2048 + colblocks - 1) / colblocks));
            L.parts = L.rowblocks;
            L.off_colpart = off;
            off = align256(off + (size_t)L.rowblocks * ncp * N * 4);
            off = colsum_layout(L, ncp, N, off);
            L.off_stats = off;
            off = align256(off + (size_t)2 * M * 4);
        }
        L.ws_bytes = off;
        return CREDIT_OK;
    }
    int k = plan.k;
    if (plan.variant == CREDIT_ROW_RESIDENT) {
        if (k != 1) return CREDIT_ERR_UNSUPPORTED;
    } else if (plan.variant == CREDIT_SPLIT_ROW) {
        bool ok = false;
        for (int kk : kSplitKs) ok |= kk == k;
        if (!ok) return CREDIT_ERR_UNSUPPORTED;
    } else {
        return CREDIT_ERR_INVALID_ARG;
    }
    L.k = k;
    const int64_t cvec = (nvec + k - 1) / k;
    const int64_t need = (cvec + kBlockThreads - 1) / kBlockThreads;
    int vpt = 0;
    for (int v : kVpts)
        if (v >= need && v <= max_vpt(k_op, dt)) { vpt = v; break; }
    if (!vpt && lds_capable(k_op, dt))  // registers plus LDS (Eq. (3) with C_res = VGPRs + LDS)
        for (int v : kLdsVpts)
            if (v >= need) { vpt = v; break; }
    if (!vpt) return CREDIT_ERR_UNSUPPORTED;  // slice exceeds register (and LDS) capacity (Eq. (3))
    L.vpt = vpt;
    L.chunk = cvec * epv;
    L.block = kBlockThreads;
    {
        // row-group slots of the one-row kernel (for the rows rule)
        const void *f1 = resident_fn(k_op, dt, vpt);
        const int occ1 = !f1 ? 0 : h ? occupancy(h, f1, kBlockThreads, 0) : model_waves(k_op, dt, vpt);
        L.rows = rows_for(h, k_op, dt, vpt, M, k, (int64_t)std::max(occ1, 1) * cus / k);
    }
    L.fn = instance_fn(k_op, dt, vpt, L.rows);
    if (!L.fn) return CREDIT_ERR_UNSUPPORTED;
    int occ = h ? occupancy(h, L.fn, L.block, 0) : model_waves(k_op, dt, vpt, L.rows);
    if (occ <= 0) return h ? CREDIT_ERR_HIP : CREDIT_ERR_UNSUPPORTED;
    if (h && k > 1) {
        // an instance that uses private memory runs split plans only at the
        // per-CU count its co-residency probe verified (dispatch of waves that
        // need private memory is also bounded by the runtime's allocation)
        auto it = h->coresident.find(L.fn);
        if (it != h->coresident.end()) occ = std::min(occ, it->second);
        if (occ <= 0) return CREDIT_ERR_UNSUPPORTED;
    }
    L.per_cu = occ;
    int64_t cap = (int64_t)occ * cus;
    int64_t gmax = cap / k;
    if (h && h->max_groups > 0) gmax = std::min<int64_t>(gmax, h->max_groups);
    if (gmax < 1) return CREDIT_ERR_UNSUPPORTED;  // k members cannot be co-resident
    const int64_t blocks = (M + L.rows - 1) / L.rows;  // row blocks of L.rows rows
    int64_t groups = std::min<int64_t>(std::max<int64_t>(blocks, 1), gmax);
    if (groups >= 8) {  // XCD-aware member mapping needs grid % 8 == 0
        groups = groups / 8 * 8;
        L.xcd = true;
    }
    L.groups = (int)groups;
    L.grid = (int)(groups * k);
    size_t off = 256;
    if (k > 1) {
        L.off_slots = off;
        off = align256(off + (size_t)blocks * kMaxStages * k * q_of(k_op) * L.rows * 8);
    }
    if (ncp) {
        L.parts = L.groups;
        L.off_colpart = off;
        off = align256(off + (size_t)L.groups * ncp * N * 4);
        off = colsum_layout(L, ncp, N, off);
    }
    L.ws_bytes = off;
    (void)recompute;
    return CREDIT_OK;
}

hipError_t launch(const void *fn, int grid, int block, size_t shmem, hipStream_t s, void **args) {
    return hipLaunchKernel(fn, dim3(grid), dim3(block), args, shmem, s);
}

// Launches whose workgroups wait for one another (split-row, the control
// kernel) need all their workgroups resident at once, and their grids fill
// the GPU.  Two of them running together on different streams could each
// hold part of the GPU and wait for slots the other holds until their bounded
// waits give up, so each one is ordered after the previous one on this
// device, whatever stream it came from: one event per device, waited on when
// the stream changes.  A launch being captured into a graph keeps the
// graph's own order (the event belongs to no capture).
struct WaitFence {
    std::mutex m;
    hipEvent_t ev = nullptr;
    hipStream_t last = nullptr;
    bool valid = false;
};

WaitFence &wait_fence(int device) {
    static WaitFence fences[64];
    return fences[device & 63];
}

hipError_t fenced_launch(int device, bool capturing, const void *fn, int grid, int block, size_t shmem,
                         hipStream_t s, void **args) {
    if (capturing) return launch(fn, grid, block, shmem, s, args);
    WaitFence &f = wait_fence(device);
    std::lock_guard<std::mutex> g(f.m);
    hipError_t e = hipSuccess;
    if (!f.ev && (e = hipEventCreateWithFlags(&f.ev, hipEventDisableTiming)) != hipSuccess) {
        f.ev = nullptr;
        return e;
    }
    if (f.valid && f.last != s && (e = hipStreamWaitEvent(s, f.ev, 0)) != hipSuccess) return e;
    if ((e = launch(fn, grid, block, shmem, s, args)) != hipSuccess) return e;
    if ((e = hipEventRecord(f.ev, s)) != hipSuccess) return e;
    f.last = s;
    f.valid = true;
    return hipSuccess;
}

hipError_t zero_words(void *p, int64_t nwords, hipStream_t s) {
    if (nwords <= 0) return hipSuccess;
    int grid = (int)std::min<int64_t>(4096, (nwords + 255) / 256);
    void *args[] = {&p, &nwords};
    return launch(zero_kernel(), grid, 256, 0, s, args);
}

bool al16(const void *p) { return ((uintptr_t)p & 15) == 0; }

struct OpCall {
    int k_op, dt;
    int64_t M, N;
    const void *in0, *in1;
    int64_t ld0, ld1;
    void *out;
    int64_t ldo;
    const float *s0, *s1;
    float *so;
    const float *gamma, *beta, *mean_in, *rstd_in;
    float *mean_out, *rstd_out;
    float *dgamma, *dbeta;
    float eps;
    void *out1;         // second output (Pearson dy, weighted-variance dw)
    int64_t ldo1;
    const float *rowg;  // per-row upstream gradient (Pearson dr, weighted-variance dv)
};

credit_status_t pick_plan(credit_handle_t h, int k_op, int dt, int64_t M, int64_t N, credit_plan_t *out, float *pred,
                          bool may_time, bool capturing);

// Issues an operator with a resolved launch on `stream`.
credit_status_t issue(credit_handle_t h, const OpCall &c, const Launch &L, void *ws, hipStream_t stream,
                      bool recompute) {
    const int B = dt_bytes(c.dt), OB = out_bytes(c.k_op, c.dt);
    RowArgs a;
    std::memset(&a, 0, sizeof(a));
    a.in0 = c.in0; a.in1 = c.in1; a.out = c.out; a.out1 = c.out1;
    a.ld0 = c.ld0; a.ld1 = c.ld1; a.ldo = c.ldo; a.ldo1 = c.ldo1;
    a.rowg = c.rowg;
    a.qs = q_of(c.k_op) * L.rows;
    a.s0 = c.s0; a.s1 = c.s1; a.so = c.so;
    a.gamma = c.gamma; a.beta = c.beta;
    a.mean_in = c.mean_in; a.rstd_in = c.rstd_in;
    a.mean_out = c.mean_out; a.rstd_out = c.rstd_out;
    a.M = c.M; a.N = c.N;
    a.eps = c.eps;
    a.errflag = h->errflag;
    a.spin_limit = (unsigned)std::min<int64_t>(h->spin_limit, 0xffffffffLL);
    int flags = 0;
    if (al16(c.in0) && (c.ld0 * B) % 16 == 0) flags |= F_ALIGN0;
    if (c.in1 && al16(c.in1) && (c.ld1 * B) % 16 == 0) flags |= F_ALIGN1;
    if (al16(c.out) && (c.ldo * OB) % 16 == 0) flags |= F_ALIGNO;
    if (c.out1 && al16(c.out1) && (c.ldo1 * B) % 16 == 0) flags |= F_ALIGNO1;
    if ((!c.gamma || al16(c.gamma)) && (!c.beta || al16(c.beta))) flags |= F_ALIGNP;
    if (recompute) flags |= F_RECOMPUTE;
    if (h->drop_publish) flags |= F_TEST_DROP_PUBLISH;
    if (h->skew) flags |= F_TEST_SKEW;
    char *w = (char *)ws;
    const int ncp = ncp_of(c.k_op);
    hipError_t e = hipSuccess;
    if (L.variant == CREDIT_TWO_PASS) {
        a.k = 1;
        a.groups = L.grid;
        a.chunk = c.N;
        if (ncp && recompute) {
            a.mean_out = (float *)(w + L.off_stats);
            a.rstd_out = a.mean_out + c.M;
        }
        a.flags = flags;
        void *args[] = {&a};
        e = launch(L.fn, L.grid, L.block, 0, stream, args);
        if (e != hipSuccess) return CREDIT_ERR_HIP;
        if (ncp && (c.dgamma || c.dbeta)) {
            RowArgs b = a;
            if (recompute) {
                b.mean_in = a.mean_out;
                b.rstd_in = a.rstd_out;
            }
            b.colpart = (float *)(w + L.off_colpart);
            int epv = dt_epv(c.dt);
            int64_t nvec = (c.N + epv - 1) / epv;
            int rb = L.rowblocks;
            void *args2[] = {&b, &rb};
            e = hipLaunchKernel(colstats_kernel(c.dt, c.k_op == OP_LN_BWD), dim3((unsigned)((nvec + 255) / 256), rb),
                                dim3(256), args2, 0, stream);
            if (e != hipSuccess) return CREDIT_ERR_HIP;
        }
    } else {
        a.k = L.k;
        a.groups = L.groups;
        a.chunk = L.chunk;
        bool capturing = false;
        if (L.k > 1) {
            a.slots = (unsigned long long *)(w + L.off_slots);
            a.epoch = next_epoch();
            // a launch being recorded into a graph would replay with this same
            // epoch and could then accept the previous replay's slot words:
            // record a bump of the device-side epoch before it instead
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return CREDIT_ERR_HIP;
            capturing = cs == hipStreamCaptureStatusActive;
            if (capturing) {
                unsigned *ctr = h->errflag + 64;  // the device epoch word of the handle
                void *bargs[] = {&ctr};
                if (launch(epoch_bump_kernel(), 1, 64, 0, stream, bargs) != hipSuccess) return CREDIT_ERR_HIP;
                a.epoch = 0;
                a.epoch_ptr = ctr;
            }
        }
        if (L.xcd) flags |= F_XCD;
        if (ncp) a.colpart = (float *)(w + L.off_colpart);
        a.flags = flags;
        void *args[] = {&a};
        e = L.k > 1 ? fenced_launch(h->device, capturing, L.fn, L.grid, L.block, 0, stream, args)
                    : launch(L.fn, L.grid, L.block, 0, stream, args);
        if (e != hipSuccess) return CREDIT_ERR_HIP;
    }
    if (ncp && (c.dgamma || c.dbeta)) {
        const float *part = (const float *)(w + L.off_colpart);
        int parts = L.parts;
        int n_cp = ncp;
        int64_t N = c.N;
        if (L.slices) {
            float *tmp = (float *)(w + L.off_colsum);
            int per = kColPer;
            void *a1[] = {&part, &parts, &n_cp, &N, &per, &tmp};
            e = hipLaunchKernel(colreduce1_kernel(), dim3((unsigned)((N + 255) / 256), (unsigned)L.slices), dim3(256),
                                a1, 0, stream);
            if (e != hipSuccess) return CREDIT_ERR_HIP;
            part = tmp;
            parts = L.slices;
        }
        float *o0 = c.dgamma, *o1 = c.dbeta;
        void *args[] = {&part, &parts, &n_cp, &N, &o0, &o1};
        e = launch(colreduce_kernel(), (int)((N + 255) / 256), 256, 0, stream, args);
        if (e != hipSuccess) return CREDIT_ERR_HIP;
    }
    return CREDIT_OK;
}

// `host_pick`: with plan == NULL and no cached plan, take the fixed rule
// (host arithmetic) instead of running the network on the device.
// Checked mode: wait for the call's launches and read the error flag, so an
// expired exchange wait is the call's own status.  A capturing stream cannot
// be waited on; its launches are checked when the graph is replayed, through
// credit_check_errors.
credit_status_t checked_wait(credit_handle_t h, hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return CREDIT_ERR_HIP;
    if (cs != hipStreamCaptureStatusNone) return CREDIT_OK;
    if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) return CREDIT_ERR_HIP;
    unsigned flag = 0;
    if (hipMemcpy(&flag, h->errflag, 4, hipMemcpyDeviceToHost) != hipSuccess) return CREDIT_ERR_HIP;
    if (flag == 0) return CREDIT_OK;
    if (hipMemset(h->errflag, 0, 4) != hipSuccess) return CREDIT_ERR_HIP;
    return CREDIT_ERR_TIMEOUT;
}

// One JSON line per operator call: the operator, the shape, the plan, whether
// the caller gave it (else the handle's selector, or CREDIT_FORCE_PLAN, chose
// it), the launch geometry and the call's status.
void log_call(credit_handle_t h, const OpCall &c, credit_plan_t p, bool given, const Launch &L,
              credit_status_t st) {
    static const char *ops[] = {"softmax_fwd", "layernorm_fwd", "rmsnorm_fwd", "softmax_bwd", "layernorm_bwd",
                                "rmsnorm_bwd", "softmax_logits_bwd", "quant_int8", "quant_fp8", "pearson_bwd",
                                "wvar_bwd", "layernorm_fwd_fp8_out"};
    static const char *dts[] = {"f32", "bf16", "fp8"};
    static const char *sels[] = {"learned", "analytic", "exhaustive", "fixed", "peak", "learned_timed"};
    const credit_selector_t sel =
        h->selector_set ? h->selector : (h->has_model ? CREDIT_SEL_LEARNED : CREDIT_SEL_FIXED);
    const bool forced = !given && h->force_set && p.variant == h->force_plan.variant && p.k == h->force_plan.k;
    std::fprintf(h->log,
                 "{\"op\": \"%s\", \"dtype\": \"%s\", \"M\": %lld, \"N\": %lld, \"plan\": [%d, %d], "
                 "\"plan_given\": %s, \"forced\": %s, \"selector\": \"%s\", \"grid\": %d, \"per_cu\": %d, "
                 "\"vpt\": %d, \"rows\": %d, \"checked\": %s, \"status\": \"%s\"}\n",
                 ops[c.k_op], dts[c.dt], (long long)c.M, (long long)c.N, (int)p.variant, (int)p.k,
                 given ? "true" : "false", forced ? "true" : "false", sels[(int)sel], L.grid, L.per_cu, L.vpt, L.rows,
                 h->checked ? "true" : "false", credit_status_string(st));
    std::fflush(h->log);
}

credit_status_t run_op(credit_handle_t h, const OpCall &c, const credit_plan_t *plan, void *ws, size_t ws_bytes,
                       void *stream, bool recompute, bool host_pick = false) {
    if (!h) return CREDIT_ERR_INVALID_ARG;
    if (c.M < 0 || c.N <= 0) return CREDIT_ERR_INVALID_ARG;
    if (!dt_ok(c.k_op, c.dt)) return CREDIT_ERR_INVALID_ARG;
    if (c.ld0 < c.N || c.ldo < c.N || (two_inputs(c.k_op) && c.ld1 < c.N)) return CREDIT_ERR_INVALID_ARG;
    if (two_out(c.k_op) && c.ldo1 < c.N) return CREDIT_ERR_INVALID_ARG;
    if (c.M == 0) {
        hipStream_t s = (hipStream_t)stream;
        if (c.dgamma && zero_words(c.dgamma, c.N, s) != hipSuccess) return CREDIT_ERR_HIP;
        if (c.dbeta && zero_words(c.dbeta, c.N, s) != hipSuccess) return CREDIT_ERR_HIP;
        return CREDIT_OK;
    }
    if (!c.in0 || !c.out || (two_inputs(c.k_op) && !c.in1)) return CREDIT_ERR_INVALID_ARG;
    if (two_out(c.k_op) && (!c.out1 || !c.rowg)) return CREDIT_ERR_INVALID_ARG;
    if (c.dt == CREDIT_FP8_E4M3) {
        if (!c.s0 || !c.so || (two_inputs(c.k_op) && !c.s1)) return CREDIT_ERR_INVALID_ARG;
    }
    if (is_quant(c.k_op) && !c.so) return CREDIT_ERR_INVALID_ARG;
    const bool norm = c.k_op == OP_LN_FWD || c.k_op == OP_RMS_FWD || c.k_op == OP_LN_BWD || c.k_op == OP_RMS_BWD ||
                      c.k_op == OP_LNQ_FWD;
    if (norm && !c.gamma) return CREDIT_ERR_INVALID_ARG;
    if ((c.k_op == OP_LN_FWD || c.k_op == OP_LNQ_FWD) && !c.beta) return CREDIT_ERR_INVALID_ARG;
    if (c.k_op == OP_LNQ_FWD && !c.so) return CREDIT_ERR_INVALID_ARG;
    if ((c.k_op == OP_LN_BWD || c.k_op == OP_RMS_BWD) && !recompute && !c.rstd_in) return CREDIT_ERR_INVALID_ARG;
    if (c.k_op == OP_LN_BWD && !recompute && !c.mean_in) return CREDIT_ERR_INVALID_ARG;
    credit_plan_t p;
    if (plan) {
        p = *plan;
    } else {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing((hipStream_t)stream, &cs) != hipSuccess) return CREDIT_ERR_HIP;
        credit_status_t st = pick_plan(h, c.k_op, c.dt, c.M, c.N, &p, nullptr, false,
                                       host_pick || cs == hipStreamCaptureStatusActive);
        if (st != CREDIT_OK) return st;
    }
    Launch L;
    std::lock_guard<std::recursive_mutex> g(h->lock);
    credit_status_t st = resolve(h, c.k_op, c.dt, c.M, c.N, p, recompute, L);
    if (st == CREDIT_OK && (!ws || ws_bytes < L.ws_bytes)) st = CREDIT_ERR_WORKSPACE;
    if (st == CREDIT_OK) st = issue(h, c, L, ws, (hipStream_t)stream, recompute);
    if (st == CREDIT_OK && h->checked) st = checked_wait(h, (hipStream_t)stream);
    if (h->log) log_call(h, c, p, plan != nullptr, L, st);
    return st;
}

// ------------------------------------------------------------ static analysis
// Byte accounting of Eq. (4) for the two-pass schedule: each statistics stage
// streams the resident inputs; the output pass streams them again and writes.
credit_workload_t workload(int k_op, int dt, bool recompute) {
    credit_workload_t w;
    std::memset(&w, 0, sizeof(w));
    const float e = (float)dt_bytes(dt);
    const int nin = two_inputs(k_op) ? 2 : 1;
    const float eo = (float)out_bytes(k_op, dt) * (two_out(k_op) ? 2.f : 1.f);  // output bytes per element
    int L = 0;
    float stage_bytes = 0.f;
    if (recompute && (k_op == OP_LN_BWD || k_op == OP_RMS_BWD)) {
        w.q[L++] = k_op == OP_LN_BWD ? 2 : 1;
        stage_bytes += e;  // reads x only
    }
    int q = (k_op == OP_SOFTMAX_FWD || k_op == OP_LN_FWD || k_op == OP_LN_BWD || k_op == OP_LNQ_FWD) ? 2 : 1;
    if (k_op == OP_SMXL_BWD || k_op == OP_WVAR_BWD) q = 3;
    if (k_op == OP_PEARSON_BWD) q = 5;
    w.q[L++] = q;
    stage_bytes += nin * e;
    if ((dt == CREDIT_FP8_E4M3 && k_op != OP_SOFTMAX_FWD && !is_quant(k_op)) || k_op == OP_LNQ_FWD) {
        w.q[L++] = 1;  // amax of the output before it can be scaled
        stage_bytes += nin * e;
    }
    w.stages = L;
    w.b_staged = nin * e + eo;
    w.b_base = stage_bytes + nin * e + eo;
    w.b_reread = w.b_base - w.b_staged;
    w.b_keep = nin * e;
    return w;
}

// Eq. (9) with MI355X terms for every split factor.  t_ctrl_us[i] is the
// control-kernel excess for kSplitKs[i].
void model_delta(credit_handle_t h, int k_op, int dt, int64_t M, int64_t N, double t_base_us, const float *t_ctrl_us,
                 float *out) {
    credit_workload_t w = workload(k_op, dt, false);
    const double t_save = t_base_us * w.b_reread / w.b_base;  // Eq. (7)
    int sumq = 0;
    for (int l = 0; l < w.stages; ++l) sumq += w.q[l];
    for (int i = 0; i < 5; ++i) {
        Launch L;
        credit_plan_t p = {CREDIT_SPLIT_ROW, kSplitKs[i]};
        if (resolve(h, k_op, dt, M, N, p, false, L) != CREDIT_OK) {
            out[i] = -INFINITY;
            continue;
        }
        // waves of row groups (Eq. (8)); a workgroup of L.rows rows exchanges
        // once per row block, with L.rows times the statistics per round
        const int64_t W = ((M + L.rows - 1) / L.rows + L.groups - 1) / L.groups;
        const double clock = h && h->cal.probed ? h->cal.clock_hz : kClockHz;
        const double slot_bpc = h && h->cal.probed ? h->cal.slot_bpc : kSlotRate;
        const double lds_bpc = h && h->cal.probed ? h->cal.lds_read_bpc : kSlotRate;
        // replay: register slots cost nothing; LDS slots are read back once per
        // pass after the load (softmax: max, sum and output; norms: statistics
        // and output) at one workgroup's LDS read rate
        const int passes = k_op == OP_SOFTMAX_FWD ? 3 : 2;
        const double t_replay = (double)W * passes * lds_vpt(L.vpt) * kBlockThreads * 16.0 / (lds_bpc * clock) * 1e6;
        const double t_deposit = 0.0;  // the deposit is the load itself (direct loads into LDS too)
        const double t_x = kSlotBytes * W * (L.k - 1) * sumq * L.rows / (clock * slot_bpc) * 1e6;
        out[i] = (float)(t_save - t_ctrl_us[i] - t_replay - t_deposit - t_x);
    }
}

// ---------------------------------------------------------------- timing
struct Bufs {
    char *in0, *in1, *out, *out1, *ws;
    float *s0, *s1, *so, *gamma, *beta, *mean, *rstd, *dgamma, *dbeta;
    size_t ws_bytes;
};

credit_status_t ensure_arena(credit_handle_t h, size_t bytes) {
    if (h->arena_bytes >= bytes && h->flushbuf) return CREDIT_OK;
    if (h->arena) (void)hipFree(h->arena);
    h->arena = nullptr;
    h->arena_bytes = 0;
    h->prepared = std::make_tuple(-1, -1, (int64_t)-1, (int64_t)-1);
    size_t want = std::max(bytes, (size_t)64 << 20);
    if (hipMalloc(&h->arena, want) != hipSuccess) {
        h->arena = nullptr;
        (void)hipGetLastError();
        return CREDIT_ERR_HIP;
    }
    h->arena_bytes = want;
    if (!h->flushbuf) {
        if (hipMalloc(&h->flushbuf, kFlushBytes) != hipSuccess) {
            h->flushbuf = nullptr;
            (void)hipGetLastError();
            return CREDIT_ERR_HIP;
        }
        if (zero_words(h->flushbuf, (int64_t)(kFlushBytes / 4), h->stream) != hipSuccess) return CREDIT_ERR_HIP;
    }
    // deterministic contents: inputs valid for every dtype, workspace zero
    int64_t nwords = (int64_t)(want / 4);
    unsigned seed = 12345u;
    int dt = CREDIT_F32;
    void *p = h->arena;
    void *args[] = {&p, &nwords, &seed, &dt};
    if (launch(fill_kernel(), 4096, 256, 0, h->stream, args) != hipSuccess) return CREDIT_ERR_HIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return CREDIT_ERR_HIP;
    return CREDIT_OK;
}

// Lays out the buffers of one operator call in the arena and fills them.
credit_status_t prepare(credit_handle_t h, int k_op, int dt, int64_t M, int64_t N, size_t ws_bytes, Bufs &b) {
    const size_t mat = align256((size_t)M * N * dt_bytes(dt));
    const size_t vecM = align256((size_t)M * 4), vecN = align256((size_t)N * 4);
    size_t total = mat * 4 + vecM * 5 + vecN * 4 + align256(ws_bytes);
    credit_status_t st = ensure_arena(h, total);
    if (st != CREDIT_OK) return st;
    char *p = h->arena;
    b.in0 = p; p += mat;
    b.in1 = p; p += mat;
    b.out = p; p += mat;
    b.out1 = p; p += mat;
    b.s0 = (float *)p; p += vecM;
    b.s1 = (float *)p; p += vecM;
    b.so = (float *)p; p += vecM;
    b.mean = (float *)p; p += vecM;
    b.rstd = (float *)p; p += vecM;
    b.gamma = (float *)p; p += vecN;
    b.beta = (float *)p; p += vecN;
    b.dgamma = (float *)p; p += vecN;
    b.dbeta = (float *)p; p += vecN;
    b.ws = p;
    b.ws_bytes = ws_bytes;
    // inputs in the dtype's format; scales / statistics as plain FP32
    auto key = std::make_tuple(k_op, dt, M, N);
    if (h->prepared != key) {
        int64_t wmat = (int64_t)(2 * mat / 4);
        unsigned seed = 7u;
        void *pin = b.in0;
        void *a1[] = {&pin, &wmat, &seed, &dt};
        if (launch(fill_kernel(), 4096, 256, 0, h->stream, a1) != hipSuccess) return CREDIT_ERR_HIP;
        h->prepared = key;
    }
    if (zero_words(b.ws, (int64_t)(align256(ws_bytes) / 4), h->stream) != hipSuccess) return CREDIT_ERR_HIP;
    return CREDIT_OK;
}

OpCall call_for(int k_op, int dt, int64_t M, int64_t N, const Bufs &b) {
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = k_op; c.dt = dt; c.M = M; c.N = N;
    c.in0 = b.in0; c.in1 = two_inputs(k_op) ? b.in1 : nullptr;
    c.ld0 = c.ld1 = c.ldo = N;
    c.out = b.out;
    c.s0 = b.s0; c.s1 = b.s1; c.so = b.so;
    c.gamma = b.gamma; c.beta = b.beta;
    c.mean_in = b.mean; c.rstd_in = b.rstd;
    c.dgamma = b.dgamma; c.dbeta = b.dbeta;
    c.eps = 1e-5f;
    if (two_out(k_op)) {
        c.out1 = b.out1;
        c.ldo1 = N;
        c.rowg = b.mean;  // any finite per-row values
    }
    return c;
}

float median(std::vector<float> v) {
    std::sort(v.begin(), v.end());
    size_t n = v.size();
    return n % 2 ? v[n / 2] : 0.5f * (v[n / 2 - 1] + v[n / 2]);
}

credit_status_t flush(credit_handle_t h) {
    const void *p = h->flushbuf;
    int64_t n = (int64_t)(kFlushBytes / 16);
    unsigned *sink = h->errflag + 32;  // never matched: the flag word stays untouched
    void *args[] = {&p, &n, &sink};
    return launch(flush_kernel(), h->cus * 8, 256, 0, h->stream, args) == hipSuccess ? CREDIT_OK : CREDIT_ERR_HIP;
}

// Spread of a set of run times: median, minimum, 90th percentile (nearest
// rank) and the median absolute deviation from the median.
credit_timing_t timing_of(std::vector<float> t) {
    credit_timing_t r;
    std::sort(t.begin(), t.end());
    const size_t n = t.size();
    r.median_us = median(t);
    r.min_us = t.front();
    r.p90_us = t[std::min(n - 1, (size_t)std::ceil(0.9 * (double)n) - 1)];
    std::vector<float> dev(n);
    for (size_t i = 0; i < n; ++i) dev[i] = std::fabs(t[i] - r.median_us);
    r.mad_us = median(dev);
    r.runs = (int32_t)n;
    return r;
}

template <class F>
credit_status_t time_median(credit_handle_t h, int reps, int do_flush, F issue_fn, float *us,
                            credit_timing_t *stats = nullptr) {
    std::vector<float> t;
    for (int r = -3; r < reps; ++r) {
        if (do_flush && flush(h) != CREDIT_OK) return CREDIT_ERR_HIP;
        if (hipEventRecord(h->ev0, h->stream) != hipSuccess) return CREDIT_ERR_HIP;
        credit_status_t st = issue_fn();
        if (st != CREDIT_OK) return st;
        if (hipEventRecord(h->ev1, h->stream) != hipSuccess) return CREDIT_ERR_HIP;
        if (hipEventSynchronize(h->ev1) != hipSuccess) return CREDIT_ERR_HIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev0, h->ev1) != hipSuccess) return CREDIT_ERR_HIP;
        if (r >= 0) t.push_back(ms * 1000.f);
    }
    *us = median(t);
    if (stats) *stats = timing_of(t);
    return CREDIT_OK;
}

credit_status_t time_plan(credit_handle_t h, int k_op, int dt, int64_t M, int64_t N, credit_plan_t p, int reps,
                          int do_flush, float *us, credit_timing_t *stats = nullptr) {
    std::lock_guard<std::recursive_mutex> g(h->lock);
    Launch L;
    credit_status_t st = resolve(h, k_op, dt, M, N, p, false, L);
    if (st != CREDIT_OK) return st;
    Bufs b;
    st = prepare(h, k_op, dt, M, N, L.ws_bytes, b);
    if (st != CREDIT_OK) return st;
    OpCall c = call_for(k_op, dt, M, N, b);
    return time_median(h, reps > 0 ? reps : 15, do_flush, [&]() { return issue(h, c, L, b.ws, h->stream, false); }, us,
                       stats);
}

credit_status_t time_control(credit_handle_t h, int k_op, int dt, int64_t M, int64_t N, int k, int reps, float *us) {
    std::lock_guard<std::recursive_mutex> g(h->lock);
    Launch L;
    credit_plan_t p = {k == 1 ? CREDIT_ROW_RESIDENT : CREDIT_SPLIT_ROW, k};
    credit_status_t st = resolve(h, k_op, dt, M, N, p, false, L);
    if (st != CREDIT_OK && k == 1) {
        p = {CREDIT_TWO_PASS, 1};
        st = resolve(h, k_op, dt, M, N, p, false, L);
        if (st == CREDIT_OK) {  // one-workgroup control at the two-pass grid, 256 threads
            L.block = kBlockThreads;
            L.groups = L.grid;
        }
    }
    if (st != CREDIT_OK) return st;
    // pin the control kernel to the same workgroups per CU
    size_t shmem = (size_t)(kLdsBytes / std::max(1, L.per_cu)) - 1024;
    if (occupancy(h, control_kernel(), kBlockThreads, shmem) > L.per_cu) shmem += 512;
    // the control kernel touches no row data: only a zeroed workspace for its slots
    st = ensure_arena(h, align256(L.ws_bytes));
    if (st != CREDIT_OK) return st;
    char *ws = h->arena + h->arena_bytes - align256(L.ws_bytes);
    if (zero_words(ws, (int64_t)(align256(L.ws_bytes) / 4), h->stream) != hipSuccess) return CREDIT_ERR_HIP;
    h->prepared = std::make_tuple(-1, -1, (int64_t)-1, (int64_t)-1);  // may overlap prepared inputs
    RowArgs a;
    std::memset(&a, 0, sizeof(a));
    a.M = (M + L.rows - 1) / L.rows;  // one exchange round per row block
    a.N = N; a.k = L.k; a.groups = L.groups;
    a.qs = q_of(k_op);
    a.slots = (unsigned long long *)(ws + L.off_slots);
    a.errflag = h->errflag;
    a.spin_limit = (unsigned)std::min<int64_t>(h->spin_limit, 0xffffffffLL);
    int stages = stages_of(k_op, dt, false);
    return time_median(h, reps > 0 ? reps : 15, 0,
                       [&]() {
                           a.epoch = next_epoch();
                           a.flags = L.xcd ? F_XCD : 0;
                           void *args[] = {&a, &stages};
                           return fenced_launch(h->device, false, control_kernel(), L.grid, kBlockThreads, shmem,
                                                h->stream, args) == hipSuccess
                                      ? CREDIT_OK
                                      : CREDIT_ERR_HIP;
                       },
                       us);
}

credit_status_t copy_bw(credit_handle_t h, size_t bytes, int reps, float *gbps) {
    std::lock_guard<std::recursive_mutex> g(h->lock);
    bytes = bytes / 64 * 64;
    credit_status_t st = ensure_arena(h, 2 * bytes);
    if (st != CREDIT_OK) return st;
    const void *src = h->arena;
    void *dst = h->arena + bytes;
    int64_t n = (int64_t)(bytes / 16);
    int grid = (int)((n + 255) / 256);
    float us = 0.f;
    st = time_median(h, reps > 0 ? reps : 15, 0,
                     [&]() {
                         void *args[] = {&src, &dst, &n};
                         return launch(copy_kernel(), grid, 256, 0, h->stream, args) == hipSuccess ? CREDIT_OK
                                                                                                  : CREDIT_ERR_HIP;
                     },
                     &us);
    if (st != CREDIT_OK) return st;
    *gbps = (float)(2.0 * bytes / (us * 1e-6) / 1e9);
    return CREDIT_OK;
}

// -------------------------------------------------------------- selectors
bool plan_ok(credit_handle_t h, int k_op, int dt, int64_t M, int64_t N, credit_plan_t p) {
    Launch L;
    return resolve(h, k_op, dt, M, N, p, false, L) == CREDIT_OK;
}

credit_plan_t class_plan(int c) {
    if (c == 0) return {CREDIT_TWO_PASS, 1};
    if (c == 1) return {CREDIT_ROW_RESIDENT, 1};
    return {CREDIT_SPLIT_ROW, kSplitKs[c - 2]};
}

credit_plan_t fixed_rule(credit_handle_t h, int k_op, int dt, int64_t M, int64_t N) {
    for (int c = 1; c < CREDIT_NUM_PLANS; ++c) {
        credit_plan_t p = class_plan(c);
        if (plan_ok(h, k_op, dt, M, N, p)) return p;
    }
    return class_plan(0);
}

// Shape features of the learned selector.  f[9] says whether rows of
// ld = N from an aligned base hold whole, 16-byte aligned vectors (N * e a
// multiple of 16): such rows take the unmasked, aligned row loop, up to 1.4x
// faster than ragged rows of the same size, which shifts the best plan.  The
// pick depends on (op, dtype, M, N) only, so a workspace sized with an
// automatic plan always fits the launch that follows.
void features(int k_op, int dt, int64_t M, int64_t N, float *f) {
    const int op = k_op % 3, dir = k_op / 3;
    for (int i = 0; i < CREDIT_NUM_FEATURES; ++i) f[i] = 0.f;
    f[0] = op == OP_SOFTMAX_FWD ? 1.f : 0.f;
    f[1] = op == OP_LN_FWD ? 1.f : 0.f;  // RMSNorm: neither
    f[2] = (float)dir;
    const double e = dt_bytes(dt);
    f[3] = (float)std::log2(e);
    f[4] = (float)std::log2((double)std::max<int64_t>(M, 1));
    f[5] = (float)std::log2((double)N);
    f[6] = ((int64_t)(N * e) % 16 == 0) ? 1.f : 0.f;
    // per split class k: log2(W_k * fill_k), where fill_k is how full the
    // slice keeps the vectors-per-thread bucket it runs in (the operator's
    // register buckets, then its LDS buckets) and W_k = ceil(M / groups) the
    // waves of row groups of Eq. (8), with the row groups of the register
    // model's workgroups per CU on 256 CUs (the host-only geometry of
    // credit_plan_geometry with no handle); -1 when the plan is illegal.  The
    // best plan changes in steps where slices cross bucket and capacity
    // boundaries (Eq. (3)) and where the last wave of row groups is partly
    // empty, which log2 M and log2 N show only indirectly.
    auto fill = [&](int k) -> double {
        const int64_t nv = (N * (int64_t)e + 15) / 16;
        const int64_t per = (nv + k - 1) / k;
        const int64_t need = (per + kBlockThreads - 1) / kBlockThreads;
        for (int v : kVpts)
            if (v >= need && v <= max_vpt(k_op, dt)) return (double)per / ((double)kBlockThreads * v);
        if (lds_capable(k_op, dt))
            for (int v : kLdsVpts)
                if (v >= need) return (double)per / ((double)kBlockThreads * v);
        return 0.0;
    };
    for (int i = 0; i < 5; ++i) {
        const int k = kSplitKs[i];
        const double fl = fill(k);
        Launch L;
        f[7 + i] = -1.f;
        if (fl <= 0.0 || resolve(nullptr, k_op, dt, M, N, {CREDIT_SPLIT_ROW, k}, false, L) != CREDIT_OK) continue;
        const int64_t groups = std::max<int64_t>(1, L.grid / k);
        const int64_t W = (std::max<int64_t>(M, 1) + groups - 1) / groups;
        f[7 + i] = (float)(std::log2((double)W) + std::log2(fl));
    }
}

credit_status_t mlp_predict_dev(credit_handle_t h, const float *feats, int64_t n, float *logits);
credit_status_t mlp_logits_one(credit_handle_t h, const float *feats, float *logits);

credit_status_t analytic_pick(credit_handle_t h, int k_op, int dt, int64_t M, int64_t N, bool peak,
                              credit_plan_t *out, float *pred) {
    credit_plan_t base = {CREDIT_ROW_RESIDENT, 1};
    if (!plan_ok(h, k_op, dt, M, N, base)) base = {CREDIT_TWO_PASS, 1};
    float tb = 0.f;
    credit_status_t st;
    credit_workload_t w = workload(k_op, dt, false);
    if (peak) {
        if (h->copy_gbps <= 0.f) {
            st = copy_bw(h, (size_t)1 << 30, 7, &h->copy_gbps);
            if (st != CREDIT_OK) return st;
        }
        // Table-V row-1 analogue: the baseline priced at copy bandwidth
        tb = (float)((double)M * N * w.b_base / (h->copy_gbps * 1e9) * 1e6);
    } else {
        st = time_plan(h, k_op, dt, M, N, base, 15, 1, &tb);
        if (st != CREDIT_OK) return st;
    }
    float c1 = 0.f;
    st = time_control(h, k_op, dt, M, N, 1, 7, &c1);
    if (st != CREDIT_OK) return st;
    float ctrl[5];
    for (int i = 0; i < 5; ++i) {
        credit_plan_t p = {CREDIT_SPLIT_ROW, kSplitKs[i]};
        ctrl[i] = 0.f;
        if (!plan_ok(h, k_op, dt, M, N, p)) continue;
        float ck = 0.f;
        st = time_control(h, k_op, dt, M, N, kSplitKs[i], 7, &ck);
        if (st != CREDIT_OK) return st;
        ctrl[i] = std::max(0.f, ck - c1);
    }
    float delta[5];
    model_delta(h, k_op, dt, M, N, tb, ctrl, delta);
    if (peak) {
        // serialized staging: the deposit is charged in full
        const double dep = (double)M * N * w.b_keep / (h->copy_gbps * 1e9) * 1e6;
        for (float &d : delta) d = (float)(d - dep);
    }
    int best = -1;
    for (int i = 0; i < 5; ++i)
        if (delta[i] > 0.f && (best < 0 || delta[i] > delta[best])) best = i;
    if (best >= 0) {
        *out = {CREDIT_SPLIT_ROW, kSplitKs[best]};
        if (pred) *pred = tb - delta[best];
    } else {
        *out = base;
        if (pred) *pred = tb;
    }
    return CREDIT_OK;
}

// Order of the plans by the bytes they move per element: the staged plans
// read every input once (the row-resident plan, then split factors by the
// exchange traffic that grows with k), the two-pass plan rereads them.
int bytes_rank(int c) { return c == 0 ? CREDIT_NUM_PLANS : c; }

// Every legal plan timed (cache flush, median of 15).  The fastest median is
// the best plan, except that plans within the timing noise of it --
// max(1%, 2 MAD of either) -- count as equally fast, and among those the one
// that moves fewer bytes (then the smaller k) is kept.
credit_status_t exhaustive_pick(credit_handle_t h, int k_op, int dt, int64_t M, int64_t N, credit_plan_t *out,
                                float *pred) {
    std::vector<std::pair<int, credit_timing_t>> all;
    float best = INFINITY;
    for (int c = 0; c < CREDIT_NUM_PLANS; ++c) {
        credit_plan_t p = class_plan(c);
        if (!plan_ok(h, k_op, dt, M, N, p)) continue;
        float t = 0.f;
        credit_timing_t ts;
        credit_status_t st = time_plan(h, k_op, dt, M, N, p, 15, 1, &t, &ts);
        if (st != CREDIT_OK) return st;
        all.push_back({c, ts});
        best = std::min(best, t);
    }
    if (!std::isfinite(best)) return CREDIT_ERR_UNSUPPORTED;
    credit_timing_t tb = {};
    for (auto &e : all)
        if (e.second.median_us == best) tb = e.second;
    int pick = -1;
    for (auto &e : all) {
        const float noise = std::max(0.01f * best, 2.f * std::max(e.second.mad_us, tb.mad_us));
        if (e.second.median_us - best > noise) continue;
        if (pick < 0 || bytes_rank(e.first) < bytes_rank(pick)) pick = e.first;
    }
    *out = class_plan(pick);
    if (pred) *pred = best;
    return CREDIT_OK;
}

// Logit margin within which the untimed pick counts two plans as tied.  The
// network is trained on soft targets exp(-(T_c / T_best - 1) / tau) with
// tau = 0.02, so a logit gap of 0.5 is a predicted 1% time difference: the
// judge's noise floor, inside which it takes the plan moving fewer bytes.
constexpr float kTieLogit = 0.5f;
// The network's best legal plan -- among the legal plans whose logits lie
// within kTieLogit of the best, the one moving the fewest bytes -- or with
// `timed` its two best legal plans, each timed (cold cache, median of 7),
// keeping the faster: the model as a screen that narrows the search, the
// final choice by measurement.
credit_status_t learned_pick(credit_handle_t h, int k_op, int dt, int64_t M, int64_t N, bool timed,
                             credit_plan_t *out, float *pred) {
    float f[CREDIT_NUM_FEATURES], logits[CREDIT_NUM_PLANS];
    features(k_op, dt, M, N, f);
    credit_status_t st = mlp_logits_one(h, f, logits);
    if (st != CREDIT_OK) return st;
    int best = -1, second = -1;
    for (int c = 0; c < CREDIT_NUM_PLANS; ++c) {
        if (!plan_ok(h, k_op, dt, M, N, class_plan(c))) continue;
        if (best < 0 || logits[c] > logits[best]) {
            second = best;
            best = c;
        } else if (second < 0 || logits[c] > logits[second]) {
            second = c;
        }
    }
    if (best < 0) return CREDIT_ERR_UNSUPPORTED;
    if (!timed) {
        int pick = best;
        for (int c = 0; c < CREDIT_NUM_PLANS; ++c)
            if (logits[best] - logits[c] <= kTieLogit && bytes_rank(c) < bytes_rank(pick) &&
                plan_ok(h, k_op, dt, M, N, class_plan(c)))
                pick = c;
        *out = class_plan(pick);
        return CREDIT_OK;
    }
    *out = class_plan(best);
    if (second < 0) return CREDIT_OK;
    float t1 = 0.f, t2 = 0.f;
    st = time_plan(h, k_op, dt, M, N, class_plan(best), 7, 1, &t1);
    if (st != CREDIT_OK) return st;
    st = time_plan(h, k_op, dt, M, N, class_plan(second), 7, 1, &t2);
    if (st != CREDIT_OK) return st;
    if (t2 < t1) *out = class_plan(second);
    if (pred) *pred = std::min(t1, t2);
    return CREDIT_OK;
}

// The plan of a shape.  Selectors that time kernels (exhaustive, analytic,
// peak, learned with timing) run only when `may_time` (credit_select): an
// operator call never times, allocates or synchronises beyond the network's
// one-row forward pass.  It uses the plan cached for the shape, else the
// network's first legal choice (the fixed rule without a model) -- and while
// its stream is being captured into a graph, where no other device work may
// run, the fixed rule, which is host arithmetic only and is not cached.
credit_status_t pick_plan(credit_handle_t h, int k_op, int dt, int64_t M, int64_t N, credit_plan_t *out,
                          float *pred, bool may_time, bool capturing) {
    std::lock_guard<std::recursive_mutex> g(h->lock);
    if (h->force_set && plan_ok(h, k_op, dt, M, N, h->force_plan)) {
        *out = h->force_plan;
        if (pred) *pred = -1.f;
        return CREDIT_OK;
    }
    credit_selector_t sel = h->selector;
    if (!h->selector_set) sel = h->has_model ? CREDIT_SEL_LEARNED : CREDIT_SEL_FIXED;
    auto key = std::make_tuple(k_op, dt, (int)sel, M, N, 0);
    if (!pred) {
        auto it = h->plan_cache.find(key);
        if (it != h->plan_cache.end()) {
            *out = it->second;
            return CREDIT_OK;
        }
    }
    if (pred) *pred = -1.f;
    credit_status_t st = CREDIT_OK;
    if (!may_time) {
        if (capturing) {
            *out = fixed_rule(h, k_op, dt, M, N);
            return CREDIT_OK;
        }
        st = CREDIT_ERR_MODEL;
        if (sel != CREDIT_SEL_FIXED && h->has_model && core_op(k_op))
            st = learned_pick(h, k_op, dt, M, N, false, out, pred);
        if (st != CREDIT_OK) *out = fixed_rule(h, k_op, dt, M, N);
        h->plan_cache[key] = *out;
        return CREDIT_OK;
    }
    switch (sel) {
    case CREDIT_SEL_LEARNED:
        // the learned selector's features cover the softmax / LayerNorm /
        // RMSNorm operators; the other workloads use the analytic model
    case CREDIT_SEL_LEARNED_TIMED:
        if (h->has_model && core_op(k_op)) {
            st = learned_pick(h, k_op, dt, M, N, sel == CREDIT_SEL_LEARNED_TIMED, out, pred);
            if (st == CREDIT_OK) break;
        }
        st = analytic_pick(h, k_op, dt, M, N, false, out, pred);
        break;
    case CREDIT_SEL_ANALYTIC: st = analytic_pick(h, k_op, dt, M, N, false, out, pred); break;
    case CREDIT_SEL_PEAK: st = analytic_pick(h, k_op, dt, M, N, true, out, pred); break;
    case CREDIT_SEL_EXHAUSTIVE: st = exhaustive_pick(h, k_op, dt, M, N, out, pred); break;
    default: *out = fixed_rule(h, k_op, dt, M, N); break;
    }
    if (st == CREDIT_OK) h->plan_cache[key] = *out;
    return st;
}

// ------------------------------------------------------ co-residency
// Every row-resident / split-row instance whose compiled code uses private
// memory (register spills, stack arrays) is launched once in probe mode at
// its full persistent grid, occupancy x CUs: every workgroup announces itself
// and waits for all the others (bounded).  Split plans of the instance then
// use the largest per-CU count at which no workgroup gave up, so their grid
// is one the device was seen to hold at once.  Instances without private
// memory are bounded by registers, LDS and wave slots alone, which the
// occupancy query reports.
credit_status_t verify_coresidency(credit_handle_t h) {
    constexpr unsigned kProbeSpins = 1u << 15;
    for (int k_op = 0; k_op < OP_COUNT; ++k_op) {
        for (int dt = CREDIT_F32; dt <= CREDIT_FP8_E4M3; ++dt) {
            if (!dt_ok(k_op, dt)) continue;
            for (int vr = 0; vr < (int)(std::size(kAllVpts) * 3); ++vr) {
                const int vpt = kAllVpts[vr / 3], rows = vr % 3 == 0 ? 1 : kMrRows[vr % 3 - 1];
                if (!instance_exists(k_op, dt, vpt)) continue;
                if (rows > 1 && !multirow_exists(k_op, dt, vpt, rows)) continue;
                const void *fn = instance_fn(k_op, dt, vpt, rows);
                if (!fn) continue;
                hipFuncAttributes at;
                if (hipFuncGetAttributes(&at, fn) != hipSuccess) return CREDIT_ERR_HIP;
                h->scratch[fn] = at.localSizeBytes;
                if (at.localSizeBytes == 0) continue;
                const int occ = occupancy(h, fn, kBlockThreads, 0);
                int ok = 0;
                for (int per = occ; per >= 1 && !ok; --per) {
                    RowArgs a;
                    std::memset(&a, 0, sizeof(a));
                    a.errflag = h->errflag;
                    a.spin_limit = kProbeSpins;
                    a.flags = F_PROBE;
                    a.k = 1;
                    void *args[] = {&a};
                    unsigned missed = 1;
                    if (hipMemsetAsync(h->errflag + 96, 0, 8, h->stream) != hipSuccess ||
                        fenced_launch(h->device, false, fn, per * h->cus, kBlockThreads, 0, h->stream, args) !=
                            hipSuccess ||
                        hipMemcpyAsync(&missed, h->errflag + 97, 4, hipMemcpyDeviceToHost, h->stream) !=
                            hipSuccess ||
                        hipStreamSynchronize(h->stream) != hipSuccess)
                        return CREDIT_ERR_HIP;
                    if (missed == 0) ok = per;
                }
                h->coresident[fn] = ok;
            }
        }
    }
    return CREDIT_OK;
}

// ------------------------------------------------------------------- MLP
const int kH = CREDIT_MLP_HIDDEN, kF = CREDIT_NUM_FEATURES, kC = CREDIT_NUM_PLANS;
const size_t oW1 = 0, ob1 = oW1 + kH * kF, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH, ob3 = oW3 + kC * kH;

struct MlpDev {
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float *raw = nullptr, *z = nullptr, *h1 = nullptr, *h2 = nullptr, *lg = nullptr, *tg = nullptr;
    float *dl = nullptr, *dh2 = nullptr, *dh1 = nullptr, *loss = nullptr, *lmean = nullptr, *mu = nullptr,
          *sd = nullptr, *dz = nullptr;
    uint8_t *mask = nullptr;
    int64_t n = 0;
    std::vector<void *> owned;
    ~MlpDev() {
        for (void *q : owned) (void)hipFree(q);
    }
    template <class T> bool alloc(T *&q, size_t count) {
        if (hipMalloc((void **)&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
        owned.push_back(q);
        return true;
    }
    bool init(int64_t n_) {
        n = n_;
        return alloc(p, kMlpParams) && alloc(g, kMlpParams) && alloc(m, kMlpParams) && alloc(v, kMlpParams) &&
               alloc(raw, n * kF) && alloc(z, n * kF) && alloc(h1, n * kH) && alloc(h2, n * kH) &&
               alloc(lg, n * kC) && alloc(tg, n * kC) && alloc(dl, n * kC) && alloc(dh2, n * kH) &&
               alloc(dh1, n * kH) && alloc(loss, n) && alloc(lmean, 1) && alloc(mu, kF) && alloc(sd, kF) &&
               alloc(dz, n * kF) && alloc(mask, n * kC);
    }
};

int blocks(int64_t n) { return (int)std::max<int64_t>(1, (n + 255) / 256); }

hipError_t mlp_forward(MlpDev &d, hipStream_t s) {
    int64_t n = d.n;
    int nf = kF;
    hipError_t e;
    {
        void *a[] = {&d.raw, &d.mu, &d.sd, &d.z, &n, &nf};
        if ((e = launch(mlp_kernel(0), blocks(n * kF), 256, 0, s, a)) != hipSuccess) return e;
    }
    auto dense = [&](float *in, size_t ow, size_t ob, float *out, int I, int O, int relu) {
        float *W = d.p + ow, *b = d.p + ob;
        void *a[] = {&in, &W, &b, &out, &n, &I, &O, &relu};
        return launch(mlp_kernel(1), blocks(n * O), 256, 0, s, a);
    };
    if ((e = dense(d.z, oW1, ob1, d.h1, kF, kH, 1)) != hipSuccess) return e;
    if ((e = dense(d.h1, oW2, ob2, d.h2, kH, kH, 1)) != hipSuccess) return e;
    return dense(d.h2, oW3, ob3, d.lg, kH, kC, 0);
}

hipError_t mlp_backward(MlpDev &d, hipStream_t s) {
    int64_t n = d.n;
    int C = kC;
    hipError_t e;
    {
        void *a[] = {&d.lg, &d.tg, &d.mask, &d.dl, &d.loss, &n, &C};
        if ((e = launch(mlp_kernel(2), blocks(n), 256, 0, s, a)) != hipSuccess) return e;
    }
    {
        void *a[] = {&d.loss, &n, &d.lmean};
        if ((e = launch(mlp_kernel(3), 1, 256, 0, s, a)) != hipSuccess) return e;
    }
    auto bw = [&](float *dout, float *in, size_t ow, size_t ob, int I, int O) {
        float *dW = d.g + ow, *db = d.g + ob;
        void *a[] = {&dout, &in, &dW, &db, &n, &I, &O};
        return launch(mlp_kernel(4), blocks((int64_t)O * (I + 1)), 256, 0, s, a);
    };
    auto bi = [&](float *dout, size_t ow, float *act, float *din, int I, int O) {
        float *W = d.p + ow;
        void *a[] = {&dout, &W, &act, &din, &n, &I, &O};
        return launch(mlp_kernel(5), blocks(n * I), 256, 0, s, a);
    };
    if ((e = bw(d.dl, d.h2, oW3, ob3, kH, kC)) != hipSuccess) return e;
    if ((e = bi(d.dl, oW3, d.h2, d.dh2, kH, kC)) != hipSuccess) return e;
    if ((e = bw(d.dh2, d.h1, oW2, ob2, kH, kH)) != hipSuccess) return e;
    if ((e = bi(d.dh2, oW2, d.h1, d.dh1, kH, kH)) != hipSuccess) return e;
    return bw(d.dh1, d.z, oW1, ob1, kF, kH);
}

bool mlp_upload(credit_handle_t h, MlpDev &d, const float *feats, const float *targets, const uint8_t *mask) {
    int64_t n = d.n;
    bool ok = hipMemcpy(d.p, h->params.data(), kMlpParams * 4, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(d.raw, feats, n * kF * 4, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(d.mu, h->mu, kF * 4, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(d.sd, h->sd, kF * 4, hipMemcpyHostToDevice) == hipSuccess;
    if (ok && targets) ok = hipMemcpy(d.tg, targets, n * kC * 4, hipMemcpyHostToDevice) == hipSuccess;
    if (ok && mask) ok = hipMemcpy(d.mask, mask, n * kC, hipMemcpyHostToDevice) == hipSuccess;
    return ok;
}

// Offsets (in floats) of the single-row inference block h->inf.
constexpr size_t iP = 0, iMu = iP + kMlpParams, iSd = iMu + kF, iRaw = iSd + kF, iZ = iRaw + kF, iH1 = iZ + kF,
                 iH2 = iH1 + kH, iLg = iH2 + kH, iEnd = iLg + kC;

// Allocates the single-row inference block (once) and uploads the current
// network into it.  Called whenever a model is set, never from an operator.
credit_status_t upload_infer(credit_handle_t h) {
    if (!h->inf && hipMalloc(&h->inf, iEnd * 4) != hipSuccess) {
        h->inf = nullptr;
        (void)hipGetLastError();
        return CREDIT_ERR_HIP;
    }
    if (hipMemcpy(h->inf + iP, h->params.data(), kMlpParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->inf + iMu, h->mu, kF * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->inf + iSd, h->sd, kF * 4, hipMemcpyHostToDevice) != hipSuccess)
        return CREDIT_ERR_HIP;
    return CREDIT_OK;
}

// The network's logits for one feature row, through the HIP kernels on the
// handle's stream, in the preallocated block: no allocation.
credit_status_t mlp_logits_one(credit_handle_t h, const float *feats, float *logits) {
    if (!h->inf) return CREDIT_ERR_MODEL;
    MlpDev d;  // a view of h->inf (owns nothing)
    d.n = 1;
    d.p = h->inf + iP;
    d.mu = h->inf + iMu;
    d.sd = h->inf + iSd;
    d.raw = h->inf + iRaw;
    d.z = h->inf + iZ;
    d.h1 = h->inf + iH1;
    d.h2 = h->inf + iH2;
    d.lg = h->inf + iLg;
    if (hipMemcpyAsync(d.raw, feats, kF * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        mlp_forward(d, h->stream) != hipSuccess ||
        hipMemcpyAsync(logits, d.lg, kC * 4, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return CREDIT_ERR_HIP;
    return CREDIT_OK;
}

credit_status_t mlp_predict_dev(credit_handle_t h, const float *feats, int64_t n, float *logits) {
    MlpDev d;
    if (!d.init(n)) return CREDIT_ERR_HIP;
    if (!mlp_upload(h, d, feats, nullptr, nullptr)) return CREDIT_ERR_HIP;
    if (mlp_forward(d, h->stream) != hipSuccess) return CREDIT_ERR_HIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return CREDIT_ERR_HIP;
    if (hipMemcpy(logits, d.lg, n * kC * 4, hipMemcpyDeviceToHost) != hipSuccess) return CREDIT_ERR_HIP;
    return CREDIT_OK;
}

// splitmix64 + Box-Muller: a portable seeded normal generator for He init.
struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() { return std::sqrt(-2.0 * std::log(uniform())) * std::cos(6.283185307179586 * uniform()); }
};

}  // namespace

// =================================================================== C ABI
extern "C" {

const char *credit_status_string(credit_status_t s) {
    switch (s) {
    case CREDIT_OK: return "CREDIT_OK";
    case CREDIT_ERR_INVALID_ARG: return "CREDIT_ERR_INVALID_ARG";
    case CREDIT_ERR_UNSUPPORTED: return "CREDIT_ERR_UNSUPPORTED";
    case CREDIT_ERR_WORKSPACE: return "CREDIT_ERR_WORKSPACE";
    case CREDIT_ERR_HIP: return "CREDIT_ERR_HIP";
    case CREDIT_ERR_TIMEOUT: return "CREDIT_ERR_TIMEOUT";
    case CREDIT_ERR_MODEL: return "CREDIT_ERR_MODEL";
    }
    return "CREDIT_ERR_UNKNOWN";
}

const char *credit_version(void) { return "credit-mi355x 0.1.0 (gfx950)"; }

// Environment configuration, read once when a handle is created:
//   CREDIT_SELECTOR    learned | analytic | exhaustive | fixed | peak
//   CREDIT_FORCE_PLAN  two_pass | resident | split:<k>   (calls with plan == NULL
//                      use it where it is legal for the shape)
//   CREDIT_SPIN_LIMIT  polls before a split-row wait gives up
//   CREDIT_CHECKED     1: operator calls wait for their launches and return
//                      CREDIT_ERR_TIMEOUT themselves
//   CREDIT_LOG         stderr | <path>: one JSON line per operator call
//                      (appended; a path that cannot be opened is ignored)
// Unrecognised values are ignored.
static void read_env(credit_handle_t h) {
    if (const char *v = std::getenv("CREDIT_SELECTOR")) {
        const std::string s(v);
        const char *names[] = {"learned", "analytic", "exhaustive", "fixed", "peak"};
        for (int i = 0; i < 5; ++i)
            if (s == names[i]) {
                h->selector = (credit_selector_t)i;
                h->selector_set = true;
            }
    }
    if (const char *v = std::getenv("CREDIT_FORCE_PLAN")) {
        const std::string s(v);
        if (s == "two_pass") {
            h->force_plan = {CREDIT_TWO_PASS, 1};
            h->force_set = true;
        } else if (s == "resident") {
            h->force_plan = {CREDIT_ROW_RESIDENT, 1};
            h->force_set = true;
        } else if (s.rfind("split:", 0) == 0) {
            const int k = std::atoi(s.c_str() + 6);
            for (int kk : kSplitKs)
                if (kk == k) {
                    h->force_plan = {CREDIT_SPLIT_ROW, k};
                    h->force_set = true;
                }
        }
    }
    if (const char *v = std::getenv("CREDIT_SPIN_LIMIT")) {
        const long long n = std::atoll(v);
        if (n > 0) h->spin_limit = n;
    }
    if (const char *v = std::getenv("CREDIT_CHECKED")) h->checked = std::string(v) == "1";
    if (const char *v = std::getenv("CREDIT_LOG")) {
        const std::string s(v);
        if (s == "stderr") {
            h->log = stderr;
        } else if (!s.empty()) {
            h->log = std::fopen(v, "a");
            h->log_owned = h->log != nullptr;
        }
    }
}

credit_status_t credit_create(int device, credit_handle_t *out) {
    if (!out) return CREDIT_ERR_INVALID_ARG;
    *out = nullptr;
    try {
        hipDeviceProp_t prop;
        if (hipSetDevice(device) != hipSuccess) return CREDIT_ERR_HIP;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) return CREDIT_ERR_HIP;
        credit_handle_t h = new credit_handle_s();
        h->device = device;
        h->cus = prop.multiProcessorCount;
        h->arch = prop.gcnArchName;
        if (hipStreamCreate(&h->stream) != hipSuccess || hipMalloc(&h->errflag, 512) != hipSuccess ||
            hipMemset(h->errflag, 0, 512) != hipSuccess || hipEventCreate(&h->ev0) != hipSuccess ||
            hipEventCreate(&h->ev1) != hipSuccess) {
            credit_destroy(h);
            return CREDIT_ERR_HIP;
        }
        read_env(h);
        // the allocation-free entry point's scratch on this device: its
        // address, and (once per device and process) its slots zeroed by a
        // fill kernel; the wait-fence event is created here too, so that no
        // operator call creates one
        void *sp = nullptr;
        if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) {
            (void)hipGetLastError();
            credit_destroy(h);
            return CREDIT_ERR_HIP;
        }
        h->scratch_dev = (char *)sp;
        {
            static std::mutex zm;
            static bool zeroed[64] = {false};
            std::lock_guard<std::mutex> zg(zm);
            if (!zeroed[device & 63]) {
                if (zero_words(sp, (int64_t)(kScratchBytes / 4), h->stream) != hipSuccess ||
                    hipStreamSynchronize(h->stream) != hipSuccess) {
                    credit_destroy(h);
                    return CREDIT_ERR_HIP;
                }
                zeroed[device & 63] = true;
            }
            WaitFence &f = wait_fence(device);
            std::lock_guard<std::mutex> fg(f.m);
            if (!f.ev && hipEventCreateWithFlags(&f.ev, hipEventDisableTiming) != hipSuccess) {
                f.ev = nullptr;
                credit_destroy(h);
                return CREDIT_ERR_HIP;
            }
        }
        if (verify_coresidency(h) != CREDIT_OK) {
            credit_destroy(h);
            return CREDIT_ERR_HIP;
        }
        *out = h;
        return CREDIT_OK;
    } catch (...) {
        return CREDIT_ERR_HIP;
    }
}

credit_status_t credit_destroy(credit_handle_t h) {
    if (!h) return CREDIT_ERR_INVALID_ARG;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->arena) (void)hipFree(h->arena);
    if (h->flushbuf) (void)hipFree(h->flushbuf);
    if (h->inf) (void)hipFree(h->inf);
    if (h->errflag) (void)hipFree(h->errflag);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    if (h->log_owned) std::fclose(h->log);
    delete h;
    return CREDIT_OK;
}

credit_status_t credit_set_selector(credit_handle_t h, credit_selector_t s) {
    if (!h || (int)s < 0 || (int)s > (int)CREDIT_SEL_LEARNED_TIMED) return CREDIT_ERR_INVALID_ARG;
    std::lock_guard<std::recursive_mutex> g(h->lock);
    h->selector = s;
    h->selector_set = true;
    return CREDIT_OK;
}

static bool valid_enum(credit_op_t op, credit_dir_t dir, credit_dtype_t dt) {
    const int k = kop((int)op, (int)dir);
    return k >= 0 && dt_ok(k, (int)dt);
}

credit_status_t credit_workspace_size(credit_handle_t h, credit_op_t op, credit_dir_t dir, credit_dtype_t dt,
                                      int64_t M, int64_t N, const credit_plan_t *plan, size_t *bytes) {
    if (!h || !bytes || !valid_enum(op, dir, dt) || M < 0 || N <= 0) return CREDIT_ERR_INVALID_ARG;
    try {
        Launch L;
        std::lock_guard<std::recursive_mutex> g(h->lock);
        if (plan) {
            credit_status_t st = resolve(h, kop(op, dir), dt, M, N, *plan, true, L);
            if (st != CREDIT_OK) return st;
            *bytes = L.ws_bytes;
            return CREDIT_OK;
        }
        // no plan: enough for any plan an automatic call may pick (the
        // largest over the legal plans), so sizing selects nothing
        size_t most = 0;
        bool any = false;
        for (int c = 0; c < CREDIT_NUM_PLANS; ++c) {
            if (resolve(h, kop(op, dir), dt, std::max<int64_t>(M, 1), N, class_plan(c), true, L) != CREDIT_OK)
                continue;
            most = std::max(most, L.ws_bytes);
            any = true;
        }
        if (!any) return CREDIT_ERR_UNSUPPORTED;
        *bytes = most;
        return CREDIT_OK;
    } catch (...) {
        return CREDIT_ERR_HIP;
    }
}

credit_status_t credit_plan_legal(credit_handle_t h, credit_op_t op, credit_dir_t dir, credit_dtype_t dt, int64_t M,
                                  int64_t N, const credit_plan_t *plan) {
    if (!plan || !valid_enum(op, dir, dt) || M < 0 || N <= 0) return CREDIT_ERR_INVALID_ARG;
    Launch L;
    if (h) {
        std::lock_guard<std::recursive_mutex> g(h->lock);
        return resolve(h, kop(op, dir), dt, M, N, *plan, false, L);
    }
    return resolve(nullptr, kop(op, dir), dt, M, N, *plan, false, L);
}

credit_status_t credit_plan_geometry(credit_handle_t h, credit_op_t op, credit_dir_t dir, credit_dtype_t dt,
                                     int64_t M, int64_t N, const credit_plan_t *plan, int32_t *grid, int32_t *block,
                                     int32_t *vpt, int32_t *per_cu, int32_t *rows) {
    if (!plan || !valid_enum(op, dir, dt) || M < 0 || N <= 0) return CREDIT_ERR_INVALID_ARG;
    Launch L;
    credit_status_t st;
    if (h) {
        std::lock_guard<std::recursive_mutex> g(h->lock);
        st = resolve(h, kop(op, dir), dt, M, N, *plan, false, L);
    } else {
        st = resolve(nullptr, kop(op, dir), dt, M, N, *plan, false, L);
    }
    if (st != CREDIT_OK) return st;
    if (grid) *grid = L.grid;
    if (block) *block = L.block;
    if (vpt) *vpt = L.vpt;
    if (per_cu) *per_cu = L.per_cu;
    if (rows) *rows = L.rows;
    return CREDIT_OK;
}

credit_status_t credit_select(credit_handle_t h, credit_op_t op, credit_dir_t dir, credit_dtype_t dt, int64_t M,
                              int64_t N, credit_plan_t *out, float *predicted_us) {
    if (!h || !out || !valid_enum(op, dir, dt) || M <= 0 || N <= 0) return CREDIT_ERR_INVALID_ARG;
    try {
        float pred = -1.f;
        credit_status_t st = pick_plan(h, kop(op, dir), dt, M, N, out, &pred, true, false);
        if (predicted_us) *predicted_us = pred;
        return st;
    } catch (...) {
        return CREDIT_ERR_HIP;
    }
}

credit_status_t credit_softmax_fwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt, const void *x,
                                   int64_t ldx, const float *x_scale, void *y, int64_t ldy, float *y_scale,
                                   const credit_plan_t *plan, void *ws, size_t ws_bytes, void *stream) {
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = OP_SOFTMAX_FWD; c.dt = dt; c.M = M; c.N = N;
    c.in0 = x; c.ld0 = ldx; c.s0 = x_scale;
    c.out = y; c.ldo = ldy; c.so = y_scale;
    c.ld1 = N;
    try { return run_op(h, c, plan, ws, ws_bytes, stream, false); } catch (...) { return CREDIT_ERR_HIP; }
}

credit_status_t credit_softmax_bwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt, const void *y,
                                   int64_t ldy, const float *y_scale, const void *dy, int64_t lddy,
                                   const float *dy_scale, void *dx, int64_t lddx, float *dx_scale,
                                   const credit_plan_t *plan, void *ws, size_t ws_bytes, void *stream) {
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = OP_SOFTMAX_BWD; c.dt = dt; c.M = M; c.N = N;
    c.in0 = y; c.ld0 = ldy; c.s0 = y_scale;
    c.in1 = dy; c.ld1 = lddy; c.s1 = dy_scale;
    c.out = dx; c.ldo = lddx; c.so = dx_scale;
    try { return run_op(h, c, plan, ws, ws_bytes, stream, false); } catch (...) { return CREDIT_ERR_HIP; }
}

credit_status_t credit_layernorm_fwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt, const void *x,
                                     int64_t ldx, const float *x_scale, const float *gamma, const float *beta,
                                     float eps, void *y, int64_t ldy, float *y_scale, float *mean, float *rstd,
                                     const credit_plan_t *plan, void *ws, size_t ws_bytes, void *stream) {
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = OP_LN_FWD; c.dt = dt; c.M = M; c.N = N;
    c.in0 = x; c.ld0 = ldx; c.s0 = x_scale;
    c.gamma = gamma; c.beta = beta; c.eps = eps;
    c.out = y; c.ldo = ldy; c.so = y_scale;
    c.mean_out = mean; c.rstd_out = rstd;
    c.ld1 = N;
    try { return run_op(h, c, plan, ws, ws_bytes, stream, false); } catch (...) { return CREDIT_ERR_HIP; }
}

credit_status_t credit_layernorm_fwd_noalloc(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                                             const void *x, int64_t ldx, const float *x_scale, const float *gamma,
                                             const float *beta, float eps, void *y, int64_t ldy, float *y_scale,
                                             float *mean, float *rstd, const credit_plan_t *plan, void *stream) {
    if (!h || !h->scratch_dev) return CREDIT_ERR_INVALID_ARG;
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = OP_LN_FWD; c.dt = dt; c.M = M; c.N = N;
    c.in0 = x; c.ld0 = ldx; c.s0 = x_scale;
    c.gamma = gamma; c.beta = beta; c.eps = eps;
    c.out = y; c.ldo = ldy; c.so = y_scale;
    c.mean_out = mean; c.rstd_out = rstd;
    c.ld1 = N;
    // a plan whose workspace exceeds the scratch returns CREDIT_ERR_WORKSPACE
    try {
        return run_op(h, c, plan, h->scratch_dev, kScratchBytes, stream, false, true);
    } catch (...) {
        return CREDIT_ERR_HIP;
    }
}

size_t credit_noalloc_scratch_bytes(void) { return kScratchBytes; }

credit_status_t credit_layernorm_bwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt, const void *x,
                                     int64_t ldx, const float *x_scale, const void *dy, int64_t lddy,
                                     const float *dy_scale, const float *gamma, const float *mean, const float *rstd,
                                     float eps, void *dx, int64_t lddx, float *dx_scale, float *dgamma,
                                     float *dbeta, const credit_plan_t *plan, void *ws, size_t ws_bytes,
                                     void *stream) {
    if ((mean == nullptr) != (rstd == nullptr)) return CREDIT_ERR_INVALID_ARG;
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = OP_LN_BWD; c.dt = dt; c.M = M; c.N = N;
    c.in0 = x; c.ld0 = ldx; c.s0 = x_scale;
    c.in1 = dy; c.ld1 = lddy; c.s1 = dy_scale;
    c.gamma = gamma; c.mean_in = mean; c.rstd_in = rstd; c.eps = eps;
    c.out = dx; c.ldo = lddx; c.so = dx_scale;
    c.dgamma = dgamma; c.dbeta = dbeta;
    try { return run_op(h, c, plan, ws, ws_bytes, stream, mean == nullptr); } catch (...) { return CREDIT_ERR_HIP; }
}

credit_status_t credit_rmsnorm_fwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt, const void *x,
                                   int64_t ldx, const float *x_scale, const float *gamma, float eps, void *y,
                                   int64_t ldy, float *y_scale, float *rstd, const credit_plan_t *plan, void *ws,
                                   size_t ws_bytes, void *stream) {
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = OP_RMS_FWD; c.dt = dt; c.M = M; c.N = N;
    c.in0 = x; c.ld0 = ldx; c.s0 = x_scale;
    c.gamma = gamma; c.eps = eps;
    c.out = y; c.ldo = ldy; c.so = y_scale;
    c.rstd_out = rstd;
    c.ld1 = N;
    try { return run_op(h, c, plan, ws, ws_bytes, stream, false); } catch (...) { return CREDIT_ERR_HIP; }
}

credit_status_t credit_rmsnorm_bwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt, const void *x,
                                   int64_t ldx, const float *x_scale, const void *dy, int64_t lddy,
                                   const float *dy_scale, const float *gamma, const float *rstd, float eps, void *dx,
                                   int64_t lddx, float *dx_scale, float *dgamma, const credit_plan_t *plan, void *ws,
                                   size_t ws_bytes, void *stream) {
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = OP_RMS_BWD; c.dt = dt; c.M = M; c.N = N;
    c.in0 = x; c.ld0 = ldx; c.s0 = x_scale;
    c.in1 = dy; c.ld1 = lddy; c.s1 = dy_scale;
    c.gamma = gamma; c.rstd_in = rstd; c.eps = eps;
    c.out = dx; c.ldo = lddx; c.so = dx_scale;
    c.dgamma = dgamma;
    try { return run_op(h, c, plan, ws, ws_bytes, stream, rstd == nullptr); } catch (...) { return CREDIT_ERR_HIP; }
}

credit_status_t credit_softmax_logits_bwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt, const void *x,
                                          int64_t ldx, const float *x_scale, const void *dy, int64_t lddy,
                                          const float *dy_scale, void *dx, int64_t lddx, float *dx_scale,
                                          const credit_plan_t *plan, void *ws, size_t ws_bytes, void *stream) {
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = OP_SMXL_BWD; c.dt = dt; c.M = M; c.N = N;
    c.in0 = x; c.ld0 = ldx; c.s0 = x_scale;
    c.in1 = dy; c.ld1 = lddy; c.s1 = dy_scale;
    c.out = dx; c.ldo = lddx; c.so = dx_scale;
    try { return run_op(h, c, plan, ws, ws_bytes, stream, false); } catch (...) { return CREDIT_ERR_HIP; }
}

credit_status_t credit_quantize_rows(credit_handle_t h, credit_op_t op, int64_t M, int64_t N, credit_dtype_t dt,
                                     const void *x, int64_t ldx, void *q, int64_t ldq, float *q_scale,
                                     const credit_plan_t *plan, void *ws, size_t ws_bytes, void *stream) {
    if (op != CREDIT_QUANT_INT8 && op != CREDIT_QUANT_FP8) return CREDIT_ERR_INVALID_ARG;
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = op == CREDIT_QUANT_INT8 ? OP_QUANT_I8 : OP_QUANT_F8; c.dt = dt; c.M = M; c.N = N;
    c.in0 = x; c.ld0 = ldx;
    c.out = q; c.ldo = ldq; c.so = q_scale;
    try { return run_op(h, c, plan, ws, ws_bytes, stream, false); } catch (...) { return CREDIT_ERR_HIP; }
}

credit_status_t credit_pearson_bwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt, const void *x,
                                   int64_t ldx, const void *y, int64_t ldy, const float *dr, void *dx, int64_t lddx,
                                   void *dy, int64_t lddy, const credit_plan_t *plan, void *ws, size_t ws_bytes,
                                   void *stream) {
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = OP_PEARSON_BWD; c.dt = dt; c.M = M; c.N = N;
    c.in0 = x; c.ld0 = ldx;
    c.in1 = y; c.ld1 = ldy;
    c.rowg = dr;
    c.out = dx; c.ldo = lddx;
    c.out1 = dy; c.ldo1 = lddy;
    try { return run_op(h, c, plan, ws, ws_bytes, stream, false); } catch (...) { return CREDIT_ERR_HIP; }
}

credit_status_t credit_wvar_bwd(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt, const void *x,
                                int64_t ldx, const void *w, int64_t ldw, const float *dv, void *dx, int64_t lddx,
                                void *dw, int64_t lddw, const credit_plan_t *plan, void *ws, size_t ws_bytes,
                                void *stream) {
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = OP_WVAR_BWD; c.dt = dt; c.M = M; c.N = N;
    c.in0 = x; c.ld0 = ldx;
    c.in1 = w; c.ld1 = ldw;
    c.rowg = dv;
    c.out = dx; c.ldo = lddx;
    c.out1 = dw; c.ldo1 = lddw;
    try { return run_op(h, c, plan, ws, ws_bytes, stream, false); } catch (...) { return CREDIT_ERR_HIP; }
}

credit_status_t credit_layernorm_fwd_fp8_out(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt,
                                             const void *x, int64_t ldx, const float *gamma, const float *beta,
                                             float eps, void *q, int64_t ldq, float *q_scale, float *mean,
                                             float *rstd, const credit_plan_t *plan, void *ws, size_t ws_bytes,
                                             void *stream) {
    OpCall c;
    std::memset(&c, 0, sizeof(c));
    c.k_op = OP_LNQ_FWD; c.dt = dt; c.M = M; c.N = N;
    c.in0 = x; c.ld0 = ldx;
    c.gamma = gamma; c.beta = beta; c.eps = eps;
    c.out = q; c.ldo = ldq; c.so = q_scale;
    c.mean_out = mean; c.rstd_out = rstd;
    try { return run_op(h, c, plan, ws, ws_bytes, stream, false); } catch (...) { return CREDIT_ERR_HIP; }
}

// ------------------------------------------------------- primitive probes
namespace {
struct ProbeOutH {
    unsigned long long cycles, ticks;
    unsigned err, xcc[2], sink;
};

credit_status_t probe_run(credit_handle_t h, int which, dim3 grid, dim3 block, void **args, ProbeOutH *dev,
                          ProbeOutH *res) {
    // the result block and the ping-pong word (the first 512 bytes) start at zero
    if (zero_words(dev, 128, h->stream) != hipSuccess) return CREDIT_ERR_HIP;
    if (hipLaunchKernel(probe_kernel(which), grid, block, args, 0, h->stream) != hipSuccess) return CREDIT_ERR_HIP;
    if (hipMemcpyAsync(res, dev, sizeof(ProbeOutH), hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        return CREDIT_ERR_HIP;
    return hipStreamSynchronize(h->stream) == hipSuccess ? CREDIT_OK : CREDIT_ERR_HIP;
}

credit_status_t probe_all(credit_handle_t h, int reps, credit_primitives_t *out) {
    std::lock_guard<std::recursive_mutex> g(h->lock);
    const int rounds = 2000, steps = 4000, xrows = 256;
    const size_t o_out = 0, o_word = 256, o_chain = 512, o_rate = o_chain + 65536,
                 o_slots = o_rate + (256 << 10);
    const size_t slot_bytes = (size_t)xrows * kMaxStages * kMaxK * 8;
    credit_status_t st = ensure_arena(h, o_slots + slot_bytes);
    if (st != CREDIT_OK) return st;
    h->prepared = std::make_tuple(-1, -1, (int64_t)-1, (int64_t)-1);
    char *base = h->arena;
    ProbeOutH *dev = (ProbeOutH *)(base + o_out);
    unsigned *word = (unsigned *)(base + o_word);
    unsigned *chain = (unsigned *)(base + o_chain);
    void *rate = base + o_rate;
    std::vector<unsigned> hc(16384);
    for (unsigned i = 0; i < 16384; ++i) hc[i] = (i + 4099u) & 16383u;  // one cycle, 16 KiB strides
    if (hipMemcpyAsync(chain, hc.data(), 65536, hipMemcpyHostToDevice, h->stream) != hipSuccess) return CREDIT_ERR_HIP;
    std::memset(out, 0, sizeof(*out));
    const int R = reps > 0 ? reps : 15;
    double mhz_c = 0, mhz_t = 0;
    auto med = [&](int which, dim3 grid, dim3 block, std::vector<void *> args, double per, float *ns,
                   float *cyc_out) -> credit_status_t {
        std::vector<float> tn, tc;
        for (int r = 0; r < R; ++r) {
            ProbeOutH res;
            credit_status_t s2 = probe_run(h, which, grid, block, args.data(), dev, &res);
            if (s2 != CREDIT_OK) return s2;
            out->errors += (int32_t)res.err;
            tn.push_back((float)(res.ticks * 10.0 / per));
            tc.push_back((float)(res.cycles / per));
            mhz_c += (double)res.cycles;
            mhz_t += (double)res.ticks;
            if (which == 2) {
                int32_t *dst = (((int *)args[2])[0] == 0 && ((int *)args[3])[0] == 8) ? out->xcd_same : out->xcd_cross;
                dst[0] = (int32_t)res.xcc[0];
                dst[1] = (int32_t)res.xcc[1];
            }
        }
        if (ns) *ns = median(tn);
        if (cyc_out) *cyc_out = median(tc);
        return CREDIT_OK;
    };
    int isteps = steps, irounds = rounds;
    unsigned spin = (unsigned)std::min<int64_t>(h->spin_limit, 0xffffffffLL);
    if ((st = med(0, dim3(1), dim3(64), {&dev, &isteps}, steps, &out->lds_load_ns, nullptr)) != CREDIT_OK) return st;
    const unsigned *cchain = chain;
    if ((st = med(1, dim3(1), dim3(64), {&dev, &cchain, &isteps}, steps, &out->l2_load_ns, nullptr)) != CREDIT_OK)
        return st;
    int a0 = 0, b8 = 8, b1 = 1;
    // a round trip is two handoffs
    if ((st = med(2, dim3(9), dim3(64), {&dev, &word, &a0, &b8, &irounds, &spin}, 2.0 * rounds,
                  &out->handoff_same_xcd_ns, nullptr)) != CREDIT_OK)
        return st;
    if ((st = med(2, dim3(9), dim3(64), {&dev, &word, &a0, &b1, &irounds, &spin}, 2.0 * rounds,
                  &out->handoff_cross_xcd_ns, nullptr)) != CREDIT_OK)
        return st;
    if ((st = med(3, dim3(1), dim3(256), {&dev, &isteps}, steps, &out->barrier_ns, nullptr)) != CREDIT_OK) return st;
    if (zero_words(base + o_slots, (int64_t)(slot_bytes / 4), h->stream) != hipSuccess) return CREDIT_ERR_HIP;
    for (int i = 0; i < 5; ++i) {
        RowArgs a;
        std::memset(&a, 0, sizeof(a));
        a.k = kSplitKs[i];
        a.qs = 1;
        a.M = xrows;
        a.slots = (unsigned long long *)(base + o_slots);
        a.errflag = h->errflag;
        a.spin_limit = spin;
        int rows = xrows;
        std::vector<float> tn;
        for (int r = 0; r < R; ++r) {
            a.epoch = next_epoch();
            void *args[] = {&dev, &a, &rows};
            ProbeOutH res;
            if ((st = probe_run(h, 4, dim3(a.k), dim3(kBlockThreads), args, dev, &res)) != CREDIT_OK) return st;
            tn.push_back((float)(res.ticks * 10.0 / rows));
        }
        out->exchange_ns[i] = median(tn);
    }
    float *rates[4] = {&out->lds_read_bpc, &out->lds_write_bpc, &out->l2_read_bpc, &out->global_write_bpc};
    const double bytes_per_rep[4] = {32768.0, 32768.0, 262144.0, 262144.0};
    for (int kind = 0; kind < 4; ++kind) {
        int k2 = kind, rp = kind < 2 ? 2000 : 200;
        float cpr = 0.f;
        if ((st = med(5, dim3(1), dim3(256), {&dev, &rate, &k2, &rp}, rp, nullptr, &cpr)) != CREDIT_OK) return st;
        *rates[kind] = (float)(bytes_per_rep[kind] / cpr);
    }
    out->clock_mhz = mhz_t > 0 ? (float)(mhz_c / mhz_t * 100.0) : 0.f;
    if (credit_check_errors(h, h->stream) != CREDIT_OK) out->errors += 1;
    return CREDIT_OK;
}
}  // namespace

credit_status_t credit_probe_primitives(credit_handle_t h, int reps, credit_primitives_t *out) {
    if (!h || !out || reps < 0) return CREDIT_ERR_INVALID_ARG;
    try {
        credit_status_t st = probe_all(h, reps, out);
        if (st == CREDIT_OK && out->errors == 0 && out->clock_mhz > 0.f && out->lds_read_bpc > 0.f &&
            out->global_write_bpc > 0.f) {
            // the analytic model's device terms from now on (Eq. (8))
            std::lock_guard<std::recursive_mutex> g(h->lock);
            h->cal.probed = true;
            h->cal.clock_hz = out->clock_mhz * 1e6;
            h->cal.slot_bpc = out->global_write_bpc;
            h->cal.lds_read_bpc = out->lds_read_bpc;
        }
        return st;
    } catch (...) {
        return CREDIT_ERR_HIP;
    }
}

credit_status_t credit_encode(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt, const float *x,
                              const float *row_scale, void *out, void *stream) {
    if (!h || M < 0 || N <= 0 || (int)dt < 0 || (int)dt > 2 || (M > 0 && (!x || !out))) return CREDIT_ERR_INVALID_ARG;
    if (M == 0) return CREDIT_OK;
    int64_t total = M * N;
    int grid = (int)std::min<int64_t>(8192, (total + 255) / 256);
    void *args[] = {&x, &row_scale, &out, &M, &N};
    return launch(encode_kernel(dt), grid, 256, 0, (hipStream_t)stream, args) == hipSuccess ? CREDIT_OK : CREDIT_ERR_HIP;
}

credit_status_t credit_decode(credit_handle_t h, int64_t M, int64_t N, credit_dtype_t dt, const void *in,
                              const float *row_scale, float *out, void *stream) {
    if (!h || M < 0 || N <= 0 || (int)dt < 0 || (int)dt > 2 || (M > 0 && (!in || !out))) return CREDIT_ERR_INVALID_ARG;
    if (M == 0) return CREDIT_OK;
    int64_t total = M * N;
    int grid = (int)std::min<int64_t>(8192, (total + 255) / 256);
    void *args[] = {&in, &row_scale, &out, &M, &N};
    return launch(decode_kernel(dt), grid, 256, 0, (hipStream_t)stream, args) == hipSuccess ? CREDIT_OK : CREDIT_ERR_HIP;
}

credit_status_t credit_check_errors(credit_handle_t h, void *stream) {
    if (!h) return CREDIT_ERR_INVALID_ARG;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return CREDIT_ERR_HIP;
    if (hipGetLastError() != hipSuccess) return CREDIT_ERR_HIP;
    unsigned flag = 0;
    if (hipMemcpy(&flag, h->errflag, 4, hipMemcpyDeviceToHost) != hipSuccess) return CREDIT_ERR_HIP;
    if (flag != 0) {
        if (hipMemset(h->errflag, 0, 4) != hipSuccess) return CREDIT_ERR_HIP;
        return CREDIT_ERR_TIMEOUT;
    }
    return CREDIT_OK;
}

credit_status_t credit_time_plan(credit_handle_t h, credit_op_t op, credit_dir_t dir, credit_dtype_t dt, int64_t M,
                                 int64_t N, const credit_plan_t *plan, int reps, int do_flush, float *median_us) {
    if (!h || !plan || !median_us || !valid_enum(op, dir, dt) || M <= 0 || N <= 0) return CREDIT_ERR_INVALID_ARG;
    try {
        return time_plan(h, kop(op, dir), dt, M, N, *plan, reps, do_flush, median_us);
    } catch (...) {
        return CREDIT_ERR_HIP;
    }
}

credit_status_t credit_time_plan_stats(credit_handle_t h, credit_op_t op, credit_dir_t dir, credit_dtype_t dt,
                                       int64_t M, int64_t N, const credit_plan_t *plan, int reps, int do_flush,
                                       credit_timing_t *out) {
    if (!h || !plan || !out || !valid_enum(op, dir, dt) || M <= 0 || N <= 0) return CREDIT_ERR_INVALID_ARG;
    try {
        float med = 0.f;
        return time_plan(h, kop(op, dir), dt, M, N, *plan, reps, do_flush, &med, out);
    } catch (...) {
        return CREDIT_ERR_HIP;
    }
}

credit_status_t credit_time_control(credit_handle_t h, credit_op_t op, credit_dir_t dir, credit_dtype_t dt,
                                    int64_t M, int64_t N, int32_t k, int reps, float *median_us) {
    if (!h || !median_us || !valid_enum(op, dir, dt) || M <= 0 || N <= 0) return CREDIT_ERR_INVALID_ARG;
    try {
        return time_control(h, kop(op, dir), dt, M, N, k, reps, median_us);
    } catch (...) {
        return CREDIT_ERR_HIP;
    }
}

credit_status_t credit_copy_bandwidth(credit_handle_t h, size_t bytes, int reps, float *gbps) {
    if (!h || !gbps || bytes < 4096) return CREDIT_ERR_INVALID_ARG;
    try {
        return copy_bw(h, bytes, reps, gbps);
    } catch (...) {
        return CREDIT_ERR_HIP;
    }
}

credit_status_t credit_model_delta(credit_handle_t h, credit_op_t op, credit_dir_t dir, credit_dtype_t dt, int64_t M,
                                   int64_t N, float t_base_us, const float *t_ctrl_us, float *out_delta_us) {
    if (!t_ctrl_us || !out_delta_us || !valid_enum(op, dir, dt) || M <= 0 || N <= 0 || !(t_base_us >= 0.f))
        return CREDIT_ERR_INVALID_ARG;
    if (h) {
        std::lock_guard<std::recursive_mutex> g(h->lock);
        model_delta(h, kop(op, dir), dt, M, N, t_base_us, t_ctrl_us, out_delta_us);
    } else {
        model_delta(nullptr, kop(op, dir), dt, M, N, t_base_us, t_ctrl_us, out_delta_us);
    }
    return CREDIT_OK;
}

credit_status_t credit_workload_info(credit_op_t op, credit_dir_t dir, credit_dtype_t dt, int recompute_stats,
                                     credit_workload_t *out) {
    if (!out || !valid_enum(op, dir, dt)) return CREDIT_ERR_INVALID_ARG;
    *out = workload(kop(op, dir), dt, recompute_stats != 0);
    return CREDIT_OK;
}

credit_status_t credit_plan_of_class(int32_t c, credit_plan_t *out) {
    if (!out || c < 0 || c >= CREDIT_NUM_PLANS) return CREDIT_ERR_INVALID_ARG;
    *out = class_plan(c);
    return CREDIT_OK;
}

credit_status_t credit_features(credit_op_t op, credit_dir_t dir, credit_dtype_t dt, int64_t M, int64_t N,
                                float *feat12) {
    if (!feat12 || !valid_enum(op, dir, dt) || M <= 0 || N <= 0) return CREDIT_ERR_INVALID_ARG;
    if (!core_op(kop(op, dir))) return CREDIT_ERR_UNSUPPORTED;
    features(kop(op, dir), dt, M, N, feat12);
    return CREDIT_OK;
}

int64_t credit_mlp_num_params(void) { return kMlpParams; }

static void reset_adam(credit_handle_t h) {
    std::fill(h->adam_m.begin(), h->adam_m.end(), 0.f);
    std::fill(h->adam_v.begin(), h->adam_v.end(), 0.f);
    h->adam_t = 0;
}

credit_status_t credit_mlp_set(credit_handle_t h, const float *params, const float *mu, const float *sd) {
    if (!h || !params || !mu || !sd) return CREDIT_ERR_INVALID_ARG;
    std::lock_guard<std::recursive_mutex> g(h->lock);
    for (int i = 0; i < kF; ++i)
        if (!(sd[i] > 0.f)) return CREDIT_ERR_INVALID_ARG;
    std::memcpy(h->params.data(), params, kMlpParams * 4);
    std::memcpy(h->mu, mu, kF * 4);
    std::memcpy(h->sd, sd, kF * 4);
    reset_adam(h);
    if (upload_infer(h) != CREDIT_OK) return CREDIT_ERR_HIP;
    h->has_model = true;
    h->plan_cache.clear();
    return CREDIT_OK;
}

credit_status_t credit_mlp_get(credit_handle_t h, float *params, float *mu, float *sd) {
    if (!h) return CREDIT_ERR_INVALID_ARG;
    std::lock_guard<std::recursive_mutex> g(h->lock);
    if (params) std::memcpy(params, h->params.data(), kMlpParams * 4);
    if (mu) std::memcpy(mu, h->mu, kF * 4);
    if (sd) std::memcpy(sd, h->sd, kF * 4);
    return CREDIT_OK;
}

credit_status_t credit_mlp_grad(credit_handle_t h, const float *feats, const float *targets, const uint8_t *mask,
                                int64_t n, float *loss, float *grad) {
    if (!h || !feats || !targets || !mask || n <= 0) return CREDIT_ERR_INVALID_ARG;
    std::lock_guard<std::recursive_mutex> g(h->lock);
    try {
        MlpDev d;
        if (!d.init(n) || !mlp_upload(h, d, feats, targets, mask)) return CREDIT_ERR_HIP;
        if (mlp_forward(d, h->stream) != hipSuccess || mlp_backward(d, h->stream) != hipSuccess) return CREDIT_ERR_HIP;
        if (hipStreamSynchronize(h->stream) != hipSuccess) return CREDIT_ERR_HIP;
        if (loss && hipMemcpy(loss, d.lmean, 4, hipMemcpyDeviceToHost) != hipSuccess) return CREDIT_ERR_HIP;
        if (grad && hipMemcpy(grad, d.g, kMlpParams * 4, hipMemcpyDeviceToHost) != hipSuccess) return CREDIT_ERR_HIP;
        return CREDIT_OK;
    } catch (...) {
        return CREDIT_ERR_HIP;
    }
}

credit_status_t credit_mlp_train(credit_handle_t h, const float *feats, const float *targets, const uint8_t *mask,
                                 int64_t n, int epochs, float lr, uint64_t seed, float *final_loss) {
    if (!h || !feats || !targets || !mask || n <= 0 || epochs < 0 || !(lr > 0.f)) return CREDIT_ERR_INVALID_ARG;
    std::lock_guard<std::recursive_mutex> g(h->lock);
    try {
        if (seed != 0) {
            // feature standardization from the training set
            for (int f = 0; f < kF; ++f) {
                double s = 0, s2 = 0;
                for (int64_t i = 0; i < n; ++i) s += feats[i * kF + f];
                double m = s / n;
                for (int64_t i = 0; i < n; ++i) s2 += (feats[i * kF + f] - m) * (feats[i * kF + f] - m);
                double sd = std::sqrt(s2 / n);
                h->mu[f] = (float)m;
                h->sd[f] = sd > 1e-6 ? (float)sd : 1.f;
            }
            // He initialisation, zero biases
            Rng r{seed};
            auto he = [&](size_t off, int O, int I) {
                double sc = std::sqrt(2.0 / I);
                for (int i = 0; i < O * I; ++i) h->params[off + i] = (float)(r.normal() * sc);
            };
            std::fill(h->params.begin(), h->params.end(), 0.f);
            he(oW1, kH, kF);
            he(oW2, kH, kH);
            he(oW3, kC, kH);
            reset_adam(h);
        }
        MlpDev d;
        if (!d.init(n) || !mlp_upload(h, d, feats, targets, mask)) return CREDIT_ERR_HIP;
        // Adam continues from the handle's moments and step count (zero after
        // a seeded initialisation, credit_mlp_set or a model without them)
        if (hipMemcpy(d.m, h->adam_m.data(), kMlpParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d.v, h->adam_v.data(), kMlpParams * 4, hipMemcpyHostToDevice) != hipSuccess)
            return CREDIT_ERR_HIP;
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        int64_t np = kMlpParams;
        double p1 = 1.0, p2 = 1.0;  // b1^t, b2^t by the same running products as the steps take
        for (int64_t t = 0; t < h->adam_t; ++t) {
            p1 *= b1;
            p2 *= b2;
        }
        for (int t = 1; t <= epochs; ++t) {
            if (mlp_forward(d, h->stream) != hipSuccess || mlp_backward(d, h->stream) != hipSuccess)
                return CREDIT_ERR_HIP;
            p1 *= b1;
            p2 *= b2;
            float bc1 = (float)(1.0 - p1), bc2 = (float)(1.0 - p2);
            float lr_ = lr, b1_ = b1, b2_ = b2, eps_ = eps;
            void *a[] = {&d.p, &d.g, &d.m, &d.v, &np, &lr_, &b1_, &b2_, &eps_, &bc1, &bc2};
            if (launch(mlp_kernel(6), blocks(np), 256, 0, h->stream, a) != hipSuccess) return CREDIT_ERR_HIP;
        }
        // loss at the final parameters
        if (mlp_forward(d, h->stream) != hipSuccess || mlp_backward(d, h->stream) != hipSuccess) return CREDIT_ERR_HIP;
        if (hipStreamSynchronize(h->stream) != hipSuccess) return CREDIT_ERR_HIP;
        if (hipMemcpy(h->params.data(), d.p, kMlpParams * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(h->adam_m.data(), d.m, kMlpParams * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(h->adam_v.data(), d.v, kMlpParams * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return CREDIT_ERR_HIP;
        h->adam_t += epochs;
        if (final_loss && hipMemcpy(final_loss, d.lmean, 4, hipMemcpyDeviceToHost) != hipSuccess)
            return CREDIT_ERR_HIP;
        if (upload_infer(h) != CREDIT_OK) return CREDIT_ERR_HIP;
        h->has_model = true;
        h->plan_cache.clear();
        return CREDIT_OK;
    } catch (...) {
        return CREDIT_ERR_HIP;
    }
}

credit_status_t credit_mlp_predict(credit_handle_t h, const float *feats, int64_t n, float *logits) {
    if (!h || !feats || !logits || n <= 0) return CREDIT_ERR_INVALID_ARG;
    std::lock_guard<std::recursive_mutex> g(h->lock);
    try {
        return mlp_predict_dev(h, feats, n, logits);
    } catch (...) {
        return CREDIT_ERR_HIP;
    }
}

static const char *kSchema = "f12-h64-h64-c7-v5";
static const char *kLibraryTag = "credit-mi355x-0.1.0";  // written into saved models (provenance)

credit_status_t credit_save_model(credit_handle_t h, const char *path) {
    if (!h || !path) return CREDIT_ERR_INVALID_ARG;
    std::lock_guard<std::recursive_mutex> g(h->lock);
    if (!h->has_model) return CREDIT_ERR_MODEL;
    FILE *f = std::fopen(path, "w");
    if (!f) return CREDIT_ERR_INVALID_ARG;
    std::string arch = h->arch.substr(0, h->arch.find(':'));
    std::fprintf(f, "CREDIT-MLP 2\narch %s\ncus %d\nschema %s\nlibrary %s\nclasses", arch.c_str(), h->cus, kSchema,
                 kLibraryTag);
    for (int c = 0; c < kC; ++c) {
        const credit_plan_t p = class_plan(c);
        std::fprintf(f, " %d:%d", (int)p.variant, (int)p.k);
    }
    std::fprintf(f, "\nmu");
    for (int i = 0; i < kF; ++i) std::fprintf(f, " %.9g", h->mu[i]);
    std::fprintf(f, "\nsd");
    for (int i = 0; i < kF; ++i) std::fprintf(f, " %.9g", h->sd[i]);
    std::fprintf(f, "\nparams %d\n", kMlpParams);
    for (int i = 0; i < kMlpParams; ++i) std::fprintf(f, "%.9g\n", h->params[i]);
    // Adam moments and step count, so that training resumes from the file
    std::fprintf(f, "adam %lld %d\n", (long long)h->adam_t, kMlpParams);
    for (int i = 0; i < kMlpParams; ++i) std::fprintf(f, "%.9g %.9g\n", h->adam_m[i], h->adam_v[i]);
    std::fprintf(f, "end\n");
    return std::fclose(f) == 0 ? CREDIT_OK : CREDIT_ERR_INVALID_ARG;
}

credit_status_t credit_load_model(credit_handle_t h, const char *path) {
    if (!h || !path) return CREDIT_ERR_INVALID_ARG;
    std::lock_guard<std::recursive_mutex> g(h->lock);
    h->has_model = false;
    h->plan_cache.clear();
    FILE *f = std::fopen(path, "r");
    if (!f) return CREDIT_ERR_MODEL;
    char arch[64] = {0}, schema[64] = {0}, tag[16] = {0}, library[64] = {0};
    int ver = 0, cus = 0, np = 0;
    bool ok = std::fscanf(f, "CREDIT-MLP %d arch %63s cus %d schema %63s", &ver, arch, &cus, schema) == 4;
    std::string want = h->arch.substr(0, h->arch.find(':'));
    ok = ok && (ver == 1 || ver == 2) && want == arch && cus == h->cus && std::strcmp(schema, kSchema) == 0;
    if (ok && ver == 2) {
        // the library that wrote it (provenance only) and the plan classes,
        // which must be this library's
        ok = std::fscanf(f, " library %63s classes", library) == 1;
        for (int c = 0; ok && c < kC; ++c) {
            int v = -1, k = -1;
            const credit_plan_t p = class_plan(c);
            ok = std::fscanf(f, " %d:%d", &v, &k) == 2 && v == (int)p.variant && k == (int)p.k;
        }
    }
    ok = ok && std::fscanf(f, " mu") == 0;
    float mu[kF], sd[kF];
    for (int i = 0; ok && i < kF; ++i) ok = std::fscanf(f, "%f", &mu[i]) == 1;
    ok = ok && std::fscanf(f, " sd") == 0;
    for (int i = 0; ok && i < kF; ++i) ok = std::fscanf(f, "%f", &sd[i]) == 1 && sd[i] > 0.f;
    ok = ok && std::fscanf(f, " params %d", &np) == 1 && np == kMlpParams;
    std::vector<float> p(kMlpParams);
    for (int i = 0; ok && i < kMlpParams; ++i) ok = std::fscanf(f, "%f", &p[i]) == 1 && std::isfinite(p[i]);
    std::vector<float> am(kMlpParams, 0.f), av(kMlpParams, 0.f);
    long long at = 0;
    if (ok && ver == 2) {
        int na = -1;
        ok = std::fscanf(f, " adam %lld %d", &at, &na) == 2 && at >= 0 && na == kMlpParams;
        for (int i = 0; ok && i < kMlpParams; ++i)
            ok = std::fscanf(f, "%f %f", &am[i], &av[i]) == 2 && std::isfinite(am[i]) && av[i] >= 0.f &&
                 std::isfinite(av[i]);
    }
    ok = ok && std::fscanf(f, "%15s", tag) == 1 && std::strcmp(tag, "end") == 0;
    std::fclose(f);
    if (!ok) return CREDIT_ERR_MODEL;
    std::memcpy(h->params.data(), p.data(), kMlpParams * 4);
    std::memcpy(h->mu, mu, sizeof(mu));
    std::memcpy(h->sd, sd, sizeof(sd));
    h->adam_m = am;
    h->adam_v = av;
    h->adam_t = at;
    if (upload_infer(h) != CREDIT_OK) return CREDIT_ERR_HIP;
    h->has_model = true;
    return CREDIT_OK;
}

credit_status_t credit_instance_info(credit_handle_t h, credit_op_t op, credit_dir_t dir, credit_dtype_t dt,
                                     int32_t vpt, int32_t rows, credit_instance_t *out) {
    if (!out || !valid_enum(op, dir, dt) || rows < 1) return CREDIT_ERR_INVALID_ARG;
    const int k_op = kop(op, dir);
    if (!instance_exists(k_op, dt, vpt)) return CREDIT_ERR_UNSUPPORTED;
    if (rows > 1 && !multirow_exists(k_op, dt, vpt, rows)) return CREDIT_ERR_UNSUPPORTED;
    const void *fn = instance_fn(k_op, dt, vpt, rows);
    if (!fn) return CREDIT_ERR_UNSUPPORTED;
    if (!h) {  // the register model only
        out->registers = out->private_bytes = out->per_cu = out->coresident_per_cu = -1;
        out->model_per_cu = model_waves(k_op, dt, vpt, rows);
        return CREDIT_OK;
    }
    std::lock_guard<std::recursive_mutex> g(h->lock);
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, fn) != hipSuccess) return CREDIT_ERR_HIP;
    out->registers = at.numRegs;
    out->private_bytes = (int32_t)at.localSizeBytes;
    out->per_cu = occupancy(h, fn, kBlockThreads, 0);
    out->model_per_cu = model_waves(k_op, dt, vpt, rows);
    auto it = h->coresident.find(fn);
    out->coresident_per_cu = it == h->coresident.end() ? -1 : it->second;
    return CREDIT_OK;
}

credit_status_t credit_set_option(credit_handle_t h, credit_option_t opt, int64_t value) {
    if (!h) return CREDIT_ERR_INVALID_ARG;
    std::lock_guard<std::recursive_mutex> g(h->lock);
    switch (opt) {
    case CREDIT_OPT_SPIN_LIMIT:
        if (value < 0) return CREDIT_ERR_INVALID_ARG;
        h->spin_limit = value;
        return CREDIT_OK;
    case CREDIT_OPT_TEST_DROP_PUBLISH: h->drop_publish = value != 0; return CREDIT_OK;
    case CREDIT_OPT_TEST_SKEW: h->skew = value != 0; return CREDIT_OK;
    case CREDIT_OPT_MAX_GROUPS:
        if (value < 0) return CREDIT_ERR_INVALID_ARG;
        h->max_groups = value;
        h->plan_cache.clear();
        return CREDIT_OK;
    case CREDIT_OPT_ROWS: {
        bool ok = value == 0 || value == 1;
        for (int r : kMrRows) ok |= value == r;
        if (!ok) return CREDIT_ERR_INVALID_ARG;
        h->rows_opt = (int)value;
        return CREDIT_OK;
    }
    }
    return CREDIT_ERR_INVALID_ARG;
}

credit_status_t credit_set_epoch(uint32_t next) {
    g_epoch.store(next == 0 ? 1 : next);
    return CREDIT_OK;
}

}  // extern "C"
