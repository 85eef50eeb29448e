/* Drives the host-only entry points of libcredit, whose host code is built
 * with AddressSanitizer and UndefinedBehaviorSanitizer: byte accounting,
 * shape features, plan classes and launch geometry, the register model of
 * every instance, the Eq. (9) model without a device, status strings,
 * argument checks, and handle creation (which fails cleanly where no GPU is
 * present).  Prints "host sanitize: ok" when every check held. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "../../include/credit.h"

static int failures = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            printf("check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                             \
        }                                                           \
    } while (0)

int main(void) {
    const long long Ms[] = {0, 1, 7, 1024, 16384, 1LL << 20};
    const long long Ns[] = {1, 15, 16, 1024, 4097, 65536, 524288, 4194304, 1LL << 25};
    const int vpts[] = {0, 1, 2, 4, 8, 12, 16, 24, 32, 48, 68, 100};
    const int rowss[] = {0, 1, 2, 4, 8};
    long long legal = 0;
    for (int op = -1; op <= 9; ++op)
        for (int dir = -1; dir <= 2; ++dir)
            for (int dt = -1; dt <= 3; ++dt) {
                const credit_op_t o = (credit_op_t)op;
                const credit_dir_t d = (credit_dir_t)dir;
                const credit_dtype_t t = (credit_dtype_t)dt;
                credit_workload_t w;
                for (int rc = 0; rc < 2; ++rc)
                    if (credit_workload_info(o, d, t, rc, &w) == CREDIT_OK)
                        CHECK(w.stages >= 1 && w.stages <= 4 && w.b_base >= w.b_staged && w.b_reread >= 0.f);
                CHECK(credit_workload_info(o, d, t, 0, NULL) != CREDIT_OK);
                for (unsigned i = 0; i < sizeof(vpts) / sizeof(vpts[0]); ++i)
                    for (unsigned r = 0; r < sizeof(rowss) / sizeof(rowss[0]); ++r) {
                        credit_instance_t inst;
                        memset(&inst, 0x5a, sizeof(inst));
                        if (credit_instance_info(NULL, o, d, t, vpts[i], rowss[r], &inst) == CREDIT_OK)
                            CHECK(inst.model_per_cu >= 1 && inst.model_per_cu <= 8 && inst.registers == -1);
                    }
                for (unsigned mi = 0; mi < sizeof(Ms) / sizeof(Ms[0]); ++mi)
                    for (unsigned ni = 0; ni < sizeof(Ns) / sizeof(Ns[0]); ++ni) {
                        const long long M = Ms[mi], N = Ns[ni];
                        float f[CREDIT_NUM_FEATURES];
                        if (credit_features(o, d, t, M, N, f) == CREDIT_OK)
                            for (int k = 0; k < CREDIT_NUM_FEATURES; ++k) CHECK(isfinite(f[k]));
                        for (int c = -1; c <= CREDIT_NUM_PLANS; ++c) {
                            credit_plan_t p;
                            if (credit_plan_of_class(c, &p) != CREDIT_OK) {
                                CHECK(c < 0 || c >= CREDIT_NUM_PLANS);
                                continue;
                            }
                            int32_t grid = -7, block = -7, vpt = -7, per_cu = -7, rows = -7;
                            if (credit_plan_geometry(NULL, o, d, t, M, N, &p, &grid, &block, &vpt, &per_cu, &rows) ==
                                CREDIT_OK) {
                                ++legal;
                                CHECK((grid >= 1 || M == 0) && block >= 64 && per_cu >= 1 && rows >= 1);
                            }
                            (void)credit_plan_geometry(NULL, o, d, t, M, N, &p, NULL, NULL, NULL, NULL, NULL);
                        }
                        CHECK(credit_plan_geometry(NULL, o, d, t, M, N, NULL, NULL, NULL, NULL, NULL, NULL) !=
                              CREDIT_OK);
                        const float ctrl[5] = {1.f, 1.5f, 2.f, 3.f, 5.f};
                        float delta[5];
                        if (credit_model_delta(NULL, o, d, t, M, N, 100.f, ctrl, delta) == CREDIT_OK)
                            for (int k = 0; k < 5; ++k) CHECK(isfinite(delta[k]) || delta[k] == -INFINITY);
                    }
            }
    CHECK(legal > 1000);
    for (int s = -1; s <= 8; ++s) CHECK(credit_status_string((credit_status_t)s) != NULL);
    CHECK(credit_version() != NULL && strlen(credit_version()) > 0);
    CHECK(credit_mlp_num_params() > 0);
    CHECK(credit_destroy(NULL) == CREDIT_ERR_INVALID_ARG);
    CHECK(credit_load_model(NULL, "missing.txt") == CREDIT_ERR_INVALID_ARG);
    CHECK(credit_create(0, NULL) == CREDIT_ERR_INVALID_ARG);
    credit_handle_t h = NULL;
    const credit_status_t st = credit_create(0, &h);
    if (st == CREDIT_OK) {
        CHECK(h != NULL);
        CHECK(credit_destroy(h) == CREDIT_OK);
    } else {
        CHECK(h == NULL);
    }
    if (failures) {
        printf("host sanitize: %d checks failed\n", failures);
        return 1;
    }
    printf("host sanitize: ok (%lld legal plan geometries)\n", legal);
    return 0;
}
