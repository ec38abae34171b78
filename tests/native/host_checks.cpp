// Host-side checks of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of every library source (no
// device code, no GPU): collocation tables, workspace sizing, argument
// validation of every entry point on seeded random and on edge-case
// arguments, plan and batch creation over a placeholder workspace address
// (never dereferenced) and their destruction.  Any sanitizer report aborts
// the run; a failed check prints it and exits 1.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "isdc.h"

static int failures = 0;
#define CHECK(cond)                                                            \
    do {                                                                       \
        if (!(cond)) {                                                         \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

// 64-bit linear congruential generator (Knuth's MMIX constants)
static uint64_t state = 20240601ull;
static uint64_t next_u64() {
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return state;
}
static int pick(int lo, int hi) { return lo + (int)((next_u64() >> 33) % (uint64_t)(hi - lo + 1)); }
static double pick_double() {
    const double vals[] = {0.0, -1.0, 1e-12, 1e-3, 0.5, 1.0, 100.0, NAN, INFINITY, -INFINITY, 1e300};
    return vals[pick(0, 10)];
}

static bool known_status(int rc) { return rc <= 0 && rc >= ISDC_E_UNSUPPORTED; }

static isdc_problem problem(int dim, int n) {
    isdc_problem p;
    std::memset(&p, 0, sizeof(p));
    p.dim = dim;
    for (int a = 0; a < 3; ++a) p.n[a] = a < dim ? n : 1;
    p.nu = 1.0;
    p.fe_kind = ISDC_FE_ZERO;
    p.stencil = ISDC_STENCIL_2ND;
    p.bc = ISDC_BC_DIRICHLET;
    return p;
}

int main() {
    void* const fake = (void*)(uintptr_t)(1ull << 40);  // 256-byte aligned, never dereferenced
    // tables: every node family and M; rows of S sum to the node spacing
    for (int kind = 0; kind <= 2; ++kind)
        for (int M = 0; M <= 10; ++M) {
            double tau[ISDC_MAX_M], Q[ISDC_MAX_M * ISDC_MAX_M], S[ISDC_MAX_M * ISDC_MAX_M], b[ISDC_MAX_M];
            const int rc = isdc_tables(kind, M, tau, Q, S);
            const bool valid = (kind == ISDC_NODES_LOBATTO ? M >= 2 : M >= 1) && M <= ISDC_MAX_M;
            CHECK((rc == ISDC_OK) == valid);
            if (rc != ISDC_OK) {
                CHECK(std::strlen(isdc_last_error()) > 0);
                continue;
            }
            double prev = 0.0;
            for (int m = 0; m < M; ++m) {
                double row = 0.0;
                for (int j = 0; j < M; ++j) row += S[m * M + j];
                CHECK(std::fabs(row - (tau[m] - prev)) < 1e-14);
                prev = tau[m];
            }
            CHECK(isdc_end_weights(kind, M, b) == ISDC_OK);
            double sum = 0.0;
            for (int j = 0; j < M; ++j) sum += b[j];
            CHECK(std::fabs(sum - 1.0) < 1e-14);
        }
    // random problems and parameters: sizing never fails outside the status set
    for (int trial = 0; trial < 20000; ++trial) {
        isdc_problem pb = problem(pick(0, 4), (1 << pick(0, 14)) - pick(0, 2));
        if (pick(0, 5) == 0) pb.n[pick(0, 2)] = pick(-1, 40);
        pb.nu = pick_double();
        pb.fe_kind = pick(-1, 3);
        pb.stencil = pick(-1, 2);
        pb.bc = pick(-1, 2);
        isdc_params pr;
        CHECK(isdc_default_params(&pr) == ISDC_OK);
        pr.node_kind = pick(-1, 3);
        pr.M = pick(-1, 11);
        pr.vcycles = pick(-1, 70);
        pr.inner_tol = pick_double();
        pr.early_exit = pick(-1, 2);
        pr.sdc_tol = pick_double();
        pr.max_sweeps = pick(-1, 3) * 50000;
        pr.smoother = pick(-1, 2);
        pr.nu_pre = pick(-1, 9);
        pr.nu_post = pick(-1, 9);
        pr.precision = pick(-1, 2);
        pr.guess = pick(-1, 3);
        pr.levels = pick(0, 3);
        size_t bytes = 0;
        const int rc = isdc_workspace_bytes(&pb, &pr, &bytes);
        CHECK(known_status(rc));
        if (rc != ISDC_OK) {
            CHECK(std::strlen(isdc_last_error()) > 0);
            isdc_plan* plan = (isdc_plan*)fake;
            CHECK(isdc_create(&pb, &pr, fake, bytes, &plan) == rc);
            continue;
        }
        CHECK(bytes > 0);
        isdc_plan* plan = nullptr;
        CHECK(isdc_create(&pb, &pr, fake, bytes - 1, &plan) == ISDC_E_WORKSPACE);
        CHECK(isdc_create(&pb, &pr, fake, bytes, &plan) == ISDC_OK && plan);
        if (!plan) continue;
        isdc_stats st;
        CHECK(isdc_get_stats(plan, &st) == ISDC_OK && st.sweeps == 0);
        int32_t shapes[32], nl = 0;
        CHECK(isdc_get_tile_shapes(plan, shapes, 32, &nl) == ISDC_OK);
        CHECK(isdc_set_tile_shapes(plan, shapes, nl) == ISDC_OK);
        CHECK(isdc_set_tile_shapes(plan, shapes, nl + 1) == ISDC_E_INVAL);
        double r = 0.0;
        CHECK(isdc_sweep(plan, nullptr, &r) == ISDC_E_INVAL);          // no step in progress
        CHECK(isdc_end(plan, (double*)fake, nullptr) == ISDC_E_INVAL);
        CHECK(isdc_begin(plan, (const double*)fake, -1.0, nullptr) == ISDC_E_INVAL);
        CHECK(isdc_step(plan, nullptr, 1e-3, nullptr, &st) == ISDC_E_INVAL);
        CHECK(isdc_vcycle(plan, -1.0, ISDC_PREC_FP64, fake, fake, 1, nullptr, nullptr) == ISDC_E_INVAL);
        CHECK(isdc_mg_op(plan, 99, 0, 1.0, ISDC_PREC_FP64, fake, fake, fake, nullptr, nullptr) == ISDC_E_INVAL);
        CHECK(isdc_probe_arm(plan, 99, 0, 1, 1) != ISDC_OK);
        CHECK(isdc_probe_read(plan, nullptr, nullptr, nullptr) == ISDC_E_INVAL);  // nothing armed
        isdc_destroy(plan);
    }
    // fixed-instance batches over the placeholder address
    for (int trial = 0; trial < 200; ++trial) {
        const int count = pick(1, 6);
        std::vector<isdc_problem> probs;
        std::vector<isdc_params> pars;
        for (int i = 0; i < count; ++i) {
            probs.push_back(problem(2, (1 << pick(2, 8)) - 1));
            isdc_params pr;
            isdc_default_params(&pr);
            pr.M = pick(2, 5);
            pr.precision = pick(0, 3) == 0 ? ISDC_PREC_FP64 : ISDC_PREC_MIXED;
            pars.push_back(pr);
        }
        size_t bytes = 0;
        const int rc = isdc_batch_bytes(count, probs.data(), pars.data(), &bytes);
        CHECK(known_status(rc));
        if (rc != ISDC_OK) continue;
        isdc_batch* b = nullptr;
        CHECK(isdc_batch_create(count, probs.data(), pars.data(), fake, bytes - 1, &b) == ISDC_E_WORKSPACE);
        CHECK(isdc_batch_create(count, probs.data(), pars.data(), fake, bytes, &b) == ISDC_OK && b);
        std::vector<double*> us(count, nullptr);
        std::vector<double> dts(count, 1e-3);
        CHECK(isdc_batch_step(b, us.data(), dts.data(), nullptr, nullptr, nullptr) == ISDC_E_INVAL);
        isdc_batch_destroy(b);
    }
    // the entry point without allocation rejects before any device work
    {
        isdc_problem big = problem(2, 1023);
        isdc_params pr;
        isdc_default_params(&pr);
        pr.M = 5;
        isdc_stats st;
        CHECK(isdc_step_noalloc(&big, &pr, (double*)fake, 1e-3, nullptr, &st) == ISDC_E_WORKSPACE);
        isdc_problem small = problem(2, 63);
        CHECK(isdc_step_noalloc(&small, &pr, nullptr, 1e-3, nullptr, &st) == ISDC_E_INVAL);
        CHECK(isdc_step_noalloc(nullptr, &pr, (double*)fake, 1e-3, nullptr, &st) == ISDC_E_INVAL);
    }
    isdc_destroy(nullptr);
    isdc_batch_destroy(nullptr);
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
