// Host-only error paths of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side of every translation unit:
// argument validation, NULL handles and pointers, the thread-local error
// message and the host-side filter derivation.  No call here reaches the
// device: each one returns its status before any device work, so the program
// runs on a machine without a GPU.  Exit status 0 = every check held.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/kpdhg.h"

static int g_fail = 0;

static void expect(int got, int want, const char* what) {
    const char* msg = kp_last_error();
    if (got != want) {
        std::printf("FAIL %s: status %d, expected %d (%s)\n", what, got, want, msg ? msg : "(null)");
        ++g_fail;
        return;
    }
    if (want != KP_OK && (!msg || !*msg)) {
        std::printf("FAIL %s: no error message\n", what);
        ++g_fail;
    }
}

static int validate(int ndim, const int64_t* shape, int64_t C, int64_t M, const void* coords, const void* maps,
                    float alpha, int W, const kp_tuning* t) {
    return nufft_plan_validate(ndim, shape, C, M, coords, maps, alpha, W, t);
}

int main() {
    const float dummy_coords[4] = {0.f, 0.f, 0.f, 0.f};  // never dereferenced by validation
    const float* coords = dummy_coords;
    const int64_t s2[2] = {16, 16}, s3[3] = {16, 16, 16};
    const int64_t odd[2] = {15, 16}, tiny[2] = {0, 16}, huge[2] = {8192, 16};
    const int64_t big3[3] = {2048, 2048, 2048};

    // ---- argument validation (Problem Setup sizes, Experiments' alpha and W)
    expect(validate(2, s2, 1, 10, coords, nullptr, 1.25f, 4, nullptr), KP_OK, "valid 2D");
    expect(validate(3, s3, 1, 10, coords, nullptr, 2.0f, 6, nullptr), KP_OK, "valid 3D");
    expect(validate(1, s2, 1, 10, coords, nullptr, 1.25f, 4, nullptr), KP_ERR_INVALID_ARG, "ndim 1");
    expect(validate(4, s3, 1, 10, coords, nullptr, 1.25f, 4, nullptr), KP_ERR_INVALID_ARG, "ndim 4");
    expect(validate(2, nullptr, 1, 10, coords, nullptr, 1.25f, 4, nullptr), KP_ERR_INVALID_ARG, "shape NULL");
    expect(validate(2, odd, 1, 10, coords, nullptr, 1.25f, 4, nullptr), KP_ERR_INVALID_ARG, "odd N");
    expect(validate(2, tiny, 1, 10, coords, nullptr, 1.25f, 4, nullptr), KP_ERR_INVALID_ARG, "N = 0");
    expect(validate(2, huge, 1, 10, coords, nullptr, 1.25f, 4, nullptr), KP_ERR_INVALID_ARG, "N > 4096");
    expect(validate(2, s2, 0, 10, coords, nullptr, 1.25f, 4, nullptr), KP_ERR_INVALID_ARG, "C = 0");
    expect(validate(2, s2, 17, 10, coords, dummy_coords, 1.25f, 4, nullptr), KP_ERR_UNSUPPORTED, "C = 17");
    expect(validate(2, s2, 1, 0, coords, nullptr, 1.25f, 4, nullptr), KP_ERR_INVALID_ARG, "M = 0");
    expect(validate(2, s2, 1, (int64_t)1 << 27, coords, nullptr, 1.25f, 4, nullptr), KP_ERR_UNSUPPORTED, "M = 2^27");
    expect(validate(2, s2, 1, 10, nullptr, nullptr, 1.25f, 4, nullptr), KP_ERR_INVALID_ARG, "coords NULL");
    expect(validate(2, s2, 3, 10, coords, nullptr, 1.25f, 4, nullptr), KP_ERR_INVALID_ARG, "maps NULL, C = 3");
    expect(validate(2, s2, 1, 10, coords, nullptr, 1.0f, 4, nullptr), KP_ERR_INVALID_ARG, "alpha 1.0");
    expect(validate(2, s2, 1, 10, coords, nullptr, 2.5f, 4, nullptr), KP_ERR_INVALID_ARG, "alpha 2.5");
    expect(validate(2, s2, 1, 10, coords, nullptr, std::nanf(""), 4, nullptr), KP_ERR_INVALID_ARG, "alpha NaN");
    expect(validate(2, s2, 1, 10, coords, nullptr, 1.25f, 3, nullptr), KP_ERR_INVALID_ARG, "W 3");
    expect(validate(2, s2, 1, 10, coords, nullptr, 1.25f, 10, nullptr), KP_ERR_INVALID_ARG, "W 10");
    expect(validate(3, big3, 1, 10, coords, nullptr, 1.25f, 4, nullptr), KP_ERR_UNSUPPORTED, "grid >= 2^31");
    const int64_t s4[2] = {2, 2};
    expect(validate(2, s4, 1, 10, coords, nullptr, 1.25f, 8, nullptr), KP_ERR_UNSUPPORTED, "grid < W");
    kp_tuning t;
    std::memset(&t, 0, sizeof(t));
    t.bin_size[0] = 7;  // 20-cell grid of N = 16 at alpha 1.25
    expect(validate(2, s2, 1, 10, coords, nullptr, 1.25f, 4, &t), KP_ERR_INVALID_ARG, "bin size not dividing G");
    std::memset(&t, 0, sizeof(t));
    t.max_chunk = -1;
    expect(validate(2, s2, 1, 10, coords, nullptr, 1.25f, 4, &t), KP_ERR_INVALID_ARG, "negative max_chunk");

    // ---- nufft_plan refuses the same arguments before any device work
    kp_plan_t plan = reinterpret_cast<kp_plan_t>(0x1);
    expect(nufft_plan(nullptr, 2, s2, 1, 10, coords, nullptr, 1.25f, 4, nullptr, nullptr), KP_ERR_INVALID_ARG,
           "plan out NULL");
    expect(nufft_plan(&plan, 2, odd, 1, 10, coords, nullptr, 1.25f, 4, nullptr, nullptr), KP_ERR_INVALID_ARG,
           "plan odd N");
    if (plan != nullptr) {
        std::printf("FAIL plan handle not cleared on error\n");
        ++g_fail;
    }

    // ---- NULL handles and pointers
    float p[4];
    float lm = 0.f;
    kp_pdhg_opts op;
    std::memset(&op, 0, sizeof(op));
    op.iters = 1;
    kp_plan_info info;
    expect(nufft_forward(nullptr, p, p, nullptr), KP_ERR_INVALID_ARG, "forward NULL plan");
    expect(nufft_adjoint(nullptr, p, p, nullptr), KP_ERR_INVALID_ARG, "adjoint NULL plan");
    expect(precond_build(nullptr, KP_PRECOND_SC, p, nullptr), KP_ERR_INVALID_ARG, "precond NULL plan");
    expect(precond_build(nullptr, KP_PRECOND_DCF, p, nullptr), KP_ERR_INVALID_ARG, "DCF precond NULL plan");
    expect(pdhg_lambda_max(nullptr, nullptr, KP_PRECOND_NONE, 30, &lm, nullptr), KP_ERR_INVALID_ARG,
           "lambda_max NULL plan");
    expect(pdhg_solve(nullptr, p, nullptr, KP_PRECOND_NONE, &op, p, nullptr, nullptr), KP_ERR_INVALID_ARG,
           "solve NULL plan");
    expect(l2_dual_cg(nullptr, p, nullptr, KP_PRECOND_NONE, 1e-3f, 1, p, nullptr, nullptr, nullptr),
           KP_ERR_INVALID_ARG, "dual cg NULL plan");
    expect(nufft_plan_info(nullptr, &info), KP_ERR_INVALID_ARG, "info NULL plan");
    expect(nufft_plan_sort(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr), KP_ERR_INVALID_ARG,
           "sort NULL plan");
    expect(nufft_plan_grid_coords(nullptr, p, nullptr), KP_ERR_INVALID_ARG, "grid coords NULL plan");
    expect(nufft_stage(nullptr, 0, 1, nullptr), KP_ERR_INVALID_ARG, "stage NULL plan");
    expect(pdhg_unrolled_forward(nullptr, p, nullptr, 0, p, 1, 1, nullptr, p, p, nullptr), KP_ERR_INVALID_ARG,
           "unrolled forward NULL plan");
    expect(nufft_batch_info(nullptr, 0, &info, nullptr), KP_ERR_INVALID_ARG, "batch info NULL");
    expect(pdhg_solve_batch(nullptr, nullptr, nullptr, 0, &op, nullptr, nullptr, nullptr), KP_ERR_INVALID_ARG,
           "batch solve NULL");
    nufft_destroy(nullptr);
    nufft_batch_destroy(nullptr);

    // ---- the host-side db4 derivation (Daubechies' N = 4 filter)
    double h[8];
    expect(kp_db4_filter(h), KP_OK, "db4 filter");
    double sum = 0, sq = 0;
    for (double v : h) {
        sum += v;
        sq += v * v;
    }
    if (std::fabs(sum - std::sqrt(2.0)) > 1e-12 || std::fabs(sq - 1.0) > 1e-12) {
        std::printf("FAIL db4 sums %.17g %.17g\n", sum, sq);
        ++g_fail;
    }
    expect(kp_db4_filter(nullptr), KP_ERR_INVALID_ARG, "db4 NULL");

    std::printf("%s: %d failed checks\n", g_fail ? "FAIL" : "OK", g_fail);
    return g_fail ? 1 : 0;
}
