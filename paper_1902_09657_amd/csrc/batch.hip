// Batched form: many independent 2D slices with uneven image sizes and
// trajectories solved together.  Every phase of a PDHG iteration (each of the
// two forward FFT passes, interpolation with the dual update, spreading,
// partial-tile reduction, each of the two inverse FFT passes with the primal
// update) is ONE kernel launch over all slices and grid lengths, driven by
// per-slice descriptor tables; the whole K iteration loop is captured once
// into a HIP graph and replayed.
//
// Tile shapes and split sizes come from a small autotuner that times the
// spreading and interpolation kernels of candidate tilings on each slice
// size class and caches the winner per (shape, coils, width, oversampling,
// sample-count class).
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

#include "kp_internal.h"

namespace kp {

// ------------------------------------------------------------- autotuner
typedef std::tuple<int64_t, int64_t, int64_t, int64_t, int, int, int> TuneKey;
static std::map<TuneKey, kp_tuning> g_tune_cache;
static std::mutex g_tune_mu;

static float time_stages(Plan& P, hipStream_t s) {
    hipEvent_t e0, e1;
    KP_HIP(hipEventCreate(&e0));
    KP_HIP(hipEventCreate(&e1));
    // warm
    InterpArgs ia{};
    ia.mode = IO_INTERNAL;
    ia.out = P.kint3.as<float2>();
    interp(P, P.bufA.as<float2>(), ia, s);
    spread_to_grid(P, P.kint.as<float2>(), (int)P.C, s);
    KP_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r) {
        interp(P, P.bufB.as<float2>(), ia, s);
        spread_to_grid(P, P.kint.as<float2>(), (int)P.C, s);
    }
    KP_HIP(hipEventRecord(e1, s));
    KP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    KP_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

static int64_t pow2_class(int64_t m) {
    int64_t c = 1;
    while (c < m) c <<= 1;
    return c;
}

kp_tuning autotune(int ndim, const int64_t* shape, int64_t C, int64_t M, const float* coords, const void* maps,
                   float alpha, int W, hipStream_t s) {
    const TuneKey key(shape[0], shape[1], ndim == 3 ? shape[2] : 0, C * 1000000 + pow2_class(M), W,
                      (int)(alpha * 1000.f), ndim);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return it->second;
    }
    std::vector<kp_tuning> cands;
    const int CG = C % 4 == 0 ? 4 : (C % 2 == 0 ? 2 : 1);
    const int ncg = (int)(C / CG);
    // split sizes for slices that run together in one launch (throughput, not
    // one slice's latency: 64 to 256 entries were up to 17 % slower there)
    const int chunks[] = {512, 1024, 2048};
    if (ndim == 2) {
        // spreading tiles b0 lines x 4 or 2 cells; sort / interpolation tiles
        // b0 x the default depth
        for (int b0 : {16, 32, 64}) {
            if (b0 * ncg > 256) continue;
            for (int depth : {4, 2}) {
                for (int ch : chunks) {
                    kp_tuning t{};
                    t.bin_size[0] = b0;
                    t.spread_bin_size[0] = b0;
                    t.spread_bin_size[1] = depth;
                    t.max_chunk = ch;
                    cands.push_back(t);
                }
            }
        }
    } else {
        for (int b : {4, 8}) {
            for (int ch : chunks) {
                kp_tuning t{};
                t.bin_size[0] = b;
                t.bin_size[1] = 8;
                t.max_chunk = ch;
                cands.push_back(t);
            }
        }
    }
    kp_tuning best{};
    float best_ms = 1e30f;
    for (const kp_tuning& t : cands) {
        std::unique_ptr<Plan> P;
        try {
            // bin sizes that do not divide the grid are skipped
            P.reset(create_plan(ndim, shape, C, M, coords, maps, alpha, W, &t, s, maps == nullptr && C > 1));
        } catch (const Error&) {
            continue;
        }
        const float ms = time_stages(*P, s);
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = best;
    return best;
}

// ------------------------------------------------------------- batch object
struct Batch {
    std::vector<std::unique_ptr<Plan>> plans;
    hipStream_t cap = nullptr;  // capture stream
    int C = 0;
    bool fast = false;          // all slices fit the one-launch-per-phase kernels
    // cached graph
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int g_K = -1, g_pkind = -1;
    float g_lambda = -1.f;
    DevBuf desc;                // descriptor tables (device)
    ~Batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

// host-side layout of the device descriptor buffer
struct DescLayout {
    size_t fA, fB, aA, aB, it, sp, hv, hl;   // byte offsets
    size_t sfA, sfB, saA, saB, sit, ssp;     // block-start arrays
    size_t total;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static DescLayout desc_layout(int n, int K, int nh) {
    DescLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    L.fA = take(sizeof(FftPass) * n);
    L.fB = take(sizeof(FftPass) * n);
    L.aA = take(sizeof(FftPass) * n);
    L.aB = take(sizeof(FftPass) * n * K);
    L.it = take(sizeof(InterpArgs) * n * K);
    L.sp = take(sizeof(SpreadArgs) * n);
    L.hv = take(sizeof(int2) * std::max(nh, 1));
    L.hl = take(sizeof(int4*) * n);
    L.sfA = take(sizeof(int64_t) * (n + 1));
    L.sfB = take(sizeof(int64_t) * (n + 1));
    L.saA = take(sizeof(int64_t) * (n + 1));
    L.saB = take(sizeof(int64_t) * (n + 1));
    L.sit = take(sizeof(int64_t) * (n + 1));
    L.ssp = take(sizeof(int64_t) * (n + 1));
    L.total = o;
    return L;
}

static void capture_fast(Batch& B, const kp_pdhg_opts& op, int p_kind, hipStream_t s) {
    const int n = (int)B.plans.size();
    const int K = op.iters;
    const int C = B.C;
    std::vector<FftPass> fA(n), fB(n), aA(n), aB((size_t)n * K);
    std::vector<InterpArgs> it((size_t)n * K);
    std::vector<SpreadArgs> sp(n);
    std::vector<int2> hv;
    std::vector<const int4*> hl(n);
    std::vector<int64_t> sfA, sfB, saA, saB, sit(n + 1, 0), ssp(n + 1, 0);
    int spread_thr = 64;
    size_t spread_lds = 0;
    int zm_max = 4;  // register line of the batched spreading kernel: the deepest slice's
    for (int i = 0; i < n; ++i) {
        Plan& P = *B.plans[i];
        float* sig = P.sched.as<float>();
        float* tau = sig + 8192;
        float* th = tau + 8192;
        const float* pint = p_kind == KP_PRECOND_NONE ? nullptr : P.pint.as<float>();
        FwdOpts fo;
        std::vector<FftPass> fw = forward_passes(P, P.img[1].as<float2>(), fo);
        fA[i] = fw[0];
        fB[i] = fw[1];
        for (int k = 0; k < K; ++k) {
            AdjOpts ao;
            ao.ex = P.img[0].as<float2>();
            ao.exbar = P.img[1].as<float2>();
            ao.tau = tau + k;
            ao.theta = th + k;
            ao.lambda = op.lambda;
            ao.epi = EPI_L2;
            std::vector<FftPass> ad = adjoint_passes(P, P.bufA.as<float2>(), P.img[2].as<float2>(), ao);
            if (k == 0) aA[i] = ad[0];
            aB[(size_t)k * n + i] = ad[1];
            InterpArgs ia{};
            ia.mode = IO_DUAL;
            ia.u = P.kint.as<float2>();
            ia.y = P.kint2.as<float2>();
            ia.p = pint;
            ia.p_mc = p_kind == KP_PRECOND_MC ? 1 : 0;
            ia.sigma = sig + k;
            it[(size_t)k * n + i] = interp_args(P, fw[1].out, ia);
        }
        sp[i] = spread_args(P, P.kint.as<float2>(), C);
        for (int h = 0; h < P.heavy_tiles; ++h) hv.push_back(make_int2(i, h));
        hl[i] = P.heavy_list.as<int4>();
        sit[i + 1] = sit[i] + (P.M * (C / 4) + 255) / 256;
        ssp[i + 1] = ssp[i] + P.nwork;
        spread_thr = std::max(spread_thr, ((spread_threads(2, P.Bs, C) + 63) / 64) * 64);
        zm_max = std::max(zm_max, spread_zm(2, P.Bs));
    }
    for (int i = 0; i < n; ++i) {
        const Plan& P = *B.plans[i];
        spread_lds = std::max(spread_lds, spread_lds_bytes(2, P.W, P.Bs, C, zm_max));
    }
    // FFT phases: one persistent launch each over the passes of every slice,
    // sorted by transform length; lines longer than 206 rows use 16-column
    // blocks (54 KB of LDS at 400) and shorter ones 32 (the passes along the
    // coils keep the coil count as their column block), LDS sized for the
    // largest column block of the phase
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return B.plans[x]->G[0] < B.plans[y]->G[0]; });
    struct Phase { int map; size_t lds; };
    Phase ph[4];
    {
        std::vector<FftPass> tA(n), tB(n), tC(n), tD((size_t)n * K);
        std::vector<int64_t> cA(n + 1, 0), cB(n + 1, 0), cC(n + 1, 0), cD(n + 1, 0);
        // the map passes (fA, aB) run along the coils: their column block is
        // the same for every slice
        const int nc_map[4] = {fA[0].Ob * fA[0].Ib, 0, 0, aB[0].Ob * aB[0].Ib};
        auto shape = [&](FftPass fp, int q) {
            const int nc = fft_mixed_columns(fp.L, nc_map[q]);
            if (nc_map[q] == 0 && fp.Ob == 1) fp.Ib = nc;
            return fp;
        };
        for (int q = 0; q < 4; ++q) ph[q] = Phase{nc_map[q], 0};
        for (int j = 0; j < n; ++j) {
            const int i = ord[j];
            tA[j] = shape(fA[i], 0);
            tB[j] = shape(fB[i], 1);
            tC[j] = shape(aA[i], 2);
            for (int k = 0; k < K; ++k) tD[(size_t)k * n + j] = shape(aB[(size_t)k * n + i], 3);
            cA[j + 1] = cA[j] + fft_pass_blocks(tA[j]);
            cB[j + 1] = cB[j] + fft_pass_blocks(tB[j]);
            cC[j + 1] = cC[j] + fft_pass_blocks(tC[j]);
            cD[j + 1] = cD[j] + fft_pass_blocks(tD[j]);
            const FftPass* t4[4] = {&tA[j], &tB[j], &tC[j], &tD[j]};
            for (int q = 0; q < 4; ++q)
                ph[q].lds = std::max(ph[q].lds, sizeof(float2) * (size_t)t4[q]->L * (t4[q]->Ob * t4[q]->Ib + 1));
        }
        fA.swap(tA);
        fB.swap(tB);
        aA.swap(tC);
        aB.swap(tD);
        sfA.swap(cA);
        sfB.swap(cB);
        saA.swap(cC);
        saB.swap(cD);
    }
    const int nh = (int)hv.size();
    const DescLayout L = desc_layout(n, K, nh);
    B.desc.alloc(L.total);
    char* d = (char*)B.desc.p;
    auto up = [&](size_t off, const void* src, size_t bytes) {
        if (bytes) KP_HIP(hipMemcpy(d + off, src, bytes, hipMemcpyHostToDevice));
    };
    up(L.fA, fA.data(), sizeof(FftPass) * n);
    up(L.fB, fB.data(), sizeof(FftPass) * n);
    up(L.aA, aA.data(), sizeof(FftPass) * n);
    up(L.aB, aB.data(), sizeof(FftPass) * n * K);
    up(L.it, it.data(), sizeof(InterpArgs) * n * K);
    up(L.sp, sp.data(), sizeof(SpreadArgs) * n);
    up(L.hv, hv.data(), sizeof(int2) * nh);
    up(L.hl, hl.data(), sizeof(int4*) * n);
    up(L.sfA, sfA.data(), sizeof(int64_t) * (n + 1));
    up(L.sfB, sfB.data(), sizeof(int64_t) * (n + 1));
    up(L.saA, saA.data(), sizeof(int64_t) * (n + 1));
    up(L.saB, saB.data(), sizeof(int64_t) * (n + 1));
    up(L.sit, sit.data(), sizeof(int64_t) * (n + 1));
    up(L.ssp, ssp.data(), sizeof(int64_t) * (n + 1));
    const KbParams kb = B.plans[0]->kb;
    // one launch per FFT phase over every slice's pass
    auto fft_phase = [&](size_t tab, size_t starts, const std::vector<int64_t>& st, size_t shift, const Phase& q) {
        launch_fft_batch_mixed((const FftPass*)(d + tab) + shift, (const int64_t*)(d + starts), n, st[n], q.map, q.lds,
                               B.cap);
    };

    if (B.exec) (void)hipGraphExecDestroy(B.exec);
    if (B.graph) (void)hipGraphDestroy(B.graph);
    B.exec = nullptr;
    B.graph = nullptr;
    KP_HIP(hipStreamBeginCapture(B.cap, hipStreamCaptureModeRelaxed));
    try {
        for (int k = 0; k < K; ++k) {
            fft_phase(L.fA, L.sfA, sfA, 0, ph[0]);
            fft_phase(L.fB, L.sfB, sfB, 0, ph[1]);
            launch_interp_batch((const InterpArgs*)(d + L.it) + (size_t)k * n, (const int64_t*)(d + L.sit), n, sit[n],
                                kb, B.cap);
            launch_spread_batch((const SpreadArgs*)(d + L.sp), (const int64_t*)(d + L.ssp), n, ssp[n], spread_thr,
                                spread_lds, zm_max, kb, B.cap);
            launch_reduce_batch((const SpreadArgs*)(d + L.sp), (const int2*)(d + L.hv), (const int4* const*)(d + L.hl),
                                nh, B.cap);
            fft_phase(L.aA, L.saA, saA, 0, ph[2]);
            fft_phase(L.aB, L.saB, saB, (size_t)k * n, ph[3]);
        }
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(B.cap, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    KP_HIP(hipStreamEndCapture(B.cap, &B.graph));
    KP_HIP(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
    B.g_K = K;
    B.g_pkind = p_kind;
    B.g_lambda = op.lambda;
    (void)s;
}

// fallback: the same iteration, slice by slice, captured into the graph
static void capture_slices(Batch& B, const kp_pdhg_opts& op, int p_kind) {
    const int K = op.iters;
    if (B.exec) (void)hipGraphExecDestroy(B.exec);
    if (B.graph) (void)hipGraphDestroy(B.graph);
    B.exec = nullptr;
    B.graph = nullptr;
    KP_HIP(hipStreamBeginCapture(B.cap, hipStreamCaptureModeRelaxed));
    try {
        for (int k = 0; k < K; ++k) {
            for (auto& Pp : B.plans) {
                Plan& P = *Pp;
                float* sig = P.sched.as<float>();
                float* tau = sig + 8192;
                float* th = tau + 8192;
                FwdOpts fo;
                float2* grid = forward_to_grid(P, P.img[1].as<float2>(), fo, B.cap);
                InterpArgs ia{};
                ia.mode = IO_DUAL;
                ia.u = P.kint.as<float2>();
                ia.y = P.kint2.as<float2>();
                ia.p = p_kind == KP_PRECOND_NONE ? nullptr : P.pint.as<float>();
                ia.p_mc = p_kind == KP_PRECOND_MC ? 1 : 0;
                ia.sigma = sig + k;
                interp(P, grid, ia, B.cap);
                float2* g2 = spread_to_grid(P, P.kint.as<float2>(), (int)P.C, B.cap);
                AdjOpts ao;
                ao.ex = P.img[0].as<float2>();
                ao.exbar = P.img[1].as<float2>();
                ao.tau = tau + k;
                ao.theta = th + k;
                ao.lambda = op.lambda;
                ao.epi = EPI_L2;
                grid_to_image(P, g2, P.img[2].as<float2>(), ao, B.cap);
            }
        }
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(B.cap, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    KP_HIP(hipStreamEndCapture(B.cap, &B.graph));
    KP_HIP(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
    B.g_K = K;
    B.g_pkind = p_kind;
    B.g_lambda = op.lambda;
}

static bool fast_eligible(const Batch& B) {
    // every slice 2D, width 4, coil groups of four, and every pass of one
    // phase on the same specialised column block
    int nc[4] = {-1, -1, -1, -1};
    for (const auto& Pp : B.plans) {
        Plan& P = *Pp;
        if (P.d != 2 || P.W != 4 || P.C % 4 != 0 || P.C != B.C) return false;
        FwdOpts fo;
        AdjOpts ao;
        ao.epi = EPI_L2;
        std::vector<FftPass> ps = forward_passes(P, P.img[1].as<float2>(), fo);
        const std::vector<FftPass> ad = adjoint_passes(P, P.bufA.as<float2>(), P.img[2].as<float2>(), ao);
        ps.insert(ps.end(), ad.begin(), ad.end());
        for (int i = 0; i < 4; ++i) {
            if (!fft_batchable(ps[i])) return false;
            const int c = ps[i].Ob * ps[i].Ib;
            if (nc[i] >= 0 && nc[i] != c) return false;
            nc[i] = c;
        }
    }
    return true;
}

}  // namespace kp

using namespace kp;

struct kp_batch {
    kp::Batch* impl;
};

extern "C" {

int nufft_autotune(int ndim, const int64_t* shape, int64_t ncoils, int64_t nsamples, const float* coords,
                   const void* maps, float oversamp, int kb_width, kp_tuning* best, void* stream) {
    return guarded([&] {
        if (!best) fail(KP_ERR_INVALID_ARG, "best is NULL");
        validate_plan_args(ndim, shape, ncoils, nsamples, coords, maps, oversamp, kb_width, nullptr, false);
        *best = autotune(ndim, shape, ncoils, nsamples, coords, maps, oversamp, kb_width, (hipStream_t)stream);
    });
}

int nufft_plan_batch(kp_batch_t* out, int nslices, const int64_t* shapes, const int64_t* nsamples, int64_t ncoils,
                     const float* const* coords, const void* const* maps, float oversamp, int kb_width, int tune,
                     void* stream) {
    return guarded([&] {
        if (!out) fail(KP_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (nslices < 1 || !shapes || !nsamples || !coords) fail(KP_ERR_INVALID_ARG, "bad batch arguments");
        hipStream_t s = (hipStream_t)stream;
        auto B = std::make_unique<Batch>();
        B->C = (int)ncoils;
        KP_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
        for (int i = 0; i < nslices; ++i) {
            const void* m = maps ? maps[i] : nullptr;
            kp_tuning t{};
            const kp_tuning* tp = nullptr;
            if (tune) {
                t = autotune(2, shapes + 2 * i, ncoils, nsamples[i], coords[i], m, oversamp, kb_width, s);
                tp = &t;
            }
            B->plans.emplace_back(create_plan(2, shapes + 2 * i, ncoils, nsamples[i], coords[i], m, oversamp, kb_width,
                                              tp, s, false));
        }
        B->fast = fast_eligible(*B);
        *out = new kp_batch{B.release()};
    });
}

int nufft_batch_info(kp_batch_t batch, int slice, kp_plan_info* info, int* fast) {
    return guarded([&] {
        if (!batch || !batch->impl) fail(KP_ERR_INVALID_ARG, "batch is NULL");
        Batch& B = *batch->impl;
        if (slice < 0 || slice >= (int)B.plans.size()) fail(KP_ERR_INVALID_ARG, "slice out of range");
        if (fast) *fast = B.fast ? 1 : 0;
        kp_plan pl{B.plans[slice].get()};
        const int rc = nufft_plan_info(&pl, info);
        if (rc != KP_OK) fail(rc, kp_last_error());
    });
}

int pdhg_solve_batch(kp_batch_t batch, const void* const* y, const float* const* p, int p_kind,
                     const kp_pdhg_opts* opts, const float* lambda_max, void* const* x_out, void* stream) {
    return guarded([&] {
        if (!batch || !batch->impl || !y || !opts || !x_out) fail(KP_ERR_INVALID_ARG, "NULL argument");
        Batch& B = *batch->impl;
        const kp_pdhg_opts& op = *opts;
        if (op.reg != KP_REG_L2) fail(KP_ERR_UNSUPPORTED, "the batched solve supports the l2 regulariser");
        if (op.objective_host || op.x0 || op.u0) fail(KP_ERR_UNSUPPORTED, "the batched solve takes no x0/u0/objective");
        if (p_kind != KP_PRECOND_NONE && !p) fail(KP_ERR_INVALID_ARG, "p is NULL");
        hipStream_t s = (hipStream_t)stream;
        const int n = (int)B.plans.size();
        require_plan_device(*B.plans[0]);
        for (int i = 0; i < n; ++i) {
            kp_pdhg_opts oi = op;
            if (lambda_max) {
                if (!(lambda_max[i] > 0.f)) fail(KP_ERR_INVALID_ARG, "lambda_max[i] must be > 0");
                oi.lambda_max = lambda_max[i];
            }
            pdhg_setup(*B.plans[i], (const float2*)y[i], p_kind == KP_PRECOND_NONE ? nullptr : p[i], p_kind, oi, s);
        }
        if (!(B.exec && B.g_K == op.iters && B.g_pkind == p_kind && B.g_lambda == op.lambda)) {
            if (B.fast)
                capture_fast(B, op, p_kind, s);
            else
                capture_slices(B, op, p_kind);
        }
        KP_HIP(hipGraphLaunch(B.exec, s));
        for (int i = 0; i < n; ++i) copy2(B.plans[i]->img[0].as<float2>(), (float2*)x_out[i], B.plans[i]->Ntot, s);
    });
}

void nufft_batch_destroy(kp_batch_t batch) {
    if (!batch) return;
    if (batch->impl) {
        for (auto& P : batch->impl->plans) (void)hipStreamSynchronize(P->stream);
        (void)hipDeviceSynchronize();
        delete batch->impl;
    }
    delete batch;
}

}  // extern "C"
