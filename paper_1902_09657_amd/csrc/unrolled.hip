// Differentiable unrolled l2 PDHG: forward with iterate checkpoints and a
// hand-written reverse recursion that uses the plan's NUFFT kernels for A
// (forward) and A^H (adjoint).
//
// Step k ("Preconditioned PDHG for simple regularizers" with free sizes):
//   ax_k       = A xbar_k
//   u_{k+1}    = (u_k + sigma_k p (ax_k - y)) / (1 + sigma_k p)
//   ahu_k      = A^H u_{k+1}
//   x_{k+1}    = (x_k - tau_k ahu_k) / (1 + tau_k lambda)
//   xbar_{k+1} = x_{k+1} + theta_k (x_{k+1} - x_k)
// Reverse of step k, for incoming gradients (gx, gxb, gu) of
// (x_{k+1}, xbar_{k+1}, u_{k+1}) (PyTorch convention: dL/dRe + i dL/dIm):
//   g_theta_k = Re<gxb, x_{k+1} - x_k>
//   gxt       = gx + (1 + theta) gxb,   d = 1 + tau lambda
//   gx'       = -theta gxb + gxt / d,   g_ahu = -tau gxt / d
//   g_tau_k   = Re<gxt, (-ahu_k - lambda x_{k+1}) / d>
//   g_lambda += Re<gxt, -tau x_{k+1} / d>
//   gut       = gu + A g_ahu,           e = 1 + sigma p
//   gu'       = gut / e,                g_ax = sigma p gut / e,   g_y -= g_ax
//   g_sigma_k = Re<gut, p (ax_k - y - u_{k+1}) / e>
//   gxb'      = A^H g_ax
// with x_0 = xbar_0 = x0 (g_x0 = gx + gxb at the end) and u_0 = 0.
//
// Memory: checkpoints of (x, xbar, u) every `ckpt_every` steps plus one
// segment of recomputed step records live in a caller-owned buffer of
// pdhg_unrolled_ckpt_bytes bytes.
#include <cmath>
#include <vector>

#include "kp_internal.h"

namespace kp {

static unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }
constexpr int kURed = 512;  // reduction blocks (fixed: deterministic sums)

struct ULayout {
    int64_t N, MC;
    int K, S, nck;
    // offsets in float2 units
    int64_t ck;         // checkpoints: nck x (x, xbar, u)
    int64_t seg;        // S x (x_k, u_k, ax_k, u1, ahu, x1)
    int64_t tmp;        // gx, gxb, gxt, gahu (N each); gu, gax, gy, Ag (MC each)
    int64_t red;        // doubles: 4K per-step + 3 x kURed partials (in float2 = 8 bytes units)
    int64_t total;      // float2 units
};

static ULayout ulayout(const Plan& P, int K, int S) {
    ULayout L{};
    L.N = P.Ntot;
    L.MC = P.M * P.C;
    L.K = K;
    L.S = S;
    L.nck = (K + S - 1) / S;
    L.ck = 0;
    L.seg = L.ck + (int64_t)L.nck * (2 * L.N + L.MC);
    L.tmp = L.seg + (int64_t)S * (3 * L.N + 3 * L.MC);
    L.red = L.tmp + 4 * L.N + 4 * L.MC;
    L.total = L.red + 4 * (int64_t)K + 3 * kURed + 16;
    return L;
}

// ---------------------------------------------------------------- kernels
__global__ void k_u_dual(const float2* u, const float2* ax, const float2* y, const float* p, int p_mc, int C,
                         int64_t n, const float* sigma, float2* u1) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float pv = p ? (p_mc ? p[i] : p[i / C]) : 1.f;
    const float sp = *sigma * pv;
    const float den = 1.f / (1.f + sp);
    const float2 a = u[i], b = ax[i], c = y[i];
    u1[i] = make_float2((a.x + sp * (b.x - c.x)) * den, (a.y + sp * (b.y - c.y)) * den);
}

__global__ void k_u_primal(const float2* x, const float2* ahu, const float* tau, const float* theta,
                           const float* lam, int64_t n, float2* x1, float2* xb1) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float t = *tau, th = *theta;
    const float den = 1.f / (1.f + t * *lam);
    const float2 a = x[i], h = ahu[i];
    const float2 xn = make_float2((a.x - t * h.x) * den, (a.y - t * h.y) * den);
    x1[i] = xn;
    xb1[i] = make_float2(xn.x + th * (xn.x - a.x), xn.y + th * (xn.y - a.y));
}

__device__ double ublock_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// image side of the reverse step; partial sums of g_theta, g_tau, g_lambda
__global__ void __launch_bounds__(256) k_b_img(float2* gx, const float2* gxb, const float2* x, const float2* x1,
                                               const float2* ahu, const float* tau, const float* theta,
                                               const float* lam, int64_t n, float2* gahu, double* part) {
    __shared__ double sh[256];
    const float t = *tau, th = *theta, l = *lam;
    const float d = 1.f + t * l;
    double s_th = 0, s_tau = 0, s_lam = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float2 b = gxb[i], a = gx[i], xo = x[i], xn = x1[i], h = ahu[i];
        s_th += (double)b.x * (xn.x - xo.x) + (double)b.y * (xn.y - xo.y);
        const float2 gt = make_float2(a.x + (1.f + th) * b.x, a.y + (1.f + th) * b.y);
        s_tau += ((double)gt.x * (-h.x - l * xn.x) + (double)gt.y * (-h.y - l * xn.y)) / d;
        s_lam += ((double)gt.x * (-t * xn.x) + (double)gt.y * (-t * xn.y)) / d;
        gx[i] = make_float2(-th * b.x + gt.x / d, -th * b.y + gt.y / d);
        gahu[i] = make_float2(-t * gt.x / d, -t * gt.y / d);
    }
    const double r0 = ublock_sum(s_tau, sh), r1 = ublock_sum(s_th, sh), r2 = ublock_sum(s_lam, sh);
    if (threadIdx.x == 0) {  // in the order of the per-step sums: tau, theta, lambda
        part[blockIdx.x] = r0;
        part[kURed + blockIdx.x] = r1;
        part[2 * kURed + blockIdx.x] = r2;
    }
}

// k-space side of the reverse step; partial sums of g_sigma
__global__ void __launch_bounds__(256) k_b_k(float2* gu, const float2* Ag, const float2* ax, const float2* y,
                                             const float2* u1, const float* p, int p_mc, int C, const float* sigma,
                                             int64_t n, float2* gax, float2* gy, double* part) {
    __shared__ double sh[256];
    const float sg = *sigma;
    double s_sig = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float pv = p ? (p_mc ? p[i] : p[i / C]) : 1.f;
        const float e = 1.f + sg * pv;
        const float2 a = gu[i], b = Ag[i];
        const float2 gt = make_float2(a.x + b.x, a.y + b.y);
        const float2 r = make_float2(ax[i].x - y[i].x - u1[i].x, ax[i].y - y[i].y - u1[i].y);
        s_sig += ((double)gt.x * r.x + (double)gt.y * r.y) * pv / e;
        gu[i] = make_float2(gt.x / e, gt.y / e);
        const float2 g = make_float2(sg * pv * gt.x / e, sg * pv * gt.y / e);
        gax[i] = g;
        gy[i] = make_float2(gy[i].x - g.x, gy[i].y - g.y);
    }
    const double r0 = ublock_sum(s_sig, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r0;
}

// sum nparts partial arrays (each kURed long) into out[j * stride]
__global__ void k_u_final(const double* part, int nparts, double* out, int stride) {
    __shared__ double sh[256];
    for (int j = 0; j < nparts; ++j) {
        double acc = 0;
        for (int i = threadIdx.x; i < kURed; i += blockDim.x) acc += part[j * kURed + i];
        const double r = ublock_sum(acc, sh);
        if (threadIdx.x == 0) out[j * stride] = r;
    }
}

// g_params from the per-step doubles; lambda summed over steps in order
__global__ void k_u_params(const double* st, int K, float* g) {
    const int i = threadIdx.x + blockIdx.x * blockDim.x;
    if (i < 3 * K) {
        // st layout: sigma[K], tau[K], theta[K], lambda[K]
        g[i] = (float)st[i];
    }
    if (i == 0) {
        double s = 0;
        for (int k = 0; k < K; ++k) s += st[3 * K + k];
        g[3 * K] = (float)s;
    }
}

__global__ void k_add2(const float2* a, const float2* b, float2* c, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = make_float2(a[i].x + b[i].x, a[i].y + b[i].y);
}

// ------------------------------------------------------------ operators
static void apply_A(Plan& P, const float2* img, float2* kout, hipStream_t s) {
    FwdOpts fo;
    float2* grid = forward_to_grid(P, img, fo, s);
    InterpArgs ia{};
    ia.mode = IO_INTERNAL;
    ia.out = kout;
    interp(P, grid, ia, s);
}
static void apply_AH(Plan& P, const float2* kin, float2* img, hipStream_t s) {
    float2* g = spread_to_grid(P, kin, (int)P.C, s);
    AdjOpts ao;
    grid_to_image(P, g, img, ao, s);
}

struct UState {
    const float2* y;     // internal y
    const float* p;      // internal p or null
    int p_mc;
    const float* prm;    // device params [3K+1]
    int K;
};

// one forward step from (x, xb, u) to (x1, xb1, u1), recording ax and ahu
static void ustep(Plan& P, const UState& U, int k, const float2* x, const float2* xb, const float2* u, float2* ax,
                  float2* u1, float2* ahu, float2* x1, float2* xb1, hipStream_t s) {
    const int64_t N = P.Ntot, MC = P.M * P.C;
    apply_A(P, xb, ax, s);
    hipLaunchKernelGGL(k_u_dual, dim3(nblk(MC)), dim3(256), 0, s, u, ax, U.y, U.p, U.p_mc, (int)P.C, MC, U.prm + k,
                       u1);
    KP_LAUNCH_CHECK();
    apply_AH(P, u1, ahu, s);
    hipLaunchKernelGGL(k_u_primal, dim3(nblk(N)), dim3(256), 0, s, x, ahu, U.prm + U.K + k, U.prm + 2 * U.K + k,
                       U.prm + 3 * U.K, N, x1, xb1);
    KP_LAUNCH_CHECK();
}

static void check_unrolled(const Plan& P, int K, int S) {
    if (K < 1 || K > 4096) fail(KP_ERR_INVALID_ARG, "K must lie in [1, 4096]");
    if (S < 1 || S > K) fail(KP_ERR_INVALID_ARG, "ckpt_every must lie in [1, K]");
    (void)P;
}

static void load_inputs(Plan& P, const void* y, const float* p, int p_kind, UState& U, hipStream_t s) {
    if (p_kind != KP_PRECOND_NONE && p_kind != KP_PRECOND_SC && p_kind != KP_PRECOND_MC)
        fail(KP_ERR_INVALID_ARG, "p_kind must be NONE, SC or MC");
    if (p_kind != KP_PRECOND_NONE && !p) fail(KP_ERR_INVALID_ARG, "p is NULL");
    permute_to_internal((const float2*)y, P.kint2.as<float2>(), P.perm.as<int32_t>(), P.M, (int)P.C, s,
                        P.iperm.as<int32_t>());
    U.y = P.kint2.as<float2>();
    U.p = load_p(P, p, p_kind, s);
    U.p_mc = p_kind == KP_PRECOND_MC ? 1 : 0;
}

void unrolled_forward(Plan& P, const void* y, const float* p, int p_kind, const float* prm, int K, int S,
                      const void* x0, void* x_out, void* ckpt, hipStream_t s) {
    check_unrolled(P, K, S);
    if (!y || !prm || !x_out || !ckpt) fail(KP_ERR_INVALID_ARG, "NULL argument");
    const ULayout L = ulayout(P, K, S);
    float2* B = (float2*)ckpt;
    UState U{};
    load_inputs(P, y, p, p_kind, U, s);
    U.prm = prm;
    U.K = K;
    const int64_t N = L.N, MC = L.MC;
    // running state: two sets of (x, xbar, u) used in turn (plan workspaces
    // and the segment area), so a step writes the other set and nothing is
    // copied; ax and A^H u of the current step are scratch
    float2* seg = B + L.seg;  // 2 MC + 3 N used of S (3 N + 3 MC)
    float2* ax = seg;
    float2* ahu = seg + MC;
    float2* xs[2] = {P.img[0].as<float2>(), seg + MC + N};
    float2* xbs[2] = {P.img[1].as<float2>(), seg + MC + 2 * N};
    float2* us[2] = {P.kint.as<float2>(), seg + MC + 3 * N};
    if (x0)
        copy2((const float2*)x0, xs[0], N, s);
    else
        fill2(xs[0], N, 0.f, 0.f, s);
    copy2(xs[0], xbs[0], N, s);
    fill2(us[0], MC, 0.f, 0.f, s);
    int cur = 0;
    for (int k = 0; k < K; ++k) {
        if (k % S == 0) {
            float2* c = B + L.ck + (int64_t)(k / S) * (2 * N + MC);
            copy2(xs[cur], c, N, s);
            copy2(xbs[cur], c + N, N, s);
            copy2(us[cur], c + 2 * N, MC, s);
        }
        ustep(P, U, k, xs[cur], xbs[cur], us[cur], ax, us[cur ^ 1], ahu, xs[cur ^ 1], xbs[cur ^ 1], s);
        cur ^= 1;
    }
    copy2(xs[cur], (float2*)x_out, N, s);
}

void unrolled_backward(Plan& P, const void* y, const float* p, int p_kind, const float* prm, int K, int S,
                       const void* x0, const void* ckpt, const void* g_x, float* g_params, void* g_y, void* g_x0,
                       hipStream_t s) {
    check_unrolled(P, K, S);
    if (!y || !prm || !ckpt || !g_x || !g_params) fail(KP_ERR_INVALID_ARG, "NULL argument");
    (void)x0;
    const ULayout L = ulayout(P, K, S);
    float2* B = (float2*)ckpt;
    UState U{};
    load_inputs(P, y, p, p_kind, U, s);
    U.prm = prm;
    U.K = K;
    const int64_t N = L.N, MC = L.MC;
    const int C = (int)P.C;
    // segment records: per step k in the segment: x_k, u_k, ax_k, u1, ahu, x1 (+ xb of the next step)
    auto rec = [&](int j) { return B + L.seg + (int64_t)j * (3 * N + 3 * MC); };
    float2* T = B + L.tmp;
    float2* gx = T;
    float2* gxb = T + N;
    float2* gxt = T + 2 * N;  // spare image (next xbar during recompute)
    float2* gahu = T + 3 * N;
    float2* gu = T + 4 * N;
    float2* gax = gu + MC;
    float2* gy = gax + MC;
    float2* Ag = gy + MC;
    double* st = (double*)(B + L.red);  // sigma[K], tau[K], theta[K], lambda[K]
    double* part = st + 4 * K;

    copy2((const float2*)g_x, gx, N, s);
    fill2(gxb, N, 0.f, 0.f, s);
    fill2(gu, MC, 0.f, 0.f, s);
    fill2(gy, MC, 0.f, 0.f, s);
    for (int sg = L.nck - 1; sg >= 0; --sg) {
        const int k0 = sg * S, k1 = std::min(K, k0 + S);
        // recompute the segment from its checkpoint; step k reads x_k and
        // u_k from the checkpoint (first step) or from the previous step's
        // record, and xbar_k from one of two spare images used in turn
        const float2* c = B + L.ck + (int64_t)sg * (2 * N + MC);
        const float2* xk = c;
        const float2* xbk = c + N;
        const float2* uk = c + 2 * N;
        float2* xbs[2] = {gxt, P.img[3].as<float2>()};
        for (int k = k0; k < k1; ++k) {
            float2* r = rec(k - k0);
            float2* rax = r + N + MC;    // ax_k
            float2* ru1 = r + N + 2 * MC;
            float2* rahu = r + N + 3 * MC;
            float2* rx1 = r + 2 * N + 3 * MC;
            float2* xb1 = xbs[(k - k0) & 1];
            ustep(P, U, k, xk, xbk, uk, rax, ru1, rahu, rx1, xb1, s);
            xk = rx1;
            xbk = xb1;
            uk = ru1;
        }
        // reverse through the segment
        for (int k = k1 - 1; k >= k0; --k) {
            float2* r = rec(k - k0);
            const float2* rx = k == k0 ? c : rec(k - 1 - k0) + 2 * N + 3 * MC;  // x_k
            const float2* rax = r + N + MC;
            const float2* ru1 = r + N + 2 * MC;
            const float2* rahu = r + N + 3 * MC;
            const float2* rx1 = r + 2 * N + 3 * MC;
            hipLaunchKernelGGL(k_b_img, dim3(kURed), dim3(256), 0, s, gx, gxb, rx, rx1, rahu, prm + K + k,
                               prm + 2 * K + k, prm + 3 * K, N, gahu, part);
            KP_LAUNCH_CHECK();
            // part[0] -> tau_k, part[1] -> theta_k, part[2] -> lambda_k (stride K)
            hipLaunchKernelGGL(k_u_final, dim3(1), dim3(256), 0, s, part, 3, st + K + k, K);
            KP_LAUNCH_CHECK();
            apply_A(P, gahu, Ag, s);
            hipLaunchKernelGGL(k_b_k, dim3(kURed), dim3(256), 0, s, gu, Ag, rax, U.y, ru1, U.p, U.p_mc, C, prm + k, MC,
                               gax, gy, part);
            KP_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_u_final, dim3(1), dim3(256), 0, s, part, 1, st + k, 0);
            KP_LAUNCH_CHECK();
            apply_AH(P, gax, gxb, s);
        }
    }
    hipLaunchKernelGGL(k_u_params, dim3(nblk(3 * K + 1)), dim3(256), 0, s, st, K, g_params);
    KP_LAUNCH_CHECK();
    if (g_x0) {
        hipLaunchKernelGGL(k_add2, dim3(nblk(N)), dim3(256), 0, s, gx, gxb, (float2*)g_x0, N);
        KP_LAUNCH_CHECK();
    }
    if (g_y) permute_to_caller(gy, (float2*)g_y, P.perm.as<int32_t>(), P.M, C, s);
}

}  // namespace kp

using namespace kp;

extern "C" {

int64_t pdhg_unrolled_ckpt_bytes(kp_plan_t plan, int K, int ckpt_every) {
    if (!plan || !plan->impl || K < 1 || ckpt_every < 1 || ckpt_every > K) return -1;
    return (int64_t)sizeof(float2) * ulayout(*plan->impl, K, ckpt_every).total;
}

int pdhg_unrolled_forward(kp_plan_t plan, const void* y, const float* p, int p_kind, const float* params, int K,
                          int ckpt_every, const void* x0, void* x_out, void* ckpt, void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl) fail(KP_ERR_INVALID_ARG, "plan is NULL");
        require_plan_device(*plan->impl);
        unrolled_forward(*plan->impl, y, p, p_kind, params, K, ckpt_every, x0, x_out, ckpt, (hipStream_t)stream);
    });
}

int pdhg_unrolled_backward(kp_plan_t plan, const void* y, const float* p, int p_kind, const float* params, int K,
                           int ckpt_every, const void* x0, const void* ckpt, const void* g_x, float* g_params,
                           void* g_y, void* g_x0, void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl) fail(KP_ERR_INVALID_ARG, "plan is NULL");
        require_plan_device(*plan->impl);
        unrolled_backward(*plan->impl, y, p, p_kind, params, K, ckpt_every, x0, ckpt, g_x, g_params, g_y, g_x0,
                          (hipStream_t)stream);
    });
}

}  // extern "C"
