// l2-optimised diagonal k-space preconditioner, efficient build
// ("Efficient computation of the multi-channel preconditioner", Fig. 2):
//
//   r_c  = sum_d autocorrelation(s_c s_d^*)      FFTs at 2N (Hermitian pairs)
//   h0   = A_2N^H(ones)                           adjoint NUFFT on the 2N image
//   p_c^{-1}[i] = 2^d / ||s_c||^2 * A_2N(r_c h0)[i]   forward NUFFT on the 2N image
//   p = 1 / Re(p^{-1})
//
// The 2N-image NUFFT (normalised by 1/sqrt(2^d N)) is a second plan over the
// same coordinates with the caller's oversampling and kernel width, run in
// channel mode (one image per channel, no coil maps).  For the
// single-channel preconditioner (C = 1, s = 1) the autocorrelation is the
// separable triangle prod_a (N_a - |k_a|) and needs no FFT.
#include <cmath>
#include <memory>

#include "kp_internal.h"

namespace kp {

static unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// q[n][j] = s_c[n] conj(s_{c+j}[n]) for j < np (maps stored [N][C])
__global__ void k_pairs(const float2* maps, int64_t N, int C, int c, int np, float2* q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * np) return;
    const int64_t n = i / np;
    const int j = (int)(i % np);
    const float2 a = maps[n * C + c], b = maps[n * C + c + j];
    q[i] = make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// R[v][c] += |Q[v][0]|^2; for j >= 1: R[v][c] += |Q[v][j]|^2, R[v][c+j] += |Q[-v][j]|^2
__global__ void k_accum_pairs(const float2* Q, int64_t Lt, int d, int L0, int L1, int L2, int np, int c, int C,
                              float2* R) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= Lt) return;
    int64_t vn;
    if (d == 2) {
        const int a0 = (int)(v / L1), a1 = (int)(v % L1);
        vn = (int64_t)((L0 - a0) % L0) * L1 + (L1 - a1) % L1;
    } else {
        const int a2 = (int)(v % L2);
        const int64_t r = v / L2;
        const int a1 = (int)(r % L1), a0 = (int)(r / L1);
        vn = ((int64_t)((L0 - a0) % L0) * L1 + (L1 - a1) % L1) * L2 + (L2 - a2) % L2;
    }
    const float2* qv = Q + v * np;
    const float2* qn = Q + vn * np;
    float2* rv = R + v * C;
    float acc = rv[c].x;
    acc += qv[0].x * qv[0].x + qv[0].y * qv[0].y;
    for (int j = 1; j < np; ++j) {
        acc += qv[j].x * qv[j].x + qv[j].y * qv[j].y;
        rv[c + j].x += qn[j].x * qn[j].x + qn[j].y * qn[j].y;
    }
    rv[c].x = acc;
}

// closed-form single-channel autocorrelation on the centred lag image:
// r[k] = prod_a (N_a - |k_a|), k_a = m_a - N_a (the -N_a lag is 0)
__global__ void k_triangle(int64_t Lt, int d, int N0, int N1, int N2, float2* r) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= Lt) return;
    const int L1 = 2 * N1, L2 = 2 * N2;
    int k0, k1, k2 = 0;
    if (d == 2) {
        k0 = (int)(v / L1) - N0;
        k1 = (int)(v % L1) - N1;
    } else {
        k2 = (int)(v % L2) - N2;
        const int64_t q = v / L2;
        k1 = (int)(q % L1) - N1;
        k0 = (int)(q / L1) - N0;
    }
    double t = (double)(N0 - abs(k0)) * (double)(N1 - abs(k1));
    if (d == 3) t *= (double)(N2 - abs(k2));
    r[v] = make_float2((float)t, 0.f);
}

__global__ void k_ones_k(float2* k, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) k[i] = make_float2(1.f, 0.f);
}

// v[n][c] = r[n][c] * h0[n] * scale
__global__ void k_rh(const float2* r, const float2* h, int64_t Lt, int C, float scale, float2* v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Lt * C) return;
    const float2 a = r[i], b = h[i / C];
    v[i] = make_float2((a.x * b.x - a.y * b.y) * scale, (a.x * b.y + a.y * b.x) * scale);
}

// per-coil ||s_c||^2 in double (one block per coil, fixed order)
__global__ void k_map_norms(const float2* maps, int64_t N, int C, double* out) {
    __shared__ double sh[256];
    const int c = blockIdx.x;
    double acc = 0;
    for (int64_t n = threadIdx.x; n < N; n += blockDim.x) {
        const float2 v = maps[n * C + c];
        acc += (double)v.x * v.x + (double)v.y * v.y;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
}

// p[s][c] = ||s_c||^2 / (2^d Re k[s][c])
__global__ void k_finish_p(const float2* k, int64_t M, int C, const double* nrm, double two_d, float* p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * C) return;
    const int c = (int)(i % C);
    p[i] = (float)(nrm[c] / (two_d * (double)k[i].x));
}

// FFT over an image laid out [shape][C]: forward order (last axis first) with
// zero-padding N_a -> L_a, or inverse order with a centred full-length
// reorder (output index m <-> lag m - L_a/2).
static void fft_image(const float2* in, float2* out, float2* tmp, int d, const int64_t* N, const int64_t* L, int C,
                      bool inverse, DevBuf* tw, hipStream_t s) {
    const float2* cur = in;
    int64_t rows[3] = {N[0], N[1], N[2]};
    for (int p = 0; p < d; ++p) {
        const int ax = inverse ? p : d - 1 - p;
        float2* dst = ((d - 1 - p) % 2 == 0) ? out : tmp;  // the last pass lands in `out`
        FftPass fp{};
        fp.L = (int)L[ax];
        fp.Lin = (int)rows[ax];
        fp.Lout = (int)L[ax];
        fp.pad_in = fp.Lin < fp.L ? 1 : 0;
        fp.crop_out = inverse ? 1 : 0;
        fp.inverse = inverse ? 1 : 0;
        int64_t O = 1, I = C;
        for (int b = 0; b < ax; ++b) O *= rows[b];
        for (int b = ax + 1; b < d; ++b) I *= rows[b];
        fp.O = O;
        fp.I = I;
        fp.in_os = (int64_t)fp.Lin * I;
        fp.in_rs = I;
        fp.out_os = (int64_t)fp.Lout * I;
        fp.out_rs = I;
        int nst = 0, rad[kMaxStages];
        fft_factor(fp.L, &nst, rad);
        fp.nst = nst;
        for (int i = 0; i < nst; ++i) fp.rad[i] = rad[i];
        fp.tw = tw[ax].as<float2>();
        fp.pre = PRE_NONE;
        fp.post = POST_NONE;
        fp.in = cur;
        fp.out = dst;
        pass_blocking(I, &fp.Ob, &fp.Ib);
        launch_fft_pass(fp, s);
        rows[ax] = L[ax];
        cur = dst;
    }
}

// ---- Pipe-Menon density compensation (Experiments: the first of the three
// k-space preconditioners compared with PDHG): w <- w / |G G^T w| from w = 1,
// with G the plan's gridding interpolation (the spreading and interpolation
// kernels on one channel, no FFT), kDcfIters times; one weight per sample.
// The raw weights have an arbitrary scale, which the fixed dual step would
// pass on to the proximal threshold through tau = 1/lambda_max(P A A^H), so
// they are scaled to lambda_max(P A A^H) = 1 (power method, 30 iterations as
// for the solver), the value the l2-optimised preconditioners approach.
constexpr int kDcfIters = 30;
constexpr int kDcfPowerIters = 30;

__global__ void k_dcf_update(float2* w, const float2* v, int64_t M) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const float2 t = v[i];
    w[i] = make_float2(w[i].x / sqrtf(t.x * t.x + t.y * t.y), 0.f);
}

__global__ void k_real_part(const float2* w, int64_t M, float* q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) q[i] = w[i].x;
}

__global__ void k_divide_by(float* q, int64_t M, const float* lam) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) q[i] = q[i] / lam[0];
}

static void dcf_build(Plan& P, float* p_out, hipStream_t s) {
    float2* w = P.kint.as<float2>();
    float2* v = P.kint3.as<float2>();
    hipLaunchKernelGGL(k_ones_k, dim3(nblk(P.M)), dim3(256), 0, s, w, P.M);
    KP_LAUNCH_CHECK();
    for (int it = 0; it < kDcfIters; ++it) {
        const float2* g = spread_to_grid(P, w, 1, s);
        InterpArgs ia{};
        ia.mode = IO_INTERNAL;
        ia.out = v;
        ia.C = 1;
        interp(P, g, ia, s);
        hipLaunchKernelGGL(k_dcf_update, dim3(nblk(P.M)), dim3(256), 0, s, w, v, P.M);
        KP_LAUNCH_CHECK();
    }
    float* q = P.pint.as<float>();
    hipLaunchKernelGGL(k_real_part, dim3(nblk(P.M)), dim3(256), 0, s, w, P.M, q);
    KP_LAUNCH_CHECK();
    DevBuf lam;
    lam.alloc(sizeof(float));
    power_method(P, q, 0, kDcfPowerIters, lam.as<float>(), s);
    hipLaunchKernelGGL(k_divide_by, dim3(nblk(P.M)), dim3(256), 0, s, q, P.M, lam.as<float>());
    KP_LAUNCH_CHECK();
    permute_p_to_caller(q, p_out, P.perm.as<int32_t>(), P.M, 1, false, s);
    KP_HIP(hipStreamSynchronize(s));
}

void precond_build_impl(Plan& P, int kind, float* p_out, hipStream_t s) {
    if (kind == KP_PRECOND_DCF) return dcf_build(P, p_out, s);
    if (kind != KP_PRECOND_SC && kind != KP_PRECOND_MC) fail(KP_ERR_INVALID_ARG, "kind must be SC, MC or DCF");
    const int d = P.d;
    const bool mc = kind == KP_PRECOND_MC;
    const int Cp = mc ? (int)P.C : 1;
    int64_t N2[3] = {1, 1, 1}, L[3] = {1, 1, 1}, N[3] = {1, 1, 1};
    int64_t Lt = 1;
    for (int a = 0; a < d; ++a) {
        N[a] = P.N[a];
        N2[a] = 2 * P.N[a];
        L[a] = 2 * P.N[a];
        Lt *= L[a];
    }
    // the 2N-image NUFFT plan (channel mode)
    std::unique_ptr<Plan> Q(create_plan(d, N2, Cp, P.M, P.coords.as<float>(), nullptr, P.alpha, P.W, nullptr, s,
                                        true));
    DevBuf tw[3];
    for (int a = 0; a < d; ++a) fft_twiddles((int)L[a], tw[a]);
    DevBuf R, img1, img2, nrm;
    R.alloc(sizeof(float2) * Lt * Cp);
    nrm.alloc(sizeof(double) * 16);
    if (mc) {
        img1.alloc(sizeof(float2) * Lt * Cp);
        img2.alloc(sizeof(float2) * Lt * Cp);
        KP_HIP(hipMemsetAsync(R.p, 0, sizeof(float2) * Lt * Cp, s));
        const int C = (int)P.C;
        for (int c = 0; c < C; ++c) {
            const int np = C - c;
            hipLaunchKernelGGL(k_pairs, dim3(nblk(P.Ntot * np)), dim3(256), 0, s, P.maps.as<float2>(), P.Ntot, C, c,
                               np, img2.as<float2>());
            KP_LAUNCH_CHECK();
            fft_image(img2.as<float2>(), img1.as<float2>(), Q->bufA.as<float2>(), d, N, L, np, false, tw, s);
            hipLaunchKernelGGL(k_accum_pairs, dim3(nblk(Lt)), dim3(256), 0, s, img1.as<float2>(), Lt, d, (int)L[0],
                               (int)L[1], (int)L[2], np, c, C, R.as<float2>());
            KP_LAUNCH_CHECK();
        }
        // r_c = IFFT(R_c) on the centred lag image
        fft_image(R.as<float2>(), img1.as<float2>(), Q->bufA.as<float2>(), d, L, L, C, true, tw, s);
        hipLaunchKernelGGL(k_map_norms, dim3(C), dim3(256), 0, s, P.maps.as<float2>(), P.Ntot, C, nrm.as<double>());
        KP_LAUNCH_CHECK();
    } else {
        img1.alloc(sizeof(float2) * Lt);
        img2.alloc(sizeof(float2) * Lt);
        hipLaunchKernelGGL(k_triangle, dim3(nblk(Lt)), dim3(256), 0, s, Lt, d, (int)N[0], (int)N[1], (int)N[2],
                           img1.as<float2>());
        KP_LAUNCH_CHECK();
        const double nN = (double)P.Ntot;
        KP_HIP(hipMemcpyAsync(nrm.p, &nN, sizeof(double), hipMemcpyHostToDevice, s));
    }
    // h0 = A_2N^H(ones) (one channel)
    hipLaunchKernelGGL(k_ones_k, dim3(nblk(Q->M)), dim3(256), 0, s, Q->kint.as<float2>(), Q->M);
    KP_LAUNCH_CHECK();
    float2* g = spread_to_grid(*Q, Q->kint.as<float2>(), 1, s);
    AdjOpts ao;
    ao.channel = true;
    ao.C = 1;
    grid_to_image(*Q, g, img2.as<float2>(), ao, s);
    // v_c = r_c h0 (the inverse FFT's 1/L^d folded in for MC)
    const float scale = mc ? (float)(1.0 / (double)Lt) : 1.f;
    hipLaunchKernelGGL(k_rh, dim3(nblk(Lt * Cp)), dim3(256), 0, s, img1.as<float2>(), img2.as<float2>(), Lt, Cp, scale,
                       R.as<float2>());
    KP_LAUNCH_CHECK();
    // p_c^{-1} = 2^d / ||s_c||^2 * A_2N(v_c)
    FwdOpts fo;
    fo.channel = true;
    fo.C = Cp;
    float2* grid = forward_to_grid(*Q, R.as<float2>(), fo, s);
    InterpArgs ia{};
    ia.mode = IO_INTERNAL;
    ia.out = Q->kint.as<float2>();
    ia.C = Cp;
    interp(*Q, grid, ia, s);
    hipLaunchKernelGGL(k_finish_p, dim3(nblk(Q->M * Cp)), dim3(256), 0, s, Q->kint.as<float2>(), Q->M, Cp,
                       nrm.as<double>(), (double)(1 << d), Q->pint.as<float>());
    KP_LAUNCH_CHECK();
    permute_p_to_caller(Q->pint.as<float>(), p_out, Q->perm.as<int32_t>(), Q->M, Cp, mc, s);
    KP_HIP(hipStreamSynchronize(s));
}

}  // namespace kp

using namespace kp;

extern "C" int precond_build(kp_plan_t plan, int kind, float* p, void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl || !p) fail(KP_ERR_INVALID_ARG, "NULL argument");
        require_plan_device(*plan->impl);
        precond_build_impl(*plan->impl, kind, p, (hipStream_t)stream);
    });
}
