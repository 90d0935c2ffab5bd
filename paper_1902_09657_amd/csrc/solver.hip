// PDHG solver: layout permutes, deterministic reductions, power method,
// step-size schedule, periodised db4 wavelet prox, the solve loop and its
// C ABI.
#include <cmath>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <set>

#include "kp_internal.h"

namespace kp {

static unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// ------------------------------------------------------------- permutes
__global__ void k_perm_in(const float2* y, float2* k, const int32_t* perm, int64_t M, int C) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * C) return;
    const int64_t s = i / C;
    const int c = (int)(i % C);
    k[i] = y[(int64_t)c * M + perm[s]];
}
__global__ void k_perm_out(const float2* k, float2* y, const int32_t* perm, int64_t M, int C) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * C) return;
    const int64_t s = i / C;
    const int c = (int)(i % C);
    y[(int64_t)c * M + perm[s]] = k[i];
}
__global__ void k_perm_p_in(const float* p, float* q, const int32_t* perm, int64_t M, int C, int mc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (mc) {
        if (i >= M * C) return;
        const int64_t s = i / C;
        const int c = (int)(i % C);
        q[i] = p[(int64_t)c * M + perm[s]];
    } else {
        if (i >= M) return;
        q[i] = p[perm[i]];
    }
}
__global__ void k_perm_p_out(const float* q, float* p, const int32_t* perm, int64_t M, int C, int mc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (mc) {
        if (i >= M * C) return;
        const int64_t s = i / C;
        const int c = (int)(i % C);
        p[(int64_t)c * M + perm[s]] = q[i];
    } else {
        if (i >= M) return;
        p[perm[i]] = q[i];
    }
}

// One thread per sorted sample, all C coils: every load instruction of a
// wave reads one coil row at 64 neighbouring sorted samples (runs of
// consecutive caller indices along a trajectory), and each thread stores its
// sample's C values as one contiguous run of 16-byte stores.
template <int C>
__global__ void k_perm_in_c(const float2* __restrict__ y, float2* __restrict__ k, const int32_t* __restrict__ perm,
                            int64_t M) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= M) return;
    const int64_t ps = perm[s];
    float2 v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = y[(int64_t)c * M + ps];
    float4* dst = reinterpret_cast<float4*>(k + s * C);
#pragma unroll
    for (int q = 0; q < C / 2; ++q) dst[q] = make_float4(v[2 * q].x, v[2 * q].y, v[2 * q + 1].x, v[2 * q + 1].y);
}

// One thread per caller sample j (inverse permutation): every load
// instruction of a wave reads 64 consecutive caller samples of one coil row,
// and each thread stores its sample's C values as one contiguous run of
// 16-byte stores at its sorted position iperm[j].
template <int C>
__global__ void k_perm_in_inv_c(const float2* __restrict__ y, float2* __restrict__ k, const int32_t* __restrict__ iperm,
                                int64_t M) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    float2 v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = y[(int64_t)c * M + j];
    float4* dst = reinterpret_cast<float4*>(k + (int64_t)iperm[j] * C);
#pragma unroll
    for (int q = 0; q < C / 2; ++q) dst[q] = make_float4(v[2 * q].x, v[2 * q].y, v[2 * q + 1].x, v[2 * q + 1].y);
}

void permute_to_internal(const float2* y, float2* k, const int32_t* perm, int64_t M, int C, hipStream_t s,
                         const int32_t* iperm) {
    if (M <= 0) return;
    if (iperm && (C == 8 || C == 12 || C == 4 || C == 2)) {
        if (C == 8)
            hipLaunchKernelGGL(k_perm_in_inv_c<8>, dim3(nblk(M)), dim3(256), 0, s, y, k, iperm, M);
        else if (C == 12)
            hipLaunchKernelGGL(k_perm_in_inv_c<12>, dim3(nblk(M)), dim3(256), 0, s, y, k, iperm, M);
        else if (C == 4)
            hipLaunchKernelGGL(k_perm_in_inv_c<4>, dim3(nblk(M)), dim3(256), 0, s, y, k, iperm, M);
        else
            hipLaunchKernelGGL(k_perm_in_inv_c<2>, dim3(nblk(M)), dim3(256), 0, s, y, k, iperm, M);
        KP_LAUNCH_CHECK();
        return;
    }
    if (C == 8)
        hipLaunchKernelGGL(k_perm_in_c<8>, dim3(nblk(M)), dim3(256), 0, s, y, k, perm, M);
    else if (C == 12)
        hipLaunchKernelGGL(k_perm_in_c<12>, dim3(nblk(M)), dim3(256), 0, s, y, k, perm, M);
    else if (C == 4)
        hipLaunchKernelGGL(k_perm_in_c<4>, dim3(nblk(M)), dim3(256), 0, s, y, k, perm, M);
    else if (C == 2)
        hipLaunchKernelGGL(k_perm_in_c<2>, dim3(nblk(M)), dim3(256), 0, s, y, k, perm, M);
    else
        hipLaunchKernelGGL(k_perm_in, dim3(nblk(M * C)), dim3(256), 0, s, y, k, perm, M, C);
    KP_LAUNCH_CHECK();
}
void permute_to_caller(const float2* k, float2* y, const int32_t* perm, int64_t M, int C, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_out, dim3(nblk(M * C)), dim3(256), 0, s, k, y, perm, M, C);
    KP_LAUNCH_CHECK();
}
void permute_p_to_internal(const float* p, float* q, const int32_t* perm, int64_t M, int C, bool mc, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_p_in, dim3(nblk(M * (mc ? C : 1))), dim3(256), 0, s, p, q, perm, M, C, (int)mc);
    KP_LAUNCH_CHECK();
}
void permute_p_to_caller(const float* q, float* p, const int32_t* perm, int64_t M, int C, bool mc, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_p_out, dim3(nblk(M * (mc ? C : 1))), dim3(256), 0, s, q, p, perm, M, C, (int)mc);
    KP_LAUNCH_CHECK();
}

// ------------------------------------------------------------- elementwise
__global__ void k_fill2(float2* x, int64_t n, float2 v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}
__global__ void k_copy2(const float2* a, float2* b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}
void fill2(float2* x, int64_t n, float re, float im, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill2, dim3(nblk(n)), dim3(256), 0, s, x, n, make_float2(re, im));
    KP_LAUNCH_CHECK();
}
void copy2(const float2* a, float2* b, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy2, dim3(nblk(n)), dim3(256), 0, s, a, b, n);
    KP_LAUNCH_CHECK();
}

// ------------------------------------------------------------- reductions
// Deterministic two-stage reductions: a fixed grid of partials, then one
// block sums them in a fixed order.
constexpr int kRedBlocks = 1024;

__device__ double block_sum(double v) {
    __shared__ double sh[256];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}
__device__ float block_min(float v) {
    __shared__ float sm[256];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sm[threadIdx.x] = fminf(sm[threadIdx.x], sm[threadIdx.x + o]);
        __syncthreads();
    }
    float r = sm[0];
    __syncthreads();
    return r;
}

// kinds: 0 = sum |a|^2, 1 = sum |a - b|^2, 2 = sum |a|, 3 = Re sum conj(a) b
__global__ void k_red_partial(const float2* a, const float2* b, int64_t n, int kind, double* part) {
    double acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float2 x = a[i];
        if (kind == 0) {
            acc += (double)x.x * x.x + (double)x.y * x.y;
        } else if (kind == 1) {
            const double dx = (double)x.x - b[i].x, dy = (double)x.y - b[i].y;
            acc += dx * dx + dy * dy;
        } else if (kind == 2) {
            acc += sqrt((double)x.x * x.x + (double)x.y * x.y);
        } else {
            const float2 y = b[i];
            acc += (double)x.x * y.x + (double)x.y * y.y;
        }
    }
    const double r = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}
__global__ void k_red_final(const double* part, int n, double* out, double scale, int accumulate) {
    double acc = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
    const double r = block_sum(acc);
    if (threadIdx.x == 0) *out = (accumulate ? *out : 0.0) + scale * r;
}
__global__ void k_min_partial(const float* p, int64_t n, float* part) {
    float acc = INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc = fminf(acc, p[i]);
    const float r = block_min(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}
__global__ void k_min_final(const float* part, int n, float* out) {
    float acc = INFINITY;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc = fminf(acc, part[i]);
    const float r = block_min(acc);
    if (threadIdx.x == 0) *out = r;
}

void reduce(const float2* a, const float2* b, int64_t n, int kind, double* out, double scale, bool accumulate,
            double* part, hipStream_t s) {
    const int nb = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_red_partial, dim3(nb), dim3(256), 0, s, a, b, n, kind, part);
    KP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_red_final, dim3(1), dim3(256), 0, s, part, nb, out, scale, (int)accumulate);
    KP_LAUNCH_CHECK();
}
void reduce_min(const float* p, int64_t n, float* out, float* part, hipStream_t s) {
    const int nb = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_min_partial, dim3(nb), dim3(256), 0, s, p, n, part);
    KP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_min_final, dim3(1), dim3(256), 0, s, part, nb, out);
    KP_LAUNCH_CHECK();
}

// lam = sqrt(nrm2); scale = 1/lam (power method bookkeeping)
__global__ void k_power_update(const double* nrm2, float* lam, float* scale) {
    const double l = sqrt(*nrm2);
    *lam = (float)l;
    *scale = (float)(l > 0 ? 1.0 / l : 0.0);
}

// sigma_k, tau_k, theta_k for k < K (computed in double)
__global__ void k_schedule(const float* lmax, const float* pmin, int K, float sigma0, int accel, float* sig,
                           float* tau, float* th) {
    double s = sigma0, t = 1.0 / ((double)sigma0 * (double)*lmax);
    const double pm = *pmin;
    for (int k = 0; k < K; ++k) {
        const double h = accel ? 1.0 / (1.0 + 2.0 * s * pm) : 1.0;
        sig[k] = (float)s;
        tau[k] = (float)t;
        th[k] = (float)h;
        s = h * s;
        t = t / h;
    }
}

__global__ void k_set_scalar(float* p, float v) { *p = v; }

// ------------------------------------------------------------- wavelet
__constant__ float c_h[8];
__constant__ float c_g[8];

// The filter constants live in each device's own copy of c_h / c_g: they are
// uploaded once per device (the current one), under a lock so that threads
// driving plans concurrently neither race on the record nor skip a device.
void upload_wavelet_constants() {
    static std::mutex mu;
    static std::set<int> done;
    int dev = 0;
    KP_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if (done.count(dev)) return;
    auto h = db4_filter_host();
    float hf[8], gf[8];
    for (int t = 0; t < 8; ++t) {
        hf[t] = (float)h[t];
        gf[t] = (float)(((t % 2) ? -1.0 : 1.0) * h[7 - t]);
    }
    KP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_h), hf, sizeof(hf)));
    KP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_g), gf, sizeof(gf)));
    done.insert(dev);
}

struct DwtArgs {
    float2* x;
    int S[3];          // element strides of the full image
    int n[3];          // extents of the current approximation block
    int d;
    int ax;
    int inverse;
    int O, I;          // outer / inner counts of the [O][L][I] view
    int Ob, Ib;        // columns per block: Ob outers x Ib inners (at most 64)
    // fused prox steps (0 / null: none)
    int soft;          // analysis: 1 = threshold the details of this level, 2 = every coefficient
    const float* tau;  // threshold = *tau * lam
    float lam;
    float2* ex;        // synthesis: write x_new to ex and ex + theta (x_new - ex_old) to exbar
    float2* exbar;
    const float* theta;
};

constexpr int kDwtK = 16;  // rows per thread at most

// Offset of column/line `c` of the [O][L][I] view: o = c / I enumerates the
// axes before `ax`, i = c % I the axes after it (C order within each).
__device__ __forceinline__ int dwt_base(const DwtArgs& a, int o, int i) {
    int off = 0, rem = o;
    for (int b = a.ax - 1; b >= 0; --b) {
        off += (rem % a.n[b]) * a.S[b];
        rem /= a.n[b];
    }
    rem = i;
    for (int b = a.d - 1; b > a.ax; --b) {
        off += (rem % a.n[b]) * a.S[b];
        rem /= a.n[b];
    }
    return off;
}

// One level along one axis of the approximation block, in place, through LDS.
// analysis: a[k] = sum_t h[t] x[(2k+t) mod L], d[k] = sum_t g[t] x[(2k+t) mod L]
// synthesis: its transpose.  A block holds NL lines of length L; every thread
// owns one line and the rows p, p + P, p + 2P, ... of it (P = 256 / NL).
// Strided axes: lines are NL consecutive inner columns, lanes run across them
// (coalesced over the columns).  Contiguous (last) axis: lanes run along a
// line (coalesced over the rows).
// FUSE: 0 plain; 1 soft threshold on the output (analysis, last axis);
// 2 write x / xbar instead of the output (synthesis).
template <bool LAST, int NL, int FUSE = 0>
__global__ void __launch_bounds__(256) k_dwt_pass(DwtArgs a) {
    extern __shared__ float2 buf[];
    constexpr int P = 256 / NL;
    const int L = a.n[a.ax];
    const int tid = threadIdx.x;
    const int l = LAST ? tid / P : tid % NL;
    const int p = LAST ? tid % P : tid / NL;
    int base = -1;
    if (LAST) {
        const int o = blockIdx.x * NL + l;
        if (o < a.O) base = dwt_base(a, o, 0);
    } else {
        const int nIb = (a.I + NL - 1) / NL;
        const int o = blockIdx.x / nIb, i = (blockIdx.x % nIb) * NL + l;
        if (i < a.I) base = dwt_base(a, o, i);
    }
    const int sr = a.S[a.ax];
    // scalars of the fused steps, read once and early (their load overlaps the
    // row loads; stores through a.x may alias them)
    const float tsoft = FUSE == 1 ? *a.tau * a.lam : 0.f;
    const float th = FUSE == 2 ? *a.theta : 0.f;
    // the line lies in the approximation sub-block of the other axes (last
    // axis only; decides which coefficients are details of this level)
    bool olow = true;
    if (LAST && FUSE == 1 && a.soft == 1) {
        int rem = blockIdx.x * NL + l;
        for (int b = a.ax - 1; b >= 0; --b) {
            olow = olow && (rem % a.n[b]) < a.n[b] / 2;
            rem /= a.n[b];
        }
    }
    // LDS: line-major rows (padded) on the last axis, row-major otherwise
    const int LP = L + 1;
    auto lds = [&](int r) { return LAST ? l * LP + r : r * (NL + 1) + l; };
    float2 v[kDwtK];
    const int bb = base < 0 ? 0 : base;
#pragma unroll
    for (int k = 0; k < kDwtK; ++k) {
        const int r = p + k * P;
        v[k] = a.x[bb + min(r, L - 1) * sr];
    }
#pragma unroll
    for (int k = 0; k < kDwtK; ++k) {
        const int r = p + k * P;
        if (r < L) buf[lds(r)] = v[k];
    }
    __syncthreads();
    if (base < 0) return;
    const int h2 = L / 2;
#pragma unroll
    for (int k = 0; k < kDwtK; ++k) {
        const int r = p + k * P;
        if (r >= L) break;
        float2 acc = make_float2(0.f, 0.f);
        if (!a.inverse) {
            const int kk = r < h2 ? r : r - h2;
            const float* f = r < h2 ? c_h : c_g;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                int src = 2 * kk + t;  // < L + 6
                src = L >= 8 ? (src >= L ? src - L : src) : src % L;
                const float2 u = buf[lds(src)];
                acc.x += f[t] * u.x;
                acc.y += f[t] * u.y;
            }
        } else {
            // x[n] = sum_k h[n-2k] a[k] + g[n-2k] d[k], n-2k taken mod L in [0, 8)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = (r & 1) + 2 * q;
                int kk = (r - t) / 2;  // r - t is even; kk >= -4
                kk = h2 >= 4 ? (kk < 0 ? kk + h2 : kk) : ((kk % h2) + h2) % h2;
                const float2 va = buf[lds(kk)];
                const float2 vd = buf[lds(h2 + kk)];
                acc.x += c_h[t] * va.x + c_g[t] * vd.x;
                acc.y += c_h[t] * va.y + c_g[t] * vd.y;
            }
        }
        if (FUSE == 1 && (a.soft == 2 || r >= h2 || !olow)) {
            // v max(1 - t/|v|, 0), as 1 - t rsqrt(|v|^2) when |v| > t
            const float t = tsoft;
            const float m2 = acc.x * acc.x + acc.y * acc.y;
            const float f = m2 > t * t ? 1.f - t * rsqrtf(m2) : 0.f;
            acc = make_float2(acc.x * f, acc.y * f);
        }
        if (FUSE == 2) {
            const int e = base + r * sr;
            const float2 xo = a.ex[e];
            a.exbar[e] = make_float2(acc.x + th * (acc.x - xo.x), acc.y + th * (acc.y - xo.y));
            a.ex[e] = acc;
        } else {
            a.x[base + r * sr] = acc;
        }
    }
}

void dwt(float2* x, const int64_t* N, int d, int levels, bool inverse, hipStream_t s, const DwtFuse* fz) {
    int64_t tot = 1;
    for (int b = 0; b < d; ++b) tot *= N[b];
    if (tot >= ((int64_t)1 << 31)) fail(KP_ERR_UNSUPPORTED, "wavelet: image too large");
    int S[3] = {1, 1, 1};
    for (int b = d - 2; b >= 0; --b) S[b] = S[b + 1] * (int)N[b + 1];
    auto run_level = [&](int lev) {
        int n[3] = {1, 1, 1};
        for (int b = 0; b < d; ++b) n[b] = (int)(N[b] >> lev);
        auto run_axis = [&](int ax) {
            DwtArgs a{};
            a.x = x;
            for (int b = 0; b < 3; ++b) {
                a.S[b] = S[b];
                a.n[b] = n[b];
            }
            a.d = d;
            a.ax = ax;
            a.inverse = inverse ? 1 : 0;
            if (fz && !inverse && ax == d - 1) {
                // the details of this level are final after its last axis
                a.soft = lev == levels - 1 ? 2 : 1;
                a.tau = fz->tau;
                a.lam = fz->lam;
            }
            if (fz && inverse && lev == 0 && ax == 0) {
                a.ex = fz->ex;
                a.exbar = fz->exbar;
                a.theta = fz->theta;
            }
            a.O = 1;
            a.I = 1;
            for (int b = 0; b < ax; ++b) a.O *= n[b];
            for (int b = ax + 1; b < d; ++b) a.I *= n[b];
            const int L = n[ax];
            // lines per block so that every thread holds at most kDwtK rows
            int NL;
            if (ax == d - 1)
                NL = L <= kDwtK * 32 ? 8 : (L <= kDwtK * 64 ? 4 : 1);
            else
                NL = L <= kDwtK * 16 ? 16 : (L <= kDwtK * 64 ? 4 : 1);
            if (L > kDwtK * 256) fail(KP_ERR_UNSUPPORTED, "wavelet: axis too long");
            const size_t lds = sizeof(float2) * (ax == d - 1 ? (size_t)NL * (L + 1) : (size_t)L * (NL + 1));
            int64_t nb;
            if (ax == d - 1)
                nb = (a.O + NL - 1) / NL;
            else
                nb = (int64_t)a.O * ((a.I + NL - 1) / NL);
            void (*fn)(DwtArgs);
            if (ax == d - 1 && a.soft)
                fn = NL == 8 ? k_dwt_pass<true, 8, 1> : (NL == 4 ? k_dwt_pass<true, 4, 1> : k_dwt_pass<true, 1, 1>);
            else if (ax == d - 1)
                fn = NL == 8 ? k_dwt_pass<true, 8> : (NL == 4 ? k_dwt_pass<true, 4> : k_dwt_pass<true, 1>);
            else if (a.ex)
                fn = NL == 16 ? k_dwt_pass<false, 16, 2>
                              : (NL == 4 ? k_dwt_pass<false, 4, 2> : k_dwt_pass<false, 1, 2>);
            else
                fn = NL == 16 ? k_dwt_pass<false, 16> : (NL == 4 ? k_dwt_pass<false, 4> : k_dwt_pass<false, 1>);
            if (lds > 65536) {
                (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                (void)hipGetLastError();
            }
            hipLaunchKernelGGL(fn, dim3((unsigned)nb), dim3(256), lds, s, a);
            KP_LAUNCH_CHECK();
        };
        if (!inverse)
            for (int ax = 0; ax < d; ++ax) run_axis(ax);
        else
            for (int ax = d - 1; ax >= 0; --ax) run_axis(ax);
    };
    if (!inverse)
        for (int l = 0; l < levels; ++l) run_level(l);
    else
        for (int l = levels - 1; l >= 0; --l) run_level(l);
}

// ---- 3D prox: one launch per level and direction
// A block transforms one brick through LDS: B x B x B coefficient positions
// of each band (analysis) or 2B x 2B x 2B image positions (synthesis).  It
// loads the (2B + 6)^3 values its filters reach (periodic), then filters the
// three axes in turn, so the level costs one read and one write of its
// block instead of three.  Levels alternate between two buffers (z and a
// scratch image), so no block reads what another block of the launch writes:
//   analysis level l reads buffer(l - 1) (z for l = 0) and writes buffer(l),
//   synthesis level l reads buffer(l) and writes the approximation of level
//   l - 1 into the origin block of buffer(l - 1) (x, xbar for l = 0),
// with buffer(l) = scratch for even l, z for odd l.  Each write lands on
// values that an earlier launch has consumed (the low octant of a finer
// level).
struct Dwt3Args {
    const float2* in;
    float2* out;
    int S0, S1;   // element strides of the full image (axis 2 contiguous)
    int n[3];     // extents of this level's approximation block
    int nb[3];    // bricks per axis
    int soft;     // analysis: 1 = threshold the details, 2 = every coefficient
    const float* tau;
    float lam;
    float2* ex;   // synthesis of level 0: x_new to ex, x_new + theta (x_new - ex_old) to exbar
    float2* exbar;
    const float* theta;
};

// Bricks: B_a coefficients per band along axis a (4 x 4 x 4; the level-0
// transform of a wide enough image uses 4 x 4 x 8, whose rows along the
// contiguous axis store 64 / 128 contiguous bytes per band and whose halo is
// 4.2 instead of 5.4 times the brick).
template <int B0, int B1, int B2>
struct Dwt3Brick {
    static constexpr int IN0 = 2 * B0 + 6, IN1 = 2 * B1 + 6, IN2 = 2 * B2 + 6;  // loaded extents
    static constexpr int OB0 = 2 * B0, OB1 = 2 * B1, OB2 = 2 * B2;              // brick outputs per axis
    static constexpr int P2 = IN2 + 1;  // LDS row length along axis 2 (odd, see dwt3_load)
    static_assert(IN0 * IN1 <= 256 && IN0 * OB2 <= 256 && OB1 * OB2 <= 256, "one thread per line of each pass");
    static constexpr size_t lds_bytes() { return sizeof(float2) * (size_t)IN0 * IN1 * P2; }
};

// Brick of this block.  Workgroups go to the 8 XCDs round-robin, so block r
// runs on XCD r % 8; the bricks are dealt so that each XCD gets one
// contiguous run of them (XCD x: bricks [x base + min(x, rem), ...) with
// base = nb / 8, rem = nb % 8, one more for x < rem; a bijection of
// [0, nb)), and a brick's neighbours, whose halos overlap its own, are read
// through the same L2 (level-0 prox 135 -> 111 us).
__device__ __forceinline__ void dwt3_brick(const Dwt3Args& a, int* q) {
    const int nb = a.nb[0] * a.nb[1] * a.nb[2];
    const int x = (int)(blockIdx.x % 8), base = nb / 8, rem = nb % 8;
    int r = x * base + min(x, rem) + (int)(blockIdx.x / 8);
    q[2] = r % a.nb[2];
    r /= a.nb[2];
    q[1] = r % a.nb[1];
    q[0] = r / a.nb[1];
}

// Brick load: the IN0 x IN1 x IN2 input values into LDS.  A thread owns a
// column (u1, u2) of the brick (two for bricks with more than 256 columns)
// and loads its IN0 values along axis 0: its axis-1/2 offset is computed
// once, the axis-0 offsets are the same for the whole block (scalar), and
// every load of the thread is issued before its first LDS write.
// pos(axis, u) gives the element index along an axis of brick row u; the
// products are 24-bit (N1 N2 < 2^24 is checked on the host).  LDS rows along
// axis 2 are padded to an odd length: the axis-2 pass reads one row per
// lane, and rows of an odd number of 8-byte elements put 16 consecutive
// lanes on 16 different bank pairs (with 14, lanes 8 apart shared banks).
template <class K, typename Pos>
__device__ __forceinline__ void dwt3_load(const Dwt3Args& a, float2* buf, Pos pos) {
    constexpr int NCOL = K::IN1 * K::IN2, NR = (NCOL + 255) / 256;
    const int tid = threadIdx.x;
    float2 v[NR][K::IN0];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int c = tid + 256 * k;
        if (c < NCOL) {
            const int u1 = c / K::IN2, u2 = c - u1 * K::IN2;
            const float2* src = a.in + __umul24(pos(1, u1), a.S1) + pos(2, u2);
#pragma unroll
            for (int u0 = 0; u0 < K::IN0; ++u0) v[k][u0] = src[__umul24(pos(0, u0), a.S0)];
        }
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int c = tid + 256 * k;
        if (c < NCOL) {
            const int u1 = c / K::IN2, u2 = c - u1 * K::IN2;
#pragma unroll
            for (int u0 = 0; u0 < K::IN0; ++u0) buf[(u0 * K::IN1 + u1) * K::P2 + u2] = v[k][u0];
        }
    }
}

// Brick load of the analysis: as dwt3_load, but a thread owns two adjacent
// columns (u1, u2), (u1, u2 + 1) with u2 even and reads both with one 16-byte
// load per row.  Along axis 2 the loaded rows 2 k B + u wrap by the even
// extent n, so an even position stays even and its pair never straddles the
// wrap; every stride of the image is even, so those loads are 16-byte aligned.
template <class K, typename Pos>
__device__ __forceinline__ void dwt3_load_pairs(const Dwt3Args& a, float2* buf, Pos pos) {
    static_assert(K::IN2 % 2 == 0, "pairs along axis 2");
    constexpr int HP = K::IN2 / 2, NPAIR = K::IN1 * HP;
    static_assert(NPAIR <= 256, "one pair of columns per thread");
    const int tid = threadIdx.x;
    if (tid >= NPAIR) return;
    const int u1 = tid / HP, u2 = 2 * (tid - u1 * HP);
    const float2* src = a.in + __umul24(pos(1, u1), a.S1) + pos(2, u2);
    float4 v[K::IN0];
#pragma unroll
    for (int u0 = 0; u0 < K::IN0; ++u0) v[u0] = *reinterpret_cast<const float4*>(src + __umul24(pos(0, u0), a.S0));
#pragma unroll
    for (int u0 = 0; u0 < K::IN0; ++u0) {
        float2* d = buf + (u0 * K::IN1 + u1) * K::P2 + u2;
        d[0] = make_float2(v[u0].x, v[u0].y);
        d[1] = make_float2(v[u0].z, v[u0].w);
    }
}

// analysis of one line held in registers: outputs r < B low band, r >= B high
template <int B, int IN>
__device__ __forceinline__ void dwt3_fwd_line(const float2* v, float2* o) {
#pragma unroll
    for (int r = 0; r < 2 * B; ++r) {
        const float* f = r < B ? c_h : c_g;
        const int k = r < B ? r : r - B;
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            acc.x += f[t] * v[2 * k + t].x;
            acc.y += f[t] * v[2 * k + t].y;
        }
        o[r] = acc;
    }
}

// synthesis of one line: v holds B + 3 low then B + 3 high coefficients
// starting 3 before the brick's first; outputs 2B image positions
template <int B>
__device__ __forceinline__ void dwt3_inv_line(const float2* v, float2* o) {
    constexpr int NB = B + 3;
#pragma unroll
    for (int m = 0; m < 2 * B; ++m) {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int t = (m & 1) + 2 * qq;
            const int u = (m - t) / 2 + 3;  // m - t is even
            acc.x += c_h[t] * v[u].x + c_g[t] * v[NB + u].x;
            acc.y += c_h[t] * v[u].y + c_g[t] * v[NB + u].y;
        }
        o[m] = acc;
    }
}

// Each axis is filtered line by line in place: a thread reads its whole line
// into registers and writes the 2B outputs over the line's first 2B entries.
template <int B0, int B1, int B2>
__global__ void __launch_bounds__(256) k_dwt3_analysis(Dwt3Args a) {
    using K = Dwt3Brick<B0, B1, B2>;
    constexpr int IN0 = K::IN0, IN1 = K::IN1, IN2 = K::IN2, OB0 = K::OB0, OB1 = K::OB1, OB2 = K::OB2, P2 = K::P2;
    extern __shared__ float2 buf[];  // [IN0][IN1][P2]
    int q[3];
    dwt3_brick(a, q);
    const int tid = threadIdx.x;
    const float tsoft = *a.tau * a.lam;
    const int h0 = a.n[0] / 2, h1 = a.n[1] / 2, h2 = a.n[2] / 2;
    // input rows 2 k B .. 2 k B + 2B + 5 of every axis, periodic: one wrap
    // needs one subtraction when the extent is at least the loaded extent, a
    // loop otherwise (deep levels of small images)
    dwt3_load_pairs<K>(a, buf, [&](int ax, int u) {
        constexpr int Bs[3] = {B0, B1, B2}, INs[3] = {IN0, IN1, IN2};
        const int n = a.n[ax];
        int sidx = 2 * q[ax] * Bs[ax] + u;
        sidx -= sidx >= n ? n : 0;
        if (n < INs[ax])
            while (sidx >= n) sidx -= n;
        return sidx;
    });
    __syncthreads();
    if (tid < IN0 * IN1) {  // axis 2: line (i0, i1)
        float2 v[IN2], o[OB2];
        float2* line = buf + tid * P2;
#pragma unroll
        for (int j = 0; j < IN2; ++j) v[j] = line[j];
        dwt3_fwd_line<B2, IN2>(v, o);
#pragma unroll
        for (int r = 0; r < OB2; ++r) line[r] = o[r];
    }
    __syncthreads();
    if (tid < IN0 * OB2) {  // axis 1: line (i0, r2)
        float2 v[IN1], o[OB1];
        float2* line = buf + (tid / OB2) * IN1 * P2 + tid % OB2;
#pragma unroll
        for (int j = 0; j < IN1; ++j) v[j] = line[j * P2];
        dwt3_fwd_line<B1, IN1>(v, o);
#pragma unroll
        for (int r = 0; r < OB1; ++r) line[r * P2] = o[r];
    }
    __syncthreads();
    if (tid < OB1 * OB2) {  // axis 0: line (r1, r2), soft threshold, store
        float2 v[IN0], o[OB0];
        const int r1 = tid / OB2, r2 = tid % OB2;
        const float2* line = buf + r1 * P2 + r2;
#pragma unroll
        for (int j = 0; j < IN0; ++j) v[j] = line[j * IN1 * P2];
        dwt3_fwd_line<B0, IN0>(v, o);
        const int c1 = q[1] * B1 + (r1 < B1 ? r1 : r1 - B1);
        const int c2 = q[2] * B2 + (r2 < B2 ? r2 : r2 - B2);
        if (c1 >= h1 || c2 >= h2) return;  // past the block (last brick of an axis)
        const int p12 = __umul24(r1 < B1 ? c1 : h1 + c1, a.S1) + (r2 < B2 ? c2 : h2 + c2);
#pragma unroll
        for (int r0 = 0; r0 < OB0; ++r0) {
            const int c0 = q[0] * B0 + (r0 < B0 ? r0 : r0 - B0);
            if (c0 >= h0) continue;
            float2 acc = o[r0];
            if (a.soft == 2 || r0 >= B0 || r1 >= B1 || r2 >= B2) {
                const float m2 = acc.x * acc.x + acc.y * acc.y;
                const float g = m2 > tsoft * tsoft ? 1.f - tsoft * rsqrtf(m2) : 0.f;
                acc = make_float2(acc.x * g, acc.y * g);
            }
            a.out[__umul24(r0 < B0 ? c0 : h0 + c0, a.S0) + p12] = acc;
        }
    }
}

// x[m] = sum_q h[t] a[(m - t) / 2] + g[t] d[(m - t) / 2], t = (m & 1) + 2q,
// indices mod n / 2; along axis a the brick holds a, d at k0 - 3 .. k0 +
// B_a - 1 (B_a + 3 each)
template <int B0, int B1, int B2, int FUSE>
__global__ void __launch_bounds__(256) k_dwt3_synthesis(Dwt3Args a) {
    using K = Dwt3Brick<B0, B1, B2>;
    constexpr int IN0 = K::IN0, IN1 = K::IN1, IN2 = K::IN2, OB0 = K::OB0, OB1 = K::OB1, OB2 = K::OB2, P2 = K::P2;
    extern __shared__ float2 buf[];  // [IN0][IN1][P2] (per axis: low band u < NB, high band NB + u)
    int q[3];
    dwt3_brick(a, q);
    const int tid = threadIdx.x;
    const float th = FUSE == 2 ? *a.theta : 0.f;
    const int hh[3] = {a.n[0] / 2, a.n[1] / 2, a.n[2] / 2};
    // x_old of the line a last-pass thread will write, loaded first so that
    // its latency hides behind the brick load and the first two passes
    float2 xo[OB0];
    const int m1 = tid / OB2, m2 = tid % OB2;
    const int g1 = 2 * q[1] * B1 + m1, g2 = 2 * q[2] * B2 + m2;
    const bool tail = tid < OB1 * OB2 && g1 < a.n[1] && g2 < a.n[2];
    const int e12 = __umul24(g1, a.S1) + g2;
    if (FUSE == 2 && tail) {
#pragma unroll
        for (int m0 = 0; m0 < OB0; ++m0) {
            const int g0 = min(2 * q[0] * B0 + m0, a.n[0] - 1);
            xo[m0] = a.ex[__umul24(g0, a.S0) + e12];
        }
    }
    // coefficient k0 - 3 + u of each band, periodic in [0, h): one
    // correction each way when h >= B + 3, a loop otherwise
    dwt3_load<K>(a, buf, [&](int ax, int u) {
        constexpr int Bs[3] = {B0, B1, B2};
        const int h = hh[ax], NB = Bs[ax] + 3;
        int kk = q[ax] * Bs[ax] - 3 + (u >= NB ? u - NB : u);
        kk += kk < 0 ? h : 0;
        kk -= kk >= h ? h : 0;
        if (h < NB) {
            while (kk < 0) kk += h;
            while (kk >= h) kk -= h;
        }
        return (u >= NB ? h : 0) + kk;
    });
    __syncthreads();
    if (tid < IN0 * IN1) {  // axis 2
        float2 v[IN2], o[OB2];
        float2* line = buf + tid * P2;
#pragma unroll
        for (int j = 0; j < IN2; ++j) v[j] = line[j];
        dwt3_inv_line<B2>(v, o);
#pragma unroll
        for (int m = 0; m < OB2; ++m) line[m] = o[m];
    }
    __syncthreads();
    if (tid < IN0 * OB2) {  // axis 1
        float2 v[IN1], o[OB1];
        float2* line = buf + (tid / OB2) * IN1 * P2 + tid % OB2;
#pragma unroll
        for (int j = 0; j < IN1; ++j) v[j] = line[j * P2];
        dwt3_inv_line<B1>(v, o);
#pragma unroll
        for (int m = 0; m < OB1; ++m) line[m * P2] = o[m];
    }
    __syncthreads();
    if (tail) {  // axis 0, store (and the x / xbar update on level 0)
        float2 v[IN0], o[OB0];
        const float2* line = buf + m1 * P2 + m2;
#pragma unroll
        for (int j = 0; j < IN0; ++j) v[j] = line[j * IN1 * P2];
        dwt3_inv_line<B0>(v, o);
#pragma unroll
        for (int m0 = 0; m0 < OB0; ++m0) {
            const int g0 = 2 * q[0] * B0 + m0;
            if (g0 >= a.n[0]) continue;
            const int e = __umul24(g0, a.S0) + e12;
            const float2 acc = o[m0];
            if (FUSE == 2) {
                a.exbar[e] = make_float2(acc.x + th * (acc.x - xo[m0].x), acc.y + th * (acc.y - xo[m0].y));
                a.ex[e] = acc;
            } else {
                a.out[e] = acc;
            }
        }
    }
}

// launches of one level with the bricks of K
template <int B0, int B1, int B2>
static void dwt3_level(Dwt3Args a, bool analysis, int fuse, hipStream_t s) {
    using K = Dwt3Brick<B0, B1, B2>;
    const int Bs[3] = {B0, B1, B2};
    for (int b = 0; b < 3; ++b) a.nb[b] = (a.n[b] / 2 + Bs[b] - 1) / Bs[b];
    const dim3 grid((unsigned)(a.nb[0] * a.nb[1] * a.nb[2]));
    const size_t lds = K::lds_bytes();
    if (analysis)
        hipLaunchKernelGGL((k_dwt3_analysis<B0, B1, B2>), grid, dim3(256), lds, s, a);
    else if (fuse == 2)
        hipLaunchKernelGGL((k_dwt3_synthesis<B0, B1, B2, 2>), grid, dim3(256), lds, s, a);
    else
        hipLaunchKernelGGL((k_dwt3_synthesis<B0, B1, B2, 0>), grid, dim3(256), lds, s, a);
    KP_LAUNCH_CHECK();
}

static void dwt3_prox(float2* z, float2* scratch, const int64_t* N, int levels, const DwtFuse& fz, hipStream_t s) {
    if (N[0] * N[1] * N[2] >= ((int64_t)1 << 31) || N[1] * N[2] >= ((int64_t)1 << 24))
        fail(KP_ERR_UNSUPPORTED, "wavelet: image too large (N < 2^31 and N1 N2 < 2^24 elements)");
    auto level_buf = [&](int l) { return (l % 2 == 0) ? scratch : z; };
    auto args = [&](int l) {
        Dwt3Args a{};
        a.S0 = (int)(N[1] * N[2]);
        a.S1 = (int)N[2];
        for (int b = 0; b < 3; ++b) a.n[b] = (int)(N[b] >> l);
        return a;
    };
    // level 0 of an image at least 32 wide along axis 2 on 4 x 4 x 8 bricks
    auto launch = [&](int l, const Dwt3Args& a, bool analysis, int fuse) {
        if (l == 0 && a.n[2] >= 32)
            dwt3_level<4, 4, 8>(a, analysis, fuse, s);
        else
            dwt3_level<4, 4, 4>(a, analysis, fuse, s);
    };
    for (int l = 0; l < levels; ++l) {
        Dwt3Args a = args(l);
        a.in = l == 0 ? z : level_buf(l - 1);
        a.out = level_buf(l);
        a.soft = l == levels - 1 ? 2 : 1;
        a.tau = fz.tau;
        a.lam = fz.lam;
        launch(l, a, true, 0);
    }
    for (int l = levels - 1; l >= 0; --l) {
        Dwt3Args a = args(l);
        a.in = level_buf(l);
        if (l == 0) {
            a.ex = fz.ex;
            a.exbar = fz.exbar;
            a.theta = fz.theta;
            launch(l, a, false, 2);
        } else {
            a.out = level_buf(l - 1);
            launch(l, a, false, 0);
        }
    }
}

// ------------------------------------------------------------- total variation
// G: periodic forward differences along every axis, (G x)_a[n] = x[n + e_a] - x[n];
// G^H v = sum_a v_a[n - e_a] - v_a[n].  The dual variable is stored [d][N].
struct TvGeom {
    int d;
    int N[3];
    int S[3];  // element strides
};

static TvGeom tv_geom(const Plan& P) {
    TvGeom g{};
    g.d = P.d;
    int st = 1;
    for (int a = P.d - 1; a >= 0; --a) {
        g.N[a] = (int)P.N[a];
        g.S[a] = st;
        st *= (int)P.N[a];
    }
    return g;
}

__device__ __forceinline__ int tv_next(const TvGeom& g, int n, int a) {
    const int c = (n / g.S[a]) % g.N[a];
    return c == g.N[a] - 1 ? n - (g.N[a] - 1) * g.S[a] : n + g.S[a];
}
__device__ __forceinline__ int tv_prev(const TvGeom& g, int n, int a) {
    const int c = (n / g.S[a]) % g.N[a];
    return c == 0 ? n + (g.N[a] - 1) * g.S[a] : n - g.S[a];
}

// v <- clip_lambda(v + sigma G xbar), the prox of sigma h* for h = lambda ||.||_1
__global__ void k_tv_dual(float2* v, const float2* xbar, TvGeom g, int n_tot, const float* sigma, float lam) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_tot) return;
    const float sg = *sigma;
    const float2 x0 = xbar[n];
    for (int a = 0; a < g.d; ++a) {
        const float2 x1 = xbar[tv_next(g, n, a)];
        float2 w = v[(int64_t)a * n_tot + n];
        w.x += sg * (x1.x - x0.x);
        w.y += sg * (x1.y - x0.y);
        const float mag = sqrtf(w.x * w.x + w.y * w.y);
        if (mag > lam) {
            const float f = lam / mag;
            w.x *= f;
            w.y *= f;
        }
        v[(int64_t)a * n_tot + n] = w;
    }
}

// x' = z - tau G^H v with z = x - tau A^H u; xbar = x' + theta (x' - x); x = x'
__global__ void k_tv_primal(const float2* z, const float2* v, float2* x, float2* xbar, TvGeom g, int n_tot,
                            const float* tau, const float* theta) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_tot) return;
    float2 gh = make_float2(0.f, 0.f);
    for (int a = 0; a < g.d; ++a) {
        const float2 vp = v[(int64_t)a * n_tot + tv_prev(g, n, a)];
        const float2 vn = v[(int64_t)a * n_tot + n];
        gh.x += vp.x - vn.x;
        gh.y += vp.y - vn.y;
    }
    const float t = *tau, th = *theta;
    const float2 zv = z[n], xo = x[n];
    const float2 xn = make_float2(zv.x - t * gh.x, zv.y - t * gh.y);
    xbar[n] = make_float2(xn.x + th * (xn.x - xo.x), xn.y + th * (xn.y - xo.y));
    x[n] = xn;
}

// sum_n sum_a |(G x)_a[n]| (per-block partial sums in FP64)
__global__ void k_red_tv(const float2* x, TvGeom g, int n_tot, double* part) {
    double acc = 0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < n_tot; n += gridDim.x * blockDim.x) {
        const float2 x0 = x[n];
        for (int a = 0; a < g.d; ++a) {
            const float2 x1 = x[tv_next(g, n, a)];
            const double dx = (double)x1.x - x0.x, dy = (double)x1.y - x0.y;
            acc += sqrt(dx * dx + dy * dy);
        }
    }
    const double r = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// lambda_max(G G^H) = sum_a max_k 2 (1 - cos(2 pi k / N_a))
static double tv_lmax(const Plan& P) {
    double t = 0;
    for (int a = 0; a < P.d; ++a) {
        double m = 0;
        for (int64_t k = 0; k < P.N[a]; ++k) m = std::max(m, 2.0 * (1.0 - std::cos(2.0 * M_PI * (double)k / (double)P.N[a])));
        t += m;
    }
    return t;
}

// constant TV steps: sigma = theta = 1, tau = 1 / (lambda_max + lambda_max(G G^H))
__global__ void k_schedule_tv(const float* lmax, double lgg, int K, float* sig, float* tau, float* th) {
    const float t = (float)(1.0 / ((double)*lmax + lgg));
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        sig[k] = 1.f;
        tau[k] = t;
        th[k] = 1.f;
    }
}

// ------------------------------------------------------------- operators
// Apply A^H P A to v (power method step), result into `out`.
static void normal_op(Plan& P, const float2* v, const float* xscale, const float* pint, int p_mc, float2* out,
                      hipStream_t s) {
    FwdOpts fo;
    fo.xscale = xscale;
    float2* grid = forward_to_grid(P, v, fo, s);
    InterpArgs ia{};
    ia.mode = IO_PMUL;
    ia.out = P.kint3.as<float2>();
    ia.p = pint;
    ia.p_mc = p_mc;
    interp(P, grid, ia, s);
    float2* g2 = spread_to_grid(P, P.kint3.as<float2>(), (int)P.C, s);
    AdjOpts ao;
    grid_to_image(P, g2, out, ao, s);
}

// scalar slots in P.sched after the 3*8192 schedule entries
enum { SL_LMAX = 0, SL_PMIN = 1, SL_SCALE = 2, SL_ONE = 3 };
static float* slot(Plan& P, int i) { return P.sched.as<float>() + 3 * 8192 + i; }

void power_method(Plan& P, const float* pint, int p_mc, int iters, float* lam_out, hipStream_t s) {
    float2* v = P.img[2].as<float2>();
    double* nrm = P.red.as<double>();
    double* part = P.red.as<double>() + 16;
    fill2(v, P.Ntot, (float)(1.0 / std::sqrt((double)P.Ntot)), 0.f, s);
    hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, slot(P, SL_SCALE), 1.f);
    KP_LAUNCH_CHECK();
    for (int it = 0; it < iters; ++it) {
        normal_op(P, v, slot(P, SL_SCALE), pint, p_mc, v, s);
        reduce(v, nullptr, P.Ntot, 0, nrm, 1.0, false, part, s);
        hipLaunchKernelGGL(k_power_update, dim3(1), dim3(1), 0, s, nrm, lam_out, slot(P, SL_SCALE));
        KP_LAUNCH_CHECK();
    }
}

// objective 1/2 ||A x - y||^2 + g(x) into host
static double objective(Plan& P, const float2* x, const float2* yint, int reg, float lam, int levels,
                        hipStream_t s) {
    double* acc = P.red.as<double>() + 8;
    double* part = P.red.as<double>() + 16;
    FwdOpts fo;
    float2* grid = forward_to_grid(P, x, fo, s);
    InterpArgs ia{};
    ia.mode = IO_INTERNAL;
    ia.out = P.kint3.as<float2>();
    interp(P, grid, ia, s);
    reduce(P.kint3.as<float2>(), yint, P.M * P.C, 1, acc, 0.5, false, part, s);
    if (reg == KP_REG_L2) {
        reduce(x, nullptr, P.Ntot, 0, acc, 0.5 * lam, true, part, s);
    } else if (reg == KP_REG_TV) {
        const int nb = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (P.Ntot + 255) / 256));
        hipLaunchKernelGGL(k_red_tv, dim3(nb), dim3(256), 0, s, x, tv_geom(P), (int)P.Ntot, part);
        KP_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_red_final, dim3(1), dim3(256), 0, s, part, nb, acc, (double)lam, 1);
        KP_LAUNCH_CHECK();
    } else {
        float2* w = P.img[3].as<float2>();
        copy2(x, w, P.Ntot, s);
        dwt(w, P.N, P.d, levels, false, s);
        reduce(w, nullptr, P.Ntot, 2, acc, lam, true, part, s);
    }
    double h = 0;
    KP_HIP(hipMemcpyAsync(&h, acc, sizeof(double), hipMemcpyDeviceToHost, s));
    KP_HIP(hipStreamSynchronize(s));
    return h;
}

static void check_p(const Plan& P, const float* p, int p_kind) {
    if (p_kind != KP_PRECOND_NONE && p_kind != KP_PRECOND_SC && p_kind != KP_PRECOND_MC)
        fail(KP_ERR_INVALID_ARG, "p_kind must be NONE, SC or MC");
    if (p_kind != KP_PRECOND_NONE && !p) fail(KP_ERR_INVALID_ARG, "p is NULL");
    (void)P;
}

// load p into P.pint (internal order); returns the pointer to pass to kernels
const float* load_p(Plan& P, const float* p, int p_kind, hipStream_t s) {
    if (p_kind == KP_PRECOND_NONE) return nullptr;
    const bool mc = p_kind == KP_PRECOND_MC;
    permute_p_to_internal(p, P.pint.as<float>(), P.perm.as<int32_t>(), P.M, (int)P.C, mc, s);
    return P.pint.as<float>();
}

// Validate options; load y, p, u0, x0 into the plan's internal buffers
// (kint2, pint, kint, img[0], img[1]); compute min p, lambda_max and the
// step schedule on the device.
void pdhg_setup(Plan& P, const float2* y, const float* p, int p_kind, const kp_pdhg_opts& op, hipStream_t s) {
    check_p(P, p, p_kind);
    if (op.iters < 1 || op.iters > 8192) fail(KP_ERR_INVALID_ARG, "iters must lie in [1, 8192]");
    if (op.reg != KP_REG_L2 && op.reg != KP_REG_L1_WAVELET && op.reg != KP_REG_TV)
        fail(KP_ERR_INVALID_ARG, "unknown regulariser");
    if (op.reg == KP_REG_TV) {
        if (!P.tvv.p) fail(KP_ERR_UNSUPPORTED, "TV needs a plan with coil maps or one coil");
        if (P.Ntot >= ((int64_t)1 << 31)) fail(KP_ERR_UNSUPPORTED, "TV: image too large");
    }
    if (!(op.lambda >= 0.f)) fail(KP_ERR_INVALID_ARG, "lambda must be >= 0");
    if (!(op.sigma0 > 0.f)) fail(KP_ERR_INVALID_ARG, "sigma0 must be > 0");
    const int levels = op.wavelet_levels;
    if (op.reg == KP_REG_L1_WAVELET) {
        if (levels < 1 || levels > 8) fail(KP_ERR_INVALID_ARG, "wavelet_levels must lie in [1, 8]");
        for (int a = 0; a < P.d; ++a)
            if (P.N[a] % (1 << levels)) fail(KP_ERR_INVALID_ARG, "every N_a must be divisible by 2^levels");
        upload_wavelet_constants();
    }
    if (op.lambda_max <= 0.f && op.power_iters < 1) fail(KP_ERR_INVALID_ARG, "power_iters must be >= 1");
    const int C = (int)P.C;
    const int K = op.iters;
    const int p_mc = p_kind == KP_PRECOND_MC ? 1 : 0;
    float* sig = P.sched.as<float>();
    float* tau = sig + 8192;
    float* th = tau + 8192;

    // y, p, u, x into internal layouts
    float2* yint = P.kint2.as<float2>();
    float2* u = P.kint.as<float2>();
    permute_to_internal(y, yint, P.perm.as<int32_t>(), P.M, C, s, P.iperm.as<int32_t>());
    const float* pint = load_p(P, p, p_kind, s);
    if (op.u0)
        permute_to_internal((const float2*)op.u0, u, P.perm.as<int32_t>(), P.M, C, s, P.iperm.as<int32_t>());
    else
        fill2(u, P.M * C, 0.f, 0.f, s);
    float2* x = P.img[0].as<float2>();
    float2* xbar = P.img[1].as<float2>();
    if (op.x0)
        copy2((const float2*)op.x0, x, P.Ntot, s);
    else
        fill2(x, P.Ntot, 0.f, 0.f, s);
    copy2(x, xbar, P.Ntot, s);

    // min p and lambda_max, then the schedule, all on the device
    if (pint)
        reduce_min(pint, P.M * (p_mc ? C : 1), slot(P, SL_PMIN), (float*)(P.red.as<double>() + 4096), s);
    else
        hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, slot(P, SL_PMIN), 1.f);
    if (op.lambda_max > 0.f) {
        hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, slot(P, SL_LMAX), op.lambda_max);
    } else {
        power_method(P, pint, p_mc, op.power_iters, slot(P, SL_LMAX), s);
    }
    KP_LAUNCH_CHECK();
    if (op.lambda_max_out)
        KP_HIP(hipMemcpyAsync(op.lambda_max_out, slot(P, SL_LMAX), sizeof(float), hipMemcpyDeviceToDevice, s));
    if (op.reg == KP_REG_TV) {
        hipLaunchKernelGGL(k_schedule_tv, dim3(1), dim3(256), 0, s, slot(P, SL_LMAX), tv_lmax(P), K, sig, tau, th);
        fill2(P.tvv.as<float2>(), P.Ntot * P.d, 0.f, 0.f, s);
    } else {
        hipLaunchKernelGGL(k_schedule, dim3(1), dim3(1), 0, s, slot(P, SL_LMAX), slot(P, SL_PMIN), K, op.sigma0,
                           op.accel, sig, tau, th);
    }
    KP_LAUNCH_CHECK();
}

void pdhg_solve_impl(Plan& P, const float2* y, const float* p, int p_kind, const kp_pdhg_opts& op, float2* x_out,
                     float2* u_out, hipStream_t s) {
    pdhg_setup(P, y, p, p_kind, op, s);
    const int C = (int)P.C;
    const int K = op.iters;
    const int levels = op.wavelet_levels;
    const int p_mc = p_kind == KP_PRECOND_MC ? 1 : 0;
    const float* pint = p_kind == KP_PRECOND_NONE ? nullptr : P.pint.as<float>();
    float* sig = P.sched.as<float>();
    float* tau = sig + 8192;
    float* th = tau + 8192;
    float2* yint = P.kint2.as<float2>();
    float2* u = P.kint.as<float2>();
    float2* x = P.img[0].as<float2>();
    float2* xbar = P.img[1].as<float2>();
    float2* z = P.img[2].as<float2>();
    if (op.objective_host) op.objective_host[0] = objective(P, x, yint, op.reg, op.lambda, levels, s);
    for (int k = 0; k < K; ++k) {
        FwdOpts fo;
        float2* grid = forward_to_grid(P, xbar, fo, s);
        InterpArgs ia{};
        ia.mode = IO_DUAL;
        ia.u = u;
        ia.y = yint;
        ia.p = pint;
        ia.p_mc = p_mc;
        ia.sigma = sig + k;
        interp(P, grid, ia, s);
        float2* g2 = spread_to_grid(P, u, C, s);
        AdjOpts ao;
        ao.ex = x;
        ao.tau = tau + k;
        ao.theta = th + k;
        ao.lambda = op.lambda;
        if (op.reg == KP_REG_L2) {
            ao.epi = EPI_L2;
            ao.exbar = xbar;
            grid_to_image(P, g2, z, ao, s);
        } else if (op.reg == KP_REG_TV) {
            // the new v uses the xbar of this iteration: update it before x changes
            const TvGeom tg = tv_geom(P);
            float2* v = P.tvv.as<float2>();
            hipLaunchKernelGGL(k_tv_dual, dim3(nblk(P.Ntot)), dim3(256), 0, s, v, xbar, tg, (int)P.Ntot, sig + k,
                               op.lambda);
            KP_LAUNCH_CHECK();
            ao.epi = EPI_Z;
            ao.exbar = z;
            grid_to_image(P, g2, z, ao, s);
            hipLaunchKernelGGL(k_tv_primal, dim3(nblk(P.Ntot)), dim3(256), 0, s, z, v, x, xbar, tg, (int)P.Ntot,
                               tau + k, th + k);
            KP_LAUNCH_CHECK();
        } else {
            ao.epi = EPI_Z;
            ao.exbar = z;
            grid_to_image(P, g2, z, ao, s);
            // x_new = W^H soft(W z): the soft threshold is fused into the
            // analysis passes, x, xbar <- x_new, x_new + theta (x_new - x)
            // into the last synthesis pass (levels >= 1 was checked)
            DwtFuse fz{tau + k, op.lambda, x, xbar, th + k};
            if (P.d == 3) {
                dwt3_prox(z, P.img[3].as<float2>(), P.N, levels, fz, s);
            } else {
                dwt(z, P.N, P.d, levels, false, s, &fz);
                dwt(z, P.N, P.d, levels, true, s, &fz);
            }
        }
        if (op.objective_host) op.objective_host[k + 1] = objective(P, x, yint, op.reg, op.lambda, levels, s);
    }
    copy2(x, x_out, P.Ntot, s);
    if (u_out) permute_to_caller(u, u_out, P.perm.as<int32_t>(), P.M, C, s);
}


// One l1-db4 prox step x = W^H soft(W z) on the plan's image workspaces (z =
// img[2], x = img[0], xbar = img[1], scratch img[3]) with the deepest level
// count up to 4 that every N_a allows, as the PDHG loop runs it: a timing aid
// (the threshold and theta are set to fixed values first).
void wavelet_prox_stage(Plan& P, hipStream_t s) {
    int levels = 0;
    while (levels < 4) {
        bool ok = true;
        for (int a = 0; a < P.d; ++a) ok = ok && P.N[a] % (2 << levels) == 0;
        if (!ok) break;
        ++levels;
    }
    if (levels == 0) fail(KP_ERR_UNSUPPORTED, "wavelet: no level fits the image shape");
    upload_wavelet_constants();
    float* tau = P.sched.as<float>() + 8192;
    float* th = tau + 8192;
    hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, tau, 1e-3f);
    hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, th, 1.f);
    KP_LAUNCH_CHECK();
    float2* z = P.img[2].as<float2>();
    DwtFuse fz{tau, 5e-3f, P.img[0].as<float2>(), P.img[1].as<float2>(), th};
    if (P.d == 3) {
        dwt3_prox(z, P.img[3].as<float2>(), P.N, levels, fz, s);
    } else {
        dwt(z, P.N, P.d, levels, false, s, &fz);
        dwt(z, P.N, P.d, levels, true, s, &fz);
    }
}


// ------------------------------------------------------------- l2 dual solver
// Supporting Materials, connection to Trzasko et al.: the dual optimum of the
// l2 problem solves (A A^H + lambda I) u = lambda y, and x = A^H u / lambda.
// Conjugate gradients with the diagonal k-space preconditioner as M^-1 = P;
// every scalar stays on the device (no host synchronisation per iteration).

// sum_i p_i |r_i|^2 (p per sample [M], per sample and coil [M][C], or 1)
__global__ void k_red_pnorm(const float2* r, const float* p, int p_mc, int C, int64_t n, double* part) {
    double acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float2 v = r[i];
        const double w = p ? (double)(p_mc ? p[i] : p[i / C]) : 1.0;
        acc += w * ((double)v.x * v.x + (double)v.y * v.y);
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// init: r = lam y (r holds y), u = 0, d = P r
__global__ void k_cg_init(float2* r, float2* u, float2* d, const float* p, int p_mc, int C, int64_t n, float lam) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 v = make_float2(lam * r[i].x, lam * r[i].y);
    const float w = p ? (p_mc ? p[i] : p[i / C]) : 1.f;
    r[i] = v;
    u[i] = make_float2(0.f, 0.f);
    d[i] = make_float2(w * v.x, w * v.y);
}

// alpha = rz / dq; u += alpha d; r -= alpha q
__global__ void k_cg_ur(float2* u, float2* r, const float2* d, const float2* q, const double* rz, const double* dq,
                        int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float al = (float)(*rz / *dq);
    const float2 dv = d[i], qv = q[i];
    u[i] = make_float2(u[i].x + al * dv.x, u[i].y + al * dv.y);
    r[i] = make_float2(r[i].x - al * qv.x, r[i].y - al * qv.y);
}

// beta = rz_new / rz; d = P r + beta d
__global__ void k_cg_d(float2* d, const float2* r, const float* p, int p_mc, int C, int64_t n, const double* rz_new,
                       const double* rz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float be = (float)(*rz_new / *rz);
    const float w = p ? (p_mc ? p[i] : p[i / C]) : 1.f;
    const float2 rv = r[i], dv = d[i];
    d[i] = make_float2(w * rv.x + be * dv.x, w * rv.y + be * dv.y);
}

__global__ void k_axpy2(float2* q, const float2* d, float a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    q[i] = make_float2(q[i].x + a * d[i].x, q[i].y + a * d[i].y);
}

__global__ void k_scale_copy(const float2* a, float2* b, float f, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = make_float2(f * a[i].x, f * a[i].y);
}

static void pnorm(const float2* r, const float* p, int p_mc, int C, int64_t n, double* out, double* part,
                  hipStream_t s) {
    const int nb = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_red_pnorm, dim3(nb), dim3(256), 0, s, r, p, p_mc, C, n, part);
    KP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_red_final, dim3(1), dim3(256), 0, s, part, nb, out, 1.0, 0);
    KP_LAUNCH_CHECK();
}

void l2_dual_cg_impl(Plan& P, const float2* y, const float* p, int p_kind, float lam, int iters, float2* x_out,
                     float2* u_out, double* res_host, hipStream_t s) {
    check_p(P, p, p_kind);
    if (iters < 1 || iters > 8192) fail(KP_ERR_INVALID_ARG, "iters must lie in [1, 8192]");
    if (!(lam > 0.f)) fail(KP_ERR_INVALID_ARG, "lambda must be > 0");
    if (!P.kint4.p) fail(KP_ERR_UNSUPPORTED, "the dual solver needs a plan with coil maps or one coil");
    const int C = (int)P.C;
    const int64_t n = P.M * C;
    const int p_mc = p_kind == KP_PRECOND_MC ? 1 : 0;
    float2* r = P.kint2.as<float2>();
    float2* d = P.kint.as<float2>();
    float2* q = P.kint3.as<float2>();
    float2* u = P.kint4.as<float2>();
    float2* img = P.img[0].as<float2>();
    double* sl = P.red.as<double>() + 2048;  // rz (two slots), dq, |r|^2, |r0|^2
    double* part = P.red.as<double>() + 16;
    permute_to_internal(y, r, P.perm.as<int32_t>(), P.M, C, s, P.iperm.as<int32_t>());
    const float* pint = load_p(P, p, p_kind, s);
    hipLaunchKernelGGL(k_cg_init, dim3(nblk(n)), dim3(256), 0, s, r, u, d, pint, p_mc, C, n, lam);
    KP_LAUNCH_CHECK();
    pnorm(r, pint, p_mc, C, n, sl + 0, part, s);
    double r0 = 0;
    if (res_host) {
        reduce(r, nullptr, n, 0, sl + 4, 1.0, false, part, s);
        KP_HIP(hipMemcpyAsync(&r0, sl + 4, sizeof(double), hipMemcpyDeviceToHost, s));
        KP_HIP(hipStreamSynchronize(s));
        r0 = std::sqrt(r0);
        res_host[0] = 1.0;
    }
    int cur = 0;
    for (int it = 0; it < iters; ++it) {
        // q = (A A^H + lam I) d
        float2* g2 = spread_to_grid(P, d, C, s);
        AdjOpts ao;
        grid_to_image(P, g2, img, ao, s);
        FwdOpts fo;
        float2* grid = forward_to_grid(P, img, fo, s);
        InterpArgs ia{};
        ia.mode = IO_INTERNAL;
        ia.out = q;
        interp(P, grid, ia, s);
        hipLaunchKernelGGL(k_axpy2, dim3(nblk(n)), dim3(256), 0, s, q, d, lam, n);
        KP_LAUNCH_CHECK();
        reduce(d, q, n, 3, sl + 2, 1.0, false, part, s);
        hipLaunchKernelGGL(k_cg_ur, dim3(nblk(n)), dim3(256), 0, s, u, r, d, q, sl + cur, sl + 2, n);
        KP_LAUNCH_CHECK();
        pnorm(r, pint, p_mc, C, n, sl + (1 - cur), part, s);
        hipLaunchKernelGGL(k_cg_d, dim3(nblk(n)), dim3(256), 0, s, d, r, pint, p_mc, C, n, sl + (1 - cur), sl + cur);
        KP_LAUNCH_CHECK();
        cur = 1 - cur;
        if (res_host) {
            double rr = 0;
            reduce(r, nullptr, n, 0, sl + 3, 1.0, false, part, s);
            KP_HIP(hipMemcpyAsync(&rr, sl + 3, sizeof(double), hipMemcpyDeviceToHost, s));
            KP_HIP(hipStreamSynchronize(s));
            res_host[it + 1] = r0 > 0 ? std::sqrt(rr) / r0 : 0.0;
        }
    }
    // x = A^H u / lam
    float2* g2 = spread_to_grid(P, u, C, s);
    AdjOpts ao;
    grid_to_image(P, g2, img, ao, s);
    hipLaunchKernelGGL(k_scale_copy, dim3(nblk(P.Ntot)), dim3(256), 0, s, img, x_out, 1.f / lam, P.Ntot);
    KP_LAUNCH_CHECK();
    if (u_out) permute_to_caller(u, u_out, P.perm.as<int32_t>(), P.M, C, s);
}

}  // namespace kp

using namespace kp;

extern "C" {

int pdhg_lambda_max(kp_plan_t plan, const float* p, int p_kind, int iters, float* out, void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl || !out) fail(KP_ERR_INVALID_ARG, "NULL argument");
        if (iters < 1) fail(KP_ERR_INVALID_ARG, "iters must be >= 1");
        Plan& P = *plan->impl;
        require_plan_device(P);
        check_p(P, p, p_kind);
        hipStream_t s = (hipStream_t)stream;
        const float* pint = load_p(P, p, p_kind, s);
        power_method(P, pint, p_kind == KP_PRECOND_MC ? 1 : 0, iters, out, s);
    });
}

int pdhg_schedule_params(kp_plan_t plan, const float* p, int p_kind, const kp_pdhg_opts* opts, float* params,
                         void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl || !opts || !params) fail(KP_ERR_INVALID_ARG, "NULL argument");
        Plan& P = *plan->impl;
        require_plan_device(P);
        const kp_pdhg_opts& op = *opts;
        check_p(P, p, p_kind);
        const int K = op.iters;
        if (K < 1 || K > 8192) fail(KP_ERR_INVALID_ARG, "iters must lie in [1, 8192]");
        if (!(op.lambda >= 0.f)) fail(KP_ERR_INVALID_ARG, "lambda must be >= 0");
        if (!(op.sigma0 > 0.f)) fail(KP_ERR_INVALID_ARG, "sigma0 must be > 0");
        if (op.lambda_max <= 0.f && op.power_iters < 1) fail(KP_ERR_INVALID_ARG, "power_iters must be >= 1");
        hipStream_t s = (hipStream_t)stream;
        const int p_mc = p_kind == KP_PRECOND_MC ? 1 : 0;
        const float* pint = load_p(P, p, p_kind, s);
        if (pint)
            reduce_min(pint, P.M * (p_mc ? P.C : 1), slot(P, SL_PMIN), (float*)(P.red.as<double>() + 4096), s);
        else
            hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, slot(P, SL_PMIN), 1.f);
        if (op.lambda_max > 0.f)
            hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, slot(P, SL_LMAX), op.lambda_max);
        else
            power_method(P, pint, p_mc, op.power_iters, slot(P, SL_LMAX), s);
        KP_LAUNCH_CHECK();
        if (op.lambda_max_out)
            KP_HIP(hipMemcpyAsync(op.lambda_max_out, slot(P, SL_LMAX), sizeof(float), hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_schedule, dim3(1), dim3(1), 0, s, slot(P, SL_LMAX), slot(P, SL_PMIN), K, op.sigma0,
                           op.accel, params, params + K, params + 2 * K);
        hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, params + 3 * K, op.lambda);
        KP_LAUNCH_CHECK();
    });
}

int l2_dual_cg(kp_plan_t plan, const void* y, const float* p, int p_kind, float lambda, int iters, void* x_out,
               void* u_out, double* residual_host, void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl || !y || !x_out) fail(KP_ERR_INVALID_ARG, "NULL argument");
        require_plan_device(*plan->impl);
        l2_dual_cg_impl(*plan->impl, (const float2*)y, p, p_kind, lambda, iters, (float2*)x_out, (float2*)u_out,
                        residual_host, (hipStream_t)stream);
    });
}

int pdhg_solve(kp_plan_t plan, const void* y, const float* p, int p_kind, const kp_pdhg_opts* opts, void* x_out,
               void* u_out, void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl || !opts || !y || !x_out) fail(KP_ERR_INVALID_ARG, "NULL argument");
        require_plan_device(*plan->impl);
        pdhg_solve_impl(*plan->impl, (const float2*)y, p, p_kind, *opts, (float2*)x_out, (float2*)u_out,
                        (hipStream_t)stream);
    });
}

}  // extern "C"
