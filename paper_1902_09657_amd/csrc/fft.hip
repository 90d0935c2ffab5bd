// LDS-staged mixed-radix Stockham FFT passes for the oversampled NUFFT grid.
//
// One pass transforms every line of a [O][L][I] view along its middle axis
// (I contiguous).  A workgroup stages `Ob x Ib` columns of length L in LDS,
// runs the Stockham stages (radices 2, 3, 4, 5, 8; twiddles exp(-2 pi i m/L)
// from a float table built in double precision on the host) between two LDS
// buffers, and writes the result back.  Pruning: a forward pass reads only the
// N non-zero input rows (centred placement n mod L, the zero rows are never
// read) and an adjoint pass writes only the N kept output rows (centred crop).
//
// Three kernels share this contract: the general pass (any length, two LDS
// buffers), the specialised LDS-staged pass (compile-time length and column
// block, stages in place in one buffer) and, for plain 32-column passes of
// lengths 160, 200, 240 and 256, a register-resident two-factor pass (one
// LDS transpose per pass; below).
//
// The first forward pass along the last image axis fuses the pre-pass of the
// NUFFT (coil multiply x s_c, deapodisation 1/(sqrt(N) Chat), and the sign
// (-1)^n that centres the spectrum so grid cell G/2 is k = 0); the last
// adjoint pass fuses the mirror post-pass (conj(s_c), deapodisation, sign,
// coil sum) and, optionally, the PDHG primal update.
#include <algorithm>
#include <type_traits>

#include "kp_internal.h"

namespace kp {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
__device__ __forceinline__ float2 rot(float2 a, int inv) {
    return inv ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// cos(2 pi/5) = (sqrt5 - 1)/4, cos(4 pi/5) = -(sqrt5 + 1)/4,
// sin(2 pi/5) = sqrt(10 + 2 sqrt5)/4, sin(4 pi/5) = sqrt(10 - 2 sqrt5)/4,
// sin(2 pi/3) = sqrt3/2, cos(pi/4) = sqrt2/2
#define KP_C51 0.30901699437494742f
#define KP_C52 -0.80901699437494742f
#define KP_S51 0.95105651629515357f
#define KP_S52 0.58778525229247313f
#define KP_S3 0.86602540378443865f
#define KP_R2 0.70710678118654752f

__device__ __forceinline__ void dft2(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}
__device__ __forceinline__ void dft3(float2* v, int inv) {
    float2 t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
    float2 m = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
    float2 r = rot(cscale(t2, KP_S3), inv);  // -i s t2 (forward)
    v[0] = cadd(v[0], t1);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}
__device__ __forceinline__ void dft4(float2* v, int inv) {
    float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    float2 b0 = cadd(v[1], v[3]), b1 = rot(csub(v[1], v[3]), inv);
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
}
__device__ __forceinline__ void dft5(float2* v, int inv) {
    float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    float2 b1 = make_float2(v[0].x + KP_C51 * t1.x + KP_C52 * t2.x, v[0].y + KP_C51 * t1.y + KP_C52 * t2.y);
    float2 b2 = make_float2(v[0].x + KP_C52 * t1.x + KP_C51 * t2.x, v[0].y + KP_C52 * t1.y + KP_C51 * t2.y);
    float2 d1 = make_float2(KP_S51 * t3.x + KP_S52 * t4.x, KP_S51 * t3.y + KP_S52 * t4.y);
    float2 d2 = make_float2(KP_S52 * t3.x - KP_S51 * t4.x, KP_S52 * t3.y - KP_S51 * t4.y);
    float2 r1 = rot(d1, inv), r2 = rot(d2, inv);  // -i d (forward)
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(b1, r1);
    v[4] = csub(b1, r1);
    v[2] = cadd(b2, r2);
    v[3] = csub(b2, r2);
}
__device__ __forceinline__ void dft8(float2* v, int inv) {
    // radix-2 split into two 4-point DFTs of even and odd samples
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft4(e, inv);
    dft4(o, inv);
    // twiddles w8^k, w8 = exp(-+ 2 pi i / 8)
    float s = inv ? 1.f : -1.f;
    float2 w1 = make_float2(KP_R2, s * KP_R2);
    float2 w3 = make_float2(-KP_R2, s * KP_R2);
    float2 o1 = cmul(o[1], w1);
    float2 o2 = rot(o[2], inv);
    float2 o3 = cmul(o[3], w3);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

__device__ __forceinline__ void dft_r(int R, float2* v, int inv) {
    switch (R) {
        case 2: dft2(v); break;
        case 3: dft3(v, inv); break;
        case 4: dft4(v, inv); break;
        case 5: dft5(v, inv); break;
        default: dft8(v, inv); break;
    }
}

__global__ void __launch_bounds__(256) k_fft_pass(FftPass p) {
    extern __shared__ float2 lds[];
    const int ncol = p.Ob * p.Ib;
    const int L = p.L;
    float2* b0 = lds;
    float2* b1 = lds + (size_t)L * ncol;
    const int64_t nIb = (p.I + p.Ib - 1) / p.Ib;
    const int64_t bid = blockIdx.x;
    const int64_t o0 = (bid / nIb) * p.Ob;
    const int64_t i0 = (bid % nIb) * p.Ib;
    const int tid = threadIdx.x, nt = blockDim.x;
    const float xs = p.xscale ? *p.xscale : 1.f;

    // ---- load (pruned: only the Lin input rows are read)
    if (p.pad_in) {
        const int gap = L - p.Lin;
        const int r0 = p.Lin / 2;
        for (int idx = tid; idx < gap * ncol; idx += nt) {
            int row = r0 + idx / ncol, col = idx % ncol;
            b0[row * ncol + col] = make_float2(0.f, 0.f);
        }
    }
    for (int idx = tid; idx < p.Lin * ncol; idx += nt) {
        const int r = idx / ncol, col = idx % ncol;
        const int64_t o = o0 + col / p.Ib, i = i0 + col % p.Ib;
        float2 v = make_float2(0.f, 0.f);
        if (o < p.O && i < p.I) {
            if (p.pre == PRE_NONE) {
                v = p.in[o * p.in_os + r * p.in_rs + i];
            } else if (p.pre == PRE_MAPS) {
                const int64_t e = o * p.Lin + r;
                const float f = p.fo[o] * p.fr[r] * xs;
                v = cscale(cmul(p.px[e], p.pmaps[e * p.I + i]), f);
            } else {
                const int64_t e = o * p.Lin + r;
                const float f = p.fo[o] * p.fr[r] * xs;
                v = cscale(p.px[e * p.I + i], f);
            }
        }
        const int pos = p.pad_in ? (r - p.Lin / 2 + L) % L : r;
        b0[pos * ncol + col] = v;
    }
    __syncthreads();

    // ---- Stockham stages
    float2* src = b0;
    float2* dst = b1;
    int Ns = 1;
    for (int s = 0; s < p.nst; ++s) {
        const int R = p.rad[s];
        const int nbf = L / R;
        const int stride = L / (Ns * R);
        for (int b = tid; b < nbf * ncol; b += nt) {
            const int col = b % ncol, j = b / ncol;
            const int k = j % Ns;
            float2 v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (t < R) v[t] = src[(j + t * nbf) * ncol + col];
            if (Ns > 1) {
#pragma unroll
                for (int t = 1; t < 8; ++t) {
                    if (t < R) {
                        float2 w = p.tw[t * k * stride];
                        if (p.inverse) w.y = -w.y;
                        v[t] = cmul(v[t], w);
                    }
                }
            }
            dft_r(R, v, p.inverse);
            const int base = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (t < R) dst[(base + t * Ns) * ncol + col] = v[t];
        }
        __syncthreads();
        float2* tmp = src;
        src = dst;
        dst = tmp;
        Ns *= R;
    }

    // ---- store (pruned: only the Lout kept rows are written)
    if (p.post == POST_MAPS) {
        // columns of one outer are the C coils: reduce conj(s_c) v_c over c
        const int C = p.Ib;
        for (int idx = tid; idx < p.Ob * p.Lout; idx += nt) {
            const int ol = idx / p.Lout, m = idx % p.Lout;
            const int64_t o = o0 + ol;
            if (o >= p.O) continue;
            const int q = p.crop_out ? (m - p.Lout / 2 + L) % L : m;
            const int64_t e = o * p.Lout + m;
            const float2* mp = p.qmaps + e * C;
            const float2* row = src + q * ncol + ol * C;
            float2 acc = make_float2(0.f, 0.f);
            for (int c = 0; c < C; ++c) acc = cadd(acc, cmulc(row[c], mp[c]));
            acc = cscale(acc, p.fo[o] * p.fr[m]);
            if (p.epi == EPI_STORE) {
                p.qx[e] = acc;
            } else if (p.epi == EPI_L2) {
                const float tau = *p.e_tau, th = *p.e_theta;
                const float2 xo = p.ex[e];
                const float den = 1.f / (1.f + tau * (p.e_lam ? *p.e_lam : p.e_lambda));
                const float2 xn = make_float2((xo.x - tau * acc.x) * den, (xo.y - tau * acc.y) * den);
                p.exbar[e] = make_float2(xn.x + th * (xn.x - xo.x), xn.y + th * (xn.y - xo.y));
                p.ex[e] = xn;
            } else {  // EPI_Z: z = x - tau A^H u
                const float tau = *p.e_tau;
                const float2 xo = p.ex[e];
                p.exbar[e] = make_float2(xo.x - tau * acc.x, xo.y - tau * acc.y);
            }
        }
        return;
    }
    for (int idx = tid; idx < p.Lout * ncol; idx += nt) {
        const int m = idx / ncol, col = idx % ncol;
        const int64_t o = o0 + col / p.Ib, i = i0 + col % p.Ib;
        if (o >= p.O || i >= p.I) continue;
        const int q = p.crop_out ? (m - p.Lout / 2 + L) % L : m;
        float2 v = src[q * ncol + col];
        if (p.post == POST_NONE) {
            p.out[o * p.out_os + m * p.out_rs + i] = v;
        } else {  // POST_CHAN
            const int64_t e = o * p.Lout + m;
            p.qx[e * p.I + i] = cscale(v, p.fo[o] * p.fr[m]);
        }
    }
}

void fft_factor(int L, int* nst, int* rad) {
    int n = 0, r = L;
    while (r % 8 == 0 && r > 8 && n < kMaxStages) { rad[n++] = 8; r /= 8; }
    while (r % 4 == 0 && n < kMaxStages) { rad[n++] = 4; r /= 4; }
    while (r % 2 == 0 && n < kMaxStages) { rad[n++] = 2; r /= 2; }
    while (r % 5 == 0 && n < kMaxStages) { rad[n++] = 5; r /= 5; }
    while (r % 3 == 0 && n < kMaxStages) { rad[n++] = 3; r /= 3; }
    if (r == 8 && n < kMaxStages) { rad[n++] = 8; r = 1; }
    if (r != 1) fail(KP_ERR_UNSUPPORTED, "FFT length " + std::to_string(L) + " is not 5-smooth");
    *nst = n;
}

size_t fft_lds_bytes(int L, int ncol) { return (size_t)2 * L * ncol * sizeof(float2); }

static int lds_limit() {
    static int lim = -1;
    if (lim < 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            lim = (int)std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);
        else
            lim = 65536;
        (void)hipFuncSetAttribute((const void*)k_fft_pass, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipGetLastError();
    }
    return lim;
}

// ------------------------------------------------------------------------
// Specialised pass for the transform lengths of the benchmark workloads: the
// length, the radix sequence and the column block (NC = 8, 16 or 32 columns,
// a divisor of the 256 threads, so every thread keeps one column) are compile
// time constants, every index is a shift or a multiply, and the stages run
// in place in a single LDS buffer with the butterfly inputs held in
// registers across the barrier.
constexpr int fft_radix_c(int L, int s) {
    int r = L, n = 0;
    int rad[16] = {};
    while (r % 8 == 0 && r > 8) { rad[n++] = 8; r /= 8; }
    while (r % 4 == 0) { rad[n++] = 4; r /= 4; }
    while (r % 2 == 0) { rad[n++] = 2; r /= 2; }
    while (r % 5 == 0) { rad[n++] = 5; r /= 5; }
    while (r % 3 == 0) { rad[n++] = 3; r /= 3; }
    return s < n ? rad[s] : 1;
}
constexpr int fft_span_c(int L, int s) {  // product of the radices before stage s
    int p = 1;
    for (int i = 0; i < s; ++i) p *= fft_radix_c(L, i);
    return p;
}

template <int R>
__device__ __forceinline__ void dft_c(float2* v, int inv) {
    if (R == 2) dft2(v);
    else if (R == 3) dft3(v, inv);
    else if (R == 4) dft4(v, inv);
    else if (R == 5) dft5(v, inv);
    else dft8(v, inv);
}

template <int L, int NC, int S, int NT>
__device__ __forceinline__ void fixed_stage(float2* buf, const float2* __restrict__ tw, int inv, int tid) {
    constexpr int R = fft_radix_c(L, S);
    if (R == 1) return;
    constexpr int NS = fft_span_c(L, S);
    constexpr int NBF = L / R;
    constexpr int TOT = NBF * NC;
    constexpr int NB = (TOT + NT - 1) / NT;
    constexpr int STRIDE = L / (NS * R);
    const int col = tid % NC;
    float2 v[NB][R];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int j = tid / NC + k * (NT / NC);
        if (k * NT + tid < TOT) {
#pragma unroll
            for (int t = 0; t < R; ++t) v[k][t] = buf[(j + t * NBF) * (NC + 1) + col];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int j = tid / NC + k * (NT / NC);
        if (k * NT + tid < TOT) {
            const int kk = j % NS;
            if (NS > 1) {  // one table read; the other twiddles as its powers
                float2 w[R];
                w[1] = tw[kk * STRIDE];
                if (inv) w[1].y = -w[1].y;
#pragma unroll
                for (int t = 2; t < R; ++t) w[t] = cmul(w[t >> 1], w[t - (t >> 1)]);
#pragma unroll
                for (int t = 1; t < R; ++t) v[k][t] = cmul(v[k][t], w[t]);
            }
            dft_c<R>(v[k], inv);
            const int base = (j / NS) * NS * R + kk;
#pragma unroll
            for (int t = 0; t < R; ++t) buf[(base + t * NS) * (NC + 1) + col] = v[k][t];
        }
    }
    __syncthreads();
}

template <int L, int NC, int NT>
__device__ __forceinline__ void fft_fixed_body(const FftPass& p, int64_t bid, float2* buf) {
    constexpr int RS = NT / NC;   // rows per sweep of the block (NT threads)
    constexpr int LS = NC + 1;    // LDS row stride (padded against bank conflicts)
    const int tid = threadIdx.x;
    const int col = tid % NC, rb = tid / NC;
    const int64_t nIb = (p.I + p.Ib - 1) / p.Ib;
    const int64_t o0 = (bid / nIb) * p.Ob;
    const int64_t i0 = (bid % nIb) * p.Ib;
    const int64_t o = o0 + col / p.Ib, i = i0 + col % p.Ib;
    const bool live = o < p.O && i < p.I;
    const float xs = p.xscale ? *p.xscale : 1.f;
    // support pruning (passes along axis 0 in 3D): rows [xlo, xhi) of this
    // thread's column, from the range of its spreading tile column
    int xlo = 0, xhi = L;
    if (p.xr_mode && live) {
        const int64_t yy = i / p.xr_G2C;
        const int zz = (int)((i % p.xr_G2C) / p.xr_C);
        const int2 r = p.xr[(yy / p.xr_B1) * p.xr_nb2 + zz / p.xr_B2];
        xlo = r.x;
        xhi = r.y;
    }
    // y-range pruning: on an axis-0 pass this thread's column (y, z) may lie
    // outside the y-range of its z (col_out); on an axis-1 pass the rows
    // [ylo, yhi) of its z are the ones that matter
    int ylo = 0, yhi = L;
    bool col_out = false;
    if (p.yr_mode && live) {
        const int zz = (int)((i % p.xr_G2C) / p.xr_C);
        const int2 r = p.yr[zz / p.xr_B2];
        if (p.yr_mode <= 2) {
            const int64_t yy = i / p.xr_G2C;
            col_out = !(yy >= r.x && yy < r.y);
        } else {
            ylo = r.x;
            yhi = r.y;
        }
    }

    // ---- load (pruned): every row load of this thread is issued before the
    // first LDS write, so the block has all its loads in flight at once
    // (addresses are clamped into range and the values of rows past Lin or of
    // dead columns are replaced by zeros afterwards, so no load is predicated)
    constexpr int NR = (L + RS - 1) / RS;
    float2 v[NR];
    const int64_t oc = live ? o : 0, ic = live ? i : 0;
    if (p.pre == PRE_NONE && (p.xr_mode == 2 || p.yr_mode == 4)) {
        // rows outside the support range are zero (spreading leaves them
        // empty, or the previous pass did not store them) and are not loaded
        const int lo = p.xr_mode == 2 ? xlo : ylo, hi = p.xr_mode == 2 ? xhi : yhi;
        const float2* src = p.in + oc * p.in_os + ic;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int r = min(rb + k * RS, p.Lin - 1);
            v[k] = (r >= lo && r < hi) ? src[(int64_t)r * p.in_rs] : make_float2(0.f, 0.f);
        }
    } else if (p.pre == PRE_NONE) {
        const float2* src = p.in + oc * p.in_os + ic;
        if (col_out) {  // a column nothing reads (yr_mode 1): not loaded
#pragma unroll
            for (int k = 0; k < NR; ++k) v[k] = make_float2(0.f, 0.f);
        } else {
#pragma unroll
            for (int k = 0; k < NR; ++k) v[k] = src[(int64_t)min(rb + k * RS, p.Lin - 1) * p.in_rs];
        }
    } else if (p.pre == PRE_MAPS) {
        float2 mv[NR];
        float fr[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int64_t e = oc * p.Lin + min(rb + k * RS, p.Lin - 1);
            v[k] = p.px[e];
            mv[k] = p.pmaps[e * p.I + ic];
            fr[k] = p.fr[min(rb + k * RS, p.Lin - 1)];
        }
        const float fo = p.fo[oc] * xs;
#pragma unroll
        for (int k = 0; k < NR; ++k) v[k] = cscale(cmul(v[k], mv[k]), fo * fr[k]);
    } else {
        float fr[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int64_t e = oc * p.Lin + min(rb + k * RS, p.Lin - 1);
            v[k] = p.px[e * p.I + ic];
            fr[k] = p.fr[min(rb + k * RS, p.Lin - 1)];
        }
        const float fo = p.fo[oc] * xs;
#pragma unroll
        for (int k = 0; k < NR; ++k) v[k] = cscale(v[k], fo * fr[k]);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k)
        if (!live) v[k] = make_float2(0.f, 0.f);
    if (p.pad_in) {
        const int g0 = p.Lin / 2, g1 = L - p.Lin + p.Lin / 2;
        for (int q = g0 + rb; q < g1; q += RS) buf[q * LS + col] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int r = rb + k * RS;
        if (r < p.Lin) {
            int pos = r;
            if (p.pad_in) {
                pos = r - p.Lin / 2;
                pos += pos < 0 ? L : 0;
            }
            buf[pos * LS + col] = v[k];
        }
    }
    __syncthreads();

    fixed_stage<L, NC, 0, NT>(buf, p.tw, p.inverse, tid);
    fixed_stage<L, NC, 1, NT>(buf, p.tw, p.inverse, tid);
    fixed_stage<L, NC, 2, NT>(buf, p.tw, p.inverse, tid);
    fixed_stage<L, NC, 3, NT>(buf, p.tw, p.inverse, tid);
    fixed_stage<L, NC, 4, NT>(buf, p.tw, p.inverse, tid);
    fixed_stage<L, NC, 5, NT>(buf, p.tw, p.inverse, tid);

    // ---- store (pruned)
    if (p.post == POST_MAPS) {
        const int C = p.Ib;
        const int tpo = NT / p.Ob;  // threads per outer
        const int ol = tid / tpo;
        const int64_t oo = o0 + ol;
        if (ol >= p.Ob || oo >= p.O) return;
        for (int m = tid % tpo; m < p.Lout; m += tpo) {
            int q = m;
            if (p.crop_out) {
                q = m - p.Lout / 2;
                q += q < 0 ? L : 0;
            }
            const int64_t e = oo * p.Lout + m;
            const float2* mp = p.qmaps + e * C;
            const float2* row = buf + q * LS + ol * C;
            float2 acc = make_float2(0.f, 0.f);
            for (int c = 0; c < C; ++c) acc = cadd(acc, cmulc(row[c], mp[c]));
            acc = cscale(acc, p.fo[oo] * p.fr[m]);
            if (p.epi == EPI_STORE) {
                p.qx[e] = acc;
            } else if (p.epi == EPI_L2) {
                const float tau = *p.e_tau, th = *p.e_theta;
                const float2 xo = p.ex[e];
                const float den = 1.f / (1.f + tau * (p.e_lam ? *p.e_lam : p.e_lambda));
                const float2 xn = make_float2((xo.x - tau * acc.x) * den, (xo.y - tau * acc.y) * den);
                p.exbar[e] = make_float2(xn.x + th * (xn.x - xo.x), xn.y + th * (xn.y - xo.y));
                p.ex[e] = xn;
            } else {
                const float tau = *p.e_tau;
                const float2 xo = p.ex[e];
                p.exbar[e] = make_float2(xo.x - tau * acc.x, xo.y - tau * acc.y);
            }
        }
        return;
    }
    if (!live) return;
    if (p.yr_mode == 2 && col_out) return;  // an empty column: the next pass takes it as zero
    for (int m = rb; m < p.Lout; m += RS) {
        if (p.xr_mode == 1 && (m < xlo || m >= xhi)) continue;  // nothing reads these rows
        if (p.yr_mode == 3 && (m < ylo || m >= yhi)) continue;  // rows of empty columns
        int q = m;
        if (p.crop_out) {
            q = m - p.Lout / 2;
            q += q < 0 ? L : 0;
        }
        const float2 v = buf[q * LS + col];
        if (p.post == POST_NONE) {
            p.out[o * p.out_os + m * p.out_rs + i] = v;
        } else {
            const int64_t e = o * p.Lout + m;
            p.qx[e * p.I + i] = cscale(v, p.fo[o] * p.fr[m]);
        }
    }
}

template <int L, int NC, int NT>
__global__ void __launch_bounds__(NT) k_fft_fixed(FftPass p) {
    extern __shared__ float2 buf[];
    fft_fixed_body<L, NC, NT>(p, blockIdx.x, buf);
}

// ------------------------------------------------------------------------
// Register-resident two-factor pass for plain lines (no fused pre- or
// post-pass): L = N1 x N2 with n = N2 n1 + n2 and k = k1 + N1 k2,
//   X[k1 + N1 k2] = sum_n2 W_N2^(n2 k2) [ W_L^(n2 k1) sum_n1 x[N2 n1 + n2] W_N1^(n1 k1) ].
// Step 1: one thread per (n2, column) takes its N1 inputs straight from
// global memory, does the N1-point DFT and the twiddle W_L^(n2 k1) in
// registers and writes the N1 results to LDS.  Step 2: one thread per
// (k1, column) reads its N2 values back and does the N2-point DFT in
// registers (its twiddles are compile-time constants), then stores the N2
// outputs straight to global memory.  One LDS round trip and one barrier per
// pass instead of one per radix stage; the only table read is W_L^n2, whose
// powers W_L^(n2 k1) are formed by complex products.

// cos and sin of 2 pi m / n (m >= 0) at compile time: quadrant reduction,
// then Taylor series on [0, pi/2) (terms to x^27: far below double rounding)
constexpr double kc_taylor_sin(double x) {
    double t = x, s = x;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / (double)((2 * k) * (2 * k + 1));
        s += t;
    }
    return s;
}
constexpr double kc_taylor_cos(double x) {
    double t = 1.0, s = 1.0;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / (double)((2 * k - 1) * (2 * k));
        s += t;
    }
    return s;
}
constexpr double kc_phase(int m, int n, int* quad) {
    const int r = m % n, q = (4 * r) / n;
    *quad = q;
    return 3.14159265358979323846 * (double)(4 * r - q * n) / (2.0 * (double)n);
}
constexpr double kc_cos(int m, int n) {
    int q = 0;
    const double ph = kc_phase(m, n, &q);
    const double c = kc_taylor_cos(ph), s = kc_taylor_sin(ph);
    return q == 0 ? c : (q == 1 ? -s : (q == 2 ? -c : s));
}
constexpr double kc_sin(int m, int n) {
    int q = 0;
    const double ph = kc_phase(m, n, &q);
    const double c = kc_taylor_cos(ph), s = kc_taylor_sin(ph);
    return q == 0 ? s : (q == 1 ? c : (q == 2 ? -s : -c));
}

// compile-time loop: f(integral_constant<int, I>) for I = B .. E - 1
template <int B, int E>
struct Unroll {
    template <typename F>
    __device__ __forceinline__ static void run(F& f) {
        if constexpr (B < E) {
            f(std::integral_constant<int, B>());
            Unroll<B + 1, E>::run(f);
        }
    }
};

// in-place N-point DFT of v (sign by INV) in registers: N = R x M split as
// above, recursively, down to the radix kernels
template <int N, int INV>
__device__ __forceinline__ void dft_reg(float2* v) {
    if constexpr (N == 2 || N == 3 || N == 4 || N == 5 || N == 8) {
        dft_c<N>(v, INV);
    } else {
        constexpr int R = fft_radix_c(N, 0), M = N / R;
        float2 y[N];
        auto col = [&](auto n2c) {
            constexpr int n2 = decltype(n2c)::value;
            float2 t[R];
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) t[n1] = v[M * n1 + n2];
            dft_c<R>(t, INV);
            y[n2] = t[0];
            auto tw = [&](auto k1c) {
                constexpr int k1 = decltype(k1c)::value;
                constexpr float wr = (float)kc_cos(n2 * k1, N);
                constexpr float wi = (float)((INV ? 1.0 : -1.0) * kc_sin(n2 * k1, N));
                y[k1 * M + n2] = n2 == 0 ? t[k1] : cmul(t[k1], make_float2(wr, wi));
            };
            Unroll<1, R>::run(tw);
        };
        Unroll<0, M>::run(col);
#pragma unroll
        for (int k1 = 0; k1 < R; ++k1) dft_reg<M, INV>(y + k1 * M);
#pragma unroll
        for (int k1 = 0; k1 < R; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < M; ++k2) v[k1 + R * k2] = y[k1 * M + k2];
    }
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufWord3 = 0x00020000;     // buffer resource word 3 (raw dword access)
constexpr uint32_t kBufOff = 0x80000000u;  // an offset past every record count used here

template <int L, int N1, int NC, int INV>
__device__ __forceinline__ void fft_reg_body(const FftPass& p, int64_t bid, float2* buf) {
    constexpr int N2 = L / N1;
    constexpr int NT = N1 * NC;
    constexpr int LS = NC + 1;                    // LDS row stride (padded)
    constexpr int NJ = (N2 * NC + NT - 1) / NT;   // step-1 tasks per thread
    static_assert(N1 * N2 == L, "L = N1 N2");
    const int tid = threadIdx.x;
    const int col = tid % NC, tr = tid / NC;      // tr < N1
    const int64_t nIb = (p.I + p.Ib - 1) / p.Ib;
    const int64_t o0 = (bid / nIb) * p.Ob;
    const int64_t i0 = (bid % nIb) * p.Ib;
    const int64_t o = o0 + col / p.Ib, i = i0 + col % p.Ib;
    const bool live = o < p.O && i < p.I;
    // support pruning, per column, as in the LDS-staged pass
    int xlo = 0, xhi = L;
    if (p.xr_mode && live) {
        const int64_t yy = i / p.xr_G2C;
        const int zz = (int)((i % p.xr_G2C) / p.xr_C);
        const int2 r = p.xr[(yy / p.xr_B1) * p.xr_nb2 + zz / p.xr_B2];
        xlo = r.x;
        xhi = r.y;
    }
    int ylo = 0, yhi = L;
    bool col_out = false;
    if (p.yr_mode && live) {
        const int zz = (int)((i % p.xr_G2C) / p.xr_C);
        const int2 r = p.yr[zz / p.xr_B2];
        if (p.yr_mode <= 2) {
            const int64_t yy = i / p.xr_G2C;
            col_out = !(yy >= r.x && yy < r.y);
        } else {
            ylo = r.x;
            yhi = r.y;
        }
    }

    // ---- step 1: loads of every task of this thread first, then the DFTs.
    // Loads and stores are buffer accesses relative to the block's first
    // element: a lane whose value is zero (padding, a pruned row, a dead
    // column, a missing task) or whose row is not stored gets the offset
    // kBufOff, past the record count, which the hardware answers with zero
    // (load) or drops (store) without a memory access, so no access needs a
    // branch.  The host keeps every valid byte offset of the pass below 2^31.
    const __amdgpu_buffer_rsrc_t rin =
        __builtin_amdgcn_make_buffer_rsrc((void*)(p.in + o0 * p.in_os + i0), (short)0, 0x7fffffff, kBufWord3);
    const uint32_t colb = (uint32_t)(((o - o0) * p.in_os + (i - i0)) * 8);
    const uint32_t rsb = (uint32_t)(p.in_rs * 8);
    int lo = 0, hi = p.Lin;  // input rows taken from memory; the others are zero
    if (p.xr_mode == 2) {
        lo = xlo;
        hi = min(xhi, p.Lin);
    } else if (p.yr_mode == 4) {
        lo = ylo;
        hi = min(yhi, p.Lin);
    }
    if (!live || (p.yr_mode == 1 && col_out)) hi = lo;
    const int half = p.Lin / 2;
    const int zlo = p.pad_in ? p.Lin - half : p.Lin, zhi = p.pad_in ? L - half : L;  // zero positions
    float2 v[NJ][N1];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int n2 = tr + j * N1;
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
            const int pos = N2 * n1 + n2;
            const int r = pos >= zhi ? pos - zhi : pos + (p.pad_in ? half : 0);  // input row at this position
            const bool ok = (n2 < N2) & ((pos < zlo) | (pos >= zhi)) & (r >= lo) & (r < hi);
            const uint32_t off = ok ? colb + (uint32_t)r * rsb : kBufOff;
            const u32x2 t = __builtin_amdgcn_raw_buffer_load_b64(rin, off, 0, 0);
            v[j][n1] = make_float2(__uint_as_float(t.x), __uint_as_float(t.y));
        }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int n2 = tr + j * N1;
        if (n2 < N2) {
            dft_reg<N1, INV>(v[j]);
            float2 w[N1];
            w[0] = make_float2(1.f, 0.f);
            w[1] = p.tw[n2];
            if (INV) w[1].y = -w[1].y;
#pragma unroll
            for (int k1 = 2; k1 < N1; ++k1) w[k1] = cmul(w[k1 >> 1], w[k1 - (k1 >> 1)]);
            buf[n2 * LS + col] = v[j][0];
#pragma unroll
            for (int k1 = 1; k1 < N1; ++k1) buf[(k1 * N2 + n2) * LS + col] = cmul(v[j][k1], w[k1]);
        }
    }
    __syncthreads();

    // ---- step 2: thread (k1 = tr, col)
    float2 y[N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) y[n2] = buf[(tr * N2 + n2) * LS + col];
    dft_reg<N2, INV>(y);
    const __amdgpu_buffer_rsrc_t rout =
        __builtin_amdgcn_make_buffer_rsrc((void*)(p.out + o0 * p.out_os + i0), (short)0, 0x7fffffff, kBufWord3);
    const uint32_t colo = (uint32_t)(((o - o0) * p.out_os + (i - i0)) * 8);
    const uint32_t rso = (uint32_t)(p.out_rs * 8);
    // rows stored: [slo, shi) of the pruning range, none for a dead or empty column
    int slo = 0, shi = p.Lout;
    if (p.xr_mode == 1) {
        slo = xlo;
        shi = min(xhi, p.Lout);
    } else if (p.yr_mode == 3) {
        slo = ylo;
        shi = min(yhi, p.Lout);
    }
    if (!live || (p.yr_mode == 2 && col_out)) shi = slo;
    const int cshift = p.crop_out ? p.Lout / 2 : 0;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
        const int q = tr + N1 * k2;
        int m = q + cshift;  // output row of transform index q (centred crop)
        m -= m >= L ? L : 0;
        const uint32_t off = ((m >= slo) & (m < shi)) ? colo + (uint32_t)m * rso : kBufOff;
        u32x2 t;
        t.x = __float_as_uint(y[k2].x);
        t.y = __float_as_uint(y[k2].y);
        __builtin_amdgcn_raw_buffer_store_b64(t, rout, off, 0, 0);
    }
}

template <int L, int N1, int NC>
__global__ void __launch_bounds__(N1 * NC) k_fft_reg(FftPass p) {
    extern __shared__ float2 buf[];
    if (p.inverse)
        fft_reg_body<L, N1, NC, 1>(p, blockIdx.x, buf);
    else
        fft_reg_body<L, N1, NC, 0>(p, blockIdx.x, buf);
}

// Column blocks of the specialised kernels: NC columns over NT threads with
// NT a multiple of NC (8, 16 or 32 columns on 256 threads; 12 columns, one
// 12-coil row, on 768 threads: on the 2D 12-coil lines 384 threads were
// 8-10 % faster than 192, and 768 a further 1-2 % (plain) to 4-6 % (batched)
// faster than 384; 960 were slower).  32 columns = 256 contiguous bytes per
// row.
static int fixed_threads(int nc) { return nc == 12 ? 768 : ((nc == 8 || nc == 16 || nc == 32) ? 256 : 0); }

// One launch over the passes of many independent transforms of mixed lengths
// (one phase of the slices of a batch): pass s owns the blocks
// blk_start[s] .. blk_start[s+1]-1 (passes sorted by length).  Each length
// has its own column block: the coil block of the passes along the coils
// (MAP > 0), else kMixCols(L): 32 columns (256 contiguous bytes of every
// row) up to length 256 and 16 above, so that every length needs at most
// 68 KB of LDS (two resident blocks per CU); LDS is sized for the largest of
// them.  With many slices in flight the wider rows pay more than a third
// resident block would (the 2D axis-0 passes read rows tens of KB apart).
__host__ __device__ constexpr int kMixCols(int L) { return L <= 256 ? 32 : 16; }

template <int NT, int MAP, int L>
__device__ __forceinline__ void mixed_body(const FftPass& p, int64_t bid, float2* buf) {
    constexpr int NC = MAP > 0 ? MAP : kMixCols(L);
    fft_fixed_body<L, NC, NT>(p, bid, buf);
}

template <int NT, int MAP>
__global__ void __launch_bounds__(NT) k_fft_batch_mixed(const FftPass* __restrict__ passes,
                                                         const int64_t* __restrict__ blk_start, int n) {
    extern __shared__ float2 buf[];
    {
        const int64_t b = blockIdx.x;
        int lo = 0, hi = n - 1;
        while (lo < hi) {  // last s with blk_start[s] <= b
            const int mid = (lo + hi + 1) / 2;
            if (blk_start[mid] <= b) lo = mid; else hi = mid - 1;
        }
        const FftPass p = passes[lo];
        const int64_t bid = b - blk_start[lo];
        switch (p.L) {
            case 160: mixed_body<NT, MAP, 160>(p, bid, buf); break;
            case 200: mixed_body<NT, MAP, 200>(p, bid, buf); break;
            case 240: mixed_body<NT, MAP, 240>(p, bid, buf); break;
            case 256: mixed_body<NT, MAP, 256>(p, bid, buf); break;
            case 320: mixed_body<NT, MAP, 320>(p, bid, buf); break;
            case 400: mixed_body<NT, MAP, 400>(p, bid, buf); break;
            default: break;
        }
    }
}

// the kernel of a phase (map = the coil column block of the passes along the
// coils, 0 for the others) and its thread count
static const void* mixed_kernel(int map, int* nt) {
    switch (map) {
        case 0: *nt = 512; return (const void*)k_fft_batch_mixed<512, 0>;
        case 8: *nt = 256; return (const void*)k_fft_batch_mixed<256, 8>;
        case 12: *nt = 768; return (const void*)k_fft_batch_mixed<768, 12>;
        case 16: *nt = 512; return (const void*)k_fft_batch_mixed<512, 16>;
        default: return nullptr;
    }
}

int fft_mixed_columns(int L, int nc_map) { return nc_map > 0 ? nc_map : kMixCols(L); }

void launch_fft_batch_mixed(const FftPass* d_passes, const int64_t* d_blk_start, int n, int64_t nblk, int map,
                            size_t lds, hipStream_t s) {
    if (nblk <= 0) return;
    int nt = 0;
    const void* fn = mixed_kernel(map, &nt);
    if (!fn) fail(KP_ERR_UNSUPPORTED, "no mixed-length FFT kernel for this column block");
    if (nblk > 0x7fffffff) fail(KP_ERR_UNSUPPORTED, "batched FFT grid too large");
    if (lds > 65536) {
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    }
    const dim3 g((unsigned)nblk);
    if (map == 0)
        hipLaunchKernelGGL((k_fft_batch_mixed<512, 0>), g, dim3(512), lds, s, d_passes, d_blk_start, n);
    else if (map == 8)
        hipLaunchKernelGGL((k_fft_batch_mixed<256, 8>), g, dim3(256), lds, s, d_passes, d_blk_start, n);
    else if (map == 12)
        hipLaunchKernelGGL((k_fft_batch_mixed<768, 12>), g, dim3(768), lds, s, d_passes, d_blk_start, n);
    else
        hipLaunchKernelGGL((k_fft_batch_mixed<512, 16>), g, dim3(512), lds, s, d_passes, d_blk_start, n);
    KP_LAUNCH_CHECK();
}

static bool batch_length(int L) { return L == 160 || L == 200 || L == 240 || L == 256 || L == 320 || L == 400; }

bool fft_batchable(const FftPass& p) {
    const int nc = p.Ob * p.Ib;
    const int nt = fixed_threads(nc);
    if (nc != 32 && nc != 16 && nc != 12 && nc != 8) return false;
    if (p.post == POST_MAPS && (nt % p.Ob) != 0) return false;
    return batch_length(p.L);
}

int64_t fft_pass_blocks(const FftPass& p) {
    return ((p.I + p.Ib - 1) / p.Ib) * ((p.O + p.Ob - 1) / p.Ob);
}

typedef void (*fft_kernel_t)(FftPass);

template <int NC, int NT>
static fft_kernel_t fixed_for(int L) {
    switch (L) {
        case 160: return k_fft_fixed<160, NC, NT>;
        case 200: return k_fft_fixed<200, NC, NT>;
        case 240: return k_fft_fixed<240, NC, NT>;
        case 256: return k_fft_fixed<256, NC, NT>;
        case 320: return k_fft_fixed<320, NC, NT>;
        case 400: return k_fft_fixed<400, NC, NT>;
        case 512: return k_fft_fixed<512, NC, NT>;
        case 640: return k_fft_fixed<640, NC, NT>;
        default: return nullptr;
    }
}

// register-resident passes: plain 32-column passes of lengths 8 x N2 with an
// N2-point DFT small enough for registers
// register-resident passes: plain 32-column passes of lengths N1 x N2 with
// an N2-point DFT small enough for registers, on N1 x 32 threads.  200 = 10 x
// 20 balances both steps (2 step-1 tasks per thread, one step-2 task; 8 x 25
// left a 4th step-1 task to an eighth of the threads: FFT stages 0.445 ->
// 0.433 ms forward); the other lengths use N1 = 8.  The fused map passes stay
// on the LDS-staged kernel: 25 values per lane cap a register pass at about
// 11 waves per CU, and those passes ran slower in that form.
static fft_kernel_t reg_for(const FftPass& p, int* n1) {
    if (p.pre != PRE_NONE || p.post != POST_NONE || p.Ob * p.Ib != 32) return nullptr;
    *n1 = 8;
    switch (p.L) {
        case 160: return k_fft_reg<160, 8, 32>;
        case 200: *n1 = 10; return k_fft_reg<200, 10, 32>;
        case 240: return k_fft_reg<240, 8, 32>;
        case 256: return k_fft_reg<256, 8, 32>;
        default: return nullptr;
    }
}

// the register-resident pass addresses a block's input and output through
// 32-bit byte offsets below 2^31
static bool reg_span_ok(const FftPass& p) {
    const int64_t lim = 0x7ffffff0;
    const int64_t in_span = ((int64_t)(p.Ob - 1) * p.in_os + (p.Ib - 1) + (int64_t)(p.Lin - 1) * p.in_rs + 1) * 8;
    const int64_t out_span = ((int64_t)(p.Ob - 1) * p.out_os + (p.Ib - 1) + (int64_t)(p.Lout - 1) * p.out_rs + 1) * 8;
    return p.in_os >= 0 && p.in_rs >= 0 && p.out_os >= 0 && p.out_rs >= 0 && in_span < lim && out_span < lim;
}

// try the specialised kernels; false if this pass fits neither
static bool launch_fixed(const FftPass& p, hipStream_t s, int lim) {
    const int nc = p.Ob * p.Ib;
    int n1 = 8;
    fft_kernel_t fr = reg_for(p, &n1);
    if (fr && reg_span_ok(p)) {
        const size_t lds = sizeof(float2) * (size_t)p.L * 33;
        if (lds <= (size_t)lim) {
            if (lds > 65536) {
                (void)hipFuncSetAttribute((const void*)fr, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
                (void)hipGetLastError();
            }
            const int64_t nblk = fft_pass_blocks(p);
            if (nblk <= 0) return true;
            if (nblk > 0x7fffffff) fail(KP_ERR_UNSUPPORTED, "FFT pass grid too large");
            hipLaunchKernelGGL(fr, dim3((unsigned)nblk), dim3(n1 * 32), lds, s, p);
            KP_LAUNCH_CHECK();
            return true;
        }
    }
    const int nt = fixed_threads(nc);
    if (nt == 0) return false;
    if (p.post == POST_MAPS && (nt % p.Ob) != 0) return false;
    fft_kernel_t fn = nc == 32   ? fixed_for<32, 256>(p.L)
                      : nc == 16 ? fixed_for<16, 256>(p.L)
                      : nc == 8  ? fixed_for<8, 256>(p.L)
                                 : fixed_for<12, 768>(p.L);
    if (!fn) return false;
    const size_t lds = sizeof(float2) * (size_t)p.L * (nc + 1);
    if (lds > (size_t)lim) return false;
    if (lds > 65536) {
        (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipGetLastError();
    }
    const int64_t nblk = fft_pass_blocks(p);
    if (nblk <= 0) return true;
    if (nblk > 0x7fffffff) fail(KP_ERR_UNSUPPORTED, "FFT pass grid too large");
    hipLaunchKernelGGL(fn, dim3((unsigned)nblk), dim3(nt), lds, s, p);
    KP_LAUNCH_CHECK();
    return true;
}

bool fft_fixed_ok(int L, int nc) {
    const int nt = fixed_threads(nc);
    if (nt == 0) return false;
    fft_kernel_t fn = nc == 32 ? fixed_for<32, 256>(L) : nc == 16 ? fixed_for<16, 256>(L)
                    : nc == 8 ? fixed_for<8, 256>(L) : fixed_for<12, 768>(L);
    return fn && sizeof(float2) * (size_t)L * (nc + 1) <= (size_t)lds_limit();
}

void launch_fft_pass(const FftPass& pin, hipStream_t s) {
    FftPass p = pin;
    const int lim = lds_limit();
    // a small transform (a 2D slice) has too few 32-column blocks to fill the
    // GPU: narrower blocks (16, 8 columns) until the pass has 1024 of them
    if (p.Ob == 1 && p.Ib == 32 && p.xr_mode == 0 && p.yr_mode == 0 && p.pre != PRE_MAPS && p.post != POST_MAPS)
        while (p.Ib > 8 && fft_pass_blocks(p) < 1024) p.Ib /= 2;
    if (launch_fixed(p, s, lim)) return;
    // support-pruned loads exist only in the specialised kernel
    if (p.xr_mode == 2 || p.yr_mode == 4) fail(KP_ERR_UNSUPPORTED, "support-pruned FFT pass needs the specialised kernel");
    // shrink the column block until both LDS buffers fit
    while (fft_lds_bytes(p.L, p.Ob * p.Ib) > (size_t)lim) {
        if (p.Ob > 1)
            p.Ob = (p.Ob + 1) / 2;
        else if (p.post != POST_MAPS && p.Ib > 1)
            p.Ib = (p.Ib + 1) / 2;
        else
            fail(KP_ERR_UNSUPPORTED, "FFT line of length " + std::to_string(p.L) + " does not fit in LDS");
    }
    const size_t lds = fft_lds_bytes(p.L, p.Ob * p.Ib);
    const int64_t nIb = (p.I + p.Ib - 1) / p.Ib;
    const int64_t nOb = (p.O + p.Ob - 1) / p.Ob;
    const int64_t nblk = nIb * nOb;
    if (nblk <= 0) return;
    if (nblk > 0x7fffffff) fail(KP_ERR_UNSUPPORTED, "FFT pass grid too large");
    hipLaunchKernelGGL(k_fft_pass, dim3((unsigned)nblk), dim3(256), lds, s, p);
    KP_LAUNCH_CHECK();
}

}  // namespace kp
