// Kaiser-Bessel interpolation (forward, gather) and spreading (adjoint).
//
// Grid layout [G_0][G_1]([G_2])[C]: the C coils of one grid cell are
// contiguous, so every tap of every sample reads or writes one contiguous
// C-vector, and the per-axis kernel weights of a sample are computed once
// and shared by all coils.
//
// Weights: C(u) = I0(beta sqrt(1 - (2u/W)^2)) / W for |u| < W/2, with I0
// from its power series sum_k (x^2/4)^k / (k!)^2 summed term by term
// (a_k = a_{k-1} t / k^2, all terms positive).  Taps of a sample at grid
// coordinate g: j = floor(g) - W/2 + 1 + t, u = g - j, t = 0..W-1, taken
// modulo G.
//
// Spreading never uses global atomics for an ordinary tile: every tile of
// the grid is owned by one work item, which gathers every sample whose
// footprint meets the tile (its touch list), accumulates the weighted values
// in an LDS copy of the tile, then stores the tile.  Tiles with more touch
// entries than a work item takes (the dense k-space centre) are split over
// several work items that add their LDS tiles into a pre-zeroed grid region.
#include "kp_internal.h"

namespace kp {

__constant__ float c_inv_k2[96];

void upload_kb_constants() {
    static bool done = false;
    if (done) return;
    float h[96];
    h[0] = 1.f;
    for (int k = 1; k < 96; ++k) h[k] = (float)(1.0 / ((double)k * (double)k));
    KP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_inv_k2), h, sizeof(h)));
    done = true;
}

int nterms_for(double beta2_4) {
    // smallest K with the series tail below 1e-9 of the sum at the largest
    // argument t = beta^2/4
    double t = beta2_4, a = 1.0, s = 1.0;
    int k = 1;
    for (; k < 95; ++k) {
        a *= t / ((double)k * k);
        s += a;
        if (a < 1e-10 * s && (double)k * k > t) break;
    }
    return k + 1 < 95 ? k + 1 : 95;
}

template <int W>
__device__ __forceinline__ float kb_weight(float u, const KbParams& kb) {
    if (u <= -(float)(W / 2)) return 0.f;  // strict support |u| < W/2
    const float r = u * kb.inv_half;
    const float arg = fmaxf(1.f - r * r, 0.f);
    const float t = kb.beta2_4 * arg;
    float term = 1.f, sum = 1.f;
    for (int k = 1; k < kb.nterms; ++k) {
        term *= t * c_inv_k2[k];
        sum += term;
    }
    return sum * kb.inv_w;
}

template <int W>
__device__ __forceinline__ void axis_taps(float g, int Ga, const KbParams& kb, float* w, int* j) {
    const float cf = floorf(g);
    const int cell = (int)cf;
    const float frac = g - cf;
#pragma unroll
    for (int t = 0; t < W; ++t) {
        w[t] = kb_weight<W>(frac + (float)(W / 2 - 1 - t), kb);
        int jj = cell - W / 2 + 1 + t;
        jj = jj < 0 ? jj + Ga : (jj >= Ga ? jj - Ga : jj);
        j[t] = jj;
    }
}

// ------------------------------------------------------------ interpolation
template <int D, int W, int CH>
__global__ void __launch_bounds__(256) k_interp(InterpArgs a, KbParams kb) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.M) return;
    float w[D][W];
    int jx[D][W];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) axis_taps<W>(a.g[s * D + ax], a.G[ax], kb, w[ax], jx[ax]);
    const int C = a.C;
    for (int c0 = 0; c0 < C; c0 += CH) {
        float2 acc[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] = make_float2(0.f, 0.f);
        if (D == 2) {
#pragma unroll
            for (int t0 = 0; t0 < W; ++t0) {
                const int64_t r0 = (int64_t)jx[0][t0] * a.G[1];
#pragma unroll
                for (int t1 = 0; t1 < W; ++t1) {
                    const float wt = w[0][t0] * w[1][t1];
                    const float2* src = a.grid + (r0 + jx[1][t1]) * C + c0;
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        if (c0 + c < C) {
                            float2 v = src[c];
                            acc[c].x += wt * v.x;
                            acc[c].y += wt * v.y;
                        }
                    }
                }
            }
        } else {
#pragma unroll
            for (int t0 = 0; t0 < W; ++t0) {
                const int64_t r0 = (int64_t)jx[0][t0] * a.G[1];
#pragma unroll
                for (int t1 = 0; t1 < W; ++t1) {
                    const int64_t r1 = (r0 + jx[1][t1]) * a.G[2];
                    const float w01 = w[0][t0] * w[1][t1];
#pragma unroll
                    for (int t2 = 0; t2 < W; ++t2) {
                        const float wt = w01 * w[2][t2];
                        const float2* src = a.grid + (r1 + jx[2][t2]) * C + c0;
#pragma unroll
                        for (int c = 0; c < CH; ++c) {
                            if (c0 + c < C) {
                                float2 v = src[c];
                                acc[c].x += wt * v.x;
                                acc[c].y += wt * v.y;
                            }
                        }
                    }
                }
            }
        }
        // epilogue
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int cc = c0 + c;
            if (cc >= C) break;
            const int64_t e = s * C + cc;
            if (a.mode == IO_CALLER) {
                a.out[(int64_t)cc * a.M + a.perm[s]] = acc[c];
            } else if (a.mode == IO_INTERNAL) {
                a.out[e] = acc[c];
            } else if (a.mode == IO_PMUL) {
                const float pv = a.p ? (a.p_mc ? a.p[e] : a.p[s]) : 1.f;
                a.out[e] = make_float2(pv * acc[c].x, pv * acc[c].y);
            } else {  // IO_DUAL
                const float pv = a.p ? (a.p_mc ? a.p[e] : a.p[s]) : 1.f;
                const float sp = *a.sigma * pv;
                const float den = 1.f / (1.f + sp);
                const float2 u = a.u[e], y = a.y[e];
                a.u[e] = make_float2((u.x + sp * (acc[c].x - y.x)) * den, (u.y + sp * (acc[c].y - y.y)) * den);
            }
        }
    }
}

template <int D, int W>
static void interp_dispatch_ch(const InterpArgs& a, const KbParams& kb, hipStream_t s) {
    const unsigned nblk = (unsigned)((a.M + 255) / 256);
    if (a.C % 4 == 0)
        hipLaunchKernelGGL((k_interp<D, W, 4>), dim3(nblk), dim3(256), 0, s, a, kb);
    else if (a.C % 2 == 0)
        hipLaunchKernelGGL((k_interp<D, W, 2>), dim3(nblk), dim3(256), 0, s, a, kb);
    else
        hipLaunchKernelGGL((k_interp<D, W, 1>), dim3(nblk), dim3(256), 0, s, a, kb);
    KP_LAUNCH_CHECK();
}

void launch_interp(int d, int W, const InterpArgs& a, const KbParams& kb, hipStream_t s) {
    if (a.M <= 0) return;
#define KP_INTERP_W(DD, WW) \
    if (d == DD && W == WW) return interp_dispatch_ch<DD, WW>(a, kb, s);
    KP_INTERP_W(2, 2) KP_INTERP_W(2, 4) KP_INTERP_W(2, 6) KP_INTERP_W(2, 8)
    KP_INTERP_W(3, 2) KP_INTERP_W(3, 4) KP_INTERP_W(3, 6) KP_INTERP_W(3, 8)
#undef KP_INTERP_W
    fail(KP_ERR_UNSUPPORTED, "interp: unsupported (d, W)");
}

// ------------------------------------------------------------ spreading
template <int D, int W>
__global__ void __launch_bounds__(256) k_spread(SpreadArgs a, KbParams kb) {
    extern __shared__ float sm[];
    const int4 wk = a.work[blockIdx.x];
    const int tile = wk.x, start = wk.y, count = wk.z, atomic = wk.w;
    const int C = a.C;
    int tc[3] = {0, 0, 0};
    {
        int rem = tile;
        for (int ax = D - 1; ax >= 0; --ax) {
            tc[ax] = rem % a.nb[ax];
            rem /= a.nb[ax];
        }
    }
    const int Bt = a.B[0] * a.B[1] * (D == 3 ? a.B[2] : 1);
    float* re = sm;
    float* im = sm + Bt * C;
    for (int i = threadIdx.x; i < 2 * Bt * C; i += blockDim.x) sm[i] = 0.f;
    __syncthreads();

    for (int e = threadIdx.x; e < count; e += blockDim.x) {
        const int s = a.touch[start + e];
        float w[D][W];
        int loc[D][W];
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            int jj[W];
            axis_taps<W>(a.g[(int64_t)s * D + ax], a.G[ax], kb, w[ax], jj);
            const int org = tc[ax] * a.B[ax];
#pragma unroll
            for (int t = 0; t < W; ++t) {
                const int l = jj[t] - org;
                loc[ax][t] = (l >= 0 && l < a.B[ax]) ? l : -1;
            }
        }
        const float2* kv = a.k + (int64_t)s * C;
        if (D == 2) {
#pragma unroll
            for (int t0 = 0; t0 < W; ++t0) {
                if (loc[0][t0] < 0) continue;
#pragma unroll
                for (int t1 = 0; t1 < W; ++t1) {
                    if (loc[1][t1] < 0) continue;
                    const float wt = w[0][t0] * w[1][t1];
                    const int l = (loc[0][t0] * a.B[1] + loc[1][t1]) * C;
                    for (int c = 0; c < C; ++c) {
                        const float2 v = kv[c];
                        atomicAdd(&re[l + c], wt * v.x);
                        atomicAdd(&im[l + c], wt * v.y);
                    }
                }
            }
        } else {
#pragma unroll
            for (int t0 = 0; t0 < W; ++t0) {
                if (loc[0][t0] < 0) continue;
#pragma unroll
                for (int t1 = 0; t1 < W; ++t1) {
                    if (loc[1][t1] < 0) continue;
                    const float w01 = w[0][t0] * w[1][t1];
                    const int l01 = (loc[0][t0] * a.B[1] + loc[1][t1]) * a.B[2];
#pragma unroll
                    for (int t2 = 0; t2 < W; ++t2) {
                        if (loc[2][t2] < 0) continue;
                        const float wt = w01 * w[2][t2];
                        const int l = (l01 + loc[2][t2]) * C;
                        for (int c = 0; c < C; ++c) {
                            const float2 v = kv[c];
                            atomicAdd(&re[l + c], wt * v.x);
                            atomicAdd(&im[l + c], wt * v.y);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();

    // write the tile back: plain stores for an owned tile, atomics for a split one
    for (int i = threadIdx.x; i < Bt * C; i += blockDim.x) {
        const int l = i / C, c = i % C;
        int64_t gidx;
        if (D == 2) {
            const int l0 = l / a.B[1], l1 = l % a.B[1];
            gidx = (int64_t)(tc[0] * a.B[0] + l0) * a.G[1] + (tc[1] * a.B[1] + l1);
        } else {
            const int l2 = l % a.B[2];
            const int l01 = l / a.B[2];
            const int l1 = l01 % a.B[1], l0 = l01 / a.B[1];
            gidx = ((int64_t)(tc[0] * a.B[0] + l0) * a.G[1] + (tc[1] * a.B[1] + l1)) * a.G[2] +
                   (tc[2] * a.B[2] + l2);
        }
        float2* dst = a.grid + gidx * C + c;
        if (atomic) {
            unsafeAtomicAdd(&dst->x, re[i]);
            unsafeAtomicAdd(&dst->y, im[i]);
        } else {
            *dst = make_float2(re[i], im[i]);
        }
    }
}

void launch_spread(int d, int W, const SpreadArgs& a, const KbParams& kb, int lds_bytes,
                   hipStream_t s) {
    if (a.nwork <= 0) return;
    const dim3 grid((unsigned)a.nwork), block(256);
#define KP_SPREAD_W(DD, WW)                                                              \
    if (d == DD && W == WW) {                                                            \
        hipLaunchKernelGGL((k_spread<DD, WW>), grid, block, lds_bytes, s, a, kb);        \
        KP_LAUNCH_CHECK();                                                               \
        return;                                                                          \
    }
    KP_SPREAD_W(2, 2) KP_SPREAD_W(2, 4) KP_SPREAD_W(2, 6) KP_SPREAD_W(2, 8)
    KP_SPREAD_W(3, 2) KP_SPREAD_W(3, 4) KP_SPREAD_W(3, 6) KP_SPREAD_W(3, 8)
#undef KP_SPREAD_W
    fail(KP_ERR_UNSUPPORTED, "spread: unsupported (d, W)");
}

}  // namespace kp
