// Kaiser-Bessel interpolation (forward, gather) and spreading (adjoint).
//
// Grid layout [G_0][G_1]([G_2])[C]: the C coils of one grid cell are
// contiguous, so every tap of a sample reads or writes one contiguous
// C-vector and the per-axis kernel weights of a sample are shared by all
// coils.
//
// Weights: C(u) = I0(beta sqrt(1 - (2u/W)^2)) / W for |u| < W/2.  The taps of
// a sample at grid coordinate g are j = floor(g) - W/2 + 1 + t, u = g - j,
// t = 0..W-1 (modulo G).  As a function of x = frac(g) - 1/2 the weight of
// tap t is smooth on [0, 1), so each tap's weight is a degree-9 polynomial in
// x fitted on the host (Chebyshev nodes, double precision; about 1e-7 of the
// peak in float32).  The last tap at frac(g) = 0 sits exactly on the support
// edge |u| = W/2 and weighs 0.
//
// Spreading is gather-by-owner: every tile of the grid is owned by one work
// item, which takes every sample whose footprint meets the tile (its touch
// list) in chunks staged in LDS, buckets the chunk by the sample's first
// tap along the leading axes, and lets each thread own one line of the tile
// along the last axis (and a group of coils) in registers.  A thread visits
// exactly the samples that cover its line, so there are no atomics at all
// for an owned tile; a tile whose touch list was split over several work
// items (the dense k-space centre) writes each piece's registers to a slot of
// partial tiles, and the slots of a tile are added in slot order afterwards,
// so results are bit-reproducible.
#include <algorithm>
#include <cmath>

#include "kp_internal.h"

namespace kp {

// ------------------------------------------------------------ KB weights
double kb_kernel_host(double u, int W, double beta) {
    const double half = W / 2.0;
    if (!(std::fabs(u) < half)) return 0.0;
    const double r = u / half;
    const double t = beta * beta * (1.0 - r * r) / 4.0;  // (x/2)^2
    // I0(x) = sum_k t^k / (k!)^2, terms positive
    double a = 1.0, s = 1.0;
    for (int k = 1; k < 200; ++k) {
        a *= t / ((double)k * k);
        s += a;
        if (a < 1e-18 * s) break;
    }
    return s / W;
}

void kb_fit(double beta, int W, KbParams* kb) {
    const int n = kPolyN;
    double nodes[kPolyN];
    for (int i = 0; i < n; ++i) nodes[i] = 0.5 * std::cos((2.0 * i + 1.0) * M_PI / (2.0 * n));
    for (int t = 0; t < 8; ++t)
        for (int k = 0; k < n; ++k) kb->poly[t][k] = 0.f;
    for (int t = 0; t < W; ++t) {
        // interpolate f_t(x) = C(x + 1/2 + W/2 - 1 - t) at the nodes (Vandermonde, partial pivoting)
        double A[kPolyN][kPolyN + 1];
        for (int i = 0; i < n; ++i) {
            double p = 1.0;
            for (int k = 0; k < n; ++k) {
                A[i][k] = p;
                p *= nodes[i];
            }
            double u = nodes[i] + 0.5 + W / 2.0 - 1.0 - t;
            // the last tap's weight tends to C(-W/2 + 0) = 1/W as frac -> 0+
            if (t == W - 1) u = std::max(u, -W / 2.0 + 1e-300);
            A[i][n] = kb_kernel_host(u, W, beta);
            if (t == W - 1 && !(std::fabs(u) < W / 2.0)) A[i][n] = 1.0 / W;
        }
        for (int c = 0; c < n; ++c) {
            int piv = c;
            for (int r = c + 1; r < n; ++r)
                if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
            for (int k = 0; k <= n; ++k) std::swap(A[c][k], A[piv][k]);
            for (int r = 0; r < n; ++r) {
                if (r == c) continue;
                const double f = A[r][c] / A[c][c];
                for (int k = c; k <= n; ++k) A[r][k] -= f * A[c][k];
            }
        }
        for (int k = 0; k < n; ++k) kb->poly[t][k] = (float)(A[k][n] / A[k][k]);
        if (2 * t < W) {
            for (int k = 0; k < kHalfN; ++k) {
                kb->ev[t][k] = (float)(A[2 * k][n] / A[2 * k][2 * k]);
                kb->od[t][k] = (float)(A[2 * k + 1][n] / A[2 * k + 1][2 * k + 1]);
            }
        }
    }
}

template <int W>
__device__ __forceinline__ void tap_weights(float frac, const KbParams& kb, float* w) {
    const float x = frac - 0.5f;
    const float x2 = x * x;
#pragma unroll
    for (int t = 0; t < W / 2; ++t) {  // mirrored pairs (t, W-1-t)
        float e = kb.ev[t][kHalfN - 1], o = kb.od[t][kHalfN - 1];
#pragma unroll
        for (int k = kHalfN - 2; k >= 0; --k) {
            e = fmaf(e, x2, kb.ev[t][k]);
            o = fmaf(o, x2, kb.od[t][k]);
        }
        w[t] = fmaf(x, o, e);
        w[W - 1 - t] = fmaf(-x, o, e);
    }
    if (frac == 0.f) w[W - 1] = 0.f;  // strict support |u| < W/2
}

template <int W>
__device__ __forceinline__ void axis_taps(float g, int Ga, const KbParams& kb, float* w, int* j) {
    const float cf = floorf(g);
    const int cell = (int)cf;
    tap_weights<W>(g - cf, kb, w);
#pragma unroll
    for (int t = 0; t < W; ++t) {
        int jj = cell - W / 2 + 1 + t;
        jj = jj < 0 ? jj + Ga : (jj >= Ga ? jj - Ga : jj);
        j[t] = jj;
    }
}

// Workgroups are dispatched to the 8 XCDs of the chip round-robin (block p
// runs on XCD p mod 8).  Remapping p so that each XCD takes one contiguous
// eighth of the logical blocks keeps neighbouring tiles, whose footprints
// share grid cells, in the same XCD's L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned p, unsigned nblk) {
    const unsigned nx = 8, q = nblk / nx, r = nblk % nx;
    const unsigned x = p % nx, k = p / nx;
    return x * q + min(x, r) + k;
}

// Output of one (sample, coil group): the interpolated values, or the dual
// update that consumes them.
template <int CH>
__device__ __forceinline__ void interp_store(const InterpArgs& a, int64_t s, int c0, const float2* acc) {
    const int C = a.C;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int cc = c0 + c;
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

// ------------------------------------------------------------ interpolation
// One thread per (sorted sample, group of CH coils), coil group fastest, so
// the lanes of one sample read one contiguous C-vector per tap.
template <int D, int W, int CH>
__device__ __forceinline__ void interp_body(const InterpArgs& a, const KbParams& kb, int64_t gid) {
    const int ncg = a.C / CH;
    if (gid >= a.M * ncg) return;
    const int64_t s = gid / ncg;
    const int c0 = (int)(gid % ncg) * CH;
    const int C = a.C;
    float w[D][W];
    int jx[D][W];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) axis_taps<W>(a.g[s * D + ax], a.G[ax], kb, w[ax], jx[ax]);
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
                    const float2 v = src[c];
                    acc[c].x += wt * v.x;
                    acc[c].y += wt * v.y;
                }
            }
        }
    } else {
#pragma unroll 1
        for (int t0 = 0; t0 < W; ++t0) {
            const int64_t r0 = (int64_t)jx[0][t0] * a.G[1];
            float wa = w[0][0];
#pragma unroll
            for (int q = 1; q < W; ++q) wa = (t0 == q) ? w[0][q] : wa;
#pragma unroll
            for (int t1 = 0; t1 < W; ++t1) {
                const int64_t r1 = (r0 + jx[1][t1]) * a.G[2];
                const float w01 = wa * w[1][t1];
#pragma unroll
                for (int t2 = 0; t2 < W; ++t2) {
                    const float wt = w01 * w[2][t2];
                    const float2* src = a.grid + (r1 + jx[2][t2]) * C + c0;
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        const float2 v = src[c];
                        acc[c].x += wt * v.x;
                        acc[c].y += wt * v.y;
                    }
                }
            }
        }
    }
    interp_store<CH>(a, s, c0, acc);
}

template <int D, int W, int CH>
__global__ void __launch_bounds__(256) k_interp(InterpArgs a, KbParams kb) {
    interp_body<D, W, CH>(a, kb, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// find s with start[s] <= b < start[s+1] (start has n+1 entries)
__device__ __forceinline__ int batch_slot(const int64_t* start, int n, int64_t b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (start[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// interpolation of many slices in one launch (2D, width 4, coil groups of 4):
// the threads of slice s are blocks start[s] .. start[s+1]-1
__global__ void __launch_bounds__(256) k_interp_batch(const InterpArgs* __restrict__ args,
                                                      const int64_t* __restrict__ start, int n, KbParams kb) {
    const int s = batch_slot(start, n, blockIdx.x);
    const InterpArgs a = args[s];
    interp_body<2, 4, 4>(a, kb, (int64_t)(blockIdx.x - start[s]) * blockDim.x + threadIdx.x);
}

void launch_interp_batch(const InterpArgs* d_args, const int64_t* d_start, int n, int64_t nblk, const KbParams& kb,
                         hipStream_t s) {
    if (nblk <= 0) return;
    if (nblk > 0x7fffffff) fail(KP_ERR_UNSUPPORTED, "batched interpolation grid too large");
    hipLaunchKernelGGL(k_interp_batch, dim3((unsigned)nblk), dim3(256), 0, s, d_args, d_start, n, kb);
    KP_LAUNCH_CHECK();
}

template <int D, int W>
static void interp_dispatch_ch(const InterpArgs& a, const KbParams& kb, hipStream_t s) {
    const int CH = a.C % 4 == 0 ? 4 : (a.C % 2 == 0 ? 2 : 1);
    const int64_t n = a.M * (a.C / CH);
    const unsigned nblk = (unsigned)((n + 255) / 256);
    if (CH == 4)
        hipLaunchKernelGGL((k_interp<D, W, 4>), dim3(nblk), dim3(256), 0, s, a, kb);
    else if (CH == 2)
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

// Tile-staged interpolation.  Samples are sorted by the tile that holds
// their cell, so the taps of every sample of tile T lie in T's halo: the
// (B_a + W - 1)-cell box starting W/2 - 1 cells before the tile.  One block
// per (piece of a tile, group of CG coils) copies that halo into LDS with
// coalesced loads, then its threads interpolate the piece's samples from LDS.
// Each grid value is read from memory once per tile instead of once per tap.
template <int D, int W, int CG>
__global__ void __launch_bounds__(256) k_interp_tile(InterpArgs a, const int4* __restrict__ items, KbParams kb) {
    extern __shared__ float2 halo[];
    const int ncg = a.C / CG;
    const int item = blockIdx.x / ncg, cg = blockIdx.x % ncg;
    const int4 wk = items[item];
    const int tile = wk.x, start = wk.y, count = wk.z;
    int org[3] = {0, 0, 0}, H[3] = {1, 1, 1};
    {
        int rem = tile;
        for (int ax = D - 1; ax >= 0; --ax) {
            org[ax] = (rem % a.nb[ax]) * a.B[ax];
            rem /= a.nb[ax];
        }
    }
#pragma unroll
    for (int ax = 0; ax < D; ++ax) H[ax] = a.B[ax] + W - 1;
    const int hcells = H[0] * H[1] * H[2];
    const int C = a.C;
    // ---- stage the halo (coil group cg), wrapping periodically
    constexpr int V = CG >= 2 ? 2 : 1;  // coils per load
    for (int i = threadIdx.x; i < hcells * (CG / V); i += blockDim.x) {
        const int cell = i / (CG / V), part = i % (CG / V);
        int h[3], rem = cell;
        for (int ax = D - 1; ax >= 0; --ax) {
            h[ax] = rem % H[ax];
            rem /= H[ax];
        }
        int64_t gi = 0;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            int j = org[ax] - W / 2 + 1 + h[ax];
            j = j < 0 ? j + a.G[ax] : (j >= a.G[ax] ? j - a.G[ax] : j);
            gi = gi * a.G[ax] + j;
        }
        const float2* src = a.grid + gi * C + cg * CG + part * V;
        if (V == 2) {
            const float4 v = *reinterpret_cast<const float4*>(src);
            halo[cell * CG + part * 2] = make_float2(v.x, v.y);
            halo[cell * CG + part * 2 + 1] = make_float2(v.z, v.w);
        } else {
            halo[cell * CG + part] = *src;
        }
    }
    __syncthreads();
    // ---- interpolate the piece's samples from LDS
    for (int64_t s = start + threadIdx.x; s < start + count; s += blockDim.x) {
        float w[D][W];
        int l[D];
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            const float g = a.g[s * D + ax];
            const float cf = floorf(g);
            tap_weights<W>(g - cf, kb, w[ax]);
            l[ax] = (int)cf - org[ax];  // halo index of the first tap
        }
        float2 acc[CG];
#pragma unroll
        for (int c = 0; c < CG; ++c) acc[c] = make_float2(0.f, 0.f);
        if (D == 2) {
#pragma unroll
            for (int t0 = 0; t0 < W; ++t0) {
                const int r0 = (l[0] + t0) * H[1] + l[1];
#pragma unroll
                for (int t1 = 0; t1 < W; ++t1) {
                    const float wt = w[0][t0] * w[1][t1];
                    const float2* src = halo + (r0 + t1) * CG;
#pragma unroll
                    for (int c = 0; c < CG; ++c) {
                        const float2 v = src[c];
                        acc[c].x = fmaf(wt, v.x, acc[c].x);
                        acc[c].y = fmaf(wt, v.y, acc[c].y);
                    }
                }
            }
        } else {
#pragma unroll 1
            for (int t0 = 0; t0 < W; ++t0) {
                float wa = w[0][0];
#pragma unroll
                for (int q = 1; q < W; ++q) wa = (t0 == q) ? w[0][q] : wa;
#pragma unroll
                for (int t1 = 0; t1 < W; ++t1) {
                    const int r1 = ((l[0] + t0) * H[1] + l[1] + t1) * H[2] + l[2];
                    const float w01 = wa * w[1][t1];
#pragma unroll
                    for (int t2 = 0; t2 < W; ++t2) {
                        const float wt = w01 * w[2][t2];
                        const float2* src = halo + (r1 + t2) * CG;
#pragma unroll
                        for (int c = 0; c < CG; ++c) {
                            const float2 v = src[c];
                            acc[c].x = fmaf(wt, v.x, acc[c].x);
                            acc[c].y = fmaf(wt, v.y, acc[c].y);
                        }
                    }
                }
            }
        }
        interp_store<CG>(a, s, cg * CG, acc);
    }
}

// 3D, width 4, CG coils per block (CG = 4 or 2): a group of 2 CG lanes
// serves one sample, each lane two coils (one 16-byte read per cell) at one
// of the 4 taps along z, so for each of the 16 (x, y) taps a group reads one
// contiguous run of 4 CG complex values of the halo; rows of one halo line
// are padded to H2P cells.  The weights of up to kTlBatch samples are
// computed once per batch into an LDS table, whose rows also take the
// interpolated values of their sample (each row is read only by its own
// sample's lanes before they write it); the 4 z-tap partial sums of a coil
// are added by a two-step DPP row shift.
__device__ __forceinline__ float dpp_row_shr4(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_row_shr1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_row_shr2(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, true));
}

constexpr int kTlThreads = 512;        // threads per block of the tap-lane interpolation
constexpr int kTlBatch = kTlThreads;   // samples whose weights sit in LDS at a time
constexpr int kTlStage = 12;           // halo loads per thread held in registers
constexpr int kTlCG = 4;       // coils per block of the tap-lane interpolation

__host__ __device__ inline int tl_h2p(int H2) { return H2 + ((12 - H2 % 8) % 8); }

// TB0..TB2: the tile shape as compile-time constants (0: taken from the
// arguments).  With constants every halo index is a multiply-shift and the
// 16 tap offsets fold into the LDS instructions' immediate offsets.
template <int TB0, int TB1, int TB2, int CG>
__global__ void __launch_bounds__(kTlThreads) k_interp_tl3(InterpArgs a, const int4* __restrict__ items, KbParams kb) {
    static_assert(CG == 2 || CG == 4, "coil groups of 2 or 4");
    constexpr int NP = CG / 2;          // float4 (two coils) per cell
    constexpr int SPW = 64 / (4 * NP);  // samples per wave
    extern __shared__ float4 tl_smem[];
    const int ncg = a.C / CG;
    // The coil groups of one piece are launched 8 blocks apart (blocks are
    // dealt to the 8 XCDs in turn, so they tend to share an L2 and the rest
    // of every grid cell's coil vector is found there).
    int item, cg;
    {
        const int b = blockIdx.x, nitems = gridDim.x / ncg;
        const int grp = b / (8 * ncg), r = b % (8 * ncg);
        if ((grp + 1) * 8 <= nitems) {
            item = grp * 8 + r % 8;
            cg = r / 8;
        } else {
            item = grp * 8 + r / ncg;
            cg = r % ncg;
        }
    }
    const int4 wk = items[item];
    const int tile = wk.x, start = wk.y, count = wk.z;
    int org[3];
    {
        int rem = tile;
        for (int ax = 2; ax >= 0; --ax) {
            org[ax] = (rem % a.nb[ax]) * a.B[ax];
            rem /= a.nb[ax];
        }
    }
    const int H0 = (TB0 ? TB0 : a.B[0]) + 3, H1 = (TB1 ? TB1 : a.B[1]) + 3, H2 = (TB2 ? TB2 : a.B[2]) + 3;
    const int H2P = tl_h2p(H2);
    const int hcells = H0 * H1 * H2;
    float2* halo = reinterpret_cast<float2*>(tl_smem);                        // [H0][H1][H2P][CG]
    float* tab = reinterpret_cast<float*>(halo + (size_t)H0 * H1 * H2P * CG);  // [kTlBatch][16]
    const int C = a.C;
    const int tid = threadIdx.x;

    // ---- halo loads into registers (two coils per float4)
    // 8^3 tiles (11^3 halo): thread t < 11 * 11 NP takes float4 t % (11 NP)
    // of the z-rows (h0, h1 = t / (11 NP)) for h0 = 0..10, so only h0 varies
    // between its loads; other shapes: the halo's float4s dealt out in order.
    constexpr bool ROWS = TB0 == 8 && TB1 == 8 && TB2 == 8;
    constexpr int RW = 11 * NP;  // float4 per z-row of the 11^3 halo
    float4 hv[kTlStage];
    if (ROWS) {
        if (tid < 11 * RW) {
            const int h1 = tid / RW, pos = tid % RW, h2 = pos / NP, part = pos % NP;
            int j1 = org[1] - 1 + h1, j2 = org[2] - 1 + h2;
            j1 = j1 < 0 ? j1 + a.G[1] : (j1 >= a.G[1] ? j1 - a.G[1] : j1);
            j2 = j2 < 0 ? j2 + a.G[2] : (j2 >= a.G[2] ? j2 - a.G[2] : j2);
            const float2* rowp = a.grid + ((int64_t)j1 * a.G[2] + j2) * C + cg * CG + part * 2;
            const int64_t plane = (int64_t)a.G[1] * a.G[2] * C;
#pragma unroll
            for (int r = 0; r < 11; ++r) {
                int j0 = org[0] - 1 + r;
                j0 = j0 < 0 ? j0 + a.G[0] : (j0 >= a.G[0] ? j0 - a.G[0] : j0);
                hv[r] = *reinterpret_cast<const float4*>(rowp + j0 * plane);
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < kTlStage; ++r) {
            const int i = tid + r * kTlThreads;
            if (i < hcells * NP) {
                const int cell = i / NP, part = i % NP;
                const int h2 = cell % H2, h01 = cell / H2, h1 = h01 % H1, h0 = h01 / H1;
                int j0 = org[0] - 1 + h0, j1 = org[1] - 1 + h1, j2 = org[2] - 1 + h2;
                j0 = j0 < 0 ? j0 + a.G[0] : (j0 >= a.G[0] ? j0 - a.G[0] : j0);
                j1 = j1 < 0 ? j1 + a.G[1] : (j1 >= a.G[1] ? j1 - a.G[1] : j1);
                j2 = j2 < 0 ? j2 + a.G[2] : (j2 >= a.G[2] ? j2 - a.G[2] : j2);
                const int64_t gi = ((int64_t)j0 * a.G[1] + j1) * a.G[2] + j2;
                hv[r] = *reinterpret_cast<const float4*>(a.grid + gi * C + cg * CG + part * 2);
            }
        }
    }

    const int lane = tid & 63, wave = tid >> 6;
    const int pr = lane % NP, t2 = (lane / NP) & 3, sub = lane / (4 * NP);
    // halo offsets (in float2) of the 16 (x, y) taps relative to a sample's base
    int toff[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) toff[t] = (((t >> 2) * H1 + (t & 3)) * H2P) * CG;
    for (int b0 = 0; b0 < count; b0 += kTlBatch) {
        const int nbt = min(kTlBatch, count - b0);
        if (b0 > 0) __syncthreads();  // the previous batch is done with the table
        // ---- weights and halo base of this batch's samples
        if (tid < nbt) {
            const int64_t s = start + b0 + tid;
            float w[3][4];
            int l[3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const float g = a.g[s * 3 + ax];
                const float cf = floorf(g);
                tap_weights<4>(g - cf, kb, w[ax]);
                l[ax] = (int)cf - org[ax];
            }
            float4* row = reinterpret_cast<float4*>(tab + tid * 16);
            row[0] = make_float4(w[0][0], w[0][1], w[0][2], w[0][3]);
            row[1] = make_float4(w[1][0], w[1][1], w[1][2], w[1][3]);
            row[2] = make_float4(w[2][0], w[2][1], w[2][2], w[2][3]);
            row[3] = make_float4(__int_as_float((l[0] * H1 + l[1]) * H2P + l[2]), 0.f, 0.f, 0.f);
        }
        if (b0 == 0 && ROWS) {
            if (tid < 11 * RW) {
                const int h1 = tid / RW, pos = tid % RW;
                float2* dst = halo + ((size_t)h1 * H2P + pos / NP) * CG + (pos % NP) * 2;
#pragma unroll
                for (int r = 0; r < 11; ++r) {
                    float2* d = dst + (size_t)r * H1 * H2P * CG;
                    d[0] = make_float2(hv[r].x, hv[r].y);
                    d[1] = make_float2(hv[r].z, hv[r].w);
                }
            }
        } else if (b0 == 0) {
#pragma unroll
            for (int r = 0; r < kTlStage; ++r) {
                const int i = tid + r * kTlThreads;
                if (i < hcells * NP) {
                    const int cell = i / NP, part = i % NP;
                    const int h2 = cell % H2, h01 = cell / H2;
                    float2* dst = halo + ((size_t)h01 * H2P + h2) * CG + part * 2;
                    dst[0] = make_float2(hv[r].x, hv[r].y);
                    dst[1] = make_float2(hv[r].z, hv[r].w);
                }
            }
        }
        __syncthreads();
        // ---- one sample per group of 4 NP lanes (two coils per lane)
        for (int i = wave * SPW + sub; i < nbt; i += (kTlThreads / 64) * SPW) {
            float* row = tab + i * 16;
            const float4 w0 = *reinterpret_cast<const float4*>(row);
            const float4 w1 = *reinterpret_cast<const float4*>(row + 4);
            const float w2 = row[8 + t2];
            const int base = __float_as_int(row[12]);
            const float w0v[4] = {w0.x, w0.y, w0.z, w0.w};
            const float w1v[4] = {w1.x * w2, w1.y * w2, w1.z * w2, w1.w * w2};
            const int hb = (base + t2) * CG + 2 * pr;
            float4 hvv[16];  // all 16 reads issued before the first use
#pragma unroll
            for (int t = 0; t < 16; ++t) hvv[t] = *reinterpret_cast<const float4*>(halo + hb + toff[t]);
            // axis-1 taps first, then the axis-0 weight once per t0
            float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
            for (int t0 = 0; t0 < 4; ++t0) {
                float s0 = w1v[0] * hvv[t0 * 4].x, s1 = w1v[0] * hvv[t0 * 4].y;
                float s2 = w1v[0] * hvv[t0 * 4].z, s3 = w1v[0] * hvv[t0 * 4].w;
#pragma unroll
                for (int t1 = 1; t1 < 4; ++t1) {
                    s0 = fmaf(w1v[t1], hvv[t0 * 4 + t1].x, s0);
                    s1 = fmaf(w1v[t1], hvv[t0 * 4 + t1].y, s1);
                    s2 = fmaf(w1v[t1], hvv[t0 * 4 + t1].z, s2);
                    s3 = fmaf(w1v[t1], hvv[t0 * 4 + t1].w, s3);
                }
                a0 = fmaf(w0v[t0], s0, a0);
                a1 = fmaf(w0v[t0], s1, a1);
                a2 = fmaf(w0v[t0], s2, a2);
                a3 = fmaf(w0v[t0], s3, a3);
            }
            // the 4 z-tap lanes of a coil pair sit NP lanes apart
            float acc[4] = {a0, a1, a2, a3};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (NP == 2) {
                    acc[q] += dpp_row_shr2(acc[q]);
                    acc[q] += dpp_row_shr4(acc[q]);
                } else {
                    acc[q] += dpp_row_shr1(acc[q]);
                    acc[q] += dpp_row_shr2(acc[q]);
                }
            }
            // the row's reads above are done (their values fed the sums), so
            // its first CG complex slots take the result
            if (t2 == 3) reinterpret_cast<float4*>(row)[pr] = make_float4(acc[0], acc[1], acc[2], acc[3]);
        }
        __syncthreads();
        // ---- output stage of the batch: one sample's CG coils per thread
        // (CG contiguous complex values of every [sample][coil] array,
        // 16-byte accesses)
        for (int i = tid; i < nbt; i += kTlThreads) {
            const int64_t s = start + b0 + i;
            const int64_t e = s * C + cg * CG;
            const float4* ob = reinterpret_cast<const float4*>(tab + i * 16);
            float4 v[NP];
#pragma unroll
            for (int q = 0; q < NP; ++q) v[q] = ob[q];
            if (a.mode == IO_CALLER) {
                const int64_t ps = a.perm[s];
                const int64_t c0 = (int64_t)(cg * CG) * a.M + ps;
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    a.out[c0 + (2 * q) * a.M] = make_float2(v[q].x, v[q].y);
                    a.out[c0 + (2 * q + 1) * a.M] = make_float2(v[q].z, v[q].w);
                }
                continue;
            }
            float4* o4 = reinterpret_cast<float4*>(a.mode == IO_DUAL ? a.u + e : a.out + e);
            if (a.mode == IO_INTERNAL) {
#pragma unroll
                for (int q = 0; q < NP; ++q) o4[q] = v[q];
                continue;
            }
            float pv[CG];
#pragma unroll
            for (int q = 0; q < CG; ++q) pv[q] = 1.f;
            if (a.p) {
                if (a.p_mc) {
#pragma unroll
                    for (int q = 0; q < NP; ++q) {
                        const float2 pp = *reinterpret_cast<const float2*>(a.p + e + 2 * q);
                        pv[2 * q] = pp.x;
                        pv[2 * q + 1] = pp.y;
                    }
                } else {
                    const float pq = a.p[s];
#pragma unroll
                    for (int q = 0; q < CG; ++q) pv[q] = pq;
                }
            }
            if (a.mode == IO_PMUL) {
#pragma unroll
                for (int q = 0; q < NP; ++q)
                    o4[q] = make_float4(pv[2 * q] * v[q].x, pv[2 * q] * v[q].y, pv[2 * q + 1] * v[q].z,
                                        pv[2 * q + 1] * v[q].w);
                continue;
            }
            // IO_DUAL: u <- (u + sigma p (v - y)) / (1 + sigma p)
            const float sg = *a.sigma;
            const float4* y4 = reinterpret_cast<const float4*>(a.y + e);
            float4 uo[NP], yo[NP];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                uo[q] = o4[q];
                yo[q] = y4[q];
            }
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const float sp0 = sg * pv[2 * q], sp1 = sg * pv[2 * q + 1];
                const float d0 = 1.f / (1.f + sp0), d1 = 1.f / (1.f + sp1);
                o4[q] = make_float4((uo[q].x + sp0 * (v[q].x - yo[q].x)) * d0, (uo[q].y + sp0 * (v[q].y - yo[q].y)) * d0,
                                    (uo[q].z + sp1 * (v[q].z - yo[q].z)) * d1, (uo[q].w + sp1 * (v[q].w - yo[q].w)) * d1);
            }
        }
    }
}

size_t interp_tl3_lds_bytes(const int* B, int CG = kTlCG) {
    const int H0 = B[0] + 3, H1 = B[1] + 3, H2P = tl_h2p(B[2] + 3);
    return (size_t)H0 * H1 * H2P * CG * sizeof(float2) + (size_t)kTlBatch * 16 * sizeof(float);
}

bool interp_tl3_ok(int d, int W, const int* B, int C) {
    return d == 3 && W == 4 && C % kTlCG == 0 && (B[0] + 3) * (B[1] + 3) * (B[2] + 3) * (kTlCG / 2) <= kTlStage * kTlThreads &&
           interp_tl3_lds_bytes(B) <= 80 * 1024;
}

size_t interp_tile_lds_bytes(int d, int W, const int* B, int C) {
    const int CG = C % 4 == 0 ? 4 : (C % 2 == 0 ? 2 : 1);
    size_t cells = 1;
    for (int ax = 0; ax < d; ++ax) cells *= (size_t)(B[ax] + W - 1);
    return cells * CG * sizeof(float2);
}

template <int D, int W>
static void interp_tile_dispatch(const InterpArgs& a, const int4* items, int64_t nitems, size_t lds, const KbParams& kb,
                                 hipStream_t s) {
    const int CG = a.C % 4 == 0 ? 4 : (a.C % 2 == 0 ? 2 : 1);
    const int64_t nb = nitems * (a.C / CG);
    if (nb > 0x7fffffff) fail(KP_ERR_UNSUPPORTED, "interpolation grid too large");
    const void* fn = CG == 4 ? (const void*)k_interp_tile<D, W, 4>
                             : (CG == 2 ? (const void*)k_interp_tile<D, W, 2> : (const void*)k_interp_tile<D, W, 1>);
    if (lds > 65536) {
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    }
    if (CG == 4)
        hipLaunchKernelGGL((k_interp_tile<D, W, 4>), dim3((unsigned)nb), dim3(256), lds, s, a, items, kb);
    else if (CG == 2)
        hipLaunchKernelGGL((k_interp_tile<D, W, 2>), dim3((unsigned)nb), dim3(256), lds, s, a, items, kb);
    else
        hipLaunchKernelGGL((k_interp_tile<D, W, 1>), dim3((unsigned)nb), dim3(256), lds, s, a, items, kb);
    KP_LAUNCH_CHECK();
}

void launch_interp_tiles(int d, int W, const InterpArgs& a, const int4* items, int64_t nitems, const KbParams& kb,
                         hipStream_t s) {
    if (a.M <= 0 || nitems <= 0) return;
    if (interp_tl3_ok(d, W, a.B, a.C)) {
        const int64_t nb = nitems * (a.C / kTlCG);
        if (nb > 0x7fffffff) fail(KP_ERR_UNSUPPORTED, "interpolation grid too large");
        const size_t lds = interp_tl3_lds_bytes(a.B);
        const bool b888 = a.B[0] == 8 && a.B[1] == 8 && a.B[2] == 8;
        const void* fn = b888 ? (const void*)k_interp_tl3<8, 8, 8, kTlCG> : (const void*)k_interp_tl3<0, 0, 0, kTlCG>;
        if (lds > 65536) {
            (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            (void)hipGetLastError();
        }
        if (b888)
            hipLaunchKernelGGL((k_interp_tl3<8, 8, 8, kTlCG>), dim3((unsigned)nb), dim3(kTlThreads), lds, s, a, items, kb);
        else
            hipLaunchKernelGGL((k_interp_tl3<0, 0, 0, kTlCG>), dim3((unsigned)nb), dim3(kTlThreads), lds, s, a, items, kb);
        KP_LAUNCH_CHECK();
        return;
    }
    const size_t lds = interp_tile_lds_bytes(d, W, a.B, a.C);
#define KP_ITILE_W(DD, WW) \
    if (d == DD && W == WW) return interp_tile_dispatch<DD, WW>(a, items, nitems, lds, kb, s);
    KP_ITILE_W(2, 2) KP_ITILE_W(2, 4) KP_ITILE_W(2, 6) KP_ITILE_W(2, 8)
    KP_ITILE_W(3, 2) KP_ITILE_W(3, 4) KP_ITILE_W(3, 6) KP_ITILE_W(3, 8)
#undef KP_ITILE_W
    fail(KP_ERR_UNSUPPORTED, "interp: unsupported (d, W)");
}

// ------------------------------------------------------------ spreading
static int coil_group(int C) { return C % 4 == 0 ? 4 : (C % 2 == 0 ? 2 : 1); }

int spread_threads(int d, const int* B, int C) {
    const int lines = d == 3 ? B[0] * B[1] : B[0];
    return lines * (C / coil_group(C));
}

// LDS carve-up for a chunk of E entries (all 4-byte words):
//   code[E] | wl[(d-1) W][E+1] | wz[ZM][E] | u[C/CG][CG][E] (float2, each coil
//   group padded by one element; C E + C/CG <= C (E+1)) | bstart[NBK+1]
// (rows of wl padded by one element and coil groups by one float2: lanes
// reading one entry from different rows, or for different coil groups, fall
// into different banks; within a group the CG coils of an entry are E float2
// apart, so one base register and two ds_read2st64_b64 reach all four)
// (entry index fastest, so lanes reading different entries hit different banks)
// buckets of a tile: first-tap positions -(W-1) .. B_a - 1 on the leading axes
int spread_nbk(int d, int W, const int* B) {
    return d == 3 ? (B[0] + W - 1) * (B[1] + W - 1) : (B[0] + W - 1);
}

// register line length of the spreading kernel for a tile depth
int spread_zm(int d, const int* B) { return B[d - 1] <= 4 ? 4 : kZMax; }

size_t spread_lds_bytes(int d, int W, const int* B, int C, int zm) {
    const size_t E = kSpreadChunk, EP = E + 1;
    const size_t nbk = (size_t)spread_nbk(d, W, B);
    if (zm <= 0) zm = spread_zm(d, B);
    const size_t words = E + EP * (size_t)(d - 1) * W + E * (size_t)zm + 2 * EP * (size_t)C + nbk + 1;
    return 4 * words;
}

// Owner-gather spreading of one work item (a tile, or a piece of a split
// tile).  Each thread owns one grid line of the tile along the last axis and
// a group of CG coils, and keeps up to kZMax cells x CG coils in registers.
// Entries arrive in chunks of E, already ordered by the bucket of their first
// tap on the leading axes (plan time), so the entries that reach a line form
// W contiguous runs of the chunk; a binary search per bucket finds them.
// PF: one entry per thread per chunk (blockDim >= E) and C <= 8; the
// coordinates and coil values of the next chunk, and the touch indices of the
// one after, are loaded while the current chunk is gathered.
template <int D, int W, int CG, int ZM = kZMax, bool PF = false>
__device__ __forceinline__ void spread_body(const SpreadArgs& a, const KbParams& kb, int64_t item, int* smem) {
    constexpr int E = kSpreadChunk;
    constexpr int NLW = (D - 1) * W;  // leading-axis weights per entry
    const int C = a.C;
    const int B0 = a.B[0];
    const int B1 = D == 3 ? a.B[1] : 1;
    const int ZL = a.B[D - 1];
    const int NB1 = D == 3 ? B1 + W - 1 : 1;
    const int NBK = D == 3 ? (B0 + W - 1) * NB1 : (B0 + W - 1);
    constexpr int EP = E + 1;
    int* code = smem;
    float* wl = (float*)(code + E);
    float* wz = wl + EP * NLW;
    float2* uu = (float2*)(wz + E * ZM);  // [C / CG][CG][E], each coil group padded by one element
    constexpr int UG = CG * E + 1;        // coil-group stride of uu
    int* bstart = (int*)(uu + EP * C);

    const int4 wk = a.work[item];
    const int tile = wk.x, start = wk.y, count = wk.z, slot = wk.w;
    int tc[3] = {0, 0, 0};
    {
        int rem = tile;
        for (int ax = D - 1; ax >= 0; --ax) {
            tc[ax] = rem % a.nb[ax];
            rem /= a.nb[ax];
        }
    }
    int org[3];
    for (int ax = 0; ax < D; ++ax) org[ax] = tc[ax] * a.B[ax];

    const int ncg = C / CG;
    const int nthr = (D == 3 ? B0 * B1 : B0) * ncg;
    const int tid = threadIdx.x;
    const bool owner = tid < nthr;
    const int line = tid / ncg, cg = tid % ncg;
    const int j0 = D == 3 ? line / B1 : line;
    const int j1 = D == 3 ? line % B1 : 0;

    float2 acc[ZM][CG];
#pragma unroll
    for (int z = 0; z < ZM; ++z)
#pragma unroll
        for (int c = 0; c < CG; ++c) acc[z][c] = make_float2(0.f, 0.f);

    // weights and bucket of entry e into LDS (and its coil values when given)
    auto stage = [&](int e, int bk, const float* gv, const float2* uv) {
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            const float g = gv[ax];
            const float cf = floorf(g);
            float w[W];
            tap_weights<W>(g - cf, kb, w);
            if (ax < D - 1) {
#pragma unroll
                for (int t = 0; t < W; ++t) wl[(ax * W + t) * EP + e] = w[t];
            } else {
                int l = (int)cf - W / 2 + 1 - org[ax];
                if (l < -(W - 1)) l += a.G[ax];
                else if (l > a.B[ax] - 1) l -= a.G[ax];
#pragma unroll
                for (int z = 0; z < ZM; ++z) {
                    const int t = z - l;
                    float v = 0.f;
#pragma unroll
                    for (int q = 0; q < W; ++q) v = (t == q) ? w[q] : v;
                    wz[z * E + e] = (z < ZL) ? v : 0.f;
                }
            }
        }
        // low 16 bits: bucket; high 16 bits (signed): the byte offset
        // 4 (e - b1 EP) with b1 the bucket's axis-1 coordinate, so that the
        // axis-1 weight of this entry for line j1 sits (2W - 1 + j1) EP floats
        // past wl plus that offset (3D)
        code[e] = bk | (int)((unsigned)(4 * (e - (D == 3 ? bk % NB1 : 0) * EP)) << 16);
        if (uv) {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c < C) uu[(c / CG) * UG + (c % CG) * E + e] = uv[c];
        }
    };
    // pipeline registers (PF): data of the current chunk's entry tid, touch
    // index and bucket of the next chunk's
    int bk0 = 0, s1 = 0, bk1 = 0;
    float g0[D];
    float2 u0[8];
    auto fetch = [&](int s) {
#pragma unroll
        for (int ax = 0; ax < D; ++ax) g0[ax] = a.g[(int64_t)s * D + ax];
        const float2* src = a.k + (int64_t)s * C;
#pragma unroll
        for (int c = 0; c < 8; ++c) u0[c] = c < C ? src[c] : make_float2(0.f, 0.f);
    };
    if (PF) {
        if (tid < count) {
            bk0 = a.code[start + tid];
            fetch(a.touch[start + tid]);
        }
        if (E + tid < count) {
            s1 = a.touch[start + E + tid];
            bk1 = a.code[start + E + tid];
        }
    }

    for (int c0 = 0; c0 < count; c0 += E) {
        const int n = min(E, count - c0);
        if (c0 > 0) __syncthreads();  // the previous chunk is consumed
        // ---- A: stage the chunk: bucket, weights, coil values
        if (PF) {
            if (tid < n) stage(tid, bk0, g0, u0);
        } else {
            for (int e = tid; e < n; e += blockDim.x) {
                const int s = a.touch[start + c0 + e];
                float gv[D];
#pragma unroll
                for (int ax = 0; ax < D; ++ax) gv[ax] = a.g[(int64_t)s * D + ax];
                const float2* src = a.k + (int64_t)s * C;
                for (int c = 0; c < C; ++c) uu[(c / CG) * UG + (c % CG) * E + e] = src[c];
                stage(e, a.code[start + c0 + e], gv, nullptr);
            }
        }
        __syncthreads();
        // ---- B: first entry of every bucket (the chunk is sorted by bucket)
        for (int b = tid; b <= NBK; b += blockDim.x) {
            int lo = 0, hi = n;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((code[mid] & 0xffff) < b) lo = mid + 1; else hi = mid;
            }
            bstart[b] = lo;
        }
        __syncthreads();
        if (PF) {  // loads for the next chunks, in flight during the gather
            if (c0 + E + tid < count) {
                bk0 = bk1;
                fetch(s1);
            }
            if (c0 + 2 * E + tid < count) {
                s1 = a.touch[start + c0 + 2 * E + tid];
                bk1 = a.code[start + c0 + 2 * E + tid];
            }
        }
        // ---- C: each owner thread gathers the entries covering its line
        if (owner) {
            const char* wly = reinterpret_cast<const char*>(wl + (2 * W - 1 + j1) * EP);
            // the W buckets of one q0 along axis 1 are consecutive, so their
            // entries form one contiguous run; the axis-1 tap of an entry
            // follows from its bucket coordinate b1
            auto gather = [&](int idx, const float* wrow) {
                float wA = wrow[idx];
                if (D == 3) wA *= *reinterpret_cast<const float*>(wly + (code[idx] >> 16));
                const float2* up = uu + cg * UG + idx;
                float2 uv[CG];
#pragma unroll
                for (int c = 0; c < CG; ++c) uv[c] = up[c * E];
#pragma unroll
                for (int z = 0; z < ZM; ++z) {
                    const float wt = wA * wz[z * E + idx];
#pragma unroll
                    for (int c = 0; c < CG; ++c) {
                        acc[z][c].x = fmaf(wt, uv[c].x, acc[z][c].x);
                        acc[z][c].y = fmaf(wt, uv[c].y, acc[z][c].y);
                    }
                }
            };
            // the W runs of this line, walked as one sequence: a lane's trip
            // count is its total over the runs, so a wave waits for its
            // busiest line once per chunk instead of once per run
            int rs[W], re[W], tot = 0;
#pragma unroll
            for (int q0 = 0; q0 < W; ++q0) {
                const int bb = D == 3 ? (j0 + q0) * NB1 + j1 : (j0 + q0);
                rs[q0] = bstart[bb];
                re[q0] = bstart[bb + (D == 3 ? W : 1)];
                tot += re[q0] - rs[q0];
            }
            int e = rs[0], end = re[0];
            const float* wrow = wl + (W - 1) * EP;  // axis-0 weight row of the current run
            auto advance = [&]() {  // to the first entry of the next non-empty run
                while (e == end) {
                    e = rs[1];
                    end = re[1];
#pragma unroll
                    for (int q = 1; q + 1 < W; ++q) {
                        rs[q] = rs[q + 1];
                        re[q] = re[q + 1];
                    }
                    wrow -= EP;
                }
            };
            int it = 0;
            for (; it + 1 < tot; it += 2) {
                advance();
                const int ea = e++;
                const float* ra = wrow;
                advance();
                const int eb = e++;
                gather(ea, ra);
                gather(eb, wrow);
            }
            if (it < tot) {
                advance();
                gather(e, wrow);
            }
        }
    }

    // ---- D: write the owned lines back
    if (owner) {
        int64_t row;
        if (D == 3)
            row = ((int64_t)(org[0] + j0) * a.G[1] + (org[1] + j1)) * a.G[2] + org[2];
        else
            row = (int64_t)(org[0] + j0) * a.G[1] + org[1];
        // a split tile writes its partial sums to its own slot; the slots of
        // a tile are added in order afterwards (k_reduce_partials)
        const int64_t cells = (int64_t)B0 * B1 * ZL;
        float2* base = slot < 0 ? a.grid + row * C : a.partial + ((int64_t)slot * cells + (int64_t)line * ZL) * C;
#pragma unroll
        for (int z = 0; z < ZM; ++z) {
            if (z >= ZL) break;
            float2* dst = base + (int64_t)z * C + cg * CG;
#pragma unroll
            for (int c = 0; c < CG; ++c) dst[c] = acc[z][c];
        }
    }
}

// Sum the partial tiles of every split tile in slot order into the grid.
// heavy[h] = (tile, first slot, number of slots).
__global__ void k_reduce_partials(SpreadArgs a, const int4* heavy, int d) {
    const int4 h = heavy[blockIdx.x];
    const int B0 = a.B[0], B1 = d == 3 ? a.B[1] : 1, ZL = a.B[d - 1];
    const int C = a.C;
    const int64_t cells = (int64_t)B0 * B1 * ZL;
    int tc[3] = {0, 0, 0}, rem = h.x;
    for (int ax = d - 1; ax >= 0; --ax) {
        tc[ax] = rem % a.nb[ax];
        rem /= a.nb[ax];
    }
    const int64_t i = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
    if (i < cells * C) {
        // slots summed in order; sixteen independent loads in flight (the
        // dense centre of a radial trajectory splits one tile into 100+ slots)
        const float2* src = a.partial + (int64_t)h.y * cells * C + i;
        const int64_t st = cells * C;
        float2 s = make_float2(0.f, 0.f);
        int q = 0;
        for (; q + 16 <= h.z; q += 16) {
            float2 v[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) v[t] = src[(q + t) * st];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                s.x += v[t].x;
                s.y += v[t].y;
            }
        }
        for (; q + 4 <= h.z; q += 4) {
            const float2 v0 = src[(q + 0) * st], v1 = src[(q + 1) * st];
            const float2 v2 = src[(q + 2) * st], v3 = src[(q + 3) * st];
            s.x += v0.x; s.y += v0.y;
            s.x += v1.x; s.y += v1.y;
            s.x += v2.x; s.y += v2.y;
            s.x += v3.x; s.y += v3.y;
        }
        for (; q < h.z; ++q) {
            const float2 v = src[q * st];
            s.x += v.x;
            s.y += v.y;
        }
        const int64_t cell = i / C;
        const int c = (int)(i % C);
        const int z = (int)(cell % ZL);
        const int64_t line = cell / ZL;
        int64_t row;
        if (d == 3) {
            const int j0 = (int)(line / B1), j1 = (int)(line % B1);
            row = ((int64_t)(tc[0] * B0 + j0) * a.G[1] + (tc[1] * B1 + j1)) * a.G[2] + tc[2] * ZL;
        } else {
            row = (int64_t)(tc[0] * B0 + line) * a.G[1] + tc[1] * ZL;
        }
        a.grid[(row + z) * C + c] = s;
    }
}

void launch_reduce_partials(const SpreadArgs& a, const int4* heavy, int nheavy, int d, hipStream_t s) {
    if (nheavy <= 0) return;
    const int64_t n = (int64_t)a.B[0] * (d == 3 ? a.B[1] : 1) * a.B[d - 1] * a.C;
    hipLaunchKernelGGL(k_reduce_partials, dim3(nheavy, (unsigned)((n + 255) / 256)), dim3(256), 0, s, a, heavy, d);
    KP_LAUNCH_CHECK();
}

template <int D, int W, int CG, int ZM, bool PF>
__global__ void __launch_bounds__(256) k_spread(SpreadArgs a, KbParams kb) {
    extern __shared__ int smem[];
    spread_body<D, W, CG, ZM, PF>(a, kb, blockIdx.x, smem);
}

// spreading of many slices in one launch (2D, width 4, coil groups of 4): the
// work items of slice s are blocks start[s] .. start[s+1]-1; ZM covers the
// deepest spreading tile of the batch
template <int ZM>
__global__ void __launch_bounds__(256) k_spread_batch(const SpreadArgs* __restrict__ args,
                                                      const int64_t* __restrict__ start, int n, KbParams kb) {
    extern __shared__ int smem[];
    const int s = batch_slot(start, n, blockIdx.x);
    const SpreadArgs a = args[s];
    spread_body<2, 4, 4, ZM>(a, kb, blockIdx.x - start[s], smem);
}

void launch_spread_batch(const SpreadArgs* d_args, const int64_t* d_start, int n, int64_t nblk, int threads,
                         size_t lds, int zm, const KbParams& kb, hipStream_t s) {
    if (nblk <= 0) return;
    if (nblk > 0x7fffffff) fail(KP_ERR_UNSUPPORTED, "batched spreading grid too large");
    if (zm != 4 && zm != kZMax) fail(KP_ERR_UNSUPPORTED, "batched spreading: register line must be 4 or 8 cells");
    const void* fn = zm == 4 ? (const void*)k_spread_batch<4> : (const void*)k_spread_batch<kZMax>;
    if (lds > 65536) {
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    }
    if (zm == 4)
        hipLaunchKernelGGL(k_spread_batch<4>, dim3((unsigned)nblk), dim3(threads), lds, s, d_args, d_start, n, kb);
    else
        hipLaunchKernelGGL(k_spread_batch<kZMax>, dim3((unsigned)nblk), dim3(threads), lds, s, d_args, d_start, n, kb);
    KP_LAUNCH_CHECK();
}

// partial-tile reduction of many slices: entry h = (slice, heavy index)
__global__ void k_reduce_batch(const SpreadArgs* __restrict__ args, const int2* __restrict__ hv,
                               const int4* const* __restrict__ heavy_lists) {
    const int2 e = hv[blockIdx.x];
    const SpreadArgs& a = args[e.x];
    const int4 h = heavy_lists[e.x][e.y];
    const int B0 = a.B[0], B1 = a.B[1], ZL = a.B[1];
    (void)B1;
    const int C = a.C;
    const int64_t cells = (int64_t)B0 * ZL;
    const int tc0 = h.x / a.nb[1], tc1 = h.x % a.nb[1];
    for (int64_t i = threadIdx.x; i < cells * C; i += blockDim.x) {
        const float2* src = a.partial + (int64_t)h.y * cells * C + i;
        float2 sm = make_float2(0.f, 0.f);
        for (int q = 0; q < h.z; ++q) {
            const float2 v = src[(int64_t)q * cells * C];
            sm.x += v.x;
            sm.y += v.y;
        }
        const int64_t cell = i / C;
        const int c = (int)(i % C);
        const int z = (int)(cell % ZL);
        const int64_t line = cell / ZL;
        const int64_t row = (int64_t)(tc0 * B0 + line) * a.G[1] + tc1 * ZL;
        a.grid[(row + z) * C + c] = sm;
    }
}

void launch_reduce_batch(const SpreadArgs* d_args, const int2* d_hv, const int4* const* d_lists, int nh,
                         hipStream_t s) {
    if (nh <= 0) return;
    hipLaunchKernelGGL(k_reduce_batch, dim3(nh), dim3(256), 0, s, d_args, d_hv, d_lists);
    KP_LAUNCH_CHECK();
}

template <int D, int W, int CG, int ZM>
static void spread_launch(const SpreadArgs& a, const KbParams& kb, size_t lds, int block, hipStream_t s) {
    const dim3 grid((unsigned)a.nwork);
    if (block >= kSpreadChunk && a.C <= 8) {
        (void)hipFuncSetAttribute((const void*)k_spread<D, W, CG, ZM, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_spread<D, W, CG, ZM, true>), grid, dim3(block), lds, s, a, kb);
    } else {
        (void)hipFuncSetAttribute((const void*)k_spread<D, W, CG, ZM, false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_spread<D, W, CG, ZM, false>), grid, dim3(block), lds, s, a, kb);
    }
    KP_LAUNCH_CHECK();
}

template <int D, int W, int ZM>
static void spread_dispatch_z(const SpreadArgs& a, const KbParams& kb, size_t lds, int block, hipStream_t s) {
    const int CG = coil_group(a.C);
    if (CG == 4)
        spread_launch<D, W, 4, ZM>(a, kb, lds, block, s);
    else if (CG == 2)
        spread_launch<D, W, 2, ZM>(a, kb, lds, block, s);
    else
        spread_launch<D, W, 1, ZM>(a, kb, lds, block, s);
}

// tiles at most 4 cells deep along the last axis keep 4-cell register lines
template <int D, int W>
static void spread_dispatch(const SpreadArgs& a, const KbParams& kb, hipStream_t s) {
    const size_t lds = spread_lds_bytes(D, W, a.B, a.C, spread_zm(D, a.B));
    const int nthr = spread_threads(D, a.B, a.C);
    const int block = ((nthr + 63) / 64) * 64;
    if (block > 256) fail(KP_ERR_UNSUPPORTED, "spreading tile needs more than 256 threads");
    if (spread_zm(D, a.B) == 4)
        spread_dispatch_z<D, W, 4>(a, kb, lds, block, s);
    else
        spread_dispatch_z<D, W, kZMax>(a, kb, lds, block, s);
}

void launch_spread(int d, int W, const SpreadArgs& a, const KbParams& kb, hipStream_t s) {
    if (a.nwork <= 0) return;
#define KP_SPREAD_W(DD, WW) \
    if (d == DD && W == WW) return spread_dispatch<DD, WW>(a, kb, s);
    KP_SPREAD_W(2, 2) KP_SPREAD_W(2, 4) KP_SPREAD_W(2, 6) KP_SPREAD_W(2, 8)
    KP_SPREAD_W(3, 2) KP_SPREAD_W(3, 4) KP_SPREAD_W(3, 6) KP_SPREAD_W(3, 8)
#undef KP_SPREAD_W
    fail(KP_ERR_UNSUPPORTED, "spread: unsupported (d, W)");
}

}  // namespace kp
