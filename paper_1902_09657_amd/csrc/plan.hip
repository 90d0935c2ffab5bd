// Plan construction: canonical grid coordinates, bit-exact stable bin sort,
// tile touch lists, spreading work items, tables and workspaces; plus the
// NUFFT forward / adjoint drivers and their C ABI.
#include <cmath>
#include <complex>
#include <memory>
#include <cstring>
#include <mutex>
#include <algorithm>
#include <climits>

#include "kp_internal.h"

namespace kp {

// ------------------------------------------------------------------ errors
static thread_local std::string t_last_error;
void set_error(const std::string& msg) { t_last_error = msg; }

void DevBuf::alloc(size_t n) {
    release();
    if (n == 0) n = 256;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        fail(KP_ERR_OOM, "hipMalloc(" + std::to_string(n) + ") failed: " + hipGetErrorString(e));
    }
    bytes = n;
}
void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

// ------------------------------------------------------------- scan (int32)
constexpr int kScanBlock = 1024;

__global__ void __launch_bounds__(256) k_scan_blocks(const int* in, int* out, int64_t n, int* bsum) {
    __shared__ int sh[256];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + tid * 4;
    int v[4], e[4], s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        e[i] = s;
        s += v[i];
    }
    sh[tid] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int t = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    const int pre = tid > 0 ? sh[tid - 1] : 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (base + i < n) out[base + i] = e[i] + pre;
    if (tid == 255) bsum[blockIdx.x] = sh[255];
}

__global__ void k_add_offsets(int* out, int64_t n, const int* boff) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += boff[i / kScanBlock];
}

// exclusive scan of n ints (in may alias out)
static void scan_exclusive(const int* in, int* out, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    DevBuf bsum, bscan;
    bsum.alloc(sizeof(int) * (nb + 1));
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(256), 0, s, in, out, n, bsum.as<int>());
    KP_LAUNCH_CHECK();
    if (nb > 1) {
        bscan.alloc(sizeof(int) * (nb + 1));
        scan_exclusive(bsum.as<int>(), bscan.as<int>(), nb, s);
        hipLaunchKernelGGL(k_add_offsets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n,
                           bscan.as<int>());
        KP_LAUNCH_CHECK();
    }
    // keep the temporaries alive until the stream has used them
    KP_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------- stable LSD radix sort
constexpr int kRsThreads = 256, kRsItems = 8, kRsTile = kRsThreads * kRsItems;

__global__ void __launch_bounds__(256) k_rs_hist(const uint32_t* keys, int64_t n, int shift, int* hist,
                                                 int nblocks) {
    __shared__ int h[16];
    if (threadIdx.x < 16) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile + threadIdx.x * kRsItems;
    for (int i = 0; i < kRsItems; ++i)
        if (base + i < n) atomicAdd(&h[(keys[base + i] >> shift) & 15], 1);
    __syncthreads();
    if (threadIdx.x < 16) hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: thread t owns items [t*8, t*8+8) of the block's tile, so
// the rank of an item among equal digits follows its index.
__global__ void __launch_bounds__(256) k_rs_scatter(const uint32_t* kin, const int32_t* vin, uint32_t* kout,
                                                    int32_t* vout, int64_t n, int shift,
                                                    const int* hscan, int nblocks) {
    __shared__ int cnt[16 * kRsThreads];
    __shared__ int run[16 * kRsThreads];
    __shared__ int tot[kRsThreads];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kRsTile + t * kRsItems;
    for (int d = 0; d < 16; ++d) {
        cnt[d * kRsThreads + t] = 0;
        run[d * kRsThreads + t] = 0;
    }
    uint32_t k[kRsItems];
    int32_t v[kRsItems];
    for (int i = 0; i < kRsItems; ++i) {
        if (base + i < n) {
            k[i] = kin[base + i];
            v[i] = vin[base + i];
            cnt[((k[i] >> shift) & 15) * kRsThreads + t] += 1;
        }
    }
    __syncthreads();
    // exclusive scan of the flattened [digit][thread] count table
    int loc[16], s = 0;
    for (int j = 0; j < 16; ++j) {
        loc[j] = s;
        s += cnt[t * 16 + j];
    }
    tot[t] = s;
    __syncthreads();
    for (int off = 1; off < kRsThreads; off <<= 1) {
        int x = t >= off ? tot[t - off] : 0;
        __syncthreads();
        tot[t] += x;
        __syncthreads();
    }
    const int pre = t > 0 ? tot[t - 1] : 0;
    __syncthreads();
    for (int j = 0; j < 16; ++j) cnt[t * 16 + j] = loc[j] + pre;
    __syncthreads();
    for (int i = 0; i < kRsItems; ++i) {
        if (base + i < n) {
            const int d = (k[i] >> shift) & 15;
            const int r = cnt[d * kRsThreads + t] - cnt[d * kRsThreads] + run[d * kRsThreads + t];
            run[d * kRsThreads + t] += 1;
            const int64_t pos = (int64_t)hscan[d * nblocks + blockIdx.x] + r;
            kout[pos] = k[i];
            vout[pos] = v[i];
        }
    }
}

// Sort (keys, vals) by key, stably; result in keys/vals.
static void radix_sort_pairs(uint32_t* keys, int32_t* vals, int64_t n, uint32_t max_key, hipStream_t s) {
    if (n <= 1) return;
    int bits = 1;
    while (bits < 32 && (max_key >> bits) != 0) ++bits;
    const int passes = (bits + 3) / 4;
    const int nblocks = (int)((n + kRsTile - 1) / kRsTile);
    DevBuf k2, v2, hist;
    k2.alloc(sizeof(uint32_t) * n);
    v2.alloc(sizeof(int32_t) * n);
    hist.alloc(sizeof(int) * 16 * (int64_t)nblocks);
    uint32_t *ka = keys, *kb = k2.as<uint32_t>();
    int32_t *va = vals, *vb = v2.as<int32_t>();
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = 4 * ps;
        hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(kRsThreads), 0, s, ka, n, shift, hist.as<int>(), nblocks);
        KP_LAUNCH_CHECK();
        scan_exclusive(hist.as<int>(), hist.as<int>(), 16 * (int64_t)nblocks, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(kRsThreads), 0, s, ka, va, kb, vb, n, shift,
                           hist.as<int>(), nblocks);
        KP_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        KP_HIP(hipMemcpyAsync(keys, ka, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
        KP_HIP(hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    }
    KP_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------ plan-time kernels
struct Geom {
    int d;
    int G[3];
    float Gf[3];
    float half[3];
    float c[3];   // fl32(G / (2 pi))
    int B[3];
    int nb[3];
    int W;
};

// Canonical float32 grid coordinates; no contraction: every product and sum
// is rounded separately (round to nearest even).
__global__ void k_coords(const float* k, int64_t M, Geom gm, float* g, uint32_t* key, int* err) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= M) return;
    uint32_t kk = 0;
    for (int ax = 0; ax < gm.d; ++ax) {
        const float t = __fmul_rn(k[s * gm.d + ax], gm.c[ax]);
        float ga = __fadd_rn(t, gm.half[ax]);
        if (ga < 0.f) ga = __fadd_rn(ga, gm.Gf[ax]);
        if (ga >= gm.Gf[ax]) ga = __fsub_rn(ga, gm.Gf[ax]);
        if (!(ga >= 0.f && ga < gm.Gf[ax])) {
            atomicOr(err, 1);
            ga = 0.f;
        }
        g[s * gm.d + ax] = ga;
        const int cell = (int)floorf(ga);
        kk = kk * (uint32_t)gm.nb[ax] + (uint32_t)(cell / gm.B[ax]);
    }
    key[s] = kk;
}

__global__ void k_invert_perm(const int32_t* perm, int32_t* iperm, int64_t n) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) iperm[perm[s]] = (int32_t)s;
}

__global__ void k_iota(int32_t* v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

// Offsets of every key in a sorted key array: off[t] = number of keys < t
// for t = 0 .. nkeys.  Thread i (0 <= i <= n) writes the keys in
// (key[i-1], key[i]] (from 0 for i = 0, up to nkeys for i = n), so no two
// threads write one entry and no atomics are needed (a count with atomics
// serialises on the long runs of equal keys).
__global__ void k_sorted_offsets(const uint32_t* key, int64_t n, int64_t nkeys, int* off) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int64_t lo = i == 0 ? 0 : (int64_t)key[i - 1] + 1;
    const int64_t hi = i == n ? nkeys : (int64_t)key[i];
    for (int64_t t = lo; t <= hi; ++t) off[t] = (int)i;
}

__global__ void k_gather_coords(const float* g, const int32_t* perm, int64_t M, int d, float* gs) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= M) return;
    const int64_t i = perm[s];
    for (int ax = 0; ax < d; ++ax) gs[s * d + ax] = g[i * d + ax];
}

// distinct tiles met by the W taps of a sample on one axis
__device__ int axis_tiles(float g, const Geom& gm, int ax, int* tl) {
    const int cell = (int)floorf(g);
    int n = 0;
    for (int t = 0; t < gm.W; ++t) {
        int j = cell - gm.W / 2 + 1 + t;
        j = j < 0 ? j + gm.G[ax] : (j >= gm.G[ax] ? j - gm.G[ax] : j);
        const int tile = j / gm.B[ax];
        bool seen = false;
        for (int q = 0; q < n; ++q) seen |= (tl[q] == tile);
        if (!seen) tl[n++] = tile;
    }
    return n;
}

__global__ void k_touch_count(const float* gs, int64_t M, Geom gm, int* cnt) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= M) return;
    int tl[8];
    int prod = 1;
    for (int ax = 0; ax < gm.d; ++ax) prod *= axis_tiles(gs[s * gm.d + ax], gm, ax, tl);
    cnt[s] = prod;
}

__global__ void k_touch_emit(const float* gs, int64_t M, Geom gm, const int* off, uint32_t* keys,
                             int32_t* vals) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= M) return;
    int tl[3][8], n[3] = {1, 1, 1};
    for (int ax = 0; ax < gm.d; ++ax) n[ax] = axis_tiles(gs[s * gm.d + ax], gm, ax, tl[ax]);
    for (int ax = gm.d; ax < 3; ++ax) tl[ax][0] = 0;
    int pos = off[s];
    for (int a = 0; a < n[0]; ++a)
        for (int b = 0; b < n[1]; ++b)
            for (int c = 0; c < n[2]; ++c) {
                uint32_t key = (uint32_t)tl[0][a] * gm.nb[1] + tl[1][b];
                if (gm.d == 3) key = key * gm.nb[2] + tl[2][c];
                keys[pos] = key;
                vals[pos] = (int32_t)s;
                ++pos;
            }
}

// Spreading order: each chunk of kSpreadChunk touch entries (the unit the
// spreading kernel stages in LDS) is stably sorted by the bucket of its
// entries' first tap on the leading axes, counted from -(W-1).  One block per
// chunk = (tile, first entry, count).
__global__ void __launch_bounds__(kSpreadChunk) k_chunk_order(const float* gs, const int32_t* touch,
                                                              const int4* chunks, Geom gm, int32_t* stouch,
                                                              uint16_t* scode) {
    __shared__ int bk_of[kSpreadChunk];
    __shared__ int cnt[512];
    const int4 ch = chunks[blockIdx.x];
    const int tile = ch.x, start = ch.y, n = ch.z;
    const int e = threadIdx.x;
    int tc[3], rem = tile;
    for (int ax = gm.d - 1; ax >= 0; --ax) {
        tc[ax] = rem % gm.nb[ax];
        rem /= gm.nb[ax];
    }
    const int NB1 = gm.d == 3 ? gm.B[1] + gm.W - 1 : 1;
    int bk = 0, s = 0;
    if (e < n) {
        s = touch[start + e];
        for (int ax = 0; ax < gm.d - 1; ++ax) {
            const int cell = (int)floorf(gs[(int64_t)s * gm.d + ax]);
            int l = cell - gm.W / 2 + 1 - tc[ax] * gm.B[ax];
            if (l < -(gm.W - 1)) l += gm.G[ax];
            else if (l > gm.B[ax] - 1) l -= gm.G[ax];
            bk = ax == 0 ? l + gm.W - 1 : bk * NB1 + (l + gm.W - 1);
        }
        bk_of[e] = bk;
    }
    for (int b = e; b < 512; b += blockDim.x) cnt[b] = 0;
    __syncthreads();
    if (e < n) atomicAdd(&cnt[bk], 1);
    __syncthreads();
    if (e == 0) {
        int run = 0;
        for (int b = 0; b < 512; ++b) {
            const int c = cnt[b];
            cnt[b] = run;
            run += c;
        }
    }
    __syncthreads();
    if (e < n) {
        int pos = cnt[bk];
        for (int q = 0; q < e; ++q) pos += bk_of[q] == bk;  // stable
        stouch[start + pos] = s;
        scode[start + pos] = (uint16_t)bk;
    }
}

// Spreading order of a whole work item (tile or piece of a split tile, at
// most kItemOrderMax entries): the entries are dealt to the item's chunks by
// their rank within their bucket (the first entry of every bucket, then the
// second of every bucket, ...), so every chunk draws evenly from all buckets
// and the owner threads of the spreading kernel get runs of similar length;
// each chunk is then stably sorted by bucket.  Ranks follow the canonical
// (ascending sample position) order, so the result is deterministic.
constexpr int kItemOrderMax = 4096;

__device__ int entry_bucket(const float* gs, int s, int tc0, int tc1, const Geom& gm) {
    const int NB1 = gm.d == 3 ? gm.B[1] + gm.W - 1 : 1;
    int bk = 0;
    for (int ax = 0; ax < gm.d - 1; ++ax) {
        const int cell = (int)floorf(gs[(int64_t)s * gm.d + ax]);
        int l = cell - gm.W / 2 + 1 - (ax == 0 ? tc0 : tc1) * gm.B[ax];
        if (l < -(gm.W - 1)) l += gm.G[ax];
        else if (l > gm.B[ax] - 1) l -= gm.G[ax];
        bk = ax == 0 ? l + gm.W - 1 : bk * NB1 + (l + gm.W - 1);
    }
    return bk;
}

__global__ void __launch_bounds__(256) k_item_order(const float* gs, const int32_t* touch, const int4* items,
                                                    Geom gm, int32_t* stouch, uint16_t* scode) {
    __shared__ int cnt[512];
    __shared__ int bk_of[kItemOrderMax];   // canonical order
    __shared__ int s_il[kItemOrderMax];    // interleaved order
    __shared__ uint16_t b_il[kItemOrderMax];
    const int4 it = items[blockIdx.x];
    const int tile = it.x, start = it.y, n = it.z;
    int tc[3] = {0, 0, 0}, rem = tile;
    for (int ax = gm.d - 1; ax >= 0; --ax) {
        tc[ax] = rem % gm.nb[ax];
        rem /= gm.nb[ax];
    }
    const int nbk = gm.d == 3 ? (gm.B[0] + gm.W - 1) * (gm.B[1] + gm.W - 1) : gm.B[0] + gm.W - 1;
    for (int b = threadIdx.x; b < 512; b += blockDim.x) cnt[b] = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int bk = entry_bucket(gs, touch[start + e], tc[0], tc[1], gm);
        bk_of[e] = bk;
        atomicAdd(&cnt[bk], 1);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int bk = bk_of[e];
        int rank = 0;  // earlier entries of the same bucket
        for (int q = 0; q < e; ++q) rank += bk_of[q] == bk;
        // position in (rank, bucket) order
        int ip = 0;
        for (int b = 0; b < nbk; ++b) {
            const int c = cnt[b];
            ip += min(c, rank) + (b < bk && c > rank ? 1 : 0);
        }
        s_il[ip] = touch[start + e];
        b_il[ip] = (uint16_t)bk;
    }
    __syncthreads();
    for (int ip = threadIdx.x; ip < n; ip += blockDim.x) {
        const int c0 = ip - ip % kSpreadChunk, c1 = min(n, c0 + kSpreadChunk);
        const int bk = b_il[ip];
        int pos = c0;
        for (int q = c0; q < c1; ++q) {
            const int bq = b_il[q];
            pos += (bq < bk || (bq == bk && q < ip)) ? 1 : 0;
        }
        stouch[start + pos] = s_il[ip];
        scode[start + pos] = (uint16_t)bk;
    }
}

__global__ void k_maps_transpose(const float2* src, int64_t N, int C, float2* dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * C) return;
    const int64_t n = i / C;
    const int c = (int)(i % C);
    dst[i] = src[(int64_t)c * N + n];
}

__global__ void k_fill_c(float2* dst, int64_t n, float2 v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = v;
}

__global__ void k_zero_tiles(float2* grid, const int* tiles, int ntiles, int d, Geom gm, int C) {
    const int tile = tiles[blockIdx.x];
    int tc[3] = {0, 0, 0};
    int rem = tile;
    for (int ax = d - 1; ax >= 0; --ax) {
        tc[ax] = rem % gm.nb[ax];
        rem /= gm.nb[ax];
    }
    const int Bt = gm.B[0] * gm.B[1] * (d == 3 ? gm.B[2] : 1);
    for (int i = threadIdx.x; i < Bt * C; i += blockDim.x) {
        const int l = i / C, c = i % C;
        int64_t gidx;
        if (d == 2) {
            gidx = (int64_t)(tc[0] * gm.B[0] + l / gm.B[1]) * gm.G[1] + tc[1] * gm.B[1] + l % gm.B[1];
        } else {
            const int l2 = l % gm.B[2], l01 = l / gm.B[2];
            gidx = ((int64_t)(tc[0] * gm.B[0] + l01 / gm.B[1]) * gm.G[1] + tc[1] * gm.B[1] + l01 % gm.B[1]) *
                       gm.G[2] +
                   tc[2] * gm.B[2] + l2;
        }
        grid[gidx * C + c] = make_float2(0.f, 0.f);
    }
}

static unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// --------------------------------------------------------------- helpers
static bool smooth5_even(int64_t g) {
    if (g <= 0 || g % 2) return false;
    for (int p : {2, 3, 5})
        while (g % p == 0) g /= p;
    return g == 1;
}

static int next_smooth_even(int64_t n) {
    int64_t m = std::max<int64_t>(2, n);
    while (!smooth5_even(m)) ++m;
    return (int)m;
}

static double kb_ft_host(double nu, int W, double beta) {
    const double z2 = beta * beta - (M_PI * W * nu) * (M_PI * W * nu);
    if (z2 > 0) {
        const double z = std::sqrt(z2);
        return z == 0 ? 1.0 : std::sinh(z) / z;
    }
    const double z = std::sqrt(-z2);
    return z == 0 ? 1.0 : std::sin(z) / z;
}

static Geom make_geom(const Plan& P, bool spreading = false) {
    Geom gm{};
    gm.d = P.d;
    gm.W = P.W;
    for (int a = 0; a < 3; ++a) {
        gm.G[a] = P.G[a];
        gm.Gf[a] = (float)P.G[a];
        gm.half[a] = (float)(P.G[a] / 2);
        gm.c[a] = (float)((double)P.G[a] / (2.0 * M_PI));
        gm.B[a] = spreading ? P.Bs[a] : P.B[a];
        gm.nb[a] = spreading ? P.nbs[a] : P.nb[a];
    }
    return gm;
}

void validate_plan_args(int ndim, const int64_t* shape, int64_t ncoils, int64_t nsamples,
                        const void* coords, const void* maps, float oversamp, int kb_width,
                        const kp_tuning* tuning, bool channel_mode) {
    if (ndim != 2 && ndim != 3) fail(KP_ERR_INVALID_ARG, "ndim must be 2 or 3");
    if (!shape) fail(KP_ERR_INVALID_ARG, "shape is NULL");
    for (int a = 0; a < ndim; ++a) {
        if (shape[a] < 2 || shape[a] > 4096) fail(KP_ERR_INVALID_ARG, "every N_a must lie in [2, 4096]");
        if (shape[a] % 2) fail(KP_ERR_INVALID_ARG, "every N_a must be even");
    }
    if (ncoils < 1) fail(KP_ERR_INVALID_ARG, "ncoils must be >= 1");
    if (ncoils > 16) fail(KP_ERR_UNSUPPORTED, "at most 16 coils are supported");
    if (nsamples < 1) fail(KP_ERR_INVALID_ARG, "nsamples must be >= 1");
    if (nsamples >= (int64_t)1 << 27) fail(KP_ERR_UNSUPPORTED, "nsamples must be < 2^27");
    if (!coords) fail(KP_ERR_INVALID_ARG, "coords is NULL");
    if (!maps && ncoils != 1 && !channel_mode) fail(KP_ERR_INVALID_ARG, "maps == NULL requires ncoils == 1");
    if (!(oversamp >= 1.25f && oversamp <= 2.0f)) fail(KP_ERR_INVALID_ARG, "oversamp must lie in [1.25, 2]");
    if (kb_width != 2 && kb_width != 4 && kb_width != 6 && kb_width != 8)
        fail(KP_ERR_INVALID_ARG, "kb_width must be 2, 4, 6 or 8");
    int64_t gtot = 1;
    for (int a = 0; a < ndim; ++a) {
        const int g = next_smooth_even((int64_t)std::ceil((double)oversamp * (double)shape[a]));
        if (g < kb_width) fail(KP_ERR_UNSUPPORTED, "grid smaller than the kernel width");
        gtot *= g;
        if (tuning && tuning->bin_size[a] > 0 && g % tuning->bin_size[a] != 0)
            fail(KP_ERR_INVALID_ARG, "tuning.bin_size must divide the grid size");
    }
    if (gtot * ncoils >= ((int64_t)1 << 31)) fail(KP_ERR_UNSUPPORTED, "grid x coils must be < 2^31 elements");
    if (tuning && tuning->max_chunk < 0) fail(KP_ERR_INVALID_ARG, "tuning.max_chunk must be >= 0");
}

static int pick_bin(int G, int target) {
    int best = 1;
    for (int b = 1; b <= G; ++b)
        if (G % b == 0 && b <= target) best = b;
    return best;
}

static void set_lds_limit(const void* fn, int bytes) {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipGetLastError();
}

Plan* create_plan(int ndim, const int64_t* shape, int64_t ncoils, int64_t nsamples, const float* coords,
                  const void* maps, float oversamp, int kb_width, const kp_tuning* tuning, hipStream_t s,
                  bool channel_mode) {
    validate_plan_args(ndim, shape, ncoils, nsamples, coords, maps, oversamp, kb_width, tuning, channel_mode);
    auto P = std::make_unique<Plan>();
    P->d = ndim;
    P->C = ncoils;
    P->M = nsamples;
    P->W = kb_width;
    P->alpha = oversamp;
    P->stream = s;
    P->Ntot = 1;
    P->Gtot = 1;
    for (int a = 0; a < ndim; ++a) {
        P->N[a] = shape[a];
        P->G[a] = next_smooth_even((int64_t)std::ceil((double)oversamp * (double)shape[a]));
        P->Ntot *= P->N[a];
        P->Gtot *= P->G[a];
    }
    const double a = (double)oversamp, w = (double)kb_width;
    P->beta = M_PI * std::sqrt((w / a) * (w / a) * (a - 0.5) * (a - 0.5) - 0.8);
    kb_fit(P->beta, kb_width, &P->kb);

    int dev = 0;
    KP_HIP(hipGetDevice(&dev));
    P->dev = dev;
    hipDeviceProp_t prop;
    KP_HIP(hipGetDeviceProperties(&prop, dev));
    P->lds_max = (int)std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);

    // tiles: the last axis at most kZMax cells (one register line per owner
    // thread); 3D leading axes 8 x 8, 2D leading axis up to 64 lines, within
    // 256 threads; every B_a divides G_a and leaves G_a >= B_a + W - 1.  The
    // spreading tiles are 4 cells deep along the last axis by default (a
    // 4-cell register line wastes fewer zero-weight taps), the sort tiles 8.
    const int C = (int)ncoils;
    const int CG = C % 4 == 0 ? 4 : (C % 2 == 0 ? 2 : 1);
    const int ncg = C / CG;
    for (int ax = 0; ax < 3; ++ax) {
        if (ax >= ndim) {
            P->B[ax] = P->Bs[ax] = 1;
            P->nb[ax] = P->nbs[ax] = 1;
            continue;
        }
        const int cap = std::max(1, P->G[ax] - kb_width + 1);
        int target;
        if (ax == ndim - 1)
            target = kZMax;
        else if (ndim == 3)
            target = 8;
        else
            target = std::max(1, std::min(64, 256 / ncg));
        int b = (tuning && tuning->bin_size[ax] > 0) ? tuning->bin_size[ax] : pick_bin(P->G[ax], std::min(target, cap));
        if (b > cap) fail(KP_ERR_INVALID_ARG, "tuning.bin_size must leave G_a >= bin + W - 1");
        if (ax == ndim - 1 && b > kZMax) fail(KP_ERR_INVALID_ARG, "tuning.bin_size on the last axis must be <= 8");
        P->B[ax] = b;
        P->nb[ax] = P->G[ax] / b;
        int bs;
        if (tuning && tuning->spread_bin_size[ax] > 0)
            bs = tuning->spread_bin_size[ax];
        else if (tuning && tuning->bin_size[ax] > 0)
            bs = b;
        else if (ax == ndim - 1)
            bs = pick_bin(P->G[ax], std::min(4, cap));
        else
            bs = b;
        if (bs > cap) fail(KP_ERR_INVALID_ARG, "tuning.spread_bin_size must leave G_a >= bin + W - 1");
        if (P->G[ax] % bs) fail(KP_ERR_INVALID_ARG, "tuning.spread_bin_size must divide the grid size");
        if (ax == ndim - 1 && bs > kZMax) fail(KP_ERR_INVALID_ARG, "tuning.spread_bin_size on the last axis must be <= 8");
        P->Bs[ax] = bs;
        P->nbs[ax] = P->G[ax] / bs;
    }
    P->nbins = (int64_t)P->nb[0] * P->nb[1] * P->nb[2];
    P->nstiles = (int64_t)P->nbs[0] * P->nbs[1] * P->nbs[2];
    if (spread_threads(ndim, P->Bs, C) > 256) fail(KP_ERR_INVALID_ARG, "spreading tiles need more than 256 threads");
    // the spreading kernel keeps a signed 16-bit LDS byte offset per entry for
    // its axis-1 weight: 4 (B_1 + W - 2)(chunk + 1) must stay below 2^15
    if (ndim == 3 && 4 * (P->Bs[1] + kb_width - 2) * (kSpreadChunk + 1) > 32767)
        fail(KP_ERR_UNSUPPORTED, "spreading tiles longer than 64 - W cells on axis 1 are not supported");
    P->spread_lds = (int)spread_lds_bytes(ndim, kb_width, P->Bs, C);
    if (P->spread_lds > P->lds_max) fail(KP_ERR_UNSUPPORTED, "spreading chunk does not fit in LDS");
    if (P->nbins >= ((int64_t)1 << 31) || P->nstiles >= ((int64_t)1 << 31)) fail(KP_ERR_UNSUPPORTED, "too many tiles");
    int max_chunk = (tuning && tuning->max_chunk > 0) ? tuning->max_chunk : 0;  // 0: chosen below

    const int64_t M = nsamples;
    const int d = ndim;
    Geom gm = make_geom(*P);
    const Geom gms = make_geom(*P, true);

    // ---- canonical coordinates and bin keys
    P->coords.alloc(sizeof(float) * M * d);
    KP_HIP(hipMemcpyAsync(P->coords.p, coords, sizeof(float) * M * d, hipMemcpyDeviceToDevice, s));
    P->g_orig.alloc(sizeof(float) * M * d);
    DevBuf keys, err;
    keys.alloc(sizeof(uint32_t) * M);
    err.alloc(sizeof(int));
    KP_HIP(hipMemsetAsync(err.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_coords, dim3(nblk(M)), dim3(256), 0, s, coords, M, gm, P->g_orig.as<float>(),
                       keys.as<uint32_t>(), err.as<int>());
    KP_LAUNCH_CHECK();
    int herr = 0;
    KP_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
    KP_HIP(hipStreamSynchronize(s));
    if (herr) fail(KP_ERR_INVALID_ARG, "coordinate out of range (|omega| beyond ~3 pi, NaN or inf)");

    // ---- stable sort of samples by tile
    P->perm.alloc(sizeof(int32_t) * M);
    hipLaunchKernelGGL(k_iota, dim3(nblk(M)), dim3(256), 0, s, P->perm.as<int32_t>(), M);
    KP_LAUNCH_CHECK();
    radix_sort_pairs(keys.as<uint32_t>(), P->perm.as<int32_t>(), M, (uint32_t)(P->nbins - 1), s);
    P->bin_off.alloc(sizeof(int) * (P->nbins + 1));
    hipLaunchKernelGGL(k_sorted_offsets, dim3(nblk(M + 1)), dim3(256), 0, s, keys.as<uint32_t>(), M, P->nbins,
                       P->bin_off.as<int>());
    KP_LAUNCH_CHECK();
    P->g_sorted.alloc(sizeof(float) * M * d);
    hipLaunchKernelGGL(k_gather_coords, dim3(nblk(M)), dim3(256), 0, s, P->g_orig.as<float>(),
                       P->perm.as<int32_t>(), M, d, P->g_sorted.as<float>());
    KP_LAUNCH_CHECK();
    P->iperm.alloc(sizeof(int32_t) * M);
    hipLaunchKernelGGL(k_invert_perm, dim3(nblk(M)), dim3(256), 0, s, P->perm.as<int32_t>(), P->iperm.as<int32_t>(), M);
    KP_LAUNCH_CHECK();

    // ---- tile touch lists
    DevBuf tcnt;
    tcnt.alloc(sizeof(int) * (M + 1));
    KP_HIP(hipMemsetAsync(tcnt.p, 0, sizeof(int) * (M + 1), s));
    hipLaunchKernelGGL(k_touch_count, dim3(nblk(M)), dim3(256), 0, s, P->g_sorted.as<float>(), M, gms,
                       tcnt.as<int>());
    KP_LAUNCH_CHECK();
    scan_exclusive(tcnt.as<int>(), tcnt.as<int>(), M + 1, s);
    int ntouch = 0;
    KP_HIP(hipMemcpyAsync(&ntouch, tcnt.as<int>() + M, sizeof(int), hipMemcpyDeviceToHost, s));
    KP_HIP(hipStreamSynchronize(s));
    P->ntouch = ntouch;
    DevBuf tkeys;
    tkeys.alloc(sizeof(uint32_t) * std::max(ntouch, 1));
    P->touch.alloc(sizeof(int32_t) * std::max(ntouch, 1));
    hipLaunchKernelGGL(k_touch_emit, dim3(nblk(M)), dim3(256), 0, s, P->g_sorted.as<float>(), M, gms,
                       tcnt.as<int>(), tkeys.as<uint32_t>(), P->touch.as<int32_t>());
    KP_LAUNCH_CHECK();
    radix_sort_pairs(tkeys.as<uint32_t>(), P->touch.as<int32_t>(), ntouch, (uint32_t)(P->nstiles - 1), s);
    P->touch_off.alloc(sizeof(int) * (P->nstiles + 1));
    hipLaunchKernelGGL(k_sorted_offsets, dim3(nblk((int64_t)ntouch + 1)), dim3(256), 0, s, tkeys.as<uint32_t>(),
                       (int64_t)ntouch, P->nstiles, P->touch_off.as<int>());
    KP_LAUNCH_CHECK();

    // ---- spreading work items (host): heavy tiles split, largest work first
    std::vector<int> toff(P->nstiles + 1);
    KP_HIP(hipMemcpyAsync(toff.data(), P->touch_off.p, sizeof(int) * (P->nstiles + 1), hipMemcpyDeviceToHost, s));
    KP_HIP(hipStreamSynchronize(s));
    // A tile with more entries than max_chunk is split; each piece gets a
    // partial-tile slot.  Work items run longest first (split pieces, then
    // owned tiles by decreasing entry count): the density of a radial
    // trajectory is concentrated in a few tiles, and this order keeps every
    // compute unit busy to the end.
    // 3D support pruning: per spreading tile column (ty, tz) the axis-0 cell
    // range holding its non-empty tiles.  Empty tiles outside these ranges are
    // then never written: the last forward FFT pass stores only the ranges
    // (interpolation reads nothing else) and the first adjoint pass takes the
    // rows outside them as zero.
    // It needs the specialised FFT kernel for the axis-0 passes (32 columns).
    // (G_1 G_2 >= 32: an axis-0 pass always has 32 columns per block)
    const bool prune = d == 3 && (int64_t)P->G[1] * P->G[2] >= 32 && fft_fixed_ok(P->G[0], 32);
    std::vector<char> skip;  // empty tiles outside their column's range
    if (prune) {
        const int nb1 = P->nbs[1], nb2 = P->nbs[2];
        std::vector<int2> xr((size_t)nb1 * nb2, make_int2(INT_MAX, 0));
        for (int64_t t = 0; t < P->nstiles; ++t) {
            if (toff[t + 1] == toff[t]) continue;
            const int tz = (int)(t % nb2), ty = (int)((t / nb2) % nb1), tx = (int)(t / ((int64_t)nb1 * nb2));
            int2& r = xr[(size_t)ty * nb2 + tz];
            r.x = std::min(r.x, tx * P->Bs[0]);
            r.y = std::max(r.y, (tx + 1) * P->Bs[0]);
        }
        for (int2& r : xr)
            if (r.y <= r.x) r = make_int2(0, 0);
        P->xrange.alloc(sizeof(int2) * xr.size());
        KP_HIP(hipMemcpy(P->xrange.p, xr.data(), sizeof(int2) * xr.size(), hipMemcpyHostToDevice));
        // per tz the axis-1 range of the tile columns that hold a non-empty
        // tile (the columns outside it are empty: zero in the adjoint, unused
        // in the forward direction)
        std::vector<int2> yr((size_t)nb2, make_int2(0, 0));
        for (int tz = 0; tz < nb2; ++tz) {
            int lo = INT_MAX, hi = 0;
            for (int ty = 0; ty < nb1; ++ty) {
                const int2 r = xr[(size_t)ty * nb2 + tz];
                if (r.y > r.x) {
                    lo = std::min(lo, ty * P->Bs[1]);
                    hi = std::max(hi, (ty + 1) * P->Bs[1]);
                }
            }
            if (hi > lo) yr[(size_t)tz] = make_int2(lo, hi);
        }
        P->yrange.alloc(sizeof(int2) * yr.size());
        KP_HIP(hipMemcpy(P->yrange.p, yr.data(), sizeof(int2) * yr.size(), hipMemcpyHostToDevice));
        // an empty tile inside its column's range is still written (zeros):
        // the first adjoint pass reads the whole range
        skip.assign((size_t)P->nstiles, 0);
        for (int64_t t = 0; t < P->nstiles; ++t) {
            if (toff[t + 1] != toff[t]) continue;
            const int tz = (int)(t % nb2), ty = (int)((t / nb2) % nb1), tx = (int)(t / ((int64_t)nb1 * nb2));
            const int2 r = xr[(size_t)ty * nb2 + tz];
            skip[t] = (tx * P->Bs[0] >= r.y || (tx + 1) * P->Bs[0] <= r.x) ? 1 : 0;
        }
    }
    // Built-in split size: 1024 entries when the plan has work for thousands
    // of such items, halved down to half a chunk otherwise.  A small plan (a
    // 2D slice) has too few tiles to fill the GPU, so its time is the longest
    // work item's gathers, and in the dense k-space centre all of an item's
    // entries reach the same few lines of its tile; a large one (3D) is
    // throughput bound, where fewer, longer items cost fewer partial tiles.
    if (max_chunk == 0) {
        const int64_t entries = toff[P->nstiles];
        max_chunk = 1024;
        while (max_chunk > kSpreadChunk / 2 && entries < (int64_t)4096 * max_chunk) max_chunk /= 2;
    }
    P->max_chunk = max_chunk;
    std::vector<int4> heavy_items, light_items;
    std::vector<int4> heavy;  // (tile, first slot, slots, 0)
    int nslots = 0;
    for (int64_t t = 0; t < P->nstiles; ++t) {
        const int o = toff[t], n = toff[t + 1] - toff[t];
        if (prune && skip[t]) continue;  // an empty tile outside the range: never read
        if (n <= max_chunk) {
            light_items.push_back(make_int4((int)t, o, n, -1));
        } else {
            const int first = nslots;
            for (int q = 0; q < n; q += max_chunk)
                heavy_items.push_back(make_int4((int)t, o + q, std::min(max_chunk, n - q), nslots++));
            heavy.push_back(make_int4((int)t, first, nslots - first, 0));
        }
    }
    std::stable_sort(light_items.begin(), light_items.end(), [](const int4& x, const int4& y) { return x.z > y.z; });

    // ---- interpolation pieces: the sorted samples of each non-empty tile in
    // runs of at most kInterpPiece, largest first
    P->interp_tiles = interp_tile_lds_bytes(d, kb_width, P->B, C) <= kInterpTileLds;
    if (P->interp_tiles) {
        std::vector<int> boff(P->nbins + 1);
        KP_HIP(hipMemcpy(boff.data(), P->bin_off.p, sizeof(int) * (P->nbins + 1), hipMemcpyDeviceToHost));
        std::vector<int4> pieces;
        for (int64_t t = 0; t < P->nbins; ++t)
            for (int q = boff[t]; q < boff[t + 1]; q += kInterpPiece)
                pieces.push_back(make_int4((int)t, q, std::min(kInterpPiece, boff[t + 1] - q), 0));
        std::stable_sort(pieces.begin(), pieces.end(), [](const int4& x, const int4& y) { return x.z > y.z; });
        P->niwork = (int64_t)pieces.size();
        P->iwork.alloc(sizeof(int4) * std::max<size_t>(pieces.size(), 1));
        if (!pieces.empty())
            KP_HIP(hipMemcpy(P->iwork.p, pieces.data(), sizeof(int4) * pieces.size(), hipMemcpyHostToDevice));
    }
    std::vector<int4> items(heavy_items);
    items.insert(items.end(), light_items.begin(), light_items.end());
    P->nwork = (int64_t)items.size();

    // ---- spreading order of the entries inside every chunk of every item
    {
        if (spread_nbk(d, kb_width, P->Bs) > 512) fail(KP_ERR_UNSUPPORTED, "too many tile buckets");
        // items of at most kItemOrderMax entries are interleaved over their
        // chunks; larger ones (only with a max_chunk above it) keep their
        // chunks of consecutive entries
        std::vector<int4> chunks, whole;
        for (const int4& it : items) {
            if (it.z <= 0) continue;
            if (it.z <= kItemOrderMax) {
                whole.push_back(it);
                continue;
            }
            for (int q = 0; q < it.z; q += kSpreadChunk)
                chunks.push_back(make_int4(it.x, it.y + q, std::min(kSpreadChunk, it.z - q), 0));
        }
        P->stouch.alloc(sizeof(int32_t) * std::max(ntouch, 1));
        P->scode.alloc(sizeof(uint16_t) * std::max(ntouch, 1));
        if (!whole.empty()) {
            DevBuf dit;
            dit.alloc(sizeof(int4) * whole.size());
            KP_HIP(hipMemcpy(dit.p, whole.data(), sizeof(int4) * whole.size(), hipMemcpyHostToDevice));
            hipLaunchKernelGGL(k_item_order, dim3((unsigned)whole.size()), dim3(256), 0, s, P->g_sorted.as<float>(),
                               P->touch.as<int32_t>(), dit.as<int4>(), gms, P->stouch.as<int32_t>(),
                               P->scode.as<uint16_t>());
            KP_LAUNCH_CHECK();
            KP_HIP(hipStreamSynchronize(s));
        }
        if (!chunks.empty()) {
            DevBuf dch;
            dch.alloc(sizeof(int4) * chunks.size());
            KP_HIP(hipMemcpy(dch.p, chunks.data(), sizeof(int4) * chunks.size(), hipMemcpyHostToDevice));
            hipLaunchKernelGGL(k_chunk_order, dim3((unsigned)chunks.size()), dim3(kSpreadChunk), 0, s,
                               P->g_sorted.as<float>(), P->touch.as<int32_t>(), dch.as<int4>(), gms,
                               P->stouch.as<int32_t>(), P->scode.as<uint16_t>());
            KP_LAUNCH_CHECK();
            KP_HIP(hipStreamSynchronize(s));
        }
    }
    P->heavy_tiles = (int64_t)heavy.size();
    P->nslots = nslots;
    P->work.alloc(sizeof(int4) * items.size());
    KP_HIP(hipMemcpy(P->work.p, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice));
    // tiles with the most slots first: their reductions are the longest
    std::stable_sort(heavy.begin(), heavy.end(), [](const int4& x, const int4& y) { return x.z > y.z; });
    P->heavy_list.alloc(sizeof(int4) * std::max<size_t>(heavy.size(), 1));
    if (!heavy.empty())
        KP_HIP(hipMemcpy(P->heavy_list.p, heavy.data(), sizeof(int4) * heavy.size(), hipMemcpyHostToDevice));
    P->partial.alloc(sizeof(float2) * std::max<int64_t>(1, (int64_t)nslots * P->Bs[0] * P->Bs[1] * P->Bs[2] * C));

    // ---- coil maps, stored [N][C]; unit maps for a single coil without maps
    P->has_maps = maps != nullptr;
    P->maps.alloc(sizeof(float2) * P->Ntot * C);
    if (maps && !channel_mode) {
        hipLaunchKernelGGL(k_maps_transpose, dim3(nblk(P->Ntot * C)), dim3(256), 0, s, (const float2*)maps, P->Ntot,
                           C, P->maps.as<float2>());
    } else {
        hipLaunchKernelGGL(k_fill_c, dim3(nblk(P->Ntot * C)), dim3(256), 0, s, P->maps.as<float2>(), P->Ntot * C,
                           make_float2(1.f, 0.f));
    }
    KP_LAUNCH_CHECK();

    // ---- deapodisation factors: f_a[m] = (-1)^n / Chat(n / G_a), n = m - N_a/2;
    // 1/sqrt(N) folded into axis 0; fo = product over the leading axes
    std::vector<std::vector<double>> f(d);
    for (int ax = 0; ax < d; ++ax) {
        f[ax].resize(P->N[ax]);
        for (int64_t m = 0; m < P->N[ax]; ++m) {
            const int64_t n = m - P->N[ax] / 2;
            const double sign = (std::llabs(n) % 2) ? -1.0 : 1.0;
            f[ax][m] = sign / kb_ft_host((double)n / P->G[ax], P->W, P->beta);
        }
    }
    for (auto& v : f[0]) v /= std::sqrt((double)P->Ntot);
    const int64_t O = P->Ntot / P->N[d - 1];
    std::vector<float> fo(O), fr(P->N[d - 1]);
    for (int64_t o = 0; o < O; ++o) {
        if (d == 2) {
            fo[o] = (float)f[0][o];
        } else {
            fo[o] = (float)(f[0][o / P->N[1]] * f[1][o % P->N[1]]);
        }
    }
    for (int64_t m = 0; m < P->N[d - 1]; ++m) fr[m] = (float)f[d - 1][m];
    P->fo_fwd.alloc(sizeof(float) * O);
    P->fr_fwd.alloc(sizeof(float) * fr.size());
    KP_HIP(hipMemcpy(P->fo_fwd.p, fo.data(), sizeof(float) * O, hipMemcpyHostToDevice));
    KP_HIP(hipMemcpy(P->fr_fwd.p, fr.data(), sizeof(float) * fr.size(), hipMemcpyHostToDevice));

    // ---- twiddles per axis
    for (int ax = 0; ax < d; ++ax) {
        const int L = P->G[ax];
        fft_twiddles(L, P->tw[ax]);
        int nst = 0, rad[kMaxStages];
        fft_factor(L, &nst, rad);
        P->fft_nst[ax].assign(1, nst);
        P->fft_rad[ax].assign(rad, rad + nst);
    }

    // ---- workspaces
    P->bufA.alloc(sizeof(float2) * P->Gtot * C);
    P->bufB.alloc(sizeof(float2) * P->Gtot * C);
    P->kint.alloc(sizeof(float2) * M * C);
    P->kint2.alloc(sizeof(float2) * M * C);
    P->kint3.alloc(sizeof(float2) * M * C);
    P->pint.alloc(sizeof(float) * M * C);
    for (auto& b : P->img) b.alloc(sizeof(float2) * P->Ntot * (channel_mode ? C : 1));
    if (!channel_mode) {
        P->tvv.alloc(sizeof(float2) * P->Ntot * ndim);
        P->kint4.alloc(sizeof(float2) * M * C);
    }
    P->red.alloc(sizeof(double) * 65536);
    P->sched.alloc(sizeof(float) * (3 * 8192 + 64));
    KP_HIP(hipStreamSynchronize(s));

    int64_t total = 0;
    for (DevBuf* b : {&P->partial, &P->coords, &P->g_sorted, &P->g_orig, &P->perm, &P->iperm, &P->bin_off, &P->xrange, &P->yrange, &P->touch_off, &P->touch, &P->work,
                      &P->heavy_list, &P->maps, &P->fo_fwd, &P->fr_fwd, &P->bufA, &P->bufB, &P->kint, &P->kint2, &P->kint3,
                      &P->pint, &P->red, &P->sched, &P->tvv, &P->kint4})
        total += (int64_t)b->bytes;
    for (auto& b : P->img) total += (int64_t)b.bytes;
    for (auto& b : P->tw) total += (int64_t)b.bytes;
    P->bytes = total;
    return P.release();
}

// ------------------------------------------------------------ operators
void fft_twiddles(int L, DevBuf& twb) {
    std::vector<float2> tw(L);
    for (int m = 0; m < L; ++m) {
        const double ang = -2.0 * M_PI * (double)m / (double)L;
        tw[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    twb.alloc(sizeof(float2) * L);
    KP_HIP(hipMemcpy(twb.p, tw.data(), sizeof(float2) * L, hipMemcpyHostToDevice));
}

void pass_blocking(int64_t I, int* Ob, int* Ib) {
    if (I >= 32) {
        *Ib = 32;
        *Ob = 1;
    } else if (I >= 16) {
        *Ib = 16;
        *Ob = 1;
    } else {
        *Ib = (int)I;
        *Ob = std::max<int>(1, 8 / (int)I);  // short inner axis (the coils): 8 columns
    }
}

static void fill_stages(const Plan& P, int ax, FftPass& fp) {
    fp.nst = P.fft_nst[ax][0];
    for (int i = 0; i < fp.nst; ++i) fp.rad[i] = P.fft_rad[ax][i];
    fp.tw = P.tw[ax].as<float2>();
}

// support pruning of an axis-0 pass over [G0][G1][G2][C] (mode 1: stores,
// mode 2: loads); the y-range pruning of the axis-0 and axis-1 passes
// (yr_mode, see FftPass)
static void set_xrange(const Plan& P, int C, int mode, FftPass& fp) {
    fp.xr = P.xrange.as<int2>();
    fp.xr_mode = mode;
    fp.xr_G2C = P.G[2] * C;
    fp.xr_C = C;
    fp.xr_B1 = P.Bs[1];
    fp.xr_B2 = P.Bs[2];
    fp.xr_nb2 = P.nbs[2];
}
static void set_yrange(const Plan& P, int C, int mode, FftPass& fp) {
    fp.yr = P.yrange.as<int2>();
    fp.yr_mode = mode;
    fp.xr_G2C = P.G[2] * C;
    fp.xr_C = C;
    fp.xr_B2 = P.Bs[2];
}
// the adjoint y-range pruning skips stores of the axis-0 pass that the axis-1
// pass must then take as zero: both passes must run on the specialised kernel
static bool yrange_ok(const Plan& P, int C) {
    if (!P.yrange.p || !kFftYPrune) return false;
    int Ob = 1, Ib = 1;
    pass_blocking((int64_t)P.G[2] * C, &Ob, &Ib);  // the column block of the axis-1 passes
    return fft_fixed_ok(P.G[0], 32) && fft_fixed_ok(P.G[1], Ob * Ib);
}

std::vector<FftPass> forward_passes(Plan& P, const float2* x, const FwdOpts& o) {
    const int C = o.C < 0 ? (int)P.C : o.C;
    const int d = P.d;
    float2* bufs[2] = {o.bufs[0] ? o.bufs[0] : P.bufA.as<float2>(), o.bufs[1] ? o.bufs[1] : P.bufB.as<float2>()};
    int which = 0;
    const float2* prev = nullptr;
    std::vector<FftPass> out;
    for (int p = 0; p < d; ++p) {
        const int ax = d - 1 - p;
        FftPass fp{};
        fp.L = P.G[ax];
        fp.Lin = (int)P.N[ax];
        fp.Lout = P.G[ax];
        fp.pad_in = 1;
        fp.crop_out = 0;
        fp.inverse = 0;
        int64_t O = 1, I = C;
        for (int b = 0; b < ax; ++b) O *= P.N[b];
        for (int b = ax + 1; b < d; ++b) I *= P.G[b];
        fp.O = O;
        fp.I = I;
        fp.in_os = (int64_t)fp.Lin * I;
        fp.in_rs = I;
        fp.out_os = (int64_t)fp.Lout * I;
        fp.out_rs = I;
        fill_stages(P, ax, fp);
        fp.out = bufs[which];
        if (p == 0) {
            fp.pre = o.channel ? PRE_CHAN : PRE_MAPS;
            fp.px = x;
            fp.pmaps = P.maps.as<float2>();
            fp.fo = P.fo_fwd.as<float>();
            fp.fr = P.fr_fwd.as<float>();
            fp.xscale = o.xscale;
        } else {
            fp.pre = PRE_NONE;
            fp.in = prev;
        }
        pass_blocking(I, &fp.Ob, &fp.Ib);
        if (ax == 0 && d == 3 && P.xrange.p) set_xrange(P, C, 1, fp);
        if (d == 3 && (ax == 0 || ax == 1) && yrange_ok(P, C)) set_yrange(P, C, ax == 0 ? 1 : 3, fp);
        out.push_back(fp);
        prev = fp.out;
        which ^= 1;
    }
    return out;
}

float2* forward_to_grid(Plan& P, const float2* x, const FwdOpts& o, hipStream_t s) {
    const std::vector<FftPass> ps = forward_passes(P, x, o);
    for (const FftPass& fp : ps) launch_fft_pass(fp, s);
    return ps.back().out;
}

std::vector<FftPass> adjoint_passes(Plan& P, float2* grid, float2* out, const AdjOpts& o) {
    const int C = o.C < 0 ? (int)P.C : o.C;
    const int d = P.d;
    const float2* cur = grid;
    std::vector<FftPass> res;
    for (int ax = 0; ax < d; ++ax) {
        float2* dst = (cur == P.bufA.as<float2>()) ? P.bufB.as<float2>() : P.bufA.as<float2>();
        FftPass fp{};
        fp.L = P.G[ax];
        fp.Lin = P.G[ax];
        fp.Lout = (int)P.N[ax];
        fp.pad_in = 0;
        fp.crop_out = 1;
        fp.inverse = 1;
        int64_t O = 1, I = C;
        for (int b = 0; b < ax; ++b) O *= P.N[b];
        for (int b = ax + 1; b < d; ++b) I *= P.G[b];
        fp.O = O;
        fp.I = I;
        fp.in_os = (int64_t)fp.Lin * I;
        fp.in_rs = I;
        fp.out_os = (int64_t)fp.Lout * I;
        fp.out_rs = I;
        fill_stages(P, ax, fp);
        fp.in = cur;
        if (ax == d - 1) {
            fp.post = o.channel ? POST_CHAN : POST_MAPS;
            fp.qx = out;
            fp.qmaps = P.maps.as<float2>();
            fp.fo = P.fo_fwd.as<float>();
            fp.fr = P.fr_fwd.as<float>();
            fp.epi = o.epi;
            fp.ex = o.ex;
            fp.exbar = o.exbar;
            fp.e_tau = o.tau;
            fp.e_theta = o.theta;
            fp.e_lambda = o.lambda;
            fp.e_lam = o.lam;
            if (!o.channel) {
                fp.Ib = C;
                fp.Ob = std::max(1, 8 / C);
            } else {
                pass_blocking(I, &fp.Ob, &fp.Ib);
            }
        } else {
            fp.post = POST_NONE;
            fp.out = dst;
            pass_blocking(I, &fp.Ob, &fp.Ib);
        }
        if (ax == 0 && d == 3 && P.xrange.p) set_xrange(P, C, 2, fp);
        if (d == 3 && (ax == 0 || ax == 1) && yrange_ok(P, C)) set_yrange(P, C, ax == 0 ? 2 : 4, fp);
        res.push_back(fp);
        cur = dst;
    }
    return res;
}

void grid_to_image(Plan& P, float2* grid, float2* out, const AdjOpts& o, hipStream_t s) {
    for (const FftPass& fp : adjoint_passes(P, grid, out, o)) launch_fft_pass(fp, s);
}

SpreadArgs spread_args(Plan& P, const float2* kint, int C) {
    SpreadArgs a{};
    a.grid = P.bufA.as<float2>();
    a.g = P.g_sorted.as<float>();
    a.k = kint;
    a.touch = P.stouch.as<int32_t>();
    a.code = P.scode.as<uint16_t>();
    a.work = P.work.as<int4>();
    a.nwork = P.nwork;
    a.partial = P.partial.as<float2>();
    a.C = C;
    for (int ax = 0; ax < 3; ++ax) {
        a.G[ax] = P.G[ax];
        a.B[ax] = P.Bs[ax];
        a.nb[ax] = P.nbs[ax];
    }
    return a;
}

float2* spread_to_grid(Plan& P, const float2* kint, int C, hipStream_t s) {
    const SpreadArgs a = spread_args(P, kint, C);
    launch_spread(P.d, P.W, a, P.kb, s);
    launch_reduce_partials(a, P.heavy_list.as<int4>(), (int)P.heavy_tiles, P.d, s);
    return a.grid;
}

InterpArgs interp_args(Plan& P, const float2* grid, const InterpArgs& tmpl) {
    InterpArgs a = tmpl;
    a.grid = grid;
    a.g = P.g_sorted.as<float>();
    a.perm = P.perm.as<int32_t>();
    a.M = P.M;
    if (a.C <= 0) a.C = (int)P.C;
    for (int ax = 0; ax < 3; ++ax) {
        a.G[ax] = P.G[ax];
        a.B[ax] = P.B[ax];
        a.nb[ax] = P.nb[ax];
    }
    return a;
}

void interp(Plan& P, const float2* grid, const InterpArgs& tmpl, hipStream_t s) {
    const InterpArgs a = interp_args(P, grid, tmpl);
    if (P.interp_tiles && a.C == (int)P.C)
        launch_interp_tiles(P.d, P.W, a, P.iwork.as<int4>(), P.niwork, P.kb, s);
    else
        launch_interp(P.d, P.W, a, P.kb, s);
}

// ------------------------------------------------------------ db4 filter
// Daubechies' construction: |m0|^2 = cos^8(xi/2) P(sin^2(xi/2)) with
// P(y) = 1 + 4y + 10y^2 + 20y^3; minimum-phase spectral factor.
std::vector<double> db4_filter_host() {
    // roots of 20 y^3 + 10 y^2 + 4 y + 1 by Durand-Kerner iteration
    typedef std::complex<double> cd;
    const double c[4] = {1.0, 4.0, 10.0, 20.0};
    auto poly = [&](cd y) { return ((c[3] * y + c[2]) * y + c[1]) * y + c[0]; };
    cd r[3] = {cd(0.4, 0.9), cd(0.4, 0.9) * cd(0.4, 0.9), cd(0.4, 0.9) * cd(0.4, 0.9) * cd(0.4, 0.9)};
    for (int it = 0; it < 500; ++it) {
        for (int i = 0; i < 3; ++i) {
            cd den = c[3];
            for (int j = 0; j < 3; ++j)
                if (j != i) den *= (r[i] - r[j]);
            r[i] -= poly(r[i]) / den;
        }
    }
    // z + 1/z = 2 - 4y; keep |z| < 1
    std::vector<cd> pz = {cd(1.0)};
    auto mul = [&](cd a0, cd a1) {  // multiply by (a0 + a1 z^-1)
        std::vector<cd> q(pz.size() + 1, cd(0.0));
        for (size_t i = 0; i < pz.size(); ++i) {
            q[i] += pz[i] * a0;
            q[i + 1] += pz[i] * a1;
        }
        pz = q;
    };
    for (int i = 0; i < 4; ++i) mul(1.0, 1.0);
    for (int i = 0; i < 3; ++i) {
        const cd b = 2.0 - 4.0 * r[i];
        const cd disc = std::sqrt(b * b - 4.0);
        cd z = (b + disc) / 2.0;
        if (std::abs(z) >= 1.0) z = (b - disc) / 2.0;
        mul(1.0, -z);
    }
    std::vector<double> h(8);
    double sum = 0;
    for (int i = 0; i < 8; ++i) {
        h[i] = pz[i].real();
        sum += h[i];
    }
    for (auto& v : h) v *= std::sqrt(2.0) / sum;
    return h;
}

void require_plan_device(const Plan& P) {
    int cur = 0;
    KP_HIP(hipGetDevice(&cur));
    if (cur != P.dev)
        fail(KP_ERR_INVALID_ARG, "the plan belongs to device " + std::to_string(P.dev) + " but device " +
                                     std::to_string(cur) + " is current");
}

}  // namespace kp

// ================================================================== C ABI
using namespace kp;

extern "C" {

const char* kp_last_error(void) { return kp::t_last_error.c_str(); }

int nufft_plan_validate(int ndim, const int64_t* shape, int64_t ncoils, int64_t nsamples, const void* coords,
                        const void* maps, float oversamp, int kb_width, const kp_tuning* tuning) {
    return guarded([&] { validate_plan_args(ndim, shape, ncoils, nsamples, coords, maps, oversamp, kb_width, tuning, false); });
}

int nufft_plan(kp_plan_t* out, int ndim, const int64_t* shape, int64_t ncoils, int64_t nsamples, const float* coords,
               const void* maps, float oversamp, int kb_width, const kp_tuning* tuning, void* stream) {
    return guarded([&] {
        if (!out) fail(KP_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        Plan* P = create_plan(ndim, shape, ncoils, nsamples, coords, maps, oversamp, kb_width, tuning,
                              (hipStream_t)stream, false);
        *out = new kp_plan{P};
    });
}

void nufft_destroy(kp_plan_t plan) {
    if (!plan) return;
    if (plan->impl) {
        (void)hipStreamSynchronize(plan->impl->stream);
        (void)hipDeviceSynchronize();
        delete plan->impl;
    }
    delete plan;
}

int nufft_forward(kp_plan_t plan, const void* x, void* y, void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl) fail(KP_ERR_INVALID_ARG, "plan is NULL");
        if (!x || !y) fail(KP_ERR_INVALID_ARG, "x or y is NULL");
        Plan& P = *plan->impl;
        require_plan_device(P);
        hipStream_t s = (hipStream_t)stream;
        P.stream = s;
        FwdOpts fo;
        float2* grid = forward_to_grid(P, (const float2*)x, fo, s);
        InterpArgs ia{};
        ia.mode = IO_CALLER;
        ia.out = (float2*)y;
        interp(P, grid, ia, s);
    });
}

int nufft_adjoint(kp_plan_t plan, const void* y, void* x, void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl) fail(KP_ERR_INVALID_ARG, "plan is NULL");
        if (!x || !y) fail(KP_ERR_INVALID_ARG, "x or y is NULL");
        Plan& P = *plan->impl;
        require_plan_device(P);
        hipStream_t s = (hipStream_t)stream;
        P.stream = s;
        permute_to_internal((const float2*)y, P.kint.as<float2>(), P.perm.as<int32_t>(), P.M, (int)P.C, s,
                            P.iperm.as<int32_t>());
        float2* grid = spread_to_grid(P, P.kint.as<float2>(), (int)P.C, s);
        AdjOpts ao;
        grid_to_image(P, grid, (float2*)x, ao, s);
    });
}

int nufft_plan_info(kp_plan_t plan, kp_plan_info* info) {
    return guarded([&] {
        if (!plan || !plan->impl || !info) fail(KP_ERR_INVALID_ARG, "NULL argument");
        const Plan& P = *plan->impl;
        std::memset(info, 0, sizeof(*info));
        info->ndim = P.d;
        for (int a = 0; a < 3; ++a) {
            info->shape[a] = a < P.d ? P.N[a] : 1;
            info->grid[a] = a < P.d ? P.G[a] : 1;
            info->bin_size[a] = P.B[a];
            info->spread_bin_size[a] = P.Bs[a];
        }
        info->nspread_tiles = P.nstiles;
        info->ncoils = P.C;
        info->nsamples = P.M;
        info->kb_width = P.W;
        info->oversamp = P.alpha;
        info->kb_beta = P.beta;
        info->nbins = P.nbins;
        info->ntouch = P.ntouch;
        info->nwork = P.nwork;
        info->heavy_tiles = P.heavy_tiles;
        info->max_chunk = P.max_chunk;
        info->workspace_bytes = P.bytes;
    });
}

int nufft_plan_sort(kp_plan_t plan, int32_t* perm, int32_t* bin_offsets, int32_t* touch_offsets, int32_t* touch,
                    void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl) fail(KP_ERR_INVALID_ARG, "plan is NULL");
        Plan& P = *plan->impl;
        require_plan_device(P);
        hipStream_t s = (hipStream_t)stream;
        if (perm) KP_HIP(hipMemcpyAsync(perm, P.perm.p, sizeof(int32_t) * P.M, hipMemcpyDeviceToDevice, s));
        if (bin_offsets)
            KP_HIP(hipMemcpyAsync(bin_offsets, P.bin_off.p, sizeof(int32_t) * (P.nbins + 1), hipMemcpyDeviceToDevice, s));
        if (touch_offsets)
            KP_HIP(hipMemcpyAsync(touch_offsets, P.touch_off.p, sizeof(int32_t) * (P.nstiles + 1), hipMemcpyDeviceToDevice, s));
        if (touch && P.ntouch > 0)
            KP_HIP(hipMemcpyAsync(touch, P.touch.p, sizeof(int32_t) * P.ntouch, hipMemcpyDeviceToDevice, s));
    });
}

int nufft_plan_grid_coords(kp_plan_t plan, float* g, void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl || !g) fail(KP_ERR_INVALID_ARG, "NULL argument");
        Plan& P = *plan->impl;
        require_plan_device(P);
        KP_HIP(hipMemcpyAsync(g, P.g_orig.p, sizeof(float) * P.M * P.d, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    });
}

int nufft_stage(kp_plan_t plan, int stage, int reps, void* stream) {
    return guarded([&] {
        if (!plan || !plan->impl) fail(KP_ERR_INVALID_ARG, "plan is NULL");
        if (stage < 0 || stage > KP_STAGE_PROX) fail(KP_ERR_INVALID_ARG, "unknown stage");
        if (reps < 1) fail(KP_ERR_INVALID_ARG, "reps must be >= 1");
        Plan& P = *plan->impl;
        require_plan_device(P);
        hipStream_t s = (hipStream_t)stream;
        for (int r = 0; r < reps; ++r) {
            if (stage == KP_STAGE_FWD_FFT) {
                FwdOpts fo;
                forward_to_grid(P, P.img[0].as<float2>(), fo, s);
            } else if (stage == KP_STAGE_INTERP) {
                InterpArgs ia{};
                ia.mode = IO_INTERNAL;
                ia.out = P.kint3.as<float2>();
                interp(P, P.d % 2 ? P.bufA.as<float2>() : P.bufB.as<float2>(), ia, s);
            } else if (stage == KP_STAGE_SPREAD) {
                spread_to_grid(P, P.kint.as<float2>(), (int)P.C, s);
            } else if (stage == KP_STAGE_SPREAD_TILES) {
                launch_spread(P.d, P.W, spread_args(P, P.kint.as<float2>(), (int)P.C), P.kb, s);
            } else if (stage == KP_STAGE_PROX) {
                wavelet_prox_stage(P, s);
            } else {
                AdjOpts ao;
                grid_to_image(P, P.bufA.as<float2>(), P.img[3].as<float2>(), ao, s);
            }
        }
    });
}

int kp_db4_filter(double* h8) {
    return guarded([&] {
        if (!h8) fail(KP_ERR_INVALID_ARG, "h8 is NULL");
        auto h = db4_filter_host();
        for (int i = 0; i < 8; ++i) h8[i] = h[i];
    });
}

}  // extern "C"
