// Internal declarations shared by the translation units of libkpdhg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/kpdhg.h"

namespace kp {

// ----------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_error(const std::string& msg);

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

#define KP_HIP(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            ::kp::fail(KP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define KP_LAUNCH_CHECK() KP_HIP(hipGetLastError())

// Run a C-ABI body, translating exceptions to status codes.
template <class F>
int guarded(F&& f) {
    try {
        f();
        return KP_OK;
    } catch (const Error& e) {
        set_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return KP_ERR_OOM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return KP_ERR_HIP;
    }
}

// ------------------------------------------------------------ device memory
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void alloc(size_t n);
    void release();
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// ------------------------------------------------------------ FFT pass
enum PreMode { PRE_NONE = 0, PRE_MAPS = 1, PRE_CHAN = 2 };
enum PostMode { POST_NONE = 0, POST_MAPS = 1, POST_CHAN = 2 };
enum Epi { EPI_STORE = 0, EPI_L2 = 1, EPI_Z = 2 };

constexpr int kMaxStages = 12;

struct FftPass {
    const float2* in;
    float2* out;
    int64_t O, I;                  // outer count, inner (contiguous) count
    int Lin, Lout, L;              // input rows, output rows, transform length
    int64_t in_os, in_rs;          // element strides of input (outer, row); inner stride 1
    int64_t out_os, out_rs;
    int Ob, Ib;                    // columns per block: Ob outers x Ib inners
    int nst;
    int rad[kMaxStages];
    const float2* tw;              // exp(-2 pi i m / L), m < L
    int inverse;
    int pad_in, crop_out;          // centred placement / centred crop
    // fused pre-pass (first forward pass along the last image axis)
    int pre;
    const float2* px;              // image [O][Lin] (PRE_MAPS) or [O][Lin][I] (PRE_CHAN)
    const float2* pmaps;           // [O][Lin][I] (PRE_MAPS)
    const float* fo;               // per-outer factor [O]
    const float* fr;               // per-row factor [Lin or Lout]
    const float* xscale;           // optional device scalar multiplier
    // fused post-pass (last adjoint pass along the last image axis)
    int post;
    float2* qx;                    // output image [O][Lout] (POST_MAPS) or channels
    const float2* qmaps;
    int epi;
    float2* ex;                    // x (read, updated) for EPI_L2 / EPI_Z
    float2* exbar;                 // xbar (written) for EPI_L2; z for EPI_Z
    const float* e_tau;            // device scalars
    const float* e_theta;
    float e_lambda;
    const float* e_lam;            // device lambda (overrides e_lambda when set)
    // support pruning of the passes along axis 0 in 3D: xr[ty nb2 + tz] is the
    // axis-0 cell range [lo, hi) holding every non-empty spreading tile of
    // tile column (ty, tz); rows outside it are not stored (xr_mode 1, the last
    // forward pass: nothing reads them) or not loaded and taken as zero
    // (xr_mode 2, the first adjoint pass: spreading leaves them zero)
    const int2* xr;
    int xr_mode;
    int xr_G2C, xr_C, xr_B1, xr_B2, xr_nb2;
    // and along axis 1: yr[tz] is the axis-1 cell range [lo, hi) holding every
    // tile column (ty, tz) that has a non-empty spreading tile; grid rows
    // (.., y, z, ..) with y outside the range of tz = z / B2 are zero in the
    // adjoint and unused in the forward direction.  yr_mode 1: forward pass
    // along axis 0, a column outside is not loaded (nothing of it is stored);
    // 2: adjoint pass along axis 0, a column outside is not stored; 3:
    // forward pass along axis 1, rows outside are not stored; 4: adjoint pass
    // along axis 1, rows outside are not loaded and taken as zero
    const int2* yr;
    int yr_mode;
};

void launch_fft_pass(const FftPass& p, hipStream_t s);
// the specialised pass kernel handles length L with nc columns per block
bool fft_fixed_ok(int L, int nc);
void fft_factor(int L, int* nst, int* rad);
size_t fft_lds_bytes(int L, int ncol);

// ------------------------------------------------------------ gridding
// Kaiser-Bessel weights of the W taps of a sample as polynomials in
// x = frac(g) - 1/2: weight of tap t = sum_k poly[t][k] x^k (degree 9,
// fitted on the host in double precision at Chebyshev nodes).  The kernel is
// even, so tap W-1-t is tap t mirrored (x -> -x): with the even and odd
// parts of tap t's polynomial as polynomials in x^2 (ev[t], od[t], degree 4),
// tap t = ev + x od and tap W-1-t = ev - x od, for t < W/2.
constexpr int kPolyN = 10;
constexpr int kHalfN = kPolyN / 2;
struct KbParams {
    float poly[8][kPolyN];
    float ev[4][kHalfN];
    float od[4][kHalfN];
};
void kb_fit(double beta, int W, KbParams* kb);
double kb_kernel_host(double u, int W, double beta);

enum InterpOut { IO_CALLER = 0, IO_INTERNAL = 1, IO_DUAL = 2, IO_PMUL = 3 };

struct InterpArgs {
    const float2* grid;       // [G][C]
    const float* g;           // sorted grid coords [M][d]
    const int32_t* perm;      // sorted -> caller
    int64_t M;
    int C;
    int G[3];
    int mode;
    float2* out;              // caller [C][M] or internal [M][C]
    // dual update / p multiply
    float2* u;                // internal [M][C]
    const float2* y;          // internal [M][C]
    const float* p;           // internal [M][C] (MC) or [M] (SC) or null
    int p_mc;
    const float* sigma;       // device scalar
    // tile geometry (tile-staged path)
    int B[3];
    int nb[3];
};

struct SpreadArgs {
    float2* grid;             // [G][C]
    const float* g;           // sorted coords [M][d]
    const float2* k;          // internal k-space [M][C]
    const int32_t* touch;     // entries (sorted sample positions), each tile's in bucket order
    const uint16_t* code;     // bucket of each entry (first tap, leading axes, local + W - 1)
    const int4* work;         // (tile, start, count, partial slot or -1)
    int64_t nwork;
    float2* partial;          // [slots][tile cells][C] partial tiles of split tiles
    int C;
    int G[3];
    int B[3];
    int nb[3];
};

// spreading launch geometry derived from the tile shape
constexpr int kSpreadChunk = 128;   // touch entries staged in LDS at a time
constexpr bool kFftYPrune = true;        // y-range pruning of the 3D axis-0 / axis-1 FFT passes
constexpr int kZMax = 8;            // tile extent along the last axis (max)
int spread_threads(int d, const int* B, int C);
int spread_nbk(int d, int W, const int* B);
int spread_zm(int d, const int* B);
size_t spread_lds_bytes(int d, int W, const int* B, int C, int zm = 0);

void launch_interp(int d, int W, const InterpArgs& a, const KbParams& kb, hipStream_t s);
// tile-staged interpolation over pieces (tile, first sorted sample, count, 0)
constexpr int kInterpPiece = 1024;          // samples per piece at most
constexpr size_t kInterpTileLds = 65536;    // halo bytes up to which the staged path is used
size_t interp_tile_lds_bytes(int d, int W, const int* B, int C);
void launch_interp_tiles(int d, int W, const InterpArgs& a, const int4* items, int64_t nitems, const KbParams& kb,
                         hipStream_t s);
void launch_spread(int d, int W, const SpreadArgs& a, const KbParams& kb, hipStream_t s);
void launch_reduce_partials(const SpreadArgs& a, const int4* heavy, int nheavy, int d, hipStream_t s);

// ------------------------------------------------------------ plan
struct Plan {
    int dev = 0;          // device current when the plan was made; every call on it must run there
    int d = 0;
    int64_t N[3] = {1, 1, 1};
    int64_t Ntot = 0;
    int64_t C = 1;
    int64_t M = 0;
    int G[3] = {1, 1, 1};
    int64_t Gtot = 0;
    int W = 4;
    float alpha = 2.f;
    double beta = 0;
    KbParams kb{};
    int B[3] = {1, 1, 1};         // sort / interpolation tiles
    int nb[3] = {1, 1, 1};
    int64_t nbins = 0;
    int Bs[3] = {1, 1, 1};        // spreading tiles
    int nbs[3] = {1, 1, 1};
    int64_t nstiles = 0;
    int64_t ntouch = 0;
    int64_t nwork = 0;
    int64_t heavy_tiles = 0;
    int max_chunk = 0;            // spreading split size in use
    bool has_maps = false;
    hipStream_t stream = nullptr;
    int lds_max = 65536;
    int spread_lds = 0;

    DevBuf coords;                // caller's coordinates [M][d]
    DevBuf g_sorted, g_orig, perm, bin_off, touch_off, touch, work, heavy_list;
    DevBuf iperm;                 // inverse of perm: sorted position of caller sample j
    DevBuf stouch, scode;         // touch entries in spreading order, their buckets
    DevBuf xrange;                // 3D: axis-0 cell range of the non-empty spreading tiles per (ty, tz)
    DevBuf yrange;                // 3D: axis-1 cell range of the tile columns with a non-empty tile, per tz
    DevBuf partial;               // partial tiles of split tiles
    DevBuf iwork;                 // interpolation pieces (tile, start, count, 0)
    int64_t niwork = 0;
    bool interp_tiles = false;    // tile-staged interpolation in use
    int64_t nslots = 0;
    DevBuf maps;                  // [N][C]
    DevBuf fo_fwd, fr_fwd;        // deapodisation factors for the first/last pass
    DevBuf tw[3];                 // twiddles per axis
    DevBuf bufA, bufB;            // FFT ping-pong [>= Gtot*C]
    DevBuf kint;                  // internal k-space [M][C]
    DevBuf kint2;                 // second internal k-space (y for the solver)
    DevBuf kint3;                 // third internal k-space (residuals, gradients)
    DevBuf kint4;                 // fourth internal k-space (the dual solver's iterate)
    DevBuf pint;                  // internal preconditioner [M][C]
    DevBuf img[4];                // image workspaces [N]
    DevBuf tvv;                   // TV dual variable [d][N]
    DevBuf red;                   // reduction scratch
    DevBuf sched;                 // schedule arrays
    std::vector<int> fft_nst[3];
    std::vector<int> fft_rad[3];
    int64_t bytes = 0;
};

// fails (KP_ERR_INVALID_ARG) unless the plan's device is the current one:
// the library never switches devices, and a plan's buffers live on one
void require_plan_device(const Plan& P);

Plan* create_plan(int ndim, const int64_t* shape, int64_t ncoils, int64_t nsamples,
                  const float* coords, const void* maps, float oversamp, int kb_width,
                  const kp_tuning* tuning, hipStream_t stream, bool channel_mode);
void validate_plan_args(int ndim, const int64_t* shape, int64_t ncoils, int64_t nsamples,
                        const void* coords, const void* maps, float oversamp, int kb_width,
                        const kp_tuning* tuning, bool channel_mode);

// Operator drivers (internal layouts).  x/out images are [N] (maps) or
// [N][C] (channel mode, no maps).
struct FwdOpts {
    const float* xscale = nullptr;   // device scalar multiplying x
    bool channel = false;            // x is [N][C] (no maps)
    int C = -1;                      // channels (<= plan C), -1 = plan C
    float2* bufs[2] = {nullptr, nullptr};  // ping-pong grids instead of the plan's bufA / bufB
};
// Pre-pass + FFT passes: image -> grid (result in plan bufA or bufB; returned)
float2* forward_to_grid(Plan& P, const float2* x, const FwdOpts& o, hipStream_t s);
// Spread internal k-space into grid (bufA)
float2* spread_to_grid(Plan& P, const float2* kint, int C, hipStream_t s);
struct AdjOpts {
    bool channel = false;
    int C = -1;
    int epi = EPI_STORE;
    float2* ex = nullptr;
    float2* exbar = nullptr;
    const float* tau = nullptr;
    const float* theta = nullptr;
    float lambda = 0.f;
    const float* lam = nullptr;      // device lambda (overrides `lambda`)
};
// Inverse FFT passes + post-pass from grid (in bufA) to image `out`
void grid_to_image(Plan& P, float2* grid, float2* out, const AdjOpts& o, hipStream_t s);

void interp(Plan& P, const float2* grid, const InterpArgs& tmpl, hipStream_t s);

// descriptor builders (what forward_to_grid / grid_to_image / spread_to_grid /
// interp launch), used to assemble one-launch-per-phase batches
std::vector<FftPass> forward_passes(Plan& P, const float2* x, const FwdOpts& o);
std::vector<FftPass> adjoint_passes(Plan& P, float2* grid, float2* out, const AdjOpts& o);
SpreadArgs spread_args(Plan& P, const float2* kint, int C);
InterpArgs interp_args(Plan& P, const float2* grid, const InterpArgs& tmpl);

// batched launches (fft.hip, grid.hip)
bool fft_batchable(const FftPass& p);
int64_t fft_pass_blocks(const FftPass& p);
// one launch over the passes of a phase of mixed lengths (sorted by length);
// map: the coil column block of the passes along the coils, else 0
int fft_mixed_columns(int L, int nc_map);
void launch_fft_batch_mixed(const FftPass* d_passes, const int64_t* d_blk_start, int n, int64_t nblk, int map,
                            size_t lds, hipStream_t s);
void launch_interp_batch(const InterpArgs* d_args, const int64_t* d_start, int n, int64_t nblk, const KbParams& kb,
                         hipStream_t s);
void launch_spread_batch(const SpreadArgs* d_args, const int64_t* d_start, int n, int64_t nblk, int threads,
                         size_t lds, int zm, const KbParams& kb, hipStream_t s);
void launch_reduce_batch(const SpreadArgs* d_args, const int2* d_hv, const int4* const* d_lists, int nh,
                         hipStream_t s);
void pdhg_setup(Plan& P, const float2* y, const float* p, int p_kind, const kp_pdhg_opts& op, hipStream_t s);

// Elementwise helpers (solver.hip)
// (with iperm, the inverse permutation, for C = 2, 4, 8 or 12: one thread
// per caller sample, coalesced reads of the coil rows, one contiguous run of
// 16-byte stores per sample at its sorted position)
void permute_to_internal(const float2* y_caller, float2* kint, const int32_t* perm, int64_t M,
                         int C, hipStream_t s, const int32_t* iperm = nullptr);
void permute_to_caller(const float2* kint, float2* y_caller, const int32_t* perm, int64_t M,
                       int C, hipStream_t s);
void permute_p_to_internal(const float* p_caller, float* pint, const int32_t* perm, int64_t M,
                           int C, bool mc, hipStream_t s);
void permute_p_to_caller(const float* pint, float* p_caller, const int32_t* perm, int64_t M,
                         int C, bool mc, hipStream_t s);


// solver helpers (solver.hip)
void fill2(float2* x, int64_t n, float re, float im, hipStream_t s);
void copy2(const float2* a, float2* b, int64_t n, hipStream_t s);
void reduce(const float2* a, const float2* b, int64_t n, int kind, double* out, double scale, bool accumulate,
            double* part, hipStream_t s);
void reduce_min(const float* p, int64_t n, float* out, float* part, hipStream_t s);
// prox steps fused into the wavelet passes: soft threshold *tau * lam on the
// analysis, x/xbar update with theta on the last synthesis pass
struct DwtFuse {
    const float* tau;
    float lam;
    float2* ex;
    float2* exbar;
    const float* theta;
};
void dwt(float2* x, const int64_t* N, int d, int levels, bool inverse, hipStream_t s, const DwtFuse* fz = nullptr);
void power_method(Plan& P, const float* pint, int p_mc, int iters, float* lam_out, hipStream_t s);
const float* load_p(Plan& P, const float* p, int p_kind, hipStream_t s);
void upload_wavelet_constants();
void wavelet_prox_stage(Plan& P, hipStream_t s);
void fft_twiddles(int L, DevBuf& tw);
void pass_blocking(int64_t I, int* Ob, int* Ib);
std::vector<double> db4_filter_host();

}  // namespace kp

struct kp_plan {
    kp::Plan* impl;
};
