/*
 * kpdhg.h - C ABI of the MI355X (gfx950) hot path of k-space-preconditioned
 * PDHG reconstruction for non-Cartesian multi-coil MRI (Ong, Uecker, Lustig,
 * "Accelerating Non-Cartesian MRI Reconstruction Convergence using k-space
 * Preconditioning").
 *
 * Conventions for every call
 * --------------------------
 *  - Pointers are DEVICE pointers unless a parameter says "host".
 *  - complex values are interleaved float pairs (re, im) == torch.complex64.
 *  - An image has shape (N_0, .., N_{d-1}), C order, last axis fastest; array
 *    index m_a sits at the centred position n_a = m_a - N_a/2.
 *  - k-space arrays are coil-major [C][M] in the caller's sample order
 *    (Problem Setup: the stacked vector y of Eq. model).
 *  - Coordinates are float32 [M][d] in radians per pixel, nominally in
 *    [-pi, pi); column a pairs with image axis a.  omega = 2 pi f / N_a with
 *    the paper's f in cycles.  Values up to about 3 pi are wrapped
 *    periodically; anything further out, NaN or inf is rejected by
 *    nufft_plan with KP_ERR_INVALID_ARG.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *    stream-ordered and asynchronous unless its comment says otherwise.  A
 *    plan serves one stream at a time and is not re-entrant.
 *  - A plan (and a batch) belongs to the device that was current when it was
 *    made; every later call on it must run with that device current, else it
 *    fails with KP_ERR_INVALID_ARG (the library never switches devices).
 *  - Every call returns KP_OK or a negative status and never throws; the
 *    message of the last failure on the calling thread is kp_last_error().
 *    Asynchronous kernel faults surface as KP_ERR_HIP at the next checked
 *    call.
 *  - Memory: nufft_plan allocates every workspace the plan's forward,
 *    adjoint and solve calls need; those calls never allocate.
 *    precond_build allocates and frees its own scratch (setup-time call).
 */
#ifndef KPDHG_H
#define KPDHG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kp_plan* kp_plan_t;
typedef struct kp_batch* kp_batch_t;

enum {
    KP_OK = 0,
    KP_ERR_INVALID_ARG = -1,  /* bad pointer, size, option or coordinate   */
    KP_ERR_UNSUPPORTED = -2,  /* valid but outside what the kernels cover  */
    KP_ERR_OOM = -3,          /* device or host allocation failed          */
    KP_ERR_HIP = -4           /* a HIP runtime call or kernel failed       */
};

enum { KP_PRECOND_NONE = 0, KP_PRECOND_SC = 1, KP_PRECOND_MC = 2, KP_PRECOND_DCF = 3 };
enum { KP_REG_L2 = 0, KP_REG_L1_WAVELET = 1, KP_REG_TV = 2 };

/* Kernel tiling.  Zeros select the built-in choice for the shape.
 * Samples are sorted by the tile (bin_size) that holds their grid cell; the
 * interpolation stages each such tile's halo.  Spreading owns the cells of its
 * own tiles (spread_bin_size), through per-tile touch lists. */
typedef struct {
    int bin_size[3];        /* sort / interpolation tile edge per axis; divides G_a */
    int max_chunk;          /* max touch-list entries per spreading work item; 0:
                               1024 for plans of 4096 x 1024 entries and more, else
                               halved (down to 128) until the plan has that many
                               items' worth                                          */
    int spread_bin_size[3]; /* spreading tile edge per axis; divides G_a; last axis
                               <= 8; in 3D axis 1 + W <= 65 (else
                               KP_ERR_UNSUPPORTED)                                   */
} kp_tuning;

/* Shape facts of a plan (filled by nufft_plan_info, host struct). */
typedef struct {
    int ndim;
    int64_t shape[3];
    int64_t grid[3];        /* oversampled grid G_a                           */
    int64_t ncoils, nsamples;
    int kb_width;
    float oversamp;
    double kb_beta;         /* Kaiser-Bessel shape parameter                  */
    int bin_size[3];        /* sort tiles                                     */
    int64_t nbins;          /* number of sort tiles                           */
    int64_t ntouch;         /* total spreading-tile touch entries             */
    int64_t nwork;          /* spreading work items                           */
    int64_t heavy_tiles;    /* spreading tiles split over several work items  */
    int64_t workspace_bytes;/* device bytes owned by the plan                 */
    int spread_bin_size[3]; /* spreading tiles                                */
    int64_t nspread_tiles;  /* number of spreading tiles                      */
    int max_chunk;          /* spreading split size in use (kp_tuning)        */
} kp_plan_info;

/* PDHG options (host struct). */
typedef struct {
    int reg;              /* KP_REG_L2, KP_REG_L1_WAVELET or KP_REG_TV               */
    float lambda;         /* regularisation weight (Problem Setup, Eq. obj)          */
    int iters;            /* PDHG iterations K >= 1                                  */
    int wavelet_levels;   /* db4 levels for KP_REG_L1_WAVELET (every N_a % 2^L == 0) */
    float lambda_max;     /* <= 0: estimate lambda_max(P A A^H) by the power method  */
    int power_iters;      /* power-method iterations (the paper uses 30)             */
    float sigma0;         /* sigma^(0) (the paper fixes 1)                           */
    int accel;            /* 1: theta_k = 1/(1+2 sigma_k min p) schedule; 0: theta=1 */
    const void* x0;       /* NULL or c64 [N] initial primal                          */
    const void* u0;       /* NULL or c64 [C][M] initial dual (caller order)          */
    double* objective_host; /* NULL or host double [iters+1]: 1/2||Ax-y||^2 + g(x)
                               before the first and after every iteration; costs one
                               extra forward and a host sync per iteration           */
    float* lambda_max_out;  /* NULL or device float [1]: the lambda_max used          */
} kp_pdhg_opts;

/* Build a plan: canonical float32 grid coordinates, bin keys, a stable
 * bit-exact sort of samples by tile, tile touch lists, Kaiser-Bessel and
 * deapodisation tables, twiddles, and every workspace.
 *   ndim       2 or 3
 *   shape      host int64[ndim], each N_a even, 2 <= N_a <= 4096
 *   ncoils     C >= 1 (maps == NULL requires C == 1: unit sensitivity)
 *   nsamples   M >= 1
 *   coords     device float32 [M][ndim]; copied (in sorted order) by the plan
 *   maps       device c64 [C][N] coil sensitivities (Problem Setup, s_c), or
 *              NULL; copied by the plan (the caller may free its copy once
 *              the stream has passed this call)
 *   oversamp   alpha in [1.25, 2]; G_a = ceil(alpha N_a) raised to the next
 *              even 5-smooth integer (Experiments: alpha = 1.25)
 *   kb_width   W in {2, 4, 6, 8} (Experiments: W = 4); Kaiser-Bessel shape
 *              beta of Beatty et al.
 *   tuning     host struct or NULL
 * Synchronises `stream` once (to size the spreading work list). */
int nufft_plan(kp_plan_t* out, int ndim, const int64_t* shape, int64_t ncoils,
               int64_t nsamples, const float* coords, const void* maps,
               float oversamp, int kb_width, const kp_tuning* tuning, void* stream);

/* y = A x  (Problem Setup, Eq. model_i without noise; NUFFT approximation):
 * coil multiply, deapodisation, zero-padded oversampled FFT, Kaiser-Bessel
 * interpolation.  x: c64 [N]; y: c64 [C][M] in the caller's sample order,
 * overwritten. */
int nufft_forward(kp_plan_t plan, const void* x, void* y, void* stream);

/* nufft_forward for callers that cannot allocate device memory where they
 * call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same operation and arguments as nufft_forward, but
 * the two FFT ping-pong grids come from a static per-device array of
 * 2 x 16 MiB that the library holds until the process ends, not from the
 * plan's workspaces.  Allocates nothing.  A plan whose grid needs more than
 * 16 MiB per buffer (G_0..G_{d-1} x C x 8 bytes; e.g. 2D 400^2 grids up to
 * 13 coils) is refused with KP_ERR_UNSUPPORTED before any launch.  Every
 * call on one device shares that device's array: calls that overlap in time
 * on one device (different streams or threads) race and must not be issued;
 * calls ordered on one stream are safe. */
int nufft_forward_noalloc(kp_plan_t plan, const void* x, void* y, void* stream);

/* x = A^H y: Kaiser-Bessel spreading accumulated per tile in LDS, inverse
 * oversampled FFT, crop, deapodisation, conj(s_c) and coil sum.
 * y: c64 [C][M] caller order; x: c64 [N], overwritten. */
int nufft_adjoint(kp_plan_t plan, const void* y, void* x, void* stream);

/* l2-optimised diagonal k-space preconditioner (section "l2 optimized
 * diagonal k-space preconditioners", Appendix A) built with the efficient
 * algorithm of "Efficient computation of the multi-channel preconditioner"
 * (Fig. 2): autocorrelations of s_c s_d^* by FFT at 2N, the point-spread
 * function by an adjoint NUFFT of ones on the 2N image, a forward NUFFT of
 * their product, p = 1/Re(.).
 *   kind KP_PRECOND_SC: Eq. sc_precond (coil maps ignored), p float [M]
 *   kind KP_PRECOND_MC: Eq. mc_precond, p float [C][M]
 *   kind KP_PRECOND_DCF: the Pipe-Menon density compensation factor, the
 *     first of the three k-space preconditioners the Experiments compare:
 *     w <- w / |G G^T w| from w = 1, 30 times, G the plan's gridding
 *     interpolation (its kernel and oversampled grid, no FFT); p float [M]
 *     (one weight per sample; pass it to the solver calls as p_kind
 *     KP_PRECOND_SC), scaled so that lambda_max(P A A^H) = 1 (power method,
 *     30 iterations): with the fixed dual step the primal step 1/lambda_max
 *     would otherwise carry the weights' arbitrary scale into the proximal
 *     threshold.  Uses the plan's internal buffers.
 * Caller sample order.  Allocates and frees scratch; synchronises. */
int precond_build(kp_plan_t plan, int kind, float* p, void* stream);

/* lambda_max(P A A^H) by the power method on A^H P A (Experiments: 30
 * iterations): v0 = ones/||ones||, v <- A^H P A v / ||A^H P A v||; the
 * estimate is the last norm.  p: NULL (P = I), float [M] (SC) or [C][M]
 * (MC) per p_kind.  out: device float [1].  No host sync. */
int pdhg_lambda_max(kp_plan_t plan, const float* p, int p_kind, int iters,
                    float* out, void* stream);

/* Preconditioned PDHG for simple regularisers (section "Preconditioned PDHG
 * for simple regularizers"): per iteration
 *   u  <- (u + sigma P (A xbar - y)) / (1 + sigma P)   (fused in interpolation)
 *   x' <- prox_{tau g}(x - tau A^H u)                   (fused in the last IFFT pass)
 *   xbar <- x' + theta (x' - x)
 * with sigma_0 = opts->sigma0, tau_0 = 1/(sigma_0 lambda_max) and the
 * accelerated schedule theta_k = 1/(1 + 2 sigma_k min p), sigma_{k+1} =
 * theta_k sigma_k, tau_{k+1} = tau_k/theta_k (or theta = 1 if !accel).
 * g = lambda||x||^2/2 (prox z/(1+tau lambda)) or lambda||W x||_1 with the
 * periodised db4 W (prox W^H soft(W z, tau lambda)).
 * KP_REG_TV, g = lambda ||G x||_1 with G the periodic forward differences
 * along every axis (anisotropic, complex modulus per component), follows
 * "Preconditioned PDHG for simple regularizers composed with linear
 * operators": a second dual v for G x,
 *   v  <- clip_lambda(v + sigma G xbar)   (prox of sigma h*, h = lambda||.||_1)
 *   x' <- x - tau (A^H u + G^H v)
 * with constant steps sigma = theta = 1, tau = 1/(lambda_max + lambda_max(G G^H)),
 * lambda_max(G G^H) = 4 d (every N_a is even); opts->sigma0 and accel are
 * not used.  x0 = u0 = 0 (and v = 0) unless given.
 * y: c64 [C][M]; p: NULL / float [M] / float [C][M] per p_kind;
 * x_out: c64 [N]; u_out: NULL or c64 [C][M] (caller order).  No host sync
 * unless opts->objective_host is set. */
int pdhg_solve(kp_plan_t plan, const void* y, const float* p, int p_kind,
               const kp_pdhg_opts* opts, void* x_out, void* u_out, void* stream);

/* l2-regularised reconstruction through its dual (Supporting Materials,
 * connection to Trzasko et al.): conjugate gradients on
 * (A A^H + lambda I) u = lambda y with the diagonal k-space preconditioner P
 * as M^-1 (P = I for KP_PRECOND_NONE), u_0 = 0, `iters` iterations (one NUFFT
 * pair each), then x = A^H u / lambda, the minimiser of
 * 1/2 ||A x - y||^2 + lambda/2 ||x||^2.  y: c64 [C][M]; p: as pdhg_solve;
 * x_out: c64 [N]; u_out: NULL or c64 [C][M] (caller order); residual_host:
 * NULL or host double [iters+1] receiving ||r_k|| / ||r_0|| (one host sync
 * per iteration when given).  lambda > 0. */
int l2_dual_cg(kp_plan_t plan, const void* y, const float* p, int p_kind, float lambda,
               int iters, void* x_out, void* u_out, double* residual_host, void* stream);

/* Unrolled differentiable l2 PDHG (same iteration as pdhg_solve, with free
 * per-step sizes): params = device float [3K+1] = sigma[K], tau[K],
 * theta[K], lambda.  Forward: runs K steps from x0 (NULL = 0), u0 = 0,
 * writes x_K and stores checkpoints of (x, xbar, u) every `ckpt_every`
 * steps into `ckpt` (device, size pdhg_unrolled_ckpt_bytes).
 * Backward: given g_x = dL/dx_K (PyTorch's complex gradient convention),
 * recomputes each segment from its checkpoint and runs the reverse
 * recursion; writes g_params float [3K+1], g_y c64 [C][M] (or NULL) and
 * g_x0 c64 [N] (or NULL).  Both use the plan's NUFFT kernels for A and A^H. */
int64_t pdhg_unrolled_ckpt_bytes(kp_plan_t plan, int K, int ckpt_every);

/* The step sizes pdhg_solve would use, as unrolled parameters: writes
 * params = device float [3K+1] (K = opts->iters) with sigma_k, tau_k,
 * theta_k of the schedule above (lambda_max from opts->lambda_max when > 0,
 * else the power method with opts->power_iters) and lambda = opts->lambda;
 * the natural initial value of learnable step sizes. */
int pdhg_schedule_params(kp_plan_t plan, const float* p, int p_kind, const kp_pdhg_opts* opts,
                         float* params, void* stream);
int pdhg_unrolled_forward(kp_plan_t plan, const void* y, const float* p, int p_kind,
                          const float* params, int K, int ckpt_every, const void* x0,
                          void* x_out, void* ckpt, void* stream);
int pdhg_unrolled_backward(kp_plan_t plan, const void* y, const float* p, int p_kind,
                           const float* params, int K, int ckpt_every, const void* x0,
                           const void* ckpt, const void* g_x, float* g_params,
                           void* g_y, void* g_x0, void* stream);

/* Release a plan after synchronising its last stream.  NULL is ignored. */
void nufft_destroy(kp_plan_t plan);

/* Host struct with the plan's sizes. */
int nufft_plan_info(kp_plan_t plan, kp_plan_info* info);

/* Copy the plan's sort to caller buffers (device int32): perm [M] (sorted
 * position -> caller sample index), bin_offsets [nbins+1] (sort tiles),
 * touch_offsets [nspread_tiles+1] and touch [ntouch] (per spreading tile, the
 * sorted sample positions whose footprint meets it, ascending).  Any pointer
 * may be NULL. */
int nufft_plan_sort(kp_plan_t plan, int32_t* perm, int32_t* bin_offsets,
                    int32_t* touch_offsets, int32_t* touch, void* stream);

/* Canonical float32 grid coordinates g [M][ndim] in caller order. */
int nufft_plan_grid_coords(kp_plan_t plan, float* g, void* stream);

/* The periodised db4 analysis filter h[8] derived by the library (host). */
int kp_db4_filter(double* h8);

/* Host-side argument validation only (no device work): returns the status
 * nufft_plan would return for these arguments before touching the device. */
int nufft_plan_validate(int ndim, const int64_t* shape, int64_t ncoils, int64_t nsamples,
                        const void* coords, const void* maps, float oversamp, int kb_width,
                        const kp_tuning* tuning);

/* Profiling aid: run one stage of the NUFFT `reps` times on the plan's own
 * workspaces (their contents are whatever the last call left), so that a
 * timer around it sees that stage alone.
 *   KP_STAGE_FWD_FFT  pre-pass + pruned forward FFT passes (d kernels)
 *   KP_STAGE_INTERP   Kaiser-Bessel interpolation into internal k-space
 *   KP_STAGE_SPREAD   tile spreading of internal k-space onto the grid
 *   KP_STAGE_ADJ_FFT  pruned inverse FFT passes + post-pass (d kernels)
 *   KP_STAGE_SPREAD_TILES  the tile kernel of KP_STAGE_SPREAD alone (split
 *                     tiles left as unreduced partial tiles)
 *   KP_STAGE_PROX     one l1-db4 proximal step of the PDHG primal update
 *                     (Preconditioned PDHG for simple regularizers, with the
 *                     l1-wavelet term: analysis, soft threshold,
 *                     synthesis, x and xbar update) on the plan's
 *                     image workspaces, with as many levels up to 4 as every
 *                     image extent allows (extents are even: at least one) */
enum { KP_STAGE_FWD_FFT = 0, KP_STAGE_INTERP = 1, KP_STAGE_SPREAD = 2, KP_STAGE_ADJ_FFT = 3,
       KP_STAGE_SPREAD_TILES = 4, KP_STAGE_PROX = 5 };
int nufft_stage(kp_plan_t plan, int stage, int reps, void* stream);

/* ---------------------------------------------------------------- batches
 * Many independent 2D reconstructions (slices) with their own image sizes
 * and trajectories, solved together: the paper treats every slice of its
 * multi-slice experiments as its own problem (Experiments), so a batch is
 * a set of independent instances of Eq. model with one coil count, one
 * oversampling and one kernel width.
 *
 * Pick tile shapes by timing candidate tilings of the spreading and
 * interpolation kernels on this problem (`best`, host struct).  Results are
 * cached per (shape, coils, sample-count class, width, oversampling), so a
 * second call for a similar slice returns at once.  Synchronises `stream`;
 * allocates and frees trial plans. */
int nufft_autotune(int ndim, const int64_t* shape, int64_t ncoils, int64_t nsamples,
                   const float* coords, const void* maps, float oversamp, int kb_width,
                   kp_tuning* best, void* stream);

/* Build one plan per slice (arguments as nufft_plan, per slice):
 *   shapes    host int64 [nslices][2]
 *   nsamples  host int64 [nslices]
 *   coords    host array of nslices device pointers, float32 [M_i][2]
 *   maps      host array of nslices device pointers c64 [C][N_i], or NULL
 *             (then C must be 1)
 *   tune      1: tile shapes from nufft_autotune per slice; 0: built-in
 * When every slice is 2D with W = 4, C a multiple of 4 and FFT lengths the
 * specialised FFT kernels cover, the solve runs each phase of an iteration
 * as ONE launch over all slices (nufft_batch_info reports it); otherwise it
 * runs slice after slice inside the same captured graph. */
int nufft_plan_batch(kp_batch_t* out, int nslices, const int64_t* shapes, const int64_t* nsamples,
                     int64_t ncoils, const float* const* coords, const void* const* maps,
                     float oversamp, int kb_width, int tune, void* stream);

/* Plan facts of one slice; *fast (may be NULL) = 1 when the one-launch-per-
 * phase path is used. */
int nufft_batch_info(kp_batch_t batch, int slice, kp_plan_info* info, int* fast);

/* l2-regularised PDHG (as pdhg_solve with reg = KP_REG_L2, no x0, u0 or
 * objective) on every slice: y, p and x_out are host arrays of nslices
 * device pointers with the per-slice layouts of pdhg_solve (p may be NULL
 * for KP_PRECOND_NONE).  p_kind applies to every slice: each p[i] must hold
 * M_i floats (SC) or C * M_i floats (MC); the library cannot check the
 * sizes behind the pointers, so a shorter buffer is read out of bounds.
 * Each slice gets its own step schedule from its
 * own lambda_max: lambda_max[i] (host float [nslices], each > 0) when the
 * array is given, else opts->lambda_max when > 0, else the power method on
 * that slice.  The K iterations are
 * captured once into a HIP graph that later calls with the same iters,
 * lambda and p_kind replay; the first call (or one that changes them)
 * allocates the graph and its descriptor tables. */
int pdhg_solve_batch(kp_batch_t batch, const void* const* y, const float* const* p, int p_kind,
                     const kp_pdhg_opts* opts, const float* lambda_max, void* const* x_out,
                     void* stream);

/* Release a batch after synchronising the device.  NULL is ignored. */
void nufft_batch_destroy(kp_batch_t batch);

/* Thread-local message of the last failure (valid until the next call). */
const char* kp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KPDHG_H */
