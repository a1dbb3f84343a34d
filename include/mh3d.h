/*
 * mh3d.h -- C ABI of the MH3D reconstruction hot path on MI355X (gfx950).
 *
 * What is computed (Sanders, Konkle, Mason, Goodwill, "Multi-Harmonic Gridded 3D
 * Deconvolution (MH3D)", arXiv 2503.13802):
 *   forward   d_k = P ( h_k (*) (b . rho) ),  k in the harmonic list
 *             -- Sec. 3.2 eq. portz / matrixModelz (z-only sensitivity, scalar b),
 *                Sec. 4.1 eq. dN (high-resolution model, final row-selector P),
 *                Table tab:ops (B Hadamard, H_k by FFT with precomputed spectrum,
 *                P a gather).  (*) is circular 3D convolution (H_k circulant).
 *   adjoint   rho = A^T d = b . sum_k h_k (x) (P^T d_k)   ((x): correlation)
 *   vector    d_k = P sum_i ( h_{k,i} (*) (b_i . rho) ) over the components i of the
 *             PSF vector and of the receive sensitivity (Sec. 3.2 eq. MH3Dcont and the
 *             stacked matrix of eq. matrixModel; App. F), user-supplied; its adjoint
 *             is sum_i b_i . sum_k h_{k,i} (x) (P^T d_k)
 *   solve     argmin_{rho >= 0} 1/2 ||A rho - d||^2 + 1/2 lambda ||T rho||^2
 *             -- Sec. 4.2 eq. Amodel with the second-order Tikhonov term, solved by
 *                the accelerated projected gradient of Sec. 4.3.
 *
 * PSF model used when no PSF array is supplied (Sec. 3.3 eq. hkapprox; the
 * transverse envelope and normalisation are readings, see the repository notes):
 *   h_k(x, y, z) = c_k L^(k + order_offset)(a x) E(r),  r = sqrt(y^2 + z^2),
 *   E(r) = L'(a r)/r (r > 0), E(0) = L'(0) * 4 asinh(1) / voxel,  ||h_k||_2 = 1,
 * with L(u) = coth u - 1/u (Sec. 2), samples at voxel centres, periodic, centred
 * at index 0, the drive axis being array axis 0 (x).
 *
 * Conventions
 *  - Volumes are FP32, C order [nx][ny][nz] (z fastest).  Portraits are FP32
 *    [n_harm][nx/ds0][ny/ds1][nz/ds2].  P keeps indices 0, ds, 2ds, ... per axis.
 *  - Every array argument is a DEVICE pointer owned by the caller, 16-byte aligned.
 *    The library never frees caller memory.  Input and output arrays must not
 *    overlap.
 *  - Calls are asynchronous on the plan's stream unless stated otherwise.
 *  - Errors are returned as mh3d_status; mh3d_last_error() gives a thread-local
 *    message.  Validation errors are detected on the host before any launch.
 *  - A plan is immutable and may be used from one host thread / stream at a time.
 */
#ifndef MH3D_H
#define MH3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MH3D_VERSION_MAJOR 0
#define MH3D_VERSION_MINOR 1

typedef enum {
  MH3D_OK = 0,
  MH3D_ERR_INVALID = 1,       /* bad argument or geometry                          */
  MH3D_ERR_UNSUPPORTED = 2,   /* valid per the paper but not built (shapes beyond the LDS budget, fold splits) */
  MH3D_ERR_OOM = 3,           /* device allocation failed                           */
  MH3D_ERR_HIP = 4,           /* a HIP runtime call failed                          */
  MH3D_ERR_NOT_CONVERGED = 5, /* solve hit max_iter before the tolerance            */
  MH3D_ERR_NONFINITE = 6      /* a reduction produced NaN/Inf                       */
} mh3d_status;

typedef struct mh3d_plan_s* mh3d_plan_t;

/* Geometry and model of one reconstruction problem. */
typedef struct {
  int32_t nx, ny, nz;        /* grid; each of the form 2^a 3^b, 4 <= n <= 256, nz even;
                                ny = 1 is a 2D image [nx][1][nz] (the projection
                                geometry of Sec. 5.2): psf required, ds[1] = 1, pad[1] = 0 */
  double voxel_mm;           /* voxel edge (mm), > 0                                     */
  int32_t ds[3];             /* decimation per axis (P), divides the grid; nz/ds2 even   */
  int32_t n_harm;            /* number of harmonics, 1..32                               */
  const int32_t* harm;       /* HOST array of harmonic indices k >= 2; strictly increasing
                                for the analytic PSF, any order with user PSFs (labels:
                                the scans of a 2D acquisition repeat them)             */
  int32_t order_offset;      /* PSF uses L^(k + order_offset); 0 by default              */
  double a_per_mm;           /* Langevin argument scale a (1/mm), > 0                    */
  const float* psf;          /* optional DEVICE [ncomp][n_harm][nx][ny][nz]; NULL -> analytic */
  const float* sens;         /* optional DEVICE [ncomp][nx][ny][nz]; NULL -> Gaussian sigma_mm */
  int32_t ncomp;             /* components of the vector model (Sec. 3.2 eq. MH3Dcont /
                                matrixModel): 0 or 1 -> scalar model; 2 or 3 -> d_k =
                                sum_i P H_{k,i} B_i rho with psf and sens both given.
                                PSF blocks h_{k,i} that are identically zero are
                                skipped; several scans of one image (Sec. 5.2) are this
                                model with one nonzero block per harmonic            */
  double sigma_mm[3];        /* Gaussian sensitivity widths (mm), peak 1 at the centre   */
  double lambda;             /* Tikhonov weight, >= 0                                    */
  int32_t reg_kind;          /* 0: stacked periodic second differences; 1: T = I         */
  double alpha;              /* boundary prior weight (eq. finalR), >= 0; 0 = off        */
  int32_t alpha_width;       /* shell depth of P_alpha in voxels: [1, min(n)/2] over the axes
                                longer than 1 if alpha > 0, else 0                      */
  int32_t pad[3];            /* boundary padding (Sec. 4.1.1): voxels of the grid on each
                                side of axis a that are modelled but not measured, a
                                multiple of ds[a].  Volumes live on the whole (padded)
                                grid; portraits cover its field of view only:
                                [n_harm][(nx-2pad0)/ds0][(ny-2pad1)/ds1][(nz-2pad2)/ds2] */
  void* stream;              /* hipStream_t all calls on this plan are enqueued on        */
} mh3d_plan_desc;

/* Solver options (Sec. 4.3). */
typedef struct {
  int32_t max_iter;          /* maximum number of updates, >= 1                          */
  double rel_tol;            /* stop after the first update with r_k <= rel_tol; 0: never */
  double tau;                /* step size; <= 0 -> 1/(1.05 L), L by power iteration,     */
                             /* computed once per plan and (power_iters, power_seed)     */
  int32_t power_iters;       /* power iterations when tau <= 0 (default 50 if 0)         */
  uint64_t power_seed;       /* Philox4x32-10 seed of the power-iteration start vector   */
  const float* rho_prev;     /* optional DEVICE rho^{k0-1} to resume; NULL -> rho_inout  */
  int32_t k0;                /* iteration counter of rho_inout (1 for a fresh start)     */
  int32_t check_every;       /* host reads the convergence flag every this many updates  */
  double* history;           /* optional HOST array receiving r_k, length history_len    */
  int32_t history_len;
} mh3d_solve_opts;

typedef struct {
  int32_t iters;             /* updates performed                                        */
  double rel_step;           /* last r_k = ||rho^{k+1} - y^k|| / ||rho^{k+1}||           */
  double tau;                /* step size used                                           */
  double lmax;               /* power-iteration estimate (0 if tau was given)            */
  float ms_total;            /* wall time of the solve on the stream (ms)                */
  float ms_per_iter;
  mh3d_status status;
} mh3d_solve_info;

/* Sizes the plan would use.  Host only: validates the descriptor and never touches
 * a GPU.  Any output pointer may be NULL. */
mh3d_status mh3d_plan_describe(const mh3d_plan_desc* desc, size_t* device_bytes,
                               int64_t* n_volume, int64_t* n_portrait);

/* Builds a plan: validates, allocates device memory, generates the PSF spectra in
 * FP64 (analytic model) or from desc->psf, and the sensitivity map.  Synchronous.
 * A plan holds its intermediate buffers and solver state, so calls on one plan must
 * not overlap (from several host threads); different plans are independent. */
mh3d_status mh3d_plan(const mh3d_plan_desc* desc, mh3d_plan_t* out);

/* Releases the plan's device memory (synchronises its stream). NULL is a no-op. */
void mh3d_destroy(mh3d_plan_t plan);

/* d = A rho (Sec. 4.1 eq. dN).  rho: [nx][ny][nz], d: [n_harm][mx][my][mz]. */
mh3d_status mh3d_forward(mh3d_plan_t plan, const float* rho, float* d);

/* rho = A^T d (adjoint of eq. dN).  d: portraits, rho: volume. */
mh3d_status mh3d_adjoint(mh3d_plan_t plan, const float* d, float* rho);

/* d = A rho and x = A^T d in one sequence of passes.  d is bitwise mh3d_forward's.
 * Without boundary padding A^T starts from the decimated spectra of d that the forward
 * pass produced (transforming d back would only reproduce them up to rounding), so x
 * equals mh3d_adjoint(d) up to that rounding.  Scalar plans run the forward and adjoint
 * class passes as one workgroup pass and write d in the launch of the adjoint plane
 * pass (three launches in all); vector plans start the adjoint class pass from d's
 * small-grid spectra (five).  With padding the pass that writes d also transforms its
 * field-of-view crop back, bitwise as mh3d_adjoint(d). */
mh3d_status mh3d_forward_adjoint(mh3d_plan_t plan, const float* rho, float* d, float* x);

/* Per-harmonic back-projections c_k = b (H_k^T P^T d_k), the terms of A^T d before
 * the sum over harmonics (adjoint of eq. dN, one harmonic at a time); sum_k c_k =
 * A^T d.  Vector model: c_k = sum_i b_i (H_{k,i}^T P^T d_k).  d: portraits, c: DEVICE
 * [n_harm][nx][ny][nz]. */
mh3d_status mh3d_backproject(mh3d_plan_t plan, const float* d, float* c);

/* Multi-harmonic anti-differentiation (App. D, eq. mhadM): the closed-form native
 * image on the portrait grid, per line along the drive axis x',
 *   rho_N^ = sum_k c_k^{-1} conj(f^)^(k-1) d_k^ / (sum_k |f^|^(2(k-1)) + lambda),
 * f the circulant central difference u[j+1] - u[j-1] (f^ = 2i sin(2 pi q / m')), with
 * the derivative order k - 1 of each harmonic (plus the plan's order_offset).  d: the
 * portraits [n_harm][mx'][my'][mz'] (field of view); c: HOST array of the n_harm
 * portrait scales c_k, or NULL for c_k = 1; lambda > 0; out: DEVICE [mx'][my'][mz'].
 * mx' must be 2^a 3^b.  Asynchronous on the plan's stream. */
mh3d_status mh3d_mhad(mh3d_plan_t plan, const float* d, double lambda, const double* c, float* out);

/* out = (A^T A + lambda T^T T) x, the normal operator of Sec. 4.3's stacked M. */
mh3d_status mh3d_normal(mh3d_plan_t plan, const float* x, float* out);

/* Power iteration on A^T A + lambda T^T T from a Philox4x32-10 uniform start vector
 * (counter (i/4, 0, 0, 0), key (seed lo, seed hi), word i%4, value (w+0.5)/2^32).
 * v_0 = x0/||x0||; w = N v; L = <v, w>; v = w/||w||, iters times.  FP32 operator
 * applications, FP64 dot products.  Writes L to *lmax (host).  Synchronous. */
mh3d_status mh3d_power_iteration(mh3d_plan_t plan, int32_t iters, uint64_t seed, double* lmax);

/* Nonnegative Tikhonov least squares by accelerated projected gradient (Sec. 4.3):
 * rho^0 = rho^1 = rho_inout (or rho_prev for rho^{k0-1}), for k = k0, k0+1, ...
 *   y^k = rho^k + (k-1)/(k+2) (rho^k - rho^{k-1}),
 *   rho^{k+1} = max(y^k - tau (A^T (A y^k - d) + lambda T^T T y^k), 0),
 * r_k = ||rho^{k+1} - y^k|| / ||rho^{k+1}|| (FP64).  On return rho_inout holds the
 * last iterate (also on MH3D_ERR_NOT_CONVERGED).  Synchronous. */
mh3d_status mh3d_solve(mh3d_plan_t plan, const float* d, float* rho_inout,
                       const mh3d_solve_opts* opts, mh3d_solve_info* info);

/* Tile shapes of the spectral passes: E spectrum elements per thread and cpw alias
 * classes per workgroup in the class passes (E in {1, 2, 3, 4, 6, 8, 9} divides
 * S = ds0 ds1 ds2 with S/E a power of two <= 64; cpw divides the class count, at
 * most 1024 threads = cpw (nx/ds0) S / E), xb decimated x-planes per
 * workgroup in the small-grid passes (divides nx/ds0; 256 threads per x'-plane, at
 * most 1024).  0 = built-in heuristic.
 * ps > 1 splits each x-plane over ps workgroups: all transform the whole plane along
 * its first axis, each takes a share of the second-axis transforms (at most
 * min(nz/2 + 1, (ny + 1)/2) workgroups).  Results do not depend on the tiles (only
 * the launch shapes change). */
typedef struct {
  int32_t E, cpw, xb;
  int32_t ps;                /* workgroups per x-plane in the plane passes: 1 to 4 */
} mh3d_tiles;
/* Sets the plan's tiles (NULL: heuristic).  Fails if a shape is invalid or does not
 * fit, or if the plan belongs to a batch.  Synchronous. */
mh3d_status mh3d_plan_set_tiles(mh3d_plan_t plan, const mh3d_tiles* tiles);
mh3d_status mh3d_plan_get_tiles(mh3d_plan_t plan, mh3d_tiles* tiles);
/* mh3d_solve without allocation, for callers that cannot allocate device memory (code
 * under stream capture, serving loops, harnesses that forbid hipMalloc): the same
 * updates, stopping rule and results as mh3d_solve with the same arguments, but the r_k
 * history that mh3d_solve keeps in a buffer it allocates on first use lives in a
 * file-scope device array of 65536 doubles (512 KiB, held by each GPU the library runs
 * on until the process ends).  No hipMalloc, hipFree or event creation; the plan's own
 * buffers (allocated by mh3d_plan) serve everything else.
 * Errors: MH3D_ERR_INVALID if opts->max_iter > 65536 or pass profiling is on (it creates
 * events), else as mh3d_solve.  info->ms_total is the call's host wall time.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (other
 * threads or streams) race, and each call overwrites the previous call's history. */
mh3d_status mh3d_solve_static(mh3d_plan_t plan, const float* d, float* rho_inout, const mh3d_solve_opts* opts,
                              mh3d_solve_info* info);

/* Pass family of the fused sequences (mh3d_forward_adjoint, mh3d_normal,
 * mh3d_power_iteration, mh3d_solve) and of the separate calls mh3d_forward,
 * mh3d_adjoint and mh3d_backproject -- the same operator (Sec. 4.1 eq. dN, Table
 * tab:ops) and solver step (Sec. 4.3) either way:
 *   1  compile-time-geometry passes, where the library has them for the plan's grid,
 *      decimation and harmonic count (scalar model, analytic PSF, no padding).  The
 *      analytic PSF is a product of an x factor per harmonic and a (y, z) factor shared
 *      by all harmonics (Sec. 2, the PSF form), so its spectra are too: a plane pass per
 *      (x-plane, y mod ds1) weights by b, transforms along z and y (the y-transform
 *      split four-step with the column pass) and folds the (y, z) aliases with the
 *      shared factor; a column pass per decimated (y, z) frequency transforms along x
 *      and applies every harmonic's x factor and x fold; the adjoint runs the same
 *      steps backwards.  The default.
 *   0  the general passes (as batches always run).
 * Results agree to FP32 rounding (the sums run in other orders).  request: 0 or 1 to
 * choose (synchronous; fails if the plan belongs to a batch), -1 to only query;
 * *active (HOST, may be NULL) receives 1 if the compile-time passes will run. */
mh3d_status mh3d_plan_path(mh3d_plan_t plan, int32_t request, int32_t* active);
/* Autotuner: times one A + A^T application (mh3d_forward_adjoint, HIP events) for candidate class tiles
 * (per valid E, the smallest cpw giving >= 64, 128, 256, 512 threads), then for
 * every small-grid xb and plane split ps with the best class tiles, each with 512 and
 * 1024 threads per workgroup in the launch that runs the adjoint plane pass beside the
 * small-grid pass writing d, and leaves the fastest on the plan.  It then times the normal operator for ps = 1, 2, 4 and keeps
 * the fastest as the plane split of the solver's passes (mh3d_normal,
 * mh3d_power_iteration, mh3d_solve run no small-grid pass, so their best split can
 * differ), which the forward plane pass of mh3d_forward_adjoint also takes (its launch
 * holds no other blocks); mh3d_plan_set_tiles sets both splits to ps, and results do not
 * depend on either.
 * A plan on the compile-time passes of mh3d_plan_path takes only xb from the tiles in
 * its own calls, but runs the general passes in a batch: it is tuned as above with those
 * passes switched off (stored under the general key), then xb alone (1, 2, 4 or 8) on
 * the compile-time A + A^T, which its "|compiled" entry keeps beside the general tiles.
 * cache_path (may be NULL): a JSON object keyed by "arch|grid|K|decimation|psf
 * kind" (plus "|compiled" for plans on the compile-time passes) with
 * E, cpw, xb, ps, ps_solve (the solver's split), tm (threads of that launch) and us; a
 * hit applies the stored tiles without timing, a miss stores the result.
 * tiles / us_per_application (HOST, may be NULL) receive the choice and its time.
 * Overwrites the plan's solver volumes; synchronous. */
mh3d_status mh3d_autotune(mh3d_plan_t plan, const char* cache_path, mh3d_tiles* tiles, double* us_per_application);

/* Batched solves of many volumes (each with its own plan: uneven grids and harmonic
 * counts allowed; analytic-PSF plans only; all on the first plan's stream).  Every
 * update of every volume runs as one launch per pass over a task table of
 * (volume, block) pairs, a chunk of updates is captured once as a hipGraph and
 * replayed, and each volume stops at its own r_k <= rel_tol (its blocks exit at
 * once afterwards).  Results equal mh3d_solve on each plan with the same options
 * (bitwise on the general passes; a plan whose own solves run the compile-time passes
 * agrees to FP32 rounding).
 * A plan may belong to one batch at a time and must not be used concurrently. */
typedef struct mh3d_batch_s* mh3d_batch_t;
mh3d_status mh3d_batch_create(int32_t n, const mh3d_plan_t* plans, mh3d_batch_t* out);
void mh3d_batch_destroy(mh3d_batch_t batch);
/* d[v], rho_inout[v]: DEVICE arrays of volume v; infos: HOST array of n (may be NULL).
 * opts applies to every volume (tau <= 0: a power iteration per volume). */
mh3d_status mh3d_solve_batch(mh3d_batch_t batch, const float* const* d, float* const* rho_inout,
                             const mh3d_solve_opts* opts, mh3d_solve_info* infos);

/* ---------------------------------------------------------------------------
 * Learned warm start (not in the paper): a 3D U-Net that maps the per-harmonic
 * back-projections c_k (mh3d_backproject) to an initial density for mh3d_solve,
 * which then refines it to the same tolerance as a cold start (Sec. 4.3 solver
 * unchanged).  BF16 weights and
 * activations, FP32 accumulation on MFMA, FP32 master weights and Adam.
 * Network: levels L, widths w_0..w_{L-1}; encoder level l = two 3x3x3 conv + ReLU,
 * 2x2x2 average pooling between levels; decoder level l = nearest 2x upsampling,
 * concatenation with the encoder output of level l, two 3x3x3 conv + ReLU; head =
 * 1x1x1 conv to one channel.  Flat FP32 parameter layout: for each layer (enc0a,
 * enc0b, ..., enc(L-1)b, dec(L-2)a, dec(L-2)b, ..., dec0b, head) the weights as
 * [Cout][tap][Cin] (tap = (dx+1)*9 + (dy+1)*3 + (dz+1)) then the bias [Cout].
 * Inputs x have C channels, channel-major [C][nx][ny][nz] (C = n_harm for the warm
 * start).  They are scaled by s = max_i |sum_c x[c][i]| (= max |A^T d| for the
 * back-projections): the network sees x/s (and targets t/s).  Grids must be powers
 * of two, at least 2^L per axis.  Calls on one network must not overlap. */
typedef struct mh3d_net_s* mh3d_net_t;
/* He-normal weights from Philox4x32-10 (key seed, stream = layer index), zero biases. */
mh3d_status mh3d_net_create(int32_t levels, const int32_t* widths, int32_t in_channels, uint64_t seed, void* stream,
                            mh3d_net_t* out);
void mh3d_net_destroy(mh3d_net_t net);
int64_t mh3d_net_param_count(mh3d_net_t net);
/* Copy the FP32 master parameters to (set = 0) or from (set = 1) a DEVICE buffer. */
mh3d_status mh3d_net_params(mh3d_net_t net, float* params, int32_t set);
/* Copy the gradient of the last mh3d_net_loss_grad to a DEVICE buffer. */
mh3d_status mh3d_net_grads(mh3d_net_t net, float* grads);
/* y = net(x / s) for DEVICE x [C][nx][ny][nz] (FP32), y [nx][ny][nz] (FP32). */
mh3d_status mh3d_net_forward(mh3d_net_t net, const float* x, int32_t nx, int32_t ny, int32_t nz, float* y);
/* Loss mean((net(x/s) - t/s)^2), t [nx][ny][nz], over a crop (HOST int[6] = offset xyz, size xyz;
 * NULL = whole volume; s over the whole volume) and its gradient (kept in the
 * network).  *loss (HOST, may be NULL) receives the loss; synchronous if given. */
mh3d_status mh3d_net_loss_grad(mh3d_net_t net, const float* x, const float* t, int32_t nx, int32_t ny, int32_t nz,
                               const int32_t* crop, double* loss);
/* One Adam step (Kingma & Ba) on the last gradient. */
mh3d_status mh3d_net_adam_step(mh3d_net_t net, float lr, float beta1, float beta2, float eps);
/* rho_init = s * max(net(c / s), 0), c = mh3d_backproject(d), s = max |A^T d|.  The
 * network has n_harm input channels; plan and net share a stream. */

mh3d_status mh3d_warm_start(mh3d_plan_t plan, mh3d_net_t net, const float* d, float* rho_init);

/* Training data on the GPU.  mh3d_phantom: n_spheres spheres (radius U(2,5) mm)
 * and n_tubes tubes (radius U(1,2.5) mm around quadratic Bezier curves with points
 * U(3, extent-3)), concentrations 10^U(-2,0), voxel-centre inclusion, drawn from
 * Philox4x32-10 (key seed, counter (j, object, 0, 0)).  mh3d_noisy_data:
 * d = A rho + sigma_k xi, sigma_k = rms_k 10^(-(snr2_db - decay_db (k-2))/20), xi
 * standard normal by Box-Muller from Philox (key seed, counter (i/2, 1, i>>33, 0)). */
mh3d_status mh3d_phantom(mh3d_plan_t plan, uint64_t seed, int32_t n_spheres, int32_t n_tubes, float* rho);
mh3d_status mh3d_noisy_data(mh3d_plan_t plan, const float* rho, uint64_t seed, double snr2_db, double decay_db,
                            float* d);

/* Copies internal plan data to a caller DEVICE buffer, for tests and tools.
 *   MH3D_FIELD_PROFILE   FP64 [n_harm][nx]      drive-axis profiles L^(k)(a x), raw
 *   MH3D_FIELD_ENVELOPE  FP64 [ny][nz]          transverse envelope E, raw
 *   MH3D_FIELD_SENS      FP32 [ncomp][nx][ny][nz]      sensitivity b
 *   MH3D_FIELD_SPECTRUM  FP32 complex [ncomp][n_harm][nx][ny][nz/2+1]  fft(h_k)
 *                        (unnormalised DFT of the PSF; the analytic one has unit norm),
 *                        read back from the plan's layout
 * *bytes receives the size needed; dst may be NULL to query it. */
typedef enum {
  MH3D_FIELD_PROFILE = 0,
  MH3D_FIELD_ENVELOPE = 1,
  MH3D_FIELD_SENS = 2,
  MH3D_FIELD_SPECTRUM = 3
} mh3d_field;
mh3d_status mh3d_plan_export(mh3d_plan_t plan, mh3d_field field, void* dst, size_t* bytes);

/* Per-kernel timing with HIP events around every launch of the plan's kernels
 * (enable = 1 starts and clears, 0 stops).  mh3d_profile_read synchronises and
 * returns the cumulative milliseconds and launch counts per kernel id, plus names. */
#define MH3D_NKERNEL 11
typedef struct {
  double ms[MH3D_NKERNEL];
  int64_t launches[MH3D_NKERNEL];
  const char* name[MH3D_NKERNEL];
} mh3d_profile_data;
mh3d_status mh3d_profile(mh3d_plan_t plan, int32_t enable);
mh3d_status mh3d_profile_read(mh3d_plan_t plan, mh3d_profile_data* out);
/* Average microseconds per launch of one pass (0 plane_fwd, 1 class_fwd, 2 small_inv,
 * 3 small_fwd, 4 class_adj, 5 plane_adj, 6 class_normal: the forward and adjoint class
 * passes in one, 7 adj_and_store: the adjoint plane pass and the small-grid inverse pass
 * in one launch, both as mh3d_forward_adjoint runs them; 6 and 7 give
 * MH3D_ERR_UNSUPPORTED for plans of the vector model or with boundary padding, which
 * keep the passes apart) over reps
 * back-to-back launches between two HIP events on the plan's stream, after one A and
 * A^T to set its inputs.  Overwrites the plan's solver volumes; profiling must be off;
 * synchronous. */
mh3d_status mh3d_time_pass(mh3d_plan_t plan, int32_t pass, int32_t reps, double* us);

/* One Philox4x32-10 block computed on the device (known-answer checks of the
 * generator used by mh3d_power_iteration).  ctr[4], key[2], out[4] are HOST
 * arrays.  Synchronous. */
mh3d_status mh3d_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out);

/* Thread-local text of the last error (never NULL). */
const char* mh3d_last_error(void);

/* Library version as MAJOR*100 + MINOR. */
int32_t mh3d_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MH3D_H */
