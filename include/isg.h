/*
 * isg.h - C ABI of the MI355X (gfx950) image-space gridding / nonrigid SENSE
 * library.
 *
 * The library computes, on one GPU, the operators of Jang, Malave and
 * Nishimura, "Image-Space Gridding for Nonrigid Motion-Corrected MR Image
 * Reconstruction" (arXiv:2501.16713):
 *
 *   T_d    forward image-space gridding, the warp m(r + d(r))   (Eq. 5, Eq. 9)
 *   T_d^H  adjoint image-space gridding                          (Eq. 7, Eq. 8)
 *   A_p    nonrigid SENSE operator G_p S T_{d_p}                 (Eq. 10, Figs. 2-3)
 *   A_p^H  its adjoint T_{d_p}^H S^H G_p^H                       (Fig. 3b)
 *   N      sum_p A_p^H A_p + lambda I, the l2 normal operator of Eq. 11
 *   CG     conjugate gradients on N x = sum_p A_p^H y_p
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Every call returns an isg_status; ISG_OK is 0.  No C++ exception crosses
 * the ABI.  On any other status isg_last_error() returns a message for the
 * calling thread.  Arguments are validated before anything is enqueued, so a
 * validation error leaves every output untouched.
 *
 * Device buffers are plain device pointers owned by the caller; they must stay
 * valid until the plan's stream has passed the call.  The library owns plans,
 * motions, trajectories and everything derived from them (tap tables, tile
 * bins, FFT twiddles, deapodization tables, scratch grids) and frees them in
 * the matching *_destroy call.
 *
 * Apply calls (warp, warp_adjoint, warp_grad_d, sense_*, normal) are
 * asynchronous on the plan's stream.  *_create calls are synchronous with
 * respect to their input buffers: the caller may reuse them on return.
 * isg_cg_solve synchronizes the stream before it returns.
 *
 * A plan is not thread-safe.  Different plans may run concurrently on
 * different streams.  A device error makes the plan fail every later call
 * with ISG_ERR_STATE until it is destroyed.
 *
 * Layouts (C order, slowest index first)
 *   image  x      complex64 (interleaved float re, im) [n0][n1][n2]   (2D: [n0][n1])
 *   field  d      float32 [ndim][n0][n1][n2], in voxels; component i
 *                 displaces along array axis i; pull convention: the warped
 *                 image at voxel r is the object at r + d(r)              (Eq. 5)
 *   coils  S      complex64 [C][n0][n1][n2]
 *   traj   k      float32 [M][ndim] in cycles/voxel, in [-0.5, 0.5);
 *                 component i is along array axis i; image voxel index j
 *                 sits at the centred position j - n/2
 *   data   y      complex64, states packed one after another; state p holds
 *                 [M_p][C] (sample-major, coils contiguous).  Sample-major
 *                 rather than coil-major ([C][M_p]): one set of 4^ndim
 *                 kernel weights per sample serves its C contiguous coil
 *                 values in one coalesced access, in the gather and the
 *                 spread alike.  Every apply call takes the number of
 *                 states P it is given (at most the plan's nphases) and P
 *                 motion and trajectory handles.
 *
 * Numerics: Kaiser-Bessel kernel of width 4 on a 2x oversampled periodic
 * grid, beta = pi*sqrt(4*(1.5)^2 - 0.8); FP32 arithmetic (FP64 for the
 * k-space coordinates at plan time and for the CG inner products and
 * scalars).  The k-space pair is scaled so that G approximates the
 * orthonormal NDFT |N|^{-1/2} sum_x z[x] exp(-2 pi i k.x); T is scaled so that
 * T_0 approximates the identity.
 */
#ifndef ISG_H
#define ISG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ISG_OK = 0,
  ISG_ERR_INVALID_ARG = 1,       /* null pointer, bad count, bad enum, size mismatch */
  ISG_ERR_UNSUPPORTED_SHAPE = 2, /* n_i not even, < 8, > 512, or with a prime factor > 7;
                                    alpha != 2, width != 4, beta > 0 and not the default;
                                    ncoils * 2 * n_last > 8192 */
  ISG_ERR_OUT_OF_MEMORY = 3,     /* a device or host allocation failed */
  ISG_ERR_DEVICE = 4,            /* no usable GPU, or a HIP runtime error */
  ISG_ERR_NOT_FINITE = 5,        /* NaN/Inf in a displacement field or trajectory */
  ISG_ERR_CG_BREAKDOWN = 6,      /* Re<p, N p> <= 0 or non-finite during CG */
  ISG_ERR_STATE = 7              /* plan previously hit a device error */
} isg_status;

/* Element type of the coil-expanded oversampled k-space grids (the
 * precision form: FP32 arithmetic in registers and LDS, results rounded to
 * nearest-even on every grid store; image-space arrays, data and CG scalars
 * are unaffected).  Half-precision grids are scaled by powers of two only,
 * so results are exactly proportional to the input: every operator call
 * scales its image input by 2^-e with 2^(e-1) <= rms < 2^e before the coil
 * expansion, and each state's spread output by 2^e' chosen from the data's
 * largest component and a per-trajectory bound on the samples reaching one
 * grid cell (the spread output then stays below 1024 in magnitude); both are
 * undone at the coil reduction or the gather output.  Both scales are
 * computed on the device (one extra reduction per call), so graph replay is
 * unaffected.  Relative error against the exact operator: about 1e-4 (FP16)
 * and 2e-3 (BF16) per result. */
typedef enum {
  ISG_STORE_FP32 = 0,
  ISG_STORE_BF16 = 1,
  ISG_STORE_FP16 = 2
} isg_storage;

typedef struct isg_plan isg_plan;     /* shape, tables, scratch; library-owned */
typedef struct isg_motion isg_motion; /* prepared displacement field d_p       */
typedef struct isg_traj isg_traj;     /* prepared trajectory k_p               */

/* Plan description.  Shapes: each n_i even, 8 <= n_i <= 512, prime factors
 * in {2, 3, 5, 7} (lengths whose factors are 2, 3 and 5 only, and whose
 * oversampled length is one of 32, 40, 48, 64, 80, 96, 128, 160, 192, 256,
 * 320, 512, run the faster two-step register FFT; the others the general
 * LDS Stockham passes).  The coil passes hold all C coils of a line in one
 * workgroup, so ncoils * 2 * n_last <= 8192.  The interpolation kernel is
 * fixed to Kaiser-Bessel of width 4 on a 2x oversampled grid (the operators'
 * tables and tap loops are built for it): alpha and width must be given as
 * 2 and 4, and beta as <= 0 (meaning pi sqrt((W/alpha)^2 (alpha - 1/2)^2 -
 * 0.8) = 8.99615...) or that value itself. */
typedef struct {
  int ndim;            /* 2 or 3 */
  int64_t n[3];        /* image shape; n[2] ignored when ndim == 2 */
  int alpha;           /* oversampling factor G_i / n_i: must be 2 */
  int width;           /* kernel width W in oversampled cells (taps per axis): must be 4 */
  double beta;         /* Kaiser-Bessel shape parameter; <= 0: the default */
  int ncoils;          /* C >= 1 (1..32) */
  int nphases;         /* P >= 1: most states one call may pass */
  isg_storage storage; /* storage of the coil-expanded k-space grids */
  void* stream;        /* hipStream_t to enqueue on; NULL = the null stream */
} isg_plan_desc;

/* Library version string, e.g. "isg 0.1 gfx950".  Never fails. */
const char* isg_version(void);

/* Message for the calling thread's last non-OK status ("" if none). */
const char* isg_last_error(void);

/* Number of visible GPUs in *count (0 on a host without one: ISG_OK). */
isg_status isg_device_count(int* count);

/* Create a plan: validates the shape, builds twiddle and deapodization
 * tables and allocates the scratch the operators need.  Errors:
 * INVALID_ARG, UNSUPPORTED_SHAPE, DEVICE (no GPU), OUT_OF_MEMORY. */
isg_status isg_plan_create(const isg_plan_desc* desc, isg_plan** plan);
/* Destroy a plan (synchronizes its stream).  Motions and trajectories
 * prepared on it may be destroyed before or after it: those still alive are
 * detached, keep their own device memory until their own destroy call, and
 * fail every apply call (INVALID_ARG: no plan). */
isg_status isg_plan_destroy(isg_plan* plan);
/* Change the stream later calls enqueue on. */
isg_status isg_plan_set_stream(isg_plan* plan, void* stream);
/* Device bytes the plan currently holds. */
isg_status isg_plan_device_bytes(const isg_plan* plan, int64_t* bytes);

/* Per-kernel timing for profiling.  With enable != 0 every kernel launch
 * whose tag starts with `prefix` ("" or NULL = every launch) is bracketed
 * by HIP events on the plan's stream; enabling or disabling clears the
 * totals.  Tags name the operator stage, e.g. "fft_coil_fwd_ax0",
 * "kgather", "warp_spread". */
isg_status isg_plan_set_timing(isg_plan* plan, int enable, const char* prefix);
/* Write the totals as JSON {"tag": [launches, total_ms], ...} into buf (len
 * bytes, NUL-terminated).  Waits for the recorded events.  INVALID_ARG if
 * buf is too small. */
isg_status isg_plan_read_timing(isg_plan* plan, char* buf, int64_t len);

/* Tunable execution options of a plan.  None of them changes the result
 * beyond floating-point summation order.
 *   ISG_OPT_SPREAD_CHUNK  samples per k-space spread work unit (tiles with
 *                         more samples are split and their partial tiles
 *                         summed in a fixed order); 32..65536, default 512;
 *                         applies to trajectories prepared (or re-tuned) later
 *   ISG_OPT_PHASE_BATCH   states whose k-space gather and spread run as one
 *                         launch (each state keeps its own grid, so device
 *                         memory grows by one coil-expanded grid per state);
 *                         1..16, default 1
 *   ISG_OPT_GRAPH         1: isg_normal captures its kernel sequence in a HIP
 *                         graph and replays it while its arguments stay the
 *                         same (not on the null stream, not while timing);
 *                         default 0
 *   ISG_OPT_KTILE_T1      extent along axis 1 of the k-space spread tiles
 *                         (4, 8 or 16; default 8 in 3D, 16 in 2D).  Smaller
 *                         tiles follow sparse trajectories more closely (the
 *                         axis-0 passes skip untouched tiles) at more
 *                         sample visits.  Trajectories prepared for another
 *                         extent fail with ISG_ERR_STATE until re-created or
 *                         passed to isg_plan_tune.
 *   ISG_OPT_KBLOCK        layout of the coil-expanded k-space arrays in 3D:
 *                         b in 1..6 keeps blocks of 2^b consecutive rows of
 *                         axis 1 together for each index of axis 0 (the
 *                         axis-0 FFT passes then step 2^b G2 C elements
 *                         rather than G1 G2 C); 0 is plain row-major.
 *                         Default 3; plain where 2^b does not divide G1 or
 *                         a length has no register FFT.  Internal arrays
 *                         only: no input or output layout changes.
 *   ISG_OPT_FFT_ADDR      1 (default): the FFT passes whose lengths and
 *                         layouts allow it address memory through buffer
 *                         resources (a scalar base per tile and element
 *                         index, one 32-bit offset per lane, untouched or
 *                         invalid elements masked by the hardware's
 *                         out-of-range rule); 0: 64-bit addresses computed
 *                         per lane and element everywhere.  Same results
 *                         bit for bit. */
typedef enum {
  ISG_OPT_SPREAD_CHUNK = 1,
  ISG_OPT_PHASE_BATCH = 2,
  ISG_OPT_GRAPH = 3,
  ISG_OPT_KTILE_T1 = 4,
  ISG_OPT_KBLOCK = 5,
  ISG_OPT_FFT_ADDR = 6
} isg_option;

/* Set / read an option.  INVALID_ARG for an unknown option or a value out of
 * range. */
isg_status isg_plan_set_option(isg_plan* plan, isg_option option, int64_t value);
isg_status isg_plan_get_option(const isg_plan* plan, isg_option option, int64_t* value);

/* Autotuner: times the normal operator sum_p A_p^H A_p x + lambda x on the
 * given inputs for candidate k-space array blockings, k-space tile extents,
 * spread chunk sizes, phase
 * batch sizes and graph replay (a coordinate search, each candidate the best
 * of `reps` timed applications after one warm-up, ending with the blockings
 * next to the chosen one under the other chosen options), keeps the fastest setting
 * in the plan and re-prepares the given trajectories for it (others prepared
 * on this plan must be re-created if the tile extent changed).  Candidates that do not
 * fit in device memory are skipped.  report (host, may be NULL) receives a
 * JSON object {"candidates": [{"kblock", "ktile_t1", "chunk", "batch", "graph",
 * "ms"}...],
 * "chosen": {...}} (NUL-terminated, truncated to len bytes).  Synchronizes
 * the stream. */
isg_status isg_plan_tune(isg_plan* plan, int nphases, const void* x, const isg_motion* const* d,
                         const void* S, isg_traj* const* k, double lambda, int reps, char* report,
                         int64_t len);

/* Prepare a displacement field d (device float32 [ndim][n...], voxels) for
 * T_d / T_d^H (Eq. 5): a copy of d and the voxel lists per tile of the
 * spreading adjoint, binned on the device on the plan's stream (a stable sort
 * by tile, so the adjoint sums in the same order on every call).  Returns
 * after the work completes (the caller may free d); only the 4-byte result of
 * the field check is copied to the host.  NOT_FINITE if d holds NaN/Inf,
 * INVALID_ARG if some |d| exceeds 1e6 voxels. */
isg_status isg_motion_create(isg_plan* plan, const float* d, isg_motion** motion);
isg_status isg_motion_destroy(isg_motion* motion);

/* Prepare a trajectory k (device float32 [M][ndim], cycles/voxel) for the
 * k-space pair (Eq. 1-3): grid coordinates G*k in FP64, split into an integer
 * tap base and an FP32 fraction, and tile bins for the spread.  Points outside
 * [-0.5, 0.5) wrap periodically.  M >= 1.  NOT_FINITE on NaN/Inf. */
isg_status isg_traj_create(isg_plan* plan, const float* k, int64_t M, isg_traj** traj);
isg_status isg_traj_destroy(isg_traj* traj);
isg_status isg_traj_count(const isg_traj* traj, int64_t* M);
/* Spread bookkeeping of a prepared trajectory: the number of (sample, tile)
 * visits, of k-space spread tiles any sample touches, and of grid points per
 * tile (for traffic accounting). */
isg_status isg_traj_info(const isg_traj* traj, int64_t* nvisits, int64_t* ntiles, int64_t* tile_points);
/* Grid cells (per coil) the axis-0 passes store in the forward direction
 * and read in the adjoint one: the runs of cells along axis 0 (of the k-space
 * tile extent along axis 0) that some sample's taps reach, per grid column;
 * 0 when the path keeps no such masks (every cell is then touched). */
isg_status isg_traj_touched_cells(const isg_traj* traj, int64_t* cells);
/* Grid columns (i1, i2) along axis 0 that hold at least one touched run: the
 * lines the axis-0 passes transform (all others are skipped); 0 when the
 * path keeps no such masks. */
isg_status isg_traj_active_columns(const isg_traj* traj, int64_t* cols);

/* y = T_d x, forward image-space gridding (Eq. 9).  x, y: device complex64
 * images; out-of-place (x != y). */
isg_status isg_warp(isg_plan* plan, const isg_motion* d, const void* x, void* y);

/* x = T_d^H y, adjoint image-space gridding (Eq. 7-8); out-of-place. */
isg_status isg_warp_adjoint(isg_plan* plan, const isg_motion* d, const void* y, void* x);

/* x = T_d^H y exactly as isg_warp_adjoint computes it (same kernels, same
 * result bit for bit), for callers that cannot allocate device memory while
 * they run: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The call allocates nothing: the oversampled grid
 * the spread's tile regions and the FFT intermediates live in one fixed
 * 64 MiB device array of the library (held on every GPU the library runs on
 * until the process ends), which fits about 290 |N| bytes in 3D and 100 |N|
 * in 2D: every 2D shape, 3D up to about 60^3 voxels.  Larger shapes fail
 * with INVALID_ARG (use isg_warp_adjoint).  The plan's device must be current.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams or threads, without ordering between them) race
 * and give wrong results.  Asynchronous on the plan's stream. */
isg_status isg_warp_adjoint_noalloc(isg_plan* plan, const isg_motion* d, const void* y, void* x);

/* grad[i][r] = Re(conj(v[r]) * d(T_d x)[r] / d d_i[r]): the gradient of
 * Re<v, T_d x> with respect to the displacement field, which is what a
 * registration or motion-refinement loss needs by the chain rule.
 * x, v: device complex64 images; grad: device float32 [ndim][n...]. */
isg_status isg_warp_grad_d(isg_plan* plan, const isg_motion* d, const void* x, const void* v,
                           float* grad);

/* y = [A_0; ...; A_{P-1}] x, the stacked nonrigid SENSE model (Eq. 10):
 * for each state p, coil c and sample j, y_p[j][c] = (G_p (S_c . T_{d_p} x))_j.
 * d, k: arrays of P handles; S: device complex64 [C][n...]; y: device,
 * sum_p M_p * C complex64 values. */
isg_status isg_sense_forward(isg_plan* plan, int nphases, const void* x,
                             const isg_motion* const* d, const void* S,
                             const isg_traj* const* k, void* y);

/* x = sum_p A_p^H y_p = sum_p T_{d_p}^H sum_c conj(S_c) . G_p^H y_{p,c} (Fig. 3b). */
isg_status isg_sense_adjoint(isg_plan* plan, int nphases, const void* y,
                             const isg_motion* const* d, const void* S,
                             const isg_traj* const* k, void* x);

/* out = sum_p A_p^H A_p x + lambda x (l2 form of Eq. 11); out != x. */
isg_status isg_normal(isg_plan* plan, int nphases, const void* x, double lambda,
                      const isg_motion* const* d, const void* S,
                      const isg_traj* const* k, void* out);

/* Gradients of the data term L = sum_p 1/2 ||A_p x - y_p||^2 given the
 * residual r = A x - y (device, packed like y):
 *   grad_x = sum_p A_p^H r_p                                   (complex64 [n...])
 *   grad_d[p][i][v] = Re(conj(v_p[v]) * d(T_{d_p} x)[v] / d d_{p,i}[v])
 *       with v_p = sum_c conj(S_c) . G_p^H r_{p,c}             (float32 [P][ndim][n...])
 * by the chain rule through the linear maps S and G_p.  Either output may
 * be NULL (not computed), not both.  grad_x != x. */
isg_status isg_sense_grad(isg_plan* plan, int nphases, const void* x, const isg_motion* const* d,
                          const void* S, const isg_traj* const* k, const void* r, void* grad_x,
                          float* grad_d);

/* Conjugate gradients on (sum_p A_p^H A_p + lambda I) x = sum_p A_p^H y_p:
 * exactly `iters` Hestenes-Stiefel iterations from the x passed in (x is
 * read as x0 and overwritten with x_iters), FP64 inner products and scalars
 * kept on the device.  resnorm (host, may be NULL) receives iters + 1 values
 * ||r_0|| .. ||r_iters||.  Synchronizes the stream.  CG_BREAKDOWN if
 * Re<p, N p> <= 0 or is not finite (x then holds the last good iterate). */
isg_status isg_cg_solve(isg_plan* plan, int nphases, const void* y,
                        const isg_motion* const* d, const void* S,
                        const isg_traj* const* k, double lambda, int iters,
                        void* x, double* resnorm);

/* ---------------------------------------------------------------------------
 * Reconstruction layer around the operators
 * ------------------------------------------------------------------------- */

/* Translate the object during the samples of a trajectory (bulk motion;
 * section "Motion Capturing for Segmented Data Acquisitions"): t (device
 * float32 [M][ndim], voxels, component i along array axis i), or NULL to
 * remove a translation set before.  Sample j of every forward model that
 * uses the trajectory is multiplied by exp(-2 pi i k_j . t_j) (the linear
 * phase of a shifted object), and the adjoints by its conjugate (which
 * corrects data acquired from a shifted object by the linear phase shift);
 * normal operators are unchanged (the phases cancel).  The phase is formed
 * in FP64.  Synchronous. */
isg_status isg_traj_set_shift(isg_traj* traj, const float* t);

/* Density compensation weights of a trajectory by the iteration of Pipe and
 * Menon: w = 1, then `iters` times w <- w / (P w), (P w)_j = sum_l w_l
 * sum_q c(kappa_j - q) c(kappa_l - q) with the interpolation kernel scaled
 * to unit integral per axis (a spread of the weights onto the oversampled
 * grid and a gather at the samples).  w: device float32 [M].  The spread
 * sums with atomic adds, so the last bits vary from run to run.
 * Synchronous. */
isg_status isg_traj_dcf(isg_plan* plan, const isg_traj* traj, int iters, float* w);

/* Direct k-space gridding reconstruction (Eq. 1-2 with the "density
 * corrected" data of the notation table), coil-combined:
 * x = sum_c conj(S_c) . G^H(w . conj(ph) . y_c), with w the weights (device
 * float32 [M], NULL: 1) and ph the trajectory's translation phases (if
 * set).  y: device complex64 [M][C]; x: device complex64 image.  A plan of
 * a lower resolution and a trajectory of the samples near the k-space origin
 * (k rescaled to that plan's cycles/voxel) give the low-resolution image
 * navigator of the paper's motion capture. */
isg_status isg_grid_recon(isg_plan* plan, const isg_traj* traj, const void* y, const float* w, const void* S,
                          void* x);

/* Orthonormal Haar wavelet transform W (the sparsifying transform of Eq. 11
 * and Eq. 13): `levels` levels of the separable one-dimensional map
 * (a, b) -> ((a + b)/sqrt2, (a - b)/sqrt2) along every axis, the Mallat
 * layout (low-pass band first along every axis, each level on the previous
 * level's low-pass box).  Every n_i must be divisible by 2^levels
 * (INVALID_ARG otherwise; levels 1..9).  x, w: device complex64 images,
 * out-of-place.  W^H = W^{-1}. */
isg_status isg_wavelet_forward(isg_plan* plan, int levels, const void* x, void* w);
isg_status isg_wavelet_inverse(isg_plan* plan, int levels, const void* w, void* x);

/* Largest eigenvalue of sum_p A_p^H A_p (isg_power_iteration) or of T_d^H
 * T_d (isg_warp_power_iteration) by the power method from the caller's
 * start vector v (device complex64 image, overwritten with the last unit
 * iterate): v <- N v / ||N v||, `iters` times; *lmax = ||N v|| of the last
 * step (host).  Twice lmax, or more, is the Lipschitz constant FISTA
 * needs.  NOT_FINITE if ||N v|| is zero or not finite.  Synchronizes. */
isg_status isg_power_iteration(isg_plan* plan, int nphases, const isg_motion* const* d, const void* S,
                               const isg_traj* const* k, int iters, void* v, double* lmax);
isg_status isg_warp_power_iteration(isg_plan* plan, const isg_motion* d, int iters, void* v, double* lmax);

/* Wavelet-FISTA (Beck and Teboulle) with constant step 1/L for
 *   min_x ||y - A x||^2 + lambda ||W x||_1                         (Eq. 11)
 * over the stacked nonrigid SENSE operators, and for
 *   min_p ||q - T_d p||^2 + lambda ||W p||_1                       (Eq. 13)
 * (isg_warp_fista_solve, Appendix 1): x_k = W^H S(W(z_k - (2/L)(A^H A z_k -
 * A^H y))), S the complex soft threshold at lambda/L of every detail
 * coefficient (the approximation coefficients are not penalised), t_{k+1} =
 * (1 + sqrt(1 + 4 t_k^2))/2, z_{k+1} = x_k + ((t_k - 1)/t_{k+1})(x_k - x_{k-1});
 * z_1 = x_0 = the x passed in, overwritten with x_iters.  lipschitz = L
 * must be at least 2 lambda_max(A^H A) (see the power iteration).
 * change (host, may be NULL) receives ||x_k - x_{k-1}|| for k = 1..iters.
 * Synchronizes. */
isg_status isg_fista_solve(isg_plan* plan, int nphases, const void* y, const isg_motion* const* d, const void* S,
                           const isg_traj* const* k, double lambda, double lipschitz, int levels, int iters, void* x,
                           double* change);
isg_status isg_warp_fista_solve(isg_plan* plan, const isg_motion* d, const void* q, double lambda, double lipschitz,
                                int levels, int iters, void* p, double* change);

/* Appendix 1, l2 form of Eq. 13: conjugate gradients on (T_d^H T_d +
 * lambda I) p = T_d^H q, exactly `iters` iterations from the p passed in
 * (overwritten with p_iters); resnorm (host, may be NULL) receives
 * ||r_0|| .. ||r_iters||.  The naive inverse of Fig. 10a is isg_warp with a
 * motion prepared from -d.  Synchronizes; CG_BREAKDOWN as isg_cg_solve. */
isg_status isg_warp_cg_solve(isg_plan* plan, const isg_motion* d, const void* q, double lambda, int iters, void* p,
                             double* resnorm);

/* Nonrigid registration by gradient descent with T_d as the warp (the
 * gradient-based alternative to the demons step of section "Nonrigid
 * Respiratory Motion Correction"): minimises
 *   E(d) = ||T_d ref - mov||^2 + mu sum_i sum_a ||D_a d_i||^2,
 * D_a the periodic forward difference along axis a, by d <- d - step
 * grad E(d), `iters` times; grad E = 2 Re(conj(T_d ref - mov) dT_d ref/dd)
 * + 2 mu (-Laplacian d).  ref, mov: device complex64 images; d: device
 * float32 [ndim][n...] (voxels), the start on entry and d_iters on return;
 * energy (host, may be NULL) receives E(d_0) .. E(d_iters).  No motion
 * handle is needed (the field is read directly).  Synchronizes. */
isg_status isg_register(isg_plan* plan, const void* ref, const void* mov, double mu, double step, int iters,
                        float* d, double* energy);

#ifdef __cplusplus
}
#endif

#endif /* ISG_H */
