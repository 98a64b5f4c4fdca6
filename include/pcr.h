/*
 * pcr.h -- C ABI of the MI355X (gfx950) library for volumetric image
 * reconstruction and tumour localisation from a single cone-beam x-ray
 * projection under a PCA lung-motion model (Li et al., "Real-time volumetric
 * image reconstruction and 3D tumor localization based on a single x-ray
 * projection image for lung cancer radiotherapy").
 *
 * Method (section 2): the deformation x = mean + U w (eq. (1), eq. (2)
 * constraint) warps the reference image f0 by trilinear interpolation
 * (pull-back, f(p) = f0(p + x(p))); the cost J = |P f - a y - b|^2 (eq. (2))
 * is minimised by alternating gradient descent on w with an Armijo line
 * search (eq. (3)) and the closed-form fit of (a, b) (eq. (4)); the gradient
 * is 2 U^T (df/dx)^T P^T (P f - a y - b); the tumour position is the inverse
 * (push-forward) deformation of its reference position (section 2.3).
 *
 * Conventions shared by every entry point:
 *   - All functions are extern "C", never throw, and return a pcr_status.
 *     On failure a description is available from pcr_last_error() (a
 *     thread-local string valid until the next call on the same thread).
 *   - Pointers named *_dev are device (HBM) pointers owned by the caller
 *     (e.g. torch tensors); *_host pointers and plain double* scalars are
 *     host memory.  The library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; the call returns without synchronising unless
 *     it has to return host values (cost, gradient, solver results,
 *     tumour position), in which case it synchronises that stream only.
 *   - Volumes are [nz][ny][nx] (x fastest, flat index i + nx*(j + ny*k)),
 *     the grid origin is the centre of voxel (0,0,0) in mm.
 *   - DVFs are pull-back displacements in mm, structure of arrays [3][N]
 *     (x, y, z components, N = nx*ny*nz).  Eigenvector fields are
 *     [K][3][N].  Projections are [nv][nu] (u fastest).
 *   - Cone-beam geometry: rotation about z through the isocentre; source
 *     iso + (SAD sin t, -SAD cos t, 0), detector centre
 *     iso + (-(SDD-SAD) sin t, (SDD-SAD) cos t, 0), detector axes
 *     e_u = (cos t, sin t, 0), e_v = (0, 0, 1); pixel (iu, iv) centre
 *     c + ((iu-(nu-1)/2) du + off_u) e_u + ((iv-(nv-1)/2) dv + off_v) e_v.
 *   - The projection P samples every ray at t = n*step_mm from the source
 *     (all integers n whose sample lies between source and pixel) with
 *     trilinear interpolation, the image being zero outside its grid, and
 *     returns step_mm * (sum of the samples).  P^T is its exact transpose.
 *   - Compute precision is PCR_F32 or PCR_F64; the reference image and the
 *     motion model may additionally be stored as PCR_BF16 or PCR_F16 (read
 *     and widened to the compute type).  Detector-wide and volume-wide
 *     reductions (cost, regression sums, gradient) accumulate in FP64.
 *   - Inputs are validated before any launch: null pointers, non-positive
 *     sizes or spacings, impossible geometry and non-finite host scalars
 *     return PCR_EINVAL and enqueue nothing.
 *   - Size limit of FP32 compute: the FP32 ray march addresses its zero-padded
 *     image, (nx+3)(ny+3)(nz+3) cells of C FP32 channels, with 32-bit byte
 *     offsets.  That image must stay below 2 GiB (with padded rows below
 *     16 MiB and (ny+3)(nz+3), (nx+3)(nz+3) below 2^24 cells).  C = 1 for
 *     pcr_forward_project; C = K + 1 rounded up to 2, 4, 6 or 8 for contexts and
 *     server streams.  A larger grid returns PCR_EINVAL from
 *     pcr_forward_project, pcr_ctx_create, pcr_cost_grad,
 *     pcr_reconstruct_from_projection and pcr_server_add_stream before any
 *     launch.  FP64 compute has no such limit.
 */
#ifndef PCR_H
#define PCR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pcr_status;
#define PCR_OK 0
#define PCR_EINVAL (-1)    /* bad shape, dtype, geometry, option or null pointer */
#define PCR_ENOMEM (-2)    /* device or host allocation failed */
#define PCR_EDEVICE (-3)   /* HIP runtime error (details in pcr_last_error) */
#define PCR_ENOCONV (-4)   /* line search exhausted or iteration cap hit before the
                              gradient tolerance; outputs hold the last accepted iterate */
#define PCR_EDIVERGE (-5)  /* fixed point did not converge; last iterate returned */
#define PCR_EBUSY (-6)     /* serving admission refused (memory budget or slots) */

typedef enum pcr_dtype { PCR_F32 = 0, PCR_F64 = 1, PCR_BF16 = 2, PCR_F16 = 3 } pcr_dtype;

typedef struct pcr_grid {
    int32_t n[3];          /* nx, ny, nz (> 0) */
    double spacing_mm[3];  /* voxel size (> 0) */
    double origin_mm[3];   /* centre of voxel (0,0,0) */
} pcr_grid;

typedef struct pcr_geom {
    double angle_rad;      /* gantry angle t */
    double sad_mm;         /* source-isocentre distance (> 0) */
    double sdd_mm;         /* source-detector distance (> sad_mm) */
    int32_t nu, nv;        /* detector columns and rows (> 0) */
    double du_mm, dv_mm;   /* pixel pitch at the detector plane (> 0) */
    double off_u_mm, off_v_mm; /* detector offsets along e_u, e_v */
    double step_mm;        /* ray sample spacing (> 0) */
    double iso_mm[3];      /* isocentre position */
} pcr_geom;

/* PCA motion model, eq. (1): x = mean + sum_k scale_k w_k U_k.  `mean` is
 * [3][N] and `U` is [K][3][N], both device pointers of dtype `storage`
 * (F32, F64, BF16 or F16).  `scale` is a host array [K] (NULL = all 1): a
 * field stored divided by scale_k (FP16 storage keeps |U_k| <= 1 so that
 * small entries stay out of the subnormal range). */
typedef struct pcr_model {
    int32_t K;             /* 1..8 */
    pcr_dtype storage;
    const void* mean;
    const void* U;
    const double* scale;
} pcr_model;

/* Gradient evaluation in the solver and in pcr_cost_grad. */
#define PCR_GRAD_FUSED 0   /* d J/d w_k = 2 <r, P h_k> with h_k = (df/dx) . u_k: one
                              (K+1)-channel ray march returns J and the gradient at
                              any (a, b) -- the same number as the adjoint form */
#define PCR_GRAD_ADJOINT 1 /* the paper's order: g = P^T (2r) by scatter, then
                              sum_v g[v] (df/dx)[v] . u_k[v] */

/* Options of the alternating algorithm (section 2.2).  The paper fixes the
 * structure (Armijo's rule on w with a, b fixed; closed-form a, b; stop on a
 * small gradient or an iteration cap); the constants are this library's:
 * defaults from pcr_solve_opts_default(). */
typedef struct pcr_solve_opts {
    int32_t max_iter;        /* iteration cap (default 50) */
    int32_t max_backtracks;  /* Armijo trials per iteration (default 30) */
    double sigma;            /* sufficient decrease: accept J' <= J - sigma mu |g|^2 (1e-4) */
    double beta;             /* step shrink per rejected trial (0.5) */
    double eps_g;            /* stop when |g_n| <= eps_g |g_0| (1e-4) */
    double step0;            /* first trial of a solve moves w by this distance (> 0);
                                a later iteration's first trial: see step_rule */
    double fixed_mu;         /* > 0: constant step mu, no line search (default 0) */
    int32_t grad_mode;       /* PCR_GRAD_FUSED (default) or PCR_GRAD_ADJOINT */
    int32_t localize;        /* nonzero: localise the tumour after the solve */
    double p_ref_mm[3];      /* tumour position in the reference image */
    double fp_tol_mm;        /* fixed-point stop: update shorter than this (1e-6) */
    int32_t fp_max_iter;     /* fixed-point iteration cap (200) */
    double mu0;              /* > 0: step size of the solve's first trial instead of
                                step0 / |g_0| -- e.g. the `mu` a previous frame's solve
                                returned, which carries the line search's scale across
                                warm-started frames (default 0) */
    int32_t step_rule;       /* first trial of each later iteration (Armijo's rule,
                                section 2.2, leaves it open): PCR_STEP_SECANT (default)
                                s.y / y.y, with s the last accepted step in w and y the
                                change of the gradient over it; PCR_STEP_QUADRATIC (or
                                the secant rule when s.y <= 0): the minimiser of the
                                quadratic through the previous line's J, slope -|g|^2
                                and accepted J', clamped to [beta, 1/beta] x the
                                accepted step */
} pcr_solve_opts;

#define PCR_STEP_SECANT 0
#define PCR_STEP_QUADRATIC 1

typedef struct pcr_solve_stats {
    int32_t status;          /* same as the return value */
    int32_t iterations;      /* accepted gradient steps */
    int32_t trials;          /* line-search trials (projections of a trial w) */
    int32_t fp_iterations;   /* fixed-point iterations of the localisation */
    int32_t fp_status;       /* PCR_OK or PCR_EDIVERGE */
    double J0, J;            /* cost after the first step 2, and at the result */
    double gnorm0, gnorm;    /* |dJ/dw| at the start and at the result */
    double a, b;             /* intensity fit at the result */
    double tumor_mm[3];      /* localised tumour position (if requested) */
    double samples;          /* ray samples marched over all projections of the solve
                                (rays are clipped to the box where the warped image
                                can be nonzero, so this is the work done) */
    double mu;               /* step size the next iteration would have tried first */
} pcr_solve_stats;

typedef struct pcr_ctx pcr_ctx;

/* ------------------------------------------------------------------------ */
const char* pcr_version(void);
const char* pcr_last_error(void);
void pcr_solve_opts_default(pcr_solve_opts* opts);

/* DVF composition (eq. (2) constraint, eq. (1)): dvf = mean + U (scale * w).
 * w_host[K] host doubles; dvf_dev [3][N] of dtype `compute` (F32 or F64),
 * overwritten. */
pcr_status pcr_dvf_compose(const pcr_grid* grid, const pcr_model* model,
                           const double* w_host, pcr_dtype compute, void* dvf_dev,
                           void* stream);

/* Pull-back warp (sections 2.2-2.3): f[v] = T[f0](v + dvf[v] / spacing),
 * trilinear, f0 = 0 outside its grid.  f0_dev [N] of dtype f0_dtype (any);
 * dvf_dev [3][N] and f_dev [N] of dtype `compute` (F32 or F64); f_dev is
 * overwritten and must not alias f0_dev. */
pcr_status pcr_warp_volume(const pcr_grid* grid, pcr_dtype f0_dtype, const void* f0_dev,
                           pcr_dtype compute, const void* dvf_dev, void* f_dev,
                           void* stream);

/* Transpose of the warp as a linear map of the reference image (the
 * gradient with respect to f0): out = W^T g.  dvf_dev [3][N], g_dev [N],
 * out_dev [N], all of dtype `compute`; out_dev is overwritten.  Uses
 * floating-point atomics: the summation order, hence the last bits, may
 * vary between runs. */
pcr_status pcr_warp_adjoint(const pcr_grid* grid, pcr_dtype compute, const void* dvf_dev,
                            const void* g_dev, void* out_dev, void* stream);

/* Gradient contraction (section 2.2: the U^T (df/dx)^T factors of the
 * gradient): grad_host[k] = scale_k * sum_v g[v] sum_a (df/dx_a)[v] U_k[a][v],
 * where df/dx is the exact derivative of the trilinear warp of f0 at the
 * displaced point of voxel v for the DVF mean + U (scale * w).  g_dev [N] of
 * dtype `compute`; f0_dev of dtype f0_dtype; FP64 accumulation in a fixed
 * order (bitwise reproducible).  Synchronises `stream`. */
pcr_status pcr_warp_contract(const pcr_grid* grid, const pcr_model* model, pcr_dtype f0_dtype,
                             const void* f0_dev, const double* w_host, pcr_dtype compute,
                             const void* g_dev, double* grad_host, void* stream);

/* Forward projection P vol (eq. (2)'s projection matrix, discretised as in
 * the conventions above).  vol_dev [N] and proj_dev [nv][nu] of dtype
 * `compute` (F32 or F64); proj_dev is overwritten.  Allocates a padded
 * device copy of the volume per call (library-owned scratch, reused). */
pcr_status pcr_forward_project(const pcr_grid* grid, const pcr_geom* geom,
                               pcr_dtype compute, const void* vol_dev, void* proj_dev,
                               void* stream);

/* Forward projection that allocates nothing, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, kernels and result
 * (bitwise) as pcr_forward_project, but the zero-padded copy of the volume,
 * (nx+3)(ny+3)(nz+3) cells of 4 (F32) or 8 (F64) bytes, lives in one fixed
 * library-owned device array of PCR_NOALLOC_SCRATCH_BYTES per GPU instead of
 * a per-thread allocation.  The array is part of the library's code object:
 * each GPU the library runs on holds it until the process ends; its device
 * address is looked up once per GPU on the first call there.  A grid whose
 * padded copy exceeds the array returns PCR_EINVAL before any launch.  Every
 * call on one GPU shares the array (and clears and refills it): calls that
 * overlap on one GPU (other host threads, or streams not ordered with each
 * other) race and give undefined projections.  Not timed by the kernel
 * profiler (pcr_profile_enable), which records events. */
#define PCR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
pcr_status pcr_forward_project_noalloc(const pcr_grid* grid, const pcr_geom* geom,
                                       pcr_dtype compute, const void* vol_dev, void* proj_dev,
                                       void* stream);

/* Backprojection P^T resid, the exact transpose of pcr_forward_project (the
 * P^T of the gradient formula in section 2.2; no factor 2).  resid_dev
 * [nv][nu], vol_dev [N] of dtype `compute`; vol_dev is overwritten.  A
 * gather: each voxel sums the weights of the samples near it in a fixed
 * order, so the result is deterministic (no atomics). */
pcr_status pcr_backproject_residual(const pcr_grid* grid, const pcr_geom* geom,
                                    pcr_dtype compute, const void* resid_dev,
                                    void* vol_dev, void* stream);

/* Solver context: binds a grid, a motion model and a reference image (all
 * caller-owned device memory that must outlive the context) and owns the
 * device scratch of the solve (a zero-padded multi-channel copy of the warped
 * image, reduction partials, pinned host staging).  compute = F32 or F64.
 * One context per host thread; calls on one context must not overlap. */
pcr_status pcr_ctx_create(const pcr_grid* grid, const pcr_model* model, pcr_dtype f0_dtype,
                          const void* f0_dev, pcr_dtype compute, pcr_ctx** out);
void pcr_ctx_destroy(pcr_ctx* ctx);
/* Bytes of device memory the context holds. */
size_t pcr_ctx_device_bytes(const pcr_ctx* ctx);
/* Element type of the context's fused image (the warped image and its K
 * tangent images that each trial marches): PCR_F32 (default) or PCR_F16
 * (FP32 compute only; each channel scaled by a power of two so that nothing
 * overflows).  FP16 halves the bytes the march gathers per sample, but its
 * rounding of the tangents adds gradient noise proportional to the residual,
 * which slows the relative-gradient stop when the model cannot fit the data.
 * Returns PCR_EINVAL for other types or FP64 compute. */
pcr_status pcr_ctx_set_image_dtype(pcr_ctx* ctx, pcr_dtype dtype);

/* Cost J(w, a, b) (eq. (2)) and its gradient dJ/dw (section 2.2, with the
 * factor 2) for the measured projection y_dev [nv][nu] (dtype = the
 * context's compute dtype) at geometry `geom`.  grad_host[K].  grad_mode is
 * PCR_GRAD_FUSED or PCR_GRAD_ADJOINT.  Synchronises `stream`. */
pcr_status pcr_cost_grad(pcr_ctx* ctx, const void* y_dev, const pcr_geom* geom,
                         const double* w_host, double a, double b, int32_t grad_mode,
                         double* cost_host, double* grad_host, void* stream);

/* One per-projection solve (section 2.2): (a, b) from step 2 at the warm
 * start w_inout, then alternate Armijo gradient steps on w and step 2 until
 * |g| <= eps_g |g_0|, max_iter, or line-search exhaustion; optionally
 * localise the tumour (section 2.3).  w_inout[K] is the warm start on entry
 * (section 4: the previous frame's w) and the result on exit; ab_out[2]
 * (may be NULL); stats may be NULL.  Returns PCR_OK or PCR_ENOCONV (result
 * still valid) or an error.  Synchronises `stream` once per line-search
 * trial. */
pcr_status pcr_reconstruct_from_projection(pcr_ctx* ctx, const void* y_dev,
                                           const pcr_geom* geom, const pcr_solve_opts* opts,
                                           double* w_inout, double* ab_out,
                                           pcr_solve_stats* stats, void* stream);

/* PCA training of the motion model (section 2.1, eq. (1); section 3): from J
 * training DVFs dvfs_dev [J][3][N] (FP32, mm), writes mean_dev [3][N] =
 * their average and U_dev [K][3][N] = the K leading left singular vectors of
 * the centred 3N x J matrix (unit norm; each flipped so that its first entry
 * within 1e-5 relative of its largest magnitude is positive), and on the host
 * sing_host[K] (singular values) and w_train_host [J][K] (training
 * coefficients <U_k, d_j - mean>), either may be NULL.  2 <= J <= 16,
 * 1 <= K <= min(8, J - 1).  The Gram matrix accumulates in FP64; the
 * eigen-solve is FP64 on the host.  Synchronises `stream`. */
pcr_status pcr_pca_train(const pcr_grid* grid, int32_t J, const float* dvfs_dev, int32_t K,
                         float* mean_dev, float* U_dev, double* sing_host, double* w_train_host,
                         void* stream);

/* Initial guess from history (section 5: the PCA coefficients predicted from
 * previous frames serve as the initial guess, useful when the imaging rate is
 * low).  w_hist [n][K] are previous results at times t_hist [n] (seconds,
 * strictly increasing); w_out[K] = the polynomial of degree
 * min(order, n - 1) through the last min(order, n - 1) + 1 points, evaluated
 * at t_next (order 0: the last result, the plain warm start; 1: linear
 * extrapolation; 2: quadratic).  Host only; no device work. */
pcr_status pcr_predict_w(const double* w_hist, const double* t_hist, int32_t n, int32_t K,
                         double t_next, int32_t order, double* w_out);

/* Tumour localisation (section 2.3): the point p with p + x(p) = p_ref for
 * the pull-back DVF x = mean + U (scale * w), by the fixed-point iteration
 * p <- p_ref - x(p) (Chen et al., the paper's ref. 13) evaluated at that
 * point only, in FP64 on the device, x interpolated trilinearly with
 * clamp-to-edge.  Stops when the update is shorter than tol_mm or after
 * max_iter iterations (then PCR_EDIVERGE with the last iterate).  iters may
 * be NULL.  Synchronises `stream`. */
pcr_status pcr_localize_tumor(const pcr_grid* grid, const pcr_model* model,
                              const double* w_host, const double p_ref_mm[3], double tol_mm,
                              int32_t max_iter, double p_out_mm[3], int32_t* iters,
                              void* stream);

/* ------------------------------------------------------------------------
 * Serving engine: continuous batching of per-projection solves for many
 * patient streams (each with its own grid, motion model, reference image,
 * detector and warm-started w).  A worker thread keeps up to max_slots solves
 * in flight, one HIP stream each; every solve advances by one line-search
 * trial per turn and new requests take slots as soon as solves finish, so
 * requests that arrive while others run overlap with them on the device.
 * Each solve runs exactly the steps of pcr_reconstruct_from_projection
 * (fused gradient, deterministic reductions): its result is bitwise the same
 * alone and in the mix.  Warm start (section 4): each stream's next solve
 * starts from its previous result.
 * ------------------------------------------------------------------------ */
typedef struct pcr_server pcr_server;

typedef struct pcr_server_opts {
    size_t hbm_budget_bytes;  /* server-owned device memory limit: stream copies of
                                 reference images and models plus per-slot scratch */
    int32_t max_slots;        /* solves in flight at once (1..64) */
    int32_t drop_stale;       /* nonzero: a queued (not yet started) request is dropped
                                 when a newer one of the same stream arrives */
    int32_t predict_order;    /* warm start of each solve: 0 = the stream's previous
                                 result; 1, 2 = pcr_predict_w over the stream's last
                                 results at their submit times */
    int32_t chain_step;       /* nonzero: each solve's first trial uses the step size
                                 the stream's previous solve ended with (opts.mu0).
                                 Not with predict_order > 0: a carried step taken
                                 from an extrapolated start can carry w into the
                                 cost's degenerate minimum (the object moved out of
                                 view, P f = 0, a = b = 0, J = 0) */
    int32_t image_f16;        /* nonzero: FP16 fused images (see pcr_ctx_set_image_dtype) */
    int32_t carry_move;       /* nonzero: each solve's first trial moves w by the distance
                                 the stream's previous solve moved it (from its start to
                                 its result), kept within [1e-3, 1] x the stream's step0;
                                 scale-free, and the first trial that suits a predicted
                                 start (predict_order > 0), whose error is about the
                                 previous prediction's.  Not with chain_step */
} pcr_server_opts;

typedef struct pcr_result {
    int64_t req_id;
    int32_t stream_id;
    int32_t status;           /* solve status (PCR_OK / PCR_ENOCONV / error), or
                                 PCR_EBUSY when the request was dropped as stale */
    int32_t iterations, trials, K, fp_status;
    double w0[8];             /* warm start the solve began from */
    double w[8];              /* result */
    double ab[2], J, tumor_mm[3];
    double t_submit_s, t_start_s, t_done_s;   /* steady-clock seconds */
    double mu0, mu;           /* step size of the first trial, and the one the solve
                                 ended with (see pcr_solve_opts.mu0) */
    double samples;           /* ray samples marched over all projections of the
                                 solve (the work it took; see pcr_solve_stats) */
    double step0;             /* distance the first trial was to move w (pcr_solve_opts.step0;
                                 0 when mu0 set the first trial) */
} pcr_result;

/* Creates the server and its worker thread on the current device. */
pcr_status pcr_server_create(const pcr_server_opts* opts, pcr_server** out);
/* Stops the worker (in-flight solves finish first) and frees all memory. */
void pcr_server_destroy(pcr_server* srv);
/* Registers a stream: copies f0 [N] (f0_dtype) and the model (mean, U, scale)
 * from the caller's device memory into server-owned memory, so the caller may
 * free its copies.  opts: solve options of every request of the stream
 * (grad_mode must be PCR_GRAD_FUSED; compute is FP32); w0: first warm start.
 * Admission by HBM footprint: PCR_EBUSY (nothing allocated) when the stream's
 * copies plus per-slot scratch large enough for every admitted grid would
 * exceed hbm_budget_bytes.  Synchronises the copies. */
pcr_status pcr_server_add_stream(pcr_server* srv, const pcr_grid* grid, const pcr_model* model,
                                 pcr_dtype f0_dtype, const void* f0_dev,
                                 const pcr_solve_opts* opts, const double* w0,
                                 int32_t* stream_id);
/* Removes a stream once its queued and in-flight requests are done or dropped. */
pcr_status pcr_server_remove_stream(pcr_server* srv, int32_t stream_id);
/* Queues one projection y_dev [nv][nu] FP32 at geometry `geom` for the stream.
 * y_dev is not copied: it must stay valid until the request's result has been
 * polled.  Returns the request id. */
pcr_status pcr_server_submit(pcr_server* srv, int32_t stream_id, const void* y_dev,
                             const pcr_geom* geom, int64_t* req_id);
/* Moves up to max finished results to out[] (oldest first); waits up to
 * wait_ms for at least one when none is ready.  *n = number written. */
pcr_status pcr_server_poll(pcr_server* srv, pcr_result* out, int32_t max, int32_t* n,
                           int32_t wait_ms);
/* Waits until no request is queued or in flight (timeout_ms < 0: forever);
 * PCR_EBUSY on timeout. */
pcr_status pcr_server_drain(pcr_server* srv, int32_t timeout_ms);
/* Snapshot / restore of a stream's warm start (checkpoint of the serving
 * state; the model itself is re-registered from its source). */
pcr_status pcr_server_get_w(pcr_server* srv, int32_t stream_id, double* w_out);
pcr_status pcr_server_set_w(pcr_server* srv, int32_t stream_id, const double* w);
/* Device bytes held (stream copies + slot scratch) and budget accounting. */
size_t pcr_server_device_bytes(const pcr_server* srv);

/* Opt-in kernel timing (tracing).  While enabled, every kernel the library
 * launches is bracketed by two HIP events on the stream it runs on.  Enabling
 * resets the totals.  pcr_profile_read resolves pending events (waiting for
 * them), fills up to `max` entries of names (static strings), total_ms and
 * counts (any may be NULL) and returns the number of kernel kinds.  Global to
 * the process; thread-safe. */
void pcr_profile_enable(int32_t on);
int32_t pcr_profile_read(int32_t max, const char** names, double* total_ms, int64_t* counts);
/* Restricts that timing to the kernel kinds whose bit is set in `mask` (bit
 * i: the i-th name pcr_profile_read reports; all bits set by default), so
 * that timing the dominant kernel leaves the others' launches free of event
 * records.  Global to the process; thread-safe. */
void pcr_profile_select(uint32_t mask);

#ifdef __cplusplus
}
#endif
#endif /* PCR_H */
