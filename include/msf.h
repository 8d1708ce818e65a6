/*
 * msf.h - C ABI of libmsf.so: the forward-model proximal map of multi-slice
 * fusion for 4D cone-beam CT (Majee et al., "Multi-Slice Fusion for
 * Sparse-View and Limited-Angle 4D CT Reconstruction"), built for MI355X
 * (gfx950).
 *
 * The operation (paper Sec. II, eq. (2), and Sec. III,
 * eq. (4)): for each time frame n,
 *
 *     x_n = argmin_z  1/2 || y_n - A_n z ||^2_{Lambda_n} + || v_n - z ||^2 / (2 sigma^2)
 *
 * which is the solution of (A_n^T Lambda_n A_n + sigma^-2 I) z = A_n^T Lambda_n y_n + sigma^-2 v_n.
 * The data term is separable over time frames (eq. (2)), so every
 * frame is an independent problem; the library solves all of them in one
 * batch.  A_n is the cone-beam system matrix: A_n[i][j] is the length of the
 * segment from the point source to the centre of detector pixel i inside
 * voxel j (exact ray-voxel intersection lengths, computed on the fly).
 *
 * Geometry (all lengths in voxel units, voxel side 1, origin at the volume
 * centre; the object-rotation of the paper's Sec. II is modelled as a
 * rotating source/detector pair):
 *   voxel (i,j,k) spans [i - nx/2, i + 1 - nx/2) x [j - ny/2, ...) x [k - nz/2, ...)
 *     (half-open on every axis);
 *   view angle t: source S = (src_iso cos t, src_iso sin t, 0), detector
 *     centre D0 = S + src_det (-cos t, -sin t, 0), detector axes
 *     e_u = (-sin t, cos t, 0), e_v = (0, 0, 1);
 *   pixel (iu, iv) centre = D0 + u e_u + v e_v with
 *     u = (iu - (nu-1)/2) du + det_off_u,  v = (iv - (nv-1)/2) dv + det_off_v.
 *
 * Layouts of caller arrays (FP32, contiguous, C order):
 *   volumes   [n_frames][nz][ny][nx]      (x fastest)
 *   sinograms the frames' views concatenated; frame n owns views
 *             view_offset[n] .. view_offset[n+1]-1; each view is [nv][nu]
 *             (u fastest).  Lambda (the diagonal weights) has the same layout.
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller unless
 * marked "host".  The library never frees or retains caller memory after a
 * call returns.  A plan owns all device workspace (sized at creation) and is
 * not thread-safe: calls on one plan must not overlap.  Work is enqueued on the
 * caller's HIP stream (`stream` is a hipStream_t; NULL = the default stream);
 * calls that return statistics synchronise that stream before returning.
 *
 * Errors: functions return msf_status.  On MSF_EINVAL nothing is written to
 * the outputs.  HIP runtime failures return MSF_EHIP.  msf_last_error() gives
 * a message for the last failing call on the calling thread.  No C++
 * exception crosses this interface.
 */
#ifndef MSF_H
#define MSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum msf_status {
    MSF_OK = 0,
    MSF_NOT_CONVERGED = 1,   /* warning: some frame hit max_iter; outputs and stats are valid */
    MSF_CNN_FALLBACK = 2,    /* warning: the learned start was rejected on some frame (v used) */
    MSF_EINVAL = -1,         /* invalid argument; outputs untouched */
    MSF_ENOMEM = -2,         /* device allocation failed */
    MSF_EHIP = -3,           /* HIP runtime error */
    MSF_EBREAKDOWN = -4      /* CG breakdown (<p, H p> <= 0 or non-finite) on some frame */
} msf_status;

/* Scan description.  view_offset and angles are HOST arrays, copied at plan
 * creation. */
typedef struct msf_geometry {
    int32_t nx, ny, nz;          /* voxels per frame (x fastest) */
    int32_t n_frames;            /* time frames (>= 1) */
    int32_t nu, nv;              /* detector columns (fast axis) and rows */
    double du, dv;               /* pixel pitch on the detector plane (> 0) */
    double src_iso;              /* source to rotation axis distance (> half volume diagonal) */
    double src_det;              /* source to detector distance (> src_iso) */
    double det_off_u, det_off_v; /* detector centre offset along e_u, e_v */
    const int64_t *view_offset;  /* host [n_frames + 1], non-decreasing, view_offset[0] = 0 */
    const double *angles;        /* host [view_offset[n_frames]], radians */
} msf_geometry;

typedef struct msf_plan msf_plan;
typedef struct msf_cnn msf_cnn;

/* Kernel launch shapes (chosen by the autotuner, or defaults). */
typedef struct msf_tiles {
    int32_t rays_per_lane;       /* rays of one detector column per lane: 1 to 6.  A geometry where a
                                    ray can cross two z planes inside one xy cell (rays steeper than 45 degrees
                                    over a cell diagonal) always runs 1: the plan stores 1 whatever is asked */
    int32_t waves_per_group;     /* projector workgroup size in 64-lane waves: 1, 2 or 4 */
    int32_t back_mode;           /* 0 = ray-driven scatter (FP64 atomic adds), 1 = voxel-driven gather computing
                                    each cell's line pieces on the fly, 2 = voxel-driven gather reading them from a
                                    per (view, xy cell) table built once per plan (default; n_views * nx * ny *
                                    (4 + 32 K) bytes, K = 2 or 3; the plan falls back to 1 if it cannot be allocated) */
    int32_t xcd_remap;           /* 1 = keep a frame's tiles on one XCD (L2 locality) */
} msf_tiles;

enum { MSF_X0_V = 0, MSF_X0_USER = 1, MSF_X0_CNN = 2 };

/* opts.cnn (MSF_X0_CNN): the solve computes g, predicts x0 with the network,
 * and per frame keeps the prediction only if it is finite and its residual
 * ||b - H x0|| is below that of v; otherwise the frame starts from v and the
 * call returns MSF_CNN_FALLBACK (a warning). */
typedef struct msf_solve_opts {
    double tol;                  /* stop frame n once ||b_n - H_n x_n|| <= tol ||b_n|| (recursive residual) */
    int32_t max_iter;            /* CG steps per frame (>= 0) */
    int32_t check_every;         /* host checks for all-frames-converged every this many steps (>= 1) */
    int32_t x0_mode;             /* MSF_X0_V: start from v; MSF_X0_USER: from x0; MSF_X0_CNN: from cnn */
    int32_t use_graph;           /* 1: replay each CG step as one captured hipGraph */
    int32_t true_residual;       /* 1: recompute ||b - H x|| / ||b|| at the end (one more A, A^T) */
    int32_t refine_every;        /* 0: off.  k > 0: iterative refinement.  At the start, every k CG steps
                                    (k rounded up to a multiple of check_every), and whenever every frame
                                    has frozen, the recursive residual is replaced by b - H x computed with
                                    FP64 ray-voxel lengths, an FP64 sinogram and FP64 sums, and each
                                    frame's CG restarts from it (p = r).  Between replacements CG freezes a
                                    frame at 0.1 tol on its recursive residual; a frame is accepted only
                                    when the FP64 residual meets tol (or at max_iter), and the status and
                                    converged flags judge that residual.  For stiff systems (large Lambda)
                                    whose error sits far above what the FP32 projector's rounding allows.
                                    Uses one FP64 sinogram of plan workspace (allocated on first use).
                                    true_rel_residual then reports the last FP64 residual. */
    const float *x0;             /* device [n_frames][nz][ny][nx], MSF_X0_USER only */
    const msf_cnn *cnn;          /* MSF_X0_CNN only */
} msf_solve_opts;

typedef struct msf_solve_stats {
    int32_t *iters;              /* host [n_frames] or NULL: CG steps taken per frame */
    double *rel_residual;        /* host [n_frames] or NULL: recursive ||r|| / ||b|| at exit */
    double *true_rel_residual;   /* host [n_frames] or NULL: recomputed (true_residual = 1), else -1 */
    uint8_t *converged;          /* host [n_frames] or NULL */
    uint8_t *cnn_used;           /* host [n_frames] or NULL: 1 if the learned start was kept */
    double *start_rel_residual;  /* host [n_frames] or NULL: ||b - H x0|| / ||b|| of the start used */
    int32_t steps;               /* out: CG steps launched for the batch */
    int32_t reserved;
    double seconds;              /* out: wall time of the call (host clock) */
} msf_solve_stats;

/* Fill *opts with defaults: tol 1e-6, max_iter 1000, check_every 8, start from v,
 * graphs on, no true residual, no refinement. */
void msf_solve_opts_default(msf_solve_opts *opts);

/* Create a plan for one geometry: validates it (EINVAL on non-positive sizes
 * or pitches, src_det <= src_iso, a source inside the volume's bounding
 * cylinder, bad view_offset), copies the view tables to the device and
 * allocates the solver workspace (5 volumes + 3 sinograms FP32).  *out is set
 * only on success. */
msf_status msf_plan_create(const msf_geometry *geom, msf_plan **out);

/* Release a plan and its workspace (NULL is a no-op).  Synchronises the device. */
void msf_plan_destroy(msf_plan *plan);

/* Replace / read the plan's launch shapes.  EINVAL on an unsupported shape. */
msf_status msf_plan_set_tiles(msf_plan *plan, const msf_tiles *tiles);
msf_status msf_plan_get_tiles(const msf_plan *plan, msf_tiles *tiles);

/* Autotuner: times the forward projector with the voxel-driven adjoint (HIP
 * events on the given stream, plan-owned buffers; the better of two runs
 * after a warm-up run) for every supported launch shape on this plan's
 * geometry, with the on-the-fly and the table-driven adjoint (the latter
 * with the forward's walk table), times the three fastest again (the best
 * of five runs), then the ray-driven adjoint at the best shape, and applies
 * the fastest (forward + adjoint) pair.
 * cache_path (may be NULL): text file of "key tiles" lines, key = GPU arch +
 * geometry sizes + a hash of the angle list; a hit is applied without timing,
 * a miss is appended.  chosen (host, may be NULL) receives the shape the plan
 * keeps (on a steep geometry with one ray per lane, see msf_tiles). */
msf_status msf_plan_autotune(msf_plan *plan, const char *cache_path, msf_tiles *chosen, void *stream);

/* Per-plan sizes (host outputs, any may be NULL). */
msf_status msf_plan_sizes(const msf_plan *plan, int64_t *n_vox_total, int64_t *n_meas_total,
                          int64_t *workspace_bytes);

/* y = A x for every frame (paper eq. (2)).  x: device volume
 * [n_frames][nz][ny][nx]; y: device sinogram (all views), overwritten. */
msf_status msf_project(msf_plan *plan, const float *x, float *y, void *stream);

/* x = A^T y for every frame, the exact adjoint of msf_project (same lengths).
 * y: device sinogram; x: device volume, overwritten. */
msf_status msf_backproject(msf_plan *plan, const float *y, float *x, void *stream);

/* The proximal map of the data term (paper eq. (4)) for every frame, by
 * conjugate gradients batched over frames: FP32 vectors, FP64 step sizes,
 * inner products and residual norms.  v: device volume; y, lambda: device
 * sinograms (lambda >= 0 and finite, else EINVAL); sigma > 0; x_out: device
 * volume (may alias v).  opts NULL = defaults.  stats: host, may be NULL.
 * Returns MSF_OK, MSF_NOT_CONVERGED (warning), MSF_CNN_FALLBACK (warning),
 * MSF_EBREAKDOWN (x_out holds the last iterate) or an error. */
msf_status msf_prox_solve(msf_plan *plan, const float *v, const float *y, const float *lambda, double sigma,
                          const msf_solve_opts *opts, float *x_out, msf_solve_stats *stats, void *stream);

/* The learned start's residual feature g = (b - H v) / d_n for every frame
 * (b - H v = A^T Lambda (y - A v), d_n = the frame's mean of
 * diag(A^T Lambda A) + 1/sigma^2): the input the network sees besides v
 * when msf_prox_solve runs with MSF_X0_CNN, exposed to build training data.
 * g_out: device volume [n_frames][nz][ny][nx], overwritten.  Synchronises. */
msf_status msf_prox_features(msf_plan *plan, const float *v, const float *y, const float *lambda, double sigma,
                             float *g_out, void *stream);

/* ---- the two networks (BF16 weights and activations on the matrix cores,
 * FP32 accumulation, FP32 master parameters; zero "same" padding) ----
 *
 * MSF_CNN_WARM_START (msf_cnn_create; not from the paper, plain CG decides
 * whether its prediction is kept): 3D CNN, 3x3x3 kernels, channels 2 -> 16 -> 16 ->
 * 16 -> 1, ReLU after the first three layers,
 *     x0 = v + c_o * f(v / c_v, g / c_g)
 * with g the feature above and scales (c_v, c_g, c_o).  15169 parameters:
 * per layer W[out][in][3][3][3] then b[out].
 *
 * MSF_CNN_DENOISER (msf_cnn_create_denoiser): the 2.5D denoiser of the
 * multi-slice fusion prior agents (paper Sec. IV): a 2D CNN, 3x3 kernels,
 * channels 5 -> 16 -> 16 -> 16 -> 1, ReLU after the first three layers,
 * whose five input channels are one 2D slice at the time points t-2, t-1,
 * t, t+1, t+2 and whose output is the denoised centre slice
 *     x_t = s_t + c_o * f(s_{t-2} / c_in, ..., s_{t+2} / c_in)
 * with scales (c_in, c_o).  5521 parameters: per layer W[out][in][3][3]
 * (kernel rows along the image's first axis) then b[out]. */
enum { MSF_CNN_WARM_START = 0, MSF_CNN_DENOISER = 1 };

msf_status msf_cnn_create(const float *params_host, int64_t n_params, const float *scales_host /* [3] */,
                          msf_cnn **out);
msf_status msf_cnn_create_denoiser(const float *params_host, int64_t n_params, const float *scales_host /* [2] */,
                                   msf_cnn **out);
void msf_cnn_destroy(msf_cnn *cnn);
/* MSF_CNN_WARM_START or MSF_CNN_DENOISER (-1 for NULL). */
int32_t msf_cnn_kind(const msf_cnn *cnn);
/* 15169 or 5521 (0 for NULL). */
int64_t msf_cnn_n_params(const msf_cnn *cnn);
/* Current FP32 parameters (host [msf_cnn_n_params]). */
msf_status msf_cnn_get_params(const msf_cnn *cnn, float *params_host);
/* The network on n images [nz][ny][nx] (device FP32), out x0 [n][nz][ny][nx].
 * Warm start: v and g are volumes [n][nz][ny][nx].  Denoiser: nz = 1, v is
 * the stacked input [n][5][ny][nx] (time points t-2 .. t+2) and g is
 * ignored (may be NULL); x0 = v[i][2] + c_o f. */
msf_status msf_cnn_infer(msf_cnn *cnn, const float *v, const float *g, int32_t n, int32_t nz, int32_t ny,
                         int32_t nx, float *x0, void *stream);
/* One training step on the mean squared error between x0 (inputs as in
 * msf_cnn_infer) and target (device FP32 [n][nz][ny][nx]): forward, backward
 * and, if apply, one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with
 * learning rate lr.  loss_out (host) receives the loss before the step;
 * grad_out (host [msf_cnn_n_params], may be NULL) the FP32 gradient.
 * Synchronises the stream. */
msf_status msf_cnn_train_step(msf_cnn *cnn, const float *v, const float *g, const float *target, int32_t n,
                              int32_t nz, int32_t ny, int32_t nx, double lr, int32_t apply, double *loss_out,
                              float *grad_out, void *stream);

/* One prior agent of multi-slice fusion (paper Sec. IV): H_xy,t (plane 1),
 * H_yz,t (plane 2) or H_zx,t (plane 3) applied to a 4D volume w [n_frames]
 * [nz][ny][nx] (device FP32).  Every 2D slice of the plane (images (y, x) at
 * fixed (t, z); (z, y) at fixed (t, x); (z, x) at fixed (t, y)) is replaced
 * by the denoiser's output with the same slice at t-2 .. t+2 as input, time
 * indices clamped to [0, n_frames).  cnn must be a MSF_CNN_DENOISER; out
 * (device, [n_frames][nz][ny][nx]) must not overlap w.  Asynchronous on
 * stream.  Planes 2 and 3 use two volumes of workspace that the network keeps
 * (allocated on first use and when a larger volume comes, freed by
 * msf_cnn_destroy).  Calls with one network must not overlap in time: they
 * share its activation and workspace buffers. */
msf_status msf_denoise25(msf_cnn *cnn, const float *w, int32_t n_frames, int32_t nz, int32_t ny, int32_t nx,
                         int32_t plane, float *out, void *stream);

/* ---- multi-agent consensus equilibrium around the proximal map ----
 * Algorithm 1 of the paper (partial-update Mann iteration, Sec. III):
 *     X <- F~(W; X);  Z <- G(2X - W);  W <- W + 2 rho (Z - X);  output X_0,
 * with F~ = [L~(W_0; X_0), H_1(W_1), H_2(W_2), H_3(W_3)] and G the weighted
 * average W_0/(1+beta) + beta/(1+beta) mean_k W_k (eqs. (8), (9)).
 * L~ is msf_prox_solve on W_0 started from the previous X_0: to tol (full
 * proximal map, partial_iters = 0) or for partial_iters CG steps (the paper's
 * partial update).  Prior agents: MSF_PRIOR_CNN = the paper's multi-slice
 * fusion agents H_xy,t, H_yz,t, H_zx,t (Sec. IV), msf_denoise25 in planes 1,
 * 2 and 3 with the denoiser opts.prior_cnn.  Stand-ins that are true
 * proximal maps: MSF_PRIOR_PLANE_GAUSS = the symmetric Gaussian smoother (std
 * prior_param voxels, 7 taps, zero outside) within the xy, yz and zx planes;
 * MSF_PRIOR_RIDGE = x / (1 + prior_param sigma^2), the proximal map of
 * (prior_param / 2) ||x||^2. */
enum { MSF_PRIOR_PLANE_GAUSS = 0, MSF_PRIOR_RIDGE = 1, MSF_PRIOR_CNN = 2 };

typedef struct msf_mace_opts {
    int32_t n_iter;              /* Mann iterations (10 in the paper's experiments) */
    int32_t prior;               /* MSF_PRIOR_PLANE_GAUSS, MSF_PRIOR_RIDGE or MSF_PRIOR_CNN */
    int32_t partial_iters;       /* 0: full solves; k > 0: k CG steps per outer iteration */
    int32_t max_iter;            /* CG step cap of a full solve */
    double beta;                 /* prior weight (1 = equal weighting) */
    double rho;                  /* Mann parameter in (0, 1); 0.5 = consensus ADMM */
    double prior_param;          /* Gaussian std (voxels) or ridge lambda */
    double tol;                  /* relative residual of a full solve */
    const msf_cnn *cnn;          /* optional learned start of the first solve */
    const msf_cnn *prior_cnn;    /* MSF_PRIOR_CNN: the 2.5D denoiser (a MSF_CNN_DENOISER network) */
} msf_mace_opts;

typedef struct msf_mace_stats {
    int64_t *cg_iters;           /* host [capacity] or NULL: CG steps summed over frames, per outer iteration */
    int32_t capacity;
    int32_t reserved;
    int64_t cg_total;            /* out */
    double seconds;              /* out */
} msf_mace_stats;

void msf_mace_opts_default(msf_mace_opts *opts);

/* Runs the MACE loop on the plan's 4D volume.  x_init: device volume (the
 * initial reconstruction x^(0)) or NULL for zeros; y, lambda: device
 * sinograms; x_out: device volume (the final X_0).  Allocates 9 volumes of
 * workspace for the call (11 with MSF_PRIOR_CNN).  Returns MSF_NOT_CONVERGED
 * if a full solve hit max_iter. */
msf_status msf_mace_run(msf_plan *plan, const float *x_init, const float *y, const float *lambda, double sigma,
                        const msf_mace_opts *opts, float *x_out, msf_mace_stats *stats, void *stream);

/* Live kernel timing.  While enabled, msf_prox_solve records HIP events on
 * the caller's stream around every forward-projector and backprojector launch
 * of its CG steps (also inside captured graphs) and accumulates the elapsed
 * times of the steps in which every frame was still iterating (launches that
 * processed the whole batch).  Enabling resets the accumulators. */
typedef struct msf_timing {
    double forward_ms;           /* summed duration of the timed forward-projector launches */
    int64_t forward_launches;
    double back_ms;              /* summed duration of the timed backprojector launches (with the
                                    voxel-driven adjoint this kernel also applies the CG update of x, r) */
    int64_t back_launches;
} msf_timing;
msf_status msf_plan_set_timing(msf_plan *plan, int32_t enable);
msf_status msf_plan_get_timing(const msf_plan *plan, msf_timing *out);

/* Blind fixture correction of every frame's sinogram (paper Appendix A,
 * algorithm "Blind fixture correction"), given a reconstruction x (device
 * [n_frames][nz][ny][nx], e.g. from msf_prox_solve or msf_mace_run):
 *   x_m    = x with the voxels farther than mask_radius (voxel units) from the
 *            rotation axis set to 0 (a cylinder slightly smaller than the field
 *            of view keeps the object and drops the edge artefacts);
 *   e      = y - A x_m (mostly the projection of fixtures outside the volume);
 *   p      = e blurred within each view by a separable Gaussian of std blur_std
 *            detector pixels over u and v (2 ceil(3 std) + 1 normalised taps,
 *            zero outside the detector);
 *   c_n    = <e, p> / <p, p> over frame n's sinogram (the least-squares fit;
 *            0 when p vanishes);
 *   y_corr = y - c_n p.
 * y, y_corr: device sinograms (public layout; may be the same buffer).
 * c_out: host [n_frames], may be NULL.  EINVAL for mask_radius <= 0 or
 * blur_std outside (0, 21.3].  Uses the plan's internal buffers and allocates
 * a temporary sinogram; synchronises the stream. */
msf_status msf_fixture_correct(msf_plan *plan, const float *x, const float *y, double mask_radius, double blur_std,
                               float *y_corr, double *c_out, void *stream);

/* Scratch limit of msf_fixture_correct_noalloc, in bytes (64 MiB). */
#define MSF_FIXTURE_SCRATCH_BYTES (64u << 20)

/* msf_fixture_correct for callers that cannot allocate device memory during
 * the call (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): same arguments, same results bit for bit, no
 * hipMalloc / hipFree or other allocating routine.  Its scratch (the blurred
 * sinogram, per-view inner products and per-frame fits:
 * 16 n_views + 8 n_frames + 4 n_meas bytes, each part rounded up to 256) is
 * a fixed device array of MSF_FIXTURE_SCRATCH_BYTES that each GPU holds
 * until the process ends; a geometry that needs more returns MSF_EINVAL
 * before any device work (128^3 x 16 with 192^2 x 256 views fits, 38 MB).
 * The plan (created beforehand) still provides the projector tables and its
 * internal buffers.  Call with the plan's device current.  Every call on one
 * GPU shares that GPU's scratch: calls that overlap in time on one GPU (from
 * any plan, stream or thread) race and give wrong results. */
msf_status msf_fixture_correct_noalloc(msf_plan *plan, const float *x, const float *y, double mask_radius,
                                       double blur_std, float *y_corr, double *c_out, void *stream);

/* Number of ray-voxel pieces of positive length (the nonzeros of A_n) per
 * frame, counted by the forward projector's own traversal.  per_frame: host
 * [n_frames].  Synchronises the stream. */
msf_status msf_count_intersections(msf_plan *plan, int64_t *per_frame, void *stream);

/* Message describing the last error on this thread ("" if none).  Valid until
 * the next call on the same thread. */
const char *msf_last_error(void);

/* Library version string (static storage). */
const char *msf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MSF_H */
