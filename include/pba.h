/*
 * pba.h -- C ABI of the MI355X photometric bundle-adjustment library (libpba.so).
 *
 * The library evaluates, for every ordered keyframe pair (s, t) -- the paper's
 * <i, j>, where the cloud of image i is warped into image j -- the multi-cue
 * photometric residuals of every source pixel with valid depth, their Huber
 * weights and SE(3) Jacobians, reduces them into the 6N x 6N normal equations
 * H dx = -b over all N poses, solves for the Gauss-Newton / Levenberg-Marquardt
 * step in FP64 and applies it as X <- X exp(dx).  All of it runs in HIP kernels
 * on one GPU; the host only marshals arguments.
 *
 * Definitions followed (paper "Photometric LiDAR and RGB-D Bundle Adjustment"):
 *   poses, inverse, projections pi_p / pi_s            Sec. III (Basics)
 *   warp u' = pi(R_j^T (R_i pi^-1(u, d) + t_i - t_j))     Sec. IV-C, Eq. (uprime)
 *   objective F = sum rho(|stacked cue residual|^2_Omega)  Sec. IV-C, Eq. (total-error-multicue)
 *   perturbation dx = [dt, dq], X boxplus dx = X exp(dx)  Supplementary (first paragraph)
 *   sensor offset, p_u, p_bar and all Jacobians           Supplementary
 *
 * Conventions (all arrays row-major, C order):
 *   pose      12 doubles: R (3x3 row-major) then t; maps platform -> world.
 *   offset    12 doubles, same layout; maps sensor -> platform.
 *   images    [H][W] float32 per keyframe: intensity and depth (pinhole: depth
 *             along the optical axis; spherical: range).  normals [H][W][3]
 *             float32, sensor frame.  Pixel (col u, row v) has integer
 *             coordinates at its centre.
 *   pinhole   pixel u looks along ((u-cx)/fx, (v-cy)/fy, 1).
 *   spherical pixel u looks along (cos el cos az, cos el sin az, sin el) with
 *             az = (u-cx)/fx, el = (v-cy)/fy.
 *   dx        6N doubles, per pose [dt (3), dq (3)]; dq is the imaginary part
 *             of a unit quaternion, so a rotation by angle a has |dq| = sin(a/2).
 *
 * Ownership: every input is copied during the call; the library never keeps a
 * caller pointer.  Outputs are caller-allocated.  `on_device` arguments say
 * whether a caller pointer is device memory (1) or host memory (0).
 *
 * Errors: every call returns a pba_status; no C++ exception crosses the ABI.
 * On error the context state is unchanged and pba_last_error() describes it.
 *
 * Streams: work is ordered on the stream given in pba_config (a borrowed
 * hipStream_t; NULL = the null stream).  Calls that return host values
 * synchronise that stream.  A context is not thread-safe.
 */
#ifndef PBA_H
#define PBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pba_ctx pba_ctx;
typedef int32_t pba_status;

enum {
    PBA_OK = 0,
    PBA_EINVAL = -1,     /* bad argument: ids, sizes, NaN or non-orthonormal pose, shape mismatch */
    PBA_ENOMEM = -2,     /* device allocation failed */
    PBA_EDEVICE = -3,    /* HIP runtime error */
    PBA_ESTATE = -4,     /* call out of order (e.g. evaluate before poses and pairs are set) */
    PBA_ENOTPD = -5,     /* Gauss-Newton system not positive definite (lambda = 0) */
    PBA_ENOVALID = -6    /* no valid correspondence at all */
};

enum { PBA_PINHOLE = 0, PBA_SPHERICAL = 1 };
enum { PBA_F32 = 0, PBA_F64 = 1 };
/* Elimination order of the pose system's Cholesky factorisation (pba_config.solve_order). */
enum { PBA_ORDER_AUTO = 0, PBA_ORDER_NATURAL = 1, PBA_ORDER_ND = 2 };

/* Length of one per-pair record written by pba_evaluate (pair_out):
 * [0,144)  H12, 12x12 row-major over [dx_s (6); dx_t (6)]
 * [144,156) b12
 * 156 F (sum of rho), 157 evaluated source pixels, 158 valid correspondences, 159 boundary-band
 * correspondences (see pba_eval_out.n_boundary_band). */
#define PBA_PAIR_OUT_LEN 160

/* A sensor model (Sec. III) and its rigid offset on the platform (Supplementary). */
typedef struct {
    int32_t model;               /* PBA_PINHOLE or PBA_SPHERICAL */
    int32_t height, width;       /* image size H, W: >= 4 each, H * W * W < 2^32, H * W <= 2^26 */
    int32_t pad;
    double fx, fy, cx, cy;       /* K: focal / angular resolution and offsets, in pixels */
    double min_depth, max_depth; /* valid depth (pinhole) or range (spherical) interval, metres */
    double offset[12];           /* sensor -> platform, R row-major then t */
} pba_sensor;

typedef struct {
    int32_t device;              /* HIP device ordinal */
    int32_t precision;           /* PBA_F32: residual/Jacobian/H path in FP32 (solve FP64);
                                    PBA_F64: the same kernels instantiated in FP64 */
    int32_t channels;            /* 2: intensity + depth; 5: + normal xyz */
    int32_t grad_mode;           /* image Jacobian: 0 = central differences at the 4 bilinear taps,
                                    blended bilinearly (Supplementary); 1 = slope of the bilinear
                                    interpolant (exact derivative of the sampled image) */
    int32_t anchor;              /* pose held fixed (gauge) */
    int32_t use_graph;           /* 1: pba_iterate replays one captured HIP graph per iteration;
                                    0: launches the same kernels one by one */
    void *stream;                /* borrowed hipStream_t, NULL = null stream */
    double omega_intensity, omega_depth, omega_normal;  /* Omega^c, scalar per cue */
    double huber_delta;          /* Huber threshold on sqrt(chi^2); <= 0: plain squares */
    double occlusion_tau_pinhole, occlusion_tau_spherical;
    /* every stencil tap's depth must be within tau of the predicted depth (Sec. IV-C,
       occlusion suppression), chosen by the target sensor's model */
    int32_t occlusion_zbuffer;   /* 1: also drop a point lying more than tau behind the nearest of
                                    the pair's own warped source points whose integer cell floor(u')
                                    is the same (a z-buffer of the pair's source points, depths as
                                    FP32; Sec. IV-C occlusion suppression, z-buffer reading).  Costs
                                    one projection-only pass over every pair per evaluation and
                                    4 bytes per target pixel per pair of device memory; 0: off */
    int32_t storage_bf16;        /* 1: intensity and normal images are kept on the device in BF16 (rounded
                                    to nearest even when loaded, and when the pyramid or normal estimation
                                    writes them); residuals, Jacobians and sums stay FP32/FP64.  FP32 path
                                    only, without occlusion_zbuffer, and pba_loss_backward is then
                                    PBA_EINVAL; 0: FP32 images */
    int32_t solve_order;         /* elimination order of the damped system's Cholesky factorisation (the
                                    solve of Sec. IV's Gauss-Newton / Levenberg-Marquardt step; the step
                                    is the same up to rounding in every order):
                                    PBA_ORDER_NATURAL: pose order, one dependent step per 64-row block
                                    column; PBA_ORDER_ND: nested dissection of the pose graph, each
                                    dissection block padded to 64 rows, one step per elimination-tree
                                    level; PBA_ORDER_AUTO (default): nested dissection when it at least
                                    halves the number of dependent steps and at most doubles the
                                    system's order (the factor takes 24 n^2 bytes at order n) */
    /* Device memory of the context (images, plans, systems, work buffers) comes from these
     * callbacks when both are set (e.g. a framework's caching allocator), else from hipMalloc.
     * dev_alloc(bytes, alloc_user) returns device memory of cfg->device usable on cfg->stream, or
     * NULL (the call then fails with PBA_ENOMEM); dev_free(ptr, bytes, alloc_user) returns it.
     * Both must stay callable until pba_destroy returns; setting only one is PBA_EINVAL. */
    void *(*dev_alloc)(size_t bytes, void *alloc_user);
    void (*dev_free)(void *ptr, size_t bytes, void *alloc_user);
    void *alloc_user;
} pba_config;

/* Fill *cfg with defaults: F32, 5 channels, grad_mode 0, anchor 0, graphs on, Omega 1,
 * Huber 0.1, tau 0.5 m (pinhole) / 1.0 m (spherical), no z-buffer, FP32 images, automatic
 * solve order. */
void pba_config_default(pba_config *cfg);

/* Create a context on cfg->device.  *out receives the handle.  PBA_EINVAL for an unknown
 * precision, channel count or grad_mode, a negative anchor, negative or non-finite Omega,
 * non-finite Huber threshold, tau <= 0 or an unknown solve_order; PBA_EDEVICE for a device
 * that does not exist. */
pba_status pba_create(const pba_config *cfg, pba_ctx **out);
pba_status pba_destroy(pba_ctx *ctx);

/* Register a sensor; *sensor_id receives its index (0, 1, ...).  Before any keyframe is loaded.
 * PBA_EINVAL for an image size outside 4 <= H, W, H W^2 < 2^32, H W <= 2^26, non-finite or zero
 * intrinsics, a bad depth interval or offset, and for a spherical sensor finer than 1550 px/rad
 * (|fx| or |fy|; a full turn in about 9700 columns): the evaluation's first projection, which
 * names the table rays of the exact one, must land within a pixel. */
pba_status pba_add_sensor(pba_ctx *ctx, const pba_sensor *sensor, int32_t *sensor_id);

/* Load n keyframes: per keyframe its sensor id and pointers to its intensity [H][W], depth [H][W]
 * and normals [H][W][3] (normals may be NULL when channels == 2).  Depth outside [min_depth,
 * max_depth] or not finite marks the pixel invalid.  If n and every keyframe's sensor equal the
 * loaded ones, only the images are replaced and poses and pairs are kept; otherwise poses and
 * pairs must be set again. */
pba_status pba_load_keyframes(pba_ctx *ctx, int32_t n, const int32_t *sensor_id,
                              const float *const *intensity, const float *const *depth,
                              const float *const *normals, int32_t on_device);

/* Poses of all n keyframes (n must equal the number loaded), or of the n pose variables after
 * pba_set_pose_groups.  Rejects non-finite values and rotations with max |R^T R - I| > 1e-6. */
pba_status pba_set_poses(pba_ctx *ctx, int32_t n, const double *poses, int32_t on_device);
pba_status pba_get_poses(pba_ctx *ctx, double *poses, int32_t on_device);

/* Keyframes that share one pose variable (the sensors of one rig frame, each with its own offset:
 * the coupled LiDAR + RGB-D formulation of the fusion experiments).  pose_of[k] in [0, n_poses)
 * for each of the N loaded keyframes, every variable used by at least one keyframe; pose_of = NULL
 * restores one pose per keyframe.  Afterwards poses, steps and pose gradients have n_poses
 * entries: pba_set_poses must be called again, and the anchor is a pose variable.  A pair inside
 * one variable contributes all four of its 6 x 6 blocks to that variable (its Jacobians cancel).
 * Loading a different keyframe set resets the grouping.  Errors: PBA_EINVAL for a bad map,
 * PBA_ESTATE before keyframes are loaded. */
pba_status pba_set_pose_groups(pba_ctx *ctx, const int32_t *pose_of, int32_t n_poses);

/* Ordered pairs (src[k] -> tgt[k]); ids in [0, n).  Replaces any previous set. */
pba_status pba_set_pairs(pba_ctx *ctx, int32_t p, const int32_t *src, const int32_t *tgt);

typedef struct {
    double F;                    /* sum over pairs and pixels of rho(chi^2) */
    int64_t n_evaluated;         /* (pair, source pixel with valid depth) evaluations */
    int64_t n_valid;             /* valid correspondences */
    int64_t n_boundary_band;     /* projected points whose stencil lies inside the target image and
                                    whose coordinate u' (column or row) is within 1e-4 px of a cell
                                    boundary: the integer cell floor(u') that decides the taps and
                                    the mask (readings of Sec. IV-C's sampling) is then sensitive to
                                    rounding, so such points may legitimately differ between the FP32
                                    and FP64 paths or from an exact evaluation */
    double *H;                   /* nullable: 6N x 6N, raw (no gauge fix, no damping) */
    double *b;                   /* nullable: 6N */
    double *pair_out;            /* nullable: P x PBA_PAIR_OUT_LEN, in the platform frames */
    int32_t on_device;           /* whether H, b, pair_out are device pointers */
    int32_t pad;
} pba_eval_out;

/* Evaluate residuals, Jacobians and the normal equations at the current poses. */
pba_status pba_evaluate(pba_ctx *ctx, pba_eval_out *out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): pba_evaluate with the same arguments and bitwise the
 * same results, whose evaluation working memory -- queue counters, per-item partial sums and
 * per-pair records -- comes from a fixed array of PBA_NOALLOC_SCRATCH_BYTES in the library's
 * device code instead of the context's buffers; the call allocates nothing (no hipMalloc or
 * hipFree, no allocator callback).  The array exists once per GPU and lives until the process
 * ends; every call on that GPU reuses it, so calls that overlap on one GPU (several streams or
 * threads, any contexts) race and must be serialised by the caller.  The system is kept in the
 * context as after pba_evaluate (pba_iterate and pba_solve_step reuse it).  Errors: those of
 * pba_evaluate, and PBA_EINVAL (state unchanged) when the context's work queue needs more than
 * the array: 256 B per work item (pba_timings.n_items) + 1280 B per pair + 1 KiB per (source,
 * target) sensor-model group (its queue counters), each part rounded up to 256 B.  Not timed (pba_get_timings counts only pba_evaluate). */
#define PBA_NOALLOC_SCRATCH_BYTES (128u << 20)
pba_status pba_evaluate_noalloc(pba_ctx *ctx, pba_eval_out *out);

/* Solve (H + lambda diag H) dx = -b at the current poses (anchor fixed), FP64 Cholesky.
 * dx (6N, N poses or pose variables, nullable) receives the step; it is also kept for
 * pba_apply_step. */
pba_status pba_solve_step(pba_ctx *ctx, double lambda, double *dx, int32_t on_device);

/* X_k <- X_k exp(dx_k) for every pose; dx NULL applies the last solved step. */
pba_status pba_apply_step(pba_ctx *ctx, const double *dx, int32_t on_device);

typedef struct {
    double F;                    /* objective after the iteration (at the accepted poses) */
    double lambda;               /* damping after the iteration (0 for Gauss-Newton) */
    double step_norm;            /* |dx| of the step tried */
    int64_t n_valid;
    int32_t accepted;            /* 1 if the step was taken */
    float ms;                    /* device time of the iteration (solve, update, evaluation,
                                    decision) from wall-clock stamps; -1 if unavailable */
} pba_iter_log;

/* Run n_iters Gauss-Newton (use_lm = 0: every solved step taken) or Levenberg-Marquardt
 * iterations (use_lm = 1: a step is kept only if F decreases; lambda /= 10 (floor 1e-12) on
 * accept, *= 10 on reject; lambda0 > 0 sets the initial damping, 0 continues from the damping
 * the previous call ended with, 1e-4 if none).  Each iteration solves at the current poses,
 * evaluates the candidate and decides on the device; the system at the current poses is
 * evaluated first only if no call has left it.  log (n_iters entries, nullable) is copied back
 * at the end.  Gauss-Newton returns PBA_ENOTPD if a system was not positive definite. */
pba_status pba_iterate(pba_ctx *ctx, int32_t n_iters, int32_t use_lm, double lambda0, pba_iter_log *log);

/* Photometric loss F(X0 boxplus delta) = sum over pairs and valid pixels of rho(chi^2)
 * (Sec. IV-C, Eq. (total-error-multicue)), with X0 the current poses and delta [N][6] float32
 * per pose (or pose variable) [dt, dq] (X0 exp(delta), Supplementary).  Evaluates at X0 boxplus delta and keeps
 * delta for pba_loss_backward.  *F_out (host) receives F, *n_valid_out (host, nullable) the number
 * of valid correspondences.  The poses X0 are not changed. */
pba_status pba_loss_forward(pba_ctx *ctx, const float *delta, int32_t on_device, double *F_out,
                            int64_t *n_valid_out);

/* Gradients of grad_F * F at the delta of the last pba_loss_forward, derived exactly for the
 * sampled images (slope of the bilinear interpolant; masks, cells and occlusion decisions held
 * as evaluated): grad_delta [N][6] (chain rule through R(dq) and the quaternion parameterisation)
 * and, per keyframe k, grad_intensity[k] [H][W], grad_depth[k] [H][W], grad_normals[k] [H][W][3]
 * (every array and every per-keyframe pointer nullable).  Image gradients are summed with atomic
 * additions, so their last bits can vary between runs.  Projections are recomputed, nothing is
 * stored per pixel between the two calls. */
pba_status pba_loss_backward(pba_ctx *ctx, double grad_F, float *grad_delta, float *const *grad_intensity,
                             float *const *grad_depth, float *const *grad_normals, int32_t on_device);

/* Coarse-to-fine image pyramid (Sec. IV-A: every keyframe is kept at several resolutions, each
 * half the one below; Sec. IV-C: optimisation runs from the coarsest level to the finest).
 * Builds n_levels levels (1..8; level 0 = the loaded images) on the device: level l + 1 takes
 * each 2x2 block of level l (odd last row/column dropped) -- depth: the block mean if all four
 * depths are valid and within the occlusion tau of each other, else no measurement; intensity:
 * the mean; normals: the mean scaled to unit length.  Level intrinsics: fx/2, fy/2,
 * (cx - 1/2)/2, (cy - 1/2)/2, floor(H/2) x floor(W/2) (pixel centres at integer coordinates).
 * Poses and pairs are shared by all levels.  PBA_ESTATE without keyframes; PBA_EINVAL if
 * n_levels is out of range or a level would be smaller than 4 x 4.  Loading keyframes drops the
 * pyramid.  The active level stays selected if it still exists, else level 0 becomes active. */
pba_status pba_build_pyramid(pba_ctx *ctx, int32_t n_levels);

/* Select the level that pba_evaluate, pba_solve_step, pba_iterate, the loss calls and
 * pba_debug_pair work on (image-sized outputs then have that level's size).  The system held
 * for the previous level is dropped; LM damping restarts at the next lambda0 > 0. */
pba_status pba_set_level(pba_ctx *ctx, int32_t level);

/* Coarse-to-fine optimisation (Sec. IV-C): for level = n_levels - 1 down to 0, select the level
 * and run up to iters[level] iterations (pba_iterate semantics, damping restarting at lambda0
 * on every level); move to the next finer level as soon as an accepted iteration lowers F by
 * less than rel_tol relative to F before it.  log (nullable, sum(iters) entries) receives the
 * iterations run, level_of (nullable, same length) their level, *n_done (nullable) their
 * number.  Level 0 is active afterwards. */
pba_status pba_optimize_pyramid(pba_ctx *ctx, const int32_t *iters, double rel_tol, int32_t use_lm, double lambda0,
                                pba_iter_log *log, int32_t *level_of, int32_t *n_done);

/* Inspection: one keyframe's images at a level, in the caller's layout (host arrays, each
 * nullable): intensity [H][W], depth [H][W] (0 where there is no measurement), normals
 * [H][W][3]; dims (nullable) receives {H, W} of that level. */
pba_status pba_get_level_image(pba_ctx *ctx, int32_t level, int32_t kf, float *intensity, float *depth,
                               float *normals, int32_t *dims);

/* Normals from depth (Sec. IV-A), replacing the loaded normal images of every keyframe: the
 * normal at u is the normal of the least-squares plane through the unprojected neighbours u' with
 * |u - u'| < tau_u pixels, tau_u = clamp(radius_m |fx| / d(u), min_px, max_px) (a fixed metric
 * radius seen at range d, so inversely proportional to it); neighbours need valid depth within the
 * sensor model's occlusion tau of d(u); at least min_count of them and a non-degenerate spread;
 * oriented towards the sensor; pixels without a normal get 0.  Needs 5 channels.  Drops any
 * pyramid (rebuild it afterwards) and the system held for the current poses. */
pba_status pba_estimate_normals(pba_ctx *ctx, double radius_m, double min_px, double max_px, int32_t min_count);

/* Matching pairs from the current poses (Sec. IV-B): an ordered pair (s, t) is kept if the angle
 * between the orientations of X_s and X_t (the rotation angle of R_s^T R_t) is below max_angle
 * (radians), the distance between their positions below max_dist, and the fraction of s's
 * pixels with valid depth that reproject validly into t (valid correspondences / evaluated
 * pixels of an evaluation at the current poses and level) at least min_ratio; with sequential
 * != 0, (k, k+1) and (k+1, k) are kept regardless (odometry-like links).  The kept pairs replace
 * the context's pairs (in (s, t) lexicographic order) and are copied to src_out / tgt_out
 * (nullable, up to cap entries); *n_out (nullable) receives their number.  PBA_ESTATE without
 * keyframes or poses; PBA_EINVAL for a negative threshold. */
pba_status pba_build_pairs(pba_ctx *ctx, double max_angle, double max_dist, double min_ratio, int32_t sequential,
                           int32_t cap, int32_t *src_out, int32_t *tgt_out, int32_t *n_out);

typedef struct {
    int32_t items_px;            /* source pixels per work item */
    int32_t grid;                /* workgroups of the persistent evaluation launch */
    double eval_ms;              /* evaluation kernel time(s) of one evaluation at this point */
} pba_tune_point;

/* Autotuner of the persistent evaluation launch (work-item size and grid): times one evaluation
 * at the current poses and level for every item size in {512, ..., 16384} (powers of 2; the source
 * pixels one wave takes at a time) and grid in {2, 4, 8} x (compute units) workgroups, keeps the
 * fastest for this context (until keyframes or pairs change the plan again) and reports the
 * measured points (points nullable, up to max_points; *n_points nullable).  Results of evaluations do not depend on the choice except in
 * the summation order of the per-pair sums. */
pba_status pba_autotune(pba_ctx *ctx, pba_tune_point *points, int32_t max_points, int32_t *n_points);

/* Per-pixel view of one pair for inspection (host outputs, each nullable, source-image sized):
 * status (0 valid, 1 no depth, 2 not projectable, 3 outside, 4 invalid or occluded tap; 5 flags a
 * point the evaluation's early depth-interval rejection would drop although it passes the
 * occlusion gate in a cell its projection can reach -- a check that should never fire),
 * uv (2 floats: projected column, row), cell (2 ints: integer cell x0, y0) and residuals
 * (5 floats).  Same kernels as pba_evaluate. */
pba_status pba_debug_pair(pba_ctx *ctx, int32_t pair, uint8_t *status, float *uv, int32_t *cell,
                          float *residuals);

typedef struct {
    double eval_ms;              /* summed duration of the evaluation kernel launches (HIP events) */
    int64_t eval_launches;
    double iterate_ms;           /* summed duration of pba_iterate iterations */
    int64_t iterations;
    int64_t n_items;             /* work items of the evaluation queue */
    int32_t items_px;            /* source pixels per work item */
    int32_t grid;                /* workgroups of the persistent evaluation launch */
    double iter_eval_ms;         /* summed duration of the evaluations inside pba_iterate (device
                                    wall-clock stamps before and after the evaluation launches of
                                    each iteration, also under graph replay) */
    int64_t iter_evals;
    int32_t solve_n;             /* order of the factored system (6 x pose variables, more with the
                                    padding of a nested-dissection order); 0 before the first plan */
    int32_t solve_steps;         /* dependent steps of the factorisation: block columns (natural order)
                                    or elimination-tree levels (nested dissection) */
    int32_t solve_nd;            /* 1 if the nested-dissection order is in use */
    int32_t reserved;
} pba_timings;

/* Kernel timing counters; reset = 1 clears them after reading. */
pba_status pba_get_timings(pba_ctx *ctx, pba_timings *out, int32_t reset);

const char *pba_status_string(pba_status status);
const char *pba_last_error(const pba_ctx *ctx);   /* valid until the next call on ctx */

#ifdef __cplusplus
}
#endif
#endif /* PBA_H */
