/*
 * ba.h -- C ABI of the MI355X (gfx950) Levenberg-Marquardt bundle-adjustment step.
 *
 * One LM iteration of the BA stage of InstantSfM (arXiv 2510.13310):
 *   - residuals of every active observation: reprojection (Eq. (2)) stacked with the
 *     weighted inverse-depth prior residual (Eqs. (6), (7)) whose reference is the masked
 *     inverse depth m / d_hat (Eq. (9)); one Huber robustifier on the stacked norm;
 *   - their SE(3) (6) and point (3) Jacobian blocks, the depth-constrained sparse Jacobian of
 *     Sec. IV-A, built in one uniform pass;
 *   - the block-sparse J^T J / J^T r of the LM system (Eq. (3), Marquardt diagonal), reduced
 *     to the camera Schur complement and solved by PCG with a 6x6 block-Jacobi preconditioner;
 *   - dynamic parameter extraction (Sec. IV-B, Eqs. (10)-(15)) at the start of every
 *     iteration, and the scatter of the compact update back into the full arrays.
 *
 * Conventions
 *   cams    C x 7 float64, row-major [qw, qx, qy, qz, cx, cy, cz]: unit quaternion of the
 *           world-to-camera rotation R and the camera centre c (the paper's {centre,
 *           quaternion} extrinsics, Sec. III-B). A world point X has camera coordinates
 *           R (X - c); pixels are (f x/z + cx, f y/z + cy).
 *   intr    C x 3 float64 [f, cx, cy] in pixels, held fixed.
 *   points  P x 3 float64.
 *   The LM update of a camera is the left SE(3) perturbation T <- Exp(xi) T, xi = (rho, phi).
 *
 * Pointers: every array argument may be host memory or device memory of the current HIP
 * device (unified addressing). Inputs are copied into library-owned device buffers before
 * the call returns; the caller keeps ownership and may free or reuse them afterwards.
 * Outputs are written to caller-provided buffers of the stated size.
 *
 * Errors: no exception crosses the ABI. On an error the context keeps its previous state
 * and ba_last_error() describes the failure. A context is not thread-safe; distinct
 * contexts are independent.
 */
#ifndef INSTANTBA_BA_H
#define INSTANTBA_BA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ba_ctx ba_ctx;

typedef int32_t ba_status;
#define BA_OK 0            /* success */
#define BA_EMPTY 1         /* no active observation: the step changed nothing */
#define BA_NOT_CONVERGED 2 /* ba_adjoint: the PCG stopped at adjoint_max_iters above
                              adjoint_rel_tol; the gradients were written from its last
                              iterate and ba_last_error() gives the residual reached */
#define BA_ERR_ARG (-1)    /* invalid argument (size, index out of range, NULL) */
#define BA_ERR_STATE (-2)  /* call out of order (e.g. lm_step before set_observations) */
#define BA_ERR_OOM (-3)    /* device allocation failed */
#define BA_ERR_DEVICE (-4) /* no usable GPU, or a HIP runtime error */
#define BA_ERR_NUMERIC (-5)/* non-finite cost at the current parameters */

#define BA_PRECISION_FP64 0  /* every stage in float64 */
#define BA_PRECISION_MIXED 1 /* float32 Jacobians, J^T J blocks and PCG matvecs; float64
                                PCG dots and norms, cost, gain ratio, 3x3 inversions. The LM
                                damping stays at or above max(lambda_min, 1e-5): a smaller
                                Marquardt damping is lost in the float32 rounding of the
                                damped blocks, whose reduced system then turns singular or
                                indefinite at float32 resolution (PCG breakdown) */

#define BA_ACTIVITY_ROWS 0    /* point active with >= 3 residual rows, camera with >= 6
                                 (rows: 2 per observation, +1 with a valid depth prior) */
#define BA_ACTIVITY_LITERAL 1 /* active with >= 1 valid observation (Eqs. (11)-(12)) */

#define BA_SOLVER_IMPLICIT 0  /* PCG on the camera Schur complement applied matrix-free: two
                                 passes over the observations per iteration (Sec. IV-B) */
#define BA_SOLVER_EXPLICIT 1  /* the same PCG on the reduced camera system assembled as D x D
                                 blocks: per extraction the block pattern (a stable sort of the
                                 camera pairs of every point), per LM step the blocks
                                 S_ij = -sum_p W_ip V*_p^-1 W_jp^T, per iteration one sparse
                                 block product. The adjoint always runs matrix-free */

#define BA_ADJOINT_FULL 0          /* the exact Hessian of the cost at the solution: the
                                      robust-corrected Gauss-Newton blocks plus, per
                                      observation, the curvature of its residual rows weighted
                                      by rho' e and the second-order part of the SE(3)
                                      retraction (the implicit derivative itself) */
#define BA_ADJOINT_GAUSS_NEWTON 1  /* sum J^T (rho' I + 2 rho'' e e^T) J only: drops those
                                      terms, which vanish with the residuals */

typedef struct ba_options {
  int32_t precision;       /* BA_PRECISION_*; default MIXED */
  int32_t img_w, img_h;    /* frustum for the validity test; default 640 x 480 */
  int32_t activity_rule;   /* BA_ACTIVITY_*; default ROWS */
  double min_depth;        /* validity needs camera-frame z > min_depth (Eq. (10)); 0.1 */
  double huber_px;         /* Huber threshold on the stacked residual norm; <= 0: L2 */
  double filter_px;        /* validity needs 2-D reprojection error <= filter_px; <= 0 off */
  double lambda_init;      /* initial LM damping; 1e-3 */
  double lambda_min, lambda_max; /* damping clamp; 1e-12, 1e12 (MIXED: at least 1e-5) */
  double diag_min, diag_max;     /* clamp of the Marquardt diagonal diag(J^T J); 1e-6, 1e32 */
  double accept_ratio;     /* accept a step when the cost drops and gain ratio > this; 1e-3 */
  int32_t pcg_max_iters;   /* 100 */
  int32_t pcg_check_every; /* PCG iterations enqueued between host convergence checks; 8 */
  double pcg_rel_tol;      /* stop when |r| <= tol |b|; 1e-6 */
  double cost_rel_tol;     /* ba_solve: stop when an accepted step lowers the cost by at most
                              this fraction (per-observation sum of the changes); 1e-10 */
  double grad_tol;         /* ba_solve: stop when max |g| <= grad_tol; 1e-10 */
  int32_t max_lm_iters;    /* ba_solve iteration cap; 100 */
  int32_t timing;          /* 1: time phases and kernels with HIP events (ba_kernel_stats) */
  int32_t adjoint_max_iters;/* PCG cap of the (undamped) adjoint solve; 5000 */
  int32_t solver;          /* BA_SOLVER_*; default IMPLICIT */
  int32_t refine_focal;    /* 1: the focal length f of each camera's intrinsics (Sec. III-B
                              lists K among the BA parameters) is a seventh camera unknown:
                              7 x 7 camera blocks, de/df = (x/z, y/z, 0), additive update, a
                              camera needs 7 residual rows; cx, cy stay fixed. The adjoint
                              needs it off. Default 0 */
  int32_t adjoint_hessian; /* BA_ADJOINT_*: the Hessian of the adjoint system; default FULL */
  double adjoint_rel_tol;  /* PCG tolerance of the adjoint solve; 1e-10 */
  double adjoint_damping;  /* Tikhonov damping of the adjoint system, added as
                              lambda clamp(diag H) like the LM damping: 0 (the exact implicit
                              derivative) fails with BA_ERR_NUMERIC when H is singular, e.g.
                              a two-view point whose observations are both in the Huber
                              regime; a small value (1e-6) regularises such blocks; 0 */
  double gp_huber;         /* Huber threshold of global positioning on |u| (unit-ray units);
                              <= 0: L2; 0.1 */
  void* hip_stream;        /* hipStream_t to run on; NULL: a stream owned by the context */
} ba_options;

typedef struct ba_step_report {
  int32_t status;          /* BA_OK or BA_EMPTY */
  int32_t accepted;        /* 1 if the step was applied */
  int32_t relinearized;    /* 1 if extraction + linearisation ran (0 after a rejection) */
  int32_t fixpoint_rounds; /* rounds of the activity fixpoint */
  int32_t pcg_iters;
  int32_t pcg_breakdown;   /* 1 if PCG met a non-positive curvature (step rejected) */
  int32_t n_cams_active, n_points_active;
  int64_t n_obs_active;
  double cost_before;      /* F = 1/2 sum rho(|e|^2) over the active observations */
  double cost_after;       /* F at the candidate, as F minus the per-observation sum of the
                              changes (+inf if a depth drops below min_depth) */
  double model_decrease;   /* -(g.delta + 1/2 sum w |J delta|^2) */
  double gain_ratio;
  double lambda;           /* damping used by this step */
  double pcg_rel_residual; /* |r| / |b| at exit (recursive residual) */
  double rms_px;           /* sqrt(mean |r_2d|^2) over the active observations, before */
  double grad_inf;         /* max |g| over the compact parameters, before */
  double ms_extract, ms_linearize, ms_setup, ms_pcg, ms_candidate, ms_total;
                           /* host wall times per phase; without timing the linearisation and
                              setup are not waited for separately, so their device time shows
                              in the next phase that synchronises */
  double pcg_true_residual;/* |b - S x| / |b| of the PCG solution x, S applied once more by the
                              solve's own matvec kernels (float32 products in MIXED, float64 in
                              FP64); computed only with opt.timing = 1 and the implicit solver,
                              else -1 */
} ba_step_report;

typedef struct ba_solve_report {
  int32_t iterations, accepted;
  int32_t stop_reason;     /* 0 max iters, 1 cost tol, 2 grad tol, 3 lambda max, 4 empty */
  int64_t total_pcg_iters;
  double initial_cost, final_cost;
  double initial_rms_px, final_rms_px;
  double lambda;
  double ms_total;
} ba_solve_report;

typedef struct ba_kernel_stat {
  char name[32];
  int64_t launches;        /* launches that did work */
  double total_ms;         /* sum of HIP-event durations on the context's stream */
  double total_bytes;      /* algorithmic bytes moved (sizes of the arrays it must read and
                              write once), summed over launches */
} ba_kernel_stat;

/* Fill *opt with the defaults listed above. */
void ba_default_options(ba_options* opt);

/* Create a context on the current HIP device holding the BA parameters of Sec. III-B: the
 * camera extrinsics {centre, quaternion} and the intrinsics K of every camera, and the 3-D
 * points. opt may be NULL (defaults). 1 <= n_cams, n_points <= 2^27 - 1 (the kernels index
 * per-point arrays with 32-bit products of up to 16 P), else BA_ERR_ARG; cams C x 7, intr
 * C x 3 and points P x 3 (layouts above) are copied in, non-finite values and zero
 * quaternions are BA_ERR_ARG. Returns BA_ERR_DEVICE when no GPU is usable. *out is NULL on
 * any error. */
ba_status ba_create(const ba_options* opt, int32_t n_cams, int32_t n_points,
                    const double* cams, const double* intr, const double* points,
                    ba_ctx** out);

/* Set the observation list: observation k is the 2-D keypoint x_ij of Eq. (2), point
 * pt_idx[k] seen in camera cam_idx[k] at pixel (xy[2k], xy[2k+1]) (float32, row-major N x 2);
 * its residual is the reprojection error pi(zeta_i, X_j, K_i) - x_ij. 0 <= n_obs <= 2^29 - 1
 * (per-observation arrays hold up to 3 values indexed with 32-bit products), else BA_ERR_ARG.
 * Indices are range-checked (BA_ERR_ARG, nothing changed). Resets the LM state (lambda),
 * clears depth priors and invalidates the linearisation. The library sorts the observations
 * point-major and renumbers points internally; every output is reported in the caller's
 * order. */
ba_status ba_set_observations(ba_ctx* ctx, int64_t n_obs, const int32_t* cam_idx,
                              const int32_t* pt_idx, const float* xy);

/* Metric depth priors d_hat (metres, camera-frame z), one per observation (N float32, the
 * order of ba_set_observations), with the optional validity mask m of Eq. (9) (N bytes, NULL:
 * all valid). Each observation then gets the inverse-depth row r^d = 1/z - m/d_hat of
 * Eq. (6) with the masked reference of Eq. (9), weighted by lambda_d and stacked with the
 * reprojection row under one robustifier (Eq. (7)). Non-finite or <= 0 depths count as
 * invalid (m = 0: target 0, a weak far-depth row). lambda_d >= 0 (px * m); 0 disables the
 * depth rows. BA_ERR_STATE before ba_set_observations; invalidates the linearisation. */
ba_status ba_set_depth_priors(ba_ctx* ctx, const float* depth, const uint8_t* valid,
                              double lambda_d);

/* Hold the listed cameras fixed (gauge anchors); they never enter the solve but their
 * observations constrain points. n = 0 clears the list. */
ba_status ba_set_fixed_cameras(ba_ctx* ctx, int32_t n, const int32_t* cam_ids);

/* Exactly one LM iteration (Eq. (3), Sec. IV-B): dynamic parameter extraction at the current
 * parameters (Eqs. (10)-(15)), linearisation, the damped normal equations reduced to the
 * camera Schur complement and solved by block-Jacobi PCG, back-substitution of the points,
 * the candidate's cost over the same observations, acceptance by gain ratio, and the scatter
 * of an accepted update into the full parameters (inactive ones untouched). After a rejected
 * step the next call reuses the extraction and linearisation with a larger damping. rep may
 * be NULL. Returns BA_EMPTY when nothing is active, BA_ERR_STATE before
 * ba_set_observations, BA_ERR_NUMERIC (parameters unchanged) for a non-finite cost. */
ba_status ba_lm_step(ba_ctx* ctx, ba_step_report* rep);

/* ba_lm_step for callers that cannot allocate device memory (serving loops, code that must
 * not call hipMalloc): the same LM iteration with the same results, but its per-step scratch
 * (fixpoint and damping flags, PCG states, reduction partials, the item partials of the camera
 * assembly and the PCG camera pass, item tables, the scan workspace) lives in a static device array of 32 MiB that each GPU holds from
 * library load to process end; the call itself allocates nothing. The context's other
 * buffers are those of ba_create and ba_set_observations. BA_ERR_ARG when the problem needs
 * more scratch than the array holds (about 2.5 bytes per point, 2 KB per camera (2.5 KB with
 * focal refinement), 0.2 MB and the scan workspace: e.g. 2M points and 5000 cameras fit), BA_ERR_STATE with opt.timing = 1 or
 * the explicit solver (both allocate). Every call on one GPU shares that GPU's array and
 * leaves its contents behind: calls that overlap in time on one GPU (from several threads or
 * streams) race and must be serialised by the caller. */
ba_status ba_lm_step_noalloc(ba_ctx* ctx, ba_step_report* rep);

/* The LM loop of Eq. (3): iterate ba_lm_step until max_lm_iters, the relative cost decrease
 * of an accepted step falls to cost_rel_tol, max |g| to grad_tol, or a rejection reaches
 * lambda_max (rep->stop_reason). rep may be NULL. Errors as ba_lm_step. */
ba_status ba_solve(ba_ctx* ctx, ba_solve_report* rep);

/* Copy the current parameters of Sec. III-B out: cams C x 7 [qw, qx, qy, qz, cx, cy, cz] and
 * points P x 3, float64, caller's order, host or device memory owned by the caller (either
 * may be NULL). */
ba_status ba_get_params(const ba_ctx* ctx, double* cams, double* points);

/* Overwrite the parameters (cams C x 7, points P x 3; either may be NULL), e.g. to warm-start
 * a re-solve. Resets lambda to lambda_init and invalidates the linearisation. */
ba_status ba_set_params(ba_ctx* ctx, const double* cams, const double* points);

/* Copy the current intrinsics out (C x 3 [f, cx, cy]): the focal lengths as refined so far
 * when refine_focal, else the values given to ba_create. */
ba_status ba_get_intrinsics(const ba_ctx* ctx, double* intr);

/* Activity of the last extraction, in the caller's order (any pointer may be NULL):
 * cams C, points P, obs N bytes, 1 = active. BA_ERR_STATE before the first step. */
ba_status ba_get_active(const ba_ctx* ctx, uint8_t* cams, uint8_t* points, uint8_t* obs);

/* The last computed LM step in tangent coordinates: cams C x d (rho, phi, and the focal step
 * when refine_focal: d = 7, else d = 6), points P x 3; zero for inactive or fixed entries. */
ba_status ba_get_last_step(const ba_ctx* ctx, double* dcams, double* dpoints);

/* The block-Jacobi preconditioner of the last LM system (the paper names PCG, Sec. IV-B, but
 * not its preconditioner): for every active camera the inverse of its D x D diagonal block
 * of the damped camera Schur complement, S_cc = U*_c - sum_k W_k V*^-1 W_k^T (Eq. (3)),
 * factorised by Cholesky in float64; a block that is not positive definite falls back to
 * the inverse of diag(U*_c). Minv: C x D x D float64, row-major, caller's camera order, zero
 * for inactive and fixed cameras; D = 7 with refine_focal, else 6. BA_ERR_STATE before the
 * first ba_lm_step. */
ba_status ba_get_preconditioner(const ba_ctx* ctx, double* Minv);

/* Undamped normal-equation blocks of the last linearisation, caller's order, zero for
 * inactive entries: U C x d*d (J_c^T W J_c, row-major d x d), gc C x d (J_c^T W e),
 * V P x 9 (J_p^T W J_p), gp P x 3 (J_p^T W e), with d = 7 when refine_focal, else 6.
 * Any pointer may be NULL. */
ba_status ba_get_normal_blocks(const ba_ctx* ctx, double* U, double* gc, double* V,
                               double* gp);

/* Implicit adjoint of the current (converged) solution: given dL/dcams (C x 7) and
 * dL/dpoints (P x 3), write dL/dxy (N x 2 float32) and dL/ddepth (N float32, zeros without
 * depth rows). Solves H v = dL/dtheta by the same Schur-PCG, with H the exact Hessian of the
 * cost (adjoint_hessian = BA_ADJOINT_FULL) or its robust-corrected Gauss-Newton part
 * sum J^T M J, M = rho' I + 2 rho'' e e^T (BA_ADJOINT_GAUSS_NEWTON), then maps v per
 * observation (implicit function theorem on the vanishing gradient at the solution). Needs at
 * least one fixed camera and a fixed scale (depth rows with lambda_d > 0, or two fixed
 * cameras): BA_ERR_STATE otherwise.
 * Inactive observations get zero gradients. Returns BA_NOT_CONVERGED when the PCG stopped at
 * adjoint_max_iters above adjoint_rel_tol (gradients written from the last iterate). */
ba_status ba_adjoint(ba_ctx* ctx, const double* grad_cams, const double* grad_points,
                     float* grad_xy, float* grad_depth);
/* (with refine_focal set, ba_adjoint returns BA_ERR_STATE: it covers poses and points) */

/* Per-kernel HIP-event statistics accumulated while opt.timing = 1. Writes up to max entries
 * and returns their count in *n. ba_reset_kernel_stats clears them. */
ba_status ba_kernel_stats(const ba_ctx* ctx, ba_kernel_stat* out, int32_t max, int32_t* n);
ba_status ba_reset_kernel_stats(ba_ctx* ctx);

/* Device bytes currently allocated by the context. */
int64_t ba_device_bytes(const ba_ctx* ctx);


/* ---------------------------------------------------------------- global positioning
 * Depth-constrained global positioning (Sec. III-A, Eq. (1); Sec. IV-A, Eqs. (4), (5), (8)) on
 * the same context: camera rotations are held at the cams' quaternions; the unknowns are the
 * camera centres (cams entries 4..6), the points and one scale s per observation, residual
 * u = v - s (X - c) on the unit world ray v = R^T K^-1 [x, y, 1] / |K^-1 [x, y, 1]|, Huber
 * (gp_huber) on |u|^2. An observation with a valid depth prior (ba_set_depth_priors; any
 * lambda_d) is pinned at s = 1 / (d_hat |K^-1 [x, y, 1]|), the inverse distance along the
 * ray of a z-depth d_hat, and its scale column leaves the system (Eq. (8)); the other scales
 * are free. Extraction keeps every observation with finite data; an observation brings 3
 * rows when pinned and 2 when free, a point needs 3 and a camera 3 (fixed cameras keep their
 * centre). One LM iteration: free scales eliminated per observation, points per point, PCG
 * with block-Jacobi on the 3 x 3 camera-centre Schur complement, back-substitution, the
 * candidate's cost over the same observations (a free scale <= 0 rejects it), Nielsen's
 * damping rule on a damping of its own. Free scales start at the inverse distance of the
 * estimate at the first GP call (again after ba_set_params, ba_set_depth_priors or
 * ba_gp_reset). A GP step leaves the BA state to re-extract at its next step. */
ba_status ba_gp_step(ba_ctx* ctx, ba_step_report* rep);   /* rms_px: RMS of |u| */
ba_status ba_gp_solve(ba_ctx* ctx, ba_solve_report* rep); /* same stopping rules as ba_solve */
/* Current scales, N doubles in the caller's observation order (pinned ones included). */
ba_status ba_gp_get_scales(const ba_ctx* ctx, double* scales);
/* Re-initialise the free scales from the current estimate and restart the GP damping. */
ba_status ba_gp_reset(ba_ctx* ctx);

/* Message of the last error on ctx (or of the last failed ba_create when ctx is NULL). */
const char* ba_last_error(const ba_ctx* ctx);

/* Release every device buffer; NULL is ignored. */
void ba_destroy(ba_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* INSTANTBA_BA_H */
