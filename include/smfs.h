/*
 * smfs -- MI355X (gfx950) library for the Stokes resistance problem of rigid
 * spheres with the method of fundamental solutions and lubrication-adapted
 * image lines (Broms, Barnett & Tornberg, arXiv 2407.03343).
 *
 * The flow is a sum of Stokeslets on an interior proxy sphere of each body
 * (Section 2.1), plus Stokeslets, rotlets and potential dipoles on an image
 * line per near contact (Section 2.3, eqs. line_points-tj; kinds chosen in
 * Section 5.1).  Strengths solve the one-body right-preconditioned square
 * system G_hat mu = b (Section 2.2, eq. resistance) by GMRES; every product
 * with G_hat applies the two-factor pseudo-inverse of each sphere's self
 * block (eq. transform), sums all off-sphere interactions directly and adds
 * the identity self blocks (eq. uAll and the self-replacement step).
 *
 * Conventions
 *  - Memory: arrays marked [host] are ordinary host memory; arrays marked
 *    [dev] are device memory of the current HIP device.  The library never
 *    allocates device memory for a problem: the caller allocates
 *    smfs_sizes.workspace_bytes of device memory and binds it with
 *    smfs_bind(), and passes the set-up scratch (smfs_setup_workspace_bytes)
 *    and the block workspaces to the calls that need them.
 *  - Streams: every device call is ordered on the hipStream_t passed in
 *    (NULL = the null stream).  Calls that return host statistics
 *    synchronise that stream before returning.
 *  - Vectors over collocation nodes (mu, b, y) are node-major, length 3 T:
 *    entry 3 i + c is component c of node i; nodes are grouped by sphere.
 *  - Source strengths (lambda) are S x 3 row-major, grouped by kind: all
 *    Stokeslets (sphere-major; proxy points first, then image nodes contact
 *    by contact), then all rotlets, then all potential dipoles.
 *  - Forces/torques are P x 6 (F, T) with F = sum of Stokeslet strengths,
 *    T = sum of rotlet strengths + sum (y - c) x f (Remark on extracting net
 *    forces and torques): the force and torque the sphere exerts on the fluid.
 *  - Errors: functions return SMFS_OK (0), a positive warning, or a negative
 *    error; smfs_last_error() gives a thread-local message.  Nothing throws
 *    across this interface.  Handles are not thread-safe; distinct handles
 *    are independent.
 */
#ifndef SMFS_H
#define SMFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *smfs_stream; /* a hipStream_t */
typedef struct smfs_problem smfs_problem;

enum {
  SMFS_OK = 0,
  SMFS_NOT_CONVERGED = 1,          /* warning: statistics still filled in */
  SMFS_GAP_BELOW_VALIDATED = 2,    /* warning: some gap < 1e-3 radii */
  SMFS_STAGNATED = 3,              /* warning: the FP64 true residual stopped falling above
                                      gmres_tol (statistics filled in, the best iterate
                                      returned) */
  SMFS_E_INVALID_ARG = -1,
  SMFS_E_OVERLAP = -2,             /* two spheres touch or overlap */
  SMFS_E_UNSUPPORTED = -3,         /* e.g. unequal radii */
  SMFS_E_NOMEM = -4,               /* workspace too small */
  SMFS_E_SVD = -5,
  SMFS_E_DEVICE = -6,              /* HIP error */
  SMFS_E_STATE = -7,               /* call out of order (e.g. apply before setup) */
  SMFS_E_AGAIN = -8                /* the server's queue is full: submit again later */
};

/* Precision of the products inside GMRES.  SMFS_MIXED: the sources of
 * contact-free spheres in FP32, both their pseudo-inverse apply (FP32 copy
 * of the shared factor) and their pair sums.  SMFS_MIXED_FAR: their pair
 * sums in FP32 from strengths computed in FP64 (the pseudo-inverse stays
 * FP64).  SMFS_MIXED_EQ: the far field of every contact-free sphere through
 * eq_points equivalent Stokeslets, fitted in FP64 and summed in FP32, for
 * target spheres at centre separation >= eq_separation; closer pairs of a
 * contact-free source, and every source of a contact sphere, exact in FP64
 * (a one-level equivalent-source replacement of the fast multipole
 * evaluation of eq. uAll, Section 2.2; needs smfs_setup_far_field, which
 * smfs_setup runs).  The proxies' strengths of a rough vector cancel by up
 * to 1e5 in their far field, which an FP32 sum of them cannot resolve; the
 * equivalent strengths are of the size of the field.  Everything else is
 * FP64 in all modes; the true-residual checks, restarts and refinement
 * residuals of a solve are FP64 products. */
enum { SMFS_FP64 = 0, SMFS_MIXED = 1, SMFS_MIXED_FAR = 2, SMFS_MIXED_EQ = 3 };
enum { SMFS_KIND_S = 1, SMFS_KIND_R = 2, SMFS_KIND_D = 4 };
/* SVD of the self blocks at set-up: SMFS_SVD_JACOBI = Householder QR
 * B = Q1 R1, a second QR R1^T = Q2 R2 (a preconditioner), one-sided Jacobi
 * on R2^T in the library's kernels, then U = Q1 U_X and V = Q2 J; ranks
 * equal LAPACK's on the default blocks.  It is the faster method for small
 * batches (two spheres: 1.1 s against 3.2 s) and for blocks of at most 768
 * columns (a 160-sphere request at 120 proxies: 2.1 s against 6-7 s), but
 * not for many large blocks (106 blocks of about 4500 x 2000: 69 s against
 * 41 s).  A block's factors do not depend on the other blocks of its batch.
 * SMFS_SVD_ROCSOLVER = rocSOLVER's bidiagonal gesvd. */
enum { SMFS_SVD_JACOBI = 0, SMFS_SVD_ROCSOLVER = 1 };

/* Discretisation and solver parameters (lengths in radii). */
typedef struct smfs_params {
  int32_t n_proxy;          /* N: proxy Stokeslets per sphere (Section 2.1) */
  double proxy_radius;      /* R_p */
  int32_t n_colloc_base;    /* base collocation nodes per sphere */
  int32_t n_image;          /* image nodes per contact; < 0: eq. (image_est) */
  uint32_t image_kinds;     /* SMFS_KIND_* mask placed at image nodes */
  double image_offset;      /* Delta in eq. (tj) */
  double image_gap_cutoff;  /* pairs with gap below this get image lines */
  double near_gap_cutoff;   /* mixed precision: pairs below this stay FP64; must not
                               exceed image_gap_cutoff (the FP32 class is the proxy
                               sources of spheres without a contact), else
                               SMFS_E_UNSUPPORTED at create */
  int32_t cap_alpha[2];     /* cap upsampling, eq. (colloc_nbr) */
  double cap_beta[2];       /* cap half-angles, eq. (thetacap) */
  int32_t left_weights;     /* row weights sqrt(area) (Remark left-precond) */
  double trunc_rel;         /* singular values kept if > trunc_rel * sigma_1 */
  double mu;                /* viscosity */
  int32_t n_check_base;     /* residual check points per sphere */
  int32_t precision;        /* SMFS_FP64, SMFS_MIXED, SMFS_MIXED_FAR or SMFS_MIXED_EQ */
  double gmres_tol;         /* relative residual target */
  int32_t gmres_max_it;
  int32_t gmres_restart;    /* Krylov vectors kept (sizes the workspace) */
  int32_t gmres_check_every;/* true-residual guard period in iterations, active once the
                               recursive estimate is below 1e-3; 0 = off.  Each check
                               forms the iterate and costs one product with G_hat */
  int32_t svd_method;       /* SMFS_SVD_ROCSOLVER (default) or SMFS_SVD_JACOBI */
  /* equivalent-source far field (SMFS_MIXED_EQ): eq_points Stokeslets on the
   * Fibonacci spiral of radius eq_radius (radii) around a sphere's centre,
   * fitted to its proxies' field at 2 eq_points check points of radius
   * eq_check_radius by a pseudo-inverse keeping singular values above
   * eq_rcond sigma_1; used for target spheres at centre separation
   * >= eq_separation, which must be at least eq_check_radius + 1 (every
   * target then lies outside the check sphere).  eq_points = 0: off. */
  int32_t eq_points;        /* default 200 */
  double eq_radius;         /* default 1.0 */
  double eq_check_radius;   /* default 2.5 */
  double eq_separation;     /* default 3.5 */
  double eq_rcond;          /* default 1e-12 */
  int32_t progress;         /* > 0: one line on stderr every `progress` GMRES iterations
                               (iteration, residual estimate); 0 (default): silent */
} smfs_params;

typedef struct smfs_sizes {
  int32_t P;
  int32_t n_factors;        /* distinct self blocks (0 = shared contact-free) */
  int32_t n_contacts;       /* directed sphere-contacts with image lines */
  int32_t min_gap_flag;     /* 1 if some gap < 1e-3 */
  int64_t T;                /* collocation nodes */
  int64_t S;                /* sources (all kinds) */
  int64_t n_kind[3];        /* Stokeslets, rotlets, dipoles */
  int64_t n_check;          /* residual check points */
  size_t workspace_bytes;   /* device bytes smfs_bind() needs */
  size_t factor_bytes;      /* part of workspace_bytes holding factors */
  int32_t svd_sweeps;       /* Jacobi sweeps the last smfs_setup needed (the most of any
                               batch; 0 with SMFS_SVD_ROCSOLVER or before set-up) */
  int64_t eq_far_pairs;     /* SMFS_MIXED_EQ product: target x equivalent-source pairs */
  int64_t eq_exact_pairs;   /* its exact FP64 pairs (contact sources, near proxies) */
  int64_t eq_near_spheres;  /* entries of all near lists (contact-free source spheres
                               closer than eq_separation to a target sphere) */
} smfs_sizes;

/* Output of a solve.  Device pointers may be NULL to skip that output. */
typedef struct smfs_out {
  double *mu;               /* [dev] 3 T: converged unknowns */
  double *lambda;           /* [dev] S x 3: strengths lambda = B^+ mu */
  double *ft;               /* [dev] P x 6: forces and torques */
  double *u_check;          /* [dev] n_check x 3: velocity at check points */
  double *rbm;              /* [dev] P x 6: rigid motions found (mobility only) */
  /* host statistics */
  int32_t iterations;       /* GMRES iterations: Krylov dimension summed over restart cycles */
  double rel_residual;      /* GMRES estimate at exit */
  double true_rel_residual; /* ||b - G_hat mu|| / ||b||, recomputed in FP64 */
  double lambda_inf;        /* max |lambda| (stability indicator, Section 3) */
  double eps_res_max;       /* max pointwise relative residual, eq. (residual) */
  double abs_res_max;       /* max |u - u_bc| / max |u_bc| */
  double t_rhs_ms, t_gmres_ms, t_post_ms;
  int64_t pair_evals;       /* pair evaluations performed by the solve */
  int64_t pair_evals_f32;   /* of which evaluated in FP32 (mixed precision) */
  int32_t refinements;      /* refinement sweeps on the FP64 true residual */
  int32_t true_checks;      /* true residuals taken by the guard (restarts included) */
  int32_t floor_iteration;  /* iteration of the smallest true residual the guard saw, -1 if none */
  double floor_rel_residual;/* that relative residual, -1 if none */
} smfs_out;

/* Defaults: N = 600, R_p = 0.7, 780 base nodes, 20 images of kinds S|R|D,
 * Delta = 0.05, image and near cutoffs 0.2, alpha = 6, beta = pi/5, pi/60,
 * left weights on, trunc 5e-12, mu = 1, 500 check points, FP64, tol 1e-10,
 * 1000 iterations, restart 400, true-residual guard every 25 iterations. */
int smfs_params_default(smfs_params *p);

/* Build the node sets on the host (Sections 2.1, 2.3, 5.1).
 * centers [host] P x 3, radii [host] P (all equal, else UNSUPPORTED).
 * Returns OVERLAP if any gap <= 0, GAP_BELOW_VALIDATED (warning, handle
 * created) if a gap is below 1e-3 radii. */
int smfs_problem_create(const smfs_params *p, int32_t P, const double *centers,
                        const double *radii, smfs_problem **out);
void smfs_problem_destroy(smfs_problem *pb);
int smfs_problem_sizes(const smfs_problem *pb, smfs_sizes *s);

/* Copy node sets out [host] (Section 2.1 proxy and collocation points;
 * Section 2.3 image lines, eqs. line_points and tj; Section 5.1 cap points
 * and weights; check points of eq. residual_x); any pointer may be NULL.
 * targets T x 3,
 * target_sphere T, target_weight T (area weights w_i), sources S x 3,
 * source_kind S (0 S, 1 R, 2 D), source_sphere S, check n_check x 3,
 * check_sphere n_check. */
int smfs_export_nodes(const smfs_problem *pb, double *targets, int32_t *target_sphere,
                      double *target_weight, double *sources, int32_t *source_kind,
                      int32_t *source_sphere, double *check, int32_t *check_sphere);

/* Factor id of sphere k (0 = the shared contact-free factor): the SVD of
 * B_k = W_k G^(kk) behind eq. transform (Section 2.2). */
int smfs_sphere_factor(const smfs_problem *pb, int32_t k, int32_t *fid);
/* Shape of self block fid: rows = 3 M, cols = 3 N', rank after truncation
 * (0 before setup/import), representative sphere. */
int smfs_factor_info(const smfs_problem *pb, int32_t fid, int32_t *rows, int32_t *cols,
                     int32_t *rank, int32_t *sphere);

/* Bind caller-provided device workspace and upload the node sets. */
int smfs_bind(smfs_problem *pb, void *dev_workspace, size_t bytes, smfs_stream stream);

/* Device scratch bytes smfs_setup needs for this problem: one batch of
 * assembled self blocks of the largest shape group, the SVD's status words
 * and the SVD's own work arrays (rocSOLVER's size query).  Host only. */
int smfs_setup_workspace_bytes(smfs_problem *pb, size_t *bytes);

/* Assemble every distinct self block B = W G^(kk) on the device and factor
 * it with a thin SVD (rocSOLVER, one batched call per group of equal shape),
 * keeping sigma_i > trunc_rel * sigma_1 (Section 2.2, eq. transform; the
 * truncation eps_trunc of Section 5); then, with eq_points > 0, fit the
 * equivalent sources (smfs_setup_far_field).  scratch [dev]: at least
 * smfs_setup_workspace_bytes bytes, 256-byte aligned, owned by the caller
 * and free again when the call returns; the library allocates no device
 * memory here (rocSOLVER works in the scratch).  Errors: SMFS_E_STATE if not
 * bound, SMFS_E_NOMEM if the scratch is too small, SMFS_E_SVD if an SVD
 * fails.  Synchronises the stream. */
int smfs_setup(smfs_problem *pb, void *scratch, size_t scratch_bytes, smfs_stream stream);

/* Equivalent sources of the contact-free spheres for SMFS_MIXED_EQ (eq_*
 * parameters; a fast evaluation of the far part of eq. uAll, Section 2.2,
 * where the paper uses a fast multipole method): assembles the Stokeslet matrices K(check, equivalent) and
 * K(check, proxies) of one sphere on the device, takes the SVD of the first
 * (rocSOLVER) and stores E = K_ce^+ K_cp (3 eq_points x 3 n_proxy, FP64) in
 * the workspace.  E depends on the node sets only, not on the factors, so a
 * caller that imports factors runs this alone.  scratch [dev]: at least
 * smfs_far_field_workspace_bytes bytes, 256-byte aligned, caller-owned and
 * free again on return.  Nothing to do (SMFS_OK) without contact-free
 * spheres or with eq_points = 0.  Errors: SMFS_E_STATE if not bound,
 * SMFS_E_NOMEM, SMFS_E_SVD.  Synchronises the stream. */
int smfs_far_field_workspace_bytes(smfs_problem *pb, size_t *bytes);
int smfs_setup_far_field(smfs_problem *pb, void *scratch, size_t scratch_bytes, smfs_stream stream);

/* Install a factor of eq. transform (Section 2.2) computed elsewhere.
 * U [host] rows x rank column-major,
 * sigma [host] rank, V [host] cols x rank row-major.  Synchronises. */
int smfs_import_factor(smfs_problem *pb, int32_t fid, int32_t rank, const double *U,
                       const double *sigma, const double *V, smfs_stream stream);

/* One product y = G_hat mu (eq. resistance): lambda_hat = V S^-1 U^T mu per
 * sphere, then y_k = mu_k + W_k sum_{k' != k} G^(kk') lambda_hat_k'.
 * mu, y [dev] 3 T (must not alias).  precision SMFS_FP64, SMFS_MIXED,
 * SMFS_MIXED_FAR or SMFS_MIXED_EQ (SMFS_E_STATE before the far-field
 * set-up). */
int smfs_apply(smfs_problem *pb, const double *mu, double *y, int32_t precision,
               smfs_stream stream);

/* lambda [dev] S x 3 = B^+ mu, eq. (transform), in FP64. */
int smfs_transform(smfs_problem *pb, const double *mu, double *lambda, smfs_stream stream);

/* b [dev] 3 T = W (v + omega x (x - c) - u_inf(x)) from rbm [dev] P x 6,
 * eq. (bc); u_inf is the background flow set by smfs_set_background (zero
 * unless set). */
int smfs_rhs(smfs_problem *pb, const double *rbm, double *b, smfs_stream stream);

/* Background flow of the boundary data, eq. (bc) (Section 1; the paper's
 * examples of fixed clusters in a shear and in a uniform flow): a linear
 * flow u_inf(x) = U + L x with U [host] 3 and the constant velocity
 * gradient L [host] 3 x 3 row-major, L[3 i + j] = d u_inf_i / d x_j
 * (absolute coordinates x).  Either pointer may be NULL (that part is zero);
 * both NULL restores the quiescent fluid, the default.  From this call on,
 * smfs_rhs, the resistance solves (single and block), the mobility solve
 * (whose velocity rows then carry -W u_inf) and the check-point residuals of
 * this problem use v + omega x (x - c) - u_inf(x); lambda, forces and
 * torques are those of the disturbance flow.  Serving requests are always
 * in a quiescent fluid.  Host-side only, no device work.  Errors:
 * SMFS_E_INVALID_ARG for a non-finite entry or a gradient that is not
 * trace-free (|L00 + L11 + L22| > 1e-12 max |L_ij|: a linear flow solves
 * the homogeneous Stokes equations only when divergence-free). */
int smfs_set_background(smfs_problem *pb, const double *U, const double *L);

/* ft [dev] P x 6 from lambda [dev] S x 3: per sphere the summed Stokeslet
 * strengths and the rotlet strengths plus the Stokeslet moments about the
 * centre (Remark "Extracting net forces and torques", Section 2.3). */
int smfs_force_torque(smfs_problem *pb, const double *lambda, double *ft, smfs_stream stream);

/* u [dev] n x 3 = sum over every source of K(x - y) lambda at points x [dev]
 * n x 3 (flow evaluation, eq. uAll with no source skipped; the velocity
 * of eq. residual_x at check points). */
int smfs_eval_velocity(smfs_problem *pb, const double *lambda, int64_t n, const double *x,
                       double *u, smfs_stream stream);

/* Resistance solve: rbm [dev] P x 6 rigid-body velocities in, outputs per
 * smfs_out; the boundary data include the background flow if one is set
 * (smfs_set_background).  Returns SMFS_OK only when the FP64 true residual
 * ||b - G_hat mu|| / ||b|| meets gmres_tol; SMFS_STAGNATED (warning) when it
 * stopped falling above the tolerance (GMRES with a true-residual check,
 * Section 2.2: the rounding of the truncated pseudo-inverses, Section 5,
 * leaves a floor that the recursive estimate does not show); SMFS_NOT_CONVERGED
 * (warning) when gmres_max_it is reached first.  Statistics are filled in for
 * every warning.
 * Refinement: when the FP64 true residual misses the tolerance, up to two
 * sweeps solve G_hat d = r on the FP64 residual r and add d (a new Krylov
 * process starts below the rounding floor of the first); in FP64 only after
 * the iteration stopped (estimate or guard), in the mixed forms always; a
 * sweep that does not lower the true residual is taken back.
 * With params.precision = SMFS_MIXED, SMFS_MIXED_FAR or SMFS_MIXED_EQ the
 * products inside GMRES take the contact-free spheres' far field in reduced
 * precision as described at the precision modes, everything else in FP64;
 * Arnoldi, the true residual, the refinement residuals, the back-transform
 * and the forces stay in FP64. */
int smfs_solve_resistance(smfs_problem *pb, const double *rbm, smfs_out *out,
                          smfs_stream stream);

/* Change the solver settings of a problem after creation (the Krylov
 * restart length sizes the workspace and cannot change).  precision is
 * one of the modes above; gmres_max_it > 0; gmres_tol > 0. */
int smfs_set_solver(smfs_problem *pb, int32_t precision, double gmres_tol, int32_t gmres_max_it);

/* Mobility solve (forces and torques in, rigid motions out; Section 1
 * names the mobility problem beside the resistance problem of Section 2.2,
 * eq. resistance, without formulating it; this is the augmented form).
 * ft [dev] P x 6 = (F, T) exerted on the fluid.  Unknowns (mu, V): the rows
 * G_hat mu - W (v + omega x (x - c)) = -W u_inf at the collocation nodes
 * (u_inf = 0 unless set by smfs_set_background) and, per sphere, the force
 * and torque of lambda = B^+ mu equal to (F, T), scaled by 1/(6 pi mu a)
 * and 1/(8 pi mu a^3).  out->rbm receives V; other outputs as for
 * resistance (the check-point residual is measured against the V found). */
int smfs_solve_mobility(smfs_problem *pb, const double *ft, smfs_out *out, smfs_stream stream);

/* ---- Many right-hand sides ------------------------------------------
 * The block forms run nrhs independent systems with one geometry: every
 * source-target pair computed once serves a run of right-hand sides, and
 * the per-sphere pseudo-inverse (eq. transform) becomes a pair of small
 * GEMMs per sphere on the matrix cores.  A block workspace of device memory
 * is allocated by the caller; its size depends on nrhs and the Krylov
 * restart length.  Block products come in FP64 and in two mixed forms: the
 * proxies of contact-free spheres summed in FP32 from FP32 copies of their
 * FP64 strengths (SMFS_MIXED, SMFS_MIXED_FAR), or their far field through
 * the equivalent sources (SMFS_MIXED_EQ: strengths for every vector, FP32
 * sums for runs of vectors, near proxies in FP64); the block pseudo-inverse
 * and every other pair in FP64.
 *
 * Vectors of a block are stored one after another: vector q starts at
 * q * ld (ld >= 3 T elements, the same for input and output blocks). */

/* Bytes of block workspace for nrhs right-hand sides; restart = 0 sizes a
 * workspace for smfs_apply_block only, restart > 0 for
 * smfs_solve_resistance_block with that Krylov restart length. */
int smfs_block_workspace_bytes(const smfs_problem *pb, int32_t nrhs, int32_t restart,
                               size_t *bytes);

/* y_q = G_hat mu_q for q < nrhs (eq. resistance with the identity self
 * blocks of Section 2.2).  precision SMFS_FP64, SMFS_MIXED / SMFS_MIXED_FAR
 * or SMFS_MIXED_EQ (the mixed block forms above).  mu, y [dev]: nrhs
 * vectors of stride ld >= 3 T; mu and y must not overlap.  ws [dev]: at
 * least smfs_block_workspace_bytes(pb, nrhs, 0) bytes, 256-byte aligned. */
int smfs_apply_block(smfs_problem *pb, int32_t nrhs, const double *mu, double *y, int64_t ld,
                     int32_t precision, void *ws, size_t ws_bytes, smfs_stream stream);

/* smfs_apply_block for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the block workspace is a library-held device array of
 * smfs_noalloc_scratch_bytes() bytes (64 MiB) per GPU, kept until the
 * process ends; nothing is allocated by this call.  Inputs and outputs as
 * for smfs_apply_block (mu, y [dev], nrhs vectors of stride ld >= 3 T, not
 * overlapping); the result is bitwise that of smfs_apply_block.  Returns
 * SMFS_E_NOMEM, launching nothing, when the problem and nrhs need more
 * scratch than that (smfs_block_workspace_bytes(pb, nrhs, 0) tells).  All
 * calls on one GPU share its array: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.  Not
 * profiled by smfs_profile. */
int smfs_apply_block_noalloc(smfs_problem *pb, int32_t nrhs, const double *mu, double *y,
                             int64_t ld, smfs_stream stream);
size_t smfs_noalloc_scratch_bytes(void);

typedef struct smfs_block_out {
  double *ft;                  /* [dev, out] nrhs x P x 6 forces/torques, or NULL */
  double *mu;                  /* [dev, out] nrhs x 3T solutions (stride 3T), or NULL */
  int32_t *iterations;         /* [host, out] nrhs GMRES iteration counts, or NULL */
  double *true_rel_residual;   /* [host, out] nrhs values ||b - G_hat mu|| / ||b||, or NULL */
  int32_t max_iterations;      /* out: block products in the Krylov iterations */
  int32_t n_converged;         /* out: systems that ended converged: the GMRES estimate,
                                  or the FP64 residual at a restart, met gmres_tol */
  double t_gmres_ms, t_post_ms;
  int64_t pair_evals;          /* out: pair x right-hand-side evaluations */
  int64_t pair_evals_f32;      /* out: of which in FP32 (mixed precision) */
  int32_t refinements;         /* out: mixed precision: restarts from FP64 true residuals
                                  once every system stood converged (at most 2) */
} smfs_block_out;

/* Resistance solves (Section 2.2, eq. resistance) for nrhs rigid motions
 * together: rbm [dev] nrhs x P x 6.  Every system runs its own
 * GMRES(restart) with the problem's gmres_tol and gmres_max_it; the Krylov
 * iterations of all systems advance in lock step through block products, a
 * system that has converged stays frozen while the others go on.  The
 * products follow params.precision: in a mixed form every restart takes the
 * FP64 true residuals, and once every system stands converged (on its
 * estimate, or on the FP64 residual of a restart) while some FP64 residual
 * misses the tolerance, the systems restart from them up to twice (those
 * above the tolerance go on); FP64 block solves take no such refinement
 * (unlike smfs_solve_resistance).  ws as above with restart > 0.  Returns
 * SMFS_OK when every FP64 true residual met gmres_tol, SMFS_STAGNATED when
 * every system stood converged but some true residual did not meet it,
 * SMFS_NOT_CONVERGED otherwise. */
int smfs_solve_resistance_block(smfs_problem *pb, int32_t nrhs, const double *rbm, int32_t restart,
                                void *ws, size_t ws_bytes, smfs_block_out *out,
                                smfs_stream stream);

/* ---- Serving --------------------------------------------------------
 * A server holds many independent resistance problems (Section 2.2, eq.
 * resistance; different sphere counts and packings, one discretisation)
 * resident on one GPU and advances them together.  Requests are admitted in
 * arrival order when their workspace fits into the server's device arena
 * and a slot is free; set-up worker threads build and factorise admitted
 * requests in batches on their own streams while the resident requests
 * keep iterating.  Every call of smfs_server_step performs iters_per_step
 * GMRES iterations of every resident request: one launch of each kernel of
 * the product with G_hat, of the Arnoldi step and of the Givens step covers
 * all of them, and a request that arrives between steps joins at the next
 * one (continuous batching).  A finished request leaves at once and its
 * memory and slot go to the next waiting request.  Every request keeps the
 * chunking and summation order of its own problem in every kernel, so a
 * result does not depend on which other requests share the launches.
 *
 * The shared factor of contact-free spheres (Section 2.2, eq. transform)
 * depends only on the discretisation: the server factorises it once and
 * copies it into each request.
 *
 * Precision: SMFS_FP64, or SMFS_MIXED_FAR (the far field of each request's
 * contact-free proxies summed in FP32 from FP64 strengths inside the
 * Krylov iterations; pseudo-inverses, contact spheres, image lines, Arnoldi
 * and every restart's true residual in FP64).  A cycle whose estimate meets
 * the tolerance restarts from the FP64 true residual (up to two such
 * refinements) before the request finishes, so the FP32 far field costs no
 * accuracy beyond the tolerance.
 *
 * Memory: the caller gives the server one block of device memory, kept
 * until smfs_server_destroy: a fixed part (smfs_server_memory_bytes: the
 * shared factor, per-slot descriptors, every set-up worker's scratch) and
 * an arena (the rest) that holds the requests' workspaces.  The server
 * allocates no device memory; rocSOLVER works in the workers' scratch. */
typedef struct smfs_server smfs_server;

typedef struct smfs_server_config {
  double radius;                /* the common sphere radius of every request */
  int32_t max_active;           /* slots: requests resident together, including those
                                   being set up, 1..4096 */
  int32_t setup_workers;        /* threads building admitted requests, 1..64, each with
                                   its own stream and rocBLAS handle */
  int32_t max_queued;           /* requests waiting for admission; smfs_server_submit returns
                                   SMFS_E_AGAIN when this many wait (0: no limit) */
  int32_t precision;            /* SMFS_FP64 or SMFS_MIXED_FAR */
  size_t worker_scratch_bytes;  /* device scratch per set-up worker: a quarter (at least
                                   64 MiB) for rocSOLVER's work arrays, the rest for the
                                   batched SVD inputs and outputs (0: 4 GiB) */
  int32_t iters_per_step;       /* GMRES iterations of the resident requests per
                                   smfs_server_step, 1..1024 (0: 8) */
  int32_t setup_batch;          /* most requests a worker sets up together, 1..64 (0: 64):
                                   smaller batches become resident sooner */
} smfs_server_config;

/* Defaults: radius 1, 64 slots, 1 worker, no queue limit, FP64, 4 GiB, 8
 * iterations per step, set-up batches of up to 64 requests. */
int smfs_server_config_default(smfs_server_config *c);

/* Bytes of the fixed part of the server's device memory for these
 * settings (host only); the arena is whatever the caller adds to it. */
int smfs_server_memory_bytes(const smfs_params *p, const smfs_server_config *c, size_t *fixed_bytes);

/* p: discretisation and solver settings of every request (gmres_restart is
 * the Krylov restart length, which sets each request's footprint;
 * p->precision is replaced by c->precision).  dev_mem [dev]: dev_bytes of
 * device memory, 256-byte aligned, owned by the caller and used by the
 * server until smfs_server_destroy; the part beyond
 * smfs_server_memory_bytes is the arena.  A worker takes every request that
 * can be admitted at that moment (up to setup_batch) and factorises the self blocks
 * of all their contact spheres together: batched SVDs per block shape, each
 * call of a fixed batch count for its shape (set by the shape and the
 * worker's scratch alone, so that a request's factors do not depend on its
 * neighbours).  Errors: SMFS_E_INVALID_ARG (bad settings or pointer),
 * SMFS_E_UNSUPPORTED (precision), SMFS_E_NOMEM (no room for an arena that
 * holds a one-sphere request). */
int smfs_server_create(const smfs_params *p, const smfs_server_config *c, void *dev_mem, size_t dev_bytes,
                       smfs_server **out);
/* Waits for the worker threads and releases the server's host resources;
 * the caller's device memory is free again afterwards. */
void smfs_server_destroy(smfs_server *srv);

/* Seconds on the clock the server stamps requests with (monotonic). */
double smfs_server_clock(void);

/* Queue a request: P spheres with centres [host] P x 3 (all of radius
 * `radius`), rigid motions rbm [host] P x 6.  t_arrival: its arrival time on
 * smfs_server_clock (latency is measured from it); a negative value means
 * now.  Geometry is built here, on the calling thread; *id receives the
 * request's handle.  SMFS_E_NOMEM when the request alone does not fit into
 * the arena; SMFS_E_AGAIN (nothing queued) when max_queued requests are
 * already waiting for admission. */
int smfs_server_submit(smfs_server *srv, int32_t P, const double *centers, const double *rbm,
                       double t_arrival, int64_t *id);

/* iters_per_step GMRES iterations of every resident request (see above),
 * with no host round trip between them: the Givens rotations, the
 * convergence estimate and the end of a restart cycle are taken on the
 * device, where each request's cycle state (Arnoldi index, rotated
 * Hessenberg columns, rotations, rotated right-hand side) lives; a request
 * that meets its estimate, its iteration limit or the end of its cycle
 * drops out of the remaining launches of the step.  The host then restarts
 * such requests from their FP64 true residual or completes them (true
 * residual, forces and torques), and finished requests leave.  *n_active:
 * requests resident after the step; *n_waiting: requests queued or being
 * set up.  Returns at once when nothing is resident. */
int smfs_server_step(smfs_server *srv, int32_t *n_active, int32_t *n_waiting);

typedef struct smfs_request_result {
  int32_t status;              /* SMFS_OK (FP64 true residual met gmres_tol), SMFS_STAGNATED
                                  (it stopped above), SMFS_NOT_CONVERGED (iteration limit)
                                  or an error code */
  int32_t P;
  int32_t iterations;
  int32_t restarts;
  double rel_residual;         /* GMRES estimate */
  double true_rel_residual;    /* ||b - G_hat mu|| / ||b|| in FP64 */
  double t_arrival, t_admitted, t_started, t_done;   /* smfs_server_clock seconds */
  int64_t pair_evals;
  int64_t pair_evals_f32;      /* of which in FP32 (SMFS_MIXED_FAR) */
  int32_t refinements;         /* restarts from the FP64 true residual after the estimate met
                                  the tolerance */
  char error[160];             /* message of a failed request (empty otherwise) */
} smfs_request_result;

/* Result of request id: returns 0 and fills *res (and ft [host] P x 6
 * forces/torques, when not NULL) once the request has finished, 1 while it
 * is waiting or running, SMFS_E_INVALID_ARG for an unknown id.  A finished
 * request's result stays available until smfs_server_release(id). */
int smfs_server_poll(smfs_server *srv, int64_t id, smfs_request_result *res, double *ft);
int smfs_server_release(smfs_server *srv, int64_t id);

typedef struct smfs_server_stats {
  int64_t steps;               /* calls of smfs_server_step that iterated */
  int64_t request_iterations;  /* GMRES iterations summed over the requests */
  int64_t completed, failed;
  size_t arena_bytes, arena_peak;
  int32_t peak_active;
  double step_ms;              /* wall time inside smfs_server_step */
  double tick_ms;              /* of which the batched iteration (launches and readback) */
  double setup_ms;             /* worker time building and factorising requests */
  int64_t setup_batches;       /* admission batches set up */
  int64_t iterations;          /* batched iterations launched (steps x iters_per_step) */
} smfs_server_stats;
int smfs_server_stats_read(smfs_server *srv, smfs_server_stats *st);

/* Pair evaluations in one product with G_hat (all off-sphere pairs). */
int64_t smfs_pairs_per_apply(const smfs_problem *pb);

/* Per-launch timing of the two kernels of each product with G_hat, taken
 * with HIP events recorded on the caller's stream around every launch.
 * Algorithmic work per product: the direct sum does 28, 25 and 30 flops per
 * Stokeslet, rotlet and dipole pair; the pseudo-inverse apply reads each
 * distinct factor once (8 bytes per kept entry of U and V; the shared
 * factor of the contact-free spheres once for all of them) plus mu and
 * lambda. */
typedef struct smfs_kernel_stats {
  int64_t direct_launches;
  double direct_ms;         /* summed over launches */
  double direct_flops;      /* algorithmic flops per launch (FP64 product) */
  int64_t pinv_launches;
  double pinv_ms;           /* U^T mu and V s kernels together */
  double pinv_bytes;        /* algorithmic bytes per launch pair (FP64 product) */
  int64_t far32_launches;   /* mixed precision: FP32 direct sum */
  double far32_ms;
  double far32_flops;       /* algorithmic flops per launch (28 per pair) */
  int64_t mixed64_launches; /* mixed precision: FP64 part of the direct sum */
  double mixed64_ms;
  double mixed64_flops;     /* FP64 direct-sum flops per mixed product */
  int64_t bdirect_launches; /* block product: direct sum over nrhs vectors */
  double bdirect_ms;
  double bdirect_flops;     /* per launch: pairs x (geometry + nrhs x per-vector flops) */
  int64_t bpinv_launches;   /* block product: MFMA pseudo-inverse GEMMs */
  double bpinv_ms;
  double bpinv_flops;       /* per launch: 2 nrhs (rank (rows + cols)) summed over spheres */
  int32_t bnrhs;            /* right-hand sides of the last profiled block product */
  int64_t eq_launches;      /* SMFS_MIXED_EQ products */
  double eq_far_ms;         /* FP32 equivalent-source sum */
  double eq_far_flops;      /* per launch: 28 per pair */
  double eq_near_ms;        /* FP64 sum of the near contact-free proxies */
  double eq_near_flops;     /* per launch: 28 per pair */
  double eq_strength_ms;    /* equivalent strengths q = E lambda_hat */
} smfs_kernel_stats;

/* enable = 1 clears the counters and starts recording; 0 stops. */
int smfs_profile(smfs_problem *pb, int32_t enable);
/* Waits for the recorded events and fills *st. */
int smfs_profile_read(smfs_problem *pb, smfs_kernel_stats *st);

const char *smfs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SMFS_H */
