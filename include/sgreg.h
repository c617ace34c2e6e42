/*
 * sgreg — shape-constrained gravitational point-cloud registration on
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Method: Agarwal & Bhowmick, "3D Point Cloud Registration with Shape
 * Constraint" (arXiv 1902.01061).  Given a template cloud Y (M points) and a
 * reference cloud X (N points) with nothing but xyz coordinates (no colour,
 * texture, correspondences or topology; Sec. I), find the translation,
 * rotation and isotropic scale that align the template to the reference.
 * Each template point is attracted by every reference point with a force
 * weighted by the similarity of the two points' local curvature (eqs. 2-5,
 * 10, 11); the net force and moment drive a Newtonian translation (eq. 5.5),
 * a Kabsch rotation (eq. 6) and an eigenvalue-ratio scale (eq. 8), iterated
 * with the G schedule of eq. (12).
 *
 * Conventions used by every call:
 *  - All array pointers are DEVICE pointers on the context's GPU, owned by
 *    the caller; the library never frees them and never keeps them past the
 *    call (except inside a graph it captured for an identical later call).
 *  - Clouds are structure-of-arrays float32 (x[n], y[n], z[n]); `m` is an
 *    optional float32 mass per point (NULL = unit masses, Sec. IV).
 *  - A pose maps template coordinates into the reference frame:
 *    T(y) = s R y + t with R row-major (13 doubles: s, R[9], t[3]).
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the
 *    default stream) unless stated otherwise.
 *  - Return value: SGR_OK (0) or a negative error code; sgr_last_error()
 *    gives a message for the calling thread.
 *  - There is no CPU code path: every step runs in HIP kernels.
 */
#ifndef SGREG_H
#define SGREG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SGR_OK 0
#define SGR_EINVAL (-1)      /* bad argument: NULL pointer, n < k+1, sigma/eps/p out of range */
#define SGR_EDEGENERATE (-2) /* a cloud with zero variance (no length scale / scale ratio) */
#define SGR_EHIP (-3)        /* a HIP runtime call failed; message has hipGetErrorString */
#define SGR_ENOMEM (-4)      /* workspace allocation failed */
#define SGR_ENUMERIC (-5)    /* device status word: non-finite or rank-deficient update */

typedef struct sgr_ctx sgr_ctx;
typedef void* sgr_stream_t; /* hipStream_t */

typedef struct {
  const float* x;
  const float* y;
  const float* z;
  const float* m; /* per-point mass or NULL (unit masses) */
  int64_t n;
} sgr_cloud;

typedef struct {
  double s;
  double R[9];
  double t[3];
} sgr_pose;

/* Parameters of the method.  Readings of passages the paper leaves open:
 *  p      distance exponent of eq. (11), h(d) n = d^(p-1) r, p >= 1
 *         (p < 1 only with eps > 0; p = -1, whose potential is a
 *         logarithm, is rejected).  1 is the default: larger p overshoots
 *         (Sec. IV warns of oscillation), p = 2 flips the template once
 *         G dt2 nears 1.
 *  g_mode 0: g = s (Sec. IV, equal weightage); 1: g = (a_i/abar)(a_j/abar) s
 *         (eq. 10), abar = mean reference curvature; 2: g = 1 (no shape
 *         term, the masses alone weight the pairs).  p = -2 with eps > 0 and
 *         g_mode 2 is the gravitational force of eq. (1) (inverse square
 *         with softening), without its velocity (friction) state.
 *  k      neighbours (self included) for the curvature descriptor.
 *  sigma  RBF spread of eq. (3); <= 0 selects the population std of the
 *         reference curvatures.
 *  eps    softening added to the distance law: h = ((d^2+eps^2)/L^2)^((p-1)/2),
 *         L = sqrt(largest eigenvalue of the reference covariance); 0 is the
 *         paper's law.
 *  G1, E  eq. (12): iteration t (0-based) uses
 *         G_t = 0.1 G1 + 0.9 G1 / (1 + exp(-(t - 1 - E/2))); E iterations.
 *  dt2    the squared time step of eq. (5.5); only G dt2 matters; <= 0
 *         selects 1/G1 so G_t dt2 runs over [0.1, 1].
 *  The force is normalised by Z = sum of reference masses. */
typedef struct {
  double p;
  int32_t g_mode;
  int32_t k;
  double sigma;
  double eps;
  double G1;
  int32_t E;
  int32_t flags; /* bit 0: no graph capture in sgr_register / batch calls;
                    bit 1: mixed precision (p = 1 only): the similarity-weighted
                    sums over the reference run as a bf16 matrix product on the
                    matrix cores (pair weights FP32, rounded to bf16; coordinates
                    split into bf16 head + tail; FP32 accumulate, FP64 wrench);
                    the energy U is then reported as 0 except for the last
                    iteration of sgr_register with stats, which runs the FP32
                    kernel; not for batch calls;
                    bit 2: vector descriptors (sgr_step_vec, sgr_register_vec)
                    with FP32 matrix products instead of the split-f16 form;
                    bit 3: pose-independent pair sums (sgr_register,
                    sgr_register_pyramid, sgr_register_batch, sgr_multistart,
                    sgr_register_vec; p = 1, g_mode 0 or 1, no mixed
                    precision; SGR_EINVAL otherwise).  With p = 1 (eq. 11,
                    h = 1) the pair weight of eq. 5 does not depend on the
                    pose, so sum_j c_ij, sum_j c_ij x_j and sum_j c_ij |x_j|^2
                    are formed once (one pass over all pairs, FP32 terms and
                    FP64 sums) and every iteration costs O(M): f_i =
                    -(G/Z) g_i (y_i sum_j c_ij - sum_j c_ij x_j).  Same
                    results as the per-iteration all-pairs kernel up to
                    rounding (workspace: about 48 bytes per template point
                    per reference chunk). */
  double dt2;
  double momentum; /* mu in [0, 1): the template's velocity state (eq. 5.5's
                      v^X, damped by eq. 1's friction -eta v, mu = 1 - the
                      friction's share).  Its velocity in the previous
                      iteration is its translation d then, and every point
                      carries mu d on top of dt2 f_i: d(t) = dt2 F / sum m +
                      mu d(t-1); the rotation is unchanged (a shift common
                      to all points).  The template starts at rest in every
                      registration (and every pyramid level).  0 (default) is
                      the paper's v = 0; calls without an iteration loop
                      (sgr_step, plans, the adjoint, sgr_step_vec) reject
                      mu != 0 with SGR_EINVAL. */
} sgr_params;

/* Context on HIP device `device`: owns the workspace, captured graphs and the
 * tile table.  The only memory the library allocates. */
int sgr_create(sgr_ctx** ctx, int device);
int sgr_destroy(sgr_ctx* ctx);
const char* sgr_last_error(void);

/* "descriptors(cloud)" (Sec. III-A, curvature; Sec. III-B, moments).
 * a_out[n] (float32): PCA surface variation lambda_0/(lambda_0+lambda_1+lambda_2)
 *   of the covariance (1/k, centred) of the k nearest neighbours, self
 *   included; neighbours ranked by float32 squared distance
 *   ((dx*dx + dy*dy) + dz*dz, each operation rounded) then by index.
 * moments_out[10] (float64, nullable): centroid[3], covariance (1/n)
 *   xx yy zz xy xz yz, largest eigenvalue.
 * Errors: SGR_EINVAL if k < 1, k > 32 or n < k. */
int sgr_descriptors(sgr_ctx* ctx, const sgr_cloud* c, int k, float* a_out, double* moments_out,
                    sgr_stream_t stream);

/* The k-nearest-neighbour lists behind sgr_descriptors: idx_out[n][k]
 * (int32), row i sorted by (float32 squared distance, index). */
int sgr_knn(sgr_ctx* ctx, const sgr_cloud* c, int k, int32_t* idx_out, sgr_stream_t stream);

/* "descriptors(cloud)" for many clouds at once (the batched registrations'
 * descriptors): the same exact k nearest neighbours and curvature (Sec.
 * III-A) as sgr_knn / sgr_descriptors on each cloud, with one launch per
 * phase of the grid search for all clouds.  a_out[c] (device float32
 * [n_c], or a_out NULL) receives cloud c's curvatures; idx_out (nullable;
 * entries nullable) its neighbour lists int32 [n_c][k] as sgr_knn writes
 * them.  Synchronises the stream once.  SGR_EINVAL for k outside [1, 32], a
 * cloud with fewer than k points, or no output. */
int sgr_descriptors_batch(sgr_ctx* ctx, int n_clouds, const sgr_cloud* clouds, int k, float* const* a_out,
                          int32_t* const* idx_out, sgr_stream_t stream);

/* "step(template, reference, pose)": exactly one iteration t of Sec. III
 * from pose `in`, writing `out` (device; may alias `in`).
 * a_t[M], a_r[N]: curvatures (e.g. from sgr_descriptors); mom_t, mom_r: the
 * moments_out of the INPUT template and of the reference.
 * wrench_out[13] (nullable): F[3] = sum_i m_i f_i, K[9] = sum_i f_i
 *   (y_i - ybar)^T row-major, U (energy whose negative gradient is f).
 * f_out[M][3] (nullable, float32): per-point force f_i at pose `in`. */
int sgr_step(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref,
             const float* a_r, const double* mom_t, const double* mom_r, const sgr_params* prm,
             int t, const sgr_pose* in, sgr_pose* out, double* wrench_out, float* f_out,
             sgr_stream_t stream);

/* sgr_step for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and kernels as sgr_step, bit for bit;
 * the step's intermediate buffers (set-up constants, packed clouds, visiting
 * order and its sort temporaries, wrench partials, per-chunk forces) come
 * from a static 64 MiB device array per GPU (SGR_STATIC_SCRATCH_BYTES)
 * instead of the context workspace, and nothing is allocated or freed.
 * The array is held from the library's loading on that GPU until the process
 * ends; its device address is taken by sgr_create.  Limit: a pair needs
 * roughly 20 N + 60 M bytes plus, with f_out, 24 M bytes per reference chunk;
 * SGR_EINVAL with the byte count when a call needs more than the array (the
 * depth-frame scene, 250 000 x 307 200, fits).  No part of the array needs
 * to start at any value.  Every call on one GPU uses the same array: calls
 * that overlap in time on one GPU (from several threads, or on several
 * streams without ordering) race and give wrong results; calls ordered on
 * one stream are safe. */
#define SGR_STATIC_SCRATCH_BYTES (64u << 20)
int sgr_step_static(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref,
                    const float* a_r, const double* mom_t, const double* mom_r, const sgr_params* prm,
                    int t, const sgr_pose* in, sgr_pose* out, double* wrench_out, float* f_out,
                    sgr_stream_t stream);

/* "register(template, reference, params) -> pose" (Sec. I's problem: the
 * translation, rotation and scale that align the template to the
 * reference): curvature descriptors of both clouds (Sec. III-A), then E
 * iterations of Sec. III from the pose in `inout` (device), written back in
 * place: the shape-weighted force (eqs. 3, 5, 10, 11), translation (eq.
 * 5.5), rotation (eq. 6), scale (eq. 8), update (eq. 9), G from eq. 12.  stats (nullable, device float64 [E][32]): per iteration G_t,
 * F[3], K[9], U, the pose after the update (13), the scale factor c and the
 * status word.  Synchronises the stream at the end to read the device
 * status word; SGR_ENUMERIC if an update went non-finite or rank deficient
 * (the pose is then frozen at the last good value). */
int sgr_register(sgr_ctx* ctx, const sgr_cloud* tmpl, const sgr_cloud* ref, const sgr_params* prm,
                 sgr_pose* inout, double* stats, sgr_stream_t stream);

/* Curvature of radius neighbourhoods (Sec. IV sets the radius of the local
 * neighbourhood to sqrt(eX) for the reference and sqrt(eY) for the template,
 * eX and eY the largest covariance eigenvalues of Sec. III-B; moments_out[9]
 * of sgr_descriptors is that eigenvalue).  The members of point i are the
 * points j whose float32 key ((dx*dx + dy*dy) + dz*dz, each operation
 * rounded, the key of sgr_knn) is <= r2, i itself included.
 * a_out[n] (float32, nullable): surface variation of the members' covariance
 *   (1/n_i, centred at their mean), 0 if its trace is 0, NaN if i has no
 *   member (a non-finite point).
 * count_out[n] (int32, nullable): n_i.
 * The points are visited in Morton order in tiles of 256; a tile whose
 * bounding box is provably farther than sqrt(r2) from a block of 64 queries
 * is skipped, so the cost falls with r2 (n^2 key evaluations at most) and the
 * counts are exactly those of the full scan.  Uses the context workspace
 * (64 bytes per point and the radix sort's temporaries); the call is
 * asynchronous on stream.
 * Errors: SGR_EINVAL if r2 is negative or not finite, or both outputs are
 * NULL; SGR_ENOMEM if the workspace cannot grow. */
int sgr_descriptors_radius(sgr_ctx* ctx, const sgr_cloud* c, float r2, float* a_out, int32_t* count_out,
                           sgr_stream_t stream);

/* One level of the pyramidal schedule (Sec. IV: for noisy data the size of
 * the neighbourhood and sigma of eq. (3) decrease with the iterations).
 *  radius_scale > 0: radius neighbourhoods of radius radius_scale *
 *                sqrt(lambda_max) of each cloud's own covariance (1 is the
 *                paper's sqrt(eX), sqrt(eY)); the float32 threshold is
 *                (float)((radius_scale * radius_scale) * lambda_max).
 *  radius_scale = 0: the k nearest neighbours (k in [1, 32]).
 *  sigma_scale > 0: multiplies the level's sigma (params.sigma if > 0, else
 *                the std of the level's reference curvatures).
 *  iters >= 1: iterations run with this level's curvatures. */
typedef struct {
  double radius_scale;
  double sigma_scale;
  int32_t iters;
  int32_t k;
} sgr_level;

/* "register" through the levels in order: each level recomputes both
 * clouds' curvatures, sigma and the packed clouds, then runs its iterations
 * from the pose the previous level reached.  t runs on across the levels,
 * so G (eq. 12) follows prm->E, which must equal the sum of the levels'
 * iters; prm->k is not used (each level names its neighbourhood).  inout,
 * stats and the errors as in sgr_register (the failing level is named);
 * levels is host memory, 1 <= n_levels <= 64. */
int sgr_register_pyramid(sgr_ctx* ctx, const sgr_cloud* tmpl, const sgr_cloud* ref, const sgr_params* prm,
                         const sgr_level* levels, int n_levels, sgr_pose* inout, double* stats,
                         sgr_stream_t stream);

/* Vector shape descriptor (Sec. III-A lists histograms of normals among
 * the local shape features): h_out[n][D] (float32, row-major), the soft
 * histogram of u = |n_i . n_j| over the k nearest neighbours j of point i
 * (self included, lists as sgr_knn), n the unit normal (eigenvector of the
 * smallest eigenvalue of the neighbourhood covariance, 1/k, centred; its sign
 * is arbitrary, hence |.|).  Bin b (centre b/(D-1)) receives the tent weight
 * max(0, 1 - (D-1)|u - b/(D-1)|); h_i sums to 1.  A point with a non-finite
 * neighbour normal gets NaN.  Where the two smallest eigenvalues coincide the
 * normal, and with it h, is not determined.
 * Errors: SGR_EINVAL if k < 1, k > 32, n < k, or D outside [2, 30]. */
int sgr_descriptors_hn(sgr_ctx* ctx, const sgr_cloud* c, int k, int D, float* h_out, sgr_stream_t stream);

/* Vector shape descriptor from local polynomial coefficients (Sec. III-A
 * lists them among the local shape features; the paper gives no definition,
 * this is the reading used).  For every point, its k nearest neighbours (the
 * neighbour lists of sgr_knn) are expressed in the frame of their covariance
 * (1/k, centred at their mean: tangent axes of the two largest eigenvalues,
 * normal of the smallest), every coordinate divided by rho = sqrt(trace);
 * a quadric h = c0 + c1 u + c2 v + c3 u^2 + c4 u v + c5 v^2 is fitted by least
 * squares (FP64 normal equations), and
 *   out[i][0..2] = (mu1, mu2, r): mu1 >= mu2 the eigenvalues of the fitted
 *   Hessian [[2 c3, c4], [c4, 2 c5]] (both negated and swapped when their
 *   sum is negative, since the normal's sign is arbitrary) and r the RMS
 *   residual of the fit,
 * float32, row-major [n][3], device, caller-owned.  The three numbers do not
 * change under rotation, translation, uniform scale, or a change of sign or
 * an in-plane rotation of the frame; they feed sgr_step_vec /
 * sgr_register_vec with D = 3.  NaN for a point whose neighbours coincide
 * (rho = 0) or lie on a line (singular normal equations).  The frame, and so
 * the descriptor, is determined only where the smallest covariance
 * eigenvalue is below the middle one.  Uses the context workspace;
 * asynchronous on stream.
 * Errors: SGR_EINVAL for NULL arguments, k outside [6, 32] or n < k. */
int sgr_descriptors_poly(sgr_ctx* ctx, const sgr_cloud* c, int k, float* out, sgr_stream_t stream);

/* sgr_step and sgr_register with vector descriptors: eq. (3) with
 * |a_i - a_j|^2 summed over D dimensions, a_t[M][D] and a_r[N][D] (device,
 * float32, row-major; e.g. from sgr_descriptors_hn).  sigma <= 0 selects
 * sigma^2 = mean_j |a_j - abar|^2 over the reference (abar its mean; the std
 * of the scalar case when D = 1).  The similarity exponents of all pairs are
 * one dense contraction on the matrix cores: by default each entry of the
 * standardised operands is split into an f16 head and tail, and head.head +
 * head.tail + tail.head is one f16 contraction of length 3 (D + 2)
 * accumulated in FP32 (about 2^-22 relative per product); FP32
 * products (flags bit 2, and automatically when a standardised descriptor
 * lies more than about 140 spreads from the mean, beyond the f16 range) are
 * about 2^-24.  The set-up synchronises the stream once to make that choice.
 * Supported:
 * p = 1, g_mode 0, no mixed precision, 1 <= D <= 30 (SGR_EINVAL otherwise).
 * Other arguments, outputs and errors as in sgr_step / sgr_register
 * (sgr_register_vec computes the moments itself; SGR_EDEGENERATE also for
 * zero descriptor spread). */
int sgr_step_vec(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                 int D, const double* mom_t, const double* mom_r, const sgr_params* prm, int t,
                 const sgr_pose* in, sgr_pose* out, double* wrench_out, float* f_out, sgr_stream_t stream);
int sgr_register_vec(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                     int D, const sgr_params* prm, sgr_pose* inout, double* stats, sgr_stream_t stream);

/* "residual": the root mean square error by which Sec. V scores a
 * registration (its protocol follows a reference that is not given, so the
 * two usual forms are offered).
 * With corr (int32[M], -1 = none): sqrt(mean |T(y_i) - x_corr(i)|^2)
 * over i with corr >= 0; with corr == NULL: one-sided nearest-neighbour RMSE
 * template -> reference (nearest by float32 distance of the float32-rounded
 * transformed point, the distance itself in float64).  rmse_out: device
 * float64 [1]. */
int sgr_residual(sgr_ctx* ctx, const sgr_cloud* tmpl, const sgr_cloud* ref, const sgr_pose* pose,
                 const int32_t* corr, double* rmse_out, sgr_stream_t stream);

/* A prepared (template, reference) pair for repeated force evaluation:
 * the per-registration constants (curvature statistics, length scale,
 * masses) and the reference packed for the pair loop are computed once, on
 * `stream`, into plan-owned device memory.  The cloud, curvature and moment
 * arrays must stay valid and unchanged while the plan is used. */
typedef struct sgr_plan sgr_plan;
int sgr_plan_create(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                    const double* mom_t, const double* mom_r, const sgr_params* prm, sgr_plan** plan,
                    sgr_stream_t stream);
int sgr_plan_destroy(sgr_plan* plan);

/* The shape-weighted all-pairs force of eq. (5) (with eqs. 3, 10, 11) at
 * pose `pose`, reduced to the wrench: wrench_out[13] = F[3], K[9], U as in
 * sgr_step; f_out[M][3] the per-point forces.  G <= 0 takes G_t of eq. (12)
 * at iteration t.  With both outputs NULL only the force kernel runs (its
 * partial sums stay in plan memory); used for timing. */
int sgr_plan_force(sgr_plan* plan, int t, double G, const sgr_pose* pose, double* wrench_out, float* f_out,
                   sgr_stream_t stream);

/* Launch shape of the pair-force kernel for the size bucket of (M, N) and
 * the distance-law mode of p (1, 3 or other): R template points per lane
 * (1, 2, 4 or 8), a target of blocks_per_cu blocks of 256 threads per
 * compute unit (each template block's reference range is cut into equal
 * chunks at multiples of 64 points to reach it; without an entry the
 * target is one wave of resident blocks, from the kernel's occupancy) and
 * the variant (0: reference tiles staged in LDS; 1: read through scalar
 * loads).  Affects plans and calls created afterwards.  R = 0 removes the
 * entry. */
int sgr_set_tiles(sgr_ctx* ctx, int64_t M, int64_t N, double p, int R, int blocks_per_cu, int variant);

/* Autotuner: times the pair-force kernel for every launch shape (R in
 * {1, 2, 4, 8}, LDS or scalar-load variant, 1 to 4 blocks per CU and 1 to 8
 * waves of resident blocks, at most 64 blocks per CU) on this pair, `reps`
 * launches each, and stores the fastest in the
 * tile table for the (M, N, p) bucket.  best (host int[3], nullable): R,
 * blocks_per_cu, variant; best_ms (host, nullable): its time per launch.
 * Synchronises the stream. */
int sgr_autotune(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                 const double* mom_t, const double* mom_r, const sgr_params* prm, int reps, int* best,
                 double* best_ms, sgr_stream_t stream);

/* Persist / restore the tile table as JSON {"arch": ..., "entries": [...]};
 * loading a table written for another architecture fails (SGR_EINVAL). */
int sgr_tiles_save(sgr_ctx* ctx, const char* path);
int sgr_tiles_load(sgr_ctx* ctx, const char* path);

/* The force field at template positions `tmpl` (used as they are, identity
 * pose): f_out[M][3] (float32) and wrench_out[13] (F, K, U as in sgr_step),
 * with force constant G > 0.  mom_r: reference moments.  The forward pass
 * of the differentiable force field. */
int sgr_force_fwd(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                  const double* mom_r, const sgr_params* prm, double G, float* f_out, double* wrench_out,
                  sgr_stream_t stream);

/* Adjoint of sgr_force_fwd.  Inputs: f[M][3] from the forward pass, the
 * upstream gradients grad_f[M][3] (float32, nullable = 0) and
 * grad_wrench[12] (F then K row-major, float64, nullable = 0).  Outputs:
 * grad_y[M][3] (float32) w.r.t. template positions, grad_m[M] (nullable)
 * w.r.t. template masses, grad_se[2] (nullable, float64) w.r.t. the
 * similarity spread sigma (which must be given, > 0) and the softening eps.
 * The curvatures are held constant (they do not depend on the pose). */
int sgr_force_bwd(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                  const double* mom_r, const sgr_params* prm, double G, const float* f, const float* grad_f,
                  const double* grad_wrench, float* grad_y, float* grad_m, double* grad_se, sgr_stream_t stream);

/* Differentiable registration, forward (Sec. III-B iterated, eq. 12): E =
 * prm->E iterations of the force (eqs. 3, 5, 10, 11) and the rigid update
 * (eqs. 5.5, 6, 8, 9) from the pose in `pose` (device, updated in place),
 * with the curvatures a_t, a_r (device float32) held constant and the input
 * moments mom_t, mom_r (device float64[10], as sgr_descriptors returns).
 * The pose before iterations 0, K, 2K, ... is stored in
 * ckpt[ceil(E / K)][13] (device float64): only poses are checkpointed.
 * sigma must be given (> 0); the FP32 force is used (the mixed flag is
 * rejected) and the update's SVD starts cold, so that a segment recomputed
 * from its checkpoint reproduces the forward poses bit for bit. */
int sgr_unrolled_fwd(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                     const double* mom_t, const double* mom_r, const sgr_params* prm, int K, sgr_pose* pose,
                     double* ckpt, sgr_stream_t stream);

/* Reverse pass of sgr_unrolled_fwd: given grad_final[13] = dL/d(final
 * pose) (device float64), writes grad_pose0[13] = dL/d(initial pose) and
 * grad_se[2] = dL/d(sigma, eps) (device float64).  Walks the iterations
 * backwards, recomputing each K-iteration segment from its checkpoint; per
 * iteration: the per-point forces and wrench at that pose, the adjoint of
 * the rigid update (Kabsch polar factor, scale, translation, re-
 * orthonormalisation), the adjoint of the force field at the posed template
 * (as sgr_force_bwd) and the pullback of its per-point gradient onto the
 * pose.  Same arguments as the forward pass, which must have run with
 * them.  Assumes every update was applied (status 0). */
int sgr_unrolled_bwd(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                     const double* mom_t, const double* mom_r, const sgr_params* prm, int K, const double* ckpt,
                     const double* grad_final, double* grad_pose0, double* grad_se, sgr_stream_t stream);

/* Change detection after registration (the application of Sec. I and
 * Sec. IV: registered template parts with no similar reference part nearby
 * show the change).  For every template point i, posed by `pose` (device,
 * 13 float64) as T(y_i) = s ((R_r0 y_0 + R_r1 y_1) + R_r2 y_2) + t_r in FP64
 * with every operation rounded on its own, then rounded to float32, and with
 * j its nearest reference point among those whose float32 key ((dx*dx +
 * dy*dy) + dz*dz) is <= (float)(tau^2), ties by index as the descriptors'
 * neighbours:
 *   flags_out[i] bit 0: there is no such point        (nothing within tau),
 *   flags_out[i] bit 1: (a_i - a_j)^2 > sigma^2 (-ln s_min) in FP64, i.e.
 *                       the shape similarity of eq. 3 is below s_min.
 * tau > 0 (+inf: the nearest point at any distance, bit 0 only for
 * non-finite points); s_min <= 0 disables the shape test, else s_min <= 1
 * and sigma > 0.  a_t, a_r: curvatures (device float32).  Outputs (device):
 * flags_out[M] uint8; nn_out[M] int32 (-1: none within tau) and d2_out[M]
 * float32 (its key, +inf if none), both nullable.  For the reverse
 * direction (reference parts missing from the template) swap the clouds and
 * pass the inverse pose. */
int sgr_change_detect(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                      const sgr_pose* pose, double tau, double sigma, double s_min, uint8_t* flags_out,
                      int32_t* nn_out, float* d2_out, sgr_stream_t stream);

/* B independent registrations of uneven sizes with shared parameters
 * (tmpls, refs: HOST arrays of B cloud views).  Descriptors of all 2B
 * clouds run in one launch; each iteration is one launch over a work list
 * of (registration, template block, reference chunk) items, one block per
 * item in decreasing cost, plus one update launch, captured in a HIP graph.  poses: device [B] (initial
 * poses in, final out).  energy_out (device [B], nullable): final energy U
 * of each.  stats (device [B][E][32], nullable) as in sgr_register.
 * Synchronises the stream; SGR_ENUMERIC / SGR_EDEGENERATE if any
 * registration failed (the others are still valid). */
int sgr_register_batch(sgr_ctx* ctx, int B, const sgr_cloud* tmpls, const sgr_cloud* refs, const sgr_params* prm,
                       sgr_pose* poses, double* energy_out, double* stats, sgr_stream_t stream);

/* Multi-start registration of one pair: S starts, start s pre-rotates the
 * template about its centroid by R0[s] (device float64 [S][9], row-major);
 * all starts run as one batch sharing the descriptors and the packed
 * reference.  poses (device [S]) receive the final poses, energy_out
 * (device [S], nullable) the final energy U, best_out (device int32 [1],
 * nullable) the start with the lowest energy (ties: lowest index). */
int sgr_multistart(sgr_ctx* ctx, const sgr_cloud* tmpl, const sgr_cloud* ref, const sgr_params* prm, int S,
                   const double* R0, sgr_pose* poses, double* energy_out, int32_t* best_out, sgr_stream_t stream);

/* One iteration (as sgr_step) on a plan: pose_out may alias pose_in. */
int sgr_plan_step(sgr_plan* plan, int t, const sgr_pose* pose_in, sgr_pose* pose_out, double* wrench_out,
                  sgr_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SGREG_H */
