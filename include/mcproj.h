/*
 * mcproj — batched projection onto constraint manifolds, collision check and
 * VJP through the projection, for AMD MI355X (gfx950).
 *
 * Method: arXiv 2604.13323 ("Vectorizing Projection in Manifold-Constrained
 * Motion Planning for Real-Time Whole-Body Control"), Alg. 2 ParallelProject
 * and getDescentStep with all constraint rows stacked in one block, followed by
 * the collision check performed after projection (Sec. IV-A). The composite
 * constraint F: R^d -> R^m and its Jacobian J follow Sec. II; a configuration
 * satisfies the constraint when ||F(q)|| < tol.
 *
 * Conventions for every call:
 *   - Return value: mc_status; MC_OK (0) on success. No call throws across the ABI.
 *     Argument errors are reported synchronously, before anything is enqueued;
 *     mc_last_error() then returns a message (thread-local, valid until the next
 *     call on the same thread).
 *   - Configuration arrays are structure-of-arrays: coordinate c of configuration i
 *     lives at q[c * ld + i], with ld >= n. Element type is given by dtype
 *     (MC_F32 = float, MC_F64 = double); resid and min_signed_dist use the same type.
 *   - Every array argument is a caller-owned DEVICE pointer. The library reads and
 *     writes them asynchronously on `stream` (a hipStream_t; 0 = the null stream);
 *     they must stay alive until the stream has passed the call. The library never
 *     keeps them. Input and output arrays must not overlap.
 *   - n == 0 is a no-op returning MC_OK.
 *   - A problem handle may be used by one stream at a time (calls on one problem
 *     share a device work-queue counter).
 *   - Numerical failure of a configuration is a per-configuration status, never a
 *     call error.
 */
#ifndef MCPROJ_H
#define MCPROJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MC_OK = 0,
  MC_ERR_INVALID_ARG = 1, /* null pointer, negative size, ld < n, bad option value */
  MC_ERR_UNSUPPORTED = 2, /* scene family or structure without a compiled kernel */
  MC_ERR_HIP = 3,         /* a HIP runtime call failed (message has the HIP error) */
  MC_ERR_OOM = 4          /* device allocation failed */
} mc_status;

typedef enum { MC_F32 = 0, MC_F64 = 1 } mc_dtype;

/* Per-configuration outcome of the projection (status array values). */
typedef enum {
  MC_CONVERGED = 0, /* ||F(q)|| < tol reached after `iters` steps                         */
  MC_MAX_ITER = 1,  /* max_iter steps taken without convergence                            */
  MC_SINGULAR = 2,  /* J J^T not factorable even in FP64 (rank-deficient Jacobian)         */
  MC_DIVERGED = 3,  /* a step longer than max_step (the paper's MaxDistance exit, Alg. 2)  */
  MC_NONFINITE = 4  /* NaN or Inf in q, F or the step                                      */
} mc_cfg_status;

/* Collision verdict values. */
enum { MC_FREE = 0, MC_COLLIDES = 1, MC_UNCHECKED = 2 };

/* Scene families with compiled kernels (the scene blob's family field). */
enum {
  MC_FAMILY_SPHERE = 0,     /* q in R^3, F = q.q - 1, the configuration is a point robot        */
  MC_FAMILY_LINEAR = 1,     /* F = A q - b, d <= 8, m <= 6, no collision geometry               */
  MC_FAMILY_PLANAR2 = 2,    /* planar 2R arm, tip position (x, y) pose block                    */
  MC_FAMILY_ARM7_AXIS = 3,  /* 7-DoF serial arm, end-effector z parallel to world z (2 rows)    */
  MC_FAMILY_DUAL14_REL = 4, /* two 7-DoF arms, relative end-effector pose of Eq. 2 (6 rows)     */
  MC_FAMILY_HUMANOID36 = 5, /* 36-DoF humanoid tree: feet poses (12), hands relative pose (6),
                               centre-of-mass xy (2)                                           */
  MC_FAMILY_DIGIT36 = 6,    /* the humanoid tree with the Digit constraint set (the paper's
                               Digit constraint figure): feet poses (12), hands relative pose
                               (6), CoM xy minus its nearest point of the support polygon (2,
                               zero inside), closed-linkage rod lengths (2)                    */
  MC_FAMILY_ARM7_TSR = 7    /* 7-DoF serial arm, TSR pose block of Eq. 1 with finite bounds B^w
                               (Sec. III): each component's excess over its interval (6)       */
};

typedef struct mc_problem mc_problem; /* opaque; device-resident scene */

typedef struct {
  mc_dtype dtype;             /* element type of q_in/q_out/resid (and of the arithmetic:
                                 MC_F32 = mixed precision, FP64 residual and iterate with an
                                 FP32 Jacobian/Gram/Cholesky step and FP64 fallback;
                                 MC_F64 = FP64 throughout)                                     */
  double tol;                 /* convergence: ||F|| < tol (2-norm of the stacked rows), > 0      */
  int32_t max_iter;           /* maximum number of Newton steps, 0..127                          */
  double alpha;               /* step scale (Alg. 2 alpha), default 1                           */
  double lambda;              /* damping (Alg. 2 lambda), >= 0, default 0                       */
  double max_step;            /* > 0: DIVERGED when ||alpha * step|| > max_step; <= 0: off       */
  double fp64_cond_threshold; /* FP32 mode: when the FP32 Cholesky of J J^T fails or its
                                 condition estimate (max L_ii / min L_ii)^2 exceeds this (1e6),
                                 the step is redone in FP64 and that configuration takes FP64
                                 steps until it terminates                                     */
  int32_t check_collision;    /* 1: collision-check CONVERGED configurations into `verdict`      */
  int32_t variant;            /* 0 auto: the fused variant, with the launch shape that
                                 mc_autotune_project stored in the problem for this dtype and mode
                                 (where the shape fields below are left at 0), else the library's
                                 default shape; 1 plain (one launch per geodesic);
                                 2 fused (persistent work-queue kernel over the whole batch)     */
  int32_t waves_per_block;    /* fused variant: 1, 2 or 4 wavefronts per workgroup (0 = auto)   */
  int32_t blocks_per_cu;      /* fused variant: resident workgroups per CU for the persistent
                                 grid (0 = auto; with auto, a stacked-mode batch larger than the
                                 lanes of the one-wave-per-SIMD launch of the 36-DoF family runs
                                 in its two-waves-per-SIMD build, same results)                  */
  int32_t mode;               /* 0 stacked: one min-norm step on all constraint rows together;
                                 1 cyclic (Sec. IV-C, Alg. 2 getDescentStep): one min-norm step
                                 per constraint block, in the scene's block order, each from the
                                 configuration the previous one left; an iteration is one cycle
                                 and max_step bounds its total displacement. Fused variant only. */
  int32_t lanes_per_config;   /* lanes that share one configuration in the projection kernels:
                                 0 = auto, 1 = one configuration per lane (the only build of the
                                 projection kernels; the check kernels pick their own lane groups) */
  int32_t step_form;          /* the pseudo-inverse of the descent step (Alg. 2 getDescentStep and
                                 Sec. IV-A, inner and outer forms): 0 inner,
                                 alpha J^T (J J^T + lambda I)^-1 F, an m x m factorisation (default);
                                 1 outer, alpha (J^T J + lambda I)^-1 J^T F, a d x d factorisation
                                 of the dense J; needs lambda > 0 (J^T J has rank <= m < d), the
                                 stacked mode, and a family with d <= 16 (MC_ERR_UNSUPPORTED
                                 otherwise: the 36-DoF factor does not fit a lane's registers).
                                 For lambda > 0 both forms give the same step up to rounding. */
} mc_project_opts;

/* Default options (tol 1e-6, max_iter 50, alpha 1, lambda 0, max_step off, threshold 1e6,
   check on, variant auto, stacked mode, launch shape auto). */
void mc_default_opts(mc_project_opts* opts);

/* Create a problem from a scene blob (magic 'MCCS', version 1 or 2: the little-endian layout
   written by Scene.to_blob in paper_2604_13323_amd/scenes.py, a 16-int header followed by joints,
   links, frames, constraint blocks, robot spheres, obstacles and the optional q_ref, A, b; in
   version 2 every block record is followed by 16 doubles of block data: the bounds lo[6], hi[6] of
   a bounded pose block, the counter-clockwise xy vertices of a support polygon):
   parses and validates the blob on the host, checks that its kinematic structure matches a
   compiled family, derives the constants the kernels need (reference poses and rod lengths of
   blocks flagged ref_from_qref, support-polygon edges and normals, subtree masses, link bounding
   spheres, obstacle clusters) and copies them to the current HIP device. The blob is not retained. *out receives the handle.
   Errors: MC_ERR_INVALID_ARG (null, malformed blob), MC_ERR_UNSUPPORTED (no kernel for this
   structure), MC_ERR_OOM / MC_ERR_HIP. */
mc_status mc_problem_create(const void* scene_blob, size_t nbytes, mc_problem** out);

/* Free the problem's device memory. Null is a no-op. The caller must make sure no enqueued
   call still uses the problem. */
void mc_problem_destroy(mc_problem* p);

int32_t mc_problem_dof(const mc_problem* p);      /* d, or -1 for null */
int32_t mc_problem_rows(const mc_problem* p);     /* m, or -1 for null */
int32_t mc_problem_family(const mc_problem* p);   /* family, or -1 for null */

/* Message of the last error on this thread ("" if none). */
const char* mc_last_error(void);

/* project_batch — Alg. 2 ParallelProject with per-configuration termination.
   For each configuration i < n: q <- q_in[:, i]; repeat { F <- F(q); stop if ||F|| < tol or
   after max_iter steps; dq <- alpha J^T (J J^T + lambda I)^-1 F; DIVERGED if max_step > 0 and
   ||dq|| > max_step; q <- q - dq }, then (check_collision) the robot spheres at the projected
   configuration are tested against the obstacle spheres (strict overlap).
   Outputs (device, caller-owned, length n unless noted):
     q_out [d][ld_out]  projected configuration (the last iterate for non-converged ones)
     status int8       mc_cfg_status
     iters  int8       steps taken
     resid  dtype      ||F|| at the last evaluation
     verdict uint8     nullable; MC_FREE / MC_COLLIDES, MC_UNCHECKED when not CONVERGED or
                       check_collision == 0
   In MC_F32 mode the iterate is held in FP64 on the device: status, iters, resid and verdict
   describe that FP64 iterate, and q_out is its rounding to float (whose residual can exceed tol
   by up to ||J|| ||q|| 2^-24).
   geo_offsets (nullable, int32[n_geo + 1], DEVICE pointer) describes the batch as n_geo geodesics
   (CSR offsets, geo_offsets[0] = 0, geo_offsets[n_geo] = n). geo_offsets_host (nullable, int32
   [n_geo + 1]) is the one HOST pointer of the call, read synchronously before the call returns:
   the plain variant launches one kernel per geodesic and needs every geodesic's bounds on the host
   (it is required there and ignored by the fused variant). geo_ok (nullable, uint8[n_geo], device)
   receives 1 when every configuration of the geodesic converged and is collision-free (the early
   exit of Alg. 2 as a per-geodesic flag).
   Workspace: in MC_F32 mode the fused variant hands configurations that need FP64 steps to a
   second kernel through a queue owned by the problem; a call with a larger n than any before
   grows it (hipFree + hipMalloc, which synchronise the device). Calls on one problem must not
   overlap (one stream at a time).
   Errors: MC_ERR_INVALID_ARG for null required pointers, n < 0, ld < n, tol <= 0,
   max_iter outside 0..127, lambda < 0, alpha <= 0, dtype mismatch, plain variant without
   geo_offsets_host. */
mc_status project_batch(const mc_problem* p, int64_t n,
                        const void* q_in, int64_t ld_in, void* q_out, int64_t ld_out,
                        int8_t* status, int8_t* iters, void* resid, uint8_t* verdict,
                        const int32_t* geo_offsets, const int32_t* geo_offsets_host, int32_t n_geo,
                        uint8_t* geo_ok, const mc_project_opts* opts, void* stream);

/* project_batch_noalloc — project_batch for callers that cannot allocate device memory: code
   under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc. Same arguments,
   kernels and results as project_batch; it calls no hipMalloc, hipFree or allocating library
   routine. Its queue counters and FP64 / exact-check queues live in a 64 MiB array of the library
   (one per device, looked up on the first call on a device with that device current, and held
   until the process ends) instead of the problem's grown buffers: n is limited to
   floor((64 MiB - 1 KiB) / (16 d + 12)) configurations, d the family's compiled dimension (114,126
   for the 36-DoF family; 8 for the linear family), and a larger n fails with MC_ERR_INVALID_ARG
   before anything is enqueued. Every call on one device shares that array and clears its counters
   itself: calls that overlap on one device (concurrent streams, or threads) race and must not be
   issued. mc_queue_counts does not report the counters of this call. */
mc_status project_batch_noalloc(const mc_problem* p, int64_t n,
                                const void* q_in, int64_t ld_in, void* q_out, int64_t ld_out,
                                int8_t* status, int8_t* iters, void* resid, uint8_t* verdict,
                                const int32_t* geo_offsets, const int32_t* geo_offsets_host, int32_t n_geo,
                                uint8_t* geo_ok, const mc_project_opts* opts, void* stream);

/* check_batch — collision check of arbitrary configurations (Sec. IV-A: robot spheres vs obstacle
   spheres, collision when ||c_i - o_j||^2 < (r_i + r_j)^2 for some pair).
   verdict uint8[n]: MC_FREE or MC_COLLIDES. min_signed_dist (nullable, dtype[n]): minimum over
   all pairs of ||c_i - o_j|| - (r_i + r_j) (+inf without geometry); requesting it forces the
   exhaustive pair loop. Without it, the kinematic families run the broad phase of the fused
   projection (link bounds against the box around all obstacles) and the exact pair tests only for
   the configurations it flags, through the problem's check queue: that queue grows to the largest
   batch seen like project_batch's (a growth allocates and synchronises; a call of the same or a
   smaller size allocates nothing), and calls on one handle must not overlap. */
mc_status check_batch(const mc_problem* p, int64_t n, const void* q, int64_t ld, mc_dtype dtype,
                      uint8_t* verdict, void* min_signed_dist, void* stream);

/* project_vjp — vector-Jacobian product through the converged projection (implicit
   differentiation at the converged point): g_in = (I - J^+ J) g_out with J = J(q_proj),
   computed as g_out - J^T (J J^T)^-1 J g_out. Exact for on-manifold inputs. In MC_F32 mode the
   Gram solve runs in FP32; configurations whose FP32 factorisation fails or whose condition
   estimate exceeds opts->fp64_cond_threshold are redone in FP64 by a second kernel (queue
   grown like project_batch's). Configurations whose status is not MC_CONVERGED get
   g_in = 0. Arrays q_proj, g_out, g_in are [d][ld] of opts->dtype. */
mc_status project_vjp(const mc_problem* p, int64_t n, const void* q_proj, int64_t ld,
                      const int8_t* status, const void* g_out, void* g_in,
                      const mc_project_opts* opts, void* stream);

/* project_vjp_exact — the exact vector-Jacobian product of the projection map at the (possibly
   off-manifold) inputs: g_in = (dP/dq_in)^T g_out, where P is the iteration of project_batch (Alg. 2
   ParallelProject, stacked mode) continued to convergence. Reverse mode through the Newton steps the
   forward call took: the output cotangent is projected on the tangent space at the converged point
   (I - J^+ J, what a further step there does), then pulled back step by step through
   q_{k+1} = q_k - alpha J^T (J J^T + lambda I)^-1 F, second derivatives of F included (Hessian-vector
   products by central differences of the analytic gradient, step 1e-5 max(1, |q|_inf)). On the manifold
   it equals project_vjp; off it, project_vjp is its first-order approximation.
   q_in [d][ld] are the inputs of the forward project_batch call, status and iters (int8[n]) its outputs,
   g_out and g_in [d][ld]; element type opts->dtype, with alpha, lambda and dtype as in that call (mode
   must be stacked). The arithmetic is FP64 in both dtypes; the iterates are recomputed from q_in
   (nothing is stored between the calls, O(iters^2) steps per configuration). Configurations whose
   status is not MC_CONVERGED get g_in = 0; where a Gram matrix on the path is not positive definite,
   g_in = NaN. */
mc_status project_vjp_exact(const mc_problem* p, int64_t n, const void* q_in, int64_t ld,
                            const int8_t* status, const int8_t* iters, const void* g_out, void* g_in,
                            const mc_project_opts* opts, void* stream);

/* interpolate_geodesics — the interpolation step of Alg. 2: geodesic g gets
   L_g = geo_offsets[g+1] - geo_offsets[g] interior points q_a + t_k (q_b - q_a),
   t_k = k / (L_g + 1), k = 1..L_g, written to q_out[:, geo_offsets[g] + k - 1].
   endpoints [d][2 * n_geo] (column 2g = q_a, 2g+1 = q_b), ld_e >= 2 n_geo. total is the
   caller's geo_offsets[n_geo] (the number of interior points; the call reads nothing back from the
   device, so it is asynchronous and capturable); points past min(total, geo_offsets[n_geo]) are
   not written. ld_out >= total. */
mc_status interpolate_geodesics(const mc_problem* p, int32_t n_geo, const int32_t* geo_offsets,
                                const void* endpoints, int64_t ld_e, int64_t total, void* q_out,
                                int64_t ld_out, mc_dtype dtype, void* stream);

/* path_length_grad — path-length loss over geodesics and its gradient:
   L = sum_g sum_i ||q_{i+1} - q_i||, g_out[:, i] = u_{i-1} - u_i with u = delta / max(||delta||, 1e-12)
   (u taken as 0 outside the geodesic; geo_offsets non-decreasing, and a configuration before
   geo_offsets[0] or from geo_offsets[n_geo] on gets g_out = 0). loss (nullable, device, one dtype scalar) receives L
   (accumulated atomically; it is zeroed by the call first). */
mc_status path_length_grad(const mc_problem* p, int64_t n, const void* q, int64_t ld,
                           const int32_t* geo_offsets, int32_t n_geo, void* g_out, void* loss,
                           mc_dtype dtype, void* stream);

/* mc_eval_residual_jacobian — diagnostic: the residual F [m][ld] and the Jacobian J [m*d][ld]
   (row r, column c at (r * d + c) * ld + i) of n configurations, both in dtype, as the
   projection kernels compute them (FP64 residual; analytic Jacobian columns in the step
   precision). */
mc_status mc_eval_residual_jacobian(const mc_problem* p, int64_t n, const void* q, int64_t ld,
                                    mc_dtype dtype, void* F, void* J, void* stream);

/* Outcome of one extension (extend_batch `result` values), in the order the steps test them. */
enum {
  MC_EXT_OK = 0,               /* q_out holds q_proj; the validated chain meets the resolution    */
  MC_EXT_ZERO = 1,             /* q_target == q_start: no direction to extend along              */
  MC_EXT_NO_PARTICLE = 2,      /* no particle projection converged                                */
  MC_EXT_COLLISION = 3,        /* the selected particle's projection is in collision              */
  MC_EXT_TOO_FAR = 4,          /* ||q_proj - q_start|| > 2 dist (first early exit)                */
  MC_EXT_INTERP_FAILED = 5,    /* an interpolated or refined point did not converge               */
  MC_EXT_INTERP_COLLISION = 6, /* an interpolated or refined point is in collision                */
  MC_EXT_GAP = 7               /* two adjacent projected points lie farther apart than the level's
                                  bound (second early exit)                                       */
};

typedef struct {
  double r;      /* extension range: q_steer lies min(||q_target - q_start||, r) from q_start, > 0 */
  double delta;  /* motion-validation resolution: refinement stops once every gap of the chain
                    is <= delta, > 0                                                           */
  int32_t n;     /* particles, and interpolated points, per extension: 1..64                      */
} mc_extend_opts;

/* extend_batch — Alg. 2 ConstrainedExtend for E independent extensions (Sec. IV-A: steer,
   particles, two-stage projection, recursive refinement; Sec. IV-B: early exits), each step batched over
   all extensions still alive and run by the projection kernels of project_batch (opts as
   there; check_collision is forced on). For extension e, with s = q_start[:, e],
   t = q_target[:, e], L = ||t - s||:
     dist = min(L, r); v = (t - s) / L; q_steer = s + dist v;
     particles p_i = q_steer + eps[e * n + i] v, i < n (eps: the N(0, sigma^2) draws, supplied
       by the caller), all projected;
     q_proj = the CONVERGED particle with the fewest steps (ties: lowest i), else NO_PARTICLE;
       COLLISION if it collides, TOO_FAR if ||q_proj - s|| > 2 dist;
     level 0: the chain s, c_1..c_n, q_proj with c_k = projection of s + k/(n+1) (q_proj - s);
     level l >= 1 (while some gap of the chain exceeds delta): the projected midpoint of every
       gap is inserted;
     a level fails with INTERP_FAILED (a new point not CONVERGED), else INTERP_COLLISION (a new
       point collides), else GAP (a gap next to a new point longer than r / (n 2^l)).
   The number of levels is at most the smallest l with r / (n 2^l) <= delta, which must be
   <= 12, and (n + 1) 2^l + 1 <= 65536.
   Arrays (device, caller-owned): q_start, q_target [d][ld] and eps [E * n] of opts->dtype;
   q_out [d][ld_out] (q_proj, written where a particle was selected: particle >= 0); result
   int8[E] (MC_EXT_*); particle int32[E] (selected particle index, -1 when none was selected);
   n_points int32[E] (points of the validated chain including both ends for MC_EXT_OK, else 0).
   Workspace: particle, chain and level buffers owned by the problem, grown to the largest call
   (synchronising the device when they grow). The call synchronises `stream` once per level to
   read how many points the level emits (not capturable into a graph).
   Errors: MC_ERR_INVALID_ARG for null required pointers, E < 0, ld < E, ld_out < E, r <= 0,
   delta <= 0, n outside 1..64, too many levels, and every project_batch option error. */
mc_status extend_batch(const mc_problem* p, int64_t E, const void* q_start, const void* q_target,
                       int64_t ld, const void* eps, const mc_extend_opts* xopts,
                       const mc_project_opts* opts, void* q_out, int64_t ld_out, int8_t* result,
                       int32_t* particle, int32_t* n_points, void* stream);

/* mc_eval_condition — diagnostic: the condition estimate that decides the FP32 -> FP64 switch,
   kappa_est = (max L_ii / min L_ii)^2 of the Cholesky factor of J J^T + lambda I, computed as the
   projection kernels compute it (MC_F32: FP32 Jacobian columns, Gram and factorisation; MC_F64:
   FP64), or +inf where the factorisation fails. q [d][ld] and kappa [n] are of dtype. */
mc_status mc_eval_condition(const mc_problem* p, int64_t n, const void* q, int64_t ld, mc_dtype dtype,
                            double lambda, void* kappa, void* stream);

/* mc_queue_counts — diagnostic: the problem's four device queue counters after the last call
   (synchronises the device): [0] work items taken from the persistent kernel's queue beyond the
   static share, [1] projections continued in FP64, [2] VJPs redone in FP64, [3] configurations
   queued for the exact collision check. */
mc_status mc_queue_counts(const mc_problem* p, uint32_t counts[4]);

/* mc_set_check_lanes — lanes per configuration of the exact collision check that project_batch
   (fused variant), extend_batch and check_batch run on the configurations their broad phase flags
   (Sec. IV-B, the collision test of every projected configuration). 0 (the default): by the length of
   the queue, a wave per configuration while it is short (at most 4 per launch workgroup), else groups
   of 4 lanes (or the size mc_autotune_project chose); 1, 2, 4, 8, 16 or 64: that many on every queue. Groups below 4 lanes exist for families
   of at most 16 coordinates and run only where the scene's staged spheres leave LDS room for them
   (else 4). Verdicts do not depend on it. MC_ERR_INVALID_ARG for other values. */
mc_status mc_set_check_lanes(mc_problem* p, int32_t lanes);

/* mc_set_kernel_timing — diagnostic: when on, project_batch brackets its main projection launch
   (the persistent kernel of the fused variant, all per-geodesic launches of the plain one) and
   project_vjp / project_vjp_exact their main VJP launch with HIP events on the call's stream; mc_last_kernel_ms waits for
   the last such call and returns the time between its two events (which = 0: projection, 1: VJP).
   The time excludes the queue reset and the FP64 and exact-check tail launches. Off by default;
   turning it on creates the events (not under stream capture). */
mc_status mc_set_kernel_timing(mc_problem* p, int32_t on);
mc_status mc_last_kernel_ms(const mc_problem* p, int32_t which, float* ms);

/* Launch shape of the fused projection. */
typedef struct {
  int32_t waves_per_block;  /* 1, 2 or 4                                        */
  int32_t blocks_per_cu;    /* 0 = occupancy limit, else 1..64                  */
  int32_t lanes_per_config; /* 1                                                */
  int32_t check_lanes;      /* lanes per configuration of the exact collision check on a long
                               queue: 1, 2, 4, 8 or 16 as mc_autotune_project chose them for
                               this batch (0 in the candidate list, and where the queue was
                               short)                                                           */
} mc_launch_shape;

/* mc_autotune_candidates — number of launch shapes mc_autotune_project tries; shapes (nullable)
   receives them in the order their timings are reported. */
int32_t mc_autotune_candidates(mc_launch_shape* shapes);

/* mc_autotune_project — the library's launch-shape autotuner: runs the fused projection of the
   batch q_in (opts as for project_batch; variant and shape fields are ignored) once per candidate
   shape to warm up and then `reps` times under HIP events on `stream`, checks that every candidate
   gives bit-identical outputs (q_out, status, iters, resid, verdict; else MC_ERR_HIP with a message
   naming the shape), and stores the fastest shape in the problem for opts->dtype and opts->mode.
   best (nullable) receives it, ms (nullable, float[mc_autotune_candidates()]) the mean time per
   call of every candidate. Where check_collision is on and the batch's exact-check queue is long (more
   entries than 16 per CU), a second stage times the check's lane groups of 1, 2 (families of at most
   16 coordinates), 4, 8 and 16 lanes per configuration in the fastest shape, checks the outputs again and keeps the fastest group size in
   the problem for every later call's long queues (best->check_lanes; mc_set_check_lanes overrides it).
   The batch itself is only read. Allocates temporary outputs and synchronises the device (a set-up
   call, not for the hot loop). reps in 1..1000. */
mc_status mc_autotune_project(mc_problem* p, int64_t n, const void* q_in, int64_t ld_in,
                              const mc_project_opts* opts, int32_t reps, void* stream,
                              mc_launch_shape* best, float* ms);

/* mc_tuned_shape — the shape stored by mc_autotune_project for (dtype, mode); MC_ERR_INVALID_ARG
   when none is stored. */
mc_status mc_tuned_shape(const mc_problem* p, mc_dtype dtype, int32_t mode, mc_launch_shape* out);

/* mc_fallback_count — number of configurations moved to FP64 (projections that switched to FP64
   steps, VJPs redone in FP64) by the calls enqueued on this problem since it was created or last
   reset (reset = 1 zeroes it after reading). Synchronises the device. */
mc_status mc_fallback_count(const mc_problem* p, int reset, uint64_t* count);

#ifdef __cplusplus
}
#endif
#endif /* MCPROJ_H */
