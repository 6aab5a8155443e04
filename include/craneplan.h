/*
 * craneplan: MI355X (gfx950) library for the GPU stochastic path optimizer of
 * an underactuated forestry crane (Vu et al., "GPU-Accelerated Motion
 * Planning of an Underactuated Forestry Crane in Cluttered Environments",
 * arXiv 2503.14160), first planning step.
 *
 * The optimizer (Algorithm 1) samples B perturbed sets of free B-spline
 * control points ("waypoints") around a mean, evaluates each path
 *   J = J_p + w_c J_c + w_l J_l                          (Sec. 4.1, path opt.)
 * over n_s checkpoints, keeps the nu cheapest ("elites"), and re-fits the mean
 * and covariance to them with log-rank weights.  Path evaluation runs forward
 * kinematics (Sec. 2) at every checkpoint and takes the signed distance d(q)
 * of the crane to the scene (Sec. 3.1) as the minimum over every
 * (link sphere, obstacle) pair.
 *
 * Conventions for every call:
 *  - Pointers named d_* are device pointers on the plan's device; everything
 *    else is host memory.  Device buffers are caller-allocated, contiguous,
 *    4-byte aligned (8-byte for double), and must not alias each other.
 *  - Floating-point data is IEEE float32 unless the name says double.
 *  - Calls marked SYNC return after the work is done; all others only enqueue
 *    work on `stream` (a hipStream_t; NULL = the default stream) and return.
 *    Device-side failures surface at the caller's next synchronisation.
 *  - Return value: CP_OK (0) or a negative CP_ERR_* code; arguments are
 *    validated on the host before anything is enqueued, and a failed call
 *    enqueues nothing.  cp_last_error() describes the last failure of the
 *    calling thread.  No C++ exception crosses this interface.
 *  - A plan / optimizer / batch must not be used from two threads at once;
 *    distinct objects are independent.  Calls on one object that are enqueued
 *    on different streams must be ordered by the caller.
 *  - Joint vectors have n_joints entries; waypoints are [B][K][n_joints].
 *
 * Layout of a path (Sec. 4.1, B-spline path and initial guess): the control
 * polygon is 4 copies of q_start, the K waypoints, 4 copies of q_goal, on a
 * uniform knot vector; the path runs over its K+3 non-constant spans, M
 * checkpoints per span, s_k = k / n_s, n_s = (K+3) M, k = 1..n_s.  In linear
 * mode the polygon is q_start, the waypoints, q_goal (n_s = (K+1) M).
 */
#ifndef CRANEPLAN_H
#define CRANEPLAN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cp_plan cp_plan;
typedef struct cp_opt cp_opt;
typedef void *cp_stream_t; /* a hipStream_t */

enum {
    CP_OK = 0,
    CP_ERR_INVALID_ARG = -1, /* null pointer, bad enum value, inconsistent description */
    CP_ERR_SIZE = -2,        /* a size outside the limits below or the plan's capacity */
    CP_ERR_HIP = -3,         /* a HIP runtime call failed (message has the HIP error) */
    CP_ERR_NOT_PD = -4,      /* covariance not positive definite after jitter retries */
    CP_ERR_STATE = -5,       /* call not valid in the object's current state */
    CP_ERR_NOMEM = -6        /* device or host allocation failed */
};

/* limits */
#define CP_MAX_JOINTS 8
#define CP_MAX_SPHERES 128
#define CP_MAX_K 64
#define CP_MAX_ELITES 4096
#define CP_MAX_DIM 96 /* K * (number of sampled joints) */
#define CP_MAX_HULLS 16

enum { CP_REVOLUTE = 0, CP_PRISMATIC = 1 };
enum { CP_INTERP_BSPLINE = 0, CP_INTERP_LINEAR = 1 };
enum { CP_JP_SQUARED = 0, CP_JP_L2 = 1 };
enum { CP_HINGE_HARD = 0, CP_HINGE_SMOOTH = 1 };
/* How much of the sphere-obstacle pair work is skipped; every mode returns
 * bitwise the same distances (see cp_cost_params.pair_filter). */
enum { CP_PAIRS_ALL = 0, CP_PAIRS_LANE = 1, CP_PAIRS_WAVE = 2, CP_PAIRS_AUTO = 3 };
/* narrow phase of d(q) (cp_scene_desc.narrow) */
enum { CP_NARROW_SPHERES = 0, CP_NARROW_SAT = 1 };

/* tape entry of a checkpoint: (sphere << 16) | obstacle, where obstacle 0 is
 * the ground, 1..n_cyl the cylinders, n_cyl+1..n_cyl+n_box the boxes, and
 * CP_OBS_SDF the signed-distance grid (scene and sphere table order); a
 * self-collision pair of spheres a < b is recorded as sphere a and obstacle
 * CP_OBS_SELF + b.  On equal distances the lower sphere wins, then its scene
 * obstacles in number order, then its self pairs by the other sphere. */
#define CP_OBS_SDF 0xFFFFu
#define CP_OBS_SELF 0xFF00u

/*
 * Crane: a serial chain (Sec. 2).  Joint j (0-based) moves frame j+1 relative
 * to frame j: a fixed translation origin[j] (in frame j), then a rotation by
 * q_j about the unit axis[j] (revolute) or a translation q_j * axis[j]
 * (prismatic).  Frame 0 is the world.  Sphere s is rigidly attached to frame
 * sphere_frame[s] in 0..n_joints at local centre sphere_center[s].
 * Joints with active[j] = 0 are not sampled; the optimizer holds them at
 * q_hold[j].  All pointers are host pointers, copied at plan creation.
 */
typedef struct {
    int32_t n_joints;            /* 1..CP_MAX_JOINTS */
    const int32_t *type;         /* [n] CP_REVOLUTE / CP_PRISMATIC */
    const float *axis;           /* [n][3] unit vectors */
    const float *origin;         /* [n][3] */
    const float *q_min, *q_max;  /* [n] joint limits (feasibility cost) */
    const float *q_hold;         /* [n] */
    const uint8_t *active;       /* [n] 1 = sampled */
    int32_t n_spheres;           /* 1..CP_MAX_SPHERES */
    const int32_t *sphere_frame; /* [S] */
    const float *sphere_center;  /* [S][3] */
    const float *sphere_radius;  /* [S] > 0 */
    /* Self-collision (Sec. 3.2 counts it with collision against the scene):
     * frame pairs (in 0..n_joints, distinct) whose spheres are checked
     * against each other; d(q) then also takes the minimum over every such
     * sphere pair of |c_a - c_b| - r_a - r_b.  0 / NULL: the scene only.
     * Repeated pairs and pairs with a frame that carries no sphere are
     * ignored. */
    int32_t n_self_pairs;        /* 0..64 */
    const int32_t *self_pairs;   /* [n_self_pairs][2] */
    /* Tip (grapple centre point) in the last frame: the end-effector point
     * of the inverse kinematics, H_g = (R of frame n, R tip + p of frame n). */
    float tip[3];
    /* Convex hulls of the links for the separating-axis narrow phase
     * (scene.narrow = CP_NARROW_SAT): oriented boxes, row = centre (3),
     * rotation (9, row-major, the box axes as its columns, orthonormal),
     * half extents (3, > 0), in the coordinates of frame hull_frame[k]
     * (0..n_joints).  0 / NULL without that narrow phase. */
    int32_t n_hulls;             /* 0..CP_MAX_HULLS */
    const int32_t *hull_frame;   /* [n_hulls] */
    const float *hull_box;       /* [n_hulls][15] */
} cp_robot_desc;

/*
 * Scene (Sec. 3.1; the paper's meshes are replaced by primitives with exact
 * signed distances): vertical solid cylinders (x, y, R, z0, z1), axis-aligned
 * solid boxes (cx, cy, cz, hx, hy, hz), the half-space z <= ground_z, and/or a
 * signed-distance grid sampled at voxel centres, queried by trilinear
 * interpolation.  cyl/box are host pointers copied at creation; d_sdf is a
 * device pointer that the plan borrows: it must stay alive and unchanged
 * while the plan is used.
 */
typedef struct {
    int32_t has_ground;
    float ground_z;
    int32_t n_cyl;               /* 0..65279 together with n_box */
    const float *cyl;            /* [n_cyl][5] */
    int32_t n_box;
    const float *box;            /* [n_box][6] */
    const float *d_sdf;          /* [nz][ny][nx] or NULL */
    int32_t sdf_dims[3];         /* nx, ny, nz (each >= 2) */
    float sdf_origin[3];         /* lower corner of voxel (0,0,0), metres */
    float voxel;                 /* voxel edge, metres */
    /* Narrow phase.  CP_NARROW_SPHERES: the robot's spheres against the
     * primitives and grid above.  CP_NARROW_SAT (the separating axis test
     * of Sec. 3.1 on convex hulls): d(q) is the minimum over every pair of a
     * robot hull and an obstacle (the ground, then the oriented boxes obb in
     * number order) of their SAT signed distance, and over the hull pairs of
     * the listed self-collision frame pairs; cyl, box and d_sdf are then not
     * used.  The SAT distance of two boxes is the largest projection gap
     * over the fifteen candidate axes (each box's three face normals and the
     * cross products of their edge directions, an edge pair within about
     * 5.7 degrees of parallel, |a x b|^2 <= 0.01, giving none): positive, a
     * lower bound of their
     * Euclidean distance (exact when the nearest features are a face and
     * anything, or two edges); otherwise minus the penetration depth.  A
     * hull against the ground: its lowest corner's height above ground_z.
     * The tape records (hull << 16) | obstacle, obstacle 0 the ground,
     * 1..n_obb the boxes, CP_OBS_SELF + m a self pair of hulls k < m; equal
     * distances keep the lowest hull, then obstacle.  This narrow phase
     * has no adjoint (cp_eval_paths_backward, the polish, the population
     * gradient and the IK refuse it) and does not run in batches.  Unless
     * cost.pair_filter is CP_PAIRS_ALL, a pair stops after the scene box's
     * three face axes when their largest gap is above the configuration's
     * running minimum (bitwise the same results). */
    int32_t narrow;              /* CP_NARROW_* */
    int32_t n_obb;               /* 0..65279 */
    const float *obb;            /* [n_obb][15], the layout of hull_box, world coordinates */
} cp_scene_desc;

/* Cost of a path (Sec. 4.1, eqs. for J_p, J_c, J_l).  The collision term is
 * phi(d) = lambda_c max(0, margin - d) (hard hinge; margin 0 is the paper's
 * ReLU(-d)), or the C1 smooth hinge lambda_c (margin/2 - d) for d < 0,
 * lambda_c (margin - d)^2 / (2 margin) for 0 <= d < margin, 0 beyond.
 * J_p sums |q_k - q_{k-1}|^2 (squared, the paper's) or |q_k - q_{k-1}| (L2). */
typedef struct {
    int32_t K;        /* free waypoints, 1..CP_MAX_K */
    int32_t M;        /* checkpoints per span, >= 1 */
    int32_t interp;   /* CP_INTERP_* */
    int32_t jp_mode;  /* CP_JP_* */
    int32_t hinge;    /* CP_HINGE_* (smooth needs margin > 0) */
    float margin;     /* metres */
    float lambda_c;
    float w_c, w_l;
    int32_t max_B;    /* largest batch any call on this plan will pass */
    /* CP_PAIRS_ALL: every sphere-obstacle pair and every grid lookup is
     * evaluated in full.  In the other modes a sphere's grid lookup is
     * skipped where a lower bound of the grid over its 2 x 2 x 2 block of
     * cells (refreshed from the grid by each evaluation call, so the borrowed
     * grid may change between calls) shows that it cannot bring the sphere
     * below the configuration's running minimum.
     * CP_PAIRS_LANE: a sphere-cylinder pair whose squared axis distance shows
     * that it cannot lower the running minimum skips its square root.
     * CP_PAIRS_WAVE: the configurations of one hardware wave that belong to
     * one path are bounded by a box per group of up to four spheres;
     * cylinders and boxes that no configuration in the box can come closer to
     * than an upper bound of its minimum are skipped for the whole wave
     * (waves that hold more than two paths are bounded as one box), and a
     * whole group of spheres is skipped when a lower bound of its distances
     * (a clearance grid built at plan creation, and the ground) is above
     * every configuration's running minimum.  CP_PAIRS_AUTO: CP_PAIRS_WAVE for
     * scenes of at least 48 cylinders and boxes, else CP_PAIRS_LANE (the
     * culling's fixed cost per wave outweighs its savings on small scenes;
     * in a batch, CP_PAIRS_WAVE if any problem qualifies; batched launches
     * do not skip grid lookups).  Skipped pairs and lookups cannot lower any
     * minimum, so distances, costs and argmin records are bitwise those of
     * CP_PAIRS_ALL in every mode. */
    int32_t pair_filter;
} cp_cost_params;

/* Algorithm 1 settings.  C_0 = sigma0^2 I; samples are xi ~ N(mu, C).  The
 * normal variates of element e of path b in iteration t come from
 * Philox4x32-10 with key (seed low word, seed high word) and counter
 * (e / 4, b, t, problem_id), four words -> two Box-Muller pairs. */
typedef struct {
    int32_t B;              /* population (lambda), 1..max_B */
    int32_t nu;             /* elites, 1..min(B, CP_MAX_ELITES) */
    float sigma0;
    double eps;             /* covariance regulariser (eps I) */
    uint64_t seed;
    uint32_t problem_id;
    int32_t polish_elites;  /* elites that take gradient steps each iteration (0 = off) */
    int32_t polish_steps;
    float polish_eta;       /* step length */
    float polish_clip;      /* gradient norm clip g_max */
} cp_opt_params;

/* Description of the last failure on the calling thread ("" if none). */
const char *cp_last_error(void);

/* Create a plan on HIP device `device` (SYNC).  Copies the robot, the
 * primitive tables and the cost parameters to the device and allocates the
 * evaluation workspace for up to cost->max_B paths.  Endpoints start at the
 * hold configuration. */
int cp_plan_create(const cp_robot_desc *robot, const cp_scene_desc *scene, const cp_cost_params *cost,
                   int device, cp_plan **out);
/* Release the caller's handle (SYNC; NULL is a no-op).  The plan's memory is
 * freed now, or, if optimizers created on it are still alive, when the last
 * of them is destroyed; the handle must not be used again either way. */
int cp_plan_destroy(cp_plan *plan);

/* Start and goal configurations q_0 and q_d (host [n_joints]) (SYNC). */
int cp_plan_set_endpoints(cp_plan *plan, const float *q_start, const float *q_goal);

/* n_s, the checkpoints per path (k = 1..n_s; the start point is not checked). */
int cp_plan_n_checkpoints(const cp_plan *plan, int32_t *n_s);

/*
 * Algorithm 1 step (2): evaluate B paths.
 *  d_waypoints [B][K][n] -> d_cost [B] (J), d_min_dist [B] (min_k d(q_k)),
 *  d_flags [B] (1 if min_dist < margin; may be NULL),
 *  d_tape [B][n_s] (argmin pair of every checkpoint; may be NULL).
 * Non-finite waypoints give a NaN cost.  B must be in 1..max_B.
 */
int cp_eval_paths(cp_plan *plan, const float *d_waypoints, int32_t B, float *d_cost, float *d_min_dist,
                  uint8_t *d_flags, uint32_t *d_tape, cp_stream_t stream);

/*
 * cp_eval_paths for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same evaluation, bitwise the same outputs, with the per-wave partial
 * sums in a static 24 MiB device array instead of the plan's workspace.  The
 * call allocates nothing.  The array is one per GPU, shared by every plan on
 * it and holding the last call's contents: calls that overlap on one GPU
 * (several streams or threads) race and must be ordered by the caller.
 * Limit: ceil(B n_s / 64) (64 / n_s + 2) * 16 bytes <= 24 MiB (for n_s >= 64
 * about B n_s <= 25 M configurations; the 65536 x 608 population fits);
 * beyond it CP_ERR_SIZE, with nothing enqueued.
 */
int cp_eval_paths_noalloc(cp_plan *plan, const float *d_waypoints, int32_t B, float *d_cost, float *d_min_dist,
                          uint8_t *d_flags, uint32_t *d_tape, cp_stream_t stream);

/*
 * Adjoint of cp_eval_paths: d_grad_waypoints[b] = d_grad_cost[b] * dJ_b/dW_b
 * [B][K][n] (every joint, sampled or not).  d_tape is the tape written by
 * cp_eval_paths for the same waypoints, or NULL to recompute the argmin
 * pairs.  Forward kinematics is recomputed, never stored.  Where the
 * minimising pair is tied the lowest (sphere, obstacle) is differentiated.
 */
int cp_eval_paths_backward(cp_plan *plan, const float *d_waypoints, int32_t B, const uint32_t *d_tape,
                           const float *d_grad_cost, float *d_grad_waypoints, cp_stream_t stream);

/* Optimizer on a plan (SYNC).  mu_0 = evenly spaced waypoints on the segment
 * from q_start to q_goal (sampled joints only), C_0 = sigma0^2 I, t = 0.  The
 * optimizer keeps the plan alive (cp_plan_destroy and cp_optimizer_destroy
 * may come in either order); the plan's endpoints are read at every step. */
int cp_optimizer_create(cp_plan *plan, const cp_opt_params *params, cp_opt **out);
int cp_optimizer_destroy(cp_opt *opt); /* SYNC; NULL is a no-op */

/* Run n_iters iterations of Algorithm 1 (Cholesky factor, sampling,
 * evaluation, selection, optional polish, log-rank weights, mean and
 * covariance update) without host synchronisation. */
int cp_optimizer_step(cp_opt *opt, int32_t n_iters, cp_stream_t stream);

/* Record the argmin tape of every population evaluation of the following
 * steps (SYNC; enable != 0 allocates B n_s 4-byte entries, 0 frees them), so
 * that the population's gradient can follow each step cheaply. */
int cp_optimizer_record_tape(cp_opt *opt, int32_t enable);
/* Gradient of the last population's summed cost, d(sum_b J_b)/dW_b, into
 * d_grad_waypoints [B][K][n] (the adjoint of the last evaluation through its
 * tape; the samples after the step are unchanged, so this is the gradient at
 * the evaluated waypoints).  Enqueued on stream; CP_ERR_STATE without a
 * recorded tape.  (The paper's Algorithm 1 is derivative free; this serves
 * gradient-based refinement of the population.) */
int cp_optimizer_population_grad(cp_opt *opt, float *d_grad_waypoints, cp_stream_t stream);

/* Timing of the evaluation launches inside cp_optimizer_step (SYNC): with
 * max_launches > 0, each of the next max_launches evaluations (Algorithm 1
 * step 2, the population's evaluation kernel alone: not the grid's bound
 * refresh before it nor the per-path sums after it) is bracketed by a pair of
 * HIP events on the step's stream; 0 switches timing off.  The call creates
 * the events (and destroys earlier ones). */
int cp_optimizer_time_eval(cp_opt *opt, int32_t max_launches);
/* Sum of the timed evaluations' durations in milliseconds and their number
 * since the last call (SYNC: waits for the last timed launch); the event
 * pairs are then reused. */
int cp_optimizer_eval_time(cp_opt *opt, double *total_ms, int32_t *launches);

/* State (SYNC): mu [D] and C [D][D] (double, D = K * sampled joints), the
 * iteration counter, the best cost seen and its waypoints [K][n].  Any
 * pointer may be NULL.  Returns CP_ERR_NOT_PD if a covariance could not be
 * factorised since the last call. */
int cp_optimizer_get_state(cp_opt *opt, double *mu, double *C, int64_t *iter, float *best_cost,
                           float *best_waypoints);
/* Replace mu, C and the iteration counter (SYNC); resets best-so-far. */
int cp_optimizer_set_state(cp_opt *opt, const double *mu, const double *C, int64_t iter);

/* Copies of the last iteration's population (enqueued on stream): the
 * waypoints [B][K][n], costs [B] and elite indices [nu] in rank order (after
 * polish: indices >= B denote polished elite slots).  Any may be NULL. */
int cp_optimizer_last(cp_opt *opt, float *d_waypoints, float *d_cost, int32_t *d_elite, cp_stream_t stream);
/* The selection of the last iteration (Algorithm 1, step 3): elite indices
 * d_idx [nu] in rank order and costs d_cost [B], enqueued on stream; the same
 * as cp_optimizer_last without the waypoints.  Either may be NULL. */
int cp_optimizer_last_elites(cp_opt *opt, int32_t *d_idx, float *d_cost, cp_stream_t stream);
/* The gradient polish of the last iteration (a setting of the differentiable
 * workload; the paper's Algorithm 1 has no such step): the polished elites'
 * waypoints d_waypoints [polish_elites][K][n] in the order of the selection
 * before polish, and their costs d_cost [polish_elites] (enqueued on stream;
 * either may be NULL).  The elite index polish_slot + B of
 * cp_optimizer_last names row polish_slot here.  CP_ERR_STATE for an
 * optimizer without polish. */
int cp_optimizer_last_polished(cp_opt *opt, float *d_waypoints, float *d_cost, cp_stream_t stream);

/*
 * Batches of independent planning problems (the paper's batch generation of
 * trajectories, Sec. 1).  Every problem has its own crane, scene, cost and
 * optimizer settings and sizes; an iteration of all of them is one sampling
 * launch, ONE persistent evaluation launch (workgroups pull work items of
 * consecutive configurations from a device queue ordered costliest problem
 * first), and one selection / update / factor launch each, with a workgroup
 * per problem.  Results are bitwise those of running each problem alone
 * through cp_optimizer_step.
 */
typedef struct cp_batch cp_batch;

/* Launch shape of the batched evaluation: configurations per work item
 * (rounds x 256) and persistent workgroups per compute unit, or 0 for one
 * workgroup per work item (the hardware dispatcher then balances the load). */
typedef struct {
    int32_t rounds;     /* 1..64 */
    int32_t wg_per_cu;  /* 0..16 */
} cp_batch_tuning;

/* Create n problems on `device` (SYNC).  robots, scenes, costs, opts are
 * arrays of n descriptors (as for cp_plan_create / cp_optimizer_create; the
 * cost's max_B must be >= the opt's B; polish is not supported in a batch);
 * q_start and q_goal hold the n endpoint vectors back to back (host). */
int cp_batch_create(int32_t n, const cp_robot_desc *robots, const cp_scene_desc *scenes, const cp_cost_params *costs,
                    const cp_opt_params *opts, const float *q_start, const float *q_goal, int device,
                    cp_batch **out);
int cp_batch_destroy(cp_batch *batch); /* SYNC; NULL is a no-op */

/* Run n_iters iterations of every problem.  The first call for a given
 * n_iters (and tuning) captures the sequence into a HIP graph on an internal
 * stream; every call replays the graph on `stream`. */
int cp_batch_run(cp_batch *batch, int32_t n_iters, cp_stream_t stream);

/* The persistent evaluation launch alone on the current populations
 * (enqueued on stream; used for tuning and timing). */
int cp_batch_eval(cp_batch *batch, cp_stream_t stream);

/* State of problem p, as cp_optimizer_get_state (SYNC). */
int cp_batch_get_state(cp_batch *batch, int32_t p, double *mu, double *C, int64_t *iter, float *best_cost,
                       float *best_waypoints);

/* The last iteration's population of problem p, as cp_optimizer_last:
 * waypoints [B_p][K_p][n_p], costs [B_p], elite indices [nu_p] in rank
 * order (enqueued on stream; any may be NULL). */
int cp_batch_last(cp_batch *batch, int32_t p, float *d_waypoints, float *d_cost, int32_t *d_elite,
                  cp_stream_t stream);

/* Set / read the launch shape (setting drops captured graphs). */
int cp_batch_set_tuning(cp_batch *batch, const cp_batch_tuning *tuning);
int cp_batch_get_tuning(const cp_batch *batch, cp_batch_tuning *tuning);

/* Autotune the launch shape (SYNC): reuse the entry for this batch's shape
 * and device from the text cache at cache_path if there is one, else time
 * every candidate shape on this batch (rounds 1, 2, 4, 8, 16, 32 times
 * workgroups per compute unit 0, 1, 2, 4, 8; each the median of three
 * evaluation launches after a warm-up), keep the fastest and append it to
 * the cache (cache_path may be NULL: no cache).  The chosen shape is applied
 * and returned in *chosen (may be NULL). */
int cp_batch_tune(cp_batch *batch, const char *cache_path, cp_batch_tuning *chosen);
/* Autotune (SYNC) whatever of plan and batch is given (either may be NULL,
 * not both).  A batch is tuned as by cp_batch_tune.  A plan has nothing to
 * time: its evaluation's launch shape follows at every call from the number
 * of paths (how many waves share a configuration's sphere groups) and its
 * pair filter from the scene, so a plan alone returns CP_OK. */
int cp_tune(cp_plan *plan, cp_batch *batch, const char *cache_path);

/* Signed-distance grid from a point cloud (for scenes given as lidar):
 * voxels holding at least one point are occupied (index floor((p - o) / h) in
 * double precision; points outside the grid are dropped); exact squared
 * distances (voxel units) to the nearest occupied / free voxel; field
 * h (sqrt(EDT_occ) - 1/2) on free voxels, -h (sqrt(EDT_free) - 1/2) on
 * occupied ones.  With no occupied (free) voxel the squared distance is
 * nx^2 + ny^2 + nz^2.  d_points [N][3]; outputs [nz][ny][nx]; d_sdf also
 * serves as scratch until the last pass writes it.  The three optional
 * outputs may be NULL: the call then allocates them (1, 4 and 4 bytes per
 * voxel), frees them and synchronises the stream; with all three given it
 * allocates nothing and returns without waiting. */
int cp_sdf_build(const float *d_points, int64_t N, const int32_t dims[3], const float origin[3], float voxel,
                 float *d_sdf, uint8_t *d_occ, int32_t *d_edt_occ, int32_t *d_edt_free, cp_stream_t stream);

/*
 * Collision-free inverse kinematics (Sec. 3.2, eq. IK opt): for each row i,
 *   q_i = argmin_q |r(q)|^2,  r = [ p_g - p_d,                  (3)
 *                                   lambda_q Log(R_d^T R_g),    (3, SO(3) log)
 *                                   lambda_c ReLU(-d(q)),       (1, scene and self)
 *                                   lambda_e |g_p|^2,           (1)
 *                                   lambda_r (q - q_ref) ]      (n_joints)
 * where (R_g, p_g) is the pose of the last frame with p_g its tip point,
 * d(q) the signed distance of the evaluation, and g_p the gravitational
 * generalised force that a unit weight at the tip exerts on the joints that
 * are not actuated (active[j] = 0): g_p,j = d z_tip / d q_j, zero when the
 * load hangs at rest.  Solved by Levenberg-Marquardt with the gain-ratio
 * damping update (Madsen, Nielsen, Tingleff 2004): mu_0 = tau max diag(J^T J);
 * per iteration (J^T J + mu I) h = -J^T r, q' = q + h (clamped to
 * [q_min, q_max] with clamp != 0), accepted when the cost decrease over the
 * decrease the linear model predicts is positive (then
 * mu *= max(1/3, 1 - (2 rho - 1)^3), else mu *= nu, nu *= 2).  A row stops
 * when max |J^T r| <= eps_grad, when |h| <= eps_step (|q| + eps_step), or
 * after max_iters trial steps.
 */
typedef struct {
    float lambda_q, lambda_c, lambda_e, lambda_r;  /* residual weights, >= 0 */
    int32_t max_iters;                             /* 0..1000 trial steps */
    float tau;                                     /* > 0 */
    float eps_grad, eps_step;                      /* >= 0 */
    int32_t clamp;                                 /* 1: keep q within the limits */
} cp_ik_params;

/*
 * Solve N independent IK rows (enqueued on stream; one hardware wave per row,
 * the wave's lanes sharing out the sphere-obstacle pairs of d(q)).
 *  d_target [N][12]: R_d row-major then p_d (metres);
 *  d_q_init [N][n]: starting configurations; d_q_ref [N][n] (NULL: q_init);
 *  d_q [N][n] out: solutions; d_info [N][6] out (may be NULL): cost
 *  F = |r|^2 / 2, |p_g - p_d|, |Log(R_d^T R_g)|, d(q), |g_p|, trial steps
 *  taken; d_status [N] out (may be NULL): 1 gradient test met, 2 step test
 *  met, 0 iteration limit.
 * With restarts > 1, rows come in groups of `restarts` (rows i*restarts ..
 * i*restarts + restarts - 1 solve target i from different starting points;
 * N must be a multiple of restarts) and d_best [N / restarts] (may be NULL)
 * receives, per group, the row with the lowest F (NaN as +inf; ties: the
 * lowest row); d_best requires d_info.  1 <= N <= 1048576.  The plan's scene
 * and robot (spheres, self pairs, tip) are used; its cost parameters are not.
 * Device buffers are the caller's, contiguous, on the plan's device.
 * Errors: CP_ERR_INVALID_ARG (null pointers, weights negative or not finite,
 * max_iters outside 0..1000, tau <= 0, d_best without d_info), CP_ERR_SIZE
 * (N out of range or not a multiple of restarts), CP_ERR_HIP (launch).
 */
int cp_ik_solve(cp_plan *plan, const cp_ik_params *params, const float *d_target, const float *d_q_init,
                const float *d_q_ref, int32_t N, int32_t restarts, float *d_q, float *d_info, int32_t *d_status,
                int32_t *d_best, cp_stream_t stream);

/* Test export: the IK residual r [N][8+n] and its Jacobian [N][8+n][n]
 * (either may be NULL) at configurations d_q [N][n] for targets d_target
 * [N][12] and references d_q_ref [N][n] (NULL: d_q), with the weights of
 * params (the solver settings are ignored). */
int cp_debug_ik_residual(cp_plan *plan, const cp_ik_params *params, const float *d_target, const float *d_q,
                         const float *d_q_ref, int32_t N, float *d_r, float *d_J, cp_stream_t stream);

/*
 * Step two of the planner (Sec. 4.2, eq. discrete): direct collocation with
 * trapezoidal defects of the reduced dynamics (Sec. 2.1).  State x = (q, qd),
 * inputs u = the accelerations of the actuated joints (active[j] = 1, in
 * joint order); the passive joints follow their rows of M qdd + b = tau with
 * no torque, M and b of a unit load at the tip on massless links (the
 * crane's mass model is not given):
 *   qdd_p = -(J_p^T J_p)^-1 J_p^T (J_a u + c + grav e_z) - damping qd_p,
 * J = d tip / dq, c = sum_ij (d^2 tip / dq_i dq_j) qd_i qd_j.  Over N
 * intervals of h = t_F / N it minimises
 *   t_F + omega_s sum_{k=1..N} |u_k|^2 + omega_t sum_{k=1..N} |q_a,k - q*_a,k|^2
 * subject to x_{k+1} - x_k = h/2 (f(x_k, u_k) + f(x_{k+1}, u_{k+1})),
 * x_0 = (q_start, 0), x_N = (q_goal, 0), the joint limits and |qd_j| <=
 * v_max[j] (q* is the path of step one at s = k / N).  Solver (IPOPT and
 * automatic differentiation are not available here): an augmented
 * Lagrangian on the defects (multipliers from 0, penalty mu0, times
 * mu_factor after each of `outer` rounds; the state bounds as quadratic
 * penalties of the same weight) around Levenberg-Marquardt on the squared
 * residual (the IK's damping schedule: mu_LM,0 = tau max diag(J^T J); at
 * most max_iters trial steps per round; stops on max |J^T r| <= eps_grad
 * or |h| <= eps_step (|z| + eps_step)), t_F = s^2 with s unknown, started
 * from the path at times k t_0 / N, t_0 = max(t_f0, t_min), with
 * velocities and inputs from its differences.  t_F >= t_min = max_j
 * |q_goal,j - q_start,j| / v_max[j], which the velocity limits imply, is
 * kept as one more penalty of weight mu (it keeps the solver off s = 0,
 * where every residual is stationary in s).  Dynamics Jacobians by central differences (step fd_q on
 * positions, 1 on velocities and inputs, where the accelerations are
 * quadratic and linear).  Everything in double precision, one workgroup
 * per problem.
 */
typedef struct {
    int32_t N;                    /* intervals, 2..400 */
    double omega_s, omega_t;      /* >= 0 */
    double grav;                  /* m/s^2 along -z */
    double damping;               /* >= 0, on the passive joints (1/s) */
    double v_max[CP_MAX_JOINTS];  /* > 0 per joint */
    double mu0, mu_factor;        /* > 0, >= 1 */
    int32_t outer, max_iters;     /* 1..20, 0..500 */
    double tau, eps_grad, eps_step, fd_q, t_f0; /* > 0, >= 0, >= 0, > 0, > 0 */
} cp_traj_params;

/* Bytes of device workspace cp_traj_refine needs for P problems (SYNC, no
 * device work).  Errors: CP_ERR_SIZE when 2 n + (actuated joints) > 16. */
int cp_traj_workspace_size(const cp_plan *plan, const cp_traj_params *params, int32_t P, size_t *bytes);

/* Refine P independent trajectories (enqueued on stream; allocates nothing):
 * d_q_start, d_q_goal [P][n]; d_q_star [P][N+1][n] the step-one paths at
 * s = k / N (row 0 and N are ignored: the endpoints are q_start, q_goal);
 * d_work: caller's device workspace of at least cp_traj_workspace_size bytes
 * (8-byte aligned; its contents on return are scratch); outputs d_x
 * [P][N+1][2n] states, d_u [P][N+1][n_act] inputs, d_t_f [P] final times,
 * d_info [P][4] (may be NULL): max |defect| without multipliers, the last
 * augmented objective |r|^2 / 2, trial steps, accepted steps.  Uses the plan's
 * robot (joints, tip, actuated set); its scene and costs are not used.
 * Errors: CP_ERR_INVALID_ARG (null pointers, parameters out of range),
 * CP_ERR_SIZE (P < 1, N out of range, workspace too small, 2 n + n_act >
 * 16), CP_ERR_HIP. */
int cp_traj_refine(cp_plan *plan, const cp_traj_params *params, const float *d_q_start, const float *d_q_goal,
                   const float *d_q_star, int32_t P, void *d_work, size_t work_bytes, float *d_x, float *d_u,
                   float *d_t_f, float *d_info, cp_stream_t stream);

/* Test exports.  Forward kinematics of N joint vectors d_q [N][n]:
 * sphere centres [N][S][3] (sphere table order) and frames [N][n+1][12]
 * (row-major rotation then position); either output may be NULL. */
int cp_debug_fk(cp_plan *plan, const float *d_q, int32_t N, float *d_centers, float *d_frames, cp_stream_t stream);
/* d(q) and the argmin pair (tape encoding) of N joint vectors. */
int cp_debug_eval_configs(cp_plan *plan, const float *d_q, int32_t N, float *d_dist, uint32_t *d_argmin,
                          cp_stream_t stream);
/* Selection step of Algorithm 1 (step 3) alone: indices of the nu smallest
 * (cost, index) pairs of d_cost [B] in rank order, NaN ranked as +inf,
 * written to d_elite [nu]; 1 <= nu <= min(B, CP_MAX_ELITES).  Runs on the
 * current device. */
int cp_debug_select(const float *d_cost, int32_t B, int32_t nu, int32_t *d_elite, cp_stream_t stream);
/* Steps (4)-(6) of Algorithm 1 alone, for tests: the log-rank weighted mean
 * and the covariance about it, from the last iteration's samples with the
 * caller's elite indices d_elite [nu] (rank order, each in 0..B-1; device
 * memory, read back and range-checked first, so the call synchronises) in
 * place of the selection.  With polish settings, the first polish_elites of
 * them are polished, re-evaluated and re-ranked first, as in a step.
 * Replaces mu and C (the factor is not refreshed) and advances the iteration
 * counter and best-so-far as a step would (the caller's first elite standing
 * for the iteration's best sample).  CP_ERR_INVALID_ARG for an index out of
 * range. */
int cp_debug_update(cp_opt *opt, const int32_t *d_elite, cp_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* CRANEPLAN_H */
