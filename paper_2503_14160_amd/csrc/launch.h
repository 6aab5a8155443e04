// Host-side launchers of the craneplan kernels (internal).
#pragma once

#include "internal.h"

namespace cp {

// evaluation (eval.hip)
int eval_slots(int ns);
size_t eval_partial_count(int B, int ns);
// events recorded on the stream right before and right after the evaluation
// kernel (the grid bound refresh before it and the per-path sums after it
// fall outside)
struct EvalEvents {
    hipEvent_t begin, end;
};
// (cost, min_dist and flags all null: only the tape is written)
hipError_t launch_eval_fwd(const PlanView &P, const float *W, int B, double2 *partial, uint32_t *tape, float *cost,
                           float *min_dist, uint8_t *flags, hipStream_t st, const EvalEvents *ev = nullptr);
// the clearance grid of a plan (P.clr_* set), into out [clr_ny][clr_nx]
hipError_t launch_clearance(const PlanView &P, float *out, hipStream_t st);
// with pol (W set): the polish's step on every path after its gradient
hipError_t launch_eval_bwd(const PlanView &P, const float *W, int B, const uint32_t *tape, const float *grad_cost,
                           float *grad_W, hipStream_t st, const PolishStep *pol = nullptr);
hipError_t launch_debug_fk(const PlanView &P, const float *Q, int N, float *centers, float *frames, hipStream_t st);
hipError_t launch_debug_configs(const PlanView &P, const float *Q, int N, float *dist, uint32_t *arg,
                                hipStream_t st);

// optimizer state on the device (opt.hip)
struct OptView {
    int32_t B, nu, D, n_act, npol;
    int32_t act[CP_MAX_JOINTS];  // sampled joint ids
    double eps;
    uint64_t seed;
    uint32_t problem_id;
    float eta, clip;
    double *mu;        // [D]
    double *C;         // [D][D]
    double *L;         // [D][D] lower Cholesky factor used for sampling
    double *xi;        // [B][D] samples
    float *W;          // [B][K][n] samples as waypoints
    float *cost;       // [B]
    float *min_dist;   // [B]
    int32_t *elite;    // [nu] elite indices in rank order (>= B: polished slot)
    int32_t *elite0;   // [nu] elite indices before polish
    float *Wp;         // [npol][K][n] polished elites
    float *Wp2;        // [npol][K][n] the other buffer of the polish steps (each step reads one, writes the other)
    float *cost_p;     // [npol]
    float *md_p;       // [npol] minimum distances of the polished elites
    float *grad_p;     // [npol][K][n]
    float *ones;       // [npol] 1.0
    double *w;         // [nu] log-rank weights
    int64_t *t;        // iteration counter
    int32_t *status;   // 0 ok, 1 covariance not positive definite
    float *best_cost;  // [1]
    float *best_W;     // [K][n]
};

// one problem of a batch (device array element); elite0 == elite (no polish)
struct BatchProblem {
    PlanView P;
    OptView O;
    int64_t partial_off;  // this problem's per-wave partial sums in the batch's shared buffer
    int32_t slots;
    int32_t pad;
};

// launch shape of the batched evaluation (chosen by the autotuner)
struct BatchTuning {
    int32_t rounds;       // 256-configuration rounds per work item
    int32_t wg_per_cu;    // persistent workgroups per compute unit
};

// persistent evaluation of every problem, then per-problem path sums (cull:
// every problem uses the wave-level culling)
hipError_t launch_batch_eval(const BatchProblem *probs, double2 *partial, int n, int max_B, const int2 *items,
                             int n_items, int rounds, int grid, bool cull, hipStream_t st);
// sampling of every problem (iteration counters unchanged)
hipError_t launch_batch_sample(const BatchProblem *probs, int n, int max_B, hipStream_t st);
// one optimizer iteration of every problem: sampling, evaluation, selection, update, factor
hipError_t launch_batch_iteration(const BatchProblem *probs, double2 *partial, int n, int max_B, const int2 *items,
                                  int n_items, int rounds, int grid, bool cull, hipStream_t st);

hipError_t launch_sample(const PlanView &P, const OptView &O, hipStream_t st);
// the per-path sums of an evaluation (launched without outputs) and the
// selection in one launch, for populations with reduce_select_fits(B)
bool reduce_select_fits(int B);
hipError_t launch_reduce_select(const double2 *partial, int slots, int ns, float margin, const OptView &O,
                                hipStream_t st);
hipError_t launch_select(const OptView &O, hipStream_t st);
// the elites to polish (elite0[0..npol)) copied from the population into dst
hipError_t launch_polish_gather(const PlanView &P, const OptView &O, float *dst, hipStream_t st);
hipError_t launch_rerank(const OptView &O, hipStream_t st);
hipError_t launch_update(const PlanView &P, const OptView &O, hipStream_t st);
hipError_t launch_chol(const OptView &O, hipStream_t st);
hipError_t launch_init_state(const PlanView &P, const OptView &O, float sigma0, hipStream_t st);

// separating-axis narrow phase (sat.hip): the forward pass into partial sums
// (and the tape), and configuration distances
hipError_t launch_eval_fwd_sat(const PlanView &P, const float *W, int B, double2 *partial, uint32_t *tape,
                               hipStream_t st);
hipError_t launch_debug_configs_sat(const PlanView &P, const float *Q, int N, float *dist, uint32_t *arg,
                                    hipStream_t st);

// collision-free inverse kinematics (ik.hip); best needs info
hipError_t launch_ik_solve(const PlanView &P, const cp_ik_params &prm, const float *target, const float *q_init,
                           const float *q_ref, int N, int restarts, float *q_out, float *info, int32_t *status,
                           int32_t *best, hipStream_t st);
hipError_t launch_ik_residual(const PlanView &P, const cp_ik_params &prm, const float *target, const float *q,
                              const float *q_ref, int N, float *r, float *J, hipStream_t st);

// step two: direct collocation (traj.hip); kMB = 16 bounds 2 n + n_act
constexpr int kTrajBlock = 16;
size_t traj_workspace_bytes(int N, int n, int na, int P);
hipError_t launch_traj_refine(const PlanView &P, const cp_traj_params &prm, const int *act, int n_act,
                              const float *q_start, const float *q_goal, const float *q_star, int n_prob, void *work,
                              float *x_out, float *u_out, float *tf_out, float *info_out, hipStream_t st);

// signed-distance grid (sdf.hip)
hipError_t launch_sdf_build(const float *points, int64_t N, const int32_t dims[3], const float origin[3], float voxel,
                            float *sdf, uint8_t *occ, int32_t *edt_occ, int32_t *edt_free, int32_t *work,
                            hipStream_t st);

}  // namespace cp
