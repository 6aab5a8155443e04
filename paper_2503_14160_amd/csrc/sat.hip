// Separating-axis narrow phase on oriented boxes (Sec. 3.1): the crane's link
// hulls against the scene's boxes and the ground, for the path evaluation
// (Algorithm 1, step 2) and configuration distances.
//
// One lane per checkpoint configuration, as in the sphere evaluation: the
// lane interpolates its configuration, then for each hull runs the chain
// from the base to the hull's frame, places the box, and takes the SAT
// distance against every scene box (wave-uniform records, scalar loads) and
// the ground; then the hull pairs of the listed self-collision frame pairs.
// A pair whose gaps along the scene box's three face axes already exceed the
// lane's running minimum stops there (about a third of the arithmetic): it
// cannot lower or tie the minimum, so results are those of every axis.
// The fifteen axes follow the separating axis test for oriented boxes of
// Gottschalk, Lin and Manocha ("OBBTree", 1996): with C = A^T B (the cosines
// between the boxes' axes) and T the centre offset in A's axes, a face axis
// gap is a difference of absolute sums, and the cross axis a_i x b_j, of
// length sqrt(1 - C_ij^2), has projection radii and centre term read off C
// and T; here each gap is divided by the axis length to give a distance.
#include "launch.h"

namespace cp {
namespace {

// edge pairs whose cross product is shorter than this (squared), about 5.7
// degrees from parallel, give no axis: the direction of a_i x b_j turns by
// about e / |a_i x b_j| for a rotation error e, so nearer to parallel the
// single-precision gap along it would be noise
constexpr float kParallel = 1e-2f;

struct Box {
    float c[3], a[3][3], h[3];  // centre, axes (a[i] = i-th axis), half extents
};

__device__ __forceinline__ Box load_box(const float4 *t, int k) {
    const float4 q0 = ldg(t, 4 * k), q1 = ldg(t, 4 * k + 1), q2 = ldg(t, 4 * k + 2), q3 = ldg(t, 4 * k + 3);
    Box b;
    b.c[0] = q0.x; b.c[1] = q0.y; b.c[2] = q0.z;
    b.h[0] = q0.w; b.h[1] = q1.w; b.h[2] = q2.w;
    // row-major rotation R: axis i is column i
    const float R[9] = {q1.x, q1.y, q1.z, q2.x, q2.y, q2.z, q3.x, q3.y, q3.z};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        b.a[i][0] = R[i]; b.a[i][1] = R[3 + i]; b.a[i][2] = R[6 + i];
    }
    return b;
}

__device__ __forceinline__ int hull_frame(const PlanView &P, int k) {
    return __float_as_int(ldg(P.hulls, 4 * k + 3).w);
}

// hull k in world coordinates at configuration q (chain from the base)
__device__ __forceinline__ Box hull_world(const PlanView &P, const float (&q)[CP_MAX_JOINTS], int k) {
    const int f = hull_frame(P, k);
    Xf T;
    xf_identity(T);
#pragma unroll
    for (int j = 0; j < CP_MAX_JOINTS; ++j)
        if (j < f) xf_joint(T, ldg(P.joints, j), q[j]);
    const Box l = load_box(P.hulls, k);
    Box w;
    xf_point(T, l.c[0], l.c[1], l.c[2], w.c[0], w.c[1], w.c[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
            w.a[i][r] = __builtin_fmaf(T.r[3 * r], l.a[i][0], __builtin_fmaf(T.r[3 * r + 1], l.a[i][1], T.r[3 * r + 2] * l.a[i][2]));
        w.h[i] = l.h[i];
    }
    return w;
}

__device__ __forceinline__ float dot3(const float (&u)[3], const float (&v)[3]) {
    return __builtin_fmaf(u[0], v[0], __builtin_fmaf(u[1], v[1], u[2] * v[2]));
}

// SAT signed distance of boxes A and B: the largest gap over the fifteen
// axes.  B's three face axes come first; if the largest of their gaps is
// already above `bound` that partial maximum is returned (a lower bound of
// the SAT value, so still above `bound`: a caller keeping the minimum below
// `bound` is unaffected), otherwise every axis is taken.  The maximum is
// exact in floating point, so the full value does not depend on the order.
__device__ __forceinline__ float sat_distance(const Box &A, const Box &B, float bound) {
    float C[3][3], Ca[3][3], Tb[3];
    const float T[3] = {B.c[0] - A.c[0], B.c[1] - A.c[1], B.c[2] - A.c[2]};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        Tb[j] = dot3(T, B.a[j]);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            C[i][j] = dot3(A.a[i], B.a[j]);
            Ca[i][j] = fabsf(C[i][j]);
        }
    }
    float best = -kInf;
    // face axes of B
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float ra = __builtin_fmaf(A.h[0], Ca[0][j], __builtin_fmaf(A.h[1], Ca[1][j], A.h[2] * Ca[2][j]));
        best = fmaxf(best, fabsf(Tb[j]) - ra - B.h[j]);
    }
    if (best > bound) return best;
    // face axes of A
    float Ta[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Ta[i] = dot3(T, A.a[i]);
        const float rb = __builtin_fmaf(B.h[0], Ca[i][0], __builtin_fmaf(B.h[1], Ca[i][1], B.h[2] * Ca[i][2]));
        best = fmaxf(best, fabsf(Ta[i]) - A.h[i] - rb);
    }
    // cross axes a_i x b_j
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            const float l2 = __builtin_fmaf(-C[i][j], C[i][j], 1.0f);
            if (l2 > kParallel) {
                const float t = fabsf(__builtin_fmaf(C[i1][j], Ta[i2], -(C[i2][j] * Ta[i1])));
                const float ra = __builtin_fmaf(A.h[i1], Ca[i2][j], A.h[i2] * Ca[i1][j]);
                const float rb = __builtin_fmaf(B.h[j1], Ca[i][j2], B.h[j2] * Ca[i][j1]);
                best = fmaxf(best, (t - ra - rb) / fsqrt(l2));
            }
        }
    }
    return best;
}

// the box's lowest corner above the ground plane
__device__ __forceinline__ float ground_distance(const Box &A, float gz) {
    const float ext = __builtin_fmaf(A.h[0], fabsf(A.a[0][2]), __builtin_fmaf(A.h[1], fabsf(A.a[1][2]), A.h[2] * fabsf(A.a[2][2])));
    return (A.c[2] - ext) - gz;
}

struct SatMin {
    float d;
    uint32_t key;  // (hull << 16) | obstacle
};

__device__ __forceinline__ void take(SatMin &m, float d, uint32_t key) {
    if (d < m.d || (d == m.d && key < m.key)) {
        m.d = d;
        m.key = key;
    }
}

// d(q) and its pair (tie order: hull, then obstacle number)
__device__ __forceinline__ SatMin sat_config_distance(const PlanView &P, const float (&q)[CP_MAX_JOINTS]) {
    SatMin m;
    m.d = kInf;
    m.key = 0xFFFFFFFFu;
    // CP_PAIRS_ALL: every axis of every pair (no early exit)
    const bool all = P.pair_filter == CP_PAIRS_ALL;
    for (int k = 0; k < P.n_hulls; ++k) {
        const Box A = hull_world(P, q, k);
        const uint32_t kk = (uint32_t)k << 16;
        if (P.has_ground) take(m, ground_distance(A, P.ground_z), kk);
        for (int o = 0; o < P.n_obb; ++o)
            take(m, sat_distance(A, load_box(P.obb, o), all ? kInf : m.d), kk | (uint32_t)(1 + o));
    }
    for (int p = 0; p < P.n_hull_self; ++p) {
        const int2 hp = ldg(P.hull_self, p);
        take(m, sat_distance(hull_world(P, q, hp.x), hull_world(P, q, hp.y), all ? kInf : m.d),
             ((uint32_t)hp.x << 16) | (CP_OBS_SELF + (uint32_t)hp.y));
    }
    return m;
}

template <bool TAPE>
__global__ __launch_bounds__(256) void k_eval_fwd_sat(PlanView P, const float *__restrict__ W, int B,
                                                      double2 *__restrict__ partial, int slots,
                                                      uint32_t *__restrict__ tape) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = (int64_t)B * P.ns;
    const bool active = g < N;
    const int b = active ? (int)(g / P.ns) : B - 1;
    const int k = active ? (int)(g - (int64_t)b * P.ns) + 1 : 1;
    const float *Wb = W + (size_t)b * P.K * P.n_joints;
    float q[CP_MAX_JOINTS], dq[CP_MAX_JOINTS], bw[4], db[4];
    int j;
    interpolate(P, Wb, k, q, dq, j, bw, db);
    float jp, jl;
    step_terms(P, q, dq, jp, jl);
    const SatMin m = sat_config_distance(P, q);
    float dphi;
    const float phi = hinge_value(P, m.d, dphi);
    const float c = __builtin_fmaf(P.w_c, phi, __builtin_fmaf(P.w_l, jl, jp));
    if (TAPE && active) tape[g] = m.key;
    const int64_t g_first = uniform_i64(g & ~(int64_t)(kWave - 1));
    const int64_t g_last = min(g_first + kWave - 1, N - 1);
    path_partials(active ? b : -1, c, m.d, (int)(g_first / P.ns), (int)(g_last / P.ns), g_first / kWave, partial,
                  slots);
}

__global__ __launch_bounds__(256) void k_debug_configs_sat(PlanView P, const float *__restrict__ Q, int N,
                                                           float *__restrict__ dist, uint32_t *__restrict__ arg) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float q[CP_MAX_JOINTS];
#pragma unroll
    for (int j = 0; j < CP_MAX_JOINTS; ++j) q[j] = j < P.n_joints ? ldg(Q, (int64_t)i * P.n_joints + j) : 0.0f;
    const SatMin m = sat_config_distance(P, q);
    dist[i] = m.d;
    if (arg) arg[i] = m.key;
}

}  // namespace

hipError_t launch_eval_fwd_sat(const PlanView &P, const float *W, int B, double2 *partial, uint32_t *tape,
                               hipStream_t st) {
    const int64_t N = (int64_t)B * P.ns;
    const dim3 grid((unsigned)((N + 255) / 256));
    const int slots = eval_slots(P.ns);
    if (tape)
        hipLaunchKernelGGL(k_eval_fwd_sat<true>, grid, dim3(256), 0, st, P, W, B, partial, slots, tape);
    else
        hipLaunchKernelGGL(k_eval_fwd_sat<false>, grid, dim3(256), 0, st, P, W, B, partial, slots, tape);
    return hipGetLastError();
}

hipError_t launch_debug_configs_sat(const PlanView &P, const float *Q, int N, float *dist, uint32_t *arg,
                                    hipStream_t st) {
    hipLaunchKernelGGL(k_debug_configs_sat, dim3((N + 255) / 256), dim3(256), 0, st, P, Q, N, dist, arg);
    return hipGetLastError();
}

}  // namespace cp
