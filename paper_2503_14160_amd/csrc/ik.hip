// Collision-free inverse kinematics (Sec. 3.2, eq. IK opt): one hardware wave
// per row.  Every lane carries the row's whole solver state (the kinematic
// chain, the residual, the normal equations), so the Levenberg-Marquardt
// arithmetic and control flow are wave-uniform; the lanes share out the
// signed distance d(q), the minimum over every (sphere, obstacle) and
// self-collision pair, which is where the work is.  Each lane holds one or
// two spheres (sorted slots lane, lane + 64) and runs them against every
// obstacle, the obstacle records being wave-uniform scalar loads (the path
// evaluation's pair loop, with its shared height term per group of trees);
// the self pairs are dealt out over the lanes from the centres in LDS.  The
// minimising pair, in the oracle's tie order, comes from a second pass over
// the obstacles, dealt out over the lanes, for the lowest-numbered sphere
// that attains the minimum.  Kernels are instantiated for at most 6 or 8
// joints (NJ) and for 1 or 2 spheres per lane (G).
#include "launch.h"

namespace cp {
namespace {

struct IkPrm {
    float lq, lc, le, lr;
    int max_iters;
    float tau, eps_grad, eps_step;
    int clamp;
};

// Order of equal distances, as in the evaluation: the lower sphere (caller
// index), then its scene obstacles in number order (ground 0, cylinders,
// boxes), the grid, then its self pairs by the other sphere.
constexpr uint32_t kKeySdf = 65280u;
constexpr uint32_t kKeySelf = 65281u;

struct PairMin {
    float d;
    uint32_t key;  // (sphere << 17) | obstacle key
};

__device__ __forceinline__ void pm_take(PairMin &b, float d, uint32_t key) {
    if (d < b.d || (d == b.d && key < b.key)) {
        b.d = d;
        b.key = key;
    }
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, kWave));
    return v;
}

// sphere centres (sorted order) with radius, and their caller indices
struct IkShared {
    float4 c[CP_MAX_SPHERES];
    int32_t orig[CP_MAX_SPHERES];
};

// The chain at q, wave-uniform: world axis and pivot (origin of the frame the
// joint moves) of every joint, the last frame's rotation, the tip point.
template <int NJ>
struct Chain {
    float aw[NJ][3], piv[NJ][3];
    float R[9];
    float p[3];
};

// This lane's spheres (sorted slots lane + 64 s, s < G): centre, radius and
// caller index; slots past the last sphere hold a far-away centre (every
// distance +inf) and radius 0.
template <int G>
struct LaneSpheres {
    float x[G], y[G], z[G], r[G];
    uint32_t orig[G];
    bool valid[G];
};

template <int NJ, int G>
__device__ __forceinline__ void chain_and_spheres(const PlanView &P, const float (&q)[NJ], Chain<NJ> &C,
                                                  LaneSpheres<G> &ls, IkShared &sh) {
    const int lane = threadIdx.x;
    SphereDev sd[G];
#pragma unroll
    for (int s = 0; s < G; ++s) {
        const int i = lane + s * kWave;
        ls.valid[s] = i < P.n_spheres;
        sd[s] = ls.valid[s] ? ldg(P.spheres, i) : SphereDev{};
        ls.x[s] = kInf; ls.y[s] = kInf; ls.z[s] = kInf;
        ls.r[s] = ls.valid[s] ? sd[s].r : 0.0f;
        ls.orig[s] = ls.valid[s] ? (uint32_t)sd[s].orig : 0xFFFFu;
    }
    Xf T;
    xf_identity(T);
#pragma unroll
    for (int f = 0; f <= NJ; ++f) {
        if (f > P.n_joints) break;
        if (f > 0) {
            const JointDev J = ldg(P.joints, f - 1);
            // world axis of joint f-1: R_{f-1} a (its own motion leaves it unchanged)
            C.aw[f - 1][0] = __builtin_fmaf(T.r[0], J.ax, __builtin_fmaf(T.r[1], J.ay, T.r[2] * J.az));
            C.aw[f - 1][1] = __builtin_fmaf(T.r[3], J.ax, __builtin_fmaf(T.r[4], J.ay, T.r[5] * J.az));
            C.aw[f - 1][2] = __builtin_fmaf(T.r[6], J.ax, __builtin_fmaf(T.r[7], J.ay, T.r[8] * J.az));
            xf_joint(T, J, q[f - 1]);
            C.piv[f - 1][0] = T.p[0]; C.piv[f - 1][1] = T.p[1]; C.piv[f - 1][2] = T.p[2];
        }
#pragma unroll
        for (int s = 0; s < G; ++s)
            if (ls.valid[s] && sd[s].frame == f) xf_point(T, sd[s].lx, sd[s].ly, sd[s].lz, ls.x[s], ls.y[s], ls.z[s]);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) C.R[i] = T.r[i];
    xf_point(T, P.tip[0], P.tip[1], P.tip[2], C.p[0], C.p[1], C.p[2]);
    __syncthreads();  // the previous evaluation's readers are done
#pragma unroll
    for (int s = 0; s < G; ++s) {
        const int i = lane + s * kWave;
        if (ls.valid[s]) {
            sh.c[i] = make_float4(ls.x[s], ls.y[s], ls.z[s], ls.r[s]);
            sh.orig[i] = (int32_t)ls.orig[s];
        }
    }
    __syncthreads();
}

// signed distance of obstacle `code` (0 ground, 1.. cylinders, then boxes, in
// the caller's order) at c, the same arithmetic as the pair loop
__device__ __forceinline__ float obstacle_sd(const PlanView &P, int code, float cx, float cy, float cz) {
    if (code == 0) return cz - P.ground_z;
    if (code <= P.n_cyl) {
        const float4 cy4 = ldg(P.cyl_orig, code - 1);
        const GroupDev gr = ldg(P.groups, __float_as_int(cy4.w));
        return cyl_combine(cyl_radial(cx, cy, cy4), fabsf(cz - gr.zc) - gr.hz);
    }
    const int o = code - 1 - P.n_cyl;
    return box_sd(cx, cy, cz, ldg(P.box, 2 * o), ldg(P.box, 2 * o + 1));
}

// d(q) and its pair, wave-uniform
template <int G>
__device__ __forceinline__ PairMin wave_distance(const PlanView &P, const LaneSpheres<G> &ls, const IkShared &sh) {
    const int lane = threadIdx.x;
    // scene: every obstacle against this lane's spheres
    float v[G], ds[G];
    spheres_min_sd<G>(P, ls.x, ls.y, ls.z, v);
    float lane_min = kInf;
#pragma unroll
    for (int s = 0; s < G; ++s) {
        ds[s] = v[s] - ls.r[s];
        if (P.sdf && ls.valid[s]) ds[s] = fminf(ds[s], sdf_query(P, ls.x[s], ls.y[s], ls.z[s], nullptr) - ls.r[s]);
        if (!ls.valid[s]) ds[s] = kInf;
        lane_min = fminf(lane_min, ds[s]);
    }
    // self-collision: the sphere pairs of each listed frame pair shared out
    PairMin bs;
    bs.d = kInf;
    bs.key = 0xFFFFFFFFu;
    for (int k = 0; k < P.n_self; ++k) {
        const int2 fp = ldg(P.self_pairs, k);
        const int a0 = ldg(P.frame_start, fp.x), na = ldg(P.frame_start, fp.x + 1) - a0;
        const int b0 = ldg(P.frame_start, fp.y), nb = ldg(P.frame_start, fp.y + 1) - b0;
        for (int t = lane; t < na * nb; t += kWave) {
            const int ia = a0 + t / nb, ib = b0 + t % nb;
            const float4 ca = sh.c[ia], cb = sh.c[ib];
            const float dx = ca.x - cb.x, dy = ca.y - cb.y, dz = ca.z - cb.z;
            const float d = fsqrt(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz))) - ca.w - cb.w;
            const uint32_t oa = (uint32_t)sh.orig[ia], ob = (uint32_t)sh.orig[ib];
            const uint32_t lo = min(oa, ob), hi = max(oa, ob);
            pm_take(bs, d, (lo << 17) | (kKeySelf + hi));
        }
    }
    lane_min = fminf(lane_min, bs.d);
    PairMin w;
    w.d = wave_min_u(lane_min);
    // the lowest-numbered sphere whose scene distance attains the minimum,
    // and its lowest obstacle among those that do
    uint32_t so = 0xFFFFFFFFu;
#pragma unroll
    for (int s = 0; s < G; ++s)
        if (ds[s] == w.d) so = min(so, ls.orig[s]);
    so = wave_min_u32(so);
    uint32_t key = 0xFFFFFFFFu;
    if (so != 0xFFFFFFFFu) {
        const float4 c = sh.c[ldg(P.sphere_slot, (int)so)];
        uint32_t kc = 0xFFFFFFFFu;
        const int n_codes = 1 + P.n_cyl + P.n_box;
        for (int code = lane; code < n_codes; code += kWave) {
            if (code == 0 && !P.has_ground) continue;
            if (obstacle_sd(P, code, c.x, c.y, c.z) - c.w == w.d) kc = min(kc, (uint32_t)code);
        }
        if (lane == 0 && P.sdf && sdf_query(P, c.x, c.y, c.z, nullptr) - c.w == w.d) kc = min(kc, kKeySdf);
        kc = wave_min_u32(kc);
        key = (so << 17) | kc;
    }
    w.key = min(key, wave_min_u32(bs.d == w.d ? bs.key : 0xFFFFFFFFu));
    return w;
}

// d d(q) / d q through the minimising pair (wave-uniform)
template <int NJ>
__device__ __forceinline__ void distance_grad(const PlanView &P, const Chain<NJ> &C, const IkShared &sh,
                                              const PairMin &pm, float (&gd)[NJ]) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) gd[j] = 0.0f;
    const int s = (int)(pm.key >> 17);
    const uint32_t ok = pm.key & 0x1FFFFu;
    if (s >= P.n_spheres) return;
    const int si = ldg(P.sphere_slot, s);
    const float4 c = sh.c[si];
    const int fs = ldg(P.spheres, si).frame;
    float g[3];
    float e[3] = {0.0f, 0.0f, 0.0f};
    int fb = 0;
    if (ok >= kKeySelf) {
        const int bo = (int)(ok - kKeySelf);
        if (bo >= P.n_spheres) return;
        const int bi = ldg(P.sphere_slot, bo);
        const float4 cb = sh.c[bi];
        fb = ldg(P.spheres, bi).frame;
        e[0] = cb.x; e[1] = cb.y; e[2] = cb.z;
        const float dx = c.x - cb.x, dy = c.y - cb.y, dz = c.z - cb.z;
        const float len = fsqrt(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
        const float inv = len > 0.0f ? 1.0f / len : 0.0f;
        g[0] = dx * inv; g[1] = dy * inv; g[2] = dz * inv;
    } else {
        obstacle_sd_grad(P, ok == kKeySdf ? CP_OBS_SDF : ok, c.x, c.y, c.z, g);
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        if (j >= P.n_joints) break;
        const bool rev = ldg(P.joints, j).type == CP_REVOLUTE;
        float v[3] = {0.0f, 0.0f, 0.0f};
        if (j < fs) {
            if (rev) {
                const float rx = c.x - C.piv[j][0], ry = c.y - C.piv[j][1], rz = c.z - C.piv[j][2];
                v[0] = C.aw[j][1] * rz - C.aw[j][2] * ry;
                v[1] = C.aw[j][2] * rx - C.aw[j][0] * rz;
                v[2] = C.aw[j][0] * ry - C.aw[j][1] * rx;
            } else {
                v[0] = C.aw[j][0]; v[1] = C.aw[j][1]; v[2] = C.aw[j][2];
            }
        }
        if (ok >= kKeySelf && j < fb) {
            if (rev) {
                const float rx = e[0] - C.piv[j][0], ry = e[1] - C.piv[j][1], rz = e[2] - C.piv[j][2];
                v[0] -= C.aw[j][1] * rz - C.aw[j][2] * ry;
                v[1] -= C.aw[j][2] * rx - C.aw[j][0] * rz;
                v[2] -= C.aw[j][0] * ry - C.aw[j][1] * rx;
            } else {
                v[0] -= C.aw[j][0]; v[1] -= C.aw[j][1]; v[2] -= C.aw[j][2];
            }
        }
        gd[j] = __builtin_fmaf(g[0], v[0], __builtin_fmaf(g[1], v[1], g[2] * v[2]));
    }
}

__device__ __forceinline__ void cross(const float a[3], const float b[3], float out[3]) {
    const float x = a[1] * b[2] - a[2] * b[1];
    const float y = a[2] * b[0] - a[0] * b[2];
    const float z = a[0] * b[1] - a[1] * b[0];
    out[0] = x; out[1] = y; out[2] = z;
}

// Log of SO(3): theta = atan2(|v| / 2, (tr E - 1) / 2) with v = vee(E - E^T)
// = 2 sin(theta) n; axis v / |v|, or near theta = pi the column of the
// symmetric part (E + E^T) / 2 - cos(theta) I = (1 - cos theta) n n^T with
// the largest diagonal entry (signed so that n . v >= 0).
__device__ __forceinline__ void so3_log(const float (&E)[9], float (&w)[3]) {
    const float v[3] = {E[7] - E[5], E[2] - E[6], E[3] - E[1]};
    const float vn = fsqrt(__builtin_fmaf(v[0], v[0], __builtin_fmaf(v[1], v[1], v[2] * v[2])));
    const float c = 0.5f * (E[0] + E[4] + E[8] - 1.0f);
    const float th = atan2f(0.5f * vn, c);
    if (c > -0.9f) {
        const float k = vn > 0.0f ? th / vn : 0.0f;
        w[0] = k * v[0]; w[1] = k * v[1]; w[2] = k * v[2];
        return;
    }
    const float d0 = E[0] - c, d1 = E[4] - c, d2 = E[8] - c;
    int k = 0;
    if (d1 > d0) k = 1;
    if (d2 > (k == 0 ? d0 : d1)) k = 2;
    const float dk = k == 0 ? d0 : (k == 1 ? d1 : d2);
    const float omc = 1.0f - c;
    const float nk = fsqrt(fmaxf(dk, 0.0f) / omc);
    float n[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        n[i] = i == k ? nk : 0.5f * (E[3 * k + i] + E[3 * i + k]) / (omc * nk);
    const float sg = (n[0] * v[0] + n[1] * v[1] + n[2] * v[2]) < 0.0f ? -th : th;
    w[0] = sg * n[0]; w[1] = sg * n[1]; w[2] = sg * n[2];
}

// inverse right Jacobian of SO(3) at w: I + [w]/2 + k [w]^2 with
// k = 1/theta^2 - (1 + cos theta) / (2 theta sin theta), by its series
// 1/12 + theta^2/720 + theta^4/30240 + theta^6/1209600 below 0.5 (in single
// precision the closed form cancels there)
__device__ __forceinline__ void so3_jr_inv(const float (&w)[3], float (&Ji)[9]) {
    const float t2 = __builtin_fmaf(w[0], w[0], __builtin_fmaf(w[1], w[1], w[2] * w[2]));
    const float th = fsqrt(t2);
    float k;
    if (th < 0.5f) {
        k = __builtin_fmaf(t2, __builtin_fmaf(t2, __builtin_fmaf(t2, 1.0f / 1209600.0f, 1.0f / 30240.0f), 1.0f / 720.0f),
                           1.0f / 12.0f);
    } else {
        float s, cth;
        sincosf(th, &s, &cth);
        k = 1.0f / t2 - (1.0f + cth) / (2.0f * th * s);
    }
    const float W[9] = {0.0f, -w[2], w[1], w[2], 0.0f, -w[0], -w[1], w[0], 0.0f};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float s2 = __builtin_fmaf(W[3 * i], W[j], __builtin_fmaf(W[3 * i + 1], W[3 + j], W[3 * i + 2] * W[6 + j]));
            Ji[3 * i + j] = (i == j ? 1.0f : 0.0f) + __builtin_fmaf(0.5f, W[3 * i + j], k * s2);
        }
}

// Residual rows 0..7 (the regularisation rows are implicit) and their
// Jacobian [8][n], wave-uniform.
template <int NJ>
struct IkEval {
    float r[8];
    float J[8][NJ];
    float pos_err, rot_err, d, gp;
};

template <int NJ, int G>
__device__ __forceinline__ void ik_eval(const PlanView &P, const IkPrm &prm, const float (&tg)[12],
                                        const float (&q)[NJ], IkShared &sh, IkEval<NJ> &E) {
    const int n = P.n_joints;
    Chain<NJ> C;
    LaneSpheres<G> ls;
    chain_and_spheres<NJ, G>(P, q, C, ls, sh);
    const PairMin pm = wave_distance<G>(P, ls, sh);
    // d p / d q_j
    float dp[NJ][3];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        dp[j][0] = dp[j][1] = dp[j][2] = 0.0f;
        if (j < n) {
            if (ldg(P.joints, j).type == CP_REVOLUTE) {
                const float r[3] = {C.p[0] - C.piv[j][0], C.p[1] - C.piv[j][1], C.p[2] - C.piv[j][2]};
                cross(C.aw[j], r, dp[j]);
            } else {
                dp[j][0] = C.aw[j][0]; dp[j][1] = C.aw[j][1]; dp[j][2] = C.aw[j][2];
            }
        }
    }
    // position
#pragma unroll
    for (int i = 0; i < 3; ++i) E.r[i] = C.p[i] - tg[9 + i];
    E.pos_err = fsqrt(__builtin_fmaf(E.r[0], E.r[0], __builtin_fmaf(E.r[1], E.r[1], E.r[2] * E.r[2])));
    // orientation: Log(R_d^T R_g)
    float Em[9], w[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            Em[3 * i + k] = __builtin_fmaf(tg[i], C.R[k], __builtin_fmaf(tg[3 + i], C.R[3 + k], tg[6 + i] * C.R[6 + k]));
    so3_log(Em, w);
#pragma unroll
    for (int i = 0; i < 3; ++i) E.r[3 + i] = prm.lq * w[i];
    E.rot_err = fsqrt(__builtin_fmaf(w[0], w[0], __builtin_fmaf(w[1], w[1], w[2] * w[2])));
    // collision
    E.d = pm.d;
    E.r[6] = pm.d < 0.0f ? prm.lc * (-pm.d) : 0.0f;
    // equilibrium of the joints that are not actuated
    float gp[NJ], gp2 = 0.0f;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        gp[j] = (j < n && !ldg(P.joints, j).active) ? dp[j][2] : 0.0f;
        gp2 = __builtin_fmaf(gp[j], gp[j], gp2);
    }
    E.r[7] = prm.le * gp2;
    E.gp = fsqrt(gp2);
    // Jacobian
    float Ji[9];
    so3_jr_inv(w, Ji);
    float gd[NJ];
    if (pm.d < 0.0f) distance_grad(P, C, sh, pm, gd);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int i = 0; i < 8; ++i) E.J[i][j] = 0.0f;
        if (j >= n) continue;
        const JointDev Jj = ldg(P.joints, j);
        E.J[0][j] = dp[j][0]; E.J[1][j] = dp[j][1]; E.J[2][j] = dp[j][2];
        if (Jj.type == CP_REVOLUTE) {
            // rotating about the world axis a_j: R_g -> R_g Exp(dq R_g^T a_j)
            float bb[3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                bb[i] = __builtin_fmaf(C.R[i], C.aw[j][0], __builtin_fmaf(C.R[3 + i], C.aw[j][1], C.R[6 + i] * C.aw[j][2]));
#pragma unroll
            for (int i = 0; i < 3; ++i)
                E.J[3 + i][j] = prm.lq * __builtin_fmaf(Ji[3 * i], bb[0], __builtin_fmaf(Ji[3 * i + 1], bb[1], Ji[3 * i + 2] * bb[2]));
        }
        if (pm.d < 0.0f) E.J[6][j] = -prm.lc * gd[j];
        // d r_e / d q_j = 2 lambda_e sum_k g_k d^2 z / dq_k dq_j, with
        // u = min(k, j), v = max(k, j): v revolute -> a_u x (a_v x (p - o_v))
        // for revolute u; v prismatic -> a_u x a_v for revolute u < v
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < NJ; ++k) {
            if (k >= n || gp[k] == 0.0f) continue;
            const int u = k < j ? k : j, v = k < j ? j : k;
            const bool ur = ldg(P.joints, u).type == CP_REVOLUTE;
            const bool vr = ldg(P.joints, v).type == CP_REVOLUTE;
            float hz = 0.0f;
            if (vr && ur) {
                const float r[3] = {C.p[0] - C.piv[v][0], C.p[1] - C.piv[v][1], C.p[2] - C.piv[v][2]};
                float t[3];
                cross(C.aw[v], r, t);
                hz = C.aw[u][0] * t[1] - C.aw[u][1] * t[0];
            } else if (!vr && ur && u < v) {
                hz = C.aw[u][0] * C.aw[v][1] - C.aw[u][1] * C.aw[v][0];
            }
            s = __builtin_fmaf(gp[k], hz, s);
        }
        E.J[7][j] = 2.0f * prm.le * s;
    }
}

__device__ __forceinline__ double sq_d(float x) { return (double)x * (double)x; }

// F = |r|^2 / 2 over the eight explicit rows and the regularisation rows
// lambda_r (q - q_ref)
template <int NJ>
__device__ __forceinline__ double half_sq_norm(const IkEval<NJ> &E, const IkPrm &prm, int n, const float (&q)[NJ],
                                               const float (&qr)[NJ]) {
    const double lr2 = (double)prm.lr * (double)prm.lr;
    double f = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) f += sq_d(E.r[k]);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const double dq = i < n ? (double)q[i] - (double)qr[i] : 0.0;
        f += lr2 * dq * dq;
    }
    return 0.5 * f;
}

// A = J^T J + lambda_r^2 I and g = J^T r + lambda_r^2 (q - q_ref) over the n
// joints, padded to NJ with identity rows (so the padded entries of the step
// are 0)
template <int NJ>
__device__ __forceinline__ void normal_eq(const IkEval<NJ> &E, const IkPrm &prm, int n, const float (&q)[NJ],
                                          const float (&qr)[NJ], double (&A)[NJ][NJ], double (&g)[NJ]) {
    const double lr2 = (double)prm.lr * (double)prm.lr;
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const double dq = i < n ? (double)q[i] - (double)qr[i] : 0.0;
        double gi = lr2 * dq;
#pragma unroll
        for (int k = 0; k < 8; ++k) gi += (double)E.J[k][i] * (double)E.r[k];
        g[i] = i < n ? gi : 0.0;
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double a = (i == j) ? lr2 : 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) a += (double)E.J[k][i] * (double)E.J[k][j];
            if (i >= n || j >= n) a = (i == j) ? 1.0 : 0.0;
            A[i][j] = a;
            A[j][i] = a;
        }
    }
}

// (A + mu I) h = -g by a Cholesky factorisation in double precision; false if
// a pivot is not positive
template <int NJ>
__device__ __forceinline__ bool damped_solve(const double (&A)[NJ][NJ], const double (&g)[NJ], double mu, int n,
                                             double (&h)[NJ]) {
    double L[NJ][NJ];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double s = A[i][j] + ((i == j && i < n) ? mu : 0.0);
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                ok = ok && s > 0.0;
                L[i][i] = sqrt(s > 0.0 ? s : 1.0);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    }
    double y[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        double s = -g[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
#pragma unroll
    for (int i = NJ - 1; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < NJ; ++k) s -= L[k][i] * h[k];
        h[i] = s / L[i][i];
    }
    return ok;
}

template <int NJ>
__device__ __forceinline__ void load_row(const float *src, int row, int n, float (&q)[NJ]) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) q[j] = j < n ? ldg(src, (int64_t)row * n + j) : 0.0f;
}

template <int NJ, int G>
__global__ __launch_bounds__(kWave) void k_ik_solve(PlanView P, IkPrm prm, const float *__restrict__ target,
                                                    const float *__restrict__ q_init, const float *__restrict__ q_ref,
                                                    int N, float *__restrict__ q_out, float *__restrict__ info,
                                                    int32_t *__restrict__ status_out) {
    __shared__ IkShared sh;
    const int row = blockIdx.x;
    if (row >= N) return;
    const int n = P.n_joints;
    float tg[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) tg[i] = ldg(target, (int64_t)row * 12 + i);
    float q[NJ], qr[NJ], lo[NJ], hi[NJ];
    load_row(q_init, row, n, q);
    load_row(q_ref ? q_ref : q_init, row, n, qr);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        lo[j] = j < n ? ldg(P.joints, j).qmin : 0.0f;
        hi[j] = j < n ? ldg(P.joints, j).qmax : 0.0f;
        if (prm.clamp) q[j] = fminf(fmaxf(q[j], lo[j]), hi[j]);
    }
    // state of the iteration: q, F(q), A = J^T J (+ lambda_r^2 I), g = J^T r
    IkEval<NJ> E;
    ik_eval<NJ, G>(P, prm, tg, q, sh, E);
    double A[NJ][NJ], g[NJ];
    double F = half_sq_norm(E, prm, n, q, qr);
    normal_eq(E, prm, n, q, qr, A, g);
    float info_pos = E.pos_err, info_rot = E.rot_err, info_d = E.d, info_gp = E.gp;
    double amax = 0.0;
#pragma unroll
    for (int i = 0; i < NJ; ++i)
        if (i < n) amax = fmax(amax, A[i][i]);
    double mu = (double)prm.tau * amax, nu = 2.0;
    int it = 0, status = 0;
    while (it < prm.max_iters) {
        double gmax = 0.0;
#pragma unroll
        for (int i = 0; i < NJ; ++i) gmax = fmax(gmax, fabs(g[i]));
        if (gmax <= (double)prm.eps_grad) {
            status = 1;
            break;
        }
        double h[NJ];
        damped_solve(A, g, mu, n, h);
        double hn = 0.0, qn2 = 0.0;
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            hn += h[i] * h[i];
            qn2 += (double)q[i] * (double)q[i];
        }
        hn = sqrt(hn);
        if (!(hn > (double)prm.eps_step * (sqrt(qn2) + (double)prm.eps_step))) {
            status = 2;
            break;
        }
        // trial point (FP32 joint values, clamped) and the decrease the
        // linear model predicts for the step actually taken:
        // L(0) - L(s) = -s.g - s.A s / 2
        float qt[NJ];
        double pred = 0.0;
        {
            double st[NJ];
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                float v = (float)((double)q[i] + h[i]);
                if (prm.clamp) v = fminf(fmaxf(v, lo[i]), hi[i]);
                qt[i] = i < n ? v : 0.0f;
                st[i] = (double)qt[i] - (double)q[i];
            }
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                double as = 0.0;
#pragma unroll
                for (int j = 0; j < NJ; ++j) as += A[i][j] * st[j];
                pred -= st[i] * g[i] + 0.5 * st[i] * as;
            }
        }
        ik_eval<NJ, G>(P, prm, tg, qt, sh, E);
        const double Ft = half_sq_norm(E, prm, n, qt, qr);
        ++it;
        if (pred > 0.0 && F - Ft > 0.0) {
            const double rho = (F - Ft) / pred;
            const double t = 2.0 * rho - 1.0;
            mu *= fmax(1.0 / 3.0, 1.0 - t * t * t);
            nu = 2.0;
#pragma unroll
            for (int i = 0; i < NJ; ++i) q[i] = qt[i];
            F = Ft;
            normal_eq(E, prm, n, q, qr, A, g);
            info_pos = E.pos_err; info_rot = E.rot_err; info_d = E.d; info_gp = E.gp;
        } else {
            mu *= nu;
            nu *= 2.0;
        }
    }
    if (threadIdx.x == 0) {
        for (int j = 0; j < n; ++j) q_out[(int64_t)row * n + j] = q[j];
        if (info) {
            float *o = info + (int64_t)row * 6;
            o[0] = (float)F; o[1] = info_pos; o[2] = info_rot; o[3] = info_d; o[4] = info_gp; o[5] = (float)it;
        }
        if (status_out) status_out[row] = status;
    }
}

// per group of `restarts` rows, the row with the lowest F (NaN as +inf; ties
// keep the lowest row)
__global__ __launch_bounds__(256) void k_ik_best(const float *__restrict__ info, int groups, int restarts,
                                                 int32_t *__restrict__ best) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= groups) return;
    int arg = t * restarts;
    uint32_t bk = cost_key(info[(int64_t)arg * 6]);
    for (int r = 1; r < restarts; ++r) {
        const int row = t * restarts + r;
        const uint32_t k = cost_key(info[(int64_t)row * 6]);
        if (k < bk) {
            bk = k;
            arg = row;
        }
    }
    best[t] = arg;
}

template <int NJ, int G>
__global__ __launch_bounds__(kWave) void k_ik_residual(PlanView P, IkPrm prm, const float *__restrict__ target,
                                                       const float *__restrict__ qv, const float *__restrict__ q_ref,
                                                       int N, float *__restrict__ r_out, float *__restrict__ J_out) {
    __shared__ IkShared sh;
    const int row = blockIdx.x;
    if (row >= N) return;
    const int n = P.n_joints, m = 8 + n;
    float tg[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) tg[i] = ldg(target, (int64_t)row * 12 + i);
    float q[NJ], qr[NJ];
    load_row(qv, row, n, q);
    load_row(q_ref ? q_ref : qv, row, n, qr);
    IkEval<NJ> E;
    ik_eval<NJ, G>(P, prm, tg, q, sh, E);
    if (threadIdx.x != 0) return;
    if (r_out) {
        float *r = r_out + (int64_t)row * m;
        for (int i = 0; i < 8; ++i) r[i] = E.r[i];
        for (int j = 0; j < n; ++j) r[8 + j] = prm.lr * (q[j] - qr[j]);
    }
    if (J_out) {
        float *J = J_out + (int64_t)row * m * n;
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < n; ++j) J[i * n + j] = E.J[i][j];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) J[(8 + i) * n + j] = i == j ? prm.lr : 0.0f;
    }
}

IkPrm to_prm(const cp_ik_params &p) {
    IkPrm d;
    d.lq = p.lambda_q; d.lc = p.lambda_c; d.le = p.lambda_e; d.lr = p.lambda_r;
    d.max_iters = p.max_iters;
    d.tau = p.tau; d.eps_grad = p.eps_grad; d.eps_step = p.eps_step;
    d.clamp = p.clamp;
    return d;
}

}  // namespace

hipError_t launch_ik_solve(const PlanView &P, const cp_ik_params &prm, const float *target, const float *q_init,
                           const float *q_ref, int N, int restarts, float *q_out, float *info, int32_t *status,
                           int32_t *best, hipStream_t st) {
    const IkPrm d = to_prm(prm);
    const bool small = P.n_joints <= 6, one = P.n_spheres <= kWave;
    if (small && one)
        hipLaunchKernelGGL((k_ik_solve<6, 1>), dim3(N), dim3(kWave), 0, st, P, d, target, q_init, q_ref, N, q_out, info,
                           status);
    else if (small)
        hipLaunchKernelGGL((k_ik_solve<6, 2>), dim3(N), dim3(kWave), 0, st, P, d, target, q_init, q_ref, N, q_out, info,
                           status);
    else if (one)
        hipLaunchKernelGGL((k_ik_solve<CP_MAX_JOINTS, 1>), dim3(N), dim3(kWave), 0, st, P, d, target, q_init, q_ref, N,
                           q_out, info, status);
    else
        hipLaunchKernelGGL((k_ik_solve<CP_MAX_JOINTS, 2>), dim3(N), dim3(kWave), 0, st, P, d, target, q_init, q_ref, N,
                           q_out, info, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !best) return e;
    const int groups = N / restarts;
    hipLaunchKernelGGL(k_ik_best, dim3((groups + 255) / 256), dim3(256), 0, st, info, groups, restarts, best);
    return hipGetLastError();
}

hipError_t launch_ik_residual(const PlanView &P, const cp_ik_params &prm, const float *target, const float *q,
                              const float *q_ref, int N, float *r, float *J, hipStream_t st) {
    const IkPrm d = to_prm(prm);
    const bool small = P.n_joints <= 6, one = P.n_spheres <= kWave;
    if (small && one)
        hipLaunchKernelGGL((k_ik_residual<6, 1>), dim3(N), dim3(kWave), 0, st, P, d, target, q, q_ref, N, r, J);
    else if (small)
        hipLaunchKernelGGL((k_ik_residual<6, 2>), dim3(N), dim3(kWave), 0, st, P, d, target, q, q_ref, N, r, J);
    else if (one)
        hipLaunchKernelGGL((k_ik_residual<CP_MAX_JOINTS, 1>), dim3(N), dim3(kWave), 0, st, P, d, target, q, q_ref, N, r,
                           J);
    else
        hipLaunchKernelGGL((k_ik_residual<CP_MAX_JOINTS, 2>), dim3(N), dim3(kWave), 0, st, P, d, target, q, q_ref, N, r,
                           J);
    return hipGetLastError();
}

}  // namespace cp
