// Step two of the planner (Sec. 4.2, eq. discrete): direct collocation of the
// reduced dynamics (Sec. 2.1) with trapezoidal defects, solved by an
// augmented Lagrangian on the defects around Levenberg-Marquardt, in double
// precision.  One workgroup of 256 threads per problem.
//
// Unknowns, per time point k = 0..N, a block [x_k (2n), u_k (n_a)] of MB =
// 2n + n_a entries (x_0 and x_N are fixed: their entries stay in the block
// with identity rows in the normal equations and no gradient), and s with
// t_F = s^2.  The normal equations J^T J + damping I are block tridiagonal
// in these blocks (a defect couples k and k + 1) with a dense last column
// for s; they are solved by a block Cholesky sweep (the block Thomas
// algorithm) for two right-hand sides and a Schur complement on s.
// The final time has the lower bound t_min = max_j |q_d,j - q_0,j| / v_max,j
// that the velocity limits imply (a penalty of weight mu on s < sqrt(t_min),
// like the state bounds): without it t_F = s^2 makes s = 0 a stationary
// point of every residual, which a low first penalty can fall into.
// Dynamics: the actuated joints' accelerations are the inputs; the passive
// joints follow a unit load at the tip on massless links:
//   qdd_p = -(J_p^T J_p)^-1 J_p^T (J_a u + c + g e_z) - damping qd_p,
// J = d tip / dq, c = sum_ij (d^2 tip / dq_i dq_j) qd_i qd_j.  Jacobians of
// the dynamics by central differences (positions: step fd_q; velocities and
// inputs, where the accelerations are quadratic and linear: step 1).
#include "launch.h"

namespace cp {
namespace {

constexpr int kTrajThreads = 256;
constexpr int kMB = kTrajBlock;  // block size 2n + n_a (padded)

struct TrajDev {
    int N, n, na, outer, max_iters;
    double omega_s, omega_t, grav, damping, mu0, mu_factor, tau, eps_grad, eps_step, fd_q, t_f0;
    double v_max[CP_MAX_JOINTS];
    int act[CP_MAX_JOINTS];
};

// per-problem workspace (doubles), offsets in units of doubles
struct TrajWork {
    double *z, *zt;      // [(N+1) MB + 1]
    double *f, *ft;      // [N+1][2n] at z and at the trial point
    double *Jx, *Ju;     // [N+1][2n][2n], [N+1][2n][na]
    double *lam;         // [N][2n]
    double *D, *E;       // [N+1][MB][MB], [N][MB][MB]
    double *c, *g;       // [(N+1) MB + 1] each (g's last entry: g_s)
    double *LD, *LX;     // factors [N+1][MB][MB], [N][MB][MB]
    double *y, *w, *h;   // [(N+1) MB + 1]
};

__host__ __device__ inline size_t traj_nz(int N) { return (size_t)(N + 1) * kMB + 1; }

__host__ __device__ inline size_t traj_work_doubles(int N, int n, int na) {
    const size_t nz = traj_nz(N);
    return 2 * nz + 2 * (size_t)(N + 1) * 2 * n + (size_t)(N + 1) * 4 * n * n + (size_t)(N + 1) * 2 * n * na +
           (size_t)N * 2 * n + 2 * (size_t)(N + 1) * kMB * kMB + 2 * (size_t)N * kMB * kMB + 5 * nz;
}

__device__ inline TrajWork traj_work(double *base, int N, int n, int na) {
    TrajWork w;
    const size_t nz = traj_nz(N);
    double *p = base;
    w.z = p; p += nz;
    w.zt = p; p += nz;
    w.f = p; p += (size_t)(N + 1) * 2 * n;
    w.ft = p; p += (size_t)(N + 1) * 2 * n;
    w.Jx = p; p += (size_t)(N + 1) * 4 * n * n;
    w.Ju = p; p += (size_t)(N + 1) * 2 * n * na;
    w.lam = p; p += (size_t)N * 2 * n;
    w.D = p; p += (size_t)(N + 1) * kMB * kMB;
    w.E = p; p += (size_t)N * kMB * kMB;
    w.LD = p; p += (size_t)(N + 1) * kMB * kMB;
    w.LX = p; p += (size_t)N * kMB * kMB;
    w.c = p; p += nz;
    w.g = p; p += nz;
    w.y = p; p += nz;
    w.w = p; p += nz;
    w.h = p; p += nz;
    return w;
}

// ---------------------------------------------------------------------------
// dynamics in double precision
// ---------------------------------------------------------------------------

// The dynamics are templated on the chain's joint count NJ (6: the crane,
// every loop bound fixed; CP_MAX_JOINTS: any chain of at most that many
// joints, the joints past n skipped), so every array below is indexed by
// constants and lives in registers.
template <int NJ>
__device__ inline int chain_n(const TrajDev &T) {
    return NJ == 6 ? 6 : T.n;
}

// joint accelerations qdd at (q, qd) with uf the actuated joints'
// accelerations (entries of passive joints unused)
template <int NJ>
__device__ void crane_accel(const PlanView &P, const TrajDev &T, const double (&q)[NJ], const double (&qd)[NJ],
                            const double (&uf)[NJ], double (&qdd)[NJ]) {
    const int n = chain_n<NJ>(T);
    double aw[NJ][3], pv[NJ][3];
    bool rev[NJ], act[NJ];
    double R[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0}, p[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        rev[j] = false;
        act[j] = true;
        for (int i = 0; i < 3; ++i) aw[j][i] = pv[j][i] = 0.0;
        if (j >= n) continue;
        const JointDev J = P.joints[j];
        const double a[3] = {J.ax, J.ay, J.az};
        rev[j] = J.type == CP_REVOLUTE;
        act[j] = J.active != 0;
        for (int i = 0; i < 3; ++i) aw[j][i] = R[3 * i] * a[0] + R[3 * i + 1] * a[1] + R[3 * i + 2] * a[2];
        // the joint's origin (moved along its axis if prismatic), then its rotation
        double o[3] = {J.ox, J.oy, J.oz};
        if (J.type == CP_PRISMATIC)
            for (int i = 0; i < 3; ++i) o[i] += q[j] * a[i];
        double np[3];
        for (int i = 0; i < 3; ++i) np[i] = R[3 * i] * o[0] + R[3 * i + 1] * o[1] + R[3 * i + 2] * o[2] + p[i];
        for (int i = 0; i < 3; ++i) p[i] = np[i];
        if (rev[j]) {
            const double sn = sin(q[j]), cs = cos(q[j]), v = 1.0 - cs;
            // rotation by q about the unit axis a (Rodrigues)
            const double Q[9] = {cs + a[0] * a[0] * v,        a[0] * a[1] * v - a[2] * sn, a[0] * a[2] * v + a[1] * sn,
                                 a[1] * a[0] * v + a[2] * sn, cs + a[1] * a[1] * v,        a[1] * a[2] * v - a[0] * sn,
                                 a[2] * a[0] * v - a[1] * sn, a[2] * a[1] * v + a[0] * sn, cs + a[2] * a[2] * v};
            double nr[9];
            for (int i = 0; i < 3; ++i)
                for (int k = 0; k < 3; ++k) nr[3 * i + k] = R[3 * i] * Q[k] + R[3 * i + 1] * Q[3 + k] + R[3 * i + 2] * Q[6 + k];
            for (int i = 0; i < 9; ++i) R[i] = nr[i];
        }
        for (int i = 0; i < 3; ++i) pv[j][i] = p[i];
    }
    const double t[3] = {P.tip[0], P.tip[1], P.tip[2]};
    double tip[3];
    for (int i = 0; i < 3; ++i) tip[i] = R[3 * i] * t[0] + R[3 * i + 1] * t[1] + R[3 * i + 2] * t[2] + p[i];
    // tip Jacobian columns and the rotation arms
    double Jc[NJ][3], arm[NJ][3];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        for (int i = 0; i < 3; ++i) arm[j][i] = tip[i] - pv[j][i];
        if (rev[j]) {
            Jc[j][0] = aw[j][1] * arm[j][2] - aw[j][2] * arm[j][1];
            Jc[j][1] = aw[j][2] * arm[j][0] - aw[j][0] * arm[j][2];
            Jc[j][2] = aw[j][0] * arm[j][1] - aw[j][1] * arm[j][0];
        } else {
            for (int i = 0; i < 3; ++i) Jc[j][i] = aw[j][i];
        }
    }
    // c = sum_ij H_ij qd_i qd_j, H_ij (i <= j, the earlier joint first):
    // revolute j: a_i x (a_j x arm_j) for revolute i, 0 for prismatic i;
    // prismatic j: a_i x a_j for revolute i < j, 0 otherwise (joints past n:
    // prismatic with a zero axis, so they add nothing)
    double c[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
#pragma unroll
        for (int j = i; j < NJ; ++j) {
            double h[3] = {0.0, 0.0, 0.0};
            if (rev[j]) {
                if (rev[i]) {
                    // a_j x arm_j is the column Jc[j]
                    h[0] = aw[i][1] * Jc[j][2] - aw[i][2] * Jc[j][1];
                    h[1] = aw[i][2] * Jc[j][0] - aw[i][0] * Jc[j][2];
                    h[2] = aw[i][0] * Jc[j][1] - aw[i][1] * Jc[j][0];
                }
            } else if (rev[i] && i < j) {
                h[0] = aw[i][1] * aw[j][2] - aw[i][2] * aw[j][1];
                h[1] = aw[i][2] * aw[j][0] - aw[i][0] * aw[j][2];
                h[2] = aw[i][0] * aw[j][1] - aw[i][1] * aw[j][0];
            }
            const double wgt = (i == j ? 1.0 : 2.0) * qd[i] * qd[j];
            for (int k = 0; k < 3; ++k) c[k] += wgt * h[k];
        }
    }
    double acc[3] = {c[0], c[1], c[2] + T.grav};
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        qdd[j] = 0.0;
        if (j < n && act[j]) {
            qdd[j] = uf[j];
            for (int k = 0; k < 3; ++k) acc[k] += Jc[j][k] * qdd[j];
        }
    }
    // passive joints: (J_p^T J_p) x = -J_p^T acc, written as one NJ x NJ
    // system G y = b that is the identity on the other joints (G is then
    // symmetric positive definite: Gaussian elimination without pivoting)
    double G[NJ][NJ], b[NJ];
#pragma unroll
    for (int r = 0; r < NJ; ++r) {
        const bool pr = r < n && !act[r];
#pragma unroll
        for (int s2 = 0; s2 < NJ; ++s2) {
            const bool ps = s2 < n && !act[s2];
            G[r][s2] = (pr && ps) ? Jc[r][0] * Jc[s2][0] + Jc[r][1] * Jc[s2][1] + Jc[r][2] * Jc[s2][2]
                                  : (r == s2 ? 1.0 : 0.0);
        }
        b[r] = pr ? -(Jc[r][0] * acc[0] + Jc[r][1] * acc[1] + Jc[r][2] * acc[2]) : 0.0;
    }
#pragma unroll
    for (int col = 0; col < NJ; ++col) {
#pragma unroll
        for (int r = col + 1; r < NJ; ++r) {
            const double fct = G[r][col] / G[col][col];
            for (int k = col; k < NJ; ++k) G[r][k] -= fct * G[col][k];
            b[r] -= fct * b[col];
        }
    }
    double y[NJ];
#pragma unroll
    for (int r = NJ - 1; r >= 0; --r) {
        double v = b[r];
        for (int k = r + 1; k < NJ; ++k) v -= G[r][k] * y[k];
        y[r] = v / G[r][r];
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        if (j < n && !act[j]) qdd[j] = y[j] - T.damping * qd[j];
}

// ---------------------------------------------------------------------------
// the problem's points
// ---------------------------------------------------------------------------

struct TrajIn {
    const float *qs, *qg, *qstar;  // [n], [n], [N+1][n]
    double t_min, s_min;           // the final-time bound and its root
};

// t_min of the problem: max_j |q_d,j - q_0,j| / v_max,j
__device__ inline double traj_t_min(const TrajDev &T, const float *qs, const float *qg) {
    double t = 0.0;
    for (int j = 0; j < T.n; ++j) t = fmax(t, fabs((double)qg[j] - (double)qs[j]) / T.v_max[j]);
    return t;
}

// x' = f(x, u) = (qd, qdd) of one point into out[2n]
template <int NJ>
__device__ inline void traj_rhs(const PlanView &P, const TrajDev &T, const double (&q)[NJ], const double (&qd)[NJ],
                                const double (&uf)[NJ], double *out) {
    const int n = chain_n<NJ>(T);
    double qdd[NJ];
    crane_accel<NJ>(P, T, q, qd, uf, qdd);
#pragma unroll
    for (int i = 0; i < NJ; ++i)
        if (i < n) {
            out[i] = qd[i];
            out[n + i] = qdd[i];
        }
}

// f at every point (and with jac its central-difference Jacobians): the
// threads share out (point, direction) tasks, a direction's two evaluations
// on one thread; the perturbed coordinate is picked by comparison, never by
// a per-lane index
template <int NJ>
__device__ void eval_points(const PlanView &P, const TrajDev &T, const TrajIn &in, const double *z, double *f,
                            double *Jx, double *Ju, bool jac) {
    const int n = chain_n<NJ>(T), na = T.na, N = T.N, nx = 2 * n;
    const int per = jac ? 1 + nx + na : 1;
    const int total = (N + 1) * per;
    for (int t = threadIdx.x; t < total; t += kTrajThreads) {
        const int k = t / per, e = t % per;
        // state and full-length inputs of point k (x_0, x_N: the fixed rest states)
        const double *b = z + (size_t)k * kMB;
        double q[NJ], qd[NJ], uf[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            q[j] = qd[j] = uf[j] = 0.0;
            if (j >= n) continue;
            if (k == 0) q[j] = in.qs[j];
            else if (k == N) q[j] = in.qg[j];
            else {
                q[j] = b[j];
                qd[j] = b[n + j];
            }
        }
#pragma unroll
        for (int a = 0; a < NJ; ++a) {
            if (a >= na) continue;
            const int ja = T.act[a];
            const double ua = b[2 * n + a];
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                if (j == ja) uf[j] = ua;
        }
        double fp[2 * NJ], fm[2 * NJ];
        if (e == 0) {
            traj_rhs<NJ>(P, T, q, qd, uf, fp);
            for (int i = 0; i < nx; ++i) f[(size_t)k * nx + i] = fp[i];
            continue;
        }
        const int d = e - 1;  // 0..n-1 positions, n..2n-1 velocities, 2n.. inputs
        const double step = d < n ? T.fd_q : 1.0;
        int ju = -1;  // the joint of the perturbed input
#pragma unroll
        for (int a = 0; a < NJ; ++a)
            if (a < na && d == nx + a) ju = T.act[a];
        double q1[NJ], qd1[NJ], u1[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            q1[j] = d == j ? q[j] + step : q[j];
            qd1[j] = d == n + j ? qd[j] + step : qd[j];
            u1[j] = j == ju ? uf[j] + step : uf[j];
        }
        traj_rhs<NJ>(P, T, q1, qd1, u1, fp);
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            q1[j] = d == j ? q[j] - step : q[j];
            qd1[j] = d == n + j ? qd[j] - step : qd[j];
            u1[j] = j == ju ? uf[j] - step : uf[j];
        }
        traj_rhs<NJ>(P, T, q1, qd1, u1, fm);
        if (d < nx) {
            for (int i = 0; i < nx; ++i) Jx[((size_t)k * nx + i) * nx + d] = (fp[i] - fm[i]) / (2.0 * step);
        } else {
            const int j = d - nx;
            for (int i = 0; i < nx; ++i) Ju[((size_t)k * nx + i) * na + j] = (fp[i] - fm[i]) / 2.0;
        }
    }
}

// block reductions over the workgroup (fixed order: thread partials, then
// a serial sum over the threads' slots)
struct TrajShared {
    double red[kTrajThreads];
    double A[kMB][kMB + 1];     // the block being factored
    double X[kMB][kMB + 1];     // L^-1 E of the previous block
    double v[2][kMB];           // v[0]: 1 / L_jj of the block being factored
};

__device__ double block_sum(TrajShared &sh, double v) {
    sh.red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kTrajThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh.red[threadIdx.x] += sh.red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh.red[0];
    __syncthreads();
    return r;
}

__device__ double block_max(TrajShared &sh, double v) {
    sh.red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kTrajThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh.red[threadIdx.x] = fmax(sh.red[threadIdx.x], sh.red[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = sh.red[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// residual pieces
// ---------------------------------------------------------------------------

// the scaled residual of defect k (row i): sqrt(mu) (d_k + lam_k / mu) with
// d_k = x_{k+1} - x_k - h/2 (f_k + f_{k+1}); and the raw defect
__device__ inline double defect_row(const TrajDev &T, const TrajIn &in, const double *z, const double *f,
                                    const double *lam, double mu, int k, int i, double *raw) {
    const int n = T.n, nx = 2 * n;
    const double s = z[(size_t)(T.N + 1) * kMB];
    const double h2 = s * s / (2.0 * T.N);
    double xa, xb;
    // state entry i of points k and k + 1
    auto st = [&](int kk) {
        if (kk == 0) return i < n ? (double)in.qs[i] : 0.0;
        if (kk == T.N) return i < n ? (double)in.qg[i] : 0.0;
        return z[(size_t)kk * kMB + i];
    };
    xa = st(k);
    xb = st(k + 1);
    const double d = xb - xa - h2 * (f[(size_t)k * nx + i] + f[(size_t)(k + 1) * nx + i]);
    if (raw) *raw = d;
    return sqrt(mu) * (d + lam[(size_t)k * nx + i] / mu);
}

// F = |r|^2 / 2 at z (f evaluated at z)
__device__ double objective(const PlanView &P, const TrajDev &T, const TrajIn &in, const double *z, const double *f,
                            const double *lam, double mu, TrajShared &sh) {
    const int n = T.n, na = T.na, N = T.N, nx = 2 * n;
    double acc = 0.0;
    // defects
    for (int t = threadIdx.x; t < N * nx; t += kTrajThreads) {
        const double r = defect_row(T, in, z, f, lam, mu, t / nx, t % nx, nullptr);
        acc += r * r;
    }
    // bounds of the interior states
    for (int t = threadIdx.x; t < (N - 1) * nx; t += kTrajThreads) {
        const int k = 1 + t / nx, i = t % nx;
        const double x = z[(size_t)k * kMB + i];
        const double lo = i < n ? (double)P.joints[i].qmin : -T.v_max[i - n];
        const double hi = i < n ? (double)P.joints[i].qmax : T.v_max[i - n];
        const double e = fmax(x - hi, 0.0) + fmax(lo - x, 0.0);
        acc += mu * e * e;
    }
    // inputs and tracking, k = 1..N
    for (int t = threadIdx.x; t < N * na; t += kTrajThreads) {
        const int k = 1 + t / na, j = t % na, a = T.act[j];
        const double u = z[(size_t)k * kMB + nx + j];
        const double qa = k == N ? (double)in.qg[a] : z[(size_t)k * kMB + a];
        const double dq = qa - (double)in.qstar[(size_t)k * n + a];
        acc += T.omega_s * u * u + T.omega_t * dq * dq;
    }
    const double s = z[(size_t)(N + 1) * kMB], lo = fmax(in.s_min - s, 0.0);
    const double tot = block_sum(sh, acc);
    return 0.5 * (tot + s * s + mu * lo * lo);
}

// ---------------------------------------------------------------------------
// normal equations J^T J (blocks D_k, E_k, column c, corner a_ss) and
// gradient g = J^T r at z
// ---------------------------------------------------------------------------

// entry (r, c) of -h/2 [Jx_k | Ju_k], 0 for the fixed states of the end
// points and the padding (the defect Jacobians are sqrt(mu) times this block
// minus or plus the identity on the free states)
__device__ inline double bentry(const TrajDev &T, const double *Jx, const double *Ju, double h2, int kk, int r, int c) {
    const int nx = 2 * T.n, na = T.na;
    if (r >= nx || c >= nx + na || ((kk == 0 || kk == T.N) && c < nx)) return 0.0;
    return c < nx ? -h2 * Jx[((size_t)kk * nx + r) * nx + c] : -h2 * Ju[((size_t)kk * nx + r) * na + (c - nx)];
}

// rr, js: scratch vectors of (N+1) MB entries (the defects' scaled residuals
// and their column for s, filled here)
__device__ void normal_equations(const PlanView &P, const TrajDev &T, const TrajIn &in, const double *z,
                                 const double *f, const double *Jx, const double *Ju, const double *lam, double mu,
                                 double *D, double *E, double *c, double *g, double &a_ss, double *rr, double *js,
                                 TrajShared &sh) {
    const int n = T.n, na = T.na, N = T.N, nx = 2 * n, MB = kMB;
    const double s = z[(size_t)(N + 1) * MB];
    const double h2 = s * s / (2.0 * N), sm = sqrt(mu);
    // the defects' scaled residuals and s-columns, once each
    for (int t = threadIdx.x; t < N * nx; t += kTrajThreads) {
        const int k = t / nx, r = t % nx;
        rr[(size_t)k * MB + r] = defect_row(T, in, z, f, lam, mu, k, r, nullptr);
        js[(size_t)k * MB + r] = -sm * (s / N) * (f[(size_t)k * nx + r] + f[(size_t)(k + 1) * nx + r]);
    }
    __syncthreads();
    const int ti = threadIdx.x / MB, tj = threadIdx.x % MB;
    // Point k's block B_k and the rows of defect k pass through LDS one step
    // ahead of their use: the block in the factorisation's two buffers (row r,
    // column c at [r][c], thread (r, c) loads it), the defect rows in a ring of
    // three slots of the reduction array (rr then js), both free here.
    double(*const buf[2])[kMB + 1] = {sh.A, sh.X};
    double *const ring = sh.red;
    buf[0][ti][tj] = bentry(T, Jx, Ju, h2, 0, ti, tj);
    double nxt = bentry(T, Jx, Ju, h2, 1, ti, tj);
    double nrr = 0.0, njs = 0.0;
    if ((int)threadIdx.x < MB) {
        ring[threadIdx.x] = rr[threadIdx.x];
        ring[MB + threadIdx.x] = js[threadIdx.x];
        nrr = rr[(size_t)MB + threadIdx.x];
        njs = js[(size_t)MB + threadIdx.x];
    }
    // bounds and tracking of entries ti and tj (point independent); their
    // entries of z and of the path, one point ahead
    auto lo_of = [&](int e) { return e < n ? (double)P.joints[e].qmin : e < nx ? -T.v_max[e - n] : 0.0; };
    auto hi_of = [&](int e) { return e < n ? (double)P.joints[e].qmax : e < nx ? T.v_max[e - n] : 0.0; };
    const double lo_i = lo_of(ti), hi_i = hi_of(ti), lo_j = lo_of(tj), hi_j = hi_of(tj);
    bool track_i = false, track_j = false;
    for (int j = 0; j < na; ++j) {
        track_i = track_i || T.act[j] == ti;
        track_j = track_j || T.act[j] == tj;
    }
    double zi = z[ti], zj = z[tj], qj = tj < n ? (double)in.qstar[tj] : 0.0;
    for (int k = 0; k <= N; ++k) {
        const bool fixed = k == 0 || k == N;
        const double zi_k = zi, zj_k = zj, qj_k = qj;
        if (k + 1 <= N) {
            zi = z[(size_t)(k + 1) * MB + ti];
            zj = z[(size_t)(k + 1) * MB + tj];
            qj = tj < n ? (double)in.qstar[(size_t)(k + 1) * n + tj] : 0.0;
        }
        if (k + 1 <= N) buf[(k + 1) & 1][ti][tj] = nxt;
        nxt = k + 2 <= N ? bentry(T, Jx, Ju, h2, k + 2, ti, tj) : 0.0;
        if ((int)threadIdx.x < MB) {
            if (k + 1 < N) {
                double *sl = ring + ((k + 1) % 3) * 2 * MB;
                sl[threadIdx.x] = nrr;
                sl[MB + threadIdx.x] = njs;
            }
            if (k + 2 < N) {
                nrr = rr[(size_t)(k + 2) * MB + threadIdx.x];
                njs = js[(size_t)(k + 2) * MB + threadIdx.x];
            }
        }
        __syncthreads();
        const double(*Bk)[kMB + 1] = buf[k & 1];
        const double(*Bn)[kMB + 1] = buf[(k + 1) & 1];
        const double *dk = ring + (k % 3) * 2 * MB;             // defect k (k < N)
        const double *dp = ring + ((k + 2) % 3) * 2 * MB;       // defect k - 1 (k > 0)
        // columns ti, tj of point k's block and column tj of point k + 1's are read
        // from LDS row by row below
        // identity parts: free state columns of point k (both defects) and k + 1
        const bool free_i = ti < nx && !fixed, free_j = tj < nx && !fixed;
        const bool free_n = tj < nx && k + 1 != N;
        // D_k (ti, tj) and E_k (ti, tj): defect k (left block L_k = sqrt(mu) (B_k - I)), defect
        // k - 1 (right block R_{k-1} = sqrt(mu) (B_k + I)), E_k = L_k^T R_k
        double dsum = 0.0, esum = 0.0;
        for (int r = 0; r < nx; ++r) {
            const double bi = Bk[r][ti], bj = Bk[r][tj];
            if (k < N) {
                const double l_i = sm * (bi + (free_i && r == ti ? -1.0 : 0.0));
                const double l_j = sm * (bj + (free_j && r == tj ? -1.0 : 0.0));
                dsum += l_i * l_j;
                esum += l_i * (sm * (Bn[r][tj] + (free_n && r == tj ? 1.0 : 0.0)));
            }
            if (k > 0) {
                const double r_i = sm * (bi + (free_i && r == ti ? 1.0 : 0.0));
                const double r_j = sm * (bj + (free_j && r == tj ? 1.0 : 0.0));
                dsum += r_i * r_j;
            }
        }
        // diagonal terms: bounds (active ones), inputs, tracking; fixed states: identity
        if (ti == tj) {
            if (fixed && ti < nx) {
                dsum = 1.0;
            } else if (ti < nx) {
                const double x = zi_k;
                if (x > hi_i || x < lo_i) dsum += mu;
                if (track_i && k < N) dsum += T.omega_t;
            } else if (ti < nx + na) {
                if (k >= 1) dsum += T.omega_s;
            } else {
                dsum = 1.0;  // padding
            }
        }
        if (fixed && ti < nx && ti != tj) dsum = 0.0;
        if (fixed && tj < nx && ti != tj) dsum = 0.0;
        if (ti >= nx + na || tj >= nx + na) dsum = ti == tj ? 1.0 : 0.0;
        D[(size_t)k * MB * MB + ti * MB + tj] = dsum;
        if (k < N) E[(size_t)k * MB * MB + ti * MB + tj] = esum;
        // c_k on the second wave (ti = 4), g_k on the third (ti = 8): one entry per thread,
        // column col = tj of B_k, so that no wave carries both beside its D and E entries
        if (ti == 4 || ti == 8) {
            const int col = tj;
            const bool is_c = ti == 4;
            const int off = is_c ? MB : 0;  // js or rr within a defect's slot
            double sum = 0.0;
            for (int r = 0; r < nx; ++r) {
                const double bj = Bk[r][tj];
                if (k < N) sum += sm * (bj + (free_j && r == col ? -1.0 : 0.0)) * dk[off + r];
                if (k > 0) sum += sm * (bj + (free_j && r == col ? 1.0 : 0.0)) * dp[off + r];
            }
            if (!(fixed && col < nx) && col < nx + na) {
                if (!is_c) {
                    if (col < nx) {
                        const double x = zj_k;
                        if (x > hi_j) sum += mu * (x - hi_j);
                        if (x < lo_j) sum -= mu * (lo_j - x);
                        if (track_j && k < N) sum += T.omega_t * (x - qj_k);
                    } else if (k >= 1) {
                        sum += T.omega_s * zj_k;
                    }
                }
            } else {
                sum = 0.0;
            }
            (is_c ? c : g)[(size_t)k * MB + col] = sum;
        }
        __syncthreads();
    }
    // corner and g_s: sums over the defect rows, plus the final-time bound
    double gs_part = 0.0, ass_part = 0.0;
    for (int t = threadIdx.x; t < N * nx; t += kTrajThreads) {
        const int k = t / nx, r = t % nx;
        const double jsv = js[(size_t)k * MB + r];
        ass_part += jsv * jsv;
        gs_part += jsv * rr[(size_t)k * MB + r];
    }
    const bool below = s < in.s_min;
    a_ss = block_sum(sh, ass_part) + 1.0 + (below ? mu : 0.0);
    const double gs = block_sum(sh, gs_part) + s + (below ? mu * (s - in.s_min) : 0.0);
    if (threadIdx.x == 0) {
        g[(size_t)(N + 1) * MB] = gs;
        c[(size_t)(N + 1) * MB] = a_ss;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// (A + damp I) h = -g: block Cholesky sweep and the Schur complement on s
// ---------------------------------------------------------------------------

// the value v holds in lane `lane` of this wave (lane: a wave-uniform index)
__device__ inline double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Cholesky of sh.A in place (lower), right-looking, on lanes 0..2 MB - 1 of
// the first wave: lane i holds row i mod MB in registers and the columns pass
// between lanes by lane reads from the first half-wave (the second repeats the
// computation, the first writes the factor back); no workgroup barrier inside
__device__ void chol_rows(TrajShared &sh) {
    const int i = threadIdx.x % kMB;
    double a[kMB];
#pragma unroll
    for (int m = 0; m < kMB; ++m) a[m] = sh.A[i][m];
#pragma unroll
    for (int j = 0; j < kMB; ++j) {
        // column j: L_jj = a_jj / sqrt(a_jj), L_ij = a_ij / sqrt(a_jj); 1 / L_jj kept for the
        // substitutions
        const double rp = rsqrt(lane_value(a[j], j));
        if (i >= j) a[j] *= rp;
        if (i == j && (int)threadIdx.x < kMB) sh.v[0][j] = rp;
#pragma unroll
        for (int m = j + 1; m < kMB; ++m) {
            const double lmj = lane_value(a[j], m);
            if (i >= m) a[m] -= a[j] * lmj;
        }
    }
    if ((int)threadIdx.x < kMB)
#pragma unroll
        for (int m = 0; m < kMB; ++m) sh.A[i][m] = a[m];
}

__device__ void factor(const double *D, const double *E, double damp, double *LD, double *LX,
                       int N, TrajShared &sh) {
    const int MB = kMB;
    const int ti = threadIdx.x / MB, tj = threadIdx.x % MB;
    double dcur = D[ti * MB + tj];
    for (int k = 0; k <= N; ++k) {
        double a = dcur;
        if (ti == tj) a += damp;
        if (k > 0) {
            // minus X_{k-1}^T X_{k-1}, X_{k-1} = L_{k-1}^-1 E_{k-1} (in sh.X)
            double s = 0.0;
            for (int m = 0; m < MB; ++m) s += sh.X[m][ti] * sh.X[m][tj];
            a -= s;
        }
        // E_k's entry and the next block's D: their loads run under the factorisation
        const double ek = k < N ? E[(size_t)k * MB * MB + ti * MB + tj] : 0.0;
        if (k < N) dcur = D[(size_t)(k + 1) * MB * MB + ti * MB + tj];
        __syncthreads();
        sh.A[ti][tj] = a;
        sh.X[ti][tj] = ek;
        __syncthreads();
        if ((int)threadIdx.x < 2 * MB) chol_rows(sh);
        __syncthreads();
        LD[(size_t)k * MB * MB + ti * MB + tj] = tj <= ti ? sh.A[ti][tj] : 0.0;
        if (k < N) {
            // X_k = L_k^-1 E_k: forward substitution, one column per thread, in place in
            // sh.X, column by column of L (each solved entry updates the rows below it, so
            // the updates of one step are independent)
            if ((int)threadIdx.x < MB) {
                const int col = threadIdx.x;
                double x[kMB];
#pragma unroll
                for (int i = 0; i < kMB; ++i) x[i] = sh.X[i][col];
#pragma unroll
                for (int m = 0; m < kMB; ++m) {
                    x[m] *= sh.v[0][m];
#pragma unroll
                    for (int i = m + 1; i < kMB; ++i) x[i] -= sh.A[i][m] * x[m];
                }
#pragma unroll
                for (int i = 0; i < kMB; ++i) sh.X[i][col] = x[i];
            }
            __syncthreads();
            LX[(size_t)k * MB * MB + ti * MB + tj] = sh.X[ti][tj];
        }
        __syncthreads();
    }
}

// solve L L^T x = b for two right-hand sides b0, b1 (length (N+1) MB), x in
// place, on lanes 0..2 MB - 1 of the first wave (lane which * MB + i holds
// entry i of right-hand side `which`; a block's unknowns pass between lanes
// by lane reads); no workgroup barrier inside, the caller synchronises
// entry m of this lane's right-hand side: lane m or MB + m
__device__ inline double of_rhs(double v, int m, int which) {
    const double v0 = lane_value(v, m), v1 = lane_value(v, kMB + m);
    return which ? v1 : v0;
}

__device__ void solve2(const double *LD, const double *LX, double *b0, double *b1, int N) {
    const int MB = kMB;
    if ((int)threadIdx.x >= 2 * MB) return;
    const int which = threadIdx.x / MB, i = threadIdx.x % MB;
    double *b = which ? b1 : b0;
    // forward: y_k = L_k^-1 (b_k - X_{k-1}^T y_{k-1})
    double prev = 0.0;
    for (int k = 0; k <= N; ++k) {
        const double *Lk = LD + (size_t)k * MB * MB;
        double row[kMB];  // row i of L_k
        for (int m = 0; m < kMB; ++m) row[m] = Lk[i * MB + m];
        const double rinv = 1.0 / Lk[i * MB + i];
        double v = b[(size_t)k * MB + i];
        if (k > 0) {
            const double *Xp = LX + (size_t)(k - 1) * MB * MB;
            double col[kMB];  // column i of X_{k-1}
            for (int m = 0; m < kMB; ++m) col[m] = Xp[m * MB + i];
#pragma unroll
            for (int m = 0; m < kMB; ++m) v -= col[m] * of_rhs(prev, m, which);
        }
#pragma unroll
        for (int j = 0; j < kMB; ++j) {
            const double xj = of_rhs(v * rinv, j, which);
            if (i > j) v -= row[j] * xj;
        }
        prev = v * rinv;
        b[(size_t)k * MB + i] = prev;
    }
    // backward: x_k = L_k^-T (y_k - X_k x_{k+1})
    for (int k = N; k >= 0; --k) {
        const double *Lk = LD + (size_t)k * MB * MB;
        double col[kMB];  // column i of L_k
        for (int m = 0; m < kMB; ++m) col[m] = Lk[m * MB + i];
        const double rinv = 1.0 / Lk[i * MB + i];
        double v = b[(size_t)k * MB + i];
        if (k < N) {
            const double *Xk = LX + (size_t)k * MB * MB;
            double row[kMB];  // row i of X_k
            for (int m = 0; m < kMB; ++m) row[m] = Xk[i * MB + m];
#pragma unroll
            for (int m = 0; m < kMB; ++m) v -= row[m] * of_rhs(prev, m, which);
        }
#pragma unroll
        for (int j = kMB - 1; j >= 0; --j) {
            const double xj = of_rhs(v * rinv, j, which);
            if (i < j) v -= col[j] * xj;
        }
        prev = v * rinv;
        b[(size_t)k * MB + i] = prev;
    }
}

// h = -(A + damp I)^-1 g with the s entry last
__device__ void damped_step(const TrajDev &T, const TrajWork &W, double a_ss, double damp, TrajShared &sh) {
    const int N = T.N;
    const size_t nb = (size_t)(N + 1) * kMB;
    factor(W.D, W.E, damp, W.LD, W.LX, N, sh);
    for (size_t t = threadIdx.x; t < nb; t += kTrajThreads) {
        W.y[t] = -W.g[t];
        W.w[t] = W.c[t];
    }
    __syncthreads();
    solve2(W.LD, W.LX, W.y, W.w, N);
    __syncthreads();
    double p0 = 0.0, p1 = 0.0;
    for (size_t t = threadIdx.x; t < nb; t += kTrajThreads) {
        p0 += W.c[t] * W.y[t];
        p1 += W.c[t] * W.w[t];
    }
    const double cy = block_sum(sh, p0), cw = block_sum(sh, p1);
    const double hs = (-W.g[nb] - cy) / (a_ss + damp - cw);
    for (size_t t = threadIdx.x; t < nb; t += kTrajThreads) W.h[t] = W.y[t] - W.w[t] * hs;
    if (threadIdx.x == 0) W.h[nb] = hs;
    __syncthreads();
}

// h . (A h) with A the undamped normal matrix
__device__ double quad_form(const TrajDev &T, const TrajWork &W, double a_ss, TrajShared &sh) {
    const int N = T.N, MB = kMB;
    const size_t nb = (size_t)(N + 1) * MB;
    double acc = 0.0;
    for (size_t t = threadIdx.x; t < nb; t += kTrajThreads) {
        const int k = (int)(t / MB), i = (int)(t % MB);
        double v = 0.0;
        for (int m = 0; m < MB; ++m) v += W.D[(size_t)k * MB * MB + i * MB + m] * W.h[(size_t)k * MB + m];
        if (k < N)
            for (int m = 0; m < MB; ++m) v += W.E[(size_t)k * MB * MB + i * MB + m] * W.h[(size_t)(k + 1) * MB + m];
        if (k > 0)
            for (int m = 0; m < MB; ++m) v += W.E[(size_t)(k - 1) * MB * MB + m * MB + i] * W.h[(size_t)(k - 1) * MB + m];
        v += W.c[t] * W.h[nb];
        acc += W.h[t] * v;
        acc += W.h[nb] * W.c[t] * W.h[t];
    }
    const double tot = block_sum(sh, acc);
    return tot + W.h[nb] * a_ss * W.h[nb];
}

// the starting point: the path's points at times k t_0 / N, velocities and
// inputs from their differences, s = sqrt(t_0), t_0 = max(t_f0, t_min)
__device__ void init_point(const TrajDev &T, const TrajIn &in, double *z) {
    const int n = T.n, na = T.na, N = T.N, nx = 2 * n, MB = kMB;
    const double t0 = fmax(T.t_f0, in.t_min), h = t0 / N;
    auto qpt = [&](int k, int i) {
        if (k <= 0) return (double)in.qs[i];
        if (k >= N) return (double)in.qg[i];
        return (double)in.qstar[(size_t)k * n + i];
    };
    auto vel = [&](int k, int i) { return (k <= 0 || k >= N) ? 0.0 : (qpt(k + 1, i) - qpt(k - 1, i)) / (2.0 * h); };
    for (size_t t = threadIdx.x; t < (size_t)(N + 1) * MB; t += kTrajThreads) {
        const int k = (int)(t / MB), i = (int)(t % MB);
        double v = 0.0;
        if (i < n) v = (k == 0 || k == N) ? qpt(k, i) : qpt(k, i);
        else if (i < nx) v = vel(k, i - n);
        else if (i < nx + na) v = k < N ? (vel(k + 1, T.act[i - nx]) - vel(k, T.act[i - nx])) / h : 0.0;
        z[t] = v;
    }
    if (threadIdx.x == 0) z[(size_t)(N + 1) * MB] = sqrt(t0);
    __syncthreads();
}

// is entry t of z an unknown (not a fixed state, not padding)?
__device__ inline bool real_entry(const TrajDev &T, size_t t) {
    const int k = (int)(t / kMB), i = (int)(t % kMB);
    if (k > T.N) return true;  // s
    if (i >= 2 * T.n + T.na) return false;
    return !((k == 0 || k == T.N) && i < 2 * T.n);
}

template <int NJ>
__global__ __launch_bounds__(kTrajThreads) void k_traj_refine(PlanView P, TrajDev T, const float *__restrict__ qs,
                                                              const float *__restrict__ qg,
                                                              const float *__restrict__ qstar, double *work,
                                                              size_t stride, float *__restrict__ x_out,
                                                              float *__restrict__ u_out, float *__restrict__ tf_out,
                                                              float *__restrict__ info_out) {
    __shared__ TrajShared sh;
    const int pr = blockIdx.x;
    const int n = T.n, na = T.na, N = T.N, nx = 2 * n, MB = kMB;
    const float *q0 = qs + (size_t)pr * n, *q1 = qg + (size_t)pr * n;
    const double t_min = traj_t_min(T, q0, q1);
    const TrajIn in{q0, q1, qstar + (size_t)pr * (N + 1) * n, t_min, sqrt(t_min)};
    const TrajWork W = traj_work(work + (size_t)pr * stride, N, n, na);
    const size_t nb = (size_t)(N + 1) * MB, nz = nb + 1;
    init_point(T, in, W.z);
    for (size_t t = threadIdx.x; t < (size_t)N * nx; t += kTrajThreads) W.lam[t] = 0.0;
    __syncthreads();
    double mu = T.mu0, F = 0.0, a_ss = 0.0;
    int iters = 0, accepted = 0;
    for (int outer = 0; outer < T.outer; ++outer) {
        eval_points<NJ>(P, T, in, W.z, W.f, W.Jx, W.Ju, true);
        __syncthreads();
        F = objective(P, T, in, W.z, W.f, W.lam, mu, sh);
        normal_equations(P, T, in, W.z, W.f, W.Jx, W.Ju, W.lam, mu, W.D, W.E, W.c, W.g, a_ss, W.y, W.w, sh);
        // initial damping: tau times the largest diagonal entry over the unknowns
        double dm = 0.0;
        for (size_t t = threadIdx.x; t < nb; t += kTrajThreads)
            if (real_entry(T, t)) dm = fmax(dm, W.D[(t / MB) * MB * MB + (t % MB) * MB + (t % MB)]);
        double damp = T.tau * fmax(block_max(sh, dm), a_ss);
        double nu = 2.0;
        int it = 0;
        while (it < T.max_iters) {
            double gm = 0.0;
            for (size_t t = threadIdx.x; t < nz; t += kTrajThreads) gm = fmax(gm, fabs(W.g[t]));
            if (block_max(sh, gm) <= T.eps_grad) break;
            damped_step(T, W, a_ss, damp, sh);
            double hh = 0.0, zz = 0.0;
            for (size_t t = threadIdx.x; t < nz; t += kTrajThreads)
                if (real_entry(T, t)) {
                    hh += W.h[t] * W.h[t];
                    zz += W.z[t] * W.z[t];
                }
            const double hn = sqrt(block_sum(sh, hh)), zn = sqrt(block_sum(sh, zz));
            if (!(hn > T.eps_step * (zn + T.eps_step))) break;
            for (size_t t = threadIdx.x; t < nz; t += kTrajThreads) W.zt[t] = W.z[t] + W.h[t];
            __syncthreads();
            eval_points<NJ>(P, T, in, W.zt, W.ft, W.Jx, W.Ju, false);
            __syncthreads();
            const double Ft = objective(P, T, in, W.zt, W.ft, W.lam, mu, sh);
            double hg = 0.0;
            for (size_t t = threadIdx.x; t < nz; t += kTrajThreads) hg += W.h[t] * W.g[t];
            const double pred = -block_sum(sh, hg) - 0.5 * quad_form(T, W, a_ss, sh);
            ++it;
            if (pred > 0.0 && F - Ft > 0.0) {
                const double rho = (F - Ft) / pred, tt = 2.0 * rho - 1.0;
                ++accepted;
                for (size_t t = threadIdx.x; t < nz; t += kTrajThreads) W.z[t] = W.zt[t];
                __syncthreads();
                F = Ft;
                eval_points<NJ>(P, T, in, W.z, W.f, W.Jx, W.Ju, true);
                __syncthreads();
                normal_equations(P, T, in, W.z, W.f, W.Jx, W.Ju, W.lam, mu, W.D, W.E, W.c, W.g, a_ss, W.y, W.w, sh);
                damp *= fmax(1.0 / 3.0, 1.0 - tt * tt * tt);
                nu = 2.0;
            } else {
                damp *= nu;
                nu *= 2.0;
            }
        }
        iters += it;
        // multipliers from the defects at z: lam += mu d
        for (size_t t = threadIdx.x; t < (size_t)N * nx; t += kTrajThreads) {
            double d;
            defect_row(T, in, W.z, W.f, W.lam, mu, (int)(t / nx), (int)(t % nx), &d);
            W.lam[t] += mu * d;
        }
        __syncthreads();
        mu *= T.mu_factor;
    }
    // outputs
    double dmax = 0.0;
    for (size_t t = threadIdx.x; t < (size_t)N * nx; t += kTrajThreads) {
        double d;
        defect_row(T, in, W.z, W.f, W.lam, 1.0, (int)(t / nx), (int)(t % nx), &d);
        dmax = fmax(dmax, fabs(d));
    }
    dmax = block_max(sh, dmax);
    for (size_t t = threadIdx.x; t < (size_t)(N + 1) * nx; t += kTrajThreads) {
        const int k = (int)(t / nx), i = (int)(t % nx);
        double v;
        if (k == 0 || k == N) v = i < n ? (double)(k == 0 ? in.qs[i] : in.qg[i]) : 0.0;
        else v = W.z[(size_t)k * MB + i];
        x_out[(size_t)pr * (N + 1) * nx + t] = (float)v;
    }
    for (size_t t = threadIdx.x; t < (size_t)(N + 1) * na; t += kTrajThreads) {
        const int k = (int)(t / na), j = (int)(t % na);
        u_out[(size_t)pr * (N + 1) * na + t] = (float)W.z[(size_t)k * MB + nx + j];
    }
    if (threadIdx.x == 0) {
        const double sv = W.z[nb];
        tf_out[pr] = (float)(sv * sv);
        if (info_out) {
            float *o = info_out + (size_t)pr * 4;
            o[0] = (float)dmax; o[1] = (float)F; o[2] = (float)iters; o[3] = (float)accepted;
        }
    }
}

}  // namespace

size_t traj_workspace_bytes(int N, int n, int na, int P) {
    return traj_work_doubles(N, n, na) * sizeof(double) * (size_t)P;
}

hipError_t launch_traj_refine(const PlanView &P, const cp_traj_params &prm, const int *act, int n_act,
                              const float *q_start, const float *q_goal, const float *q_star, int n_prob, void *work,
                              float *x_out, float *u_out, float *tf_out, float *info_out, hipStream_t st) {
    TrajDev T{};
    T.N = prm.N;
    T.n = P.n_joints;
    T.na = n_act;
    for (int j = 0; j < CP_MAX_JOINTS; ++j) T.act[j] = j < n_act ? act[j] : 0;
    T.outer = prm.outer;
    T.max_iters = prm.max_iters;
    T.omega_s = prm.omega_s; T.omega_t = prm.omega_t; T.grav = prm.grav; T.damping = prm.damping;
    T.mu0 = prm.mu0; T.mu_factor = prm.mu_factor; T.tau = prm.tau; T.eps_grad = prm.eps_grad;
    T.eps_step = prm.eps_step; T.fd_q = prm.fd_q; T.t_f0 = prm.t_f0;
    for (int j = 0; j < CP_MAX_JOINTS; ++j) T.v_max[j] = j < T.n ? prm.v_max[j] : 0.0;
    const size_t stride = traj_work_doubles(T.N, T.n, T.na);
    if (T.n == 6)
        hipLaunchKernelGGL(k_traj_refine<6>, dim3(n_prob), dim3(kTrajThreads), 0, st, P, T, q_start, q_goal, q_star,
                           static_cast<double *>(work), stride, x_out, u_out, tf_out, info_out);
    else
        hipLaunchKernelGGL(k_traj_refine<CP_MAX_JOINTS>, dim3(n_prob), dim3(kTrajThreads), 0, st, P, T, q_start,
                           q_goal, q_star, static_cast<double *>(work), stride, x_out, u_out, tf_out, info_out);
    return hipGetLastError();
}

}  // namespace cp
