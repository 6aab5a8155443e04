"""Plain CPU oracle of the crane path optimizer (FP64).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product path (the HIP library and its
binding) never imports this package, and this package imports nothing of the
product except the seeded input generator.

The heavy loops (kinematics, distances, spline, cost, gradient, Philox, EDT,
the IK residual and its Jacobian, the reduced crane dynamics) are in
``oracle.c``; the optimizer of Algorithm 1 (sampling, selection, log-rank
weights, mean and covariance update), the Levenberg-Marquardt loop of the
collision-free IK (Sec. 3.2) and step two's collocation problem and solver
(Sec. 4.2) are written out here with numpy, step by step.

Readings of the paper taken here (each is also listed in the design notes):
* the spline keeps the paper's four copies of the start and goal control
  points on a uniform knot vector and runs over its K+3 non-constant spans;
* the collision term uses the scalar d(q), the minimum over every sphere and
  obstacle pair; sums over checkpoints run over k = 1..n_s;
* the sampling distribution is N(mu, C) with sigma folded into C
  (C_0 = sigma0^2 I), sampled through the lower Cholesky factor;
* the covariance update uses the freshly updated mean;
* elites are the first nu of the stable order on (cost, index), NaN ranked
  as +inf (a NaN and a +inf then go by index);
* step two: a unit load at the tip on massless links stands for the crane's
  mass model (passive rows of Sec. 2.1's state-space form with M = J^T J,
  b = J^T (c + g e_z)), viscous damping on the passive joints, R = I,
  defects over k = 0..N-1, the final-time bound t_F >= t_min that the
  velocity limits imply, and an augmented-Lagrangian Levenberg-Marquardt
  solver in place of IPOPT.

Parity status: every function here is pinned by a CPU test (closed forms,
invariants, brute force, finite differences, published Philox vectors, scipy's
rotation maps, MINPACK's Levenberg-Marquardt, exact box distances from a
bound-constrained least-squares solve, the pendulum frequency, energy
conservation, an exact KKT optimum and SLSQP) except two chaotic iterations, which
are "parity unpinned": multi-iteration optimizer trajectories beyond one step
(one-step parity and convergence properties are checked), and IK trajectories
that cross the collision term, where a switch of the minimising pair changes
the rest of the solve (the residual, its Jacobian, single solves that stay
clear of collision and the validity of every row are checked).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Robot(ctypes.Structure):
    _fields_ = [("n_joints", ctypes.c_int32), ("type", ctypes.c_void_p), ("axis", ctypes.c_void_p),
                ("origin", ctypes.c_void_p), ("q_min", ctypes.c_void_p), ("q_max", ctypes.c_void_p),
                ("q_hold", ctypes.c_void_p), ("active", ctypes.c_void_p), ("n_spheres", ctypes.c_int32),
                ("sphere_frame", ctypes.c_void_p), ("sphere_center", ctypes.c_void_p),
                ("sphere_radius", ctypes.c_void_p), ("tip", ctypes.c_void_p), ("n_self", ctypes.c_int32),
                ("self_pairs", ctypes.c_void_p), ("n_hulls", ctypes.c_int32), ("hull_frame", ctypes.c_void_p),
                ("hull_box", ctypes.c_void_p)]


class _Scene(ctypes.Structure):
    _fields_ = [("has_ground", ctypes.c_int32), ("ground_z", ctypes.c_float), ("n_cyl", ctypes.c_int32),
                ("cyl", ctypes.c_void_p), ("n_box", ctypes.c_int32), ("box", ctypes.c_void_p),
                ("sdf", ctypes.c_void_p), ("sdf_dims", ctypes.c_int32 * 3),
                ("sdf_origin", ctypes.c_float * 3), ("voxel", ctypes.c_float), ("narrow", ctypes.c_int32),
                ("n_obb", ctypes.c_int32), ("obb", ctypes.c_void_p)]


class _Cost(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("M", ctypes.c_int32), ("interp", ctypes.c_int32),
                ("jp_mode", ctypes.c_int32), ("hinge", ctypes.c_int32), ("margin", ctypes.c_float),
                ("lambda_c", ctypes.c_float), ("w_c", ctypes.c_float), ("w_l", ctypes.c_float)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.orc_fk.argtypes = [vp, vp, vp, vp, vp]
        L.orc_sd_cylinder.argtypes = [vp, vp, vp]
        L.orc_sd_cylinder.restype = ctypes.c_double
        L.orc_sd_box.argtypes = [vp, vp, vp]
        L.orc_sd_box.restype = ctypes.c_double
        L.orc_sdf_query.argtypes = [vp, vp, vp]
        L.orc_sdf_query.restype = ctypes.c_double
        L.orc_config_distance.argtypes = [vp, vp, vp, vp, vp, vp]
        L.orc_config_distance.restype = ctypes.c_double
        L.orc_n_checkpoints.argtypes = [vp]
        L.orc_n_checkpoints.restype = ctypes.c_int
        L.orc_path_points.argtypes = [vp, vp, vp, vp, vp, vp]
        L.orc_eval_paths.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp]
        L.orc_grad_paths.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp, vp]
        L.orc_eval_configs.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, i64, i32, vp]
        L.orc_occupancy.argtypes = [vp, i64, vp, vp, ctypes.c_float, vp]
        L.orc_edt_brute.argtypes = [vp, ctypes.c_uint8, vp, vp]
        L.orc_edt_separable.argtypes = [vp, ctypes.c_uint8, vp, vp]
        L.orc_sdf_from_edt.argtypes = [vp, vp, vp, ctypes.c_size_t, ctypes.c_float, vp]
        L.orc_sat_obb_f.argtypes = [vp, vp]
        L.orc_sat_obb_f.restype = ctypes.c_double
        L.orc_hulls_world.argtypes = [vp, vp, vp]
        L.orc_crane_accel.argtypes = [vp, vp, vp, vp, ctypes.c_double, ctypes.c_double, vp]
        L.orc_so3_log.argtypes = [vp, vp]
        L.orc_so3_jr_inv.argtypes = [vp, vp]
        L.orc_ik_residual.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class Model:
    """Robot + scene + cost parameters marshalled for the C oracle.  Arrays are
    kept referenced so the raw pointers stay valid."""

    def __init__(self, robot, scene, cost, sdf: Optional[np.ndarray] = None, sdf_spec=None):
        self.robot, self.scene, self.cost = robot, scene, cost
        self._keep = []

        def keep(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a.ctypes.data

        r = _Robot()
        r.n_joints = robot.n_joints
        r.type = keep(robot.joint_type, np.int32)
        r.axis = keep(robot.axis, np.float32)
        r.origin = keep(robot.origin, np.float32)
        r.q_min = keep(robot.q_min, np.float32)
        r.q_max = keep(robot.q_max, np.float32)
        r.q_hold = keep(robot.q_hold, np.float32)
        r.active = keep(robot.active, np.uint8)
        r.n_spheres = robot.n_spheres
        r.sphere_frame = keep(robot.sphere_frame, np.int32)
        r.sphere_center = keep(robot.sphere_center, np.float32)
        r.sphere_radius = keep(robot.sphere_radius, np.float32)
        r.tip = keep(robot.tip, np.float32)
        pairs = np.asarray(getattr(robot, "self_pairs", np.zeros((0, 2))), np.int32).reshape(-1, 2)
        r.n_self = int(pairs.shape[0])
        r.self_pairs = keep(pairs if pairs.size else np.zeros((1, 2)), np.int32)
        hb = np.asarray(getattr(robot, "hull_box", np.zeros((0, 15))), np.float32).reshape(-1, 15)
        r.n_hulls = int(hb.shape[0])
        r.hull_frame = keep(getattr(robot, "hull_frame", np.zeros(0)) if hb.size else np.zeros(1), np.int32)
        r.hull_box = keep(hb if hb.size else np.zeros((1, 15)), np.float32)
        s = _Scene()
        s.has_ground = int(scene.has_ground)
        s.ground_z = float(scene.ground_z)
        s.n_cyl = scene.n_cyl
        s.cyl = keep(scene.cyl if scene.n_cyl else np.zeros((1, 5)), np.float32)
        s.n_box = scene.n_box
        s.box = keep(scene.box if scene.n_box else np.zeros((1, 6)), np.float32)
        if sdf is not None:
            s.sdf = keep(sdf, np.float32)
            for a in range(3):
                s.sdf_dims[a] = int(sdf_spec.dims[a])
                s.sdf_origin[a] = float(sdf_spec.origin[a])
            s.voxel = float(sdf_spec.voxel)
        else:
            s.sdf = None
        s.narrow = int(getattr(scene, "narrow", 0))
        ob = np.asarray(getattr(scene, "obb", np.zeros((0, 15))), np.float32).reshape(-1, 15)
        s.n_obb = int(ob.shape[0])
        s.obb = keep(ob if ob.size else np.zeros((1, 15)), np.float32)
        if s.narrow == 1 and r.n_hulls == 0:
            raise ValueError("the separating-axis narrow phase needs the robot's hulls")
        self.sat = s.narrow == 1
        c = _Cost()
        if cost is not None:
            c.K, c.M, c.interp, c.jp_mode, c.hinge = cost.K, cost.M, cost.interp, cost.jp_mode, cost.hinge
            c.margin, c.lambda_c, c.w_c, c.w_l = cost.margin, cost.lambda_c, cost.w_c, cost.w_l
        self.r, self.s, self.c = r, s, c

    # pointers
    @property
    def pr(self):
        return ctypes.addressof(self.r)

    @property
    def ps(self):
        return ctypes.addressof(self.s)

    @property
    def pc(self):
        return ctypes.addressof(self.c)

    def n_s(self) -> int:
        return lib().orc_n_checkpoints(self.pc)


# ----------------------------------------------------------------------------
# kinematics, distances, path, cost
# ----------------------------------------------------------------------------

def fk(model: Model, q):
    """Frames [n+1,12], sphere centres [S,3], tip [3] at joint vector q."""
    q = np.ascontiguousarray(q, np.float64)
    n, S = model.robot.n_joints, model.robot.n_spheres
    frames = np.zeros((n + 1, 12))
    cen = np.zeros((S, 3))
    tip = np.zeros(3)
    lib().orc_fk(model.pr, _p(q), _p(frames), _p(cen), _p(tip))
    return frames, cen, tip


def sat_obb(a, b) -> float:
    """SAT signed distance of two oriented boxes (rows of 15: centre,
    rotation row-major with the box axes as columns, half extents)."""
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    return float(lib().orc_sat_obb_f(_p(a), _p(b)))


def hulls_world(model: Model, q) -> np.ndarray:
    """The robot's hulls in world coordinates at q, [H,15]."""
    q = np.ascontiguousarray(q, np.float64)
    out = np.zeros((model.r.n_hulls, 15))
    lib().orc_hulls_world(model.pr, _p(q), _p(out))
    return out


def sd_cylinder(c, cyl, grad=False):
    c = np.ascontiguousarray(c, np.float64)
    cyl = np.ascontiguousarray(cyl, np.float32)
    g = np.zeros(3)
    d = lib().orc_sd_cylinder(_p(c), _p(cyl), _p(g))
    return (d, g) if grad else d


def sd_box(c, box, grad=False):
    c = np.ascontiguousarray(c, np.float64)
    box = np.ascontiguousarray(box, np.float32)
    g = np.zeros(3)
    d = lib().orc_sd_box(_p(c), _p(box), _p(g))
    return (d, g) if grad else d


def sdf_query(model: Model, c, grad=False):
    c = np.ascontiguousarray(c, np.float64)
    g = np.zeros(3)
    d = lib().orc_sdf_query(model.ps, _p(c), _p(g))
    return (d, g) if grad else d


def eval_configs(model: Model, Q):
    """d(q), argmin sphere, argmin obstacle and runner-up pair distance for
    joint vectors Q [N,n]."""
    Q = np.ascontiguousarray(Q, np.float64)
    N = Q.shape[0]
    d = np.zeros(N)
    s = np.zeros(N, np.int32)
    o = np.zeros(N, np.int32)
    sec = np.zeros(N)
    lib().orc_eval_configs(model.pr, model.ps, _p(Q), N, _p(d), _p(s), _p(o), _p(sec))
    return d, s, o, sec


def path_points(model: Model, q_start, q_goal, W):
    """q(s_k), k = 0..n_s, for one path W [K,n] -> [n_s+1, n]."""
    W = np.ascontiguousarray(W, np.float64)
    qs = np.ascontiguousarray(q_start, np.float64)
    qg = np.ascontiguousarray(q_goal, np.float64)
    out = np.zeros((model.n_s() + 1, model.robot.n_joints))
    lib().orc_path_points(model.pr, model.pc, _p(qs), _p(qg), _p(W), _p(out))
    return out


def eval_paths(model: Model, q_start, q_goal, W, per_checkpoint: bool = False):
    """Cost, min distance and flag of each path W [B,K,n].  With
    ``per_checkpoint`` also d_k, the tape (sphere << 16 | obstacle), the
    runner-up pair distance [B,n_s] and (J_p, J_c, J_l) [B,3]."""
    W = np.ascontiguousarray(W, np.float64)
    B = W.shape[0]
    qs = np.ascontiguousarray(q_start, np.float64)
    qg = np.ascontiguousarray(q_goal, np.float64)
    cost = np.zeros(B)
    md = np.zeros(B)
    fl = np.zeros(B, np.uint8)
    out = {"cost": cost, "min_dist": md, "flags": fl}
    dk = tape = sec = parts = None
    if per_checkpoint:
        ns = model.n_s()
        dk = np.zeros((B, ns))
        tape = np.zeros((B, ns), np.int32)
        sec = np.zeros((B, ns))
        parts = np.zeros((B, 3))
        out.update(d=dk, tape=tape, second=sec, parts=parts)
    lib().orc_eval_paths(model.pr, model.ps, model.pc, _p(qs), _p(qg), _p(W), B, _p(cost), _p(md), _p(fl),
                         _p(dk), _p(tape), _p(sec), _p(parts))
    return out


def grad_paths(model: Model, q_start, q_goal, W):
    """Analytic d cost / d W [B,K,n] and the cost [B]."""
    if model.sat:
        raise ValueError("the separating-axis narrow phase has no gradient here")
    W = np.ascontiguousarray(W, np.float64)
    B = W.shape[0]
    qs = np.ascontiguousarray(q_start, np.float64)
    qg = np.ascontiguousarray(q_goal, np.float64)
    cost = np.zeros(B)
    g = np.zeros(W.shape)
    lib().orc_grad_paths(model.pr, model.ps, model.pc, _p(qs), _p(qg), _p(W), B, _p(cost), _p(g))
    return cost, g


def fd_grad(model: Model, q_start, q_goal, W, h: float = 1e-6):
    """Central finite differences of the double-precision cost of each path,
    (J(W + h e) - J(W - h e)) / 2h for every waypoint entry -> [B,K,n]."""
    W = np.asarray(W, np.float64)
    B, K, n = W.shape
    g = np.zeros(W.shape)
    for i in range(K):
        for j in range(n):
            Wp = W.copy()
            Wm = W.copy()
            Wp[:, i, j] += h
            Wm[:, i, j] -= h
            cp = eval_paths(model, q_start, q_goal, Wp)["cost"]
            cm = eval_paths(model, q_start, q_goal, Wm)["cost"]
            g[:, i, j] = (cp - cm) / (2.0 * h)
    return g



# ----------------------------------------------------------------------------
# collision-free inverse kinematics (Sec. 3.2, eq. IK opt)
# ----------------------------------------------------------------------------

def so3_log(R):
    """Rotation vector w (|w| in [0, pi]) of the rotation matrix R [3,3]."""
    R = np.ascontiguousarray(R, np.float64)
    w = np.zeros(3)
    lib().orc_so3_log(_p(R), _p(w))
    return w


def so3_jr_inv(w):
    """Inverse right Jacobian of SO(3) at the rotation vector w [3] -> [3,3]."""
    w = np.ascontiguousarray(w, np.float64)
    J = np.zeros((3, 3))
    lib().orc_so3_jr_inv(_p(w), _p(J))
    return J


def ik_weights(par) -> np.ndarray:
    return np.array([par.lambda_q, par.lambda_c, par.lambda_e, par.lambda_r], np.float64)


def ik_residual(model: Model, par, target, q, q_ref, jacobian: bool = True):
    """Residual r [8+n] of the IK problem at q, its Jacobian [8+n, n] (or
    None) and info = (|p_g - p_d|, |Log(R_d^T R_g)|, d(q), |g_p|, argmin
    sphere, argmin obstacle).  ``target`` is R_d row-major then p_d [12]."""
    if model.sat:
        raise ValueError("the IK takes the sphere narrow phase")
    n = model.robot.n_joints
    lam = ik_weights(par)
    t = np.ascontiguousarray(target, np.float64)
    q = np.ascontiguousarray(q, np.float64)
    qr = np.ascontiguousarray(q_ref, np.float64)
    r = np.zeros(8 + n)
    J = np.zeros((8 + n, n)) if jacobian else None
    info = np.zeros(6)
    lib().orc_ik_residual(model.pr, model.ps, _p(lam), _p(t), _p(q), _p(qr), _p(r), _p(J), _p(info))
    return r, J, info


def ik_solve(model: Model, par, target, q_init, q_ref, trace: Optional[list] = None):
    """Levenberg-Marquardt on F(q) = |r(q)|^2 / 2 (eq. IK opt), with the
    damping schedule of Madsen, Nielsen and Tingleff ("Methods for non-linear
    least squares problems", 2004, Sec. 3.2): mu_0 = tau max diag(J^T J);
    each iteration solves (J^T J + mu I) h = -J^T r, takes q' = q + h (clamped
    to the joint limits if ``par.clamp``), and accepts it when the gain ratio
    rho = (F(q) - F(q')) / (L(0) - L(q' - q)) is positive, with
    L(0) - L(s) = -s.g - s.A s / 2 the decrease predicted by the linear model;
    then mu *= max(1/3, 1 - (2 rho - 1)^3), nu = 2, else mu *= nu, nu *= 2.
    Stops when max |J^T r| <= eps_grad (status 1), when
    |h| <= eps_step (|q| + eps_step) (status 2), or after max_iters trial
    steps (status 0).  Returns (q, F, info, iterations, status); with
    ``trace`` the accepted iterates (q, F) are appended to it."""
    lo = np.asarray(model.robot.q_min, np.float64)
    hi = np.asarray(model.robot.q_max, np.float64)
    q = np.array(q_init, np.float64)
    if par.clamp:
        q = np.clip(q, lo, hi)
    r, J, info = ik_residual(model, par, target, q, q_ref)
    F = 0.5 * float(r @ r)
    A = J.T @ J
    g = J.T @ r
    mu = par.tau * float(np.max(np.diag(A)))
    nu = 2.0
    it = 0
    status = 0
    if trace is not None:
        trace.append((q.copy(), F))
    while it < par.max_iters:
        if float(np.max(np.abs(g))) <= par.eps_grad:
            status = 1
            break
        h = np.linalg.solve(A + mu * np.eye(A.shape[0]), -g)
        if float(np.linalg.norm(h)) <= par.eps_step * (float(np.linalg.norm(q)) + par.eps_step):
            status = 2
            break
        qn = q + h
        if par.clamp:
            qn = np.clip(qn, lo, hi)
        s = qn - q
        rn, Jn, infon = ik_residual(model, par, target, qn, q_ref)
        Fn = 0.5 * float(rn @ rn)
        pred = -float(s @ g) - 0.5 * float(s @ A @ s)
        it += 1
        if pred > 0.0 and F - Fn > 0.0:
            rho = (F - Fn) / pred
            q, r, J, info, F = qn, rn, Jn, infon, Fn
            A = J.T @ J
            g = J.T @ r
            mu *= max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
            nu = 2.0
            if trace is not None:
                trace.append((q.copy(), F))
        else:
            mu *= nu
            nu *= 2.0
    return q, F, info, it, status

# ----------------------------------------------------------------------------
# step two: reduced dynamics and direct collocation (Sec. 2.1, Sec. 4.2)
# ----------------------------------------------------------------------------

def crane_accel(model: Model, q, qd, u, grav: float, damping: float) -> np.ndarray:
    """Joint accelerations of the reduced dynamics (u: the actuated joints'
    accelerations in joint order)."""
    n = model.robot.n_joints
    q = np.ascontiguousarray(q, np.float64)
    qd = np.ascontiguousarray(qd, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    out = np.zeros(n)
    lib().orc_crane_accel(model.pr, _p(q), _p(qd), _p(u), float(grav), float(damping), _p(out))
    return out


def traj_f(model: Model, par, x, u) -> np.ndarray:
    """Right-hand side of x' = f(x, u), x = (q, qd)."""
    n = model.robot.n_joints
    return np.concatenate([x[n:], crane_accel(model, x[:n], x[n:], u, par.grav, par.damping)])


def traj_f_jac(model: Model, par, x, u):
    """df/dx [2n, 2n] and df/du [2n, n_a] by central differences (steps
    par.fd_q on positions, 1 on velocities and inputs)."""
    n = model.robot.n_joints
    na = len(u)
    Jx = np.zeros((2 * n, 2 * n))
    Ju = np.zeros((2 * n, na))
    for i in range(2 * n):
        h = par.fd_q if i < n else 1.0
        e = np.zeros(2 * n)
        e[i] = h
        Jx[:, i] = (traj_f(model, par, x + e, u) - traj_f(model, par, x - e, u)) / (2.0 * h)
    for i in range(na):
        e = np.zeros(na)
        e[i] = 1.0
        Ju[:, i] = (traj_f(model, par, x, u + e) - traj_f(model, par, x, u - e)) / 2.0
    return Jx, Ju


class TrajLayout:
    """Unknowns z of the collocation problem: per time point k = 0..N the
    state x_k (for 1 <= k <= N-1; x_0 and x_N are fixed) and the input u_k,
    time-major, then s with t_F = s^2.  Residuals r: the N defects (2n each,
    scaled), the state bounds of the interior points (4n each: q above its
    upper limit, below its lower one, qd above v_max, below -v_max), the
    input terms sqrt(omega_s) u_k and tracking terms sqrt(omega_t)
    (q_a,k - q*_a,k) for k = 1..N (n_a each), then s, then the penalty of
    the final-time bound s >= sqrt(t_min)."""

    def __init__(self, n: int, na: int, N: int):
        self.n, self.na, self.N = n, na, N
        self.off = np.zeros(N + 2, np.int64)
        for k in range(N + 1):
            size = na + (2 * n if 0 < k < N else 0)
            self.off[k + 1] = self.off[k] + size
        self.s = int(self.off[N + 1])
        self.nz = self.s + 1
        self.r_def = 0
        self.r_bnd = N * 2 * n
        self.r_u = self.r_bnd + (N - 1) * 4 * n
        self.r_q = self.r_u + N * na
        self.r_s = self.r_q + N * na
        self.r_t = self.r_s + 1
        self.nr = self.r_t + 1

    def x_at(self, z, k):
        return None if k in (0, self.N) else z[self.off[k]:self.off[k] + 2 * self.n]

    def u_at(self, z, k):
        o = self.off[k] + (2 * self.n if 0 < k < self.N else 0)
        return z[o:o + self.na]


def _traj_bounds(model, par):
    rb = model.robot
    lo = np.concatenate([np.asarray(rb.q_min, np.float64), -np.asarray(par.v_max, np.float64)])
    hi = np.concatenate([np.asarray(rb.q_max, np.float64), np.asarray(par.v_max, np.float64)])
    return lo, hi


def traj_t_min(model: Model, par, q_start, q_goal):
    """The shortest final time the velocity limits allow: every joint moves
    |q_d,j - q_0,j| at speed at most v_max,j, so t_F >= max_j |q_d,j -
    q_0,j| / v_max,j.  The trapezoidal defects imply the same bound on the
    discrete problem (q_N - q_0 = sum_k h (qd_k + qd_k+1) / 2), so adding
    it leaves the feasible set unchanged; it keeps the solver away from
    t_F = 0, where t_F = s^2 makes every residual stationary in s."""
    dq = np.abs(np.asarray(q_goal, np.float64) - np.asarray(q_start, np.float64))
    return float(np.max(dq / np.asarray(par.v_max, np.float64)[:len(dq)]))


def traj_residual(model: Model, par, q_start, q_goal, q_star, z, lam, mu, jacobian: bool = True):
    """Residual r [nr] of the collocation problem at z (augmented Lagrangian
    with multipliers lam [N, 2n] and penalty mu on the defects) and its
    Jacobian [nr, nz] (or None).  q_star [N+1, n]: the path's points."""
    rb = model.robot
    n = rb.n_joints
    act = np.where(np.asarray(rb.active) != 0)[0]
    na = len(act)
    N = par.N
    L = TrajLayout(n, na, N)
    xs = np.concatenate([np.asarray(q_start, np.float64), np.zeros(n)])
    xg = np.concatenate([np.asarray(q_goal, np.float64), np.zeros(n)])
    X = [xs] + [L.x_at(z, k) for k in range(1, N)] + [xg]
    U = [L.u_at(z, k) for k in range(N + 1)]
    s = z[L.s]
    h2 = s * s / (2.0 * N)  # h / 2 with h = t_F / N
    F = [traj_f(model, par, X[k], U[k]) for k in range(N + 1)]
    r = np.zeros(L.nr)
    J = np.zeros((L.nr, L.nz)) if jacobian else None
    sm = math.sqrt(mu)
    for k in range(N):
        d = X[k + 1] - X[k] - h2 * (F[k] + F[k + 1])
        r[2 * n * k:2 * n * (k + 1)] = sm * (d + lam[k] / mu)
    lo, hi = _traj_bounds(model, par)
    for k in range(1, N):
        o = L.r_bnd + 4 * n * (k - 1)
        x = X[k]
        r[o:o + 2 * n] = sm * np.maximum(x - hi, 0.0)
        r[o + 2 * n:o + 4 * n] = sm * np.maximum(lo - x, 0.0)
    for k in range(1, N + 1):
        r[L.r_u + na * (k - 1):L.r_u + na * k] = math.sqrt(par.omega_s) * U[k]
        r[L.r_q + na * (k - 1):L.r_q + na * k] = math.sqrt(par.omega_t) * (X[k][act] - np.asarray(q_star[k], np.float64)[act])
    r[L.r_s] = s
    s_min = math.sqrt(traj_t_min(model, par, q_start, q_goal))
    r[L.r_t] = sm * max(s_min - s, 0.0)
    if not jacobian:
        return r, None
    Jf = [traj_f_jac(model, par, X[k], U[k]) for k in range(N + 1)]
    I = np.eye(2 * n)
    for k in range(N):
        rows = slice(2 * n * k, 2 * n * (k + 1))
        for kk, sign in ((k, -1.0), (k + 1, 1.0)):
            Jx, Ju = Jf[kk]
            if 0 < kk < N:
                J[rows, L.off[kk]:L.off[kk] + 2 * n] = sm * (sign * I - h2 * Jx)
            uo = L.off[kk] + (2 * n if 0 < kk < N else 0)
            J[rows, uo:uo + na] = sm * (-h2 * Ju)
        J[rows, L.s] = sm * (-(s / N) * (F[k] + F[k + 1]))
    for k in range(1, N):
        o = L.r_bnd + 4 * n * (k - 1)
        x = X[k]
        for i in range(2 * n):
            if x[i] > hi[i]:
                J[o + i, L.off[k] + i] = sm
            if x[i] < lo[i]:
                J[o + 2 * n + i, L.off[k] + i] = -sm
    for k in range(1, N + 1):
        uo = L.off[k] + (2 * n if 0 < k < N else 0)
        for i in range(na):
            J[L.r_u + na * (k - 1) + i, uo + i] = math.sqrt(par.omega_s)
            if k < N:
                J[L.r_q + na * (k - 1) + i, L.off[k] + act[i]] = math.sqrt(par.omega_t)
    J[L.r_s, L.s] = 1.0
    if s < s_min:
        J[L.r_t, L.s] = -sm
    return r, J


def traj_initial(model: Model, par, q_start, q_goal, q_star):
    """Starting point: the path's points at times k t_0 / N, velocities and
    inputs from their differences, s = sqrt(t_0), t_0 = max(t_f0, t_min)."""
    rb = model.robot
    n = rb.n_joints
    act = np.where(np.asarray(rb.active) != 0)[0]
    N = par.N
    L = TrajLayout(n, len(act), N)
    t0 = max(par.t_f0, traj_t_min(model, par, q_start, q_goal))
    h = t0 / N
    Q = np.asarray(q_star, np.float64).copy()
    Q[0], Q[N] = q_start, q_goal
    V = np.zeros_like(Q)
    V[1:N] = (Q[2:] - Q[:N - 1]) / (2.0 * h)
    z = np.zeros(L.nz)
    for k in range(N + 1):
        if 0 < k < N:
            z[L.off[k]:L.off[k] + n] = Q[k]
            z[L.off[k] + n:L.off[k] + 2 * n] = V[k]
        uo = L.off[k] + (2 * n if 0 < k < N else 0)
        z[uo:uo + len(act)] = ((V[k + 1] - V[k]) / h)[act] if k < N else 0.0
    z[L.s] = math.sqrt(t0)
    return z


def traj_refine(model: Model, par, q_start, q_goal, q_star, trace: Optional[list] = None):
    """Step two (Sec. 4.2, eq. discrete): augmented Lagrangian on the
    trapezoidal defects around Levenberg-Marquardt (the damping schedule of
    the IK).  Per outer iteration: minimise |r|^2 / 2 by LM from the current
    point, then lam += mu d (d the defects), mu *= mu_factor.  Returns
    dict(t_f, X [N+1, 2n], U [N+1, n_a], z, defect (max |d|), F (the last
    |r|^2 / 2), iters (trial steps over all outer iterations), accepted (the
    trial steps taken), t_min)."""
    rb = model.robot
    n = rb.n_joints
    act = np.where(np.asarray(rb.active) != 0)[0]
    N = par.N
    L = TrajLayout(n, len(act), N)
    z = traj_initial(model, par, q_start, q_goal, q_star)
    lam = np.zeros((N, 2 * n))
    mu = par.mu0
    iters = 0
    accepted = 0
    F = 0.0
    for _ in range(par.outer):
        r, J = traj_residual(model, par, q_start, q_goal, q_star, z, lam, mu)
        F = 0.5 * float(r @ r)
        A = J.T @ J
        g = J.T @ r
        damp = par.tau * float(np.max(np.diag(A)))
        nu = 2.0
        it = 0
        while it < par.max_iters:
            if float(np.max(np.abs(g))) <= par.eps_grad:
                break
            hstep = np.linalg.solve(A + damp * np.eye(L.nz), -g)
            if float(np.linalg.norm(hstep)) <= par.eps_step * (float(np.linalg.norm(z)) + par.eps_step):
                break
            zn = z + hstep
            rn, Jn = traj_residual(model, par, q_start, q_goal, q_star, zn, lam, mu)
            Fn = 0.5 * float(rn @ rn)
            pred = -float(hstep @ g) - 0.5 * float(hstep @ A @ hstep)
            it += 1
            if pred > 0.0 and F - Fn > 0.0:
                rho = (F - Fn) / pred
                accepted += 1
                z, r, J, F = zn, rn, Jn, Fn
                A = J.T @ J
                g = J.T @ r
                damp *= max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
                nu = 2.0
            else:
                damp *= nu
                nu *= 2.0
        iters += it
        # multiplier update from the defects at z
        d = r[:N * 2 * n].reshape(N, 2 * n) / math.sqrt(mu) - lam / mu
        lam = lam + mu * d
        mu *= par.mu_factor
        if trace is not None:
            trace.append((z.copy(), F, float(np.max(np.abs(d)))))
    X = np.zeros((N + 1, 2 * n))
    U = np.zeros((N + 1, len(act)))
    X[0, :n], X[N, :n] = q_start, q_goal
    for k in range(N + 1):
        if 0 < k < N:
            X[k] = L.x_at(z, k)
        U[k] = L.u_at(z, k)
    r0, _ = traj_residual(model, par, q_start, q_goal, q_star, z, np.zeros((N, 2 * n)), 1.0, jacobian=False)
    return dict(t_f=float(z[L.s] ** 2), X=X, U=U, z=z, defect=float(np.max(np.abs(r0[:N * 2 * n]))), F=F,
                iters=iters, accepted=accepted, t_min=traj_t_min(model, par, q_start, q_goal))


# ----------------------------------------------------------------------------
# RNG
# ----------------------------------------------------------------------------

def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def normals(seed: int, t: int, B: int, D: int, problem: int = 0):
    z = np.zeros((B, D))
    lib().orc_normals(ctypes.c_uint64(seed), t, problem, B, D, _p(z))
    return z


# ----------------------------------------------------------------------------
# signed-distance grid
# ----------------------------------------------------------------------------

def occupancy(points, dims, origin, voxel):
    pts = np.ascontiguousarray(points, np.float32)
    d = np.ascontiguousarray(dims, np.int32)
    o = np.ascontiguousarray(origin, np.float32)
    occ = np.zeros((dims[2], dims[1], dims[0]), np.uint8)
    lib().orc_occupancy(_p(pts), pts.shape[0], _p(d), _p(o), float(voxel), _p(occ))
    return occ


def edt(mask, target: int = 1, brute: bool = False):
    """Squared Euclidean distance (voxel units) from every voxel of ``mask``
    [nz,ny,nx] to the nearest voxel whose value equals ``target``."""
    mask = np.ascontiguousarray(mask, np.uint8)
    nz, ny, nx = mask.shape
    d = np.array([nx, ny, nz], np.int32)
    out = np.zeros(mask.shape, np.int64)
    fn = lib().orc_edt_brute if brute else lib().orc_edt_separable
    fn(_p(mask), target, _p(d), _p(out))
    return out


def sdf_from_occupancy(occ, voxel):
    occ = np.ascontiguousarray(occ, np.uint8)
    e_occ = edt(occ, 1)
    e_free = edt(occ, 0)
    phi = np.zeros(occ.shape)
    lib().orc_sdf_from_edt(_p(occ), _p(e_occ), _p(e_free), occ.size, float(voxel), _p(phi))
    return phi, e_occ, e_free


def sdf_build(points, spec):
    occ = occupancy(points, spec.dims, spec.origin, spec.voxel)
    phi, e_occ, e_free = sdf_from_occupancy(occ, spec.voxel)
    return phi, occ, e_occ, e_free


# ----------------------------------------------------------------------------
# Algorithm 1: stochastic optimization with log-rank weights
# ----------------------------------------------------------------------------

class NotPositiveDefinite(RuntimeError):
    pass


def log_rank_weights(nu: int) -> np.ndarray:
    """Step (4): w_j = (ln(nu + 1/2) - ln j) / sum_k (ln(nu + 1/2) - ln k)."""
    j = np.arange(1, nu + 1, dtype=np.float64)
    a = math.log(nu + 0.5) - np.log(j)
    return a / a.sum()


def initial_mean(robot, q_start, q_goal, K: int) -> np.ndarray:
    """Control points evenly spaced on the segment from start to goal
    (Sec. 4.1 initial guess): W_i = q_s + (i+1)/(K+1) (q_g - q_s), active
    joints only, flattened [K * n_active] (waypoint-major)."""
    act = robot.active.astype(bool)
    qs = np.asarray(q_start, np.float64)[act]
    qg = np.asarray(q_goal, np.float64)[act]
    i = np.arange(K, dtype=np.float64)[:, None]
    return (qs[None, :] + (i + 1.0) / (K + 1.0) * (qg - qs)[None, :]).reshape(-1)


def cholesky_jitter(C: np.ndarray, eps: float) -> np.ndarray:
    """Lower Cholesky factor of C; if C is not numerically positive definite,
    retry with C + 10^k eps I for k = 1, 2, 3."""
    D = C.shape[0]
    for k in range(4):
        A = C if k == 0 else C + (10.0 ** k) * eps * np.eye(D)
        try:
            return np.linalg.cholesky(A)
        except np.linalg.LinAlgError:
            continue
    raise NotPositiveDefinite("covariance is not positive definite")


def expand(robot, xi: np.ndarray, K: int) -> np.ndarray:
    """Samples xi [B, K*n_active] -> waypoints [B,K,n] (double); joints that
    are not sampled take their hold value."""
    B = xi.shape[0]
    n = robot.n_joints
    act = robot.active.astype(bool)
    W = np.empty((B, K, n), np.float64)
    W[:, :, act] = xi.reshape(B, K, int(act.sum()))
    W[:, :, ~act] = robot.q_hold[~act]
    return W


def select(cost: np.ndarray, nu: int) -> np.ndarray:
    """Step (3): indices of the nu lowest costs, stable on (cost, index), NaN
    ranked as +inf (so a NaN and a +inf go by index) and -0 equal to +0."""
    key = np.where(np.isnan(cost), np.inf, cost)
    order = np.lexsort((np.arange(cost.shape[0]), key))
    return order[:nu]


def update(xi_elite: np.ndarray, w: np.ndarray, eps: float):
    """Steps (5)-(6): mu' = sum_j w_j x_(j);
    C' = sum_j w_j (x_(j) - mu')(x_(j) - mu')^T + eps I."""
    mu = w @ xi_elite
    diff = xi_elite - mu[None, :]
    C = (diff * w[:, None]).T @ diff + eps * np.eye(xi_elite.shape[1])
    return mu, C


class Optimizer:
    """Algorithm 1 on one problem, step by step, in double precision."""

    def __init__(self, problem, model: Optional[Model] = None, problem_id: int = 0):
        self.p = problem
        self.model = model or Model(problem.robot, problem.scene, problem.cost)
        K = problem.cost.K
        self.K = K
        self.D = K * problem.robot.n_active
        self.mu = initial_mean(problem.robot, problem.q_start, problem.q_goal, K)
        # sigma0 is a single-precision parameter of the problem statement
        s0 = float(np.float32(problem.opt.sigma0))
        self.C = (s0 * s0) * np.eye(self.D)
        self.t = 0
        self.problem_id = problem_id
        self.w = log_rank_weights(problem.opt.nu)
        self.best_cost = math.inf
        self.best_xi = None
        self.history = []

    def set_state(self, mu, C, t):
        self.mu = np.array(mu, np.float64)
        self.C = np.array(C, np.float64)
        self.t = int(t)

    def sample(self):
        """Step (1): xi_b = mu + L z_b with z from Philox/Box-Muller."""
        L = cholesky_jitter(self.C, self.p.opt.eps)
        z = normals(self.p.opt.seed, self.t, self.p.opt.B, self.D, self.problem_id)
        return self.mu[None, :] + z @ L.T

    def polish(self, xi_elite, trace: Optional[list] = None):
        """Gradient polish of the elites (a workload setting, not in the
        paper): each takes ``polish_steps`` steps
        W <- W - eta g / max(1, |g| / g_max), where g is the analytic gradient
        of the path cost restricted to the sampled joints and |g| its norm
        over those joints only; joints that are not sampled keep their hold
        value.  With ``trace`` (a list), the iterate before every step is
        appended to it."""
        o = self.p.opt
        act = self.p.robot.active.astype(bool)
        xi = xi_elite.copy()
        for _ in range(o.polish_steps):
            if trace is not None:
                trace.append(xi.copy())
            W = expand(self.p.robot, xi, self.K)
            _, g = grad_paths(self.model, self.p.q_start, self.p.q_goal, W)
            g = g[:, :, act].reshape(xi.shape[0], -1)
            nrm = np.sqrt((g * g).sum(1))
            scale = o.polish_eta / np.maximum(1.0, nrm / o.polish_clip)
            xi = xi - scale[:, None] * g
        return xi

    def step(self):
        o = self.p.opt
        xi = self.sample()
        W = expand(self.p.robot, xi, self.K)
        r = eval_paths(self.model, self.p.q_start, self.p.q_goal, W)
        cost = r["cost"]
        elite = select(cost, o.nu)
        xe = xi[elite]
        ce = cost[elite]
        if o.polish_steps > 0 and o.polish_elites > 0:
            npol = min(o.polish_elites, o.nu)
            xe = xe.copy()
            xe[:npol] = self.polish(xe[:npol])
            rp = eval_paths(self.model, self.p.q_start, self.p.q_goal, expand(self.p.robot, xe, self.K))
            ce = rp["cost"]
            order = select(ce, o.nu)
            xe, ce = xe[order], ce[order]
        mu, C = update(xe, self.w, o.eps)
        # best-so-far over every evaluated sample, ties by (iteration, index)
        kb = int(select(cost, 1)[0])
        if cost[kb] < self.best_cost:
            self.best_cost = float(cost[kb])
            self.best_xi = xi[kb].copy()
        if o.polish_steps > 0 and ce.size and ce[0] < self.best_cost:
            self.best_cost = float(ce[0])
            self.best_xi = xe[0].copy()
        self.history.append(dict(t=self.t, elite=elite, cost=cost, mu=mu, C=C))
        self.mu, self.C = mu, C
        self.t += 1
        return dict(xi=xi, cost=cost, elite=elite, mu=mu, C=C)
