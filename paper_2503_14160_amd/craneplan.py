"""Python binding of the craneplan C-ABI library (argument marshalling only).

Every computation runs in the HIP kernels of ``libcraneplan.so``; this module
only converts arguments, hands device pointers of torch tensors to the
library, and enqueues on torch's current HIP stream.  It raises if the
library has not been built (``python -m paper_2503_14160_amd.build``); there
is no fallback path.

Robot, scene and parameter arguments are read by attribute name (the field
names of the declarations in ``include/craneplan.h``), so any object with
those attributes works, e.g. the dataclasses of ``paper_2503_14160_amd.synth``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcraneplan.so")

_c_i32, _c_f32, _c_f64, _c_u64, _c_u32, _vp = (ctypes.c_int32, ctypes.c_float, ctypes.c_double, ctypes.c_uint64,
                                               ctypes.c_uint32, ctypes.c_void_p)

CP_OBS_SDF = 0xFFFF
# cp_cost_params.pair_filter: every pair / lane-level square-root skip / wave-level culling /
# culling for scenes of at least 48 obstacles, else the lane filter
PAIRS_ALL, PAIRS_LANE, PAIRS_WAVE, PAIRS_AUTO = 0, 1, 2, 3
# cp_scene_desc.narrow: spheres against primitives / grid, or the separating axis test on hulls
NARROW_SPHERES, NARROW_SAT = 0, 1
EXPORTS = ["cp_last_error", "cp_plan_create", "cp_plan_destroy", "cp_plan_set_endpoints", "cp_plan_n_checkpoints",
           "cp_eval_paths", "cp_eval_paths_backward", "cp_optimizer_create", "cp_optimizer_destroy",
           "cp_optimizer_step", "cp_optimizer_get_state", "cp_optimizer_set_state", "cp_optimizer_last",
           "cp_sdf_build", "cp_debug_fk", "cp_debug_eval_configs", "cp_debug_select", "cp_batch_create",
           "cp_batch_destroy", "cp_batch_run", "cp_batch_eval", "cp_batch_get_state", "cp_batch_set_tuning",
           "cp_batch_get_tuning", "cp_batch_tune", "cp_optimizer_last_elites", "cp_tune",
           "cp_debug_update", "cp_optimizer_last_polished", "cp_batch_last", "cp_eval_paths_noalloc",
           "cp_optimizer_time_eval", "cp_optimizer_eval_time", "cp_optimizer_record_tape",
           "cp_optimizer_population_grad", "cp_ik_solve", "cp_debug_ik_residual", "cp_traj_workspace_size",
           "cp_traj_refine"]


class CranePlanError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"craneplan error {code}: {msg}")
        self.code = code


class _Robot(ctypes.Structure):
    _fields_ = [("n_joints", _c_i32), ("type", _vp), ("axis", _vp), ("origin", _vp), ("q_min", _vp),
                ("q_max", _vp), ("q_hold", _vp), ("active", _vp), ("n_spheres", _c_i32), ("sphere_frame", _vp),
                ("sphere_center", _vp), ("sphere_radius", _vp), ("n_self_pairs", _c_i32), ("self_pairs", _vp),
                ("tip", _c_f32 * 3), ("n_hulls", _c_i32), ("hull_frame", _vp), ("hull_box", _vp)]


class _Scene(ctypes.Structure):
    _fields_ = [("has_ground", _c_i32), ("ground_z", _c_f32), ("n_cyl", _c_i32), ("cyl", _vp), ("n_box", _c_i32),
                ("box", _vp), ("d_sdf", _vp), ("sdf_dims", _c_i32 * 3), ("sdf_origin", _c_f32 * 3),
                ("voxel", _c_f32), ("narrow", _c_i32), ("n_obb", _c_i32), ("obb", _vp)]


class _Cost(ctypes.Structure):
    _fields_ = [("K", _c_i32), ("M", _c_i32), ("interp", _c_i32), ("jp_mode", _c_i32), ("hinge", _c_i32),
                ("margin", _c_f32), ("lambda_c", _c_f32), ("w_c", _c_f32), ("w_l", _c_f32), ("max_B", _c_i32),
                ("pair_filter", _c_i32)]


class _Ik(ctypes.Structure):
    _fields_ = [("lambda_q", _c_f32), ("lambda_c", _c_f32), ("lambda_e", _c_f32), ("lambda_r", _c_f32),
                ("max_iters", _c_i32), ("tau", _c_f32), ("eps_grad", _c_f32), ("eps_step", _c_f32),
                ("clamp", _c_i32)]


class _Traj(ctypes.Structure):
    _fields_ = [("N", _c_i32), ("omega_s", _c_f64), ("omega_t", _c_f64), ("grav", _c_f64), ("damping", _c_f64),
                ("v_max", _c_f64 * 8), ("mu0", _c_f64), ("mu_factor", _c_f64), ("outer", _c_i32),
                ("max_iters", _c_i32), ("tau", _c_f64), ("eps_grad", _c_f64), ("eps_step", _c_f64),
                ("fd_q", _c_f64), ("t_f0", _c_f64)]


def _fill_traj(t, par, n):
    t.N = int(par.N)
    t.omega_s, t.omega_t, t.grav, t.damping = float(par.omega_s), float(par.omega_t), float(par.grav), float(par.damping)
    vm = list(par.v_max)
    for j in range(8):
        t.v_max[j] = float(vm[j]) if j < len(vm) else 1.0
    t.mu0, t.mu_factor = float(par.mu0), float(par.mu_factor)
    t.outer, t.max_iters = int(par.outer), int(par.max_iters)
    t.tau, t.eps_grad, t.eps_step, t.fd_q, t.t_f0 = (float(par.tau), float(par.eps_grad), float(par.eps_step),
                                                      float(par.fd_q), float(par.t_f0))


class _Opt(ctypes.Structure):
    _fields_ = [("B", _c_i32), ("nu", _c_i32), ("sigma0", _c_f32), ("eps", _c_f64), ("seed", _c_u64),
                ("problem_id", _c_u32), ("polish_elites", _c_i32), ("polish_steps", _c_i32),
                ("polish_eta", _c_f32), ("polish_clip", _c_f32)]


_lib = None


def lib():
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2503_14160_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64 = _c_i32, ctypes.c_int64
        L.cp_last_error.restype = ctypes.c_char_p
        L.cp_plan_create.argtypes = [_vp, _vp, _vp, ctypes.c_int, _vp]
        L.cp_plan_destroy.argtypes = [_vp]
        L.cp_plan_set_endpoints.argtypes = [_vp, _vp, _vp]
        L.cp_plan_n_checkpoints.argtypes = [_vp, _vp]
        L.cp_eval_paths.argtypes = [_vp, _vp, i32, _vp, _vp, _vp, _vp, _vp]
        L.cp_eval_paths_backward.argtypes = [_vp, _vp, i32, _vp, _vp, _vp, _vp]
        L.cp_optimizer_create.argtypes = [_vp, _vp, _vp]
        L.cp_optimizer_destroy.argtypes = [_vp]
        L.cp_optimizer_step.argtypes = [_vp, i32, _vp]
        L.cp_optimizer_get_state.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
        L.cp_optimizer_set_state.argtypes = [_vp, _vp, _vp, ctypes.c_int64]
        L.cp_optimizer_last.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.cp_sdf_build.argtypes = [_vp, i64, _vp, _vp, _c_f32, _vp, _vp, _vp, _vp, _vp]
        L.cp_debug_fk.argtypes = [_vp, _vp, i32, _vp, _vp, _vp]
        L.cp_debug_eval_configs.argtypes = [_vp, _vp, i32, _vp, _vp, _vp]
        L.cp_debug_select.argtypes = [_vp, i32, i32, _vp, _vp]
        L.cp_batch_create.argtypes = [i32, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp]
        L.cp_batch_destroy.argtypes = [_vp]
        L.cp_batch_run.argtypes = [_vp, i32, _vp]
        L.cp_batch_eval.argtypes = [_vp, _vp]
        L.cp_batch_get_state.argtypes = [_vp, i32, _vp, _vp, _vp, _vp, _vp]
        L.cp_batch_set_tuning.argtypes = [_vp, _vp]
        L.cp_batch_get_tuning.argtypes = [_vp, _vp]
        L.cp_batch_tune.argtypes = [_vp, ctypes.c_char_p, _vp]
        L.cp_optimizer_last_elites.argtypes = [_vp, _vp, _vp, _vp]
        L.cp_tune.argtypes = [_vp, _vp, ctypes.c_char_p]
        L.cp_debug_update.argtypes = [_vp, _vp, _vp]
        L.cp_optimizer_last_polished.argtypes = [_vp, _vp, _vp, _vp]
        L.cp_batch_last.argtypes = [_vp, i32, _vp, _vp, _vp, _vp]
        L.cp_eval_paths_noalloc.argtypes = [_vp, _vp, i32, _vp, _vp, _vp, _vp, _vp]
        L.cp_optimizer_time_eval.argtypes = [_vp, i32]
        L.cp_optimizer_eval_time.argtypes = [_vp, _vp, _vp]
        L.cp_optimizer_record_tape.argtypes = [_vp, i32]
        L.cp_optimizer_population_grad.argtypes = [_vp, _vp, _vp]
        L.cp_ik_solve.argtypes = [_vp, _vp, _vp, _vp, _vp, i32, i32, _vp, _vp, _vp, _vp, _vp]
        L.cp_debug_ik_residual.argtypes = [_vp, _vp, _vp, _vp, _vp, i32, _vp, _vp, _vp]
        L.cp_traj_workspace_size.argtypes = [_vp, _vp, i32, _vp]
        L.cp_traj_refine.argtypes = [_vp, _vp, _vp, _vp, _vp, i32, _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp]
        for name in EXPORTS[1:]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise CranePlanError(rc, lib().cp_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _host(a, dt):
    return np.ascontiguousarray(np.asarray(a), dtype=dt)


def _keep_ptr(keep, a, dt):
    a = _host(a, dt)
    keep.append(a)
    return a.ctypes.data


def _fill_robot(r, robot, keep):
    r.n_joints = int(len(robot.joint_type))
    r.type = _keep_ptr(keep, robot.joint_type, np.int32)
    r.axis = _keep_ptr(keep, robot.axis, np.float32)
    r.origin = _keep_ptr(keep, robot.origin, np.float32)
    r.q_min = _keep_ptr(keep, robot.q_min, np.float32)
    r.q_max = _keep_ptr(keep, robot.q_max, np.float32)
    r.q_hold = _keep_ptr(keep, robot.q_hold, np.float32)
    r.active = _keep_ptr(keep, robot.active, np.uint8)
    r.n_spheres = int(len(robot.sphere_radius))
    r.sphere_frame = _keep_ptr(keep, robot.sphere_frame, np.int32)
    r.sphere_center = _keep_ptr(keep, robot.sphere_center, np.float32)
    r.sphere_radius = _keep_ptr(keep, robot.sphere_radius, np.float32)
    pairs = _host(getattr(robot, "self_pairs", np.zeros((0, 2))), np.int32).reshape(-1, 2)
    r.n_self_pairs = int(pairs.shape[0])
    r.self_pairs = _keep_ptr(keep, pairs, np.int32) if pairs.size else None
    tip = _host(getattr(robot, "tip", np.zeros(3)), np.float32).reshape(3)
    for a in range(3):
        r.tip[a] = float(tip[a])
    hb = _host(getattr(robot, "hull_box", np.zeros((0, 15))), np.float32).reshape(-1, 15)
    r.n_hulls = int(hb.shape[0])
    r.hull_frame = _keep_ptr(keep, robot.hull_frame, np.int32) if hb.size else None
    r.hull_box = _keep_ptr(keep, hb, np.float32) if hb.size else None


def _fill_scene(s, scene, keep, sdf=None, sdf_spec=None):
    s.has_ground = int(scene.has_ground)
    s.ground_z = float(scene.ground_z)
    s.n_cyl = int(scene.cyl.shape[0])
    s.cyl = _keep_ptr(keep, scene.cyl, np.float32) if s.n_cyl else None
    s.n_box = int(scene.box.shape[0])
    s.box = _keep_ptr(keep, scene.box, np.float32) if s.n_box else None
    s.narrow = int(getattr(scene, "narrow", 0))
    ob = _host(getattr(scene, "obb", np.zeros((0, 15))), np.float32).reshape(-1, 15)
    s.n_obb = int(ob.shape[0])
    s.obb = _keep_ptr(keep, ob, np.float32) if ob.size else None
    if sdf is not None:
        s.d_sdf = sdf.data_ptr()
        for a in range(3):
            s.sdf_dims[a] = int(sdf_spec.dims[a])
            s.sdf_origin[a] = float(sdf_spec.origin[a])
        s.voxel = float(sdf_spec.voxel)


def _fill_cost(c, cost, max_B, pair_filter=PAIRS_AUTO):
    c.K, c.M, c.interp, c.jp_mode, c.hinge = cost.K, cost.M, cost.interp, cost.jp_mode, cost.hinge
    c.margin, c.lambda_c, c.w_c, c.w_l = cost.margin, cost.lambda_c, cost.w_c, cost.w_l
    c.max_B = int(max_B)
    c.pair_filter = int(pair_filter)


def _fill_ik(k, par):
    k.lambda_q, k.lambda_c = float(par.lambda_q), float(par.lambda_c)
    k.lambda_e, k.lambda_r = float(par.lambda_e), float(par.lambda_r)
    k.max_iters, k.tau = int(par.max_iters), float(par.tau)
    k.eps_grad, k.eps_step = float(par.eps_grad), float(par.eps_step)
    k.clamp = int(par.clamp)


def _fill_opt(o, opt, problem_id=0):
    o.B, o.nu, o.sigma0, o.eps, o.seed = int(opt.B), int(opt.nu), float(opt.sigma0), float(opt.eps), int(opt.seed)
    o.problem_id = int(problem_id)
    o.polish_elites = int(getattr(opt, "polish_elites", 0))
    o.polish_steps = int(getattr(opt, "polish_steps", 0))
    o.polish_eta = float(getattr(opt, "polish_eta", 0.0))
    o.polish_clip = float(getattr(opt, "polish_clip", 1.0))


class Plan:
    """A crane, a scene and a path cost on one device (cp_plan_create)."""

    def __init__(self, robot, scene, cost, max_B: int, device: int = 0, sdf: Optional[torch.Tensor] = None,
                 sdf_spec=None, pair_filter: int = PAIRS_AUTO):
        L = lib()
        self._keep = []
        r, s, c = _Robot(), _Scene(), _Cost()
        _fill_robot(r, robot, self._keep)
        _fill_scene(s, scene, self._keep, sdf, sdf_spec)
        _fill_cost(c, cost, max_B, pair_filter)
        self.sdf = sdf
        h = ctypes.c_void_p()
        _check(L.cp_plan_create(ctypes.byref(r), ctypes.byref(s), ctypes.byref(c), int(device), ctypes.byref(h)))
        self._h = h
        self.device = torch.device("cuda", device)
        self.n_joints = r.n_joints
        self.n_spheres = r.n_spheres
        self.n_active = int(np.count_nonzero(_host(robot.active, np.uint8)))
        self.K = cost.K
        self.max_B = int(max_B)
        ns = _c_i32()
        _check(L.cp_plan_n_checkpoints(h, ctypes.byref(ns)))
        self.n_s = ns.value

    def close(self):
        if getattr(self, "_h", None):
            lib().cp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_endpoints(self, q_start, q_goal):
        qs = _host(q_start, np.float32)
        qg = _host(q_goal, np.float32)
        _check(lib().cp_plan_set_endpoints(self._h, qs.ctypes.data, qg.ctypes.data))

    def _w(self, W: torch.Tensor) -> torch.Tensor:
        if W.dtype != torch.float32 or W.dim() != 3 or W.shape[1] != self.K or W.shape[2] != self.n_joints:
            raise ValueError(f"waypoints must be float32 [B,{self.K},{self.n_joints}]")
        return W.contiguous()

    def eval(self, W: torch.Tensor, tape: bool = False):
        """cost [B], min_dist [B], flags [B] (and tape [B, n_s] if asked)."""
        W = self._w(W)
        B = W.shape[0]
        cost = torch.empty(B, dtype=torch.float32, device=W.device)
        md = torch.empty(B, dtype=torch.float32, device=W.device)
        fl = torch.empty(B, dtype=torch.uint8, device=W.device)
        tp = torch.empty((B, self.n_s), dtype=torch.int32, device=W.device) if tape else None
        _check(lib().cp_eval_paths(self._h, _ptr(W), B, _ptr(cost), _ptr(md), _ptr(fl), _ptr(tp), _stream()))
        return (cost, md, fl, tp) if tape else (cost, md, fl)

    def eval_into(self, W, cost, md, fl=None, tape=None):
        """Enqueue an evaluation into caller-provided buffers (no allocation)."""
        _check(lib().cp_eval_paths(self._h, _ptr(W), W.shape[0], _ptr(cost), _ptr(md), _ptr(fl), _ptr(tape),
                                   _stream()))

    def eval_noalloc_into(self, W, cost, md, fl=None, tape=None):
        """cp_eval_paths_noalloc: the evaluation into caller-provided buffers,
        with the library allocating nothing (static per-GPU scratch)."""
        _check(lib().cp_eval_paths_noalloc(self._h, _ptr(W), W.shape[0], _ptr(cost), _ptr(md), _ptr(fl), _ptr(tape),
                                           _stream()))

    def backward(self, W: torch.Tensor, grad_cost: torch.Tensor, tape: Optional[torch.Tensor] = None):
        """d(sum_b grad_cost[b] J_b) / dW, [B,K,n]."""
        W = self._w(W)
        g = torch.empty_like(W)
        gc = grad_cost.to(torch.float32).contiguous()
        _check(lib().cp_eval_paths_backward(self._h, _ptr(W), W.shape[0], _ptr(tape), _ptr(gc), _ptr(g), _stream()))
        return g

    def backward_into(self, W, grad_cost, grad_W, tape=None):
        _check(lib().cp_eval_paths_backward(self._h, _ptr(W), W.shape[0], _ptr(tape), _ptr(grad_cost),
                                            _ptr(grad_W), _stream()))

    def debug_fk(self, Q: torch.Tensor):
        Q = Q.to(torch.float32).contiguous()
        N = Q.shape[0]
        cen = torch.empty((N, self.n_spheres, 3), dtype=torch.float32, device=Q.device)
        fr = torch.empty((N, self.n_joints + 1, 12), dtype=torch.float32, device=Q.device)
        _check(lib().cp_debug_fk(self._h, _ptr(Q), N, _ptr(cen), _ptr(fr), _stream()))
        return cen, fr

    def debug_configs(self, Q: torch.Tensor):
        Q = Q.to(torch.float32).contiguous()
        N = Q.shape[0]
        d = torch.empty(N, dtype=torch.float32, device=Q.device)
        a = torch.empty(N, dtype=torch.int32, device=Q.device)
        _check(lib().cp_debug_eval_configs(self._h, _ptr(Q), N, _ptr(d), _ptr(a), _stream()))
        return d, a


    def _rows(self, a: torch.Tensor, N: int, width: int, name: str) -> torch.Tensor:
        if a.dtype != torch.float32 or a.shape != (N, width) or a.device != self.device:
            raise ValueError(f"{name} must be float32 [{N},{width}] on {self.device}")
        return a.contiguous()

    def ik_solve(self, params, target: torch.Tensor, q_init: torch.Tensor, q_ref: Optional[torch.Tensor] = None,
                 restarts: int = 1):
        """cp_ik_solve: (q [N,n], info [N,6], status [N], best [N/restarts])
        for targets [N,12] (R_d row-major, p_d), starts q_init [N,n] and
        regularisation references q_ref [N,n] (None: q_init)."""
        N = q_init.shape[0]
        n = self.n_joints
        target = self._rows(target, N, 12, "target")
        q_init = self._rows(q_init, N, n, "q_init")
        if q_ref is not None:
            q_ref = self._rows(q_ref, N, n, "q_ref")
        k = _Ik()
        _fill_ik(k, params)
        q = torch.empty((N, n), dtype=torch.float32, device=self.device)
        info = torch.empty((N, 6), dtype=torch.float32, device=self.device)
        status = torch.empty(N, dtype=torch.int32, device=self.device)
        best = torch.empty(max(1, N // int(restarts)), dtype=torch.int32, device=self.device)
        _check(lib().cp_ik_solve(self._h, ctypes.byref(k), _ptr(target), _ptr(q_init), _ptr(q_ref), N, int(restarts),
                                 _ptr(q), _ptr(info), _ptr(status), _ptr(best), _stream()))
        return q, info, status, best

    def ik_residual(self, params, target: torch.Tensor, q: torch.Tensor, q_ref: Optional[torch.Tensor] = None):
        """cp_debug_ik_residual: residual [N,8+n] and Jacobian [N,8+n,n]."""
        N = q.shape[0]
        n = self.n_joints
        target = self._rows(target, N, 12, "target")
        q = self._rows(q, N, n, "q")
        if q_ref is not None:
            q_ref = self._rows(q_ref, N, n, "q_ref")
        k = _Ik()
        _fill_ik(k, params)
        r = torch.empty((N, 8 + n), dtype=torch.float32, device=self.device)
        J = torch.empty((N, 8 + n, n), dtype=torch.float32, device=self.device)
        _check(lib().cp_debug_ik_residual(self._h, ctypes.byref(k), _ptr(target), _ptr(q), _ptr(q_ref), N, _ptr(r),
                                          _ptr(J), _stream()))
        return r, J


    def traj_refine(self, params, q_start: torch.Tensor, q_goal: torch.Tensor, q_star: torch.Tensor):
        """cp_traj_refine: states [P,N+1,2n], inputs [P,N+1,n_act], final
        times [P] and info [P,4] for P problems (q_start, q_goal [P,n], the
        step-one paths q_star [P,N+1,n]); the workspace is allocated here."""
        P = q_start.shape[0]
        n = self.n_joints
        N = int(params.N)
        q_start = self._rows(q_start, P, n, "q_start")
        q_goal = self._rows(q_goal, P, n, "q_goal")
        if q_star.dtype != torch.float32 or tuple(q_star.shape) != (P, N + 1, n) or q_star.device != self.device:
            raise ValueError(f"q_star must be float32 [{P},{N + 1},{n}] on {self.device}")
        q_star = q_star.contiguous()
        t = _Traj()
        _fill_traj(t, params, n)
        nbytes = ctypes.c_size_t()
        _check(lib().cp_traj_workspace_size(self._h, ctypes.byref(t), P, ctypes.byref(nbytes)))
        work = torch.empty(max(8, nbytes.value), dtype=torch.uint8, device=self.device)
        X = torch.empty((P, N + 1, 2 * n), dtype=torch.float32, device=self.device)
        U = torch.empty((P, N + 1, self.n_active), dtype=torch.float32, device=self.device)
        tf = torch.empty(P, dtype=torch.float32, device=self.device)
        info = torch.empty((P, 4), dtype=torch.float32, device=self.device)
        _check(lib().cp_traj_refine(self._h, ctypes.byref(t), _ptr(q_start), _ptr(q_goal), _ptr(q_star), P, _ptr(work),
                                    nbytes.value, _ptr(X), _ptr(U), _ptr(tf), _ptr(info), _stream()))
        return X, U, tf, info


class EvalPaths(torch.autograd.Function):
    """cost = J(W) with the hand-written adjoint as its backward; the argmin
    tape is saved, forward kinematics is recomputed in the backward pass."""

    @staticmethod
    def forward(ctx, W, plan):
        cost, md, fl, tape = plan.eval(W.detach(), tape=True)
        ctx.plan = plan
        ctx.save_for_backward(W.detach(), tape)
        ctx.mark_non_differentiable(md, fl)
        return cost, md, fl

    @staticmethod
    def backward(ctx, grad_cost, _g_md=None, _g_fl=None):
        W, tape = ctx.saved_tensors
        return ctx.plan.backward(W, grad_cost.contiguous(), tape), None


class Optimizer:
    """Algorithm 1 on a plan (cp_optimizer_create)."""

    def __init__(self, plan: Plan, opt, problem_id: int = 0):
        o = _Opt()
        _fill_opt(o, opt, problem_id)
        h = ctypes.c_void_p()
        _check(lib().cp_optimizer_create(plan._h, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.plan = plan
        self.B, self.nu = o.B, o.nu
        self.npol = o.polish_elites if o.polish_steps > 0 else 0
        self.D = plan.K * plan.n_active

    def close(self):
        if getattr(self, "_h", None):
            lib().cp_optimizer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n_iters: int = 1):
        _check(lib().cp_optimizer_step(self._h, int(n_iters), _stream()))

    def get_state(self):
        D = self.D
        mu = np.zeros(D)
        C = np.zeros((D, D))
        t = ctypes.c_int64()
        bc = ctypes.c_float()
        bw = np.zeros((self.plan.K, self.plan.n_joints), np.float32)
        rc = lib().cp_optimizer_get_state(self._h, mu.ctypes.data, C.ctypes.data, ctypes.byref(t), ctypes.byref(bc),
                                          bw.ctypes.data)
        _check(rc)
        return dict(mu=mu, C=C, t=t.value, best_cost=bc.value, best_W=bw)

    def set_state(self, mu, C, t: int):
        mu = _host(mu, np.float64)
        C = _host(C, np.float64)
        _check(lib().cp_optimizer_set_state(self._h, mu.ctypes.data, C.ctypes.data, int(t)))

    def last(self):
        dev = self.plan.device
        W = torch.empty((self.B, self.plan.K, self.plan.n_joints), dtype=torch.float32, device=dev)
        cost = torch.empty(self.B, dtype=torch.float32, device=dev)
        elite = torch.empty(self.nu, dtype=torch.int32, device=dev)
        _check(lib().cp_optimizer_last(self._h, _ptr(W), _ptr(cost), _ptr(elite), _stream()))
        return W, cost, elite

    def record_tape(self, enable: bool = True):
        """Record the argmin tape of every population evaluation (enables
        population_grad)."""
        _check(lib().cp_optimizer_record_tape(self._h, int(bool(enable))))

    def population_grad(self, out: Optional[torch.Tensor] = None):
        """d(sum_b J_b)/dW of the last population [B,K,n] (needs record_tape)."""
        if out is None:
            out = torch.empty((self.B, self.plan.K, self.plan.n_joints), dtype=torch.float32,
                              device=self.plan.device)
        _check(lib().cp_optimizer_population_grad(self._h, _ptr(out), _stream()))
        return out

    def time_eval(self, max_launches: int):
        """Bracket the next max_launches evaluation kernels of step() with HIP
        events (0: off)."""
        _check(lib().cp_optimizer_time_eval(self._h, int(max_launches)))

    def eval_time(self):
        """(total milliseconds, launches) of the evaluations timed since the
        last call."""
        ms = ctypes.c_double()
        n = _c_i32()
        _check(lib().cp_optimizer_eval_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def last_polished(self):
        """The last iteration's polished elites [polish_elites,K,n] (in the
        order of the selection before polish) and their costs."""
        dev = self.plan.device
        npol = self.npol
        W = torch.empty((npol, self.plan.K, self.plan.n_joints), dtype=torch.float32, device=dev)
        cost = torch.empty(npol, dtype=torch.float32, device=dev)
        _check(lib().cp_optimizer_last_polished(self._h, _ptr(W), _ptr(cost), _stream()))
        return W, cost

    def debug_update(self, elite: torch.Tensor):
        """Steps (4)-(6) alone on the last samples with the given elite indices
        (rank order), in place of the selection, after the polish of the
        first polish_elites of them if the optimizer polishes (tests)."""
        elite = elite.to(device=self.plan.device, dtype=torch.int32).contiguous()
        _check(lib().cp_debug_update(self._h, _ptr(elite), _stream()))

    def last_elites(self):
        """The last iteration's elite indices [nu] (rank order) and costs [B]."""
        dev = self.plan.device
        elite = torch.empty(self.nu, dtype=torch.int32, device=dev)
        cost = torch.empty(self.B, dtype=torch.float32, device=dev)
        _check(lib().cp_optimizer_last_elites(self._h, _ptr(elite), _ptr(cost), _stream()))
        return elite, cost


class _Tuning(ctypes.Structure):
    _fields_ = [("rounds", _c_i32), ("wg_per_cu", _c_i32)]


class Batch:
    """Independent problems run together (cp_batch_create): one persistent
    evaluation launch per iteration, iterations replayed from a HIP graph.
    ``problems`` are objects with robot, scene, cost, opt, q_start, q_goal;
    problem i uses Philox problem id i."""

    def __init__(self, problems, device: int = 0, pair_filter: int = PAIRS_AUTO):
        L = lib()
        n = len(problems)
        self._keep = []
        robots, scenes = (_Robot * n)(), (_Scene * n)()
        costs, opts = (_Cost * n)(), (_Opt * n)()
        for i, p in enumerate(problems):
            _fill_robot(robots[i], p.robot, self._keep)
            _fill_scene(scenes[i], p.scene, self._keep)
            _fill_cost(costs[i], p.cost, p.opt.B, pair_filter)
            _fill_opt(opts[i], p.opt, i)
        qs = _host(np.concatenate([np.asarray(p.q_start, np.float32) for p in problems]), np.float32)
        qg = _host(np.concatenate([np.asarray(p.q_goal, np.float32) for p in problems]), np.float32)
        h = ctypes.c_void_p()
        _check(L.cp_batch_create(n, robots, scenes, costs, opts, qs.ctypes.data, qg.ctypes.data, int(device),
                                 ctypes.byref(h)))
        self._h = h
        self.n = n
        self.shapes = [(p.cost.K, p.robot.n_joints, int(p.cost.K * int(np.count_nonzero(p.robot.active))))
                       for p in problems]
        self.pops = [(int(p.opt.B), int(p.opt.nu)) for p in problems]

    def close(self):
        if getattr(self, "_h", None):
            lib().cp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, n_iters: int):
        _check(lib().cp_batch_run(self._h, int(n_iters), _stream()))

    def eval(self):
        _check(lib().cp_batch_eval(self._h, _stream()))

    def get_state(self, p: int):
        K, n, D = self.shapes[p]
        mu = np.zeros(D)
        C = np.zeros((D, D))
        t = ctypes.c_int64()
        bc = ctypes.c_float()
        bw = np.zeros((K, n), np.float32)
        _check(lib().cp_batch_get_state(self._h, int(p), mu.ctypes.data, C.ctypes.data, ctypes.byref(t),
                                        ctypes.byref(bc), bw.ctypes.data))
        return dict(mu=mu, C=C, t=t.value, best_cost=bc.value, best_W=bw)

    def last(self, p: int, device: int = 0):
        """Problem p's last population: waypoints [B,K,n], costs [B], elite
        indices [nu] in rank order (cp_batch_last)."""
        K, n, _ = self.shapes[p]
        B, nu = self.pops[p]
        dev = torch.device("cuda", device)
        W = torch.empty((B, K, n), dtype=torch.float32, device=dev)
        cost = torch.empty(B, dtype=torch.float32, device=dev)
        elite = torch.empty(nu, dtype=torch.int32, device=dev)
        _check(lib().cp_batch_last(self._h, int(p), _ptr(W), _ptr(cost), _ptr(elite), _stream()))
        return W, cost, elite

    def set_tuning(self, rounds: int, wg_per_cu: int):
        t = _Tuning(int(rounds), int(wg_per_cu))
        _check(lib().cp_batch_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self):
        t = _Tuning()
        _check(lib().cp_batch_get_tuning(self._h, ctypes.byref(t)))
        return t.rounds, t.wg_per_cu

    def tune(self, cache_path: Optional[str] = None):
        t = _Tuning()
        path = cache_path.encode() if cache_path else None
        _check(lib().cp_batch_tune(self._h, path, ctypes.byref(t)))
        return t.rounds, t.wg_per_cu


def tune(plan: Optional["Plan"] = None, batch: Optional["Batch"] = None, cache_path: Optional[str] = None):
    """cp_tune: autotune a batch (a plan alone has no launch parameters to time)."""
    path = cache_path.encode() if cache_path else None
    _check(lib().cp_tune(plan._h if plan is not None else None, batch._h if batch is not None else None, path))


def select(cost: torch.Tensor, nu: int) -> torch.Tensor:
    """Indices of the nu smallest (cost, index) pairs in rank order, NaN as +inf
    (the selection step of the optimizer, exported for tests)."""
    cost = cost.to(torch.float32).contiguous()
    out = torch.empty(nu, dtype=torch.int32, device=cost.device)
    _check(lib().cp_debug_select(_ptr(cost), cost.shape[0], int(nu), _ptr(out), _stream()))
    return out


def sdf_build(points: torch.Tensor, spec, with_edt: bool = False):
    """Signed-distance grid [nz,ny,nx] from a device point cloud [N,3]."""
    nx, ny, nz = (int(v) for v in spec.dims)
    dev = points.device
    pts = points.to(torch.float32).contiguous()
    sdf = torch.empty((nz, ny, nx), dtype=torch.float32, device=dev)
    occ = eo = ef = None
    if with_edt:
        occ = torch.empty((nz, ny, nx), dtype=torch.uint8, device=dev)
        eo = torch.empty((nz, ny, nx), dtype=torch.int32, device=dev)
        ef = torch.empty((nz, ny, nx), dtype=torch.int32, device=dev)
    dims = np.array([nx, ny, nz], np.int32)
    org = np.array(spec.origin, np.float32)
    _check(lib().cp_sdf_build(_ptr(pts), pts.shape[0], dims.ctypes.data, org.ctypes.data, float(spec.voxel),
                              _ptr(sdf), _ptr(occ), _ptr(eo), _ptr(ef), _stream()))
    return (sdf, occ, eo, ef) if with_edt else sdf
