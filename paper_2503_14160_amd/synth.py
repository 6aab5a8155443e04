"""Seeded synthetic inputs for the crane path optimizer (input data only).

This module draws crane models, obstacle scenes, start/goal configurations and
lidar point clouds from integer seeds.  It holds none of the method's
arithmetic: no kinematics, no distance, no interpolation, no cost and no
optimizer step.  Both the HIP library and the CPU oracle take its arrays as
inputs, so the two sides always see the same (FP32-representable) numbers.

The paper's own crane (an 8-DOF Denavit-Hartenberg chain, Sec. 2), its 32
collision meshes (Fig. 2) and its two benchmark environments (Fig. 3) are not
published with it, so seeded stand-ins are drawn here:

* the crane is a 6-joint serial chain (slew, boom, arm, telescope and two
  passive grapple-swing joints held at 0) whose links carry bounding spheres;
* the scene is a forest of vertical cylinders (trees) plus axis-aligned boxes
  (log piles) and a ground plane, or a lidar cloud of such a forest that is
  turned into a signed-distance grid.

Every array is numpy, C-contiguous, float32 (int32/uint8 for indices/flags).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

REVOLUTE = 0
PRISMATIC = 1

INTERP_BSPLINE = 0
INTERP_LINEAR = 1
JP_SQUARED = 0
JP_L2 = 1
HINGE_HARD = 0
HINGE_SMOOTH = 1


@dataclasses.dataclass
class Robot:
    """A serial chain with link-bounding spheres.

    Joint j (0-based) moves frame j+1 relative to frame j: first a fixed
    translation ``origin[j]`` (in frame j), then a rotation about, or a
    translation along, the unit ``axis[j]``.  Frame 0 is the world.  Sphere s
    is rigidly attached to frame ``sphere_frame[s]`` (0..n) at local centre
    ``sphere_center[s]``.  ``tip`` is a point in the last frame.
    """

    joint_type: np.ndarray   # int32 [n]   REVOLUTE / PRISMATIC
    axis: np.ndarray         # f32 [n,3]
    origin: np.ndarray       # f32 [n,3]
    q_min: np.ndarray        # f32 [n]
    q_max: np.ndarray        # f32 [n]
    q_hold: np.ndarray       # f32 [n]  value of joints that are not sampled
    active: np.ndarray       # uint8 [n] 1 = sampled by the optimizer
    sphere_frame: np.ndarray   # int32 [S]
    sphere_center: np.ndarray  # f32 [S,3]
    sphere_radius: np.ndarray  # f32 [S]
    tip: np.ndarray          # f32 [3]
    link_lengths: np.ndarray  # f32 [5]  L1..L5 (column, boom, arm, telescope, hanger)
    # frame pairs whose spheres are checked against each other (self-collision);
    # empty: the environment only
    self_pairs: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 2), np.int32))
    # convex hulls of the links for the separating-axis narrow phase: oriented
    # boxes, row = centre (3), rotation (9, row-major, the box axes as its
    # columns), half extents (3), in the coordinates of frame hull_frame[k]
    hull_frame: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int32))
    hull_box: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 15), np.float32))

    @property
    def n_joints(self) -> int:
        return int(self.joint_type.shape[0])

    @property
    def n_spheres(self) -> int:
        return int(self.sphere_radius.shape[0])

    @property
    def n_active(self) -> int:
        return int(self.active.sum())


@dataclasses.dataclass
class Scene:
    """Obstacles.  ``cyl`` rows are (x, y, R, z0, z1): a vertical solid
    cylinder of radius R over z in [z0, z1].  ``box`` rows are
    (cx, cy, cz, hx, hy, hz): an axis-aligned solid box (centre, half sides).
    ``has_ground`` adds the half-space z <= ground_z."""

    cyl: np.ndarray          # f32 [Oc,5]
    box: np.ndarray          # f32 [Ob,6]
    has_ground: int = 1
    ground_z: float = 0.0
    # separating-axis narrow phase (narrow = 1): the robot's hulls against
    # these oriented boxes (rows as Robot.hull_box, world coordinates) and the
    # ground; cyl and box are then not used
    narrow: int = 0
    obb: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 15), np.float32))

    @property
    def n_cyl(self) -> int:
        return int(self.cyl.shape[0])

    @property
    def n_box(self) -> int:
        return int(self.box.shape[0])

    @property
    def n_obb(self) -> int:
        return int(self.obb.shape[0])


@dataclasses.dataclass
class SdfSpec:
    """A regular grid of voxels: dims (nx, ny, nz), lower corner ``origin``
    and edge ``voxel`` (metres).  Voxel (i, j, k) covers
    [origin + (i, j, k) * voxel, origin + (i+1, j+1, k+1) * voxel)."""

    dims: tuple
    origin: tuple
    voxel: float


@dataclasses.dataclass
class CostParams:
    K: int                   # free waypoints (control points that are optimised)
    M: int                   # checkpoints per spline span (or per linear segment)
    interp: int = INTERP_BSPLINE
    jp_mode: int = JP_SQUARED
    hinge: int = HINGE_HARD
    margin: float = 0.0
    lambda_c: float = 1.0
    w_c: float = 100.0
    w_l: float = 100.0

    @property
    def n_spans(self) -> int:
        return self.K + 3 if self.interp == INTERP_BSPLINE else self.K + 1

    @property
    def n_s(self) -> int:
        """Checkpoints per path, excluding the start point s_0 = 0."""
        return self.n_spans * self.M


@dataclasses.dataclass
class OptParams:
    B: int                   # population (paths per iteration)
    nu: int                  # elites
    sigma0: float            # initial standard deviation of every sampled dimension
    eps: float               # covariance regulariser
    seed: int                # RNG key
    T: int                   # iterations
    polish_elites: int = 0
    polish_steps: int = 0
    polish_eta: float = 1e-3
    polish_clip: float = 10.0


@dataclasses.dataclass
class IkParams:
    """Weights and solver settings of the collision-free IK (Sec. 3.2): the
    residual is [p_g - p_d, lambda_q Log(R_d^T R_g), lambda_c ReLU(-d(q)),
    lambda_e |g_p|^2, lambda_r (q - q_ref)], minimised by Levenberg-Marquardt
    (``max_iters`` trial steps, initial damping ``tau`` max diag(J^T J),
    stops on max |J^T r| <= eps_grad or |h| <= eps_step (|q| + eps_step);
    ``clamp`` keeps q within the joint limits)."""

    lambda_q: float = 1.0
    lambda_c: float = 10.0
    lambda_e: float = 1.0
    lambda_r: float = 1e-2
    max_iters: int = 50
    tau: float = 1e-3
    eps_grad: float = 1e-6
    eps_step: float = 1e-7
    clamp: int = 1


@dataclasses.dataclass
class TrajParams:
    """Step two of the planner (Sec. 4.2, eq. discrete): direct collocation
    with trapezoidal defects over N intervals of the reduced dynamics (Sec.
    2.1: the actuated joints' accelerations are the inputs, the passive
    joints follow a unit load at the tip, with viscous damping ``damping``
    1/s on them), minimising t_F + omega_s sum |u_k|^2 + omega_t sum
    |q_a,k - q*_a,k|^2 from rest at q_0 to rest at q_d, within the joint
    limits and |qd_j| <= v_max[j].  Solved by an augmented Lagrangian on the
    defects (penalty ``mu0``, times ``mu_factor`` per outer iteration,
    ``outer`` of them; the state bounds as quadratic penalties of the same
    weight) around Levenberg-Marquardt (``max_iters`` trial steps per outer
    iteration, initial damping ``tau`` max diag(J^T J), stops on
    max |J^T r| <= eps_grad or |h| <= eps_step (|z| + eps_step)); t_F = s^2
    with s the unknown, kept above t_min = max_j |q_d,j - q_0,j| / v_max[j]
    (a bound the velocity limits imply) by one more penalty, and started at
    max(t_f0, t_min).  Jacobians of the dynamics by central differences
    (steps fd_q on positions, 1 on velocities and inputs, where the
    accelerations are quadratic and linear).  The defaults reach defects
    near 1e-12 at N = 100 on the crane's moves."""

    N: int = 100
    omega_s: float = 0.1
    omega_t: float = 10.0
    grav: float = 9.81
    damping: float = 0.5
    v_max: tuple = (0.6, 0.4, 0.4, 0.5, 2.0, 2.0)
    mu0: float = 1e3
    mu_factor: float = 10.0
    outer: int = 5
    max_iters: int = 60
    tau: float = 1e-6
    eps_grad: float = 1e-9
    eps_step: float = 1e-12
    fd_q: float = 1e-5
    t_f0: float = 12.0


@dataclasses.dataclass
class IkProblem:
    """Batched IK: the tip poses of the configurations ``q_star`` [N,n] are the
    targets; ``q_init`` [N*R,n] holds R starting configurations per target
    (rows i*R .. i*R+R-1 belong to target i); ``q_ref`` [n] is the crane's
    current configuration (regularisation).  As drawn, ``q_star`` holds
    candidate configurations, more than ``n_targets``; a workload is the first
    ``n_targets`` of them whose grasp pose is clear of the scene (``pick``),
    clearance being judged by whoever uses the workload."""

    name: str
    robot: Robot
    scene: Scene
    q_star: np.ndarray
    q_init: np.ndarray
    q_ref: np.ndarray
    restarts: int
    params: IkParams
    n_targets: int = 0

    def pick(self, clear: np.ndarray) -> "IkProblem":
        """The first ``n_targets`` candidates with ``clear`` set (a boolean per
        candidate) and their starting configurations."""
        idx = np.flatnonzero(np.asarray(clear, bool))[: self.n_targets]
        if len(idx) < self.n_targets:
            raise ValueError(f"only {len(idx)} clear candidates for {self.n_targets} targets")
        n = self.robot.n_joints
        q_init = self.q_init.reshape(-1, self.restarts, n)[idx].reshape(-1, n)
        return dataclasses.replace(self, q_star=self.q_star[idx], q_init=np.ascontiguousarray(q_init))


@dataclasses.dataclass
class Problem:
    name: str
    robot: Robot
    scene: Scene
    q_start: np.ndarray      # f32 [n]
    q_goal: np.ndarray       # f32 [n]
    cost: CostParams
    opt: OptParams
    sdf: Optional[SdfSpec] = None
    lidar: Optional[np.ndarray] = None  # f32 [N,3]


# ----------------------------------------------------------------------------
# crane
# ----------------------------------------------------------------------------

def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def make_robot(seed: int, n_spheres: int) -> Robot:
    """The 6-joint synthetic forestry crane.

    Joints: slew (revolute +z at the base), boom (revolute -y, offset L1 up
    the column), arm (revolute -y, offset L2 along the boom), telescope
    (prismatic +x, offset L3 along the arm, 0..3 m), and two passive swing
    joints (revolute +x at offset L4, revolute +y) that are held at 0.  Link
    lengths are U(2, 5) m.  Spheres of radius U(0.15, 0.4) m are spread over
    the five link segments in proportion to segment length (largest
    remainder, at least one each), centred at (i + 1/2)/n along a segment.
    """
    if n_spheres < 5:
        raise ValueError("need at least one sphere per link segment (5)")
    rng = np.random.default_rng(seed)
    L = _f32(rng.uniform(2.0, 5.0, size=5))
    L1, L2, L3, L4, L5 = (float(x) for x in L)
    joint_type = np.array([REVOLUTE, REVOLUTE, REVOLUTE, PRISMATIC, REVOLUTE, REVOLUTE], np.int32)
    axis = _f32([[0, 0, 1], [0, -1, 0], [0, -1, 0], [1, 0, 0], [1, 0, 0], [0, 1, 0]])
    origin = _f32([[0, 0, 0], [0, 0, L1], [L2, 0, 0], [L3, 0, 0], [L4, 0, 0], [0, 0, 0]])
    q_min = _f32([-math.pi, -0.2, -2.4, 0.0, -math.pi / 2, -math.pi / 2])
    q_max = _f32([math.pi, 1.2, 0.4, 3.0, math.pi / 2, math.pi / 2])
    q_hold = _f32([0, 0, 0, 0, 0, 0])
    active = np.array([1, 1, 1, 1, 0, 0], np.uint8)

    # segments: (frame, start point, end point) in that frame
    col0 = 1.0
    segs = [
        (1, (0.0, 0.0, col0), (0.0, 0.0, L1)),
        (2, (0.0, 0.0, 0.0), (L2, 0.0, 0.0)),
        (3, (0.0, 0.0, 0.0), (L3, 0.0, 0.0)),
        (4, (0.0, 0.0, 0.0), (L4, 0.0, 0.0)),
        (6, (0.0, 0.0, 0.0), (0.0, 0.0, -L5)),
    ]
    lens = np.array([L1 - col0, L2, L3, L4, L5], np.float64)
    quota = n_spheres * lens / lens.sum()
    counts = np.maximum(np.floor(quota).astype(np.int64), 1)
    while counts.sum() < n_spheres:
        frac = quota - counts
        counts[int(np.argmax(frac))] += 1
    while counts.sum() > n_spheres:
        cand = np.where(counts > 1)[0]
        counts[cand[int(np.argmax(counts[cand] - quota[cand]))]] -= 1
    frames, centers = [], []
    for (f, a, b), n in zip(segs, counts):
        a = np.array(a)
        b = np.array(b)
        for i in range(int(n)):
            frames.append(f)
            centers.append(a + (i + 0.5) / n * (b - a))
    radius = _f32(rng.uniform(0.15, 0.4, size=n_spheres))
    return Robot(joint_type=joint_type, axis=axis, origin=origin, q_min=q_min, q_max=q_max,
                 q_hold=q_hold, active=active,
                 sphere_frame=np.array(frames, np.int32), sphere_center=_f32(centers),
                 sphere_radius=radius, tip=_f32([0.0, 0.0, -L5]), link_lengths=L)


def crane_self_pairs(robot: Robot) -> np.ndarray:
    """Frame pairs of the crane's links that are not adjacent: the sphere-
    carrying frames in chain order are the column (1), boom (2), arm (3),
    telescope (4) and hanger (6, joined to the telescope through the
    sphere-less frame 5); links next to each other in that order share a
    joint and are not checked."""
    frames = sorted(set(int(f) for f in robot.sphere_frame if f > 0))
    pairs = [(a, b) for i, a in enumerate(frames) for b in frames[i + 2:]]
    return np.array(pairs, np.int32).reshape(-1, 2)


def with_self_collision(robot: Robot) -> Robot:
    """The same crane with its non-adjacent link pairs checked for
    self-collision."""
    return dataclasses.replace(robot, self_pairs=crane_self_pairs(robot))


def _obb_row(c, R, h) -> np.ndarray:
    return np.concatenate([np.asarray(c, np.float64), np.asarray(R, np.float64).reshape(9),
                           np.asarray(h, np.float64)])


def with_hulls(robot: Robot) -> Robot:
    """The crane with one oriented box per link segment for the
    separating-axis narrow phase: the segment's extent along its own
    direction plus, across it and beyond its ends, the largest radius of the
    segment's spheres (the box holds every sphere of the segment).  Segments
    run along a frame axis, so each box's axes are its frame's."""
    L1, L2, L3, L4, L5 = (float(x) for x in robot.link_lengths)
    segs = [(1, (0.0, 0.0, 1.0), (0.0, 0.0, L1)), (2, (0.0, 0.0, 0.0), (L2, 0.0, 0.0)),
            (3, (0.0, 0.0, 0.0), (L3, 0.0, 0.0)), (4, (0.0, 0.0, 0.0), (L4, 0.0, 0.0)),
            (6, (0.0, 0.0, 0.0), (0.0, 0.0, -L5))]
    frames, rows = [], []
    for f, a, b in segs:
        a, b = np.array(a), np.array(b)
        r = float(robot.sphere_radius[robot.sphere_frame == f].max())
        h = np.abs(b - a) / 2.0 + r
        frames.append(f)
        rows.append(_obb_row((a + b) / 2.0, np.eye(3), h))
    return dataclasses.replace(robot, hull_frame=np.array(frames, np.int32), hull_box=_f32(rows))


def hull_scene(rng: np.random.Generator, scene: Scene) -> Scene:
    """The scene's obstacles as oriented boxes for the separating-axis narrow
    phase: a tree of radius R over [z0, z1] becomes an upright square prism
    of half width R turned about z by an angle U(0, pi/2); a log pile keeps
    its box."""
    rows = []
    for x, y, R, z0, z1 in scene.cyl.astype(np.float64):
        t = rng.uniform(0.0, math.pi / 2)
        c, s = math.cos(t), math.sin(t)
        rows.append(_obb_row((x, y, 0.5 * (z0 + z1)), [[c, -s, 0], [s, c, 0], [0, 0, 1]], (R, R, 0.5 * (z1 - z0))))
    for cx, cy, cz, hx, hy, hz in scene.box.astype(np.float64):
        rows.append(_obb_row((cx, cy, cz), np.eye(3), (hx, hy, hz)))
    return dataclasses.replace(scene, narrow=1, obb=_f32(np.array(rows).reshape(-1, 15)))


def make_endpoints(rng: np.random.Generator, robot: Robot):
    """Start and goal configurations.

    The slew angles lie in [-0.9 pi, 0.9 pi] and differ by at least pi/2, so
    a path has to sweep through the forest.  Boom angle U(0.75, 1.15) rad, arm
    pitch relative to the horizon (boom + arm angle) U(0.25, 0.6) rad,
    telescope U(0.5, 2.7) m; passive joints at their hold value.
    """
    while True:
        s1, g1 = rng.uniform(-0.9 * math.pi, 0.9 * math.pi, size=2)
        if abs(g1 - s1) >= math.pi / 2:
            break
    out = []
    for q1 in (s1, g1):
        q2 = rng.uniform(0.75, 1.15)
        alpha = rng.uniform(0.25, 0.6)
        q4 = rng.uniform(0.5, 2.7)
        q = np.array(robot.q_hold, np.float64)
        q[0], q[1], q[2], q[3] = q1, q2, alpha - q2, q4
        out.append(_f32(q))
    return out[0], out[1]


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------

def _ray_clearance(px: float, py: float, angles) -> float:
    """2-D distance from (px, py) to the nearest of the rays from the origin
    at the given azimuths (used to keep obstacles off the start and goal
    poses, which lie in the vertical half-plane at their slew angle)."""
    best = math.inf
    for th in angles:
        ux, uy = math.cos(th), math.sin(th)
        t = max(0.0, px * ux + py * uy)
        best = min(best, math.hypot(px - t * ux, py - t * uy))
    return best


def make_scene(rng: np.random.Generator, robot: Robot, q_start, q_goal, n_cyl: int, n_box: int,
               half_extent: float, r_range=(0.1, 0.5), height=15.0, box_side=(1.0, 6.0)) -> Scene:
    """Trees and log piles on a square of side 2*half_extent around the base.

    Tree radius U(r_range), z in [0, height]; box sides U(box_side) per axis,
    resting on the ground.  An obstacle is redrawn if its footprint comes
    within 1.5 m of the base axis, or within (largest sphere radius + 0.15 m)
    of the vertical half-planes that hold the start and goal poses.
    """
    r_max = float(robot.sphere_radius.max())
    angles = (float(q_start[0]), float(q_goal[0]))

    def ok(x, y, rad):
        if math.hypot(x, y) < rad + 1.5:
            return False
        return _ray_clearance(x, y, angles) >= rad + r_max + 0.15

    cyl = []
    while len(cyl) < n_cyl:
        x, y = rng.uniform(-half_extent, half_extent, size=2)
        R = rng.uniform(*r_range)
        if ok(x, y, R):
            cyl.append((x, y, R, 0.0, height))
    box = []
    while len(box) < n_box:
        x, y = rng.uniform(-half_extent, half_extent, size=2)
        h = rng.uniform(*box_side, size=3) / 2
        if ok(x, y, math.hypot(h[0], h[1])):
            box.append((x, y, h[2], h[0], h[1], h[2]))
    cyl_a = _f32(cyl).reshape(-1, 5)
    box_a = _f32(box).reshape(-1, 6)
    return Scene(cyl=cyl_a, box=box_a, has_ground=1, ground_z=0.0)


def make_lidar(rng: np.random.Generator, trees: np.ndarray, n_points: int, spec: SdfSpec,
               ground_frac=0.4, noise=0.05, z_top=12.4) -> np.ndarray:
    """A synthetic lidar cloud: a fraction ``ground_frac`` of the points on the
    ground (x, y uniform over the grid footprint, z ~ N(0, noise)) and the rest
    on tree trunk surfaces (tree chosen with probability proportional to its
    radius, angle U(0, 2 pi), height U(0, z_top), radius R + N(0, noise))."""
    n_ground = int(round(ground_frac * n_points))
    n_trunk = n_points - n_ground
    ox, oy, _ = spec.origin
    nx, ny, _ = spec.dims
    gx = rng.uniform(ox, ox + nx * spec.voxel, size=n_ground)
    gy = rng.uniform(oy, oy + ny * spec.voxel, size=n_ground)
    gz = rng.normal(0.0, noise, size=n_ground)
    p = trees[:, 2].astype(np.float64)
    which = rng.choice(trees.shape[0], size=n_trunk, p=p / p.sum())
    th = rng.uniform(0.0, 2 * math.pi, size=n_trunk)
    z = rng.uniform(0.0, z_top, size=n_trunk)
    r = trees[which, 2] + rng.normal(0.0, noise, size=n_trunk)
    tx = trees[which, 0] + r * np.cos(th)
    ty = trees[which, 1] + r * np.sin(th)
    pts = np.concatenate([np.stack([gx, gy, gz], 1), np.stack([tx, ty, z], 1)], 0)
    pts = pts[rng.permutation(n_points)]
    return _f32(pts)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

ROBOT_SEED = 1000
SCENE_SEED = 2000
RNG_SEED = 3000


def c0_plain() -> Problem:
    """256 paths x 8 waypoints x 16 points per span, 24 spheres, 32 trees in a
    20 x 20 m square plus ground, 10 % elites, 20 iterations, sigma 0.2 rad."""
    robot = make_robot(ROBOT_SEED + 0, 24)
    rng = np.random.default_rng(SCENE_SEED + 0)
    qs, qg = make_endpoints(rng, robot)
    scene = make_scene(rng, robot, qs, qg, n_cyl=32, n_box=0, half_extent=10.0, r_range=(0.1, 0.4))
    cost = CostParams(K=8, M=16)
    opt = OptParams(B=256, nu=25, sigma0=0.2, eps=1e-6, seed=RNG_SEED + 0, T=20)
    return Problem("c0_plain", robot, scene, qs, qg, cost, opt)


def c1_full() -> Problem:
    """16384 paths x 16 waypoints x 32 points per span, 64 spheres, 512 trees
    and 16 log piles in a 40 x 40 m square plus ground, 5 % elites, 50
    iterations."""
    robot = make_robot(ROBOT_SEED + 1, 64)
    rng = np.random.default_rng(SCENE_SEED + 1)
    qs, qg = make_endpoints(rng, robot)
    scene = make_scene(rng, robot, qs, qg, n_cyl=512, n_box=16, half_extent=20.0)
    cost = CostParams(K=16, M=32)
    opt = OptParams(B=16384, nu=819, sigma0=0.2, eps=1e-6, seed=RNG_SEED + 1, T=50)
    return Problem("c1_full", robot, scene, qs, qg, cost, opt)


def c2_diff() -> Problem:
    """The c1_full crane and scene with a smooth hinge (margin 0.1 m), 1024
    paths, 64 elites, and 50 gradient-polish steps on the elites."""
    base = c1_full()
    cost = CostParams(K=16, M=32, hinge=HINGE_SMOOTH, margin=0.1)
    opt = OptParams(B=1024, nu=64, sigma0=0.2, eps=1e-6, seed=RNG_SEED + 2, T=20,
                    polish_elites=64, polish_steps=50, polish_eta=1e-3, polish_clip=10.0)
    return Problem("c2_diff", base.robot, base.scene, base.q_start, base.q_goal, cost, opt)


def c3_batch(n_problems: int = 256) -> List[Problem]:
    """Independent problems of uneven size: paths U{512..8192}, waypoints
    U{8..24}, obstacles U{64..1024} (one box per 32), each with its own crane
    seed offset, start and goal; 16 points per span, 64 spheres, 5 % elites,
    30 iterations."""
    out = []
    meta = np.random.default_rng(SCENE_SEED + 3)
    for p in range(n_problems):
        B = int(meta.integers(512, 8193))
        K = int(meta.integers(8, 25))
        O = int(meta.integers(64, 1025))
        robot = make_robot(ROBOT_SEED + 3 + 7919 * (p + 1), 64)
        rng = np.random.default_rng(SCENE_SEED + 3 + 7919 * (p + 1))
        qs, qg = make_endpoints(rng, robot)
        nb = O // 32
        scene = make_scene(rng, robot, qs, qg, n_cyl=O - nb, n_box=nb, half_extent=20.0)
        cost = CostParams(K=K, M=16)
        opt = OptParams(B=B, nu=max(1, int(0.05 * B)), sigma0=0.2, eps=1e-6,
                        seed=RNG_SEED + 3 + 7919 * (p + 1), T=30)
        out.append(Problem(f"c3_batch[{p}]", robot, scene, qs, qg, cost, opt))
    return out


C4_SPEC = SdfSpec(dims=(256, 256, 128), origin=(-12.8, -12.8, -0.4), voxel=0.1)


def c4_sdf(n_points: int = 1_000_000) -> Problem:
    """A 1 M-point lidar cloud of 64 trees and the ground, to be turned into a
    256 x 256 x 128 signed-distance grid at 0.1 m; 65536 paths x 16 waypoints
    x 32 points per span, 64 spheres, smooth hinge, 50 iterations."""
    robot = make_robot(ROBOT_SEED + 4, 64)
    rng = np.random.default_rng(SCENE_SEED + 4)
    qs, qg = make_endpoints(rng, robot)
    trees = make_scene(rng, robot, qs, qg, n_cyl=64, n_box=0, half_extent=12.0, height=12.4)
    lidar = make_lidar(rng, trees.cyl, n_points, C4_SPEC)
    cost = CostParams(K=16, M=32, hinge=HINGE_SMOOTH, margin=0.1)
    opt = OptParams(B=65536, nu=3276, sigma0=0.2, eps=1e-6, seed=RNG_SEED + 4, T=50)
    scene = Scene(cyl=_f32(np.zeros((0, 5))), box=_f32(np.zeros((0, 6))), has_ground=0)
    return Problem("c4_sdf", robot, scene, qs, qg, cost, opt, sdf=C4_SPEC, lidar=lidar)


def hanging_configs(rng: np.random.Generator, robot: Robot, N: int) -> np.ndarray:
    """N crane configurations [N,n] with the grapple hanging at rest: slew
    U(-pi, pi), boom U(0.2, 1.1) rad, arm pitch relative to the horizon
    alpha = boom + arm U(-0.4, 0.5) rad, telescope U(0.2, 2.8) m, first swing
    joint 0 and second swing joint alpha (the hanger then points straight
    down, where a weight at its end exerts no torque on either swing joint)."""
    q = np.zeros((N, robot.n_joints), np.float64)
    q[:, 0] = rng.uniform(-math.pi, math.pi, size=N)
    q[:, 1] = rng.uniform(0.2, 1.1, size=N)
    alpha = rng.uniform(-0.4, 0.5, size=N)
    q[:, 2] = alpha - q[:, 1]
    q[:, 3] = rng.uniform(0.2, 2.8, size=N)
    q[:, 4] = 0.0
    q[:, 5] = alpha
    return _f32(q)


def ik_c1(n_targets: int = 1024, restarts: int = 8, oversample: int = 24) -> IkProblem:
    """Batched collision-free IK on the c1_full crane (with its non-adjacent
    link pairs checked for self-collision) and forest: ``oversample`` times
    ``n_targets`` candidate hanging configurations, whose grasp poses are the
    targets once the clear ones are picked (about 8 % of them keep 0.1 m from
    every tree, log pile and link of the crane), ``restarts`` starting points
    each (the crane's start configuration, then configurations uniform
    within the joint limits with the swing joints at 0)."""
    base = c1_full()
    robot = with_self_collision(base.robot)
    rng = np.random.default_rng(SCENE_SEED + 5)
    n_cand = n_targets * oversample
    q_star = hanging_configs(rng, robot, n_cand)
    q_init = np.empty((n_cand, restarts, robot.n_joints), np.float64)
    q_init[:, 0, :] = base.q_start
    lo = robot.q_min.astype(np.float64)
    hi = robot.q_max.astype(np.float64)
    q_init[:, 1:, :] = rng.uniform(lo, hi, size=(n_cand, restarts - 1, robot.n_joints))
    q_init[:, 1:, 4:] = 0.0
    return IkProblem("ik_c1", robot, base.scene, q_star, _f32(q_init.reshape(-1, robot.n_joints)),
                     _f32(base.q_start), restarts, IkParams(), n_targets=n_targets)


# clearance of a grasp pose's configuration from the scene and the crane itself (m)
IK_TARGET_CLEARANCE = 0.1


def traj_problems(robot: Robot, P: int, N: int, seed: int):
    """P step-two problems: start/goal pairs (hanging configurations, then a
    slew of U(-0.8, 0.8) rad, a boom move of U(-0.15, 0.15) rad and a
    telescope move of U(-0.5, 0.5) m clipped to [0.1, 2.9], the grapple
    kept hanging) and bent paths between them sampled at s = k / N: the
    straight line plus a smooth bump of 0.1 sin(pi s) rad on the boom, as a
    step-one path bends over an obstacle.  float32 [P, n], [P, n],
    [P, N+1, n]."""
    rng = np.random.default_rng(seed)
    q0 = hanging_configs(rng, robot, P).astype(np.float64)
    qg = q0.copy()
    qg[:, 0] += rng.uniform(-0.8, 0.8, P)
    qg[:, 1] += rng.uniform(-0.15, 0.15, P)
    qg[:, 3] = np.clip(qg[:, 3] + rng.uniform(-0.5, 0.5, P), 0.1, 2.9)
    qg[:, 5] = qg[:, 1] + qg[:, 2]
    s = np.linspace(0.0, 1.0, N + 1)
    qstar = q0[:, None, :] + s[None, :, None] * (qg - q0)[:, None, :]
    qstar[:, :, 1] += 0.1 * np.sin(np.pi * s)[None, :]
    return _f32(q0), _f32(qg), _f32(qstar)


WORKLOADS = {"c0_plain": c0_plain, "c1_full": c1_full, "c2_diff": c2_diff, "c4_sdf": c4_sdf}


# ----------------------------------------------------------------------------
# generic random inputs for tests
# ----------------------------------------------------------------------------

def random_waypoints(rng: np.random.Generator, robot: Robot, q_start, q_goal, B: int, K: int,
                     sigma: float = 0.2) -> np.ndarray:
    """B paths of K waypoints [B,K,n]: evenly spaced points on the segment
    from start to goal plus N(0, sigma^2) noise on the active joints."""
    n = robot.n_joints
    t = (np.arange(K, dtype=np.float64) + 1.0) / (K + 1.0)
    base = q_start[None, :].astype(np.float64) + t[:, None] * (q_goal - q_start)[None, :].astype(np.float64)
    W = np.broadcast_to(base, (B, K, n)).copy()
    act = robot.active.astype(bool)
    W[:, :, act] += rng.normal(0.0, sigma, size=(B, K, int(act.sum())))
    W[:, :, ~act] = robot.q_hold[~act]
    return _f32(W)


def random_configs(rng: np.random.Generator, robot: Robot, N: int, margin: float = 0.2) -> np.ndarray:
    """N joint vectors [N,n] uniform in the joint limits widened by ``margin``."""
    lo = robot.q_min.astype(np.float64) - margin
    hi = robot.q_max.astype(np.float64) + margin
    return _f32(rng.uniform(lo, hi, size=(N, robot.n_joints)))
