"""Pins of the oracle's separating-axis narrow phase on oriented boxes (Sec. 3.1).

The SAT distance of two boxes is checked against closed forms for
axis-aligned boxes, against the exact Euclidean distance from a
bound-constrained least-squares solve (never above it; equal when a face
separates them), against the largest projection gap over thousands of random
directions (for intersecting boxes the best of the fifteen axes is the
largest gap over all directions), for symmetry and rigid-motion invariance;
the configuration distance against an explicit enumeration, the hulls
against the forward kinematics and against the link spheres they hold.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.spatial.transform import Rotation

from paper_2503_14160_amd import synth


def _box(c, R, h):
    return np.concatenate([np.asarray(c, float), np.asarray(R, float).reshape(9), np.asarray(h, float)])


def _parts(b):
    return b[:3], b[3:12].reshape(3, 3), b[12:15]


def _exact_distance(a, b):
    """min |x - y| over x in box a, y in box b (convex; bound-constrained)."""
    ca, Ra, ha = _parts(a)
    cb, Rb, hb = _parts(b)
    Ma, Mb = Ra * ha, Rb * hb

    def f(z):
        r = ca + Ma @ z[:3] - cb - Mb @ z[3:]
        return float(r @ r), np.concatenate([2 * Ma.T @ r, -2 * Mb.T @ r])

    best = math.inf
    for z0 in (np.zeros(6), np.full(6, 0.5), np.full(6, -0.5)):
        res = minimize(f, z0, jac=True, method="L-BFGS-B", bounds=[(-1, 1)] * 6,
                       options=dict(ftol=1e-15, gtol=1e-12, maxiter=2000))
        best = min(best, res.fun)
    return math.sqrt(max(best, 0.0))


def _gap(a, b, n):
    ca, Ra, ha = _parts(a)
    cb, Rb, hb = _parts(b)
    return abs((cb - ca) @ n) - np.abs(Ra.T @ n) @ ha - np.abs(Rb.T @ n) @ hb


def _random_box(rng, spread=2.0):
    return _box(rng.uniform(-spread, spread, 3), Rotation.random(random_state=rng).as_matrix(),
                rng.uniform(0.2, 1.5, 3))


def test_axis_aligned_closed_form(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        ca, cb = rng.uniform(-3, 3, 3), rng.uniform(-3, 3, 3)
        ha, hb = rng.uniform(0.1, 2, 3), rng.uniform(0.1, 2, 3)
        a, b = _box(ca, np.eye(3), ha), _box(cb, np.eye(3), hb)
        g = np.abs(cb - ca) - ha - hb
        # parallel edges contribute no cross axis; the face axes give the per-axis gaps
        assert orc.sat_obb(a, b) == pytest.approx(g.max(), abs=1e-12)
        if g.max() > 0 and (g > 0).sum() == 1:
            assert orc.sat_obb(a, b) == pytest.approx(_exact_distance(a, b), abs=1e-7)


def test_symmetry_and_rigid_motion(orc):
    rng = np.random.default_rng(2)
    for _ in range(100):
        a, b = _random_box(rng), _random_box(rng)
        d = orc.sat_obb(a, b)
        assert orc.sat_obb(b, a) == pytest.approx(d, abs=1e-12)
        Q = Rotation.random(random_state=rng).as_matrix()
        t = rng.uniform(-10, 10, 3)

        def move(x):
            c, R, h = _parts(x)
            return _box(Q @ c + t, Q @ R, h)
        assert orc.sat_obb(move(a), move(b)) == pytest.approx(d, abs=1e-11)


def test_never_above_the_exact_distance_and_positive_only_when_disjoint(orc):
    rng = np.random.default_rng(3)
    n_sep = n_int = 0
    for _ in range(150):
        a, b = _random_box(rng, 2.5), _random_box(rng, 2.5)
        d = orc.sat_obb(a, b)
        ex = _exact_distance(a, b)
        assert d <= ex + 1e-7, (d, ex)
        if d > 1e-6:
            assert ex > 0
            n_sep += 1
        if ex < 1e-9:
            assert d <= 1e-9
            n_int += 1
    assert n_sep >= 20 and n_int >= 20


def test_face_separation_is_exact(orc):
    """B beyond A's +a_k face with its lowest point along a_k at gap g and its
    projection inside the face: the distance is g, and so is the SAT value."""
    rng = np.random.default_rng(4)
    for _ in range(60):
        RA = Rotation.random(random_state=rng).as_matrix()
        ha = rng.uniform(1.0, 2.0, 3)
        k = int(rng.integers(3))
        RB = Rotation.random(random_state=rng).as_matrix()
        hb = rng.uniform(0.05, 0.3, 3)
        g = rng.uniform(0.01, 1.0)
        ext = np.abs(RB.T @ RA[:, k]) @ hb  # B's half-width along a_k
        cb_local = rng.uniform(-0.4, 0.4, 3) * ha
        cb_local[k] = ha[k] + g + ext
        a = _box(np.zeros(3), RA, ha)
        b = _box(RA @ cb_local, RB, hb)
        assert orc.sat_obb(a, b) == pytest.approx(g, abs=1e-12)
        assert _exact_distance(a, b) == pytest.approx(g, abs=1e-6)


def test_intersecting_value_is_the_largest_gap_over_all_directions(orc):
    rng = np.random.default_rng(5)
    dirs = rng.normal(size=(20000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    n_done = 0
    for _ in range(60):
        a, b = _random_box(rng, 0.8), _random_box(rng, 0.8)
        d = orc.sat_obb(a, b)
        if d >= 0:
            continue
        n_done += 1
        ca, Ra, ha = _parts(a)
        cb, Rb, hb = _parts(b)
        gaps = np.abs(dirs @ (cb - ca)) - np.abs(dirs @ Ra) @ ha - np.abs(dirs @ Rb) @ hb
        # no direction separates more than the best candidate axis ...
        assert gaps.max() <= d + 1e-12
        # ... and directions near it come close (sampling resolution ~ 0.03 rad)
        assert gaps.max() >= d - 0.15 * (ha.sum() + hb.sum() + np.linalg.norm(cb - ca))
    assert n_done >= 20


def _sat_crane(orc, n_obb=40, seed=6):
    base = synth.c1_full()
    robot = synth.with_self_collision(synth.with_hulls(base.robot))
    rng = np.random.default_rng(seed)
    scene = synth.hull_scene(rng, dataclasses.replace(base.scene, cyl=base.scene.cyl[:n_obb], box=base.scene.box[:4]))
    return robot, scene, orc.Model(robot, scene, None)


def test_hulls_follow_the_frames_and_hold_the_link_spheres(orc):
    robot, scene, m = _sat_crane(orc)
    plain = orc.Model(synth.with_hulls(synth.c1_full().robot), scene, None)
    rng = np.random.default_rng(7)
    for q in synth.random_configs(rng, robot, 20).astype(np.float64):
        frames, centres, _ = orc.fk(plain, q)
        hw = orc.hulls_world(m, q)
        for k, f in enumerate(robot.hull_frame):
            R = frames[f, :9].reshape(3, 3)
            p = frames[f, 9:12]
            c, Rl, h = _parts(robot.hull_box[k].astype(np.float64))
            np.testing.assert_allclose(hw[k, :3], R @ c + p, atol=1e-12)
            np.testing.assert_allclose(hw[k, 3:12].reshape(3, 3), R @ Rl, atol=1e-14)
            # every sphere of the link lies inside its hull
            for s in np.where(robot.sphere_frame == f)[0]:
                loc = (R @ Rl).T @ (centres[s] - hw[k, :3])
                assert np.all(np.abs(loc) + robot.sphere_radius[s] <= h + 1e-6)


def test_configuration_distance_is_min_over_hull_pairs(orc):
    robot, scene, m = _sat_crane(orc)
    rng = np.random.default_rng(8)
    Q = synth.random_configs(rng, robot, 30).astype(np.float64)
    Q[:, 4:] = rng.uniform(-1.0, 1.0, size=(30, 2))
    d, s, o, sec = orc.eval_configs(m, Q)
    n_self = 0
    for i, q in enumerate(Q):
        hw = orc.hulls_world(m, q)
        vals = []
        for k in range(len(hw)):
            c, R, h = _parts(hw[k])
            corners = c[:, None] + (R * h) @ np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)]).T
            vals.append((corners[2].min() - scene.ground_z, k, 0))
            for j in range(scene.n_obb):
                vals.append((orc.sat_obb(hw[k], scene.obb[j].astype(np.float64)), k, 1 + j))
            for k2 in range(k + 1, len(hw)):
                fa, fb = robot.hull_frame[k], robot.hull_frame[k2]
                if any({fa, fb} == {int(x), int(y)} for x, y in robot.self_pairs):
                    vals.append((orc.sat_obb(hw[k], hw[k2]), k, 0xFF00 + k2))
        best = min(vals)
        assert d[i] == pytest.approx(best[0], abs=1e-12)
        assert (s[i], o[i]) == (best[1], best[2])
        n_self += o[i] >= 0xFF00
    assert sec.shape == d.shape


def test_sat_path_cost_uses_the_hull_distance(orc):
    """The path cost's collision term in SAT mode is the hinge of the hull
    distance at every checkpoint (per-checkpoint distances from the path
    evaluation equal the configuration distances of the path's points)."""
    robot, scene, _ = _sat_crane(orc)
    base = synth.c1_full()
    cost = dataclasses.replace(base.cost, K=4, M=4)
    m = orc.Model(robot, scene, cost)
    rng = np.random.default_rng(9)
    W = synth.random_waypoints(rng, robot, base.q_start, base.q_goal, 4, 4, sigma=0.3).astype(np.float64)
    ref = orc.eval_paths(m, base.q_start, base.q_goal, W, per_checkpoint=True)
    for b in range(4):
        pts = orc.path_points(m, base.q_start, base.q_goal, W[b])
        d, _, _, _ = orc.eval_configs(m, pts[1:])
        np.testing.assert_allclose(ref["d"][b], d, atol=0)
        assert ref["min_dist"][b] == pytest.approx(d.min(), abs=0)
    with pytest.raises(ValueError):
        orc.grad_paths(m, base.q_start, base.q_goal, W)
