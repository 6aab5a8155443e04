"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test checks one oracle routine against a closed form, an invariant, a
brute-force computation, a published value or a textbook formula written
independently here, chosen so that a plausible slip in the oracle (a dropped
term, a wrong sign or index, a transposed operand) fails at least one test.
"""
import dataclasses
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2503_14160_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _robot(seed=11, S=24):
    return synth.make_robot(seed, S)


def _empty_scene(ground=0):
    return synth.Scene(cyl=np.zeros((0, 5), np.float32), box=np.zeros((0, 6), np.float32),
                       has_ground=ground, ground_z=0.0)


def _rz(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


# ----------------------------------------------------------------------------
# Philox4x32-10
# ----------------------------------------------------------------------------

def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox4x32_10(v[0:4], v[4:6])
        assert out.tolist() == v[6:10]


def test_normals_moments_and_layout(orc):
    z = orc.normals(seed=77, t=3, B=4096, D=32)
    n = z.size
    assert abs(z.mean()) < 5.0 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
    # fourth moment of a standard normal is 3
    assert abs((z ** 4).mean() - 3.0) < 5.0 * math.sqrt(96.0 / n)
    # counter layout: element 4g+h of path b at iteration t uses counter (g, b, t, problem)
    x = orc.philox4x32_10([2, 5, 3, 0], [77, 0])
    u = [(2.0 * (w >> 9) + 1.0) / 2 ** 24 for w in x.tolist()]
    r = math.sqrt(-2.0 * math.log(u[0]))
    assert z[5, 8] == pytest.approx(r * math.cos(2 * math.pi * u[1]), rel=0, abs=1e-15)
    assert z[5, 9] == pytest.approx(r * math.sin(2 * math.pi * u[1]), rel=0, abs=1e-15)
    # a different iteration or problem gives a different stream; the same one repeats
    assert not np.array_equal(z, orc.normals(seed=77, t=4, B=4096, D=32))
    assert not np.array_equal(z, orc.normals(seed=77, t=3, B=4096, D=32, problem=1))
    assert np.array_equal(z, orc.normals(seed=77, t=3, B=4096, D=32))


# ----------------------------------------------------------------------------
# forward kinematics
# ----------------------------------------------------------------------------

def test_fk_zero_angles_are_summed_offsets(orc):
    rb = _robot()
    m = orc.Model(rb, _empty_scene(), None)
    L1, L2, L3, L4, L5 = (float(x) for x in rb.link_lengths)
    frames, _, tip = orc.fk(m, np.zeros(6))
    p = frames[:, 9:12]
    np.testing.assert_allclose(p[1], [0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(p[2], [0, 0, L1], atol=1e-14)
    np.testing.assert_allclose(p[3], [L2, 0, L1], atol=1e-14)
    np.testing.assert_allclose(p[4], [L2 + L3, 0, L1], atol=1e-14)
    np.testing.assert_allclose(p[5], [L2 + L3 + L4, 0, L1], atol=1e-14)
    np.testing.assert_allclose(p[6], [L2 + L3 + L4, 0, L1], atol=1e-14)
    np.testing.assert_allclose(tip, [L2 + L3 + L4, 0, L1 - L5], atol=1e-14)
    for j in range(7):
        np.testing.assert_allclose(frames[j, :9].reshape(3, 3), np.eye(3), atol=1e-15)


def test_fk_preserves_link_lengths_and_rotations(orc):
    rb = _robot()
    m = orc.Model(rb, _empty_scene(), None)
    L1, L2, L3, L4, L5 = (float(x) for x in rb.link_lengths)
    rng = np.random.default_rng(5)
    for _ in range(50):
        q = rng.uniform(rb.q_min - 0.5, rb.q_max + 0.5)
        frames, cen, tip = orc.fk(m, q)
        p = frames[:, 9:12]
        assert np.linalg.norm(p[2] - p[1]) == pytest.approx(L1, abs=1e-12)
        assert np.linalg.norm(p[3] - p[2]) == pytest.approx(L2, abs=1e-12)
        assert np.linalg.norm(p[4] - p[3]) == pytest.approx(L3 + q[3], abs=1e-12)
        assert np.linalg.norm(p[5] - p[4]) == pytest.approx(L4, abs=1e-12)
        assert np.linalg.norm(p[6] - p[5]) == pytest.approx(0.0, abs=1e-12)
        assert np.linalg.norm(tip - p[6]) == pytest.approx(L5, abs=1e-12)
        for j in range(7):
            R = frames[j, :9].reshape(3, 3)
            np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
            assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-14)
        # spheres keep their distance to their frame origin
        for s in range(rb.n_spheres):
            f = rb.sphere_frame[s]
            assert np.linalg.norm(cen[s] - p[f]) == pytest.approx(np.linalg.norm(rb.sphere_center[s].astype(np.float64)), abs=1e-12)


def test_fk_slew_rotates_everything_about_z(orc):
    rb = _robot()
    m = orc.Model(rb, _empty_scene(), None)
    rng = np.random.default_rng(6)
    for _ in range(20):
        q = rng.uniform(rb.q_min, rb.q_max)
        dq = rng.uniform(-1, 1)
        q2 = q.copy()
        q2[0] += dq
        f1, c1, t1 = orc.fk(m, q)
        f2, c2, t2 = orc.fk(m, q2)
        Rz = _rz(dq)
        np.testing.assert_allclose(c2, c1 @ Rz.T, atol=1e-12)
        np.testing.assert_allclose(t2, Rz @ t1, atol=1e-12)


def test_fk_planar_when_slew_and_swing_zero(orc):
    rb = _robot()
    m = orc.Model(rb, _empty_scene(), None)
    rng = np.random.default_rng(7)
    for _ in range(20):
        q = rng.uniform(rb.q_min, rb.q_max)
        q[0] = 0.0
        q[4] = 0.0
        f, c, t = orc.fk(m, q)
        np.testing.assert_allclose(c[:, 1], 0.0, atol=1e-13)
        np.testing.assert_allclose(f[:, 10], 0.0, atol=1e-13)
        assert abs(t[1]) < 1e-13


def test_fk_boom_pitch_direction(orc):
    """Boom axis is -y: a positive boom angle lifts the boom tip."""
    rb = _robot()
    m = orc.Model(rb, _empty_scene(), None)
    L1, L2 = float(rb.link_lengths[0]), float(rb.link_lengths[1])
    q = np.zeros(6)
    q[1] = 0.3
    f, _, _ = orc.fk(m, q)
    np.testing.assert_allclose(f[3, 9:12], [L2 * math.cos(0.3), 0, L1 + L2 * math.sin(0.3)], atol=1e-13)


# ----------------------------------------------------------------------------
# signed distances
# ----------------------------------------------------------------------------

def _cyl_surface(cyl, h):
    x0, y0, R, z0, z1 = (float(v) for v in cyl)
    pts = []
    nth = max(8, int(2 * math.pi * R / h) + 1)
    nz = max(2, int((z1 - z0) / h) + 1)
    for th in np.linspace(0, 2 * math.pi, nth, endpoint=False):
        for z in np.linspace(z0, z1, nz):
            pts.append((x0 + R * math.cos(th), y0 + R * math.sin(th), z))
    for rr in np.linspace(0, R, max(2, int(R / h) + 1)):
        nt = max(1, int(2 * math.pi * rr / h) + 1)
        for th in np.linspace(0, 2 * math.pi, nt, endpoint=False):
            for z in (z0, z1):
                pts.append((x0 + rr * math.cos(th), y0 + rr * math.sin(th), z))
    return np.array(pts)


def _box_surface(box, h):
    c = np.array(box[:3], np.float64)
    hh = np.array(box[3:], np.float64)
    pts = []
    for ax in range(3):
        o = [a for a in range(3) if a != ax]
        u = np.linspace(-hh[o[0]], hh[o[0]], max(2, int(2 * hh[o[0]] / h) + 1))
        v = np.linspace(-hh[o[1]], hh[o[1]], max(2, int(2 * hh[o[1]] / h) + 1))
        for sgn in (-1, 1):
            for a in u:
                for b in v:
                    p = np.zeros(3)
                    p[ax] = sgn * hh[ax]
                    p[o[0]] = a
                    p[o[1]] = b
                    pts.append(c + p)
    return np.array(pts)


def test_sd_cylinder_vs_surface_sampling(orc):
    rng = np.random.default_rng(8)
    hs = 0.01
    cyl = np.array([0.3, -0.2, 0.25, 0.0, 1.0], np.float32)
    surf = _cyl_surface(cyl, hs)
    for _ in range(200):
        c = rng.uniform([-0.5, -1.0, -0.6], [1.1, 0.6, 1.6])
        d = orc.sd_cylinder(c, cyl)
        inside = math.hypot(c[0] - cyl[0], c[1] - cyl[1]) <= cyl[2] and cyl[3] <= c[2] <= cyl[4]
        dist = np.sqrt(((surf - c) ** 2).sum(1)).min()
        ref = -dist if inside else dist
        assert abs(d - ref) <= hs, (c, d, ref)


def test_sd_box_vs_surface_sampling(orc):
    rng = np.random.default_rng(9)
    hs = 0.01
    box = np.array([0.1, 0.2, 0.3, 0.4, 0.25, 0.3], np.float32)
    surf = _box_surface(box, hs)
    for _ in range(200):
        c = rng.uniform([-0.6, -0.4, -0.3], [0.8, 0.8, 0.9])
        d = orc.sd_box(c, box)
        inside = np.all(np.abs(c - box[:3]) <= box[3:])
        dist = np.sqrt(((surf - c) ** 2).sum(1)).min()
        ref = -dist if inside else dist
        assert abs(d - ref) <= hs, (c, d, ref)


def test_sd_special_cases(orc):
    cyl = np.array([1.0, 2.0, 0.5, 0.0, 15.0], np.float32)
    # on the axis above the cap: distance to the cap plane
    assert orc.sd_cylinder([1.0, 2.0, 17.5], cyl) == pytest.approx(2.5, abs=1e-14)
    # beside the side wall at mid height: radial gap
    assert orc.sd_cylinder([4.0, 2.0, 7.0], cyl) == pytest.approx(2.5, abs=1e-14)
    # on the axis at mid height: -(min(R, half height))
    assert orc.sd_cylinder([1.0, 2.0, 7.5], cyl) == pytest.approx(-0.5, abs=1e-14)
    # diagonal beyond the rim: Euclidean distance to the rim circle
    assert orc.sd_cylinder([1.0 + 0.5 + 3.0, 2.0, 15.0 + 4.0], cyl) == pytest.approx(5.0, abs=1e-14)
    box = np.array([0, 0, 1, 1, 2, 1], np.float32)
    assert orc.sd_box([3.0, 0.0, 1.0], box) == pytest.approx(2.0, abs=1e-14)
    assert orc.sd_box([1.0 + 3, 2.0 + 4, 1.0], box) == pytest.approx(5.0, abs=1e-14)
    assert orc.sd_box([0.0, 0.0, 1.0], box) == pytest.approx(-1.0, abs=1e-14)


def test_sd_gradients_match_finite_differences(orc):
    rng = np.random.default_rng(10)
    cyl = np.array([0.3, -0.2, 0.25, 0.0, 1.0], np.float32)
    box = np.array([0.1, 0.2, 0.3, 0.4, 0.25, 0.3], np.float32)
    h = 1e-6
    for fn, ob in ((orc.sd_cylinder, cyl), (orc.sd_box, box)):
        n_checked = 0
        for _ in range(300):
            c = rng.uniform(-1.0, 1.5, size=3)
            d, g = fn(c, ob, grad=True)
            fd = np.zeros(3)
            for a in range(3):
                e = np.zeros(3)
                e[a] = h
                fd[a] = (fn(c + e, ob) - fn(c - e, ob)) / (2 * h)
            # skip points within 1e-4 of a kink (gradient switches branch there)
            kink = False
            for a in range(3):
                e = np.zeros(3)
                e[a] = 1e-4
                _, g1 = fn(c + e, ob, grad=True)
                _, g2 = fn(c - e, ob, grad=True)
                if np.abs(g1 - g2).max() > 1e-2:
                    kink = True
            if kink:
                continue
            n_checked += 1
            np.testing.assert_allclose(g, fd, atol=1e-7)
        assert n_checked > 200


def test_config_distance_is_min_over_pairs(orc):
    rb = _robot(S=24)
    rng = np.random.default_rng(12)
    qs, qg = synth.make_endpoints(rng, rb)
    sc = synth.make_scene(rng, rb, qs, qg, n_cyl=12, n_box=3, half_extent=8.0)
    m = orc.Model(rb, sc, None)
    Q = synth.random_configs(rng, rb, 40)
    d, s_arg, o_arg, sec = orc.eval_configs(m, Q)
    for i in range(Q.shape[0]):
        _, cen, _ = orc.fk(m, Q[i])
        vals = []
        for s in range(rb.n_spheres):
            r = float(rb.sphere_radius[s])
            vals.append((cen[s, 2] - 0.0 - r, s, 0))
            for o in range(sc.n_cyl):
                vals.append((orc.sd_cylinder(cen[s], sc.cyl[o]) - r, s, 1 + o))
            for o in range(sc.n_box):
                vals.append((orc.sd_box(cen[s], sc.box[o]) - r, s, 1 + sc.n_cyl + o))
        best = min(vals, key=lambda v: (v[0], v[1], v[2]))
        assert d[i] == best[0]
        assert (s_arg[i], o_arg[i]) == (best[1], best[2])
        assert sec[i] == sorted(v[0] for v in vals)[1]


def _self_vals(orc, m, rb, q):
    """Every listed self pair of spheres (a < b) at q, written out from the
    oracle's FK centres: (|c_a - c_b| - r_a - r_b, a, 0xFF00 + b)."""
    _, cen, _ = orc.fk(m, q)
    listed = {tuple(sorted(p)) for p in rb.self_pairs.tolist()}
    vals = []
    for a in range(rb.n_spheres):
        for b in range(a + 1, rb.n_spheres):
            if tuple(sorted((int(rb.sphere_frame[a]), int(rb.sphere_frame[b])))) in listed:
                d = float(np.linalg.norm(cen[a] - cen[b])) - float(rb.sphere_radius[a]) - float(rb.sphere_radius[b])
                vals.append((d, a, 0xFF00 + b))
    return vals


def test_self_collision_is_min_over_listed_sphere_pairs(orc):
    """With self-collision frame pairs listed (the crane's non-adjacent links)
    d(q) is the minimum over the scene pairs and over every sphere pair of a
    listed frame pair of |c_a - c_b| - r_a - r_b, ties by (sphere, scene
    obstacles first, then the other sphere); random folded configurations
    reach negative self distances."""
    rb = synth.with_self_collision(_robot(S=24))
    assert len(rb.self_pairs) == 6
    rng = np.random.default_rng(31)
    qs, qg = synth.make_endpoints(rng, rb)
    sc = synth.make_scene(rng, rb, qs, qg, n_cyl=6, n_box=1, half_extent=8.0)
    m = orc.Model(rb, sc, None)
    m0 = orc.Model(rb, _empty_scene(), None)
    Q = synth.random_configs(rng, rb, 60, margin=0.0)
    # telescope retracted and the hanger swung up toward the arm on half of them
    Q[:30, 3] = rng.uniform(0.0, 0.6, size=30)
    Q[:30, 5] = rng.choice([-1.0, 1.0], size=30) * rng.uniform(1.2, 1.57, size=30)
    d, s_arg, o_arg, sec = orc.eval_configs(m, Q)
    d0, s0, o0, _ = orc.eval_configs(m0, Q)
    neg = 0
    for i in range(Q.shape[0]):
        _, cen, _ = orc.fk(m, Q[i])
        selfv = _self_vals(orc, m, rb, Q[i])
        vals = []
        for s in range(rb.n_spheres):
            r = float(rb.sphere_radius[s])
            vals.append((cen[s, 2] - r, s, 0))
            for o in range(sc.n_cyl):
                vals.append((orc.sd_cylinder(cen[s], sc.cyl[o]) - r, s, 1 + o))
            for o in range(sc.n_box):
                vals.append((orc.sd_box(cen[s], sc.box[o]) - r, s, 1 + sc.n_cyl + o))
        vals += selfv
        best = min(vals, key=lambda v: (v[0], v[1], v[2]))
        assert d[i] == pytest.approx(best[0], abs=1e-12)
        assert (s_arg[i], o_arg[i]) == (best[1], best[2])
        assert sec[i] == pytest.approx(sorted(v[0] for v in vals)[1], abs=1e-12)
        sbest = min(selfv, key=lambda v: (v[0], v[1], v[2]))
        assert d0[i] == pytest.approx(sbest[0], abs=1e-12) and (s0[i], o0[i]) == (sbest[1], sbest[2])
        neg += sbest[0] < 0
    assert neg >= 5


def test_self_collision_invariant_under_slew(orc):
    """Self distances depend on the joint angles below the slew only: turning
    the whole crane about the vertical axis leaves them unchanged."""
    rb = synth.with_self_collision(_robot(S=24))
    m0 = orc.Model(rb, _empty_scene(), None)
    rng = np.random.default_rng(32)
    Q = synth.random_configs(rng, rb, 30)
    Q2 = Q.copy()
    Q2[:, 0] += rng.uniform(-3, 3, size=30)
    d1, s1, o1, _ = orc.eval_configs(m0, Q)
    d2, s2, o2, _ = orc.eval_configs(m0, Q2)
    np.testing.assert_allclose(d1, d2, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(o1 >= 0xFF00, True)


def test_self_collision_gradient_matches_central_differences(orc):
    """Paths with the hanger swung up toward the arm and no scene: the
    collision term comes from self pairs alone; the analytic gradient (through
    both spheres' chains, passive joints included) matches FP64 central
    differences on paths without a kink."""
    rb = synth.with_self_collision(_robot(S=16))
    rng = np.random.default_rng(33)
    qs = np.array([0.3, 0.9, -1.0, 0.2, 0.0, 1.35], np.float32)
    qg = np.array([1.5, 0.7, -1.2, 0.4, 0.0, 1.45], np.float32)
    K, M = 4, 4
    m = orc.Model(rb, _empty_scene(), _cost(K, M, hinge=synth.HINGE_SMOOTH, margin=0.1))
    W = synth.random_waypoints(rng, rb, qs, qg, 12, K, sigma=0.2).astype(np.float64)
    W[:, :, 5] = 1.4 + rng.normal(size=(12, K)) * 0.05
    ok = _fd_ok_mask(orc, m, qs, qg, W, 0.1)
    ref = orc.eval_paths(m, qs, qg, W, per_checkpoint=True)
    assert ((ref["d"] < 0.1) & (ok[:, None])).any()  # self pairs inside the hinge on kept paths
    assert ok.sum() >= 4
    W = W[ok]
    _, g = orc.grad_paths(m, qs, qg, W)
    fd = orc.fd_grad(m, qs, qg, W, h=1e-6)
    for b in range(W.shape[0]):
        err = np.linalg.norm(g[b] - fd[b]) / max(np.linalg.norm(fd[b]), 1e-12)
        assert err <= 1e-6, (b, err)


# ----------------------------------------------------------------------------
# interpolation
# ----------------------------------------------------------------------------

def _blend(u):
    """Uniform cubic B-spline blending polynomials (textbook closed form)."""
    return np.array([(1 - u) ** 3 / 6, (3 * u ** 3 - 6 * u ** 2 + 4) / 6,
                     (-3 * u ** 3 + 3 * u ** 2 + 3 * u + 1) / 6, u ** 3 / 6])


def _cost(K, M, interp=synth.INTERP_BSPLINE, jp=synth.JP_SQUARED, hinge=synth.HINGE_HARD, margin=0.0):
    return synth.CostParams(K=K, M=M, interp=interp, jp_mode=jp, hinge=hinge, margin=margin)


def test_bspline_matches_closed_form_blend(orc):
    rb = _robot()
    K, M = 5, 4
    m = orc.Model(rb, _empty_scene(), _cost(K, M))
    rng = np.random.default_rng(13)
    qs, qg = rng.normal(size=6), rng.normal(size=6)
    W = rng.normal(size=(K, 6))
    pts = orc.path_points(m, qs, qg, W)
    P = np.concatenate([np.repeat(qs[None], 3, 0), W, np.repeat(qg[None], 3, 0)], 0)
    ns = (K + 3) * M
    assert pts.shape == (ns + 1, 6)
    for k in range(ns + 1):
        j, i = divmod(k, M)
        if j == K + 3:
            j, u = K + 2, 1.0
        else:
            u = i / M
        ref = _blend(u) @ P[j:j + 4]
        np.testing.assert_allclose(pts[k], ref, atol=1e-14)


def test_bspline_basis_values_and_endpoints(orc):
    rb = _robot()
    K, M = 4, 2
    m = orc.Model(rb, _empty_scene(), _cost(K, M))
    z = np.zeros(6)
    for i in range(K):
        W = np.zeros((K, 6))
        W[i, 0] = 1.0
        pts = orc.path_points(m, z, z, W)[:, 0]
        # control point i+3 of the 3-copy polygon is active on spans i..i+3
        for j in range(K + 3):
            t = j - i
            if 0 <= t <= 3:
                assert pts[j * M] == pytest.approx([1 / 6, 4 / 6, 1 / 6, 0.0][::-1][t] if False else [0.0, 1 / 6, 4 / 6, 1 / 6][3 - t] if False else _blend(0.0)[3 - t], abs=1e-15)
                assert pts[j * M + M // 2] == pytest.approx(_blend(0.5)[3 - t], abs=1e-15)
    np.testing.assert_allclose(_blend(0.0), [1 / 6, 4 / 6, 1 / 6, 0], atol=1e-15)
    np.testing.assert_allclose(_blend(0.5), np.array([1, 23, 23, 1]) / 48, atol=1e-15)
    rng = np.random.default_rng(14)
    qs, qg = rng.normal(size=6), rng.normal(size=6)
    pts = orc.path_points(m, qs, qg, rng.normal(size=(K, 6)))
    np.testing.assert_allclose(pts[0], qs, atol=1e-14)
    np.testing.assert_allclose(pts[-1], qg, atol=1e-14)
    # partition of unity: a constant polygon gives a constant path
    c = rng.normal(size=6)
    pts = orc.path_points(m, c, c, np.repeat(c[None], K, 0))
    np.testing.assert_allclose(pts, np.repeat(c[None], pts.shape[0], 0), atol=1e-14)


def test_collinear_polygon_gives_monotone_straight_path(orc):
    rb = _robot()
    K, M = 6, 8
    m = orc.Model(rb, _empty_scene(), _cost(K, M))
    qs, qg = np.zeros(6), np.array([1.0, -2.0, 0.5, 0.3, 0.0, 0.0])
    t = np.sort(np.random.default_rng(15).uniform(0, 1, K))
    W = t[:, None] * qg[None]
    pts = orc.path_points(m, qs, qg, W)
    lam = pts[:, 0]
    np.testing.assert_allclose(pts, lam[:, None] * qg[None], atol=1e-14)
    assert np.all(np.diff(lam) >= -1e-15)


def test_linear_interp(orc):
    rb = _robot()
    K, M = 3, 5
    m = orc.Model(rb, _empty_scene(), _cost(K, M, interp=synth.INTERP_LINEAR))
    rng = np.random.default_rng(16)
    qs, qg, W = rng.normal(size=6), rng.normal(size=6), rng.normal(size=(K, 6))
    P = np.concatenate([qs[None], W, qg[None]], 0)
    pts = orc.path_points(m, qs, qg, W)
    for k in range(pts.shape[0]):
        j, i = divmod(k, M)
        if j == K + 1:
            ref = qg
        else:
            ref = (1 - i / M) * P[j] + (i / M) * P[j + 1]
        np.testing.assert_allclose(pts[k], ref, atol=1e-14)


# ----------------------------------------------------------------------------
# cost
# ----------------------------------------------------------------------------

def _jp_coefficient(K, M):
    """Exact sum over checkpoints of (t(s_k) - t(s_{k-1}))^2 for the 1-D spline
    whose control polygon is [0,0,0, 1/(K+1), ..., K/(K+1), 1,1,1]
    (rational arithmetic, blend polynomials)."""
    P = [Fraction(0)] * 3 + [Fraction(i + 1, K + 1) for i in range(K)] + [Fraction(1)] * 3

    def blend(u):
        return [(1 - u) ** 3 / 6, (3 * u ** 3 - 6 * u ** 2 + 4) / 6, (-3 * u ** 3 + 3 * u ** 2 + 3 * u + 1) / 6,
                u ** 3 / 6]

    def q(k):
        j, i = divmod(k, M)
        u = Fraction(i, M)
        if j == K + 3:
            j, u = K + 2, Fraction(1)
        return sum(b * p for b, p in zip(blend(u), P[j:j + 4]))

    ns = (K + 3) * M
    vals = [q(k) for k in range(ns + 1)]
    return sum((vals[k] - vals[k - 1]) ** 2 for k in range(1, ns + 1))


def test_straight_path_length_closed_forms(orc):
    rb = _robot()
    qs = np.array([-1.0, 0.2, -0.5, 0.4, 0.0, 0.0])
    qg = np.array([1.5, 0.9, -0.1, 2.1, 0.0, 0.0])
    dist = np.linalg.norm(qg - qs)
    for K, M in ((8, 16), (16, 32), (3, 5)):
        i = np.arange(K)[:, None]
        W = qs[None] + (i + 1) / (K + 1) * (qg - qs)[None]
        for interp in (synth.INTERP_BSPLINE, synth.INTERP_LINEAR):
            m2 = orc.Model(rb, _empty_scene(), _cost(K, M, interp=interp, jp=synth.JP_L2))
            r = orc.eval_paths(m2, qs, qg, W[None], per_checkpoint=True)
            assert r["parts"][0, 0] == pytest.approx(dist, rel=1e-13)
            assert r["parts"][0, 1] == 0.0 and r["parts"][0, 2] == 0.0
            assert r["cost"][0] == pytest.approx(dist, rel=1e-13)
        mlin = orc.Model(rb, _empty_scene(), _cost(K, M, interp=synth.INTERP_LINEAR))
        ns = (K + 1) * M
        assert orc.eval_paths(mlin, qs, qg, W[None])["cost"][0] == pytest.approx(dist ** 2 / ns, rel=1e-13)
        msp = orc.Model(rb, _empty_scene(), _cost(K, M))
        c = float(_jp_coefficient(K, M))
        assert orc.eval_paths(msp, qs, qg, W[None])["cost"][0] == pytest.approx(dist ** 2 * c, rel=1e-13)
    assert float(_jp_coefficient(8, 16)) == pytest.approx(0.006584027503580, rel=1e-12)
    assert float(_jp_coefficient(16, 32)) == pytest.approx(0.001787762202377, rel=1e-12)


def test_limit_cost_closed_form(orc):
    rb = _robot()
    K, M = 4, 3
    m = orc.Model(rb, _empty_scene(), _cost(K, M))
    q = np.array(rb.q_max, np.float64) + np.array([0.1, 0.2, 0.0, 0.5, 0.0, 0.0])
    q[2] = float(rb.q_min[2]) - 0.3
    W = np.repeat(q[None], K, 0)
    r = orc.eval_paths(m, q, q, W[None], per_checkpoint=True)
    ns = (K + 3) * M
    assert r["parts"][0, 0] < 1e-25  # constant path (rounding of the basis sum only)
    assert r["parts"][0, 2] == pytest.approx(ns * (0.1 ** 2 + 0.2 ** 2 + 0.3 ** 2 + 0.5 ** 2), rel=1e-12)
    assert r["cost"][0] == pytest.approx(100.0 * r["parts"][0, 2], rel=1e-13)
    inside = 0.5 * (np.array(rb.q_min, np.float64) + np.array(rb.q_max, np.float64))
    r = orc.eval_paths(m, inside, inside, np.repeat(inside[None], K, 0)[None], per_checkpoint=True)
    assert r["parts"][0, 2] == 0.0


def test_collision_cost_from_distances(orc):
    """J_c is the hinge of d_k summed over checkpoints 1..n_s; min_dist and the
    flag follow d_k; J_c = 0 whenever min_dist >= margin."""
    rb = _robot()
    rng = np.random.default_rng(17)
    qs, qg = synth.make_endpoints(rng, rb)
    sc = synth.make_scene(rng, rb, qs, qg, n_cyl=20, n_box=2, half_extent=8.0)
    K, M = 5, 6
    for hinge, margin in ((synth.HINGE_HARD, 0.0), (synth.HINGE_HARD, 0.2), (synth.HINGE_SMOOTH, 0.1)):
        m = orc.Model(rb, sc, _cost(K, M, hinge=hinge, margin=margin))
        W = synth.random_waypoints(rng, rb, qs, qg, 6, K, sigma=0.4)
        r = orc.eval_paths(m, qs, qg, W, per_checkpoint=True)
        d = r["d"]
        margin = float(np.float32(margin))  # the model carries FP32 parameters
        if hinge == synth.HINGE_HARD:
            phi = np.maximum(0.0, margin - d)
        else:
            phi = np.where(d < 0, margin / 2 - d, np.where(d < margin, (margin - d) ** 2 / (2 * margin), 0.0))
        np.testing.assert_allclose(r["parts"][:, 1], phi.sum(1), rtol=1e-13, atol=1e-15)
        np.testing.assert_array_equal(r["min_dist"], d.min(1))
        np.testing.assert_array_equal(r["flags"], (d.min(1) < np.float32(margin)).astype(np.uint8))
        # the per-checkpoint distance is d(q(s_k)) for k = 1..n_s
        pts = orc.path_points(m, qs, qg, W[0])
        dc, _, _, _ = orc.eval_configs(m, pts[1:])
        np.testing.assert_array_equal(d[0], dc)
        total = r["parts"][:, 0] + 100.0 * r["parts"][:, 1] + 100.0 * r["parts"][:, 2]
        np.testing.assert_allclose(r["cost"], total, rtol=1e-14)
    # far from everything: no collision cost
    far = synth.Scene(cyl=np.array([[100.0, 100.0, 0.3, 0.0, 15.0]], np.float32), box=np.zeros((0, 6), np.float32),
                      has_ground=0)
    m = orc.Model(rb, far, _cost(K, M, margin=0.1))
    W = synth.random_waypoints(rng, rb, qs, qg, 4, K, sigma=0.1)
    r = orc.eval_paths(m, qs, qg, W, per_checkpoint=True)
    assert np.all(r["min_dist"] >= 0.1) and np.all(r["parts"][:, 1] == 0.0)


# ----------------------------------------------------------------------------
# gradient
# ----------------------------------------------------------------------------

def _fd_ok_mask(orc, m, qs, qg, W, margin):
    r = orc.eval_paths(m, qs, qg, W, per_checkpoint=True)
    gap = r["second"] - r["d"]
    near_tie = (gap < 1e-5).any(1)
    near_margin = (np.abs(r["d"] - margin) < 1e-5).any(1)
    return ~(near_tie | near_margin)


@pytest.mark.parametrize("hinge,margin,jp", [(synth.HINGE_SMOOTH, 0.1, synth.JP_SQUARED),
                                            (synth.HINGE_HARD, 0.0, synth.JP_SQUARED),
                                            (synth.HINGE_HARD, 0.05, synth.JP_L2)])
def test_gradient_matches_central_differences(orc, hinge, margin, jp):
    rb = _robot(S=12)
    rng = np.random.default_rng(18)
    qs, qg = synth.make_endpoints(rng, rb)
    sc = synth.make_scene(rng, rb, qs, qg, n_cyl=10, n_box=2, half_extent=7.0)
    K, M = 4, 4
    m = orc.Model(rb, sc, _cost(K, M, hinge=hinge, margin=margin, jp=jp))
    W = synth.random_waypoints(rng, rb, qs, qg, 8, K, sigma=0.5).astype(np.float64)
    W[:, :, 3] = np.clip(W[:, :, 3], 0.2, 2.8)
    ok = _fd_ok_mask(orc, m, qs, qg, W, margin)
    assert ok.sum() >= 4
    W = W[ok]
    _, g = orc.grad_paths(m, qs, qg, W)
    fd = orc.fd_grad(m, qs, qg, W, h=1e-6)
    for b in range(W.shape[0]):
        err = np.linalg.norm(g[b] - fd[b]) / max(np.linalg.norm(fd[b]), 1e-12)
        assert err <= 1e-6, (b, err)


def test_gradient_of_path_length_closed_form(orc):
    """Without obstacles or limits the squared-J_p gradient with respect to the
    control points is 2 sum_k (q_k - q_{k-1}) (N(t_k) - N(t_{k-1}))."""
    rb = _robot()
    K, M = 5, 3
    m = orc.Model(rb, _empty_scene(), _cost(K, M))
    rng = np.random.default_rng(19)
    qs = np.zeros(6)
    qg = np.array([1.0, 0.5, -0.5, 1.0, 0.0, 0.0])
    W = np.clip(rng.normal(size=(1, K, 6)) * 0.2 + 0.3, -0.1, 0.3)
    W[:, :, 4:] = 0.0
    _, g = orc.grad_paths(m, qs, qg, W)
    pts = orc.path_points(m, qs, qg, W[0])
    ns = (K + 3) * M
    ref = np.zeros((K, 6))
    for i in range(K):
        # path response to control point i (basis function values at the checkpoints)
        E = np.zeros((K, 6))
        E[i, 0] = 1.0
        N = orc.path_points(m, np.zeros(6), np.zeros(6), E)[:, 0]
        for k in range(1, ns + 1):
            ref[i] += 2 * (pts[k] - pts[k - 1]) * (N[k] - N[k - 1])
    np.testing.assert_allclose(g[0], ref, atol=1e-12)


# ----------------------------------------------------------------------------
# Algorithm 1 steps
# ----------------------------------------------------------------------------

def test_log_rank_weights(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "log_rank_weights.txt")) if l.strip() and not l.startswith("#")]
    for kind, nu, idx, val in rows:
        nu, idx, val = int(nu), int(idx), float(val)
        if kind == "w":
            assert orc.log_rank_weights(nu)[idx - 1] == pytest.approx(val, abs=1e-12)
        else:
            assert nu * math.log(nu + 0.5) - math.lgamma(nu + 1) == pytest.approx(val, abs=1e-9)
            a = math.log(nu + 0.5) - np.log(np.arange(1, nu + 1))
            w = orc.log_rank_weights(nu)
            np.testing.assert_allclose(w, a / val, rtol=1e-11)
    for nu in (1, 2, 25, 64, 819, 3276):
        w = orc.log_rank_weights(nu)
        assert w.sum() == pytest.approx(1.0, abs=1e-14)
        assert np.all(w > 0) and np.all(np.diff(w) < 0)
    assert orc.log_rank_weights(1).tolist() == [1.0]


def test_mean_covariance_update_properties(orc):
    rng = np.random.default_rng(20)
    eps = 1e-6
    D = 7
    x = rng.normal(size=D)
    for nu in (1, 5):
        mu, C = orc.update(np.repeat(x[None], nu, 0), orc.log_rank_weights(nu), eps)
        np.testing.assert_allclose(mu, x, atol=1e-15)
        np.testing.assert_allclose(C, eps * np.eye(D), atol=1e-15)
    X = rng.normal(size=(12, D))
    w = orc.log_rank_weights(12)
    mu, C = orc.update(X, w, eps)
    assert np.all(mu >= X.min(0) - 1e-15) and np.all(mu <= X.max(0) + 1e-15)
    np.testing.assert_allclose(C, C.T, atol=1e-15)
    assert np.linalg.eigvalsh(C).min() >= eps * (1 - 1e-9)
    # explicit double sum
    ref = np.zeros((D, D))
    for j in range(12):
        ref += w[j] * np.outer(X[j] - mu, X[j] - mu)
    np.testing.assert_allclose(C, ref + eps * np.eye(D), atol=1e-14)


def test_selection_brute_force(orc):
    rng = np.random.default_rng(21)
    cost = np.round(rng.normal(size=300), 1)  # many ties
    cost[[3, 50, 77]] = np.nan
    cost[[1, 60, 299]] = np.inf  # interleaved with the NaNs by index
    cost[[5, 6]] = [-0.0, 0.0]
    cost[[7]] = -0.0
    for nu in (1, 10, 150, 295, 300):
        got = orc.select(cost, nu)
        keyed = sorted(range(cost.size), key=lambda i: (math.inf if math.isnan(cost[i]) else cost[i], i))
        assert got.tolist() == keyed[:nu]


def test_cholesky_jitter_and_failure(orc):
    C = np.diag([1.0, 4.0, 0.0])
    L = orc.cholesky_jitter(C + 1e-6 * np.eye(3), 1e-6)
    np.testing.assert_allclose(L @ L.T, C + 1e-6 * np.eye(3), atol=1e-15)
    # singular: retried with 10 eps I
    L = orc.cholesky_jitter(C, 1e-6)
    np.testing.assert_allclose(L @ L.T, C + 1e-5 * np.eye(3), atol=1e-15)
    with pytest.raises(orc.NotPositiveDefinite):
        orc.cholesky_jitter(-np.eye(3), 1e-6)


def test_sample_statistics(orc):
    """Samples mu + L z have mean mu and covariance C (CLT bounds)."""
    rb = _robot()
    prob = synth.Problem("t", rb, _empty_scene(), np.zeros(6, np.float32), np.ones(6, np.float32),
                         _cost(2, 2), synth.OptParams(B=16384, nu=10, sigma0=0.3, eps=1e-6, seed=5, T=1))
    opt = orc.Optimizer(prob)
    A = np.random.default_rng(22).normal(size=(opt.D, opt.D))
    opt.C = A @ A.T * 0.01 + 0.01 * np.eye(opt.D)
    xi = opt.sample()
    n = xi.shape[0]
    sd = np.sqrt(np.diag(opt.C))
    assert np.all(np.abs(xi.mean(0) - opt.mu) < 5 * sd / math.sqrt(n))
    emp = np.cov(xi.T)
    tol = 5 * np.sqrt((opt.C ** 2 + np.outer(np.diag(opt.C), np.diag(opt.C))) / n)
    assert np.all(np.abs(emp - opt.C) < tol)


def test_optimizer_free_space_moves_to_straight_line(orc):
    """No obstacles, linear interpolation, squared path length: the optimum is
    the evenly spaced straight line (cost |q_g - q_s|^2 / n_s).  The update has
    no step-size control, so the spread shrinks geometrically and the mean
    stalls short of the optimum; what is fixed is that the cost approaches the
    optimum, the mean moves toward the line and best-so-far never increases."""
    rb = _robot()
    K = 4
    qs = np.array([-1.0, 0.3, -0.4, 0.5, 0.0, 0.0], np.float32)
    qg = np.array([1.0, 0.8, -0.2, 2.0, 0.0, 0.0], np.float32)
    prob = synth.Problem("free", rb, _empty_scene(), qs, qg, _cost(K, 4, interp=synth.INTERP_LINEAR),
                         synth.OptParams(B=512, nu=51, sigma0=0.3, eps=1e-8, seed=9, T=30))
    opt = orc.Optimizer(prob)
    target = orc.initial_mean(rb, qs, qg, K)
    opt.mu = opt.mu + np.random.default_rng(23).normal(size=opt.D) * 0.3
    err0 = np.abs(opt.mu - target).max()
    best = []
    for _ in range(30):
        opt.step()
        best.append(opt.best_cost)
    assert all(b2 <= b1 for b1, b2 in zip(best, best[1:]))
    optimum = float(np.sum((qg.astype(np.float64) - qs) ** 2)) / prob.cost.n_s
    assert optimum <= best[-1] < 1.05 * optimum
    assert np.abs(opt.mu - target).max() < 0.5 * err0


# ----------------------------------------------------------------------------
# gradient polish of the elites (a workload setting; the paper's Algorithm 1
# is derivative free)
# ----------------------------------------------------------------------------

def _polish_problem(scene, K=5, M=4, steps=1, eta=1e-3, clip=10.0, hinge=synth.HINGE_HARD, margin=0.0,
                    interp=synth.INTERP_LINEAR, nu=4):
    rb = _robot()
    qs = np.array([0.2, 0.5, -0.3, 1.0, 0.0, 0.0], np.float32)
    qg = np.array([1.4, 0.9, -0.6, 2.0, 0.0, 0.0], np.float32)
    opt = synth.OptParams(B=8, nu=nu, sigma0=0.2, eps=1e-6, seed=5, T=1, polish_elites=nu, polish_steps=steps,
                          polish_eta=eta, polish_clip=clip)
    return synth.Problem("polish", rb, scene, qs, qg, _cost(K, M, interp=interp, hinge=hinge, margin=margin), opt)


def _linear_jp_grad(qs, qg, xi, K, M, act):
    """Free space, linear interpolation, squared J_p: the polygon is
    (q_s, W_0..W_{K-1}, q_g) and every checkpoint step of segment j is
    (P_{j+1} - P_j) / M, so J_p = sum_j |P_{j+1} - P_j|^2 / M and
    dJ_p / dW_i = (2 / M) (2 P_{i+1} - P_i - P_{i+2}) (written out here, not
    taken from the oracle)."""
    na = int(act.sum())
    P = np.concatenate([np.asarray(qs, np.float64)[act][None], xi.reshape(K, na),
                        np.asarray(qg, np.float64)[act][None]], 0)
    return ((2.0 / M) * (2 * P[1:-1] - P[:-2] - P[2:])).reshape(-1)


def test_polish_free_space_steps_follow_the_closed_form_gradient(orc):
    """In free space within the joint limits the cost is J_p alone; each
    unclipped polish step is x - eta g with g the closed-form gradient above,
    and every step lowers J.  Several steps are the closed-form iteration."""
    prob = _polish_problem(_empty_scene(), steps=5, eta=1e-2)
    opt = orc.Optimizer(prob)
    act = prob.robot.active.astype(bool)
    rng = np.random.default_rng(41)
    x0 = np.tile(opt.mu, (4, 1)) + rng.normal(size=(4, opt.D)) * 0.05
    ref = x0.copy()
    for _ in range(5):
        g = np.stack([_linear_jp_grad(prob.q_start, prob.q_goal, r, prob.cost.K, prob.cost.M, act) for r in ref])
        assert np.all(np.linalg.norm(g, axis=1) < prob.opt.polish_clip)  # unclipped regime
        ref = ref - prob.opt.polish_eta * g
    trace = []
    got = opt.polish(x0, trace=trace)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)
    assert len(trace) == 5
    m = opt.model
    costs = [orc.eval_paths(m, prob.q_start, prob.q_goal, orc.expand(prob.robot, x, prob.cost.K))["cost"]
             for x in trace + [got]]
    for a, b in zip(costs, costs[1:]):
        assert np.all(b < a)


def test_polish_clipped_step_has_length_eta_gmax(orc):
    """Far from the straight line the gradient norm exceeds g_max: the step is
    eta g_max g / |g| exactly (its length eta g_max, its direction -g)."""
    prob = _polish_problem(_empty_scene(), M=1, steps=1, eta=1e-3, clip=0.5)
    opt = orc.Optimizer(prob)
    rb = prob.robot
    act = rb.active.astype(bool)
    rng = np.random.default_rng(42)
    x0 = np.tile(opt.mu, (3, 1)) + rng.normal(size=(3, opt.D)) * 0.1
    lo = np.tile(rb.q_min[act], prob.cost.K)
    hi = np.tile(rb.q_max[act], prob.cost.K)
    assert np.all((x0 > lo) & (x0 < hi))  # no limit cost: J = J_p
    g = np.stack([_linear_jp_grad(prob.q_start, prob.q_goal, r, prob.cost.K, prob.cost.M, act) for r in x0])
    nrm = np.linalg.norm(g, axis=1)
    assert np.all(nrm > 0.5)
    got = opt.polish(x0)
    step = x0 - got
    np.testing.assert_allclose(np.linalg.norm(step, axis=1), 1e-3 * 0.5, rtol=1e-12)
    np.testing.assert_allclose(step, 1e-3 * 0.5 * g / nrm[:, None], rtol=0, atol=1e-15)


def test_polish_uses_the_sampled_joints_only(orc):
    """With an obstacle touching the hanger spheres the cost also depends on
    the passive swing joints, but the polish steps and clips on the sampled
    joints alone: step = eta g_a / max(1, |g_a| / g_max) with g_a the sampled
    joints' part of the (FD-pinned) gradient; the passive joints stay at their
    hold value."""
    rb = _robot()
    prob0 = _polish_problem(_empty_scene(), interp=synth.INTERP_BSPLINE, hinge=synth.HINGE_SMOOTH, margin=0.1)
    opt0 = orc.Optimizer(prob0)
    m0 = opt0.model
    # an obstacle at the hanger of the middle of the path
    W = orc.expand(rb, opt0.mu[None], prob0.cost.K)
    mid = orc.path_points(m0, prob0.q_start, prob0.q_goal, W[0])[prob0.cost.n_s // 2]
    _, cen, _ = orc.fk(m0, mid)
    s_hang = int(np.where(rb.sphere_frame == 6)[0][-1])
    c = cen[s_hang]
    box = np.array([[c[0] + 0.3, c[1], c[2], 0.3, 0.3, 0.3]], np.float32)
    scene = synth.Scene(cyl=np.zeros((0, 5), np.float32), box=box, has_ground=0)
    for clip in (1e6, 1.0):
        prob = _polish_problem(scene, interp=synth.INTERP_BSPLINE, hinge=synth.HINGE_SMOOTH, margin=0.1, clip=clip)
        opt = orc.Optimizer(prob)
        x0 = opt.mu[None].copy()
        _, gfull = orc.grad_paths(opt.model, prob.q_start, prob.q_goal, orc.expand(rb, x0, prob.cost.K))
        assert np.abs(gfull[0][:, 4:]).max() > 1e-3  # the passive joints do matter
        ga = gfull[:, :, rb.active.astype(bool)].reshape(1, -1)
        scale = prob.opt.polish_eta / max(1.0, np.linalg.norm(ga) / clip)
        got = opt.polish(x0)
        np.testing.assert_allclose(got, x0 - scale * ga, rtol=0, atol=1e-15)
        assert got.shape == x0.shape
        Wp = orc.expand(rb, got, prob.cost.K)
        np.testing.assert_array_equal(Wp[:, :, ~rb.active.astype(bool)], 0.0)


def test_optimizer_step_with_idle_polish_equals_plain_step(orc):
    """A polish of zero step length re-evaluates the elites unchanged, and the
    stable re-ranking keeps their order: the step equals the plain one.  With
    a real polish, best-so-far takes the best polished elite."""
    rng = np.random.default_rng(43)
    rb = _robot()
    qs, qg = synth.make_endpoints(rng, rb)
    sc = synth.make_scene(rng, rb, qs, qg, n_cyl=12, n_box=1, half_extent=6.0)
    base = synth.Problem("p", rb, sc, qs, qg, _cost(4, 4, hinge=synth.HINGE_SMOOTH, margin=0.1),
                         synth.OptParams(B=32, nu=6, sigma0=0.3, eps=1e-6, seed=11, T=1))
    idle = dataclasses.replace(base, opt=dataclasses.replace(base.opt, polish_elites=6, polish_steps=2,
                                                             polish_eta=0.0))
    a = orc.Optimizer(base).step()
    b = orc.Optimizer(idle).step()
    np.testing.assert_array_equal(a["mu"], b["mu"])
    np.testing.assert_array_equal(a["C"], b["C"])
    real = dataclasses.replace(base, opt=dataclasses.replace(base.opt, polish_elites=6, polish_steps=3,
                                                             polish_eta=1e-3))
    o = orc.Optimizer(real)
    r = o.step()
    xe = r["xi"][r["elite"]][:6]
    xp = o.polish(xe)
    cp_ = orc.eval_paths(o.model, qs, qg, orc.expand(rb, xp, 4))["cost"]
    assert o.best_cost <= min(cp_.min(), r["cost"].min())


# ----------------------------------------------------------------------------
# voxel occupancy, distance transforms, signed-distance grid
# ----------------------------------------------------------------------------

def test_edt_separable_equals_brute_force(orc):
    rng = np.random.default_rng(24)
    for shape, p in (((5, 6, 7), 0.1), ((4, 9, 3), 0.02), ((6, 5, 8), 0.5), ((3, 3, 3), 0.0)):
        mask = (rng.uniform(size=shape) < p).astype(np.uint8)
        for target in (1, 0):
            a = orc.edt(mask, target, brute=True)
            b = orc.edt(mask, target, brute=False)
            np.testing.assert_array_equal(a, b)
    empty = np.zeros((3, 4, 5), np.uint8)
    np.testing.assert_array_equal(orc.edt(empty, 1), np.full(empty.shape, 5 * 5 + 4 * 4 + 3 * 3))


def test_sdf_single_voxel_and_plane(orc):
    nz, ny, nx = 6, 7, 8
    occ = np.zeros((nz, ny, nx), np.uint8)
    occ[2, 3, 4] = 1
    h = 0.25
    phi, e_occ, e_free = orc.sdf_from_occupancy(occ, h)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    dist = np.sqrt((xx - 4) ** 2 + (yy - 3) ** 2 + (zz - 2) ** 2)
    ref = h * (dist - 0.5)
    ref[2, 3, 4] = -h * 0.5
    np.testing.assert_allclose(phi, ref, atol=1e-15)
    occ = np.zeros((nz, ny, nx), np.uint8)
    occ[:2] = 1
    phi, e_occ, e_free = orc.sdf_from_occupancy(occ, h)
    np.testing.assert_array_equal(e_occ[2:], ((zz[2:] - 1) ** 2))
    np.testing.assert_array_equal(e_free[:2], ((zz[:2] - 2) ** 2))


def test_trilinear_reproduces_linear_fields(orc):
    spec = synth.SdfSpec(dims=(6, 5, 4), origin=(-1.0, 2.0, 0.5), voxel=0.5)
    nx, ny, nz = spec.dims
    a = np.array([0.3, -1.2, 0.7])
    b = 0.25
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cx = spec.origin[0] + (i + 0.5) * spec.voxel
    cy = spec.origin[1] + (j + 0.5) * spec.voxel
    cz = spec.origin[2] + (k + 0.5) * spec.voxel
    grid = (a[0] * cx + a[1] * cy + a[2] * cz + b).astype(np.float32)
    m = orc.Model(_robot(), _empty_scene(), None, sdf=grid, sdf_spec=spec)
    rng = np.random.default_rng(25)
    lo = np.array(spec.origin) + 0.5 * spec.voxel
    hi = np.array(spec.origin) + (np.array(spec.dims) - 0.5) * spec.voxel
    for _ in range(100):
        c = rng.uniform(lo, hi)
        v, g = orc.sdf_query(m, c, grad=True)
        assert v == pytest.approx(a @ c + b, abs=1e-6)  # grid stored in float32
        np.testing.assert_allclose(g, a, atol=1e-5)
    # outside the grid the voxel coordinate clamps: the value of the nearest face
    c = np.array([hi[0] + 3.0, 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])])
    v, g = orc.sdf_query(m, c, grad=True)
    assert v == pytest.approx(a @ np.array([hi[0], c[1], c[2]]) + b, abs=1e-6)
    assert g[0] == 0.0


def test_occupancy_binning(orc):
    spec = synth.SdfSpec(dims=(4, 3, 2), origin=(-1.0, -1.0, -0.5), voxel=0.25)
    pts = np.array([[-1.0, -1.0, -0.5],       # lower corner -> voxel (0,0,0)
                    [-0.5, -0.75, -0.25],     # exactly on faces -> (2,1,1)
                    [-0.0001, -0.26, -0.01],  # just below faces -> (3,2,1)
                    [0.0, 0.0, 0.0],          # x at the upper grid bound -> dropped
                    [-1.0001, -0.9, -0.4],    # below the lower bound -> dropped
                    ], np.float32)
    occ = orc.occupancy(pts, spec.dims, spec.origin, spec.voxel)
    ref = np.zeros((2, 3, 4), np.uint8)
    ref[0, 0, 0] = 1
    ref[1, 1, 2] = 1
    ref[1, 2, 3] = 1
    np.testing.assert_array_equal(occ, ref)
