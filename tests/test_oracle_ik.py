"""Pins of the oracle's collision-free inverse kinematics (Sec. 3.2, eq. IK opt).

The SO(3) logarithm and its inverse right Jacobian are checked against
scipy's rotation-vector conversions (an independent implementation of the
exponential and logarithm maps); the residual against the oracle's forward
kinematics and distances (pinned elsewhere) term by term; its Jacobian
against central differences of the residual; the passive-joint term against
the hanging equilibrium of the load; and the Levenberg-Marquardt loop
against MINPACK's (scipy.optimize.least_squares, method 'lm') on the same
residual, and against exact reachability (FK(q_d) = H_d).
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy.optimize import least_squares
from scipy.spatial.transform import Rotation

from paper_2503_14160_amd import synth


def _exp(w):
    return Rotation.from_rotvec(np.asarray(w, np.float64)).as_matrix()


def _crane():
    base = synth.c1_full()
    return base, synth.with_self_collision(base.robot)


def _open(orc, robot):
    """The crane over bare ground (the c1 forest is too dense for most poses)."""
    ground = synth.Scene(cyl=np.zeros((0, 5), np.float32), box=np.zeros((0, 6), np.float32), has_ground=1,
                         ground_z=0.0)
    return orc.Model(robot, ground, None)


def _pose(orc, m, q):
    frames, _, tip = orc.fk(m, q)
    return np.concatenate([frames[-1, :9], tip])


# ----------------------------------------------------------------------------
# SO(3)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("theta", [0.0, 1e-9, 1e-4, 0.3, 1.0, 2.0, 2.6, 2.8, 3.0, math.pi - 1e-6])
def test_so3_log_inverts_exp(orc, theta):
    rng = np.random.default_rng(int(theta * 1000) + 3)
    for _ in range(20):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        w = theta * n
        got = orc.so3_log(_exp(w))
        # near pi the axis comes from the symmetric part (accuracy ~ sqrt(eps) / (pi - theta) there)
        tol = 1e-12 if theta < 2.5 else 2e-8
        np.testing.assert_allclose(got, w, rtol=0, atol=tol)
        assert np.linalg.norm(got) <= math.pi + 1e-12


def test_so3_log_at_pi_and_identity(orc):
    assert np.array_equal(orc.so3_log(np.eye(3)), np.zeros(3))
    rng = np.random.default_rng(5)
    for _ in range(20):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        R = _exp(math.pi * n)
        w = orc.so3_log(R)
        # a half turn has two rotation vectors, +-pi n: either maps back to R
        assert abs(np.linalg.norm(w) - math.pi) < 1e-12
        assert min(np.linalg.norm(w - math.pi * n), np.linalg.norm(w + math.pi * n)) < 1e-7
        np.testing.assert_allclose(_exp(w), R, atol=1e-12)
    # agrees with scipy's logarithm on random rotations
    for R in Rotation.random(50, random_state=9).as_matrix():
        np.testing.assert_allclose(orc.so3_log(R), Rotation.from_matrix(R).as_rotvec(), atol=1e-9)


@pytest.mark.parametrize("theta", [0.0, 1e-3, 5e-3, 0.02, 0.5, 1.5, 2.5, 3.0])
def test_so3_jr_inv_is_the_derivative_of_log(orc, theta):
    """J_r^-1(w) e = d/dt Log(Exp(w) Exp(t e)) at t = 0 (central differences
    through scipy's maps)."""
    rng = np.random.default_rng(17)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    w = theta * n
    Ji = orc.so3_jr_inv(w)
    h = 1e-6
    fd = np.zeros((3, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        wp = Rotation.from_matrix(_exp(w) @ _exp(e)).as_rotvec()
        wm = Rotation.from_matrix(_exp(w) @ _exp(-e)).as_rotvec()
        fd[:, k] = (wp - wm) / (2 * h)
    np.testing.assert_allclose(Ji, fd, atol=2e-8)
    # at w = 0 it is the identity; its inverse is the right Jacobian of Exp
    if theta == 0.0:
        assert np.array_equal(Ji, np.eye(3))


# ----------------------------------------------------------------------------
# residual
# ----------------------------------------------------------------------------

def test_residual_terms(orc):
    base, robot = _crane()
    m = orc.Model(robot, base.scene, None)
    par = synth.IkParams(lambda_q=0.7, lambda_c=3.0, lambda_e=0.4, lambda_r=0.05)
    rng = np.random.default_rng(2)
    Q = synth.random_configs(rng, robot, 40).astype(np.float64)
    Q[:, 4:] = rng.uniform(-1.0, 1.0, size=(40, 2))
    qstar = synth.random_configs(rng, robot, 40).astype(np.float64)
    d_all, _, _, _ = orc.eval_configs(m, Q)
    n_coll = 0
    for i in range(40):
        tgt = _pose(orc, m, qstar[i])
        q, qr = Q[i], qstar[(i + 1) % 40]
        r, _, info = orc.ik_residual(m, par, tgt, q, qr, jacobian=False)
        frames, _, tip = orc.fk(m, q)
        Rg = frames[-1, :9].reshape(3, 3)
        Rd = tgt[:9].reshape(3, 3)
        np.testing.assert_allclose(r[:3], tip - tgt[9:], atol=1e-13)
        np.testing.assert_allclose(r[3:6], 0.7 * Rotation.from_matrix(Rd.T @ Rg).as_rotvec(), atol=1e-9)
        assert r[6] == pytest.approx(3.0 * max(0.0, -d_all[i]), abs=1e-13)
        n_coll += d_all[i] < 0
        # g_p,j = d z_tip / d q_j over the passive joints, by central differences of the tip
        gp = []
        for j in np.where(robot.active == 0)[0]:
            e = np.zeros(6)
            e[j] = 1e-6
            gp.append((orc.fk(m, q + e)[2][2] - orc.fk(m, q - e)[2][2]) / 2e-6)
        assert r[7] == pytest.approx(0.4 * float(np.dot(gp, gp)), rel=1e-7, abs=1e-12)
        np.testing.assert_allclose(r[8:], 0.05 * (q - qr), atol=1e-15)
        assert info[0] == pytest.approx(np.linalg.norm(tip - tgt[9:]), abs=1e-13)
        assert info[2] == pytest.approx(d_all[i], abs=1e-13)
    assert n_coll >= 3  # the collision term is exercised


def test_residual_vanishes_at_the_target_configuration(orc):
    base, robot = _crane()
    m = orc.Model(robot, base.scene, None)
    par = synth.IkParams()
    rng = np.random.default_rng(4)
    for q in synth.hanging_configs(rng, robot, 16).astype(np.float64):
        q[5] = q[1] + q[2]  # the swing cancels the arm's pitch exactly (the generator rounds to FP32)
        r, _, info = orc.ik_residual(m, par, _pose(orc, m, q), q, q, jacobian=False)
        assert np.max(np.abs(r[:6])) < 1e-13
        assert np.all(r[8:] == 0.0)
        # the hanger hangs straight down: no gravity torque on the swing joints
        assert r[7] < 1e-28 and info[3] < 1e-14
        frames, _, tip = orc.fk(m, q)
        hang = tip - frames[-1, 9:12]
        np.testing.assert_allclose(hang / np.linalg.norm(hang), [0, 0, -1], atol=1e-14)


def test_residual_jacobian_matches_central_differences(orc):
    base, robot = _crane()
    m = orc.Model(robot, base.scene, None)
    par = synth.IkParams(lambda_q=0.8, lambda_c=5.0, lambda_e=2.0, lambda_r=0.1)
    rng = np.random.default_rng(6)
    Q = synth.random_configs(rng, robot, 200).astype(np.float64)
    Q[:, 4:] = rng.uniform(-1.2, 1.2, size=(200, 2))
    d, _, _, sec = orc.eval_configs(m, Q)
    # away from argmin switches and from the hinge's kink
    keep = (np.abs(sec - d) > 1e-4) & (np.abs(d) > 1e-4)
    Q = Q[keep][:60]
    tgt = _pose(orc, m, synth.random_configs(rng, robot, 1)[0].astype(np.float64))
    qr = np.zeros(6)
    n_coll = 0
    for q in Q:
        r, J, _ = orc.ik_residual(m, par, tgt, q, qr)
        # stay off the cut locus of Log (|w| = pi)
        if np.linalg.norm(r[3:6]) / 0.8 > 3.0:
            continue
        n_coll += r[6] > 0
        h = 1e-6
        fd = np.zeros_like(J)
        for j in range(6):
            e = np.zeros(6)
            e[j] = h
            fd[:, j] = (orc.ik_residual(m, par, tgt, q + e, qr, False)[0] -
                        orc.ik_residual(m, par, tgt, q - e, qr, False)[0]) / (2 * h)
        np.testing.assert_allclose(J, fd, rtol=1e-6, atol=1e-7)
    assert n_coll >= 3


# ----------------------------------------------------------------------------
# Levenberg-Marquardt
# ----------------------------------------------------------------------------

def test_lm_reaches_reachable_poses_exactly(orc):
    """lambda_r = 0, collision-free targets: the solver drives the pose error
    to zero from a start near the generating configuration."""
    base, robot = _crane()
    m = _open(orc, robot)
    par = synth.IkParams(lambda_r=0.0, max_iters=100, eps_grad=1e-14, eps_step=1e-15)
    rng = np.random.default_rng(8)
    Q = synth.hanging_configs(rng, robot, 60).astype(np.float64)
    d, _, _, _ = orc.eval_configs(m, Q)
    Q = Q[d > 0.3][:12]
    assert len(Q) == 12
    for q in Q:
        q0 = q + rng.uniform(-0.15, 0.15, size=6)
        trace = []
        qs, F, info, it, status = orc.ik_solve(m, par, _pose(orc, m, q), q0, q, trace=trace)
        assert info[0] < 1e-10 and info[1] < 1e-10, (info, it, status)
        # accepted iterates never raise the cost
        Fs = [t[1] for t in trace]
        assert all(b < a for a, b in zip(Fs, Fs[1:]))
        assert F == Fs[-1]


def test_lm_stops_on_the_gradient_and_step_tests(orc):
    base, robot = _crane()
    m = _open(orc, robot)
    rng = np.random.default_rng(10)
    q = synth.hanging_configs(rng, robot, 1)[0].astype(np.float64)
    q[5] = q[1] + q[2]
    tgt = _pose(orc, m, q)
    # started at the solution: the gradient test passes before any step
    par = synth.IkParams(eps_grad=1e-9)
    qs, F, info, it, status = orc.ik_solve(m, par, tgt, q, q)
    assert (status, it) == (1, 0) and np.array_equal(qs, q) and F == 0.0
    # no iterations allowed: the start (clamped to the limits) is returned
    par0 = synth.IkParams(max_iters=0)
    q_out = q.copy()
    q_out[3] = 5.0
    qs, F, info, it, status = orc.ik_solve(m, par0, tgt, q_out, q)
    assert status == 0 and it == 0 and qs[3] == pytest.approx(robot.q_max[3])
    # a huge step tolerance stops at once with status 2
    par2 = synth.IkParams(eps_step=1e6, eps_grad=0.0)
    qs, F, info, it, status = orc.ik_solve(m, par2, tgt, q + 0.1, q)
    assert (status, it) == (2, 0)


def test_lm_matches_minpack_on_the_same_residual(orc):
    """Unclamped, from the same start, the oracle's LM and MINPACK's reach the
    same local minimum of |r|^2 (collision-free targets, regularised)."""
    base, robot = _crane()
    m = _open(orc, robot)
    par = synth.IkParams(lambda_q=0.5, lambda_c=10.0, lambda_e=1.0, lambda_r=0.05, max_iters=200,
                         eps_grad=1e-13, eps_step=1e-14, clamp=0)
    rng = np.random.default_rng(12)
    Q = synth.hanging_configs(rng, robot, 60).astype(np.float64)
    d, _, _, _ = orc.eval_configs(m, Q)
    Q = Q[d > 0.3][:8]
    q_ref = base.q_start.astype(np.float64)
    for q in Q:
        tgt = _pose(orc, m, q)
        q0 = q + rng.uniform(-0.2, 0.2, size=6)
        qs, F, info, it, status = orc.ik_solve(m, par, tgt, q0, q_ref)
        ref = least_squares(lambda x: orc.ik_residual(m, par, tgt, x, q_ref, False)[0], q0,
                            jac=lambda x: orc.ik_residual(m, par, tgt, x, q_ref)[1], method="lm",
                            xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=2000)
        assert status in (1, 2)
        assert F == pytest.approx(0.5 * float(ref.fun @ ref.fun), rel=1e-9, abs=1e-20)
        np.testing.assert_allclose(qs, ref.x, atol=1e-7)


def test_lm_collision_term_pushes_out_of_obstacles(orc):
    """A target whose exact solution puts the crane inside a tree: with a
    large collision weight the solution is pushed out to near contact, with
    the pose error traded for it; with lambda_c = 0 the pose is reached."""
    base, robot = _crane()
    rng = np.random.default_rng(14)
    q = synth.hanging_configs(rng, robot, 1)[0].astype(np.float64)
    empty = synth.Scene(cyl=np.zeros((0, 5), np.float32), box=np.zeros((0, 6), np.float32), has_ground=1,
                        ground_z=0.0)
    m0 = orc.Model(robot, empty, None)
    frames, cen, tip = orc.fk(m0, q)
    # a tree of radius 0.3 m through the middle of the hanger
    mid = 0.5 * (frames[-1, 9:12] + tip)
    scene = dataclasses.replace(empty, cyl=np.array([[mid[0], mid[1], 0.3, 0.0, 15.0]], np.float32))
    m = orc.Model(robot, scene, None)
    assert orc.eval_configs(m, q[None])[0][0] < -0.2
    tgt = _pose(orc, m, q)
    free = synth.IkParams(lambda_c=0.0, lambda_r=0.0, max_iters=100)
    qs, F, info, it, status = orc.ik_solve(m, free, tgt, q + 0.05, q)
    assert info[0] < 1e-8 and info[2] < -0.2
    hard = synth.IkParams(lambda_c=100.0, lambda_r=0.0, max_iters=200)
    qs, F, info, it, status = orc.ik_solve(m, hard, tgt, q + 0.05, q)
    assert info[2] > -0.05 and info[0] > 0.1
