"""Pins of the oracle's step two (Sec. 4.2, eq. discrete) and of its reduced
dynamics (Sec. 2.1, state-space form).

Dynamics: rest at a hanging configuration, the pendulum frequency sqrt(g/l)
of the load, energy conservation of a free swing integrated by Runge-Kutta,
d'Alembert's principle on the passive joints against second differences of
the tip, the actuated rows equal to the inputs, the damping term.
Collocation: a one-joint double integrator against its exact solution
(linear KKT system for fixed t_F, then a golden-section search on t_F), and
the crane on a short horizon against scipy's SLSQP on the same nonlinear
programme; defects and boundary conditions at the solution.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

from paper_2503_14160_amd import synth


def _crane():
    base = synth.c1_full()
    return base, base.robot


def _hanging(robot, seed=3):
    q = synth.hanging_configs(np.random.default_rng(seed), robot, 1)[0].astype(np.float64)
    q[5] = q[1] + q[2]
    return q


def _empty():
    return synth.Scene(cyl=np.zeros((0, 5), np.float32), box=np.zeros((0, 6), np.float32), has_ground=0)


def _tip(orc, m, q):
    return orc.fk(m, q)[2]


# ----------------------------------------------------------------------------
# dynamics
# ----------------------------------------------------------------------------

def test_rest_at_a_hanging_configuration(orc):
    base, robot = _crane()
    m = orc.Model(robot, _empty(), None)
    q = _hanging(robot)
    qdd = orc.crane_accel(m, q, np.zeros(6), np.zeros(4), 9.81, 0.5)
    assert np.max(np.abs(qdd)) < 1e-12


def test_actuated_rows_and_damping(orc):
    base, robot = _crane()
    m = orc.Model(robot, _empty(), None)
    rng = np.random.default_rng(4)
    for _ in range(20):
        q = synth.random_configs(rng, robot, 1)[0].astype(np.float64)
        qd = rng.normal(size=6) * 0.3
        u = rng.normal(size=4)
        a0 = orc.crane_accel(m, q, qd, u, 9.81, 0.0)
        a1 = orc.crane_accel(m, q, qd, u, 9.81, 0.7)
        np.testing.assert_array_equal(a0[:4], u)
        np.testing.assert_allclose(a1[4:], a0[4:] - 0.7 * qd[4:], atol=1e-12)


def test_small_swings_have_the_pendulum_frequency(orc):
    """Crane at rest, load hanging: the passive joints' stiffness matrix
    d qdd_p / d q_p has both eigenvalues -g / l, l the hanger length."""
    base, robot = _crane()
    m = orc.Model(robot, _empty(), None)
    q = _hanging(robot)
    l = float(robot.link_lengths[4])
    K = np.zeros((2, 2))
    h = 1e-6
    for j in range(2):
        e = np.zeros(6)
        e[4 + j] = h
        K[:, j] = (orc.crane_accel(m, q + e, np.zeros(6), np.zeros(4), 9.81, 0.0)[4:] -
                   orc.crane_accel(m, q - e, np.zeros(6), np.zeros(4), 9.81, 0.0)[4:]) / (2 * h)
    np.testing.assert_allclose(np.sort(np.linalg.eigvals(K).real), [-9.81 / l] * 2, rtol=1e-7)


def test_free_swing_conserves_energy(orc):
    """Actuated joints at rest, no damping: the load's energy
    |v_tip|^2 / 2 + g z_tip is constant along the motion (RK4, 1 ms steps)."""
    base, robot = _crane()
    m = orc.Model(robot, _empty(), None)
    q = _hanging(robot)
    q[4] += 0.3
    q[5] -= 0.25
    x = np.concatenate([q, np.zeros(6)])

    def f(x):
        return np.concatenate([x[6:], orc.crane_accel(m, x[:6], x[6:], np.zeros(4), 9.81, 0.0)])

    def energy(x):
        h = 1e-6
        v = (_tip(orc, m, x[:6] + h * x[6:]) - _tip(orc, m, x[:6] - h * x[6:])) / (2 * h)
        return 0.5 * float(v @ v) + 9.81 * float(_tip(orc, m, x[:6])[2])

    E0 = energy(x)
    dt = 1e-3
    swing = 0.0
    for _ in range(2000):
        k1 = f(x)
        k2 = f(x + 0.5 * dt * k1)
        k3 = f(x + 0.5 * dt * k2)
        k4 = f(x + dt * k3)
        x = x + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        swing = max(swing, abs(x[10]))
    assert swing > 0.5  # it did swing
    assert abs(energy(x) - E0) < 1e-8 * max(abs(E0), 1.0)
    np.testing.assert_array_equal(x[:4], q[:4])


def test_passive_joints_feel_no_force(orc):
    """d'Alembert on the passive joints: J_p^T (tip'' + g e_z) = 0, the tip's
    acceleration taken by second differences of its position along
    q + t qd + t^2 qdd / 2."""
    base, robot = _crane()
    m = orc.Model(robot, _empty(), None)
    rng = np.random.default_rng(5)
    for _ in range(20):
        q = synth.random_configs(rng, robot, 1)[0].astype(np.float64)
        q[4:] = rng.uniform(-0.8, 0.8, 2)
        qd = rng.normal(size=6) * 0.4
        u = rng.normal(size=4) * 0.5
        qdd = orc.crane_accel(m, q, qd, u, 9.81, 0.0)
        t = 1e-4
        pos = [_tip(orc, m, q + s * qd + 0.5 * s * s * qdd) for s in (-t, 0.0, t)]
        acc = (pos[0] - 2 * pos[1] + pos[2]) / (t * t)
        for j in (4, 5):
            e = np.zeros(6)
            e[j] = 1e-6
            Jj = (_tip(orc, m, q + e) - _tip(orc, m, q - e)) / 2e-6
            assert abs(Jj @ (acc + np.array([0, 0, 9.81]))) < 1e-5 * (1 + np.linalg.norm(acc))


# ----------------------------------------------------------------------------
# collocation
# ----------------------------------------------------------------------------

def _slider():
    """One prismatic joint along x, actuated: a double integrator."""
    f32 = np.float32
    return synth.Robot(joint_type=np.array([synth.PRISMATIC], np.int32), axis=f32([[1, 0, 0]]), origin=f32([[0, 0, 0]]),
                       q_min=f32([-10.0]), q_max=f32([10.0]), q_hold=f32([0.0]), active=np.array([1], np.uint8),
                       sphere_frame=np.array([1], np.int32), sphere_center=f32([[0, 0, 0]]),
                       sphere_radius=f32([0.1]), tip=f32([0, 0, 0]), link_lengths=f32([1, 1, 1, 1, 1]))


def test_double_integrator_against_its_exact_solution(orc):
    """For the slider the defects are linear in (x, u) once t_F is fixed, so
    the problem is an equality-constrained least squares solved exactly by
    its KKT system; a golden-section search over t_F then gives the
    optimum, which the augmented-Lagrangian LM must reach."""
    robot = _slider()
    m = orc.Model(robot, _empty(), None)
    N = 10
    par = synth.TrajParams(N=N, omega_s=0.5, omega_t=0.0, v_max=(10.0,), damping=0.0, t_f0=3.0, outer=6,
                           max_iters=60)
    q0, qd = np.array([0.0]), np.array([2.0])
    qstar = np.linspace(0.0, 2.0, N + 1)[:, None]
    res = orc.traj_refine(m, par, q0, qd, qstar)

    def inner(T):
        # unknowns per point k: x_k = (p, v) for 1..N-1 and u_k for 0..N
        h = T / N
        nx = 2 * (N - 1)
        nz = nx + N + 1
        xi = lambda k: 2 * (k - 1)
        ui = lambda k: nx + k
        A = np.zeros((2 * N, nz))
        b = np.zeros(2 * N)
        X0, XN = np.array([0.0, 0.0]), np.array([2.0, 0.0])
        for k in range(N):
            # p_{k+1} - p_k - h/2 (v_k + v_{k+1}) = 0 ; v_{k+1} - v_k - h/2 (u_k + u_{k+1}) = 0
            for which, sign in ((k, -1.0), (k + 1, 1.0)):
                if 0 < which < N:
                    A[2 * k, xi(which)] += sign
                    A[2 * k, xi(which) + 1] += -h / 2
                    A[2 * k + 1, xi(which) + 1] += sign
                else:
                    Xf = X0 if which == 0 else XN
                    b[2 * k] -= sign * Xf[0] - h / 2 * Xf[1]
                    b[2 * k + 1] -= sign * Xf[1]
                A[2 * k + 1, ui(which)] += -h / 2
        H = np.zeros((nz, nz))
        for k in range(1, N + 1):
            H[ui(k), ui(k)] = 2 * par.omega_s
        K = np.block([[H, A.T], [A, np.zeros((2 * N, 2 * N))]])
        sol = np.linalg.solve(K, np.concatenate([np.zeros(nz), b]))
        z = sol[:nz]
        return T + 0.5 * z @ H @ z

    best = minimize_scalar(inner, bounds=(0.5, 10.0), method="bounded", options=dict(xatol=1e-10))
    assert res["defect"] < 1e-7
    assert res["t_f"] == pytest.approx(best.x, rel=1e-5)
    J_res = res["t_f"] + par.omega_s * float(np.sum(res["U"][1:] ** 2))
    assert J_res == pytest.approx(best.fun, rel=1e-7)


def test_crane_against_slsqp(orc):
    """The crane on a short horizon (N = 5, a small slew and boom move):
    SLSQP on the same nonlinear programme (objective, defect equalities,
    state bounds as inequalities) reaches the same t_F and trajectory."""
    base, robot = _crane()
    m = orc.Model(robot, _empty(), None)
    N = 5
    par = synth.TrajParams(N=N, omega_s=0.2, omega_t=5.0, t_f0=6.0, outer=6, max_iters=80, damping=0.5)
    q0 = _hanging(robot, 7)
    qd = q0.copy()
    qd[0] += 0.4
    qd[1] += 0.1
    qd[5] += 0.1
    qstar = q0 + np.linspace(0, 1, N + 1)[:, None] * (qd - q0)
    res = orc.traj_refine(m, par, q0, qd, qstar)
    assert res["defect"] < 1e-7
    L = orc.TrajLayout(6, 4, N)
    lam0 = np.zeros((N, 12))

    def obj(z):
        r, _ = orc.traj_residual(m, par, q0, qd, qstar, z, lam0, 1.0, jacobian=False)
        return float(r[L.r_u:L.r_t] @ r[L.r_u:L.r_t])

    def defects(z):
        r, _ = orc.traj_residual(m, par, q0, qd, qstar, z, lam0, 1.0, jacobian=False)
        return r[:N * 12]

    lo, hi = orc._traj_bounds(m, par)
    cons = [dict(type="eq", fun=defects)]
    bounds = [(None, None)] * L.nz
    for k in range(1, N):
        for i in range(12):
            bounds[L.off[k] + i] = (lo[i], hi[i])
    ref = minimize(obj, orc.traj_initial(m, par, q0, qd, qstar), method="SLSQP", constraints=cons, bounds=bounds,
                   options=dict(ftol=1e-14, maxiter=2000))
    assert ref.success, ref.message
    assert res["t_f"] == pytest.approx(ref.x[L.s] ** 2, rel=1e-4)
    np.testing.assert_allclose(res["z"][:L.s], ref.x[:L.s], atol=2e-4)
    assert np.all(np.abs(defects(ref.x)) < 1e-8)


def test_low_first_penalty_does_not_collapse_the_final_time(orc):
    """With a first penalty of 100 a long move can be cheaper to leave
    infeasible at t_F -> 0 (the defects then cost about mu |q_d - q_0|^2 /
    (2 N), less than the time the move takes), and at s = 0 every residual
    is stationary in s: without a bound this case ends at t_F ~ 1e-136 with
    defects of 0.03.  The bound t_F >= t_min, which the velocity limits
    imply, keeps the solver off that point: it must end feasible, within
    the velocity limits, and so above t_min."""
    from traj_cases import problems
    base, robot = _crane()
    m = orc.Model(robot, _empty(), None)
    N = 12
    par = synth.TrajParams(N=N, t_f0=6.0, mu0=100.0, outer=6, max_iters=200)
    q0, qd, qstar = (a[2].astype(np.float64) for a in problems(robot, 4, N, 501))
    t_min = orc.traj_t_min(m, par, q0, qd)
    assert t_min == pytest.approx(np.max(np.abs(qd - q0) / np.asarray(par.v_max)))
    res = orc.traj_refine(m, par, q0, qd, qstar)
    assert res["defect"] < 1e-8
    assert res["t_f"] > t_min
    v = res["X"][:, 6:]
    assert np.all(np.abs(v) <= np.asarray(par.v_max) + 1e-4)
    # the discrete bound the defects imply: |q_N - q_0| <= t_F max |qd|
    assert np.all(np.abs(qd - q0) <= res["t_f"] * np.abs(v).max(axis=0) + 1e-9)
