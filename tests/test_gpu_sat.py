"""The separating-axis narrow phase on the GPU (Sec. 3.1) against the oracle,
through the C ABI: the c1 crane's link hulls (with its non-adjacent link
pairs) against the c1 forest as oriented boxes (512 upright prisms turned
about z, 16 log piles) and the ground.

Tolerances: SAT distances within EPS_SAT = 3e-4 m.  FP32 placement of the
boxes at 20-40 m from the origin carries about 2e-5 m of position error (as
for the spheres) and about 1e-6 of rotation error in the cosines between box
axes; a cross axis a_i x b_j turns by that error over its length, at least
sqrt(0.01) = 0.1, and the gap along it moves by the turn times the lever
|T| + the half extents (at most about 20 m here): 2e-5 + 20 x 1e-6 / 0.1 =
2.2e-4 m.  The argmin pair is compared where the oracle's runner-up is more
than 2 EPS_SAT away; costs as the sphere evaluation's with EPS_SAT in place
of its distance tolerance; flags unless the oracle's minimum distance is
within EPS_SAT of the margin.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2503_14160_amd import synth

pytestmark = pytest.mark.gpu

EPS_SAT = 3e-4


@pytest.fixture(scope="module")
def cp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_14160_amd import craneplan
    craneplan.lib()
    return craneplan


def _sat_problem(n_cyl=None, seed=77):
    base = synth.c1_full()
    robot = synth.with_self_collision(synth.with_hulls(base.robot))
    scene = base.scene if n_cyl is None else dataclasses.replace(base.scene, cyl=base.scene.cyl[:n_cyl])
    scene = synth.hull_scene(np.random.default_rng(seed), scene)
    return base, robot, scene


def test_sat_config_distance_parity(cp):
    base, robot, scene = _sat_problem()
    rng = np.random.default_rng(401)
    N = 1024
    Q = synth.random_configs(rng, robot, N)
    Q[:, 4:] = rng.uniform(-1.2, 1.2, size=(N, 2)).astype(np.float32)
    plan = cp.Plan(robot, scene, base.cost, max_B=1)
    print(f"[sat configs] N={N}, {scene.n_obb} boxes, {len(robot.hull_box)} hulls", flush=True)
    d, a = plan.debug_configs(torch.from_numpy(Q).cuda())
    d = d.cpu().numpy().astype(np.float64)
    a = a.cpu().numpy().view(np.uint32)
    m = oracle.Model(robot, scene, None)
    dr, sr, orr, sec = oracle.eval_configs(m, Q.astype(np.float64))
    err = np.abs(d - dr)
    print(f"[sat configs] max |dd| = {err.max():.2e} m, collisions {np.mean(dr < 0):.2f}", flush=True)
    assert np.all(err <= EPS_SAT), (np.argmax(err), err.max())
    uniq = (sec - dr) > 2 * EPS_SAT
    assert uniq.mean() > 0.8
    np.testing.assert_array_equal(a[uniq] >> 16, sr[uniq])
    np.testing.assert_array_equal(a[uniq] & 0xFFFF, orr[uniq])
    # every kind of obstacle takes part: ground, boxes, self pairs
    kinds = orr[uniq]
    assert (kinds == 0).any() and ((kinds > 0) & (kinds < 0xFF00)).any() and (kinds >= 0xFF00).any()


def test_sat_eval_parity(cp):
    """Path costs, minimum distances, flags and tapes in SAT mode (reduced
    checkpoint count so the oracle finishes in seconds; several tiles and a
    ragged last wave)."""
    base, robot, scene = _sat_problem()
    cost = dataclasses.replace(base.cost, M=8)
    B = 12
    rng = np.random.default_rng(402)
    W = synth.random_waypoints(rng, robot, base.q_start, base.q_goal, B, cost.K, sigma=0.3)
    plan = cp.Plan(robot, scene, cost, max_B=B)
    plan.set_endpoints(base.q_start, base.q_goal)
    print(f"[sat eval] B={B} n_s={plan.n_s}", flush=True)
    c, md, fl, tape = plan.eval(torch.from_numpy(W).cuda(), tape=True)
    m = oracle.Model(robot, scene, cost)
    ref = oracle.eval_paths(m, base.q_start, base.q_goal, W.astype(np.float64), per_checkpoint=True)
    c = c.cpu().numpy().astype(np.float64)
    md = md.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(md - ref["min_dist"]) <= EPS_SAT)
    near = np.abs(ref["min_dist"] - cost.margin) <= EPS_SAT
    np.testing.assert_array_equal(fl.cpu().numpy()[~near], (ref["min_dist"] < cost.margin)[~near])
    n_act = ((ref["d"] < cost.margin + EPS_SAT)).sum(1)
    tol = 1e-5 * np.abs(ref["cost"]) + cost.w_c * cost.lambda_c * EPS_SAT * n_act + 2 * cost.w_l * 1e-6 * np.sqrt(
        plan.n_s * 6 * np.maximum(ref["cost"], 0)) + 1e-6
    assert np.all(np.abs(c - ref["cost"]) <= tol), np.max(np.abs(c - ref["cost"]) / tol)
    tp = tape.cpu().numpy().view(np.uint32)
    uniq = (ref["second"] - ref["d"]) > 2 * EPS_SAT
    tr = ref["tape"].view(np.uint32)
    np.testing.assert_array_equal(tp[uniq], tr[uniq])


def test_sat_eval_full_size_sampled(cp):
    """The c1 population size (16384 paths x 608 checkpoints) in one launch;
    sampled paths (first and last included) against the oracle."""
    base, robot, scene = _sat_problem()
    cost = base.cost
    B = base.opt.B
    rng = np.random.default_rng(403)
    W = synth.random_waypoints(rng, robot, base.q_start, base.q_goal, B, cost.K, sigma=0.25)
    plan = cp.Plan(robot, scene, cost, max_B=B)
    plan.set_endpoints(base.q_start, base.q_goal)
    print(f"[sat eval full] B={B} n_s={plan.n_s}", flush=True)
    c, md, fl = plan.eval(torch.from_numpy(W).cuda())
    idx = np.array([0, B - 1, 4097, 9999])
    m = oracle.Model(robot, scene, cost)
    ref = oracle.eval_paths(m, base.q_start, base.q_goal, W[idx].astype(np.float64))
    c = c.cpu().numpy()[idx].astype(np.float64)
    md = md.cpu().numpy()[idx].astype(np.float64)
    assert np.all(np.abs(md - ref["min_dist"]) <= EPS_SAT)
    assert np.all(np.abs(c - ref["cost"]) <= 1e-5 * np.abs(ref["cost"]) + cost.w_c * cost.lambda_c * EPS_SAT *
                  plan.n_s + 1e-3)


def test_sat_optimizer_one_step(cp):
    """One optimizer iteration in SAT mode: the device's samples evaluated by
    the oracle match the device's costs, and the elites are the first nu of
    the stable order on the device's costs."""
    base, robot, scene = _sat_problem(n_cyl=128)
    cost = dataclasses.replace(base.cost, K=6, M=8)
    opt = synth.OptParams(B=256, nu=16, sigma0=0.2, eps=1e-6, seed=9, T=1)
    plan = cp.Plan(robot, scene, cost, max_B=opt.B)
    plan.set_endpoints(base.q_start, base.q_goal)
    o = cp.Optimizer(plan, opt)
    o.step(1)
    W, costs, elite = o.last()
    W = W.cpu().numpy().astype(np.float64)
    costs = costs.cpu().numpy().astype(np.float64)
    elite = elite.cpu().numpy()
    m = oracle.Model(robot, scene, cost)
    ref = oracle.eval_paths(m, base.q_start, base.q_goal, W)
    tol = 1e-5 * np.abs(ref["cost"]) + cost.w_c * cost.lambda_c * EPS_SAT * plan.n_s + 1e-6
    assert np.all(np.abs(costs - ref["cost"]) <= tol)
    # the elite set of the device's own costs is the stable order's first nu
    order = np.lexsort((np.arange(opt.B), costs.astype(np.float32)))
    np.testing.assert_array_equal(elite, order[:opt.nu])


def test_sat_refusals(cp):
    """No adjoint in SAT mode: the backward pass, the polish, the population
    gradient and the IK refuse it; batches take the sphere narrow phase."""
    base, robot, scene = _sat_problem(n_cyl=32)
    plan = cp.Plan(robot, scene, base.cost, max_B=4)
    plan.set_endpoints(base.q_start, base.q_goal)
    W = torch.zeros((4, base.cost.K, 6), device="cuda")
    with pytest.raises(cp.CranePlanError) as ei:
        plan.backward(W, torch.ones(4, device="cuda"))
    assert "adjoint" in str(ei.value)
    with pytest.raises(cp.CranePlanError):
        cp.Optimizer(plan, synth.OptParams(B=4, nu=2, sigma0=0.2, eps=1e-6, seed=1, T=1, polish_elites=2,
                                           polish_steps=3))
    o = cp.Optimizer(plan, synth.OptParams(B=4, nu=2, sigma0=0.2, eps=1e-6, seed=1, T=1))
    with pytest.raises(cp.CranePlanError):
        o.record_tape(True)
    T = torch.zeros((1, 12), device="cuda")
    with pytest.raises(cp.CranePlanError):
        plan.ik_solve(synth.IkParams(), T, torch.zeros((1, 6), device="cuda"))
    p = dataclasses.replace(synth.c0_plain(), scene=scene, robot=robot)
    p.opt = synth.OptParams(B=16, nu=2, sigma0=0.2, eps=1e-6, seed=1, T=1)
    with pytest.raises(cp.CranePlanError):
        cp.Batch([p])


def test_sat_early_exit_is_exact(cp):
    """Stopping a pair after the box's face axes (every pair_filter but
    CP_PAIRS_ALL) gives bitwise the results of taking every axis: costs,
    minimum distances, flags, tapes and configuration distances with their
    pairs, on random paths and random configurations (many in collision)."""
    base, robot, scene = _sat_problem()
    cost = dataclasses.replace(base.cost, M=16)
    B = 300
    rng = np.random.default_rng(404)
    W = torch.from_numpy(synth.random_waypoints(rng, robot, base.q_start, base.q_goal, B, cost.K, sigma=0.4)).cuda()
    Q = synth.random_configs(rng, robot, 2000)
    Q[:, 4:] = rng.uniform(-1.2, 1.2, size=(2000, 2)).astype(np.float32)
    Q = torch.from_numpy(Q).cuda()
    out = {}
    for mode in (cp.PAIRS_ALL, cp.PAIRS_LANE, cp.PAIRS_WAVE, cp.PAIRS_AUTO):
        plan = cp.Plan(robot, scene, cost, max_B=B, pair_filter=mode)
        plan.set_endpoints(base.q_start, base.q_goal)
        out[mode] = plan.eval(W, tape=True) + plan.debug_configs(Q)
    for mode in (cp.PAIRS_LANE, cp.PAIRS_WAVE, cp.PAIRS_AUTO):
        for a, b in zip(out[cp.PAIRS_ALL], out[mode]):
            assert torch.equal(a, b), mode
