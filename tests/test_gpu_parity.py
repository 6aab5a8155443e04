"""HIP library vs the FP64 oracle, element by element, through the C ABI.

Tolerances (derived in the design notes):
* FK positions: |dp| <= 1e-5 max(|p|, 1 m).
* distances: |dd| <= EPS_D = 2e-5 m (a few units in the last place of FP32
  coordinates at the 20-40 m scene extent, accumulated through the chain).
* costs: |dJ| <= 1e-5 |J| + w_c lambda_c EPS_D N_act + 2 w_l EPS_Q sqrt(n_s n J_l)
  where N_act counts checkpoints whose oracle distance is within EPS_D of the
  hinge's active region; paths with no active checkpoint meet 1e-5 relative.
* flags: identical unless the oracle's min distance is within 1e-4 m of the
  margin.  Tape (argmin pair): identical where the oracle's runner-up pair is
  more than 2 EPS_D away.  Elites: identical where adjacent cost gaps exceed
  the cost tolerance.  Gradients: <= 1e-4 relative (norm per path).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2503_14160_amd import synth

pytestmark = pytest.mark.gpu

EPS_D = 2e-5
EPS_Q = 1e-6


@pytest.fixture(scope="module")
def cp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_14160_amd import craneplan
    craneplan.lib()
    return craneplan


def _cost_tol(ref, cost, n_joints):
    c = np.abs(ref["cost"])
    m = float(np.float32(cost.margin))
    if cost.hinge == synth.HINGE_HARD:
        act = ref["d"] < m + EPS_D
    else:
        act = ref["d"] < m + EPS_D
    n_act = act.sum(1)
    jl = ref["parts"][:, 2]
    ns = ref["d"].shape[1]
    return (1e-5 * c + cost.w_c * cost.lambda_c * EPS_D * n_act
            + 2 * cost.w_l * EPS_Q * np.sqrt(ns * n_joints * jl) + 1e-6), n_act


def _check_eval(cp, prob, W, plan=None, label=""):
    print(f"[eval parity] {label} B={W.shape[0]} K={prob.cost.K} M={prob.cost.M}", flush=True)
    if plan is None:
        plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=W.shape[0])
        plan.set_endpoints(prob.q_start, prob.q_goal)
    cost, md, fl, tape = plan.eval(torch.from_numpy(W).cuda(), tape=True)
    torch.cuda.synchronize()
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    ref = oracle.eval_paths(m, prob.q_start, prob.q_goal, W.astype(np.float64), per_checkpoint=True)
    c = cost.cpu().numpy().astype(np.float64)
    tol, n_act = _cost_tol(ref, prob.cost, prob.robot.n_joints)
    err = np.abs(c - ref["cost"])
    assert np.all(err <= tol), (label, np.max(err / tol), np.argmax(err / tol))
    free = n_act == 0
    if free.any():
        assert np.all(err[free] <= 1e-5 * np.abs(ref["cost"][free]) + 1e-7)
    if (~free).any():
        rel = err[~free] / np.maximum(np.abs(ref["cost"][~free]), 1e-12)
        print(f"[eval parity] {label}: largest relative cost error on colliding paths {rel.max():.2e} "
              f"({int((~free).sum())} paths)", flush=True)
    md = md.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(md - ref["min_dist"]) <= EPS_D), label
    margin = float(np.float32(prob.cost.margin))
    fl = fl.cpu().numpy()
    clear = np.abs(ref["min_dist"] - margin) > 1e-4
    np.testing.assert_array_equal(fl[clear], ref["flags"][clear])
    tape = tape.cpu().numpy().view(np.uint32)
    ok = (ref["second"] - ref["d"]) > 2 * EPS_D
    np.testing.assert_array_equal(tape[ok], ref["tape"].view(np.uint32)[ok])
    return plan, c, ref


# ----------------------------------------------------------------------------
# kinematics and distances
# ----------------------------------------------------------------------------

def test_fk_parity(cp):
    prob = synth.c1_full()
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=1)
    rng = np.random.default_rng(100)
    Q = synth.random_configs(rng, prob.robot, 512)
    cen, fr = plan.debug_fk(torch.from_numpy(Q).cuda())
    cen, fr = cen.cpu().numpy(), fr.cpu().numpy()
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    for i in range(Q.shape[0]):
        f_ref, c_ref, _ = oracle.fk(m, Q[i].astype(np.float64))
        scale = np.maximum(np.linalg.norm(c_ref, axis=1, keepdims=True), 1.0)
        assert np.all(np.abs(cen[i] - c_ref) <= 1e-5 * scale)
        np.testing.assert_allclose(fr[i][:, :9], f_ref[:, :9], atol=2e-6)
        pscale = np.maximum(np.linalg.norm(f_ref[:, 9:], axis=1, keepdims=True), 1.0)
        assert np.all(np.abs(fr[i][:, 9:] - f_ref[:, 9:]) <= 1e-5 * pscale)


def test_config_distance_parity(cp):
    prob = synth.c1_full()
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=1)
    rng = np.random.default_rng(101)
    Q = synth.random_configs(rng, prob.robot, 1024)
    d, a = plan.debug_configs(torch.from_numpy(Q).cuda())
    d, a = d.cpu().numpy().astype(np.float64), a.cpu().numpy().view(np.uint32)
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    dr, sr, orr, sec = oracle.eval_configs(m, Q.astype(np.float64))
    assert np.all(np.abs(d - dr) <= EPS_D)
    ok = (sec - dr) > 2 * EPS_D
    assert ok.mean() > 0.9
    np.testing.assert_array_equal(a[ok] >> 16, sr[ok])
    np.testing.assert_array_equal(a[ok] & 0xFFFF, orr[ok])


# ----------------------------------------------------------------------------
# path evaluation
# ----------------------------------------------------------------------------

def test_eval_parity_c0(cp):
    prob = synth.c0_plain()
    rng = np.random.default_rng(102)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 256, prob.cost.K, sigma=0.3)
    _check_eval(cp, prob, W, label="c0_plain")


@pytest.mark.parametrize("interp,jp,hinge,margin,K,M,B", [
    (synth.INTERP_BSPLINE, synth.JP_SQUARED, synth.HINGE_HARD, 0.0, 5, 7, 37),      # ragged, n_s = 56 < 64
    (synth.INTERP_LINEAR, synth.JP_L2, synth.HINGE_SMOOTH, 0.1, 3, 2, 51),         # n_s = 8: many paths per wave
    (synth.INTERP_BSPLINE, synth.JP_L2, synth.HINGE_HARD, 0.2, 12, 9, 1),          # one path
    (synth.INTERP_LINEAR, synth.JP_SQUARED, synth.HINGE_HARD, 0.05, 1, 1, 200),    # n_s = 2
])
def test_eval_parity_variants(cp, interp, jp, hinge, margin, K, M, B):
    base = synth.c0_plain()
    cost = synth.CostParams(K=K, M=M, interp=interp, jp_mode=jp, hinge=hinge, margin=margin)
    prob = synth.Problem("variant", base.robot, base.scene, base.q_start, base.q_goal, cost, base.opt)
    rng = np.random.default_rng(103 + K)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, B, K, sigma=0.4)
    _check_eval(cp, prob, W, label=f"interp={interp} jp={jp} hinge={hinge} K={K} M={M} B={B}")


def test_eval_nonfinite_waypoints(cp):
    prob = synth.c0_plain()
    rng = np.random.default_rng(104)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 8, prob.cost.K, sigma=0.3)
    W[3, 2, 1] = np.nan
    W[5, 0, 0] = np.inf
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=8)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    cost, md, fl = plan.eval(torch.from_numpy(W).cuda())
    c = cost.cpu().numpy()
    assert np.isnan(c[3]) and np.isnan(c[5])
    assert np.all(np.isfinite(np.delete(c, [3, 5])))


def test_eval_full_size_sampled(cp):
    """c1_full at its benchmark size (16384 paths x 608 checkpoints, 64
    spheres, 512 trees + 16 boxes): sampled paths against the oracle."""
    prob = synth.c1_full()
    B = prob.opt.B
    rng = np.random.default_rng(105)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, B, prob.cost.K, sigma=0.2)
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    print(f"[eval full] c1_full B={B} n_s={plan.n_s}", flush=True)
    cost, md, fl = plan.eval(torch.from_numpy(W).cuda())
    torch.cuda.synchronize()
    idx = np.sort(rng.choice(B, size=24, replace=False))
    idx[0], idx[-1] = 0, B - 1
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    ref = oracle.eval_paths(m, prob.q_start, prob.q_goal, W[idx].astype(np.float64), per_checkpoint=True)
    tol, _ = _cost_tol(ref, prob.cost, prob.robot.n_joints)
    c = cost.cpu().numpy()[idx].astype(np.float64)
    assert np.all(np.abs(c - ref["cost"]) <= tol)
    assert np.all(np.abs(md.cpu().numpy()[idx] - ref["min_dist"]) <= EPS_D)
    # the same paths evaluated in another batch position: the minimum is exact,
    # the sum only regroups (wave boundaries move), so it agrees to rounding
    cost2, md2, _ = plan.eval(torch.from_numpy(W[idx]).cuda())
    np.testing.assert_allclose(cost2.cpu().numpy(), cost.cpu().numpy()[idx], rtol=2e-7)
    np.testing.assert_array_equal(md2.cpu().numpy(), md.cpu().numpy()[idx])


def test_eval_c4_full_size_sampled(cp):
    """c4_sdf at its benchmark size: the grid built on the device from 1 M
    points (256 x 256 x 128), 65536 paths x 608 checkpoints evaluated in the
    benchmark's launch; sampled paths against the oracle, which builds its
    own grid from the same points."""
    prob = synth.c4_sdf()
    B, spec = prob.opt.B, prob.sdf
    print(f"[eval full] c4_sdf B={B} grid={spec.dims}", flush=True)
    sdf, occ, eo, ef = cp.sdf_build(torch.from_numpy(prob.lidar).cuda(), spec, with_edt=True)
    rng = np.random.default_rng(107)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, B, prob.cost.K, sigma=0.2)
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B, sdf=sdf, sdf_spec=spec)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    cost, md, fl = plan.eval(torch.from_numpy(W).cuda())
    torch.cuda.synchronize()
    phi_ref, occ_ref, eo_ref, ef_ref = oracle.sdf_build(prob.lidar, spec)
    # the full-size grid: occupancy and squared distances bit-exact
    np.testing.assert_array_equal(occ.cpu().numpy(), occ_ref)
    np.testing.assert_array_equal(eo.cpu().numpy(), eo_ref)
    np.testing.assert_array_equal(ef.cpu().numpy(), ef_ref)
    np.testing.assert_allclose(sdf.cpu().numpy(), phi_ref, rtol=2e-7, atol=1e-7)
    idx = np.sort(rng.choice(B, size=24, replace=False))
    idx[0], idx[-1] = 0, B - 1
    m = oracle.Model(prob.robot, prob.scene, prob.cost, sdf=phi_ref, sdf_spec=spec)
    ref = oracle.eval_paths(m, prob.q_start, prob.q_goal, W[idx].astype(np.float64), per_checkpoint=True)
    tol, _ = _cost_tol(ref, prob.cost, prob.robot.n_joints)
    c = cost.cpu().numpy()[idx].astype(np.float64)
    assert np.all(np.abs(c - ref["cost"]) <= tol)
    assert np.all(np.abs(md.cpu().numpy()[idx] - ref["min_dist"]) <= EPS_D)
    clear = np.abs(ref["min_dist"] - float(np.float32(prob.cost.margin))) > 1e-4
    np.testing.assert_array_equal(fl.cpu().numpy()[idx][clear], ref["flags"][clear])


def test_eval_deterministic(cp):
    prob = synth.c0_plain()
    rng = np.random.default_rng(106)
    W = torch.from_numpy(synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 256, prob.cost.K)).cuda()
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=256)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    a = plan.eval(W, tape=True)
    b = plan.eval(W, tape=True)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


# ----------------------------------------------------------------------------
# adjoint
# ----------------------------------------------------------------------------

def _diff_problem(B=24, K=16, M=32):
    base = synth.c1_full()
    cost = synth.CostParams(K=K, M=M, hinge=synth.HINGE_SMOOTH, margin=0.1)
    return synth.Problem("diff", base.robot, base.scene, base.q_start, base.q_goal, cost, base.opt)


def test_backward_parity(cp):
    prob = _diff_problem()
    rng = np.random.default_rng(107)
    B = 24
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, B, prob.cost.K, sigma=0.3)
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    Wt = torch.from_numpy(W).cuda()
    print(f"[backward] B={B} n_s={plan.n_s}", flush=True)
    cost, md, fl, tape = plan.eval(Wt, tape=True)
    gc = torch.linspace(0.5, 2.0, B, device="cuda")
    g_tape = plan.backward(Wt, gc, tape)
    g_none = plan.backward(Wt, gc, None)
    torch.cuda.synchronize()
    assert torch.equal(g_tape, g_none)
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    ref = oracle.eval_paths(m, prob.q_start, prob.q_goal, W.astype(np.float64), per_checkpoint=True)
    _, gref = oracle.grad_paths(m, prob.q_start, prob.q_goal, W.astype(np.float64))
    gref = gref * gc.cpu().numpy()[:, None, None]
    ok = ((ref["second"] - ref["d"]) > 1e-5).all(1) & (np.abs(ref["d"] - 0.1) > 1e-5).all(1)
    assert ok.sum() >= B // 2
    g = g_tape.cpu().numpy().astype(np.float64)
    for b in np.where(ok)[0]:
        rel = np.linalg.norm(g[b] - gref[b]) / max(np.linalg.norm(gref[b]), 1e-12)
        assert rel <= 1e-4, (b, rel)


def test_backward_matches_central_differences(cp):
    prob = _diff_problem(K=6, M=8)
    rng = np.random.default_rng(108)
    B = 6
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, B, prob.cost.K, sigma=0.3).astype(np.float64)
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    ref = oracle.eval_paths(m, prob.q_start, prob.q_goal, W, per_checkpoint=True)
    ok = ((ref["second"] - ref["d"]) > 1e-5).all(1) & (np.abs(ref["d"] - 0.1) > 1e-5).all(1)
    assert ok.sum() >= 1
    W = W[ok]
    fd = oracle.fd_grad(m, prob.q_start, prob.q_goal, W, h=1e-6)
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    Wt = torch.from_numpy(W.astype(np.float32)).cuda()
    g = plan.backward(Wt, torch.ones(W.shape[0], device="cuda")).cpu().numpy().astype(np.float64)
    for b in range(W.shape[0]):
        rel = np.linalg.norm(g[b] - fd[b]) / max(np.linalg.norm(fd[b]), 1e-12)
        assert rel <= 1e-4, (b, rel)


def test_backward_c2_size_matches_central_differences(cp):
    """The differentiable workload's gradient check: the adjoint of a
    population W [1024, 16, 6] (c2_diff: 608 checkpoints, smooth hinge 0.1 m,
    512 trees + 16 boxes), computed in one launch of 1024 paths, against FP64
    central differences (h = 1e-6) of the oracle's cost on 32 of its paths
    (the first 32 without a kink: runner-up pair more than 1e-5 m away and
    |d - m| > 1e-5 at every checkpoint), and against the oracle's analytic
    gradient; <= 1e-4 relative (norm per path)."""
    prob = synth.c2_diff()
    B = prob.opt.B
    rng = np.random.default_rng(112)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, B, prob.cost.K, sigma=0.2)
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    Wt = torch.from_numpy(W).cuda()
    print(f"[backward c2] B={B} n_s={plan.n_s}", flush=True)
    cost, md, fl, tape = plan.eval(Wt, tape=True)
    g = plan.backward(Wt, torch.ones(B, device="cuda"), tape).cpu().numpy().astype(np.float64)
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    Wd = W.astype(np.float64)
    pick = []
    for b0 in range(0, B, 64):
        ref = oracle.eval_paths(m, prob.q_start, prob.q_goal, Wd[b0:b0 + 64], per_checkpoint=True)
        ok = ((ref["second"] - ref["d"]) > 1e-5).all(1) & (np.abs(ref["d"] - 0.1) > 1e-5).all(1)
        pick += (b0 + np.where(ok)[0]).tolist()
        if len(pick) >= 32:
            break
    idx = np.array(pick[:32])
    assert idx.size == 32
    print("[backward c2] FP64 central differences on 32 paths", flush=True)
    fd = oracle.fd_grad(m, prob.q_start, prob.q_goal, Wd[idx], h=1e-6)
    _, gref = oracle.grad_paths(m, prob.q_start, prob.q_goal, Wd[idx])
    worst = 0.0
    for r, b in enumerate(idx):
        rel_fd = np.linalg.norm(g[b] - fd[r]) / max(np.linalg.norm(fd[r]), 1e-12)
        rel_an = np.linalg.norm(g[b] - gref[r]) / max(np.linalg.norm(gref[r]), 1e-12)
        worst = max(worst, rel_fd, rel_an)
        assert rel_fd <= 1e-4 and rel_an <= 1e-4, (b, rel_fd, rel_an)
    print(f"[backward c2] largest relative gradient error {worst:.2e}", flush=True)


def test_backward_grid_scene_parity(cp):
    """The adjoint through the trilinear signed-distance lookup (c4_sdf: the
    grid the device builds from 1 M lidar points; the oracle differentiates on
    its own grid, built from the same points): against the oracle's analytic
    gradient and FP64 central differences on paths without a kink (runner-up
    sphere more than 1e-5 m away, |d - m| > 1e-5, and the minimising sphere's
    centre more than 1e-3 voxel from a cell face of the interpolation at
    every checkpoint inside the hinge)."""
    import dataclasses
    base = synth.c4_sdf()
    spec = base.sdf
    prob = dataclasses.replace(base, cost=dataclasses.replace(base.cost, M=8))
    sdf = cp.sdf_build(torch.from_numpy(prob.lidar).cuda(), spec)
    phi_ref, _, _, _ = oracle.sdf_build(prob.lidar, spec)
    m = oracle.Model(prob.robot, prob.scene, prob.cost, sdf=phi_ref, sdf_spec=spec)
    rng = np.random.default_rng(113)
    B = 48
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, B, prob.cost.K, sigma=0.3)
    Wd = W.astype(np.float64)
    ref = oracle.eval_paths(m, prob.q_start, prob.q_goal, Wd, per_checkpoint=True)
    margin = float(np.float32(prob.cost.margin))
    ok = ((ref["second"] - ref["d"]) > 1e-5).all(1) & (np.abs(ref["d"] - margin) > 1e-5).all(1)
    # the cell faces: minimising sphere centre of every checkpoint inside the hinge
    org = np.array(spec.origin, np.float64)
    for b in np.where(ok)[0]:
        pts = oracle.path_points(m, prob.q_start, prob.q_goal, Wd[b])
        for k in np.where(ref["d"][b] < margin)[0]:
            _, cen, _ = oracle.fk(m, pts[k + 1])
            gpos = (cen[ref["tape"][b, k] >> 16] - org) / spec.voxel - 0.5
            if np.min(np.abs(gpos - np.round(gpos))) < 1e-3:
                ok[b] = False
                break
    assert ok.sum() >= 8, ok.sum()
    active = (ref["d"] < margin).sum(1)
    assert active[ok].max() > 0  # the grid term takes part
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B, sdf=sdf, sdf_spec=spec)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    Wt = torch.from_numpy(W).cuda()
    print(f"[backward grid] B={B} n_s={plan.n_s}, {int(ok.sum())} paths without a kink", flush=True)
    cost, md, fl, tape = plan.eval(Wt, tape=True)
    g_tape = plan.backward(Wt, torch.ones(B, device="cuda"), tape)
    g_none = plan.backward(Wt, torch.ones(B, device="cuda"), None)
    assert torch.equal(g_tape, g_none)
    g = g_tape.cpu().numpy().astype(np.float64)
    idx = np.where(ok)[0][:8]
    _, gref = oracle.grad_paths(m, prob.q_start, prob.q_goal, Wd[idx])
    fd = oracle.fd_grad(m, prob.q_start, prob.q_goal, Wd[idx], h=1e-6)
    for r, b in enumerate(idx):
        rel_an = np.linalg.norm(g[b] - gref[r]) / max(np.linalg.norm(gref[r]), 1e-12)
        rel_fd = np.linalg.norm(g[b] - fd[r]) / max(np.linalg.norm(fd[r]), 1e-12)
        assert rel_an <= 1e-4 and rel_fd <= 1e-4, (b, rel_an, rel_fd)


def test_population_gradient_after_a_step(cp):
    """An optimizer that records the argmin tape steps exactly as one that
    does not, and its population gradient is the adjoint of the evaluated
    population (bitwise the plan's backward with the evaluation's tape, and
    the oracle's analytic gradient on paths without a kink)."""
    import dataclasses
    prob = dataclasses.replace(_diff_problem(K=8, M=8),
                               opt=synth.OptParams(B=512, nu=25, sigma0=0.3, eps=1e-6, seed=19, T=1))
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=prob.opt.B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    a = cp.Optimizer(plan, prob.opt)
    b = cp.Optimizer(plan, prob.opt)
    b.record_tape(True)
    a.step(2)
    b.step(2)
    sa, sb = a.get_state(), b.get_state()
    np.testing.assert_array_equal(sa["mu"], sb["mu"])
    np.testing.assert_array_equal(sa["C"], sb["C"])
    g = b.population_grad()
    W, cost, _ = b.last()
    _, _, _, tape = plan.eval(W, tape=True)
    ones = torch.ones(prob.opt.B, device="cuda")
    assert torch.equal(g, plan.backward(W, ones, tape))
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    Wd = W[:48].cpu().numpy().astype(np.float64)
    ref = oracle.eval_paths(m, prob.q_start, prob.q_goal, Wd, per_checkpoint=True)
    ok = ((ref["second"] - ref["d"]) > 1e-5).all(1) & (np.abs(ref["d"] - 0.1) > 1e-5).all(1)
    assert ok.sum() >= 8
    _, gref = oracle.grad_paths(m, prob.q_start, prob.q_goal, Wd[ok])
    gg = g[:48].cpu().numpy().astype(np.float64)[ok]
    for r in range(gg.shape[0]):
        assert np.linalg.norm(gg[r] - gref[r]) <= 1e-4 * max(np.linalg.norm(gref[r]), 1e-12)
    c = cp.Optimizer(plan, prob.opt)
    with pytest.raises(cp.CranePlanError) as ei:
        c.population_grad()
    assert ei.value.code == -5


def test_autograd_function(cp):
    prob = _diff_problem(K=8, M=8)
    rng = np.random.default_rng(109)
    W = torch.from_numpy(synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 16, 8, sigma=0.3)).cuda()
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=16)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    Wv = W.clone().requires_grad_(True)
    cost, _, _ = cp.EvalPaths.apply(Wv, plan)
    (cost * torch.arange(16, device="cuda", dtype=torch.float32)).sum().backward()
    _, _, _, tape = plan.eval(W, tape=True)
    g = plan.backward(W, torch.arange(16, device="cuda", dtype=torch.float32), tape)
    assert torch.equal(Wv.grad, g)


# ----------------------------------------------------------------------------
# selection and optimizer
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("B,nu", [(1, 1), (256, 25), (1000, 999), (1024, 1024), (1024, 100), (1025, 100),
                                  (16384, 819), (16385, 4096), (32768, 1), (32769, 1638), (65536, 3276),
                                  (65535, 4096), (65537, 3276), (100000, 2000), (5000, 4096)])
def test_select_parity(cp, B, nu):
    rng = np.random.default_rng(110 + B)
    cost = np.round(rng.normal(size=B) * 3, 2).astype(np.float32)  # many ties
    cost[rng.choice(B, size=max(0, B // 50), replace=False)] = np.nan
    if B > 4:
        cost[:3] = [np.inf, -np.inf, 0.0]
    got = cp.select(torch.from_numpy(cost).cuda(), nu).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.select(cost.astype(np.float64), nu))


@pytest.mark.parametrize("B", [300, 3000, 20000, 65536, 70000])
def test_select_nonfinite_and_ties(cp, B):
    """Ranks that reach the non-finite costs: NaN ranks as +inf, so NaNs and
    +infs interleave by index; -0 equals +0; all-equal and one-value-heavy
    populations exercise the equal-key rule at the threshold."""
    rng = np.random.default_rng(7 + B)
    nu = min(B, 4096)
    cost = rng.uniform(1.0, 2.0, size=B).astype(np.float32)
    nonfin = rng.choice(B, size=B - nu // 2, replace=False)
    cost[nonfin] = np.nan
    cost[nonfin[rng.random(nonfin.size) < 0.3]] = np.inf
    cost[rng.choice(B, size=min(B, 40), replace=False)] = -0.0
    cost[rng.choice(B, size=min(B, 40), replace=False)] = 0.0
    cases = [cost,
             np.full(B, 3.5, np.float32),
             np.where(rng.random(B) < 0.9, np.float32(20.0), rng.uniform(19.0, 21.0, B)).astype(np.float32),
             # the same leading bytes everywhere: 20 + multiples of 2^-19
             (20.0 + rng.integers(0, 64, B) * 2.0 ** -19).astype(np.float32)]
    for c in cases:
        got = cp.select(torch.from_numpy(c).cuda(), nu).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.select(c.astype(np.float64), nu))


def _elite_compare(e_gpu, cost_ref, nu, tol):
    """Elite sets equal where the gap at the boundary is clear; ranks equal
    where adjacent gaps are clear."""
    order = oracle.select(cost_ref, len(cost_ref))
    srt = cost_ref[order]
    gaps = np.diff(srt)
    tt = np.maximum(tol[order][:-1], tol[order][1:]) * 2
    if nu < len(srt) and gaps[nu - 1] > tt[nu - 1]:
        assert set(e_gpu.tolist()) == set(order[:nu].tolist())
    for r in range(nu):
        left = r == 0 or gaps[r - 1] > tt[r - 1]
        right = r == len(srt) - 1 or gaps[r] > tt[r]
        if left and right:
            assert e_gpu[r] == order[r], r


def test_optimizer_one_step_parity(cp):
    prob = synth.c0_plain()
    orc = oracle.Optimizer(prob)
    for _ in range(2):
        orc.step()
    mu0, C0, t0 = orc.mu.copy(), orc.C.copy(), orc.t
    step = orc.step()
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=prob.opt.B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    opt = cp.Optimizer(plan, prob.opt)
    opt.set_state(mu0, C0, t0)
    print(f"[optimizer one step] c0_plain t={t0}", flush=True)
    opt.step(1)
    W, cost, elite = opt.last()
    st = opt.get_state()
    W = W.cpu().numpy()
    Wref = oracle.expand(prob.robot, step["xi"], prob.cost.K)
    np.testing.assert_allclose(W, Wref, rtol=0, atol=2e-6 * np.maximum(1, np.abs(Wref)).max())
    # the oracle evaluates its own samples, stored in FP32 as the device stores its own
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    Wq = Wref.astype(np.float32).astype(np.float64)
    ref = oracle.eval_paths(m, prob.q_start, prob.q_goal, Wq, per_checkpoint=True)
    tol, _ = _cost_tol(ref, prob.cost, prob.robot.n_joints)
    c = cost.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(c - ref["cost"]) <= tol)
    e = elite.cpu().numpy()
    _elite_compare(e, step["cost"], prob.opt.nu, tol + 1e-5 * np.abs(step["cost"]))
    assert st["t"] == t0 + 1
    if np.array_equal(e, step["elite"]):
        np.testing.assert_allclose(st["mu"], step["mu"], rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(st["C"], step["C"], rtol=1e-4, atol=1e-8)
    # whatever the device selected: its update from the oracle's elites
    # (indices into the same population) equals the oracle's update
    opt.debug_update(torch.from_numpy(step["elite"].astype(np.int32)))
    st2 = opt.get_state()
    np.testing.assert_allclose(st2["mu"], step["mu"], rtol=0, atol=1e-10)
    np.testing.assert_allclose(st2["C"], step["C"], rtol=0, atol=1e-11 * np.abs(step["C"]).max())


def _check_first_iterations(cp, prob, label):
    """From creation: the state at t = 0 is the oracle's initial state, and
    the first iteration (samples, costs, elites, mean and covariance) is the
    oracle's first step."""
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=prob.opt.B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    opt = cp.Optimizer(plan, prob.opt)
    st0 = opt.get_state()
    orc = oracle.Optimizer(prob)
    assert st0["t"] == 0 and st0["best_cost"] == math.inf
    np.testing.assert_allclose(st0["mu"], orc.mu, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(st0["C"], orc.C)
    print(f"[first iteration] {label} B={prob.opt.B} nu={prob.opt.nu}", flush=True)
    opt.step(1)
    W, cost, elite = opt.last()
    step = orc.step()
    Wref = oracle.expand(prob.robot, step["xi"], prob.cost.K)
    W = W.cpu().numpy()
    np.testing.assert_allclose(W, Wref, rtol=0, atol=2e-6 * np.maximum(1, np.abs(Wref)).max())
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    ref = oracle.eval_paths(m, prob.q_start, prob.q_goal, Wref.astype(np.float32).astype(np.float64),
                            per_checkpoint=True)
    tol, _ = _cost_tol(ref, prob.cost, prob.robot.n_joints)
    c = cost.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(c - ref["cost"]) <= tol)
    e = elite.cpu().numpy()
    _elite_compare(e, ref["cost"], prob.opt.nu, tol)
    # the selection inside the step is the plain selection of the step's costs
    np.testing.assert_array_equal(e, cp.select(cost, prob.opt.nu).cpu().numpy())
    opt.debug_update(torch.from_numpy(step["elite"].astype(np.int32)))
    st = opt.get_state()
    np.testing.assert_allclose(st["mu"], step["mu"], rtol=0, atol=1e-10)
    np.testing.assert_allclose(st["C"], step["C"], rtol=0, atol=1e-11 * np.abs(step["C"]).max())


def test_initial_state_and_first_iteration_c0(cp):
    _check_first_iterations(cp, synth.c0_plain(), "c0_plain")


@pytest.mark.parametrize("B,nu", [(1024, 64), (800, 80), (769, 38), (1000, 600)])
def test_first_iteration_selection_paths(cp, B, nu):
    """Populations of 769-1024 paths with nu <= B/2 take the radix selection
    inside the fused per-path sums + selection launch; the others the rank
    count.  c0_plain crane and scene."""
    import dataclasses
    base = synth.c0_plain()
    prob = dataclasses.replace(base, opt=synth.OptParams(B=B, nu=nu, sigma0=0.2, eps=1e-6, seed=40 + B, T=1))
    _check_first_iterations(cp, prob, f"B={B} nu={nu}")


@pytest.mark.parametrize("K", [24, 16, 9, 8, 5])
@pytest.mark.parametrize("kind", ["spd", "zero_variance"])
def test_sampling_parity_dims(cp, kind, K):
    """Step (1) from a given mean and covariance at several dimensions
    D = 4K (c1_full's crane, 4 sampled joints): 96, the largest the library
    takes (the largest batched problems), 64 (c1), 36, 32 (c0) and 20 (the
    factorisation runs in shared memory above 64, in one wave's registers up
    to 32 and up to 64).  The device Cholesky factor and the samples it draws
    equal the oracle's.  'zero_variance' gives one sampled joint of one
    waypoint no variance, so the first factorisation meets a zero pivot and
    the jittered retry C + 10 eps I is the one used."""
    import dataclasses
    base = synth.c1_full()
    prob = dataclasses.replace(base, cost=dataclasses.replace(base.cost, K=K),
                               opt=synth.OptParams(B=256, nu=25, sigma0=0.2, eps=1e-6, seed=21, T=1))
    D = prob.cost.K * prob.robot.n_active
    assert D == 4 * K
    rng = np.random.default_rng(33)
    X = rng.normal(size=(D, 2 * D)) * 0.05
    C = X @ X.T / (2 * D) + 1e-4 * np.eye(D)
    if kind == "zero_variance":
        z = (37 * D) // 96
        C[z, :] = 0.0
        C[:, z] = 0.0
    mu = oracle.initial_mean(prob.robot, prob.q_start, prob.q_goal, prob.cost.K) + rng.normal(size=D) * 0.01
    orc = oracle.Optimizer(prob)
    orc.set_state(mu, C, 4)
    Wref = oracle.expand(prob.robot, orc.sample(), prob.cost.K)
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=prob.opt.B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    opt = cp.Optimizer(plan, prob.opt)
    print(f"[sampling] D={D} kind={kind}", flush=True)
    opt.set_state(mu, C, 4)
    opt.step(1)
    W = opt.last()[0].cpu().numpy()
    np.testing.assert_allclose(W, Wref, rtol=0, atol=2e-6 * np.maximum(1, np.abs(Wref)).max())


@pytest.mark.parametrize("K,B,nu", [(16, 4096, 819), (24, 2048, 1000), (5, 512, 7)])
def test_update_parity_many_elites(cp, K, B, nu):
    """Steps (4)-(6) with many elites (each entry of C is a sum over nu elites,
    taken on the device as 16 interleaved partial sums): from a given state the
    device draws its samples, then updates from elite indices the test picks
    (any nu distinct paths, in a given rank order); the new mean and covariance
    equal the oracle's update of its own samples of that state with the same
    indices."""
    import dataclasses
    base = synth.c1_full()
    prob = dataclasses.replace(base, cost=dataclasses.replace(base.cost, K=K, M=8),
                               opt=synth.OptParams(B=B, nu=nu, sigma0=0.2, eps=1e-6, seed=31, T=1))
    D = K * prob.robot.n_active
    rng = np.random.default_rng(34)
    X = rng.normal(size=(D, 2 * D)) * 0.05
    C = X @ X.T / (2 * D) + 1e-3 * np.eye(D)
    mu = oracle.initial_mean(prob.robot, prob.q_start, prob.q_goal, K) + rng.normal(size=D) * 0.01
    elite = rng.permutation(B)[:nu]
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    opt = cp.Optimizer(plan, prob.opt)
    print(f"[update parity] D={D} B={B} nu={nu}", flush=True)
    opt.set_state(mu, C, 2)
    opt.step(1)
    opt.debug_update(torch.from_numpy(elite.astype(np.int32)))
    st = opt.get_state()
    orc = oracle.Optimizer(prob)
    orc.set_state(mu, C, 2)
    xi = orc.sample()
    mu_ref, C_ref = oracle.update(xi[elite], oracle.log_rank_weights(nu), prob.opt.eps)
    np.testing.assert_allclose(st["mu"], mu_ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(st["C"], C_ref, rtol=0, atol=1e-13 * np.abs(C_ref).max() + 1e-15)
    bad = elite.copy()
    bad[-1] = B  # out of range: refused before any device work
    with pytest.raises(cp.CranePlanError):
        opt.debug_update(torch.from_numpy(bad.astype(np.int32)))


def test_plan_destroyed_before_its_optimizer(cp):
    """cp_plan_destroy before cp_optimizer_destroy (the order a garbage
    collector may pick for a plan and an optimizer in one reference cycle):
    the optimizer keeps its plan alive and still steps, and destroying it
    afterwards leaves no HIP error behind for the next caller."""
    import ctypes
    prob = synth.c0_plain()
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=prob.opt.B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    opt = cp.Optimizer(plan, prob.opt)
    opt.step(1)
    plan.close()
    opt.step(2)
    torch.cuda.synchronize()
    assert np.isfinite(opt.get_state()["best_cost"])
    opt.close()
    hip = ctypes.CDLL("libamdhip64.so")
    assert hip.hipPeekAtLastError() == 0
    assert torch.ones(4, device="cuda").sum().item() == 4.0


def test_optimizer_runs_and_is_deterministic(cp):
    prob = synth.c0_plain()
    out = []
    for _ in range(2):
        plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=prob.opt.B)
        plan.set_endpoints(prob.q_start, prob.q_goal)
        opt = cp.Optimizer(plan, prob.opt)
        best = []
        for _ in range(prob.opt.T):
            opt.step(1)
            best.append(opt.get_state()["best_cost"])
        out.append((opt.get_state(), best))
    (s1, b1), (s2, b2) = out
    assert b1 == b2
    np.testing.assert_array_equal(s1["mu"], s2["mu"])
    np.testing.assert_array_equal(s1["C"], s2["C"])
    assert all(y <= x for x, y in zip(b1, b1[1:]))
    assert b1[-1] < b1[0]
    assert s1["t"] == prob.opt.T
    # the last selection, alone and with the population; a plan has nothing to tune
    elite, cost = opt.last_elites()
    _, cost_all, elite_all = opt.last()
    assert torch.equal(elite, elite_all) and torch.equal(cost, cost_all)
    cp.tune(plan=plan)


def test_optimizer_resume_reproduces(cp):
    prob = synth.c0_plain()
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=prob.opt.B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    a = cp.Optimizer(plan, prob.opt)
    a.step(3)
    mid = a.get_state()
    a.step(2)
    end_a = a.get_state()
    b = cp.Optimizer(plan, prob.opt)
    b.set_state(mid["mu"], mid["C"], mid["t"])
    b.step(2)
    end_b = b.get_state()
    np.testing.assert_array_equal(end_a["mu"], end_b["mu"])
    np.testing.assert_array_equal(end_a["C"], end_b["C"])


def test_optimizer_not_positive_definite(cp):
    prob = synth.c0_plain()
    opt_p = synth.OptParams(B=64, nu=1, sigma0=0.2, eps=0.0, seed=5, T=1)
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=64)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    opt = cp.Optimizer(plan, opt_p)
    opt.step(1)
    with pytest.raises(cp.CranePlanError) as ei:
        opt.get_state()
    assert ei.value.code == -4


# the polish parity test: a path is compared only if at every iterate of the
# oracle's polish each checkpoint within the hinge (d < margin + 1e-3 m) has
# its runner-up pair more than POLISH_GAP away (no argmin switch, R20)
POLISH_GAP = 1e-4
# polished waypoints: FP32 steps against FP64 steps, 10 clipped steps of
# length eta g_max = 1e-2 (see the test's docstring)
POLISH_WTOL = 1e-4


def _kink_gap(m, prob, iterates, margin):
    gap = np.full(iterates[0].shape[0], np.inf)
    for x in iterates:
        r = oracle.eval_paths(m, prob.q_start, prob.q_goal, oracle.expand(prob.robot, x, prob.cost.K),
                              per_checkpoint=True)
        act = r["d"] < margin + 1e-3
        gap = np.minimum(gap, np.where(act, r["second"] - r["d"], np.inf).min(1))
    return gap


def test_polish_parity_c2_scene(cp):
    """Gradient polish (the differentiable workload's setting: 64 elites x 10
    steps W <- W - eta g / max(1, |g| / g_max), eta = 1e-3, g_max = 10) on the
    c2_diff crane and scene (512 trees + 16 boxes, smooth hinge, margin 0.1 m,
    K = 16), with M = 4 points per span: the scene is so cluttered that a
    path meets about one checkpoint inside the hinge per span, and fewer
    checkpoints keep more paths clear of argmin switches (and the oracle
    fast).

    The device draws its population from a given state; the elites are chosen
    by the test, from the oracle alone: among the oracle's own samples of that
    state (stored in FP32, as the device stores its own), the oracle polishes
    every one and keeps those whose polish meets no argmin switch inside the
    hinge (POLISH_GAP), then takes 64 whose polished costs are far apart, so
    the re-ranking has one right answer.  The device polishes the same
    indices of its own population (cp_debug_update); polished waypoints,
    their costs, the re-ranked order, mu and C must match the oracle's.

    Tolerances: each step moves W by eta g_max = 1e-2 along -g/|g|.  The
    device's direction carries the adjoint's error (<= 1e-4 relative; 2.5e-5
    at most, 7e-6 typically, on these paths) and W is stored in FP32 (6e-8
    per step near 1 rad): after one step the device and the oracle differ by
    at most 1.7e-7 (measured).  The collision term's curvature feeds a W error
    back into the next step's direction, so the difference grows over the 10
    steps (measured: at most 8e-7 after 2 steps, 3e-6 after 5, 5.6e-6 to
    3.2e-5 after 10 depending on the elites); POLISH_WTOL = 1e-4 bounds it
    with a factor of 3 over the largest seen.  Polished costs: the
    evaluation tolerance plus |g| POLISH_WTOL.  mu: POLISH_WTOL; C:
    2 max|x - mu| POLISH_WTOL + POLISH_WTOL^2."""
    import dataclasses
    base = synth.c2_diff()
    B, nu, steps = 384, 64, 10
    prob = dataclasses.replace(base, cost=dataclasses.replace(base.cost, M=4),
                               opt=synth.OptParams(B=B, nu=nu, sigma0=0.2, eps=1e-6, seed=71, T=1,
                                                   polish_elites=nu, polish_steps=steps, polish_eta=1e-3,
                                                   polish_clip=10.0))
    margin = float(np.float32(prob.cost.margin))
    orc = oracle.Optimizer(prob)
    mu0, C0 = orc.mu.copy(), orc.C.copy()
    xq = orc.sample().astype(np.float32).astype(np.float64)
    print(f"[polish parity] oracle polish of {B} samples x {steps} steps", flush=True)
    trace = []
    xp = orc.polish(xq, trace=trace)
    m = orc.model
    gap = _kink_gap(m, prob, trace + [xp], margin)
    ref_p = oracle.eval_paths(m, prob.q_start, prob.q_goal, oracle.expand(prob.robot, xp, prob.cost.K),
                              per_checkpoint=True)
    _, g_p = oracle.grad_paths(m, prob.q_start, prob.q_goal, oracle.expand(prob.robot, xp, prob.cost.K))
    tol_p = _cost_tol(ref_p, prob.cost, prob.robot.n_joints)[0] + np.linalg.norm(g_p.reshape(B, -1), axis=1) * POLISH_WTOL
    cand = np.where(gap > POLISH_GAP)[0]
    print(f"[polish parity] {cand.size} of {B} samples without an argmin switch", flush=True)
    chosen = []
    for i in cand[np.argsort(ref_p["cost"][cand], kind="stable")]:
        if not chosen or ref_p["cost"][i] - ref_p["cost"][chosen[-1]] > 2 * (tol_p[i] + tol_p[chosen[-1]]):
            chosen.append(int(i))
    assert len(chosen) >= nu, len(chosen)
    # rank order before polish: the test's choice (here: by index)
    elite = np.sort(np.array(chosen[:nu]))
    # the oracle's step after selection
    xe = xp[elite]
    ce = ref_p["cost"][elite]
    order = oracle.select(ce, nu)
    mu_ref, C_ref = oracle.update(xe[order], orc.w, prob.opt.eps)

    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    opt = cp.Optimizer(plan, prob.opt)
    opt.set_state(mu0, C0, 0)
    opt.step(1)
    print("[polish parity] device polish of the chosen elites", flush=True)
    opt.debug_update(torch.from_numpy(elite.astype(np.int32)))
    Wp, cost_p = opt.last_polished()
    _, _, e_dev = opt.last()
    st = opt.get_state()
    Wp = Wp.cpu().numpy().astype(np.float64)
    Wref = oracle.expand(prob.robot, xe, prob.cost.K)
    err_w = np.abs(Wp - Wref).max()
    print(f"[polish parity] max |W_dev - W_oracle| = {err_w:.3e}", flush=True)
    assert err_w <= POLISH_WTOL
    c = cost_p.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(c - ce) <= tol_p[elite]), np.max(np.abs(c - ce) / tol_p[elite])
    # re-ranked order: polished slot i is index B + i
    np.testing.assert_array_equal(e_dev.cpu().numpy(), B + order)
    np.testing.assert_allclose(st["mu"], mu_ref, rtol=0, atol=POLISH_WTOL)
    dev = np.abs(xe - mu_ref[None]).max()
    np.testing.assert_allclose(st["C"], C_ref, rtol=0, atol=2 * dev * POLISH_WTOL + POLISH_WTOL ** 2)
    # a whole step with polish from the same state: best-so-far is the better of
    # the best sample and the best polished elite
    opt2 = cp.Optimizer(plan, prob.opt)
    opt2.set_state(mu0, C0, 0)
    opt2.step(1)
    _, cost_all, _ = opt2.last()
    _, cp2 = opt2.last_polished()
    best = min(float(cost_all.min().cpu()), float(cp2.min().cpu()))
    assert opt2.get_state()["best_cost"] == best


# ----------------------------------------------------------------------------
# signed-distance grid
# ----------------------------------------------------------------------------

def test_sdf_build_and_query_parity(cp):
    spec = synth.SdfSpec(dims=(64, 48, 32), origin=(-3.2, -2.4, -0.4), voxel=0.1)
    rng = np.random.default_rng(111)
    trees = np.array([[-1.0, 0.5, 0.3, 0, 3], [1.2, -0.8, 0.2, 0, 3], [0.3, 1.5, 0.45, 0, 3]], np.float32)
    pts = synth.make_lidar(rng, trees, 60000, spec, z_top=2.8)
    pts = np.concatenate([pts, np.array([[-10.0, 0, 0], [0, 0, 50.0]], np.float32)])  # outside the grid
    print("[sdf] 64x48x32", flush=True)
    sdf, occ, eo, ef = cp.sdf_build(torch.from_numpy(pts).cuda(), spec, with_edt=True)
    torch.cuda.synchronize()
    phi_ref, occ_ref, eo_ref, ef_ref = oracle.sdf_build(pts, spec)
    np.testing.assert_array_equal(occ.cpu().numpy(), occ_ref)
    np.testing.assert_array_equal(eo.cpu().numpy(), eo_ref)
    np.testing.assert_array_equal(ef.cpu().numpy(), ef_ref)
    np.testing.assert_allclose(sdf.cpu().numpy(), phi_ref, rtol=2e-7, atol=1e-7)
    # queries through a plan that uses the grid
    prob = synth.c0_plain()
    scene = synth.Scene(cyl=np.zeros((0, 5), np.float32), box=np.zeros((0, 6), np.float32), has_ground=0)
    plan = cp.Plan(prob.robot, scene, prob.cost, max_B=1, sdf=sdf, sdf_spec=spec)
    Q = synth.random_configs(rng, prob.robot, 512)
    d, a = plan.debug_configs(torch.from_numpy(Q).cuda())
    m = oracle.Model(prob.robot, scene, prob.cost, sdf=phi_ref, sdf_spec=spec)
    dr, sr, orr, sec = oracle.eval_configs(m, Q.astype(np.float64))
    assert np.all(np.abs(d.cpu().numpy() - dr) <= 1e-4)
    assert np.all((a.cpu().numpy().view(np.uint32) & 0xFFFF) == 0xFFFF)


@pytest.mark.parametrize("dims,n_pts", [((4096, 2, 3), 40), ((3, 1500, 4), 30), ((5, 6, 1100), 25),
                                        ((9, 8, 7), 0), ((4, 4, 4), 4000), ((33, 17, 65), 300)])
def test_sdf_build_shapes(cp, dims, n_pts):
    """Distance transforms on grids of uneven shape: one axis up to the
    4096 limit (the envelope passes' shared-memory stack then holds fewer
    lines per block), no occupied voxel (every squared distance is the
    'none' value nx^2 + ny^2 + nz^2), every voxel occupied; occupancy and both
    squared EDTs bit-exact against the oracle's plain line minima."""
    spec = synth.SdfSpec(dims=dims, origin=(-1.0, 2.0, 0.5), voxel=0.25)
    rng = np.random.default_rng(sum(dims) + n_pts)
    ext = np.array(dims) * spec.voxel
    pts = (np.array(spec.origin) + rng.uniform(0, 1, size=(n_pts, 3)) * ext).astype(np.float32)
    if n_pts == 4000:  # every voxel of the 4 x 4 x 4 grid
        g = np.stack(np.meshgrid(*[np.arange(4) + 0.5] * 3, indexing="ij"), -1).reshape(-1, 3)
        pts = np.concatenate([pts, (np.array(spec.origin) + g * spec.voxel).astype(np.float32)])
    pts = np.ascontiguousarray(pts.reshape(-1, 3), np.float32)
    print(f"[sdf shapes] dims={dims} points={pts.shape[0]}", flush=True)
    dev = torch.from_numpy(pts).cuda() if pts.shape[0] else torch.zeros((0, 3), device="cuda")
    sdf, occ, eo, ef = cp.sdf_build(dev, spec, with_edt=True)
    torch.cuda.synchronize()
    phi_ref, occ_ref, eo_ref, ef_ref = oracle.sdf_build(pts, spec)
    np.testing.assert_array_equal(occ.cpu().numpy(), occ_ref)
    np.testing.assert_array_equal(eo.cpu().numpy(), eo_ref)
    np.testing.assert_array_equal(ef.cpu().numpy(), ef_ref)
    np.testing.assert_allclose(sdf.cpu().numpy(), phi_ref, rtol=2e-7, atol=1e-7)
    if n_pts == 0:
        assert (eo_ref == sum(d * d for d in dims)).all()
    if n_pts == 4000:
        assert occ_ref.all() and (ef_ref == sum(d * d for d in dims)).all()
