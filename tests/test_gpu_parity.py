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
    sdf = cp.sdf_build(torch.from_numpy(prob.lidar).cuda(), spec)
    rng = np.random.default_rng(107)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, B, prob.cost.K, sigma=0.2)
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B, sdf=sdf, sdf_spec=spec)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    cost, md, fl = plan.eval(torch.from_numpy(W).cuda())
    torch.cuda.synchronize()
    phi_ref, _, _, _ = oracle.sdf_build(prob.lidar, spec)
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
    W = W[ok]
    fd = oracle.fd_grad(m, prob.q_start, prob.q_goal, W, h=1e-6)
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    Wt = torch.from_numpy(W.astype(np.float32)).cuda()
    g = plan.backward(Wt, torch.ones(W.shape[0], device="cuda")).cpu().numpy().astype(np.float64)
    for b in range(W.shape[0]):
        rel = np.linalg.norm(g[b] - fd[b]) / max(np.linalg.norm(fd[b]), 1e-12)
        assert rel <= 1e-4, (b, rel)


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
    if set(e.tolist()) == set(step["elite"].tolist()) and np.array_equal(e, step["elite"]):
        np.testing.assert_allclose(st["mu"], step["mu"], rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(st["C"], step["C"], rtol=1e-4, atol=1e-8)


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


def test_polish_one_step(cp):
    """Gradient polish (c2_diff settings, reduced): the polished elites'
    costs do not exceed their unpolished costs by more than the tolerance and
    the best-so-far improves on the sampled best."""
    base = synth.c2_diff()
    opt_p = synth.OptParams(B=256, nu=16, sigma0=0.2, eps=1e-6, seed=7, T=2, polish_elites=16, polish_steps=10,
                            polish_eta=1e-3, polish_clip=10.0)
    plan = cp.Plan(base.robot, base.scene, base.cost, max_B=256)
    plan.set_endpoints(base.q_start, base.q_goal)
    opt = cp.Optimizer(plan, opt_p)
    opt.step(2)
    st = opt.get_state()
    W, cost, elite = opt.last()
    assert np.isfinite(st["best_cost"])
    assert st["best_cost"] <= float(cost.min().cpu()) + 1e-6


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
