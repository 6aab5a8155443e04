"""Batched problems (one persistent evaluation launch, graph replay,
autotuned launch shape) against the same problems run one at a time."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2503_14160_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_14160_amd import craneplan
    craneplan.lib()
    return craneplan


def _problems(n=6, seed=500):
    """Problems of uneven size: spheres, waypoints, checkpoints, obstacles,
    population and elites all differ."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed + i)
        robot = synth.make_robot(seed + 100 + i, 16 + 4 * i)
        qs, qg = synth.make_endpoints(rng, robot)
        scene = synth.make_scene(rng, robot, qs, qg, n_cyl=8 + 13 * i, n_box=i % 3, half_extent=10.0)
        K = 4 + i
        cost = synth.CostParams(K=K, M=8 if i % 2 else 5)
        B = 64 + 41 * i
        opt = synth.OptParams(B=B, nu=max(1, B // 10), sigma0=0.2, eps=1e-6, seed=seed + 200 + i, T=4)
        out.append(synth.Problem(f"batch[{i}]", robot, scene, qs, qg, cost, opt))
    return out


def _sequential(cp, probs, iters):
    states = []
    for i, p in enumerate(probs):
        plan = cp.Plan(p.robot, p.scene, p.cost, max_B=p.opt.B)
        plan.set_endpoints(p.q_start, p.q_goal)
        opt = cp.Optimizer(plan, p.opt, problem_id=i)
        opt.step(iters)
        states.append(opt.get_state())
    return states


def _same(a, b):
    np.testing.assert_array_equal(a["mu"], b["mu"])
    np.testing.assert_array_equal(a["C"], b["C"])
    assert a["t"] == b["t"]
    assert a["best_cost"] == b["best_cost"]
    np.testing.assert_array_equal(a["best_W"], b["best_W"])


def test_batch_matches_sequential(cp):
    probs = _problems()
    print("[batch] 6 problems, 3 iterations via graph", flush=True)
    batch = cp.Batch(probs)
    batch.run(3)
    torch.cuda.synchronize()
    seq = _sequential(cp, probs, 3)
    for i in range(len(probs)):
        _same(batch.get_state(i), seq[i])


def test_batch_graph_replays_with_eager_work_between(cp):
    probs = _problems(n=4, seed=520)
    batch = cp.Batch(probs)
    print("[batch] replay 2+2 with eager work between", flush=True)
    batch.run(2)
    torch.cuda.synchronize()
    mid = [batch.get_state(i) for i in range(len(probs))]
    x = torch.randn(1 << 20, device="cuda")
    y = (x * 2.0).sum()
    torch.cuda.synchronize()
    batch.run(2)  # same captured graph, replayed
    torch.cuda.synchronize()
    seq2 = _sequential(cp, probs, 2)
    seq4 = _sequential(cp, probs, 4)
    for i in range(len(probs)):
        _same(mid[i], seq2[i])
        _same(batch.get_state(i), seq4[i])
    assert torch.isfinite(y)


def test_batch_result_does_not_depend_on_tuning(cp):
    probs = _problems(n=5, seed=540)
    ref = None
    for rounds, wg in ((1, 2), (8, 8), (3, 5), (2, 0)):
        batch = cp.Batch(probs)
        batch.set_tuning(rounds, wg)
        assert batch.get_tuning() == (rounds, wg)
        print(f"[batch] tuning rounds={rounds} wg_per_cu={wg}", flush=True)
        batch.run(2)
        torch.cuda.synchronize()
        st = [batch.get_state(i) for i in range(len(probs))]
        if ref is None:
            ref = st
        else:
            for a, b in zip(ref, st):
                _same(a, b)


def test_batch_autotune_and_cache(cp, tmp_path):
    probs = _problems(n=4, seed=560)
    cache = str(tmp_path / "tune.txt")
    batch = cp.Batch(probs)
    print("[batch] autotune", flush=True)
    chosen = batch.tune(cache)
    assert chosen[0] >= 1 and chosen[1] >= 0  # 0: one workgroup per work item
    assert batch.get_tuning() == chosen
    lines = open(cache).read().split("\n")
    assert len([l for l in lines if l.strip()]) == 1
    batch2 = cp.Batch(probs)
    assert batch2.tune(cache) == chosen
    assert len([l for l in open(cache).read().split("\n") if l.strip()]) == 1
    batch2.run(1)
    torch.cuda.synchronize()
    seq = _sequential(cp, probs, 1)
    for i in range(len(probs)):
        _same(batch2.get_state(i), seq[i])


EPS_D = 2e-5


def _c3_span():
    """Problems of the batched workload (c3_batch) that span its ranges: the
    least work, the median, the most work (K = 24, so D = 96: the factor runs
    in shared memory), the largest population (8153 paths: radix selection)
    and one of more than 1000 obstacles."""
    probs = synth.c3_batch(256)
    work = np.array([p.opt.B * p.cost.n_s * (p.scene.n_cyl + p.scene.n_box + 1) for p in probs])
    order = np.argsort(work, kind="stable")
    Bs = np.array([p.opt.B for p in probs])
    Os = np.array([p.scene.n_cyl + p.scene.n_box for p in probs])
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1]), int(np.argmax(Bs)),
            int(np.where(Os >= 1000)[0][0])]
    out = []
    for i in pick:
        if i not in out:
            out.append(i)
    return [probs[i] for i in out]


def test_batch_c3_sizes_against_oracle(cp):
    """A batch of problems spanning c3_batch (paths 1158..8153, waypoints
    8..24, obstacles 85..1000+): after one batched iteration from creation
    every problem's state equals its own run through cp_optimizer_step
    (bitwise), its samples are the oracle's, sampled paths' costs match the
    oracle's evaluation of its own samples (stored in FP32), and the problem
    of least work matches the oracle's whole first step (elites, mean,
    covariance)."""
    probs = _c3_span()
    n = len(probs)
    assert max(p.cost.K for p in probs) == 24 and max(p.opt.B for p in probs) > 8000
    assert max(p.scene.n_cyl + p.scene.n_box for p in probs) >= 1000
    print(f"[batch c3] {n} problems, 1 iteration", flush=True)
    batch = cp.Batch(probs)
    batch.run(1)
    torch.cuda.synchronize()
    seq = _sequential(cp, probs, 1)
    for i in range(n):
        _same(batch.get_state(i), seq[i])
    rng = np.random.default_rng(900)
    for i, p in enumerate(probs):
        W, cost, elite = batch.last(i)
        W = W.cpu().numpy()
        orc = oracle.Optimizer(p, problem_id=i)
        xi = orc.sample()
        Wref = oracle.expand(p.robot, xi, p.cost.K)
        np.testing.assert_allclose(W, Wref, rtol=0, atol=2e-6 * np.maximum(1, np.abs(Wref)).max())
        idx = np.sort(rng.choice(p.opt.B, size=16, replace=False))
        idx[0], idx[-1] = 0, p.opt.B - 1
        m = oracle.Model(p.robot, p.scene, p.cost)
        print(f"[batch c3] problem {i}: B={p.opt.B} K={p.cost.K} obstacles={p.scene.n_cyl + p.scene.n_box}",
              flush=True)
        ref = oracle.eval_paths(m, p.q_start, p.q_goal, Wref[idx].astype(np.float32).astype(np.float64),
                                per_checkpoint=True)
        act = (ref["d"] < float(np.float32(p.cost.margin)) + EPS_D).sum(1)
        tol = 1e-5 * np.abs(ref["cost"]) + p.cost.w_c * p.cost.lambda_c * EPS_D * act + 1e-6 \
            + 2 * p.cost.w_l * 1e-6 * np.sqrt(p.cost.n_s * p.robot.n_joints * ref["parts"][:, 2])
        c = cost.cpu().numpy()[idx].astype(np.float64)
        assert np.all(np.abs(c - ref["cost"]) <= tol), (i, np.max(np.abs(c - ref["cost"]) / tol))
    # the problem of least work: the oracle's whole first step
    i = 0
    p = probs[i]
    orc = oracle.Optimizer(p, problem_id=i)
    step = orc.step()
    m = oracle.Model(p.robot, p.scene, p.cost)
    Wq = oracle.expand(p.robot, step["xi"], p.cost.K).astype(np.float32).astype(np.float64)
    ref = oracle.eval_paths(m, p.q_start, p.q_goal, Wq, per_checkpoint=True)
    act = (ref["d"] < float(np.float32(p.cost.margin)) + EPS_D).sum(1)
    tol = 1e-5 * np.abs(ref["cost"]) + p.cost.w_c * p.cost.lambda_c * EPS_D * act + 1e-6 \
        + 2 * p.cost.w_l * 1e-6 * np.sqrt(p.cost.n_s * p.robot.n_joints * ref["parts"][:, 2])
    # elites: the set where the boundary gap is clear, each rank where both
    # adjacent gaps are clear (a gap is clear above twice the two costs'
    # tolerances)
    srt = oracle.select(ref["cost"], p.opt.B)
    gaps = np.diff(ref["cost"][srt])
    clear = gaps > 2 * (tol[srt][:-1] + tol[srt][1:])
    nu = p.opt.nu
    assert clear[nu - 1]
    _, cost, elite = batch.last(i)
    e = elite.cpu().numpy()
    assert set(e.tolist()) == set(srt[:nu].tolist())
    ranks_ok = np.array([(r == 0 or clear[r - 1]) and clear[r] for r in range(nu)])
    assert ranks_ok.sum() >= nu // 2
    np.testing.assert_array_equal(e[ranks_ok], srt[:nu][ranks_ok])
    # the update at this size from the oracle's elites (the batch equals the
    # problem run alone, bitwise, as checked above)
    plan = cp.Plan(p.robot, p.scene, p.cost, max_B=p.opt.B)
    plan.set_endpoints(p.q_start, p.q_goal)
    opt = cp.Optimizer(plan, p.opt, problem_id=i)
    opt.step(1)
    opt.debug_update(torch.from_numpy(step["elite"].astype(np.int32)))
    st = opt.get_state()
    np.testing.assert_allclose(st["mu"], step["mu"], rtol=0, atol=1e-10)
    np.testing.assert_allclose(st["C"], step["C"], rtol=0, atol=1e-11 * np.abs(step["C"]).max())
