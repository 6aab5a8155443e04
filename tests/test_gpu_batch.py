"""Batched problems (one persistent evaluation launch, graph replay,
autotuned launch shape) against the same problems run one at a time."""
import os

import numpy as np
import pytest
import torch

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
