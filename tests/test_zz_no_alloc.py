"""The allocation-free evaluation entry point (cp_eval_paths_noalloc) through
the C ABI against cp_eval_paths: bitwise equal costs, minimum distances,
flags and argmin tapes, on two calls in a row (the second with fewer paths,
so it runs on scratch the first call left filled), and the size limit."""
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


def _outputs(B, ns):
    return (torch.empty(B, device="cuda"), torch.empty(B, device="cuda"),
            torch.empty(B, dtype=torch.uint8, device="cuda"), torch.empty((B, ns), dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("workload", ["c1_full", "c0_plain"])
def test_noalloc_eval_matches_eval(cp, workload):
    prob = synth.WORKLOADS[workload]()
    B0 = 8192 if workload == "c1_full" else 256
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B0)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    rng = np.random.default_rng(77)
    for B in (B0, B0 // 3 + 1):
        print(f"[noalloc] {workload} B={B}", flush=True)
        W = torch.from_numpy(synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, B, prob.cost.K,
                                                    sigma=0.3)).cuda()
        ref = _outputs(B, plan.n_s)
        got = _outputs(B, plan.n_s)
        plan.eval_into(W, *ref)
        plan.eval_noalloc_into(W, *got)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b)
        assert torch.isfinite(got[0]).all()


def test_noalloc_eval_rejects_sizes_beyond_its_scratch(cp):
    base = synth.c0_plain()
    cost = synth.CostParams(K=1, M=1, interp=synth.INTERP_LINEAR)  # n_s = 2: 34 partial slots per wave
    B = 1 << 21
    plan = cp.Plan(base.robot, base.scene, cost, max_B=B)
    W = torch.zeros((B, 1, base.robot.n_joints), device="cuda")
    cost_t, md = torch.empty(B, device="cuda"), torch.empty(B, device="cuda")
    with pytest.raises(cp.CranePlanError) as ei:
        plan.eval_noalloc_into(W, cost_t, md)
    assert ei.value.code == -2 and "scratch" in str(ei.value)
    # within the limit the same plan evaluates
    plan.eval_noalloc_into(W[:1024], cost_t[:1024], md[:1024])
    torch.cuda.synchronize()
    assert torch.isfinite(cost_t[:1024]).all()
