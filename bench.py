"""Benchmark: one optimizer iteration of the crane path planner per step.

A step is one pass of the whole hot path on the c1_full workload (16384
sampled paths x 16 waypoints x 32 checkpoints per span = 608 checkpoints,
64 link spheres, 512 trees + 16 boxes + ground, 819 elites): sampling,
evaluation (interpolation, forward kinematics, sphere-obstacle distances,
cost), elite selection, mean/covariance update and the Cholesky factor.
Inputs are seeded synthetic data already resident on the GPU.

Prints one JSON line: configurations checked per second over the timed
optimizer iterations, planner iterations per second, the evaluation kernel
against the FP32 vector roofline, and the CPU oracle's rate on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic flops of one checked configuration (plain formulas, counted as
# add/sub/mul/min/max/sqrt = 1, fma = 2): a sphere-cylinder pair 15, a
# sphere-box pair 20, per sphere 7 (height term of the shared tree extent and
# the ground), interpolation + forward kinematics 1500
F_CYL, F_BOX, F_SPHERE, F_CONFIG = 15, 20, 7, 1500
PEAK_FP32 = 157.3e12  # MI355X FP32 vector peak (256 CU x 2.4 GHz x 256 flop/clk)
# HBM bytes per k_eval_fwd launch on c1_full from rocprofv3 FETCH_SIZE / WRITE_SIZE, each
# scaled by the same counter on a plain 1 GiB copy (profiles/k_eval_fwd_c1_full_hbm_bytes.md);
# None once the kernel has changed since the counters were taken
TRAFFIC_BYTES = None


def flops_per_config(n_spheres, n_cyl, n_box):
    return n_spheres * (n_cyl * F_CYL + n_box * F_BOX + F_SPHERE) + F_CONFIG


def cpu_baseline(prob, n_paths=1536, seed=7):
    import oracle
    oracle.build()
    rng = np.random.default_rng(seed)
    W = oracle.expand(prob.robot, oracle.Optimizer(prob).sample()[:n_paths], prob.cost.K)
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    t0 = time.perf_counter()
    oracle.eval_paths(m, prob.q_start, prob.q_goal, W)
    dt = time.perf_counter() - t0
    n_cfg = n_paths * prob.cost.n_s
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n_cfg / dt, "unit": "configs/s", "cores": min(threads, n_paths), "kind": "oracle",
            "sample": f"{n_paths} of {prob.opt.B} sampled paths of the first c1_full iteration "
                      f"({n_cfg} configurations, evaluation only), FP64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eval-reps", type=int, default=10)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path is single-GPU in this build",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n}))
        return
    from paper_2503_14160_amd import craneplan as cp
    from paper_2503_14160_amd import synth

    prob = synth.c1_full()
    B, ns = prob.opt.B, prob.cost.n_s
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    opt = cp.Optimizer(plan, prob.opt)
    torch.cuda.synchronize()

    print(f"[bench] c1_full warmup {args.warmup}", file=sys.stderr, flush=True)
    opt.step(args.warmup)
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} iterations", file=sys.stderr, flush=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    opt.step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_step = ms / args.steps
    st = opt.get_state()

    # evaluation kernel alone, on the same stream, on the last population
    W, cost, _ = opt.last()
    md = torch.empty_like(cost)
    plan.eval_into(W, cost, md)
    torch.cuda.synchronize()
    print(f"[bench] eval kernel x{args.eval_reps}", file=sys.stderr, flush=True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.eval_reps):
        plan.eval_into(W, cost, md)
    ev1.record()
    torch.cuda.synchronize()
    eval_ms = ev0.elapsed_time(ev1) / args.eval_reps
    fpc = flops_per_config(prob.robot.n_spheres, prob.scene.n_cyl, prob.scene.n_box)
    flops = fpc * B * ns
    achieved = flops / (eval_ms * 1e-3)

    # the same evaluation with every pair in full (no square-root skipping):
    # identical results, the brute-force reference for the roofline
    plain = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B, pair_filter=False)
    plain.set_endpoints(prob.q_start, prob.q_goal)
    c_plain = torch.empty_like(cost)
    plain.eval_into(W, c_plain, md)
    torch.cuda.synchronize()
    reps_plain = max(1, args.eval_reps // 3)
    ev0.record()
    for _ in range(reps_plain):
        plain.eval_into(W, c_plain, md)
    ev1.record()
    torch.cuda.synchronize()
    plain_ms = ev0.elapsed_time(ev1) / reps_plain
    same = bool(torch.equal(c_plain, cost))

    configs = B * ns
    out = {
        "metric": "configs checked/s (FK+collision)",
        "value": configs * args.steps / (ms * 1e-3),
        "unit": "configs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "planner_iters_per_s": 1e3 / ms_step,
        "eval_ms": eval_ms,
        "eval_configs_per_s": configs / (eval_ms * 1e-3),
        "best_cost": st["best_cost"],
        "wall_s": wall,
        "config": {"workload": "c1_full", "paths": B, "waypoints": prob.cost.K, "points_per_span": prob.cost.M,
                   "checkpoints": ns, "spheres": prob.robot.n_spheres, "cylinders": prob.scene.n_cyl,
                   "boxes": prob.scene.n_box, "elites": prob.opt.nu},
        "roofline": {"bound": "alu", "kernel": "k_eval_fwd", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": TRAFFIC_BYTES,
                     "flops_per_config": fpc,
                     "note": "algorithmic flops of the all-pairs definition; the kernel skips the square root of "
                             "pairs that cannot lower the minimum (bitwise-identical results), so this rate can "
                             "exceed the hardware peak; all_pairs_kernel is the same launch evaluating every pair",
                     "all_pairs_kernel": {"ms": plain_ms, "achieved": flops / (plain_ms * 1e-3) / 1e12,
                                          "frac": flops / (plain_ms * 1e-3) / PEAK_FP32,
                                          "identical_costs": same}},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
