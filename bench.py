"""Benchmark of the crane path planner on one MI355X.

Default (``--workload c1_full``): a step is one optimizer iteration of the
whole hot path on the 16384-path workload (16 waypoints, 32 checkpoints per
span = 608 checkpoints, 64 link spheres, 512 trees + 16 boxes + ground,
819 elites): sampling, evaluation (interpolation, forward kinematics,
sphere-obstacle distances, cost), elite selection, mean/covariance update and
the Cholesky factor.  Inputs are seeded synthetic data already resident on
the GPU.  Prints one JSON line: configurations checked per second over the
timed iterations, planner iterations per second, the evaluation kernel
against the FP32 vector roofline, and the CPU oracle's rate on a bounded
sample of the same workload.

Other workloads print their own line: c0_plain (small single problem),
c2_diff (adjoint: fwd+bwd vs fwd, gradient error, polished iterations),
c3_batch (many problems: batched graph launch vs one problem at a time),
c4_sdf (lidar -> signed-distance grid, trilinear queries, fwd+bwd),
ik (batched collision-free inverse kinematics with restarts),
sat (the separating-axis narrow phase on link hulls and oriented boxes),
traj (step two: batched trajectory refinement by direct collocation).
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
# a sphere-cylinder pair with its own height term (no shared extent): radial term 7, height term 2,
# combination 9, minus the radius 1, running minimum 1; a sphere-sphere self pair: difference 3,
# squared length 5, square root 1, radii 2, minimum 1; a sphere against the ground 3
F_CYL_FULL, F_SELF, F_GROUND = 20, 12, 3
PEAK_FP32 = 157.3e12  # MI355X FP32 vector peak (256 CU x 2.4 GHz x 256 flop/clk)
PEAK_HBM = 8.0e12     # MI355X HBM3E bytes/s
# algorithmic bytes of one trilinear signed-distance query: 8 FP32 corners
SDF_QUERY_BYTES = 32
# counter figures of the timed evaluation launches (rocprofv3 summaries); each
# file names the command it was taken with and a hash of the kernel sources,
# and its figures are used only while both still match
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_2503_14160_amd/csrc/eval.hip", "paper_2503_14160_amd/csrc/internal.h",
                  "paper_2503_14160_amd/csrc/launch.h", "include/craneplan.h"]


def kernel_source_hash():
    """Hash of what the evaluation kernels are compiled from: their sources,
    the headers they include and the compiler flags."""
    import hashlib

    from paper_2503_14160_amd import build
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(build.FLAGS).encode())
    return h.hexdigest()[:16]


def profile_figures(name, workload, steps, warmup):
    """The 'figure: key = value' lines of profiles/<name> if the file was taken
    on the current kernel sources with the same workload, steps and warmup;
    else None (with the reason)."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None, f"{name} missing"
    fig = {}
    for line in open(path):
        line = line.strip()
        if line.startswith("figure:") and "=" in line:
            k, v = line[len("figure:"):].split("=", 1)
            fig[k.strip()] = v.strip()
    want = {"source_sha16": kernel_source_hash(), "workload": workload, "steps": str(steps), "warmup": str(warmup)}
    for k, v in want.items():
        if fig.get(k) != v:
            return None, f"{name}: {k} is {fig.get(k)}, this run has {v}"
    return fig, name


def flops_per_config(n_spheres, n_cyl, n_box):
    return n_spheres * (n_cyl * F_CYL + n_box * F_BOX + F_SPHERE) + F_CONFIG


def _timed(torch, fn, reps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(prob, n_paths=1536):
    import oracle
    oracle.build()
    W = oracle.expand(prob.robot, oracle.Optimizer(prob).sample()[:n_paths], prob.cost.K)
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    t0 = time.perf_counter()
    oracle.eval_paths(m, prob.q_start, prob.q_goal, W)
    dt = time.perf_counter() - t0
    n_cfg = n_paths * prob.cost.n_s
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n_cfg / dt, "unit": "configs/s", "cores": min(threads, n_paths), "kind": "oracle",
            "sample": f"{n_paths} of {prob.opt.B} sampled paths of the first {prob.name} iteration "
                      f"({n_cfg} configurations, evaluation only), FP64, {dt:.1f} s"}


def base_line(args, metric, value, unit, ms_step, config, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": config}
    out.update(extra)
    return out


# ----------------------------------------------------------------------------
# c1_full / c0_plain: optimizer iterations
# ----------------------------------------------------------------------------

def bench_iterations(args, torch, cp, prob, with_roofline):
    """Optimizer iterations from creation: the timed region runs the
    workload's whole loop (K iterations from t = 0, after W warm-up
    iterations and a reset to the initial state), and every evaluation
    kernel inside it is bracketed by HIP events on the step's stream."""
    B, ns = prob.opt.B, prob.cost.n_s
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    opt = cp.Optimizer(plan, prob.opt)
    st0 = opt.get_state()
    torch.cuda.synchronize()
    print(f"[bench] {prob.name} warmup {args.warmup}", file=sys.stderr, flush=True)
    opt.step(args.warmup)
    opt.set_state(st0["mu"], st0["C"], 0)
    opt.time_eval(args.steps)
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} iterations from t = 0", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ms = _timed(torch, lambda: opt.step(args.steps), 1)
    wall = time.perf_counter() - t0
    eval_total_ms, launches = opt.eval_time()
    opt.time_eval(0)
    eval_ms = eval_total_ms / max(launches, 1)
    ms_step = ms / args.steps
    st = opt.get_state()
    configs = B * ns
    config = {"workload": prob.name, "paths": B, "waypoints": prob.cost.K, "points_per_span": prob.cost.M,
              "checkpoints": ns, "spheres": prob.robot.n_spheres, "cylinders": prob.scene.n_cyl,
              "boxes": prob.scene.n_box, "elites": prob.opt.nu, "iterations_timed": args.steps,
              "from_iteration": 0}
    out = base_line(args, "configs checked/s (FK+collision)", configs * args.steps / (ms * 1e-3), "configs/s",
                    ms_step, config, planner_iters_per_s=1e3 / ms_step, best_cost=st["best_cost"], wall_s=wall,
                    eval_ms=eval_ms, eval_launches_timed=launches, eval_configs_per_s=configs / (eval_ms * 1e-3))
    if not with_roofline:
        return out, plan, opt

    # executed FP32 work of the timed launches, from the counters
    fig, why = profile_figures("k_eval_fwd_c1_full_counters.md", prob.name, args.steps, args.warmup)
    fpc = flops_per_config(prob.robot.n_spheres, prob.scene.n_cyl, prob.scene.n_box)
    alg_flops = fpc * configs
    # the same evaluation with every pair in full (identical results) on the
    # last population: the all-pairs definition's own roofline
    W, cost, _ = opt.last()
    md = torch.empty_like(cost)
    plain = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B, pair_filter=cp.PAIRS_ALL)
    plain.set_endpoints(prob.q_start, prob.q_goal)
    c_plain = torch.empty_like(cost)
    c_cull = torch.empty_like(cost)
    plain.eval_into(W, c_plain, md)
    plan.eval_into(W, c_cull, md)
    torch.cuda.synchronize()
    print("[bench] all-pairs evaluation", file=sys.stderr, flush=True)
    plain_ms = _timed(torch, lambda: plain.eval_into(W, c_plain, md), max(1, args.eval_reps // 3))
    roof = {"bound": "alu", "kernel": "k_eval_fwd<false, true> (wave culling)", "unit": "TFLOP/s",
            "peak": PEAK_FP32 / 1e12, "launch_ms": eval_ms, "launches": launches,
            "achieved": None, "frac": None, "traffic": None, "counters": why,
            "effective": {"achieved": alg_flops / (eval_ms * 1e-3) / 1e12, "unit": "TFLOP/s",
                          "flops_per_config": fpc,
                          "note": "algorithmic flops of the all-pairs definition over the culling kernel's time: the "
                                  "kernel skips pairs that cannot lower any minimum (bitwise-identical results), so "
                                  "this rate is not a fraction of the hardware peak"},
            "all_pairs_kernel": {"ms": plain_ms, "achieved": alg_flops / (plain_ms * 1e-3) / 1e12,
                                 "frac": alg_flops / (plain_ms * 1e-3) / PEAK_FP32,
                                 "identical_costs": bool(torch.equal(c_plain, c_cull))}}
    if fig is not None:
        flops = float(fig["fp32_flops_per_launch"])
        roof.update({"achieved": flops / (eval_ms * 1e-3) / 1e12, "frac": flops / (eval_ms * 1e-3) / PEAK_FP32,
                     "flops_per_launch": flops, "profile_kernel_trace_ms": float(fig["kernel_trace_ms"]),
                     "flops_definition": "executed FP32 VALU flops per launch: 64 lanes x rocprofv3 "
                                         "SQ_INSTS_VALU_FLOPS_FP32 (ADD + MUL + 2 FMA + TRANS per wave "
                                         "instruction), averaged over the timed launches (profiles/" + why + ")"})
        if fig.get("hbm_bytes_per_launch") not in (None, "null"):
            roof["traffic"] = float(fig["hbm_bytes_per_launch"])
    out["roofline"] = roof
    return out, plan, opt


# ----------------------------------------------------------------------------
# c2_diff: adjoint
# ----------------------------------------------------------------------------

def bench_diff(args, torch, cp, prob):
    import oracle
    B = prob.opt.B
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    opt = cp.Optimizer(plan, synth_opt_no_polish(prob))
    opt.step(1)
    W, _, _ = opt.last()
    cost = torch.empty(B, device="cuda")
    md = torch.empty_like(cost)
    tape = torch.empty((B, plan.n_s), dtype=torch.int32, device="cuda")
    g = torch.empty_like(W)
    ones = torch.ones(B, device="cuda")
    plan.eval_into(W, cost, md)
    plan.eval_into(W, cost, md, tape=tape)
    plan.backward_into(W, ones, g, tape)
    torch.cuda.synchronize()
    print("[bench] c2_diff fwd / fwd+bwd", file=sys.stderr, flush=True)
    reps = args.eval_reps
    fwd_ms = _timed(torch, lambda: plan.eval_into(W, cost, md), reps)
    fwd_tape_ms = _timed(torch, lambda: plan.eval_into(W, cost, md, tape=tape), reps)

    def fb():
        plan.eval_into(W, cost, md, tape=tape)
        plan.backward_into(W, ones, g, tape)
    fb_ms = _timed(torch, fb, reps)

    def fb_nt():
        plan.eval_into(W, cost, md)
        plan.backward_into(W, ones, g, None)
    fb_nt_ms = _timed(torch, fb_nt, max(1, reps // 3))
    # gradient error of 8 paths against the oracle's analytic FP64 gradient
    Wn = W[:8].cpu().numpy().astype(np.float64)
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    _, gref = oracle.grad_paths(m, prob.q_start, prob.q_goal, Wn)
    gg = g[:8].cpu().numpy().astype(np.float64)
    rel = [float(np.linalg.norm(gg[b] - gref[b]) / max(np.linalg.norm(gref[b]), 1e-12)) for b in range(8)]
    # optimizer iterations with the gradient polish of the elites
    popt = cp.Optimizer(plan, prob.opt)
    popt.step(1)
    torch.cuda.synchronize()
    it_ms = _timed(torch, lambda: popt.step(args.steps), 1) / args.steps
    ns = plan.n_s
    config = {"workload": prob.name, "paths": B, "waypoints": prob.cost.K, "checkpoints": ns,
              "spheres": prob.robot.n_spheres, "cylinders": prob.scene.n_cyl, "boxes": prob.scene.n_box,
              "hinge": "smooth", "margin": prob.cost.margin, "polish": [prob.opt.polish_elites, prob.opt.polish_steps]}
    return base_line(args, "fwd+bwd time / fwd time", fb_ms / fwd_ms, "ratio", it_ms, config,
                     higher_is_better=False, fwd_ms=fwd_ms, fwd_with_tape_ms=fwd_tape_ms, fwd_bwd_ms=fb_ms,
                     fwd_bwd_without_tape_ms=fb_nt_ms, grad_rel_err_max=max(rel),
                     fwd_configs_per_s=B * ns / (fwd_ms * 1e-3), polished_iters_per_s=1e3 / it_ms)


def synth_opt_no_polish(prob):
    from paper_2503_14160_amd import synth
    o = prob.opt
    return synth.OptParams(B=o.B, nu=o.nu, sigma0=o.sigma0, eps=o.eps, seed=o.seed, T=o.T)


# ----------------------------------------------------------------------------
# c3_batch: many problems in one launch vs one at a time
# ----------------------------------------------------------------------------

def bench_batch(args, torch, cp, probs):
    n = len(probs)
    T = args.batch_iters
    work = np.array([p.opt.B * p.cost.n_s for p in probs], np.float64)
    print(f"[bench] c3_batch: {n} problems, building", file=sys.stderr, flush=True)
    batch = cp.Batch(probs)
    cache = args.tune_cache
    t0 = time.perf_counter()
    tuning = batch.tune(cache)
    tune_s = time.perf_counter() - t0
    print(f"[bench] tuned {tuning} in {tune_s:.1f} s; graph of {T} iterations", file=sys.stderr, flush=True)
    batch.run(1)  # warm-up iteration (its own small graph)
    batch.run(T)  # captures the T-iteration graph and runs it once
    torch.cuda.synchronize()
    ms_b = _timed(torch, lambda: batch.run(T), 1)  # replays the graph
    # the batched evaluation alone (one persistent launch and the per-path sums) on the current populations
    eval_b = _timed(torch, batch.eval, 5)
    print(f"[bench] batched {ms_b:.1f} ms (evaluation {eval_b:.2f} ms per iteration); sequential", file=sys.stderr,
          flush=True)
    # one problem at a time: same kernels, eager launches, synchronised per problem; then the evaluation alone
    # of each problem's last population, back to back
    per = np.zeros(n)
    eval_s = 0.0
    for i, p in enumerate(probs):
        plan = cp.Plan(p.robot, p.scene, p.cost, max_B=p.opt.B)
        plan.set_endpoints(p.q_start, p.q_goal)
        opt = cp.Optimizer(plan, p.opt, problem_id=i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        opt.step(T)
        torch.cuda.synchronize()
        per[i] = (time.perf_counter() - t0) * 1e3
        W, c_last, _ = opt.last()
        md = torch.empty_like(c_last)
        plan.eval_into(W, c_last, md)
        eval_s += _timed(torch, lambda: plan.eval_into(W, c_last, md), 3)
        if i % 32 == 0:
            print(f"[bench] sequential {i}/{n}", file=sys.stderr, flush=True)
    ms_s = per.sum()
    total_cfg = work.sum() * T
    # per-size buckets: ratio of the bucket's sequential time to its share of the batched time
    order = np.argsort(work)
    buckets = {}
    for name, idx in (("small", order[: n // 3]), ("medium", order[n // 3: 2 * n // 3]), ("large", order[2 * n // 3:])):
        share = ms_b * work[idx].sum() / work.sum()
        buckets[name] = {"problems": int(len(idx)), "sequential_ms": float(per[idx].sum()),
                         "batched_share_ms": float(share), "ratio": float(per[idx].sum() / share)}
    config = {"workload": "c3_batch", "problems": n, "iterations": T,
              "paths": [int(min(p.opt.B for p in probs)), int(max(p.opt.B for p in probs))],
              "waypoints": [int(min(p.cost.K for p in probs)), int(max(p.cost.K for p in probs))],
              "obstacles": [int(min(p.scene.n_cyl + p.scene.n_box for p in probs)),
                            int(max(p.scene.n_cyl + p.scene.n_box for p in probs))],
              "tuning": {"rounds": tuning[0], "wg_per_cu": tuning[1]}}
    # where the time goes, per iteration: evaluation and the rest, each way
    o_s, o_b = ms_s / T - eval_s, ms_b / T - eval_b
    model = {"per_iteration_ms": {"sequential_eval": eval_s, "sequential_rest": o_s, "batched_eval": eval_b,
                                  "batched_rest": o_b},
             "eval_only_ratio": eval_s / eval_b,
             "bound_with_no_batched_rest": (eval_s + o_s) / eval_b,
             "note": "the batched run can beat one problem at a time by at most (sequential evaluation + "
                     "sequential rest) / batched evaluation; the evaluation of one problem already fills the chip "
                     "for all but the smallest problems, so the batched evaluation is about as fast as the "
                     "sequential ones added up"}
    return base_line(args, "configs checked/s (FK+collision), batched", total_cfg / (ms_b * 1e-3), "configs/s",
                     ms_b / T, config, batched_ms=ms_b, sequential_ms=ms_s, batched_over_sequential=ms_s / ms_b,
                     model=model,
                     sequential_configs_per_s=total_cfg / (ms_s * 1e-3), planner_iters_per_s=T * n / (ms_b * 1e-3),
                     buckets=buckets, tune_s=tune_s)


# ----------------------------------------------------------------------------
# c4_sdf: lidar -> signed-distance grid, trilinear queries
# ----------------------------------------------------------------------------

def bench_sdf(args, torch, cp, prob):
    """c4_sdf: the grid built on the device from the lidar cloud, then
    optimizer iterations from t = 0 in which every iteration also takes the
    population's gradient (forward with the argmin tape, then the adjoint)."""
    spec = prob.sdf
    pts = torch.from_numpy(prob.lidar).cuda()
    cp.sdf_build(pts, spec)
    torch.cuda.synchronize()
    print("[bench] c4_sdf build", file=sys.stderr, flush=True)
    # with every optional output supplied the call allocates nothing, so the
    # events time the build kernels alone
    build_ms = _timed(torch, lambda: cp.sdf_build(pts, spec, with_edt=True), 5)
    sdf = cp.sdf_build(pts, spec)
    torch.cuda.synchronize()
    # algorithmic bytes of the build: the points once, then per voxel the
    # occupancy fill and write (2 B), two distance transforms (per transform:
    # x pass 1 B in + 4 B out, y and z passes 4 + 4 B each, final fix-up 4 + 4 B)
    # and the sign pass (1 + 4 + 4 B in, 4 B out)
    n_vox = int(np.prod(spec.dims))
    build_bytes = 12 * int(prob.lidar.shape[0]) + n_vox * (2 + 2 * (5 + 8 + 8 + 8) + 13)
    B = prob.opt.B
    plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=B, sdf=sdf, sdf_spec=spec)
    plan.set_endpoints(prob.q_start, prob.q_goal)
    opt = cp.Optimizer(plan, prob.opt)
    opt.record_tape(True)
    st0 = opt.get_state()
    g = torch.empty((B, prob.cost.K, prob.robot.n_joints), dtype=torch.float32, device="cuda")

    def step():
        opt.step(1)
        opt.population_grad(g)
    for _ in range(args.warmup):
        step()
    opt.set_state(st0["mu"], st0["C"], 0)
    opt.time_eval(args.steps)
    torch.cuda.synchronize()
    print(f"[bench] c4_sdf {args.steps} iterations with the population gradient", file=sys.stderr, flush=True)

    def loop():
        for _ in range(args.steps):
            step()
    ms = _timed(torch, loop, 1)
    eval_total_ms, launches = opt.eval_time()
    opt.time_eval(0)
    eval_ms = eval_total_ms / max(launches, 1)
    ms_step = ms / args.steps
    # forward alone and forward + backward on the last population
    W, cost, _ = opt.last()
    md = torch.empty_like(cost)
    tape = torch.empty((B, plan.n_s), dtype=torch.int32, device="cuda")
    ones = torch.ones(B, device="cuda")
    plan.eval_into(W, cost, md, tape=tape)
    plan.backward_into(W, ones, g, tape)
    torch.cuda.synchronize()
    fwd_ms = _timed(torch, lambda: plan.eval_into(W, cost, md), args.eval_reps)

    def fb():
        plan.eval_into(W, cost, md, tape=tape)
        plan.backward_into(W, ones, g, tape)
    fb_ms = _timed(torch, fb, args.eval_reps)
    ns = plan.n_s
    queries = B * ns * prob.robot.n_spheres
    config = {"workload": "c4_sdf", "points": int(prob.lidar.shape[0]), "grid": list(spec.dims),
              "voxel": spec.voxel, "paths": B, "waypoints": prob.cost.K, "checkpoints": ns,
              "spheres": prob.robot.n_spheres, "iterations_timed": args.steps, "from_iteration": 0,
              "step": "sample, evaluate (with argmin tape), select, update, factor, population gradient"}
    roof = {"kernel": "k_eval_fwd<true, false> (grid lookups, argmin tape)", "launch_ms": eval_ms,
            "launches": launches, "bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
            "traffic": None,
            "effective": {"achieved": queries * SDF_QUERY_BYTES / (eval_ms * 1e-3) / 1e9, "unit": "GB/s",
                          "note": "algorithmic bytes, 8 FP32 corners for every sphere's query, over the launch: "
                                  "the kernel skips the lookups that the grid's 2x2x2-block lower bounds show "
                                  "cannot lower the minimum (bitwise-identical results) and the 32 MiB grid is "
                                  "cache resident, so this is not a fraction of HBM bandwidth"}}
    fig, why = profile_figures("k_eval_fwd_c4_sdf_counters.md", "c4_sdf", args.steps, args.warmup)
    roof["counters"] = why
    if fig is not None:
        flops = float(fig["fp32_flops_per_launch"])
        hbm = float(fig["hbm_bytes_per_launch"])
        f_alu = flops / (eval_ms * 1e-3) / PEAK_FP32
        f_hbm = hbm / (eval_ms * 1e-3) / PEAK_HBM
        roof["traffic"] = hbm
        roof["fp32"] = {"achieved": flops / (eval_ms * 1e-3) / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                        "frac": f_alu}
        roof["hbm"] = {"achieved": hbm / (eval_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                       "frac": f_hbm}
        if f_alu >= f_hbm:
            roof.update(bound="alu", achieved=roof["fp32"]["achieved"], peak=PEAK_FP32 / 1e12, unit="TFLOP/s",
                        frac=f_alu)
        else:
            roof.update(bound="hbm", achieved=roof["hbm"]["achieved"], peak=PEAK_HBM / 1e9, unit="GB/s",
                        frac=f_hbm)
    return base_line(args, "configs checked/s (FK+collision)", B * ns * args.steps / (ms * 1e-3), "configs/s",
                     ms_step, config, planner_iters_per_s=1e3 / ms_step, sdf_build_ms=build_ms,
                     sdf_build_roofline={"bound": "hbm", "unit": "GB/s", "bytes": build_bytes,
                                         "achieved": build_bytes / (build_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                                         "frac": build_bytes / (build_ms * 1e-3) / PEAK_HBM}, fwd_ms=fwd_ms,
                     fwd_bwd_ms=fb_ms, fwd_bwd_over_fwd=fb_ms / fwd_ms, eval_ms=eval_ms, roofline=roof)


# ----------------------------------------------------------------------------
# ik: batched collision-free inverse kinematics
# ----------------------------------------------------------------------------

def bench_ik(args, torch, cp, cand):
    """ik: the grasp poses of hanging configurations on the c1 crane (with its
    self pairs) in the c1 forest, picked where the configuration keeps 0.1 m
    from the scene and itself (by the library's own distance), several
    starting points per target, one launch solving every row by
    Levenberg-Marquardt; reports rows and targets per second and the launch
    against the FP32 vector roofline, counting each d(q) evaluation's
    all-pairs flops (the kernel takes every pair)."""
    from paper_2503_14160_amd import synth
    plan = cp.Plan(cand.robot, cand.scene, synth_cost_any(), max_B=1)
    dist, _ = plan.debug_configs(torch.from_numpy(cand.q_star).cuda())
    prob = cand.pick(dist.cpu().numpy() > synth.IK_TARGET_CLEARANCE)
    n = prob.robot.n_joints
    N = prob.q_init.shape[0]
    R = prob.restarts
    # targets: the last frame's rotation and its tip point at q_star (the library's own kinematics)
    qs = torch.from_numpy(prob.q_star).cuda()
    _, frames = plan.debug_fk(qs)
    Rm = frames[:, n, :9].reshape(-1, 3, 3)
    tip = torch.from_numpy(np.asarray(prob.robot.tip, np.float32)).cuda()
    p = torch.matmul(Rm, tip) + frames[:, n, 9:12]
    T = torch.cat([frames[:, n, :9], p], dim=1).repeat_interleave(R, dim=0).contiguous()
    q0 = torch.from_numpy(prob.q_init).cuda()
    qr = torch.from_numpy(np.broadcast_to(prob.q_ref, (N, n)).copy()).cuda()
    par = prob.params
    for _ in range(max(1, args.warmup)):
        q, info, status, best = plan.ik_solve(par, T, q0, qr, restarts=R)
    torch.cuda.synchronize()
    print(f"[bench] ik: {N} rows ({N // R} targets x {R} starts), {args.steps} timed launches", file=sys.stderr,
          flush=True)
    ms = _timed(torch, lambda: plan.ik_solve(par, T, q0, qr, restarts=R), args.steps)
    q, info, status, best = plan.ik_solve(par, T, q0, qr, restarts=R)
    inf = info.cpu().numpy()
    evals = float(np.sum(1.0 + inf[:, 5]))
    S = prob.robot.n_spheres
    n_self = self_sphere_pairs(prob.robot)
    # per d(q) evaluation: every sphere against the ground, the cylinders (each with its own height
    # term) and the boxes, and the self pairs; the chain, the residual and Jacobian rows and the normal
    # equations of each row and evaluation are not counted
    f_eval = S * (prob.scene.n_cyl * F_CYL_FULL + prob.scene.n_box * F_BOX + F_GROUND) + n_self * F_SELF
    flops = evals * f_eval
    bi = best.cpu().numpy()
    Fb = inf[bi, 0]
    config = {"workload": "ik_c1", "targets": N // R, "restarts": R, "rows": N, "max_iters": par.max_iters,
              "target_clearance_m": synth.IK_TARGET_CLEARANCE, "candidates": int(cand.q_star.shape[0]),
              "spheres": S, "cylinders": prob.scene.n_cyl, "boxes": prob.scene.n_box, "self_sphere_pairs": n_self,
              "weights": [par.lambda_q, par.lambda_c, par.lambda_e, par.lambda_r]}
    roof = {"bound": "alu", "kernel": "k_ik_solve", "unit": "TFLOP/s", "peak": PEAK_FP32 / 1e12,
            "launch_ms": ms, "achieved": flops / (ms * 1e-3) / 1e12, "frac": flops / (ms * 1e-3) / PEAK_FP32,
            "traffic": None, "flops_per_launch": flops, "flops_per_distance": f_eval,
            "distance_evaluations": evals,
            "note": "algorithmic flops of the distance evaluations (every sphere-obstacle and self pair per trial "
                    "step) over the launch; the wave-uniform solver arithmetic is not counted"}
    out = base_line(args, "IK rows solved/s", N / (ms * 1e-3), "rows/s", ms, config,
                    targets_per_s=(N // R) / (ms * 1e-3), mean_trial_steps=float(inf[:, 5].mean()),
                    status_counts={str(k): int(v) for k, v in zip(*np.unique(status.cpu().numpy(),
                                                                               return_counts=True))},
                    best_pos_err_median=float(np.median(inf[bi, 1])), best_cost_median=float(np.median(Fb)),
                    best_in_collision=float(np.mean(inf[bi, 3] < 0)), roofline=roof)
    return out, T, prob


def synth_cost_any():
    from paper_2503_14160_amd import synth
    return synth.CostParams(K=4, M=4)


def self_sphere_pairs(robot):
    counts = np.bincount(np.asarray(robot.sphere_frame), minlength=robot.n_joints + 1)
    return int(sum(counts[a] * counts[b] for a, b in np.asarray(robot.self_pairs).reshape(-1, 2)))


def cpu_baseline_ik(prob, T, rows=1024):
    import oracle
    oracle.build()
    m = oracle.Model(prob.robot, prob.scene, None)
    Tn = T[:rows].cpu().numpy().astype(np.float64)
    t0 = time.perf_counter()
    for i in range(rows):
        oracle.ik_solve(m, prob.params, Tn[i], prob.q_init[i].astype(np.float64), prob.q_ref.astype(np.float64))
    dt = time.perf_counter() - t0
    return {"value": rows / dt, "unit": "rows/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {rows} of {prob.q_init.shape[0]} rows of the ik workload, solved one after "
                      f"another (C residual + numpy Levenberg-Marquardt, FP64), {dt:.1f} s"}


# ----------------------------------------------------------------------------
# sat: the separating-axis narrow phase on hulls
# ----------------------------------------------------------------------------

# algorithmic flops of the SAT distance of two oriented boxes: centre offset 3,
# its components along both boxes' axes 6 x 5, the cosine matrix 9 x 5, six
# face axes (half-width sum 5, |T| - two half-widths 2, maximum 1) 6 x 8, nine
# cross axes (length 2, centre term 3, two half-widths 3 + 3, difference 2,
# square root 1, division 1, maximum 1) 9 x 16; placing a hull (its chain,
# centre and axes) 400, its ground distance 8; interpolation and step terms 200
F_SAT_PAIR, F_HULL, F_HULL_GROUND, F_SAT_CONFIG = 270, 400, 8, 200


def sat_problem():
    import dataclasses

    from paper_2503_14160_amd import synth
    base = synth.c1_full()
    robot = synth.with_self_collision(synth.with_hulls(base.robot))
    scene = synth.hull_scene(np.random.default_rng(synth.SCENE_SEED + 7), base.scene)
    return dataclasses.replace(base, name="c1_sat", robot=robot, scene=scene)


def bench_sat(args, torch, cp, prob):
    """sat: the c1 population (16384 paths x 608 checkpoints) with the
    separating-axis narrow phase, 5 link hulls against the c1 forest as 528
    oriented boxes and the ground (and the hull pairs of the non-adjacent
    links): optimizer iterations from t = 0; plus the paper's collision
    benchmark shape, 100 paths x 100 points in one evaluation launch."""
    import dataclasses

    from paper_2503_14160_amd import synth
    out, plan, opt = bench_iterations(args, torch, cp, prob, with_roofline=False)
    H = len(prob.robot.hull_box)
    n_self = sum(1 for k in range(H) for m in range(k + 1, H)
                 if any({int(prob.robot.hull_frame[k]), int(prob.robot.hull_frame[m])} == {int(a), int(b)}
                        for a, b in prob.robot.self_pairs))
    fpc = (H * (F_HULL + F_HULL_GROUND + prob.scene.n_obb * F_SAT_PAIR) + n_self * (F_SAT_PAIR + 2 * F_HULL)
           + F_SAT_CONFIG)
    configs = prob.opt.B * plan.n_s
    eval_ms = out["eval_ms"]
    out["config"].update(hulls=H, oriented_boxes=prob.scene.n_obb, hull_self_pairs=n_self, narrow="sat")
    # the same launch with every axis of every pair (CP_PAIRS_ALL, identical results) on the last population:
    # the definition's own roofline
    W, cost_b, _ = opt.last()
    md = torch.empty_like(cost_b)
    c_all, c_cut = torch.empty_like(cost_b), torch.empty_like(cost_b)
    plain = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=prob.opt.B, pair_filter=cp.PAIRS_ALL)
    plain.set_endpoints(prob.q_start, prob.q_goal)
    plain.eval_into(W, c_all, md)
    plan.eval_into(W, c_cut, md)
    torch.cuda.synchronize()
    all_ms = _timed(torch, lambda: plain.eval_into(W, c_all, md), max(1, args.eval_reps // 3))
    alg = fpc * configs
    out["roofline"] = {"bound": "alu", "kernel": "k_eval_fwd_sat<false> (every axis of every pair)",
                       "unit": "TFLOP/s", "peak": PEAK_FP32 / 1e12, "launch_ms": all_ms,
                       "achieved": alg / (all_ms * 1e-3) / 1e12, "frac": alg / (all_ms * 1e-3) / PEAK_FP32,
                       "flops_per_config": fpc, "traffic": None,
                       "identical_costs": bool(torch.equal(c_all, c_cut)),
                       "early_exit_kernel": {"launch_ms": eval_ms, "launches": out["eval_launches_timed"],
                                             "effective": alg / (eval_ms * 1e-3) / 1e12,
                                             "note": "the timed launches stop a pair after the box's face axes when "
                                                     "they show it cannot lower the minimum (bitwise the same "
                                                     "results); algorithmic flops over their time are not a "
                                                     "fraction of the peak"},
                       "note": "algorithmic flops of every hull-box SAT test (15 axes), every hull placement and "
                               "self pair, over the every-axis launch on the last population"}
    # the paper's shape: 100 paths, 100 checkpoints each (K = 7, M = 10: (7 + 3) x 10)
    cost = dataclasses.replace(prob.cost, K=7, M=10)
    small = cp.Plan(prob.robot, prob.scene, cost, max_B=100)
    small.set_endpoints(prob.q_start, prob.q_goal)
    rng = np.random.default_rng(5)
    W = torch.from_numpy(synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 100, 7, sigma=0.3)).cuda()
    c = torch.empty(100, device="cuda")
    md = torch.empty_like(c)
    small.eval_into(W, c, md)
    torch.cuda.synchronize()
    e1_ms = _timed(torch, lambda: small.eval_into(W, c, md), args.eval_reps)
    out["paper_shape"] = {"paths": 100, "checkpoints": small.n_s, "configs": 100 * small.n_s, "ms": e1_ms,
                          "configs_per_s": 100 * small.n_s / (e1_ms * 1e-3),
                          "paper_context": "10^4 configurations in 0.014 s on an RTX 4090 with MJX SAT on 32 "
                                           "meshes (other hardware, other geometry)"}
    return out


def cpu_baseline_sat(prob, n_paths=1024):
    import oracle
    oracle.build()
    rng = np.random.default_rng(6)
    from paper_2503_14160_amd import synth
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, n_paths, prob.cost.K, sigma=0.3)
    m = oracle.Model(prob.robot, prob.scene, prob.cost)
    t0 = time.perf_counter()
    oracle.eval_paths(m, prob.q_start, prob.q_goal, W.astype(np.float64))
    dt = time.perf_counter() - t0
    n_cfg = n_paths * prob.cost.n_s
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n_cfg / dt, "unit": "configs/s", "cores": min(threads, n_paths), "kind": "oracle",
            "sample": f"{n_paths} random paths of the c1 shape with the SAT narrow phase ({n_cfg} configurations, "
                      f"evaluation only), FP64, {dt:.1f} s"}


# ----------------------------------------------------------------------------
# traj: step two, batched trajectory refinement
# ----------------------------------------------------------------------------

PEAK_FP64 = 78.6e12  # MI355X FP64 vector peak


def traj_flops(N, n, na, robot):
    """Algorithmic FP64 flops of one assembly (dynamics Jacobians by central
    differences and the normal equations) and of one trial step (block
    factorisation, two solves, the trial point's dynamics and objective, the
    predicted decrease) at the kernel's block of MB = 16 entries per point.
    One evaluation of the dynamics: the chain (a revolute joint 107, a
    prismatic one 40: world axis 15, origin 18, rotation 27 + 2, product
    45), the tip 18, the Jacobian columns 12 per joint, the velocity term
    (a revolute pair 27, a revolute-prismatic pair 18), the inputs and the
    passive joints' 2 x 2 solve 50."""
    jt = np.asarray(robot.joint_type)
    rev = int(np.sum(jt == 0))
    pri = len(jt) - rev
    f_dyn = 107 * rev + 40 * pri + 18 + 12 * n + 27 * rev * (rev + 1) // 2 + 18 * rev * pri + 50
    MB, nx = 16, 2 * n
    jac = (N + 1) * (1 + 2 * (nx + na)) * f_dyn + (N + 1) * (nx + na) * nx * 2
    normal = (N + 1) * MB * MB * 2 * nx * 2 + N * MB * MB * nx * 2 + (N + 1) * MB * 2 * nx * 2 * 2 + N * nx * 4
    chol = sum((MB - 1 - j) * (MB - j) for j in range(MB)) + MB + MB * (MB - 1) // 2
    factor = (N + 1) * (MB * MB * MB * 2 + chol + MB * MB * (MB + 1))
    solve = (N + 1) * 2 * 2 * (MB * MB * 2 + MB * (MB + 1)) + 2 * (N + 1) * MB * 2 * 2
    trial = (N + 1) * f_dyn + (N * nx + (N - 1) * nx + N * na) * 4 + (N + 1) * MB * (3 * MB * 2 + 4)
    return {"assembly": jac + normal, "trial": factor + solve + trial, "dynamics": f_dyn}


def bench_traj(args, torch, cp):
    """traj: step two on P problems at the paper's 100 collocation intervals
    (the c1 crane's chain; start/goal moves and bent step-one paths from the
    seeded recipe), default solver settings, one launch refining all of
    them; reports trajectories per second and the launch against the FP64
    vector roofline (algorithmic flops from each problem's own counts of
    assemblies and trial steps)."""
    from paper_2503_14160_amd import synth
    robot = synth.c1_full().robot
    par = synth.TrajParams(N=100)
    P = args.batch_problems
    q0, qg, qs = synth.traj_problems(robot, P, par.N, synth.SCENE_SEED + 11)
    plan = cp.Plan(robot, synth.c0_plain().scene, synth_cost_any(), max_B=1)
    a = [torch.from_numpy(x).cuda() for x in (q0, qg, qs)]
    for _ in range(max(1, args.warmup)):
        plan.traj_refine(par, *a)
    torch.cuda.synchronize()
    print(f"[bench] traj: {P} problems, N = {par.N}, {args.steps} timed launches", file=sys.stderr, flush=True)
    ms = _timed(torch, lambda: plan.traj_refine(par, *a), args.steps)
    X, U, tf, info = plan.traj_refine(par, *a)
    inf = info.cpu().numpy().astype(np.float64)
    n = robot.n_joints
    na = int(np.sum(robot.active))
    fl = traj_flops(par.N, n, na, robot)
    flops = float(np.sum(inf[:, 2]) * fl["trial"] + np.sum(inf[:, 3] + par.outer) * fl["assembly"])
    config = {"workload": "traj_n100", "problems": P, "intervals": par.N, "unknowns_per_problem": 16 * (par.N - 1) + 4 * 2 + 1,
              "outer": par.outer, "max_iters": par.max_iters, "mu0": par.mu0, "omega_s": par.omega_s,
              "omega_t": par.omega_t}
    roof = {"bound": "alu", "kernel": "k_traj_refine", "unit": "TFLOP/s", "peak": PEAK_FP64 / 1e12, "launch_ms": ms,
            "achieved": flops / (ms * 1e-3) / 1e12, "frac": flops / (ms * 1e-3) / PEAK_FP64, "traffic": None,
            "flops_per_launch": flops, "flops_per_assembly": fl["assembly"], "flops_per_trial": fl["trial"],
            "note": "algorithmic FP64 flops of the assemblies (accepted steps plus one per outer round) and trial "
                    "steps each problem took, over the launch; the solve is a sequential sweep over the 101 blocks "
                    "of each problem, bound by latency rather than by the vector units"}
    out = base_line(args, "trajectories refined/s", P / (ms * 1e-3), "trajectories/s", ms, config,
                    ms_per_trajectory_in_batch=ms / P, trial_steps_mean=float(inf[:, 2].mean()),
                    accepted_steps_mean=float(inf[:, 3].mean()), defect_median=float(np.median(inf[:, 0])),
                    defect_below_1e_8=float(np.mean(inf[:, 0] < 1e-8)), t_f_median=float(np.median(tf.cpu().numpy())),
                    roofline=roof)
    out["dtype"] = "f64"
    return out, (robot, par, q0, qg, qs)


def cpu_baseline_traj(robot, par, q0, qg, qs, problems=1):
    import oracle
    oracle.build()
    m = oracle.Model(robot, synth_scene_empty(), None)
    t0 = time.perf_counter()
    for p in range(problems):
        oracle.traj_refine(m, par, q0[p].astype(np.float64), qg[p].astype(np.float64), qs[p].astype(np.float64))
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": problems / dt, "unit": "trajectories/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {problems} of the traj workload's problems (N = {par.N}, dense FP64 "
                      f"Levenberg-Marquardt in numpy, the C dynamics), {dt:.1f} s"}


def synth_scene_empty():
    from paper_2503_14160_amd import synth
    return synth.c0_plain().scene


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed iterations (default: the workload's iteration count, 50 for c1_full; 20 otherwise)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c1_full",
                    choices=["c1_full", "c1_self", "c0_plain", "c2_diff", "c3_batch", "c4_sdf", "ik", "sat", "traj"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eval-reps", type=int, default=10)
    ap.add_argument("--batch-problems", type=int, default=256)
    ap.add_argument("--batch-iters", type=int, default=30)
    ap.add_argument("--tune-cache", default=None, metavar="PATH",
                    help="c3_batch: text cache of tuned launch shapes (default: none, the tuner times every shape)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library evaluates and optimizes "
              f"on a single device", file=sys.stderr)
        sys.exit(2)

    if args.steps is None:
        args.steps = 50 if args.workload in ("c1_full", "c1_self", "c4_sdf") else 20
        if args.workload == "sat":
            args.steps = 10
        if args.workload == "traj":
            args.steps = 3
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

    if args.workload == "c1_full":
        prob = synth.c1_full()
        out, _, _ = bench_iterations(args, torch, cp, prob, with_roofline=True)
        if not args.no_cpu_baseline:
            print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
            out["cpu_baseline"] = cpu_baseline(prob)
    elif args.workload == "c1_self":
        # c1_full with the crane's non-adjacent link pairs also checked against each other
        import dataclasses
        prob = synth.c1_full()
        prob = dataclasses.replace(prob, name="c1_self", robot=synth.with_self_collision(prob.robot))
        out, _, _ = bench_iterations(args, torch, cp, prob, with_roofline=False)
        out["config"]["self_pairs"] = prob.robot.self_pairs.tolist()
    elif args.workload == "c0_plain":
        out, _, _ = bench_iterations(args, torch, cp, synth.c0_plain(), with_roofline=False)
    elif args.workload == "c2_diff":
        out = bench_diff(args, torch, cp, synth.c2_diff())
    elif args.workload == "c3_batch":
        out = bench_batch(args, torch, cp, synth.c3_batch(args.batch_problems))
    elif args.workload == "sat":
        prob = sat_problem()
        out = bench_sat(args, torch, cp, prob)
        if not args.no_cpu_baseline:
            print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
            out["cpu_baseline"] = cpu_baseline_sat(prob)
    elif args.workload == "traj":
        out, ctx = bench_traj(args, torch, cp)
        if not args.no_cpu_baseline:
            print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
            out["cpu_baseline"] = cpu_baseline_traj(*ctx)
    elif args.workload == "ik":
        out, T, prob = bench_ik(args, torch, cp, synth.ik_c1())
        if not args.no_cpu_baseline:
            print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
            out["cpu_baseline"] = cpu_baseline_ik(prob, T)
    else:
        out = bench_sdf(args, torch, cp, synth.c4_sdf())
    print(json.dumps(out))


if __name__ == "__main__":
    main()
