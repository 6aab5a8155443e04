"""The three pair modes of cp_cost_params.pair_filter (every pair, the
lane-level square-root skip, the wave-level culling) must give bitwise the
same distances, costs, flags and argmin records: skipped pairs are exactly
those that cannot lower a minimum.  Cases cover waves that hold one path, two
paths and many paths, wide and narrow perturbations, boxes overlapping the
crane, centres inside obstacles, non-finite waypoints, a scene thousands of
metres away (rounding at large coordinates) and the batched launch."""
import dataclasses

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


def _bits(t):
    return t.contiguous().view(torch.int32).cpu().numpy() if t.dtype == torch.float32 else t.cpu().numpy()


def _eval_modes(cp, prob, W, label, backward=False):
    print(f"[pairs] {label} B={W.shape[0]} K={prob.cost.K} M={prob.cost.M}", flush=True)
    Wt = torch.from_numpy(np.ascontiguousarray(W, dtype=np.float32)).cuda()
    out = {}
    for mode in (cp.PAIRS_ALL, cp.PAIRS_LANE, cp.PAIRS_WAVE, cp.PAIRS_AUTO):
        plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=W.shape[0], pair_filter=mode)
        plan.set_endpoints(prob.q_start, prob.q_goal)
        cost, md, fl, tape = plan.eval(Wt, tape=True)
        res = [_bits(cost), _bits(md), _bits(fl), _bits(tape)]
        if backward:
            gc = torch.linspace(0.5, 2.0, W.shape[0], device="cuda")
            res.append(_bits(plan.backward(Wt, gc, None)))
        torch.cuda.synchronize()
        out[mode] = res
    for mode in (cp.PAIRS_LANE, cp.PAIRS_WAVE, cp.PAIRS_AUTO):
        for name, a, b in zip(("cost", "min_dist", "flags", "tape", "grad"), out[cp.PAIRS_ALL], out[mode]):
            np.testing.assert_array_equal(a, b, err_msg=f"{label}: {name} differs in mode {mode}")
    return out[cp.PAIRS_ALL]


def test_pairs_c0(cp):
    prob = synth.c0_plain()
    rng = np.random.default_rng(700)
    for sigma in (0.05, 0.3, 1.0):
        W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 256, prob.cost.K, sigma=sigma)
        _eval_modes(cp, prob, W, f"c0 sigma={sigma}")


def test_pairs_c1_subset(cp):
    prob = synth.c1_full()
    rng = np.random.default_rng(701)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 512, prob.cost.K, sigma=0.2)
    _eval_modes(cp, prob, W, "c1 512 paths")


def test_pairs_smooth_hinge_and_backward(cp):
    base = synth.c1_full()
    cost = synth.CostParams(K=8, M=16, hinge=synth.HINGE_SMOOTH, margin=0.1)
    prob = synth.Problem("diff", base.robot, base.scene, base.q_start, base.q_goal, cost, base.opt)
    rng = np.random.default_rng(702)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 48, cost.K, sigma=0.4)
    _eval_modes(cp, prob, W, "smooth hinge", backward=True)


@pytest.mark.parametrize("K,M,B", [(5, 7, 37), (3, 2, 51), (1, 1, 200), (12, 9, 1)])
def test_pairs_many_paths_per_wave(cp, K, M, B):
    base = synth.c0_plain()
    cost = synth.CostParams(K=K, M=M, interp=synth.INTERP_LINEAR if M < 4 else synth.INTERP_BSPLINE)
    prob = synth.Problem("variant", base.robot, base.scene, base.q_start, base.q_goal, cost, base.opt)
    rng = np.random.default_rng(703 + K)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, B, K, sigma=0.5)
    _eval_modes(cp, prob, W, f"K={K} M={M} B={B}")


def test_pairs_dense_overlapping_scene(cp):
    """Boxes and trees right on the crane's sweep: centres inside obstacles,
    negative distances, boxes whose slabs overlap the wave's box."""
    base = synth.c0_plain()
    rng = np.random.default_rng(704)
    r = rng.uniform(2.0, 12.0, 300)
    a = rng.uniform(-np.pi, np.pi, 300)
    cyl = np.stack([r * np.cos(a), r * np.sin(a), rng.uniform(0.05, 0.8, 300),
                    np.zeros(300), rng.uniform(2.0, 15.0, 300)], 1).astype(np.float32)
    rb = rng.uniform(2.0, 12.0, 40)
    ab = rng.uniform(-np.pi, np.pi, 40)
    box = np.stack([rb * np.cos(ab), rb * np.sin(ab), rng.uniform(0.5, 6.0, 40),
                    rng.uniform(0.2, 3.0, 40), rng.uniform(0.2, 3.0, 40), rng.uniform(0.2, 3.0, 40)], 1)
    scene = synth.Scene(cyl=cyl, box=box.astype(np.float32), has_ground=1, ground_z=0.0)
    prob = dataclasses.replace(base, scene=scene)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 128, prob.cost.K, sigma=0.5)
    _eval_modes(cp, prob, W, "dense overlapping")


def test_pairs_far_scene(cp):
    """Obstacles about 3 km away: distances near 3000 m, where a float's unit
    in the last place is 0.25 mm and the relative slack decides."""
    base = synth.c0_plain()
    rng = np.random.default_rng(705)
    n = 200
    cyl = np.stack([3000.0 + rng.uniform(-5, 5, n), rng.uniform(-5, 5, n), rng.uniform(0.1, 0.5, n),
                    np.zeros(n), np.full(n, 15.0)], 1).astype(np.float32)
    box = np.array([[-2990.0, 3.0, 1.0, 1.0, 2.0, 1.0], [-2995.0, -3.0, 2.0, 0.5, 0.5, 2.0]], np.float32)
    scene = synth.Scene(cyl=cyl, box=box, has_ground=0, ground_z=0.0)
    prob = dataclasses.replace(base, scene=scene)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 128, prob.cost.K, sigma=0.3)
    _eval_modes(cp, prob, W, "far scene")


def test_pairs_nonfinite(cp):
    prob = synth.c0_plain()
    rng = np.random.default_rng(706)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 24, prob.cost.K, sigma=0.3)
    W[3, 2, 1] = np.nan
    W[5, 0, 0] = np.inf
    W[11, 4, 0] = -np.inf  # slew only: x, y non-finite, z finite
    ref = _eval_modes(cp, prob, W, "non-finite")
    assert not np.isfinite(ref[0].view(np.float32)[[3, 5, 11]]).any()


def test_pairs_random_configs(cp):
    prob = synth.c1_full()
    rng = np.random.default_rng(707)
    Q = torch.from_numpy(synth.random_configs(rng, prob.robot, 2048)).cuda()
    res = {}
    for mode in (cp.PAIRS_ALL, cp.PAIRS_LANE, cp.PAIRS_WAVE):
        plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=1, pair_filter=mode)
        d, a = plan.debug_configs(Q)
        res[mode] = (_bits(d), _bits(a))
    for mode in (cp.PAIRS_LANE, cp.PAIRS_WAVE):
        np.testing.assert_array_equal(res[cp.PAIRS_ALL][0], res[mode][0])
        np.testing.assert_array_equal(res[cp.PAIRS_ALL][1], res[mode][1])


@pytest.mark.parametrize("scene", ["grid_only", "mixed"])
def test_pairs_sdf_scene(cp, scene):
    """A grid alone, and a grid together with trees, boxes and the ground:
    every mode but CP_PAIRS_ALL skips grid lookups by the block lower bounds
    (and culls the primitives), with bitwise the same results, forward with
    the tape and backward without it.  The grid is then changed in place and
    the results must follow it (the bounds are refreshed by every call)."""
    prob = synth.c4_sdf(n_points=100_000)
    spec = prob.sdf
    sdf = cp.sdf_build(torch.from_numpy(prob.lidar).cuda(), spec)
    rng = np.random.default_rng(708)
    if scene == "mixed":
        prob = dataclasses.replace(prob, scene=synth.c0_plain().scene)
    W = torch.from_numpy(synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 192, prob.cost.K,
                                                sigma=0.3)).cuda()
    gc = torch.linspace(0.5, 2.0, W.shape[0], device="cuda")
    plans = {}
    for mode in (cp.PAIRS_ALL, cp.PAIRS_LANE, cp.PAIRS_WAVE, cp.PAIRS_AUTO):
        plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=W.shape[0], sdf=sdf, sdf_spec=spec, pair_filter=mode)
        plan.set_endpoints(prob.q_start, prob.q_goal)
        plans[mode] = plan
    for step in ("built", "changed"):
        print(f"[pairs] sdf {scene} {step}", flush=True)
        out = {}
        for mode, plan in plans.items():
            out[mode] = [_bits(x) for x in plan.eval(W, tape=True)] + [_bits(plan.backward(W, gc, None))]
        for mode in (cp.PAIRS_LANE, cp.PAIRS_WAVE, cp.PAIRS_AUTO):
            for name, a, b in zip(("cost", "min_dist", "flags", "tape", "grad"), out[cp.PAIRS_ALL], out[mode]):
                np.testing.assert_array_equal(a, b, err_msg=f"sdf {scene} {step}: {name} differs in mode {mode}")
        if step == "built":
            before = out[cp.PAIRS_ALL][1].copy()
            sdf.sub_(0.25)  # every distance 25 cm smaller: bounds from the old grid would skip wrongly
            torch.cuda.synchronize()
    assert not np.array_equal(before, out[cp.PAIRS_ALL][1])


def test_pairs_batch(cp):
    probs = []
    for i in range(5):
        rng = np.random.default_rng(720 + i)
        robot = synth.make_robot(820 + i, 16 + 8 * i)
        qs, qg = synth.make_endpoints(rng, robot)
        scene = synth.make_scene(rng, robot, qs, qg, n_cyl=20 + 40 * i, n_box=i, half_extent=12.0)
        cost = synth.CostParams(K=4 + 2 * i, M=8 + 4 * i)
        B = 96 + 50 * i
        opt = synth.OptParams(B=B, nu=max(1, B // 10), sigma0=0.3, eps=1e-6, seed=900 + i, T=3)
        probs.append(synth.Problem(f"p{i}", robot, scene, qs, qg, cost, opt))
    states = {}
    for mode in (cp.PAIRS_LANE, cp.PAIRS_WAVE):
        b = cp.Batch(probs, pair_filter=mode)
        b.run(3)
        torch.cuda.synchronize()
        states[mode] = [b.get_state(i) for i in range(len(probs))]
        b.close()
    for sa, sb in zip(states[cp.PAIRS_LANE], states[cp.PAIRS_WAVE]):
        np.testing.assert_array_equal(sa["mu"], sb["mu"])
        np.testing.assert_array_equal(sa["C"], sb["C"])
        assert sa["best_cost"] == sb["best_cost"]
        np.testing.assert_array_equal(sa["best_W"], sb["best_W"])


def test_pair_filter_validated(cp):
    prob = synth.c0_plain()
    with pytest.raises(cp.CranePlanError):
        cp.Plan(prob.robot, prob.scene, prob.cost, max_B=1, pair_filter=4)


def _scene_variants():
    rng = np.random.default_rng(730)
    out = {}
    # several vertical extents: one cylinder group (and grid) per extent
    n = 200
    ext = np.array([[0.0, 15.0], [0.0, 4.0], [2.0, 9.0], [-1.0, 30.0], [5.0, 6.0]])[rng.integers(0, 5, n)]
    r = rng.uniform(2.0, 14.0, n)
    a = rng.uniform(-np.pi, np.pi, n)
    out["groups"] = np.stack([r * np.cos(a), r * np.sin(a), rng.uniform(0.1, 0.5, n), ext[:, 0], ext[:, 1]], 1)
    # every cylinder on one line (a grid of one row)
    xs = rng.uniform(-15, 15, 120)
    out["line"] = np.stack([xs, np.full(120, 4.0), rng.uniform(0.1, 0.4, 120), np.zeros(120), np.full(120, 15.0)], 1)
    # duplicated centres with different radii
    base = np.stack([rng.uniform(-12, 12, 40), rng.uniform(-12, 12, 40)], 1)
    dup = np.concatenate([base, base, base])
    out["duplicates"] = np.concatenate([dup, rng.uniform(0.1, 0.6, (120, 1)), np.zeros((120, 1)),
                                        np.full((120, 1), 15.0)], 1)
    # a single tree
    out["single"] = np.array([[3.0, 2.0, 0.3, 0.0, 15.0]])
    # a huge trunk around part of the sweep (centres inside it) among ordinary trees
    big = np.array([[6.0, 0.0, 4.0, 0.0, 15.0]])
    r = rng.uniform(3.0, 14.0, 80)
    a = rng.uniform(-np.pi, np.pi, 80)
    small = np.stack([r * np.cos(a), r * np.sin(a), rng.uniform(0.1, 0.4, 80), np.zeros(80), np.full(80, 15.0)], 1)
    out["huge"] = np.concatenate([big, small])
    # everything far away but one tree close to the base
    far = np.stack([rng.uniform(200, 260, 100), rng.uniform(-30, 30, 100), rng.uniform(0.1, 0.5, 100), np.zeros(100),
                    np.full(100, 15.0)], 1)
    out["far_and_one"] = np.concatenate([far, np.array([[2.5, -3.0, 0.4, 0.0, 15.0]])])
    return out


@pytest.mark.parametrize("name", ["groups", "line", "duplicates", "single", "huge", "far_and_one"])
def test_pairs_degenerate_scenes(cp, name):
    """Scenes that stress the cell and hint grids: several cylinder groups,
    one-row grids, duplicated centres, a single cylinder, centres inside a
    huge trunk, and nearly everything out of reach."""
    base = synth.c1_full()
    cyl = _scene_variants()[name].astype(np.float32)
    box = np.array([[4.0, -6.0, 1.0, 1.0, 1.0, 1.0]], np.float32) if name in ("groups", "huge") else \
        np.zeros((0, 6), np.float32)
    scene = synth.Scene(cyl=cyl, box=box, has_ground=1, ground_z=0.0)
    prob = dataclasses.replace(base, scene=scene, cost=synth.CostParams(K=6, M=12))
    rng = np.random.default_rng(731)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 96, prob.cost.K, sigma=0.4)
    _eval_modes(cp, prob, W, f"degenerate {name}")


@pytest.mark.parametrize("wl,n_big,n_small", [("c1", 512, (64, 200, 7)), ("c0", 2048, (256, 1000, 1)),
                                              ("ragged", 6000, (100, 333, 2000))])
def test_small_launch_split_matches_full_launch(cp, wl, n_big, n_small):
    """Launches of few waves share each wave's sphere groups out over 2, 4 or 8
    waves, and the adjoint of few paths runs 16 waves per path instead of 4; a
    path's cost, distance, flag, argmin record and gradient must not depend on
    that: the first n paths evaluated alone (split launches) equal the same
    paths inside a population large enough for the plain launches."""
    if wl == "c1":
        prob = synth.c1_full()
    elif wl == "c0":
        prob = synth.c0_plain()
    else:
        base = synth.c1_full()
        prob = dataclasses.replace(base, cost=synth.CostParams(K=5, M=7, hinge=synth.HINGE_SMOOTH, margin=0.1))
    rng = np.random.default_rng(720)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, n_big, prob.cost.K, sigma=0.3)
    Wt = torch.from_numpy(np.ascontiguousarray(W, dtype=np.float32)).cuda()
    gc = torch.linspace(0.5, 2.0, n_big, device="cuda")
    for mode in (cp.PAIRS_ALL, cp.PAIRS_LANE, cp.PAIRS_WAVE):
        plan = cp.Plan(prob.robot, prob.scene, prob.cost, max_B=n_big, pair_filter=mode)
        plan.set_endpoints(prob.q_start, prob.q_goal)
        cost, md, fl, tape = plan.eval(Wt, tape=True)
        big = [_bits(t) for t in (cost, md, fl, tape)]
        big += [_bits(plan.backward(Wt, gc, tape)), _bits(plan.backward(Wt, gc, None))]
        for n in n_small:
            print(f"[split] {wl} mode={mode} {n} of {n_big} paths", flush=True)
            Ws = Wt[:n].contiguous()
            cost, md, fl, tape = plan.eval(Ws, tape=True)
            small = [_bits(t) for t in (cost, md, fl, tape)]
            small += [_bits(plan.backward(Ws, gc[:n].contiguous(), tape)),
                      _bits(plan.backward(Ws, gc[:n].contiguous(), None))]
            for name, a, b in zip(("cost", "min_dist", "flags", "tape", "grad", "grad without tape"), big, small):
                np.testing.assert_array_equal(a[:n], b, err_msg=f"{wl} mode {mode} n={n}: {name}")


@pytest.mark.parametrize("counts", [(1, 5, 6, 7, 2, 3, 9), (0, 4, 0, 13, 1, 0, 8), (3, 3, 3, 3, 3, 3, 3)])
def test_pairs_sphere_group_sizes(cp, counts):
    """Frames holding 0 to 13 spheres, so that sphere groups of every size
    from 1 to 4 and frames without spheres occur: the crane of c1_full with
    its spheres reassigned to frames in the given counts."""
    base = synth.c1_full()
    rb = base.robot
    S = sum(counts)
    frame = np.repeat(np.arange(len(counts)), counts).astype(np.int32)
    robot = dataclasses.replace(rb, sphere_frame=frame, sphere_center=rb.sphere_center[:S].copy(),
                                sphere_radius=rb.sphere_radius[:S].copy())
    cost = synth.CostParams(K=6, M=12, hinge=synth.HINGE_SMOOTH, margin=0.1)
    prob = dataclasses.replace(base, robot=robot, cost=cost)
    rng = np.random.default_rng(740 + S)
    W = synth.random_waypoints(rng, prob.robot, prob.q_start, prob.q_goal, 80, cost.K, sigma=0.4)
    _eval_modes(cp, prob, W, f"sphere counts {counts}", backward=True)


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
def test_pairs_random_scenes(cp, seed):
    """Random cranes and scenes (tree counts and radii, several tree heights,
    box counts and sizes, scene extents, perturbation widths): the culling
    with its group skip and lead frame equals the every-pair evaluation bit
    for bit, forward with the tape and backward without it."""
    rng = np.random.default_rng(760 + seed)
    robot = synth.make_robot(7000 + seed, int(rng.integers(8, 72)))
    qs, qg = synth.make_endpoints(rng, robot)
    scene = synth.make_scene(rng, robot, qs, qg, n_cyl=int(rng.integers(48, 900)), n_box=int(rng.integers(0, 40)),
                             half_extent=float(rng.uniform(6.0, 30.0)),
                             r_range=(0.05, float(rng.uniform(0.2, 1.5))), height=float(rng.uniform(2.0, 20.0)),
                             box_side=(0.3, float(rng.uniform(1.0, 8.0))))
    if seed % 2:
        # a second tree height: two cylinder groups
        cyl = scene.cyl.copy()
        cyl[::3, 4] = cyl[::3, 3] + 4.0
        scene = dataclasses.replace(scene, cyl=cyl)
    cost = synth.CostParams(K=int(rng.integers(3, 10)), M=int(rng.integers(5, 20)), hinge=synth.HINGE_SMOOTH,
                            margin=0.1)
    prob = synth.Problem("random", robot, scene, qs, qg, cost, synth.c1_full().opt)
    W = synth.random_waypoints(rng, robot, qs, qg, int(rng.integers(40, 300)), cost.K,
                               sigma=float(rng.uniform(0.05, 0.8)))
    _eval_modes(cp, prob, W, f"random scene {seed}", backward=True)
