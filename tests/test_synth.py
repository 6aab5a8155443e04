"""The seeded workloads are well formed: shapes, sizes and start/goal poses
clear of every obstacle (checked with the oracle's distances)."""
import numpy as np
import pytest

from paper_2503_14160_amd import synth


def test_robot_layout():
    for S in (24, 64):
        rb = synth.make_robot(1000, S)
        assert rb.n_joints == 6 and rb.n_spheres == S and rb.n_active == 4
        counts = np.bincount(rb.sphere_frame, minlength=7)
        assert counts[[1, 2, 3, 4, 6]].min() >= 1 and counts[0] == 0 and counts[5] == 0
        assert np.all((rb.sphere_radius >= 0.15) & (rb.sphere_radius <= 0.4))
        assert np.all((rb.link_lengths >= 2) & (rb.link_lengths <= 5))


@pytest.mark.parametrize("name", ["c0_plain", "c1_full", "c2_diff"])
def test_workload_endpoints_clear(orc, name):
    p = synth.WORKLOADS[name]()
    assert p.q_start.shape == (6,) and p.q_goal.shape == (6,)
    assert abs(float(p.q_goal[0] - p.q_start[0])) >= np.pi / 2 - 1e-6
    m = orc.Model(p.robot, p.scene, p.cost)
    d, _, _, _ = orc.eval_configs(m, np.stack([p.q_start, p.q_goal]).astype(np.float64))
    assert np.all(d > 0.0), d
    _, _, tip = orc.fk(m, p.q_start)
    assert tip[2] >= 0.5


def test_sizes():
    p0 = synth.c0_plain()
    assert (p0.opt.B, p0.cost.K, p0.cost.M, p0.cost.n_s, p0.robot.n_spheres, p0.scene.n_cyl) == (256, 8, 16, 176, 24, 32)
    p1 = synth.c1_full()
    assert (p1.opt.B, p1.cost.K, p1.cost.M, p1.cost.n_s, p1.robot.n_spheres, p1.scene.n_cyl, p1.scene.n_box,
            p1.opt.nu) == (16384, 16, 32, 608, 64, 512, 16, 819)


def test_batch_problems_clear(orc):
    probs = synth.c3_batch(24)
    for p in probs:
        assert 512 <= p.opt.B <= 8192 and 8 <= p.cost.K <= 24
        assert 64 <= p.scene.n_cyl + p.scene.n_box <= 1024
        m = orc.Model(p.robot, p.scene, p.cost)
        d, _, _, _ = orc.eval_configs(m, np.stack([p.q_start, p.q_goal]).astype(np.float64))
        assert np.all(d > 0.0), (p.name, d)


@pytest.mark.parametrize("name", ["c0_plain", "c1_full", "c2_diff"])
def test_workload_endpoints_clear_of_self_collision(orc, name):
    """The crane's non-adjacent link pairs (self-collision) are clear at every
    workload's start and goal."""
    p = synth.WORKLOADS[name]()
    rb = synth.with_self_collision(p.robot)
    empty = synth.Scene(cyl=np.zeros((0, 5), np.float32), box=np.zeros((0, 6), np.float32), has_ground=0)
    m = orc.Model(rb, empty, p.cost)
    d, _, o, _ = orc.eval_configs(m, np.stack([p.q_start, p.q_goal]).astype(np.float64))
    assert np.all(d > 0.0), d
    assert np.all(o >= 0xFF00)


def test_ik_workload_layout():
    p = synth.ik_c1(n_targets=32, restarts=4, oversample=3)
    n = p.robot.n_joints
    assert p.q_star.shape == (96, n) and p.q_init.shape == (96 * 4, n)
    assert p.q_star.dtype == np.float32 and p.q_init.dtype == np.float32
    lo, hi = p.robot.q_min, p.robot.q_max
    assert np.all(p.q_init >= lo) and np.all(p.q_init <= hi)
    assert np.all(p.q_star >= lo) and np.all(p.q_star <= hi)
    # the first start of every target is the crane's start configuration
    np.testing.assert_array_equal(p.q_init.reshape(96, 4, n)[:, 0], np.broadcast_to(p.q_ref, (96, n)))
    assert len(p.robot.self_pairs) > 0
    # picking keeps the first n_targets marked candidates with their own starts
    mask = np.zeros(96, bool)
    mask[1::2] = True
    q = p.pick(mask)
    assert q.q_star.shape == (32, n) and q.q_init.shape == (128, n)
    np.testing.assert_array_equal(q.q_star, p.q_star[1:64:2])
    np.testing.assert_array_equal(q.q_init.reshape(32, 4, n), p.q_init.reshape(96, 4, n)[1:64:2])
    with pytest.raises(ValueError):
        p.pick(np.zeros(96, bool))
