"""Seeded step-two problems shared by the oracle's and the device's tests
(input generation only)."""
import numpy as np

from paper_2503_14160_amd import synth


def problems(robot, P, N, seed):
    """P start/goal pairs (hanging configurations, slew, boom and telescope
    moves) and bent paths between them: the straight line plus a smooth bump
    of 0.1 rad on the boom, as a step-one path bends over an obstacle.
    float32 [P, n], [P, n], [P, N+1, n]."""
    rng = np.random.default_rng(seed)
    q0 = synth.hanging_configs(rng, robot, P).astype(np.float64)
    qg = q0.copy()
    qg[:, 0] += rng.uniform(-0.8, 0.8, P)
    qg[:, 1] += rng.uniform(-0.15, 0.15, P)
    qg[:, 3] = np.clip(qg[:, 3] + rng.uniform(-0.5, 0.5, P), 0.1, 2.9)
    qg[:, 5] = qg[:, 1] + qg[:, 2]
    s = np.linspace(0.0, 1.0, N + 1)
    qstar = q0[:, None, :] + s[None, :, None] * (qg - q0)[:, None, :]
    qstar[:, :, 1] += 0.1 * np.sin(np.pi * s)[None, :]
    return q0.astype(np.float32), qg.astype(np.float32), qstar.astype(np.float32)
