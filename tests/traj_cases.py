"""Seeded step-two problems shared by the oracle's and the device's tests
(input generation only)."""
from paper_2503_14160_amd import synth


def problems(robot, P, N, seed):
    return synth.traj_problems(robot, P, N, seed)
