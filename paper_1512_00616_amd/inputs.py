"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds no arithmetic of the method: only problem sizes, nominal parameters and
seeded random draws (numpy PCG64).  Both the HIP path and the CPU oracle
receive the same arrays from here.
"""
import math

import numpy as np

# nominal kinematics: h0 = 0.25, theta0 = 10 deg (in radians), phi = pi/2
MU_NOMINAL = (0.25, math.radians(10.0), math.pi / 2)

# discretisations of the workloads: O-grid Nr x Nth, degree p, steps per period
WORKLOADS = {
    # 8x24 O-grid, p=1, 20 steps: free stream + N(0, 1e-3), seed 1
    "circle-8x24-p1-nt20": dict(Nr=8, Nth=24, p=1, Nt=20),
    # 32x96 O-grid, p=3 (40x40 blocks), 100 steps, free-stream start
    "circle-32x96-p3-nt100": dict(Nr=32, Nth=96, p=3, Nt=100),
    # 16x48, p=2, 60 steps (batched instances)
    "circle-16x48-p2-nt60": dict(Nr=16, Nth=48, p=2, Nt=60),
    # 64x192, p=3, 200 steps
    "circle-64x192-p3-nt200": dict(Nr=64, Nth=192, p=3, Nt=200),
}

PHYSICS = dict(mach=0.2, re=1000.0, gamma=1.4, pr=0.72, T=1.0)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def perturbation(n, seed=1, sigma=1e-3):
    """iid N(0, sigma^2) on every entry of a state vector of length n."""
    return sigma * rng(seed).standard_normal(n)


def random_vectors(n, k=2, seed=7):
    """k independent standard-normal vectors of length n (dot-product tests)."""
    g = rng(seed)
    return [g.standard_normal(n) for _ in range(k)]


def warmstart_params(count, seed):
    """Kinematics for the learned warm start: training draws (seed 5) and
    held-out draws (seed 55), same ranges as batch_params."""
    return batch_params(count, seed=seed)


def batch_params(count, seed=4):
    """(h0, theta0 [rad], phi) with h0 ~ U[0.1, 0.5], theta0 ~ U[0, 30 deg], phi ~ U[0, pi]."""
    g = rng(seed)
    h0 = g.uniform(0.1, 0.5, count)
    th = np.radians(g.uniform(0.0, 30.0, count))
    ph = g.uniform(0.0, math.pi, count)
    return np.stack([h0, th, ph], axis=1)
