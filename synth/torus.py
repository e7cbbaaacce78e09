"""Noisy points on a torus in R^3 (the small plain-method workload).

Area-uniform sampling: the toroidal angle phi is uniform on [0, 2 pi); the
poloidal angle theta is drawn by rejection with acceptance probability
(R + r cos theta) / (R + r), which makes the density proportional to the
surface element.  Each coordinate then gets iid N(0, noise^2) noise.  Draw
order from numpy.random.default_rng(seed): batches of (theta, accept-uniform)
pairs until n are accepted, then the n phi values, then the 3n noise values.
"""
import numpy as np


def torus_points(n, R=2.0, r=1.0, noise=0.01, seed=0):
    rng = np.random.default_rng(seed)
    thetas = []
    have = 0
    while have < n:
        m = max(2 * (n - have), 16)
        th = rng.uniform(0.0, 2.0 * np.pi, size=m)
        acc = rng.uniform(0.0, 1.0, size=m) < (R + r * np.cos(th)) / (R + r)
        th = th[acc][: n - have]
        thetas.append(th)
        have += th.size
    theta = np.concatenate(thetas)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n)
    x = np.stack(
        [(R + r * np.cos(theta)) * np.cos(phi), (R + r * np.cos(theta)) * np.sin(phi), r * np.sin(theta)],
        axis=1,
    )
    x = x + noise * rng.standard_normal(size=(n, 3))
    return x.astype(np.float32)
