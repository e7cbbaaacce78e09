"""Many small problems for the batched form.

Sixty-four datasets, each the KS delay embedding of its own trajectory (KS
seed s = 1..64): N_s log-uniform on [5e3, 2e5], (d_s, q_s) uniform over
{(32, 1), (128, 2), (512, 8)} (the leading d_s coordinates of the q_s-delay
embedding), rank budget r_s uniform over {64, 128, 256, 512}; drawn from
numpy.random.default_rng(seed) in the order N, (d, q), r per dataset.  Each
dataset is decomposed at eight bandwidths m * median, m in
BANDWIDTH_MULTIPLIERS, giving 512 jobs.
"""
import numpy as np

from .bandwidth import median_sq_distance
from .ks import ks_points

BANDWIDTH_MULTIPLIERS = (0.25, 0.5, 1.0, 2.0, 4.0, 8.0, 16.0, 32.0)
DIMS = ((32, 1), (128, 2), (512, 8))
RANKS = (64, 128, 256, 512)


def batch_specs(n_datasets=64, seed=0, n_min=5e3, n_max=2e5):
    rng = np.random.default_rng(seed)
    specs = []
    for s in range(1, n_datasets + 1):
        N = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        d, q = DIMS[int(rng.integers(len(DIMS)))]
        r = RANKS[int(rng.integers(len(RANKS)))]
        specs.append({"seed": s, "N": N, "d": d, "q": q, "r": r})
    return specs


def batch_points(spec):
    """float32 N x d points of one dataset and its median-heuristic bandwidth."""
    X = ks_points(spec["N"], q=spec["q"], seed=spec["seed"], d=spec["d"])
    return X, median_sq_distance(X, seed=spec["seed"])
