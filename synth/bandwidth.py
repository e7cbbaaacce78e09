"""Median-heuristic kernel bandwidth.

eps = median of the squared pairwise distances |x_i - x_j|^2 over all pairs
i < j of a subsample of `m` rows drawn without replacement by
numpy.random.default_rng(seed).choice(N, m, replace=False).  With an even
number of pairs the median is the mean of the two middle values.  Computed in
float64 from the stored (float32) coordinates.
"""
import numpy as np


def median_sq_distance(X, m=500, seed=0):
    X = np.asarray(X)
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    idx = rng.choice(n, min(m, n), replace=False)
    S = X[idx].astype(np.float64)
    iu, ju = np.triu_indices(S.shape[0], k=1)
    d2 = ((S[iu] - S[ju]) ** 2).sum(axis=1)
    return float(np.median(d2))
