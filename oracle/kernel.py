"""Gaussian kernel evaluated directly (oracle; test infrastructure only).

Kernel: k(x, y) = exp(-|x - y|^2 / eps) (the Gaussian kernel of the
Application section, eq. data-kernel, with its eps*J written as one bandwidth
eps).  It satisfies Assumption 1 (continuous, bounded, PSD, positive) and
k(x, x) = 1.

Squared distances are formed as sum_j (x_j - y_j)^2, never through the
|x|^2 + |y|^2 - 2<x, y> expansion, so the oracle does not share the GPU's
arithmetic.
"""
import numpy as np


def sq_distances(A, B, max_elems=1 << 24):
    """D[i, j] = sum_l (A[i, l] - B[j, l])^2 in float64, formed entry by entry.

    Rows of A are processed in blocks so the difference tensor stays small.
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    D = np.empty((A.shape[0], B.shape[0]), dtype=np.float64)
    per_row = max(1, B.shape[0] * max(1, A.shape[1]))
    rb = max(1, max_elems // per_row)
    for i0 in range(0, A.shape[0], rb):
        diff = A[i0:i0 + rb, None, :] - B[None, :, :]
        D[i0:i0 + rb] = np.einsum("ijk,ijk->ij", diff, diff)
    return D


def gaussian_kernel(A, B, eps):
    """K[i, j] = exp(-|A_i - B_j|^2 / eps)."""
    return np.exp(-sq_distances(A, B) / eps)
