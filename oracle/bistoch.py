"""Approximate EVD of the bistochastic kernel from a partial Cholesky factor
(oracle; test infrastructure only).

Follows the paper's Section "Bistochastic normalization" (the factored form
P~ = B C B^T with B = D~^{-1} F and C = F^T Q~^{-1} F) and Algorithm 1, with
the general QR-then-small-EVD route of the opening of the "Normalized kernel
approximation" section.  The Nystrom extension uses the extension formula of
the "Nystrom method connection" section applied to P~.

Readings of points the paper leaves open:

* QR: the paper suggests CGS2 or CholQR2; the oracle uses Householder QR
  (numpy.linalg.qr).  The sign convention of R cancels in U = Q V.
* gamma: the optional regulariser of the QR step is added to the entries
  (i, i), i < k, of the N x k matrix D~^{-1} F (default 0).
* Eigenvalues are sorted in decreasing order; each eigenvector column gets
  the sign that makes its largest-magnitude entry (lowest index on ties)
  positive.
* The optional constant leading eigenvector is followed by a QR with a
  positive diagonal in R.
* Extension matrix: E = C R^T V Lambda^{-1} (k x nev).  With
  f(y) = F(S, :)^{-1} k(X_S, y) the extended eigenvector values are
  (f(y)^T E) / (c^T f(y)), c = F^T 1; at a training point they reproduce the
  row of U.
"""
import numpy as np
import scipy.linalg as sla

from .kernel import gaussian_kernel


class DegreeError(ArithmeticError):
    """An assert of Algorithm 1 (diag(D~) > 0 or diag(Q~) > 0) failed."""


def bistoch_degrees(F):
    """Algorithm 1 normalisation vectors from F alone.

    c = F^T 1, d~ = F c = diag(F F^T 1), w = F^T (1 / d~), q~ = F w
    = diag(F F^T D~^{-1} 1).  Raises DegreeError when a degree is not > 0.
    """
    F = np.asarray(F, dtype=np.float64)
    N = F.shape[0]
    c = F.T @ np.ones(N)
    d = F @ c
    if not np.all(d > 0):
        raise DegreeError("diag(D~) > 0 failed")
    w = F.T @ (1.0 / d)
    q = F @ w
    if not np.all(q > 0):
        raise DegreeError("diag(Q~) > 0 failed")
    return c, d, q


def sign_normalize(U):
    """Flip each column so its largest-|entry| (first on ties) is positive."""
    U = np.array(U, dtype=np.float64, copy=True)
    for j in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, j])))
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
    return U


def bistoch_eig(F, nev, gamma=0.0, fix_const=False):
    """Algorithm 1 after the factorisation: top-nev eigenpairs of P~.

    Returns dict with U (N x nev), lam (nev, decreasing), c, d, q, C, GB
    (= B^T B), R1, M (= R1 C R1^T), lam_all (all k eigenvalues) and E.
    """
    F = np.asarray(F, dtype=np.float64)
    N, k = F.shape
    if not 1 <= nev <= k:
        raise ValueError("need 1 <= nev <= k")
    c, d, q = bistoch_degrees(F)
    B = F / d[:, None]
    if gamma:
        idx = np.arange(min(N, k))
        B[idx, idx] += gamma
    Q1, R1 = np.linalg.qr(B, mode="reduced")
    C = F.T @ (F / q[:, None])
    M = R1 @ C @ R1.T
    M = 0.5 * (M + M.T)
    lam, V = np.linalg.eigh(M)
    lam = lam[::-1]
    V = V[:, ::-1]
    U = Q1 @ V[:, :nev]
    if fix_const:
        U[:, 0] = 1.0 / np.sqrt(N)
        U, Rq = np.linalg.qr(U, mode="reduced")
        U = U * np.sign(np.diag(Rq))[None, :]
    U = sign_normalize(U)
    # Extension matrix with the same column signs as U: V's columns are
    # matched to U through U = Q1 V.
    Vn = V[:, :nev]
    if not fix_const:
        sgn = np.sign(np.sum(U * (Q1 @ Vn), axis=0))
        Vn = Vn * sgn[None, :]
    E = C @ R1.T @ Vn / lam[None, :nev]
    return {
        "U": U,
        "lam": lam[:nev].copy(),
        "lam_all": lam.copy(),
        "c": c,
        "d": d,
        "q": q,
        "C": C,
        "GB": B.T @ B,
        "R1": R1,
        "M": M,
        "E": E,
    }


def nystrom_extend(Y, X, S, F, c, E, eps):
    """Extended eigenvector values at new points Y (rows).

    f(y) = F(S, :)^{-1} k(X_S, y) (F(S, :) is lower triangular in pivot
    order), value = (f(y)^T E) / (c^T f(y)).
    """
    S = np.asarray(S, dtype=np.int64)
    Kys = gaussian_kernel(X[S], Y, eps)  # k x M
    f = sla.solve_triangular(np.asarray(F, dtype=np.float64)[S, :], Kys, lower=True)
    num = f.T @ E
    den = f.T @ c
    return num / den[:, None]


def dense_bistochastic(K):
    """P = D^{-1} K Q^{-1} K D^{-1} with D = diag(K 1), Q = diag(K D^{-1} 1)
    (eq. bistoch-kernel, discrete form), formed densely for brute-force checks.
    Returns (P, d, q)."""
    K = np.asarray(K, dtype=np.float64)
    one = np.ones(K.shape[0])
    d = K @ one
    q = K @ (one / d)
    P = (K / d[:, None] / q[None, :]) @ (K / d[None, :])
    return P, d, q


def dense_symmetric(K):
    """L = D^{-1/2} K D^{-1/2}, D = diag(K 1) (Section on the symmetric
    normalisation), formed densely.  Returns (L, d)."""
    K = np.asarray(K, dtype=np.float64)
    d = K @ np.ones(K.shape[0])
    s = 1.0 / np.sqrt(d)
    return K * s[:, None] * s[None, :], d


def symmetric_eig(F, nev):
    """Symmetric normalisation route (Section "Symmetric normalization"):
    L~ = (D~^{-1/2} F)(D~^{-1/2} F)^T, EVD via QR of B = D~^{-1/2} F and EVD of
    R R^T (the general route with C = I).  E = R^T V Lambda^{-1} (k x nev,
    signed like U) is the extension matrix: from L~ U = U Lambda and
    B^T U = R^T V, U = B E, so a new point y with f(y) = F(S, :)^{-1} k(X_S, y)
    and d~(y) = c^T f(y) gets the values f(y)^T E / sqrt(d~(y))."""
    F = np.asarray(F, dtype=np.float64)
    c = F.T @ np.ones(F.shape[0])
    d = F @ c
    if not np.all(d > 0):
        raise DegreeError("diag(D~) > 0 failed")
    B = F / np.sqrt(d)[:, None]
    Q, R = np.linalg.qr(B, mode="reduced")
    lam, V = np.linalg.eigh(R @ R.T)
    lam, V = lam[::-1], V[:, ::-1]
    U = sign_normalize(Q @ V[:, :nev])
    Vn = V[:, :nev] * np.sign(np.sum(U * (Q @ V[:, :nev]), axis=0))[None, :]
    E = R.T @ Vn / lam[None, :nev]
    return {"U": U, "lam": lam[:nev].copy(), "lam_all": lam.copy(), "d": d, "c": c, "E": E}


def symmetric_extend(Y, X, S, F, c, E, eps):
    """Extension of the eigenvectors of L~ to new points Y (rows):
    f(y) = F(S, :)^{-1} k(X_S, y), value = (f(y)^T E) / sqrt(c^T f(y))."""
    S = np.asarray(S, dtype=np.int64)
    Kys = gaussian_kernel(X[S], Y, eps)
    f = sla.solve_triangular(np.asarray(F, dtype=np.float64)[S, :], Kys, lower=True)
    return (f.T @ E) / np.sqrt(f.T @ c)[:, None]


def gaussian_dense(X, eps):
    """Full kernel matrix (brute force only)."""
    return gaussian_kernel(X, X, eps)
