"""Accelerated randomly pivoted partial Cholesky (oracle; test infrastructure only).

Follows the paper's Appendix "Randomly pivoted Cholesky": Algorithm 2 (ARPC)
and Algorithm 3 (its accept/reject check), with zero-based indexing.  The
kernel matrix is never formed: only the columns of accepted pivots and the
b x b proposal blocks are evaluated.

Readings of points the paper leaves open (each also listed in the design
notes):

* Sampling distribution.  Algorithm 2 samples "from d/sum(d)"; the text of the
  same appendix defines the law as rho/sum(rho), rho the residual diagonal.
  We sample from rho.
* Exact, order-independent sampling.  rho is quantised to integers
  rho_q = floor(rho * 2^40) (rho lies in [0, 1] for the Gaussian kernel, whose
  diagonal is 1).  With T = sum rho_q and m the 53-bit integer of the uniform
  u (u = m 2^-53), the pivot is the smallest j whose inclusive prefix sum
  C_j exceeds floor(m T / 2^53).  The deviation from rho/sum(rho) is at most
  2^-40 per entry, and any implementation that sums integers gets the same
  pivot.
* Uniform stream layout.  Round i reads u[2 b i + j] for proposal j and
  u[2 b i + b + j] for the accept test of proposal j (both always consumed).
* t = ceil(r / b) rounds; the last one proposes r - (t - 1) b pivots.
* Algorithm 3 compares z * rho_loc(i) with the current (updated) H(i, i),
  rho_loc = diag(H) at block start, with strict "<"; a proposal equal to an
  earlier accepted proposal of the same block is rejected (in exact arithmetic
  its updated H(i, i) is 0); a proposal whose updated H(i, i) <= tau is
  rejected.
* After each round rho[S_i] is set to 0 exactly (true in exact arithmetic).
* Greedy mode (the deterministic extreme named in the same appendix) needs
  b = 1 and takes the argmax of rho, lowest index on ties.
* The run stops early when the quantised total is 0; unused columns of F are
  zero and are dropped (F has k <= r columns).
* Replay mode feeds a given ordered pivot list, all accepted, so runs that
  differ only in arithmetic precision can be compared with identical pivots.
"""
import math

import numpy as np

from .kernel import gaussian_kernel

QBITS = 40
QSCALE = float(2 ** QBITS)


def quantize_rho(rho):
    """rho_q = floor(max(rho, 0) * 2^40) as Python-exact int64 values."""
    r = np.maximum(np.asarray(rho, dtype=np.float64), 0.0)
    return np.floor(r * QSCALE).astype(np.int64)


def inverse_cdf_pivot(rho_q, u):
    """Smallest j with C_j > floor(m * T / 2^53), m = u * 2^53 (exact integers).

    Returns -1 when T = 0.
    """
    rho_q = [int(v) for v in rho_q]
    T = sum(rho_q)
    if T == 0:
        return -1
    m = int(round(float(u) * (2.0 ** 53)))
    if not (0 <= m < 2 ** 53) or m != float(u) * (2.0 ** 53):
        raise ValueError("uniform must be a multiple of 2^-53 in [0, 1)")
    target = (m * T) >> 53
    c = 0
    for j, v in enumerate(rho_q):
        c += v
        if c > target:
            return j
    raise AssertionError("unreachable: target < T")


def greedy_pivot(rho):
    """argmax rho, lowest index among ties (the first maximum)."""
    rho = np.asarray(rho, dtype=np.float64)
    best = 0
    for j in range(1, rho.size):
        if rho[j] > rho[best]:
            best = j
    return best


def accept_reject(H, z, proposals, tau=0.0, force_accept=False):
    """Algorithm 3: accept/reject check with in-block pivoted Cholesky.

    H: b x b proposal block (residual kernel on the proposals), z: b uniforms,
    proposals: the b proposed indices (used only to reject repeats of an
    already accepted index).  Returns (T, L) with T the accepted positions in
    proposal order and L = L(T, T) the |T| x |T| lower Cholesky factor.
    With force_accept every proposal is taken (replay); a pivot <= tau then
    raises FloatingPointError (breakdown).
    """
    H = np.array(H, dtype=np.float64, copy=True)
    b = H.shape[0]
    rho_loc = np.diag(H).copy()
    L = np.zeros((b, b))
    T = []
    for i in range(b):
        if not force_accept and any(proposals[j] == proposals[i] for j in T):
            continue
        hii = H[i, i]
        if force_accept:
            if not hii > tau:
                raise FloatingPointError("replayed pivot block is not positive definite")
            ok = True
        else:
            ok = hii > tau and z[i] * rho_loc[i] < hii
        if ok:
            T.append(i)
            L[i:, i] = H[i:, i] / math.sqrt(hii)
            H[i + 1:, i + 1:] -= np.outer(L[i + 1:, i], L[i + 1:, i])
    T = np.array(T, dtype=np.int64)
    return T, L[np.ix_(T, T)]


def arpc(X, eps, r, b, mode="sampled", uniforms=None, tau=0.0, replay=None, return_trace=False):
    """Algorithm 2 (ARPC) on the Gaussian kernel of the rows of X.

    Returns dict with F (N x k, float64), S (k pivots, in acceptance order),
    rho (final residual diagonal), k, and per round the accepted counts and
    trace errors sum(rho)/N.
    """
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    if mode not in ("sampled", "greedy", "replay"):
        raise ValueError(mode)
    if r < 1 or r > N or b < 1 or not eps > 0:
        raise ValueError("invalid arguments")
    if mode == "greedy" and b != 1:
        raise ValueError("greedy pivoting needs b = 1")
    t = -(-r // b)
    if mode == "sampled":
        uniforms = np.asarray(uniforms, dtype=np.float64)
        if uniforms.size < 2 * b * t:
            raise ValueError("need 2*b*ceil(r/b) uniforms")
    if mode == "replay":
        replay = np.asarray(replay, dtype=np.int64)
        t = -(-replay.size // b)

    F = np.zeros((N, r))
    rho = np.ones(N)  # diag K = k(x, x) = 1 for the Gaussian kernel
    S = []
    k = 0
    accepted, trace = [], []
    for i in range(t):
        bi = min(b, r - i * b) if mode != "replay" else min(b, replay.size - i * b)
        if mode == "sampled":
            rho_q = quantize_rho(rho)
            if int(rho_q.sum()) == 0:
                break
            prop = [inverse_cdf_pivot(rho_q, uniforms[2 * b * i + j]) for j in range(bi)]
            z = [uniforms[2 * b * i + b + j] for j in range(bi)]
        elif mode == "greedy":
            if not np.max(rho) > 0:
                break
            prop = [greedy_pivot(rho)]
            z = [0.0]
        else:
            prop = list(replay[i * b:i * b + bi])
            z = [0.0] * bi
        prop = np.array(prop, dtype=np.int64)
        # H = K(S', S') - F(S', :) F(S', :)^T
        H = gaussian_kernel(X[prop], X[prop], eps) - F[prop, :k] @ F[prop, :k].T
        T, L = accept_reject(H, z, prop, tau=tau, force_accept=(mode == "replay"))
        Si = prop[T]
        if Si.size:
            # G = (K(:, S_i) - F F(S_i, :)^T) L^{-T}, as a solve with L
            R = gaussian_kernel(X, X[Si], eps) - F[:, :k] @ F[Si, :k].T
            G = np.linalg.solve(L, R.T).T
            F[:, k:k + Si.size] = G
            k += Si.size
            S.extend(int(s) for s in Si)
            rho = rho - np.sum(G * G, axis=1)
            rho = np.maximum(rho, 0.0)
            rho[Si] = 0.0
        accepted.append(int(Si.size))
        trace.append(float(rho.sum() / N))
    out = {
        "F": F[:, :k].copy(),
        "S": np.array(S, dtype=np.int64),
        "rho": rho,
        "k": k,
        "accepted": accepted,
        "trace_err": trace,
    }
    return out
