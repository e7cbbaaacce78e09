"""Pins of the float64 CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine computing the same object by another route (LAPACK's pivoted
Cholesky, a dense eigendecomposition), a closed form (the Nystrom identity),
an invariant (row sums of the bistochastic matrix), an exact probability law
(enumerated), or an inequality the paper proves.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.spatial.distance import cdist
from scipy.stats import chi2

import oracle
from oracle.arpc import accept_reject, arpc, inverse_cdf_pivot, quantize_rho
from oracle.bistoch import (
    DegreeError,
    bistoch_degrees,
    bistoch_eig,
    dense_bistochastic,
    dense_symmetric,
    nystrom_extend,
    symmetric_eig,
)
from oracle.kernel import gaussian_kernel
from synth import median_sq_distance, torus_points, uniform_stream


def _torus(n, seed=0):
    X = torus_points(n, seed=seed)
    return X, median_sq_distance(X, seed=seed)


def _angles(U, V):
    """Largest principal angle between the column spans of U and V."""
    Qu, _ = np.linalg.qr(U)
    Qv, _ = np.linalg.qr(V)
    s = np.linalg.norm(Qv - Qu @ (Qu.T @ Qv), 2)  # sine of the largest angle
    return float(np.arcsin(min(s, 1.0)))


# ---------------------------------------------------------------- kernel


def test_kernel_matches_library_distance():
    rng = np.random.default_rng(1)
    A, B = rng.standard_normal((37, 5)), rng.standard_normal((11, 5))
    K = gaussian_kernel(A, B, 3.0)
    ref = np.exp(-cdist(A, B, "sqeuclidean") / 3.0)
    assert np.max(np.abs(K - ref)) < 1e-14
    # a value by hand: |(1,2) - (0,0)|^2 = 5
    assert abs(gaussian_kernel([[1.0, 2.0]], [[0.0, 0.0]], 2.0)[0, 0] - math.exp(-2.5)) < 1e-16
    Kxx = gaussian_kernel(A, A, 3.0)
    assert np.all(np.diag(Kxx) == 1.0) and np.allclose(Kxx, Kxx.T)


# ---------------------------------------------------------- pivot sampling


def test_inverse_cdf_hand_cases():
    rho = np.array([0.0, 0.5, 0.0, 0.5])
    q = quantize_rho(rho)
    assert inverse_cdf_pivot(q, 0.0) == 1
    assert inverse_cdf_pivot(q, 0.5 - 2.0 ** -53) == 1
    assert inverse_cdf_pivot(q, 0.5) == 3
    assert inverse_cdf_pivot(q, 1.0 - 2.0 ** -53) == 3
    assert inverse_cdf_pivot(quantize_rho(np.zeros(5)), 0.3) == -1
    # negative residuals (round-off) count as zero
    assert inverse_cdf_pivot(quantize_rho([-1e-17, 1e-3]), 0.0) == 1


def test_inverse_cdf_exact_law():
    """Exact enumeration: the number of 53-bit m that select j equals
    ceil(C_j 2^53 / T) - ceil(C_{j-1} 2^53 / T), so P(j) = rho_q[j]/T up to 2^-53."""
    rng = np.random.default_rng(2)
    rho = rng.uniform(0, 1, 9)
    rho[3] = 0.0
    q = [int(v) for v in quantize_rho(rho)]
    T = sum(q)
    C = np.cumsum(q).tolist()
    lo = 0
    for j in range(len(q)):
        hi = -(-C[j] * 2 ** 53 // T)
        count = hi - lo
        assert abs(count / 2 ** 53 - q[j] / T) <= 2.0 ** -52
        if count > 0:  # first and last m of the range select j
            assert inverse_cdf_pivot(q, lo * 2.0 ** -53) == j
            assert inverse_cdf_pivot(q, (hi - 1) * 2.0 ** -53) == j
        lo = hi
    # quantisation error vs the real-valued law
    assert np.max(np.abs(np.array(q) / T - rho / rho.sum())) < 1e-11


def test_inverse_cdf_frequencies():
    rho = np.array([0.1, 0.0, 0.25, 0.05, 0.6])
    q = quantize_rho(rho)
    u = uniform_stream(20000, seed=7)
    counts = np.bincount([inverse_cdf_pivot(q, x) for x in u], minlength=5)
    assert counts[1] == 0
    p = rho / rho.sum()
    nz = p > 0
    stat = np.sum((counts[nz] - 20000 * p[nz]) ** 2 / (20000 * p[nz]))
    assert stat < chi2.ppf(0.999, nz.sum() - 1)


# ------------------------------------------------------- Algorithm 3 alone


def test_accept_reject_full_accept_is_cholesky():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6, 6))
    H = A @ A.T + 6 * np.eye(6)
    T, L = accept_reject(H, np.zeros(6), np.arange(6))
    assert list(T) == list(range(6))
    assert np.allclose(L, np.linalg.cholesky(H), atol=1e-13)


def test_accept_reject_rejects_duplicates_and_tiny_pivots():
    X = np.array([[0.0], [1.0], [0.0]])
    H = gaussian_kernel(X, X, 1.0)
    T, L = accept_reject(H, np.zeros(3), np.array([4, 7, 4]))
    assert list(T) == [0, 1]
    assert np.allclose(L @ L.T, H[:2, :2])
    # an accepted pivot whose updated diagonal is below tau is rejected
    H2 = np.array([[1.0, 0.999999], [0.999999, 1.0]])
    T2, _ = accept_reject(H2, np.zeros(2), np.array([0, 1]), tau=1e-5)
    assert list(T2) == [0]


def test_accept_reject_uses_updated_diagonal():
    """Pivot i is accepted iff z * H0(i,i) < H(i,i) after earlier updates."""
    H = np.array([[1.0, 0.8], [0.8, 1.0]])  # updated H(1,1) = 1 - 0.64 = 0.36
    assert list(accept_reject(H, [0.9, 0.35], [0, 1])[0]) == [0, 1]
    assert list(accept_reject(H, [0.9, 0.37], [0, 1])[0]) == [0]


# ------------------------------------------------------ Algorithm 2 pins


def test_greedy_order_matches_lapack_pstrf():
    """Greedy b=1 pivots = LAPACK dpstrf (complete pivoting) pivot order."""
    X, eps = _torus(300)
    K = gaussian_kernel(X, X, eps)
    out = arpc(X, eps, r=40, b=1, mode="greedy")
    c, piv, rank, info = sla.lapack.dpstrf(K, lower=1, tol=-1.0)
    assert list(out["S"]) == list(piv[:40] - 1)
    # the factor columns agree with LAPACK's (lower triangular, permuted)
    Lp = np.tril(c)[:, :40]
    Fl = np.zeros_like(Lp)
    Fl[piv - 1] = Lp
    assert np.max(np.abs(Fl - out["F"])) < 1e-10


@pytest.mark.parametrize("b", [1, 8, 12])
def test_factor_closed_form_and_residual(b):
    """p1-p3: F = K(:,S) chol(K(S,S))^{-T}; F(S,:) lower triangular with
    F(S,:)F(S,:)^T = K(S,S); rho = diag(K - F F^T) >= 0; K - F F^T is PSD."""
    X, eps = _torus(400, seed=b)
    u = uniform_stream(2 * b * (-(-64 // b)), seed=b)
    out = arpc(X, eps, r=64, b=b, mode="sampled", uniforms=u)
    F, S = out["F"], out["S"]
    k = out["k"]
    assert 0 < k <= 64 and len(set(S.tolist())) == k
    K = gaussian_kernel(X, X, eps)
    Lc = np.linalg.cholesky(K[np.ix_(S, S)])
    Fc = sla.solve_triangular(Lc, K[:, S].T, lower=True).T
    assert np.max(np.abs(F - Fc)) < 1e-8
    FS = F[S]
    assert np.max(np.abs(np.triu(FS, 1))) < 1e-12
    assert np.max(np.abs(FS @ FS.T - K[np.ix_(S, S)])) < 1e-12
    Rm = K - F @ F.T
    assert np.all(out["rho"] >= 0)
    assert np.max(np.abs(np.maximum(np.diag(Rm), 0) - out["rho"]) * (out["rho"] > 0)) < 1e-10
    assert np.all(out["rho"][S] == 0)
    assert np.linalg.eigvalsh(Rm).min() > -1e-10
    # Nystrom identity: F F^T = K(:,S) K(S,S)^{-1} K(S,:)
    Kn = K[:, S] @ np.linalg.solve(K[np.ix_(S, S)], K[S, :])
    assert np.max(np.abs(F @ F.T - Kn)) < 1e-7
    # trace error reported per round
    assert abs(out["trace_err"][-1] - out["rho"].sum() / 400) < 1e-15


def test_b1_is_rpc():
    """ARPC with b = 1 is RPC: every round accepts its single proposal and
    the factor equals a one-column-at-a-time RPC written from the text."""
    X, eps = _torus(200, seed=5)
    r = 30
    u = uniform_stream(2 * r, seed=11)
    out = arpc(X, eps, r=r, b=1, mode="sampled", uniforms=u)
    assert out["accepted"] == [1] * r
    N = X.shape[0]
    F = np.zeros((N, r))
    rho = np.ones(N)
    S = []
    for i in range(r):
        s = inverse_cdf_pivot(quantize_rho(rho), u[2 * i])
        col = np.exp(-((X.astype(np.float64) - X[s].astype(np.float64)) ** 2).sum(1) / eps)
        g = (col - F[:, :i] @ F[s, :i]) / math.sqrt(col[s] - F[s, :i] @ F[s, :i])
        F[:, i] = g
        rho = np.maximum(rho - g * g, 0.0)
        rho[s] = 0.0
        S.append(s)
    assert list(out["S"]) == S
    assert np.max(np.abs(out["F"] - F)) < 1e-10


def test_arpc_acceptance_law_matches_rpc():
    """The first two accepted pivots of one ARPC round (b = 2) follow RPC's
    law: s1 ~ rho/sum(rho); s2 = j accepted w.p. rho'_j/sum(rho), rho' the
    residual after s1, else only one pivot is accepted."""
    X = np.array([[0.0, 0.0], [0.3, 0.0], [1.0, 0.5], [2.0, 2.0]])
    eps = 1.0
    N = 4
    K = gaussian_kernel(X, X, eps)
    probs = {}
    for i in range(N):
        p1 = 1.0 / N
        resid = K - np.outer(K[:, i], K[:, i]) / K[i, i]
        rp = np.diag(resid).copy()
        rp[i] = 0.0
        for j in range(N):
            probs[(i, j)] = p1 * rp[j] / N
        probs[(i, None)] = p1 * (1 - rp.sum() / N)
    trials = 6000
    counts = {key: 0 for key in probs}
    for t in range(trials):
        u = uniform_stream(4, seed=1000 + t)
        out = arpc(X, eps, r=2, b=2, mode="sampled", uniforms=u)
        S = out["S"].tolist()
        counts[(S[0], S[1] if len(S) > 1 else None)] += 1
    keys = [k for k in probs if probs[k] > 1e-9]
    exp_ = np.array([trials * probs[k] for k in keys])
    obs = np.array([counts[k] for k in keys])
    assert sum(counts[k] for k in probs if probs[k] <= 1e-9) == 0
    stat = np.sum((obs - exp_) ** 2 / exp_)
    assert stat < chi2.ppf(0.999, len(keys) - 1), (stat, list(zip(keys, obs, exp_)))


def test_thm1_expected_trace_error_bound():
    """Theorem 1: E tr(K - K~) <= (1 + e) tr(K - [K]_r') when
    r >= r'/e + r' log(1/(e eta)); checked on the mean over seeds (RPC, b=1)."""
    X, eps = _torus(250, seed=3)
    K = gaussian_kernel(X, X, eps)
    lam = np.sort(np.linalg.eigvalsh(K))[::-1]
    rp, e = 4, 0.5
    tail = lam[rp:].sum()
    eta = tail / np.trace(K)
    r = int(math.ceil(rp / e + rp * math.log(1 / (e * eta))))
    errs = []
    for s in range(40):
        out = arpc(X, eps, r=r, b=1, mode="sampled", uniforms=uniform_stream(2 * r, seed=500 + s))
        errs.append(np.trace(K) - np.sum(out["F"] ** 2))
    assert np.mean(errs) <= (1 + e) * tail


def test_recovery_at_full_rank():
    """r = N with a narrow bandwidth (well-conditioned K): K~ = K and P~ = P."""
    X, eps = _torus(120, seed=9)
    eps = 0.1 * eps
    K = gaussian_kernel(X, X, eps)
    out = arpc(X, eps, r=120, b=1, mode="greedy")
    F = out["F"]
    assert out["k"] == 120
    assert np.max(np.abs(F @ F.T - K)) < 1e-10
    P, _, _ = dense_bistochastic(K)
    Pt, _, _ = dense_bistochastic(F @ F.T)
    assert np.max(np.abs(P - Pt)) < 1e-9
    res = bistoch_eig(F, 10)
    lam_true = np.sort(np.linalg.eigvalsh(P))[::-1][:10]
    assert np.max(np.abs(res["lam"] - lam_true) / lam_true) < 1e-9


def test_degenerate_all_points_equal():
    """All points equal: K = 11^T has rank 1; one pivot, then sum(rho_q) = 0 stops."""
    X = np.ones((50, 3), dtype=np.float32)
    out = arpc(X, 1.0, r=16, b=4, mode="sampled", uniforms=uniform_stream(2 * 4 * 4, seed=1))
    assert out["k"] == 1 and np.allclose(out["F"], 1.0) and np.all(out["rho"] == 0)
    res = bistoch_eig(out["F"], 1)
    assert abs(res["lam"][0] - 1.0) < 1e-14


def test_ragged_last_round():
    """r not divisible by b: t = ceil(r/b) rounds, the last proposes r-(t-1)b."""
    X, eps = _torus(300, seed=4)
    out = arpc(X, eps, r=20, b=8, mode="sampled", uniforms=uniform_stream(2 * 8 * 3, seed=4))
    assert len(out["accepted"]) == 3 and out["accepted"][2] <= 4 and out["k"] <= 20


def test_replay_reproduces_factor():
    X, eps = _torus(300, seed=6)
    out = arpc(X, eps, r=48, b=16, mode="sampled", uniforms=uniform_stream(2 * 16 * 3, seed=6))
    rep = arpc(X, eps, r=48, b=16, mode="replay", replay=out["S"])
    assert list(rep["S"]) == list(out["S"])
    assert np.max(np.abs(rep["F"] - out["F"])) < 1e-10
    # F depends only on the ordered pivots, not on the block size
    rep1 = arpc(X, eps, r=48, b=5, mode="replay", replay=out["S"])
    assert np.max(np.abs(rep1["F"] - out["F"])) < 1e-10


# ------------------------------------------------------ Algorithm 1 pins


def _factor(n=500, r=64, b=8, seed=0):
    X, eps = _torus(n, seed=seed)
    out = arpc(X, eps, r=r, b=b, mode="sampled", uniforms=uniform_stream(2 * b * (-(-r // b)), seed=seed))
    return X, eps, out


def test_degrees_row_sums_and_structure():
    """p9: P~ 1 = 1, P~ symmetric PSD, eigenpair (1, 1/sqrt(N)); 1 = B c."""
    X, eps, out = _factor()
    F = out["F"]
    N = F.shape[0]
    c, d, q = bistoch_degrees(F)
    Kt = F @ F.T
    assert np.allclose(d, Kt.sum(1), rtol=1e-12)
    assert np.allclose(q, Kt @ (1 / d), rtol=1e-12)
    Pt, _, _ = dense_bistochastic(Kt)
    assert np.max(np.abs(Pt.sum(1) - 1)) < 1e-12
    assert np.max(np.abs(Pt - Pt.T)) < 1e-14
    assert np.linalg.eigvalsh(Pt).min() > -1e-12
    assert np.max(np.abs((F / d[:, None]) @ c - 1)) < 1e-12
    res = bistoch_eig(F, 8)
    j = int(np.argmin(np.abs(res["lam_all"] - 1)))
    assert abs(res["lam_all"][j] - 1) < 1e-10
    lam_dense, V = np.linalg.eigh(Pt)
    jj = int(np.argmin(np.abs(lam_dense - 1)))
    assert abs(abs(V[:, jj].sum()) / math.sqrt(N) - 1) < 1e-8


def test_factored_evd_matches_dense():
    """p10: eigenpairs from Algorithm 1 = dense eigh of the explicitly formed P~."""
    X, eps, out = _factor(n=600, r=64, b=8, seed=1)
    F = out["F"]
    nev = 12
    res = bistoch_eig(F, nev)
    Pt, _, _ = dense_bistochastic(F @ F.T)
    lam, V = np.linalg.eigh(Pt)
    lam, V = lam[::-1], V[:, ::-1]
    assert np.max(np.abs(res["lam"] - lam[:nev]) / np.abs(lam[:nev])) < 1e-10
    # compare subspaces up to the last clear gap within the top nev
    gaps = [i for i in range(1, nev) if lam[i - 1] / lam[i] - 1 > 1e-3]
    m = gaps[-1]
    assert _angles(res["U"][:, :m], V[:, :m]) < 1e-8
    for j in range(m):  # individual vectors up to sign where isolated
        if (j == 0 or lam[j - 1] / lam[j] - 1 > 1e-3) and lam[j] / lam[j + 1] - 1 > 1e-3:
            assert min(np.max(np.abs(res["U"][:, j] - V[:, j])), np.max(np.abs(res["U"][:, j] + V[:, j]))) < 1e-8


def test_symmetric_route_matches_svd_and_dense():
    """Symmetric normalisation: QR + EVD of R R^T = SVD of D~^{-1/2} F = dense
    EVD of L~ (eigenvectors up to sign)."""
    X, eps, out = _factor(n=400, r=48, b=6, seed=2)
    F = out["F"]
    res = symmetric_eig(F, 6)
    d = (F @ F.T).sum(1)
    Us, s, _ = np.linalg.svd(F / np.sqrt(d)[:, None], full_matrices=False)
    assert np.max(np.abs(res["lam"] - s[:6] ** 2)) < 1e-12
    L, _ = dense_symmetric(F @ F.T)
    lam = np.sort(np.linalg.eigvalsh(L))[::-1]
    assert np.max(np.abs(res["lam"] - lam[:6])) < 1e-12
    assert _angles(res["U"][:, :3], Us[:, :3]) < 1e-8


def test_nystrom_route_matches_factor_route():
    """EVD of K~ by the Nystrom route (K(S,S) = V Z V^T, extend, QR, EVD) equals
    the factor route (QR of F, EVD of R R^T) up to sign."""
    X, eps, out = _factor(n=400, r=40, b=5, seed=3)
    F, S = out["F"], out["S"]
    K = gaussian_kernel(X, X, eps)
    Z, V = np.linalg.eigh(K[np.ix_(S, S)])
    Vt = K[:, S] @ V
    Q, R = np.linalg.qr(Vt)
    lam_n, W = np.linalg.eigh(R @ np.diag(1 / Z) @ R.T)
    Q2, R2 = np.linalg.qr(F)
    lam_f, W2 = np.linalg.eigh(R2 @ R2.T)
    assert np.max(np.abs(np.sort(lam_n) - np.sort(lam_f)) / np.max(lam_f)) < 1e-8
    top_n = (Q @ W)[:, ::-1][:, :3]
    top_f = (Q2 @ W2)[:, ::-1][:, :3]
    assert _angles(top_n, top_f) < 1e-6


def test_nystrom_extension_reproduces_training_rows():
    """Extension of P~'s eigenvectors evaluated at training points = rows of U."""
    X, eps, out = _factor(n=500, r=64, b=8, seed=4)
    F, S = out["F"], out["S"]
    res = bistoch_eig(F, 10)
    rows = np.array([0, 7, 123, 499, int(S[3])])
    phi = nystrom_extend(X[rows], X, S, F, res["c"], res["E"], eps)
    assert np.max(np.abs(phi - res["U"][rows])) < 1e-8


def test_degree_assert_raises():
    F = np.array([[1.0, 0.0], [-3.0, 0.1], [0.5, 0.2]])
    with pytest.raises(DegreeError, match="D~"):
        bistoch_degrees(F)
    # d~ = (2.375, 2.4375, 3.3125, 3.75, 1.25, 0.5) > 0 by hand, but
    # q~[0] = F[0] . F^T (1/d~) = -0.065 < 0: the second assert fires
    F = np.array([[0.5, 1.0], [0.0, 0.75], [-0.5, 0.75], [-0.75, 0.75], [-0.25, 0.25], [-0.75, -0.25]])
    assert np.allclose(F @ (F.T @ np.ones(6)), [2.375, 2.4375, 3.3125, 3.75, 1.25, 0.5])
    with pytest.raises(DegreeError, match="Q~"):
        bistoch_degrees(F)


def test_fix_const_column():
    X, eps, out = _factor(n=300, r=32, b=4, seed=5)
    res = bistoch_eig(out["F"], 6, fix_const=True)
    U = res["U"]
    assert np.allclose(U[:, 0], 1 / math.sqrt(300), atol=1e-12)
    assert np.allclose(U.T @ U, np.eye(6), atol=1e-12)


def test_error_bounds_lemma12_lemma14_thm7():
    """Lemma 12, Lemma 14 and Theorem 7 hold for every realisation."""
    X, eps = _torus(350, seed=8)
    K = gaussian_kernel(X, X, eps)
    N = K.shape[0]
    P, d, q = dense_bistochastic(K)
    normK = np.linalg.eigvalsh(K).max()
    for r, b in [(16, 4), (40, 8), (80, 8)]:
        out = arpc(X, eps, r=r, b=b, mode="sampled", uniforms=uniform_stream(2 * b * (-(-r // b)), seed=r))
        F = out["F"]
        Kt = F @ F.T
        tr_err = np.trace(K - Kt)
        Pt, dt, qt = dense_bistochastic(Kt)
        assert np.all(dt > 0) and np.all(qt > 0)
        # Lemma 12
        assert np.sum((d - dt) ** 2) <= N * tr_err ** 2 * (1 + 1e-12)
        assert np.max(np.abs(d - dt)) <= math.sqrt(N) * tr_err * (1 + 1e-12)
        # Lemma 14
        dd = min(d.min(), dt.min())
        assert np.max(np.abs(q - qt)) <= math.sqrt(N) / dd * (1 + normK / dd) * tr_err * (1 + 1e-12)
        # Theorem 7
        dq = min(q.min(), qt.min())
        Gnorm = math.sqrt(max(np.linalg.eigvalsh(Pt).max(), 0))
        bound = (1 + Gnorm) * (
            1 / (math.sqrt(q.min()) * d.min())
            + math.sqrt(N) * np.trace(K) / (math.sqrt(dq) * dd ** 2)
            + math.sqrt(N) * np.trace(K) / (2 * dq ** 1.5 * dd ** 2) * (1 + normK / dd)
        ) * tr_err
        lhs = np.abs(np.linalg.eigvalsh(P - Pt)).sum()
        assert lhs <= bound


@pytest.mark.parametrize("gamma", [1e-6, 1e-3, 0.1])
def test_gamma_regularised_qr_matches_dense(gamma):
    """The regularised QR of the "Numerical experiments" section (gamma added
    to the entries (i, i), i < k, of D~^{-1} F): the oracle's eigenpairs equal
    those of the dense N x N matrix B' C B'^T with B' = D~^{-1} F + gamma E_k
    formed explicitly, its U is orthonormal, and U = B' E (the extension
    identity, which for gamma > 0 holds with B' and not with D~^{-1} F)."""
    X, eps, out = _factor(n=500, r=48, b=8, seed=9)
    F = out["F"]
    N, k = F.shape
    nev = 10
    res = bistoch_eig(F, nev, gamma=gamma)
    c, d, q = bistoch_degrees(F)
    Bp = F / d[:, None]
    Bp[np.arange(k), np.arange(k)] += gamma
    C = F.T @ (F / q[:, None])
    lam, V = np.linalg.eigh(Bp @ C @ Bp.T)
    lam, V = lam[::-1], V[:, ::-1]
    assert np.max(np.abs(res["lam"] - lam[:nev]) / np.abs(lam[:nev])) < 1e-10
    m = max(i for i in range(1, nev + 1) if i == nev or lam[i - 1] / lam[i] - 1 > 1e-3)
    assert _angles(res["U"][:, :m], V[:, :m]) < 1e-8
    assert np.max(np.abs(res["U"].T @ res["U"] - np.eye(nev))) < 1e-12
    assert np.max(np.abs(Bp @ res["E"] - res["U"])) < 1e-10
    # the regulariser moves the spectrum: without it the eigenvalues differ
    if gamma >= 1e-3:
        assert np.max(np.abs(bistoch_eig(F, nev)["lam"] - res["lam"])) > 1e-6


# ------------------------------------------- symmetric normalisation pins


def test_symmetric_extension_reproduces_training_rows():
    """Extension of L~'s eigenvectors (f(y)^T E / sqrt(d~(y))) evaluated at
    training points = rows of U; at a new point it is the dense formula
    d~(y)^{-1/2} k~(y, X) D~^{-1/2} U Lambda^{-1} with k~(y, X) = f(y)^T F^T."""
    from oracle.bistoch import symmetric_extend

    X, eps, out = _factor(n=400, r=48, b=6, seed=12)
    F, S = out["F"], out["S"]
    res = symmetric_eig(F, 8)
    rows = np.array([0, 9, 200, 399, int(S[5])])
    phi = symmetric_extend(X[rows], X, S, F, res["c"], res["E"], eps)
    assert np.max(np.abs(phi - res["U"][rows])) < 1e-8
    Y = torus_points(30, seed=77)
    f = sla.solve_triangular(F[S, :], gaussian_kernel(X[S], Y, eps), lower=True)  # k x M
    kt = f.T @ F.T  # k~(y, X)
    dy = kt.sum(axis=1)
    dense = (kt / np.sqrt(dy)[:, None]) @ (res["U"] / np.sqrt(res["d"])[:, None]) / res["lam"][None, :]
    assert np.max(np.abs(symmetric_extend(Y, X, S, F, res["c"], res["E"], eps) - dense)) < 1e-9


def _sym_bound(dmin, delta, N, trK, err):
    """Theorem 3's bound on the trace norm of L - L~."""
    return (1.0 / dmin + math.sqrt(N) / delta ** 2 * trK + N / (4.0 * delta ** 3) * trK * err) * err


def test_theorem3_and_remark4_symmetric_bounds():
    """Theorem 3: |L - L~|_* <= [1/d_min + sqrt(N) tr K / delta^2 + N tr K
    tr(K - K~) / (4 delta^3)] tr(K - K~) for every realisation; Remark 4: with
    the exact degrees D in place of D~, L - L~_D is PSD with trace norm at most
    tr(K - K~) / d_min.  The oracle's symmetric eigenvalues satisfy Mirsky's
    sum |lambda_i(L) - lambda_i(L~)| <= |L - L~|_*."""
    X, eps = _torus(220, seed=13)
    K = gaussian_kernel(X, X, eps)
    N = K.shape[0]
    L, d = dense_symmetric(K)
    lamL = np.sort(np.linalg.eigvalsh(L))[::-1]
    trK = np.trace(K)
    for r, b in [(12, 4), (30, 6), (60, 10)]:
        out = arpc(X, eps, r=r, b=b, mode="sampled", uniforms=uniform_stream(2 * b * (-(-r // b)), seed=r + 5))
        F = out["F"]
        Kt = F @ F.T
        err = trK - np.trace(Kt)
        Lt, dt = dense_symmetric(Kt)
        assert np.all(dt > 0)
        tn = np.abs(np.linalg.eigvalsh(L - Lt)).sum()
        assert tn <= _sym_bound(d.min(), min(d.min(), dt.min()), N, trK, err)
        sD = 1.0 / np.sqrt(d)
        LD = Kt * sD[:, None] * sD[None, :]
        ev = np.linalg.eigvalsh(L - LD)
        assert ev.min() >= -1e-12 and ev.sum() <= err / d.min() * (1 + 1e-12)
        lo = np.zeros(N)
        lo[:out["k"]] = symmetric_eig(F, 1)["lam_all"]
        assert np.abs(lamL - np.sort(lo)[::-1]).sum() <= tn * (1 + 1e-9)


def test_corollary5_probability_bound():
    """Corollary 5 for RPC: with zeta from Theorem 1 (r' = 10, e = 1/2, r set
    by its rank condition) and 1 < t < d_min / (sqrt(N) zeta), with
    probability at least 1 - 1/t both d~_min > d_min - sqrt(N) t zeta and
    |L - L~|_* < [1/d_min + sqrt(N) tr K / a_t^2 + N tr K t zeta / (4 a_t^3)]
    t zeta, a_t = d_min - sqrt(N) t zeta.  Checked as a frequency over 60
    seeds against 1 - 1/t less three binomial standard deviations."""
    X, eps = _torus(200, seed=3)
    eps = 4.0 * eps  # a wide kernel: fast spectral decay, so the corollary applies
    K = gaussian_kernel(X, X, eps)
    N = K.shape[0]
    L, d = dense_symmetric(K)
    lam = np.sort(np.linalg.eigvalsh(K))[::-1]
    trK = np.trace(K)
    rp, e = 10, 0.5
    tail = lam[rp:].sum()
    r = int(math.ceil(rp / e + rp * math.log(trK / (e * tail))))
    zeta = (1 + e) * tail
    dmin = d.min()
    tmax = dmin / (math.sqrt(N) * zeta)
    assert tmax > 4
    seeds = 60
    hits = {2.0: 0, 4.0: 0}
    for s in range(seeds):
        out = arpc(X, eps, r=r, b=1, mode="sampled", uniforms=uniform_stream(2 * r, seed=900 + s))
        Kt = out["F"] @ out["F"].T
        Lt, dt = dense_symmetric(Kt)
        tn = np.abs(np.linalg.eigvalsh(L - Lt)).sum()
        for t in hits:
            a = dmin - math.sqrt(N) * t * zeta
            bound = (1 / dmin + math.sqrt(N) * trK / a ** 2 + N * trK * t * zeta / (4 * a ** 3)) * t * zeta
            if dt.min() > a and tn < bound:
                hits[t] += 1
    for t, h in hits.items():
        p = 1 - 1 / t
        assert h / seeds >= p - 3 * math.sqrt(p * (1 - p) / seeds)
