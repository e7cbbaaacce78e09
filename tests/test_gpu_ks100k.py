"""The plain method at paper shape against the oracle: KS delay embedding,
N = 100 000, d = 512, median bandwidth, r = 512, b = 64 (8 rounds), top 32
eigenpairs of P~ (Algorithms 2, 3 and 1).

The oracle's result is stored in tests/golden/ks100k_r512_b64.npz, written by
tests/golden/make_ks100k_golden.py, which calls only the oracle and the input
generators (the oracle takes about two minutes here).  Checks:
  * float64, free-running sampled pivots: the accepted pivots and per-round
    counts identical to the oracle's; F at sampled rows against the closed
    form K(n, S) chol(K(S, S))^{-T} (float64 error model of the products and
    block solves); eigenvalues within 1e-6 relative and the leading subspace
    (up to a clear gap) within 1e-4 rad;
  * float32 (float32 MFMA products, float32 factor and Grams), replaying the
    oracle's pivots: the same eigen bars, 1e-6 and 1e-4;
  * bf16 distance products (the mixed form), replaying the pivots: 1e-3 and
    1e-2.
The oracle's eigenvectors are U = D~^{-1} F Z with its Z = R^{-1} V stored;
the test forms them with the device's float64 factor and degrees (equal to the
oracle's to the float64 bars checked first).
"""
import hashlib
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from synth import ks_points, median_sq_distance, uniform_stream

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ks100k_r512_b64.npz")
N, Q, R, B, NEV = 100_000, 8, 512, 64, 32


@pytest.fixture(scope="module")
def case():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_26574_amd as rp

    rp.load_library()
    g = np.load(GOLD, allow_pickle=False)
    X = ks_points(N, q=Q, seed=0)
    assert hashlib.sha256(X.tobytes()).digest() == g["x_sha256"].tobytes(), "input generator changed"
    eps = float(g["eps"])
    assert eps == median_sq_distance(X, seed=0)
    u = uniform_stream(2 * B * (R // B), seed=0)
    Xd = torch.from_numpy(X).cuda()
    print("ks100k: float64 free-running factorisation", flush=True)
    out = rp.rpchol_factor(Xd, eps, R, B, mode="sampled", uniforms=torch.from_numpy(u).cuda())
    assert rp.status_sync(out["status"]) == 0
    deg = rp.bistoch_degrees(out["F"], out["k"])
    assert rp.status_sync(deg["status"]) == 0
    eig = rp.bistoch_eig(out["F"], out["k"], deg["d"], deg["q"], NEV)
    assert rp.status_sync(eig["status"]) == 0
    k = int(out["k"].item())
    # the oracle's eigenvectors from its Z and the device's float64 factor
    Uref = ((out["F"][:, :k] / deg["d"][:, None]) @ torch.from_numpy(g["Z"]).cuda()).cpu().numpy()
    return dict(torch=torch, rp=rp, g=g, X=X, Xd=Xd, eps=eps, out=out, deg=deg, eig=eig, k=k, Uref=Uref)


def _gap_index(lam, nev, rel=1e-3):
    for m in range(nev, 0, -1):
        if lam[m - 1] / lam[m] - 1 > rel:
            return m
    return nev


def _angle(U, V):
    Qu, _ = np.linalg.qr(U)
    Qv, _ = np.linalg.qr(V)
    s = np.linalg.norm(Qv - Qu @ (Qu.T @ Qv), 2)
    return float(np.arcsin(min(s, 1.0)))


def _eig_errors(c, eig):
    lam_o = c["g"]["lam"]
    lam = eig["lam"].cpu().numpy()
    m = _gap_index(lam_o, NEV)
    le = float(np.abs(lam / lam_o[:NEV] - 1).max())
    ae = _angle(eig["U"].double().cpu().numpy()[:, :m], c["Uref"][:, :m])
    return le, ae, m


def test_f64_pivots_factor_and_eigenpairs(case):
    c = case
    g, out, k = c["g"], c["out"], c["k"]
    piv = out["pivots"].cpu().numpy()
    assert k == len(g["pivots"]) and list(piv[:k]) == list(g["pivots"])
    assert list(out["round_accepted"].cpu().numpy()) == list(g["accepted"])
    trace = out["round_trace"].cpu().numpy()  # sum(rho) / N after each round
    assert np.abs(trace / g["trace_err"] - 1).max() < 1e-9
    # F at sampled rows (and a few pivots) against the closed form
    S = g["pivots"]
    rows = np.unique(np.concatenate([np.random.default_rng(7).choice(N, 384, replace=False), S[:: 37]]))
    Lss = sla.cholesky(oracle.gaussian_kernel(c["X"][S], c["X"][S], c["eps"]), lower=True)
    Fcf = sla.solve_triangular(Lss, oracle.gaussian_kernel(c["X"][S], c["X"][rows], c["eps"]), lower=True).T
    F = out["F"][:, :k].cpu().numpy()[rows]
    err = np.abs(F - Fcf).max() / np.abs(Fcf).max()
    bar = 10.0 * math.sqrt(k) * 2.0 ** -53 * np.linalg.cond(Lss)
    le, ae, m = _eig_errors(c, c["eig"])
    print(f"ks100k f64: k={k}, F error {err:.3g} (bar {bar:.3g}), eigenvalues {le:.3g}, "
          f"angle {ae:.3g} over {m}")
    assert err < bar
    assert le < 1e-6 and ae < 1e-4


@pytest.mark.parametrize("gemm,fac,gram,ltol,atol", [("f32", "f32", "f32", 1e-6, 1e-4),
                                                     ("bf16", "f32", "f32", 1e-3, 1e-2),
                                                     ("bf16", "f32", "split16", 1e-3, 1e-2)])
def test_reduced_precision_replay(case, gemm, fac, gram, ltol, atol):
    c = case
    torch, rp = c["torch"], c["rp"]
    rep = torch.from_numpy(np.asarray(c["g"]["pivots"], dtype=np.int64)).cuda()
    print(f"ks100k replay {gemm}/{fac}/{gram}", flush=True)
    out = rp.rpchol_factor(c["Xd"], c["eps"], R, B, mode="replay", replay=rep, gemm_dtype=gemm,
                           factor_dtype=fac)
    assert rp.status_sync(out["status"]) == 0
    deg = rp.bistoch_degrees(out["F"], out["k"])
    eig = rp.bistoch_eig(out["F"], out["k"], deg["d"], deg["q"], NEV, gram_dtype=gram)
    assert rp.status_sync(eig["status"]) == 0
    le, ae, m = _eig_errors(c, eig)
    print(f"ks100k {gemm}/{fac}/{gram}: eigenvalues {le:.3g}, angle {ae:.3g} over {m}")
    assert le < ltol and ae < atol
