"""GPU parity: the HIP path (through the C-ABI) against the float64 CPU oracle.

Bars (the contract of the method's precision forms):
  * pivots identical (greedy and sampled mode share the integer CDF, so any
    difference is a defect; cross-precision runs use replay);
  * F within 1e-12 (FP64) of the oracle relative to max |F|; in FP32 within
    5e-5: kernel entries carry a relative error of about u32 (|x|^2+|s|^2)/eps
    ~ 2e-7 from the norm expansion, which the pivot-block solves L^{-T}
    amplify by up to ~1e2 at r = 64; in BF16 products within 1e-2 on
    delay-embedded (d = 512) points, whose rounding errors average over
    the coordinates;
  * eigenvalues within 1e-6 relative at FP64/FP32 (1e-10 is asked at FP64)
    and 1e-3 at BF16; principal angles of the leading eigenvector subspace
    within 1e-4 rad (FP64/FP32) and 1e-2 (BF16).
"""
import math

import numpy as np
import pytest

import oracle
from synth import median_sq_distance, torus_points, uniform_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_26574_amd as rp

    rp.load_library()
    return torch, rp


def _angle(U, V):
    Qu, _ = np.linalg.qr(U)
    Qv, _ = np.linalg.qr(V)
    s = np.linalg.norm(Qv - Qu @ (Qu.T @ Qv), 2)
    return float(np.arcsin(min(s, 1.0)))


def _gap_index(lam, nev, rel=1e-3):
    """Largest m <= nev with a relative gap between lam[m-1] and lam[m]."""
    for m in range(nev, 0, -1):
        if m < len(lam) and lam[m - 1] / lam[m] - 1 > rel:
            return m
    return nev


def _torus_case(n=2000, seed=0):
    X = torus_points(n, seed=seed)
    return X, median_sq_distance(X, seed=seed)


def _run_factor(gpu, X, eps, r, b, mode, u=None, replay=None, gdt="f64", fdt="f64", tau=0.0):
    torch, rp = gpu
    Xd = torch.from_numpy(X).cuda()
    kw = {}
    if u is not None:
        kw["uniforms"] = torch.from_numpy(u).cuda()
    if replay is not None:
        kw["replay"] = torch.as_tensor(np.asarray(replay, dtype=np.int64)).cuda()
    out = rp.rpchol_factor(Xd, eps, r, b, mode=mode, gemm_dtype=gdt, factor_dtype=fdt, tau=tau, **kw)
    st = rp.status_sync(out["status"])
    assert st == 0, rp.STATUS_NAMES.get(st, st)
    k = int(out["k"].item())
    F = out["F"].double().cpu().numpy()
    return out, k, F, out["pivots"].cpu().numpy(), out["rho"].cpu().numpy()


def test_library_loads(gpu):
    torch, rp = gpu
    assert "gfx950" in rp.version()


def test_greedy_c1_pivots_and_factor(gpu):
    X, eps = _torus_case()
    ref = oracle.arpc(X, eps, r=64, b=1, mode="greedy")
    out, k, F, piv, rho = _run_factor(gpu, X, eps, 64, 1, "greedy")
    assert k == ref["k"] == 64
    assert list(piv[:k]) == list(ref["S"])
    scale = np.abs(ref["F"]).max()
    assert np.abs(F[:, :k] - ref["F"]).max() / scale < 1e-12
    assert np.all(F[:, k:] == 0)
    assert np.abs(rho - ref["rho"]).max() < 1e-12


@pytest.mark.parametrize("b", [1, 8, 16])
def test_sampled_c1_pivots_and_factor(gpu, b):
    X, eps = _torus_case(seed=b)
    r = 64
    u = uniform_stream(2 * b * (-(-r // b)), seed=100 + b)
    ref = oracle.arpc(X, eps, r=r, b=b, mode="sampled", uniforms=u)
    out, k, F, piv, rho = _run_factor(gpu, X, eps, r, b, "sampled", u=u)
    assert k == ref["k"]
    assert list(piv[:k]) == list(ref["S"])
    assert np.all(piv[k:] == -1)
    scale = np.abs(ref["F"]).max()
    assert np.abs(F[:, :k] - ref["F"]).max() / scale < 1e-12
    assert np.abs(rho - ref["rho"]).max() < 1e-12
    assert np.all(rho[ref["S"]] == 0)
    # per-round trace error sum(rho) / N after each round
    tr = out["round_trace"].cpu().numpy()
    assert len(tr) == len(ref["trace_err"])
    assert np.abs(tr - np.asarray(ref["trace_err"])).max() < 1e-12


def test_sampled_ragged_shapes(gpu):
    """N not a multiple of the tiles, d not a multiple of the k-step, r not a
    multiple of b (last round proposes r - (t-1) b)."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((1337, 37)).astype(np.float32)
    eps = median_sq_distance(X, seed=5)
    r, b = 100, 16
    u = uniform_stream(2 * b * 7, seed=77)
    ref = oracle.arpc(X, eps, r=r, b=b, mode="sampled", uniforms=u)
    out, k, F, piv, rho = _run_factor(gpu, X, eps, r, b, "sampled", u=u)
    assert k == ref["k"] and list(piv[:k]) == list(ref["S"])
    assert np.abs(F[:, :k] - ref["F"]).max() / np.abs(ref["F"]).max() < 1e-12


@pytest.mark.parametrize("fdt,gdt", [("f64", "f64"), ("f32", "f32"), ("f32", "bf16")])
def test_factor_leading_dimension_and_ragged_tail(gpu, fdt, gdt):
    """F stored with two leading dimensions (the default 1344 and 1352, both
    multiples of 8 as the ABI asks) at N = 1337, whose last 16-row block of
    the solve is ragged (element stores) while the others take vector stores:
    pivots, F and the residual diagonal are equal bit for bit."""
    torch, rp = gpu
    rng = np.random.default_rng(9)
    X = rng.standard_normal((1337, 37)).astype(np.float32)
    eps = median_sq_distance(X, seed=9)
    r, b = 200, 64
    u = torch.from_numpy(uniform_stream(2 * b * 4, seed=9)).cuda()
    Xd = torch.from_numpy(X).cuda()
    outs = [rp.rpchol_factor(Xd, eps, r, b, uniforms=u, gemm_dtype=gdt, factor_dtype=fdt, ldf=ld)
            for ld in (None, 1352)]
    assert outs[0]["ldf"] == 1344 and outs[1]["ldf"] == 1352
    for o in outs:
        assert rp.status_sync(o["status"]) == 0
    k = int(outs[0]["k"].item())
    assert k == int(outs[1]["k"].item()) and k > 100
    assert torch.equal(outs[0]["pivots"], outs[1]["pivots"])
    assert torch.equal(outs[0]["F"][:, :k], outs[1]["F"][:, :k])
    assert torch.equal(outs[0]["rho"], outs[1]["rho"])


@pytest.mark.parametrize("n,d,unfused", [(77, 1, False), (1337, 37, False), (1337, 37, True),
                                         (2051, 70, False), (300, 130, True)])
def test_split16_ragged_shapes(gpu, n, d, unfused):
    """The split-fp16 distance form on shapes that leave partial tiles: N below
    or not a multiple of the 128-row tile, d not a multiple of the 64-deep
    split stage (a stage that is partly or wholly padding), r not a multiple
    of b; fused and two-kernel paths, replaying the oracle's pivots, to the
    split form's F bar 2e-4."""
    torch, rp = gpu
    rng = np.random.default_rng(n + d)
    X = rng.standard_normal((n, d)).astype(np.float32)
    eps = median_sq_distance(X, seed=n)
    r, b = min(60, n), 16
    u = uniform_stream(2 * b * (-(-r // b)), seed=n)
    ref = oracle.arpc(X, eps, r=r, b=b, mode="sampled", uniforms=u)
    Xd = torch.from_numpy(X).cuda()
    rep = torch.as_tensor(np.asarray(ref["S"], dtype=np.int64)).cuda()
    out = rp.rpchol_factor(Xd, eps, r, b, mode="replay", replay=rep, gemm_dtype="split16",
                           factor_dtype="f32", unfused=unfused)
    assert rp.status_sync(out["status"]) == 0
    k = int(out["k"].item())
    assert k == ref["k"]
    F = out["F"][:, :k].double().cpu().numpy()
    err = np.abs(F - ref["F"]).max() / np.abs(ref["F"]).max()
    print(f"split16 N={n} d={d} unfused={unfused}: F error {err:.3g}")
    assert err < 2e-4
    assert not out["F"][:, k:].any().item()


def test_sampled_large_rank_f64(gpu):
    """Ranks in the hundreds: the proposal block's factor product spans several
    slices of the split proposal-block kernel (coordinates and factor columns
    in one index range), many rounds of b = 64; pivots identical to the
    oracle's.  F is held to the float64 error model of its products and block
    solves, 10 sqrt(k) u cond(F(S, :)) (u = 2^-53; the two sides sum and block
    differently), which at this rank exceeds the small cases' 1e-12."""
    X = torus_points(3000, seed=41)
    eps = median_sq_distance(X, seed=41) / 16.0  # narrow kernel: slow spectral decay, many pivots
    r, b = 600, 64
    u = uniform_stream(2 * b * (-(-r // b)), seed=41)
    ref = oracle.arpc(X, eps, r=r, b=b, mode="sampled", uniforms=u)
    out, k, F, piv, rho = _run_factor(gpu, X, eps, r, b, "sampled", u=u)
    assert ref["k"] > 300
    assert k == ref["k"] and list(piv[:k]) == list(ref["S"])
    err = np.abs(F[:, :k] - ref["F"]).max() / np.abs(ref["F"]).max()
    bar = 10.0 * math.sqrt(k) * 2.0 ** -53 * np.linalg.cond(ref["F"][np.asarray(ref["S"]), :])
    print(f"k = {k}: F error {err:.3g}, bar {bar:.3g}")
    assert err < bar


@pytest.mark.parametrize("gdt,fdt,ftol", [("f64", "f64", 1e-12), ("f32", "f32", 5e-5), ("bf16", "f32", 1e-2),
                                           ("split16", "f32", 2e-4)])
def test_wide_points(gpu, gdt, fdt, ftol):
    """Points of width d = 2050 (the padded width 2080 spans 65 k-stages of 32
    and 33 of 64 with a ragged last stage, and the proposal block's joint
    coordinate/column range runs over nine slices of 256): float64 pivots are
    the oracle's and F within 1e-12; the reduced-precision forms replay the
    oracle's pivots and hold F to their bars."""
    rng = np.random.default_rng(61)
    X = rng.standard_normal((600, 2050)).astype(np.float32)
    eps = median_sq_distance(X, seed=61)
    r, b = 96, 32
    u = uniform_stream(2 * b * (r // b), seed=61)
    ref = oracle.arpc(X, eps, r=r, b=b, mode="sampled", uniforms=u)
    mode, kw = ("sampled", {"u": u}) if gdt == "f64" else ("replay", {"replay": ref["S"]})
    out, k, F, piv, rho = _run_factor(gpu, X, eps, r, b, mode, gdt=gdt, fdt=fdt, **kw)
    assert k == ref["k"] and list(piv[:k]) == list(ref["S"])
    err = np.abs(F[:, :k] - ref["F"]).max() / np.abs(ref["F"]).max()
    print(f"{gdt}: k = {k}, F error {err:.3g}")
    assert err < ftol


def test_full_budget_f64(gpu):
    """The whole budget r = N (200 points in R^8, b = 40: five rounds whose
    proposals run out of fresh points, so repeats and rejections spend part
    of the budget): pivots and F are the oracle's, and the residual K - F F^T,
    positive semidefinite, has no entry above its largest diagonal entry
    (the returned rho)."""
    rng = np.random.default_rng(62)
    X = rng.standard_normal((200, 8)).astype(np.float32)
    eps = median_sq_distance(X, seed=62)
    r, b = 200, 40
    u = uniform_stream(2 * b * (r // b), seed=62)
    ref = oracle.arpc(X, eps, r=r, b=b, mode="sampled", uniforms=u)
    out, k, F, piv, rho = _run_factor(gpu, X, eps, r, b, "sampled", u=u)
    assert k == ref["k"] and k > 100 and list(piv[:k]) == list(ref["S"])
    assert np.abs(F[:, :k] - ref["F"]).max() / np.abs(ref["F"]).max() < 1e-12
    K = oracle.gaussian_kernel(X.astype(np.float64), X.astype(np.float64), eps)
    Fk = F[:, :k]
    assert np.abs(Fk @ Fk.T - K).max() <= rho.max() + 1e-12


def test_repeated_proposals(gpu):
    """A block that proposes the same point several times (32 draws from 50
    points, 8 of them repeats in the first round): Algorithm 3 accepts a point
    at most once; pivots identical to the oracle's, F within the float64 bar."""
    rng = np.random.default_rng(51)
    X = rng.standard_normal((50, 4)).astype(np.float32)
    eps = median_sq_distance(X, seed=51)
    u = uniform_stream(2 * 32 * 2, seed=51)
    ref = oracle.arpc(X, eps, r=40, b=32, mode="sampled", uniforms=u)
    out, k, F, piv, rho = _run_factor(gpu, X, eps, 40, 32, "sampled", u=u)
    assert k == ref["k"] and list(piv[:k]) == list(ref["S"])
    assert len(set(piv[:k].tolist())) == k
    assert np.abs(F[:, :k] - ref["F"]).max() / np.abs(ref["F"]).max() < 1e-12


def test_degenerate_all_equal_points(gpu):
    X = np.ones((300, 4), dtype=np.float32)
    u = uniform_stream(2 * 4 * 4, seed=1)
    out, k, F, piv, rho = _run_factor(gpu, X, 1.0, 16, 4, "sampled", u=u)
    assert k == 1 and np.allclose(F[:, 0], 1.0) and np.all(F[:, 1:] == 0) and np.all(rho == 0)


def test_replay_f64_matches_oracle(gpu):
    X, eps = _torus_case(seed=3)
    u = uniform_stream(2 * 16 * 4, seed=3)
    ref = oracle.arpc(X, eps, r=64, b=16, mode="sampled", uniforms=u)
    out, k, F, piv, rho = _run_factor(gpu, X, eps, 64, 16, "replay", replay=ref["S"])
    assert k == ref["k"] and list(piv[:k]) == list(ref["S"])
    assert np.abs(F[:, :k] - ref["F"]).max() / np.abs(ref["F"]).max() < 1e-12


def _ks_case(n=2000, seed=0, q=8):
    from synth import ks_points

    X = ks_points(n, q=q, seed=seed)
    return X, median_sq_distance(X, seed=seed)


# split16: float32 points with split-fp16 distance and Schur products (unit
# roundoff 2^-22 per product), so 4 x the float32 bar
@pytest.mark.parametrize("gdt,fdt,case,ftol", [("f32", "f32", "torus", 5e-5), ("bf16", "f32", "ks", 1e-2),
                                               ("split16", "f32", "torus", 2e-4),
                                               ("split16", "f32", "ks", 2e-4)])
def test_replay_reduced_precision(gpu, gdt, fdt, case, ftol):
    X, eps = _torus_case(seed=4) if case == "torus" else _ks_case(seed=4)
    u = uniform_stream(2 * 16 * 4, seed=4)
    ref = oracle.arpc(X, eps, r=64, b=16, mode="sampled", uniforms=u)
    out, k, F, piv, rho = _run_factor(gpu, X, eps, 64, 16, "replay", replay=ref["S"], gdt=gdt, fdt=fdt)
    assert k == ref["k"]
    err = np.abs(F[:, :k] - ref["F"]).max() / np.abs(ref["F"]).max()
    print(f"{gdt}/{case}: F error {err:.3g}")
    assert err < ftol


def _eig_case(gpu, X, eps, r, b, nev, seed, gdt="f64", fdt="f64", gram="f64", fix_const=False):
    torch, rp = gpu
    u = uniform_stream(2 * b * (-(-r // b)), seed=seed)
    ref = oracle.arpc(X, eps, r=r, b=b, mode="sampled", uniforms=u)
    mode, kw = ("sampled", {"u": u}) if gdt == "f64" else ("replay", {"replay": ref["S"]})
    out, k, F, piv, rho = _run_factor(gpu, X, eps, r, b, mode, gdt=gdt, fdt=fdt, **kw)
    deg = rp.bistoch_degrees(out["F"], out["k"])
    eig = rp.bistoch_eig(out["F"], out["k"], deg["d"], deg["q"], nev, gram_dtype=gram, fix_const=fix_const)
    assert rp.status_sync(eig["status"]) == 0
    assert rp.status_sync(deg["status"]) == 0
    res = oracle.bistoch_eig(ref["F"], nev, fix_const=fix_const)
    return ref, out, deg, eig, res


def test_degrees_and_eig_c1_f64(gpu):
    X, eps = _torus_case()
    nev = 16
    ref, out, deg, eig, res = _eig_case(gpu, X, eps, 64, 8, nev, seed=21)
    c, d, q = (deg[x].cpu().numpy() for x in ("c", "d", "q"))
    k = ref["k"]
    assert np.abs(c[:k] - res["c"]).max() / np.abs(res["c"]).max() < 1e-12
    assert np.all(c[k:] == 0)
    assert np.abs(d / res["d"] - 1).max() < 1e-12
    assert np.abs(q / res["q"] - 1).max() < 1e-12
    lam = eig["lam"].cpu().numpy()
    assert np.abs(lam / res["lam"] - 1).max() < 1e-10
    U = eig["U"].cpu().numpy()
    m = _gap_index(res["lam_all"], nev)
    assert _angle(U[:, :m], res["U"][:, :m]) < 1e-8
    # sign convention: largest-magnitude entry positive
    for j in range(nev):
        i = int(np.argmax(np.abs(U[:, j])))
        assert U[i, j] > 0
    # P~ 1 = 1 means the constant vector is an eigenvector with eigenvalue 1
    assert np.min(np.abs(lam - 1.0)) < 1e-10


def test_eig_fix_const(gpu):
    X, eps = _torus_case(seed=2)
    ref, out, deg, eig, res = _eig_case(gpu, X, eps, 64, 8, 8, seed=22, fix_const=True)
    U = eig["U"].cpu().numpy()
    assert np.abs(U[:, 0] - 1 / math.sqrt(U.shape[0])).max() < 1e-12
    assert np.abs(U.T @ U - np.eye(8)).max() < 1e-12
    assert _angle(U, res["U"]) < 1e-8


@pytest.mark.parametrize("gdt,fdt,gram,case,ltol,atol", [
    ("f32", "f32", "f32", "torus", 1e-6, 1e-4),
    ("bf16", "f32", "f32", "ks", 1e-3, 1e-2),
    # the split-fp16 Gram keeps 22 of float32's 24 bits per operand (unit
    # roundoff 2^-22 = 4 x float32's), so its bars are 4 x the float32 ones
    ("f32", "f32", "split16", "torus", 4e-6, 4e-4),
    ("bf16", "f32", "split16", "ks", 1e-3, 1e-2),
    # split-fp16 distances, Schur products and Grams: the same 2^-22 bars
    ("split16", "f32", "split16", "torus", 4e-6, 4e-4),
    ("split16", "f32", "split16", "ks", 4e-6, 4e-4),
])
def test_eig_reduced_precision(gpu, gdt, fdt, gram, case, ltol, atol):
    X, eps = _torus_case(seed=6) if case == "torus" else _ks_case(seed=6)
    nev = 16
    ref, out, deg, eig, res = _eig_case(gpu, X, eps, 64, 16, nev, seed=23, gdt=gdt, fdt=fdt, gram=gram)
    lam = eig["lam"].cpu().numpy()
    m = _gap_index(res["lam_all"], nev)
    le = np.abs(lam / res["lam"] - 1).max()
    U = eig["U"].cpu().numpy()
    ae = _angle(U[:, :m], res["U"][:, :m])
    print(f"{gdt}/{gram}/{case}: eigenvalue error {le:.3g}, angle {ae:.3g}")
    assert le < ltol
    assert ae < atol
    # the sign rule on the returned columns (the split form finds the column
    # maxima inside its U kernel): the largest |U(:, j)|, lowest row on ties, is positive
    top = np.argmax(np.abs(U), axis=0)
    assert np.all(U[top, np.arange(U.shape[1])] > 0)


@pytest.mark.parametrize("gram,ltol,atol", [("f32", 1e-6, 1e-4), ("split16", 4e-6, 4e-4)])
def test_float32_grams_many_chunks(gpu, gram, ltol, atol):
    """The float32 Gram forms over 28 row chunks with a ragged last chunk and
    a ragged last column tile (N = 40 003, r = 256, k = 192 accepted),
    subspace-iteration eigensolver, against the oracle on its own pivots
    (replayed)."""
    rng = np.random.default_rng(11)
    X = rng.standard_normal((40_003, 6)).astype(np.float32)
    eps = median_sq_distance(X, seed=11)
    nev = 24
    ref, out, deg, eig, res = _eig_case(gpu, X, eps, 256, 32, nev, seed=26, gdt="f32", fdt="f32",
                                        gram=gram)
    assert ref["k"] > 128
    lam = eig["lam"].cpu().numpy()
    m = _gap_index(res["lam_all"], nev)
    le = np.abs(lam / res["lam"] - 1).max()
    ae = _angle(eig["U"].cpu().numpy()[:, :m], res["U"][:, :m])
    print(f"{gram}: eigenvalue error {le:.3g}, angle {ae:.3g}")
    assert le < ltol
    assert ae < atol


@pytest.mark.parametrize("N", [1_500_000, 2_200_000])
def test_split16_grams_long_chunks(gpu, N):
    """Split-fp16 Grams over long row chunks (r = 128, one column tile): at
    N = 1.5e6 a chunk holds 46 runs of 256 rows (both Grams from one pass over
    F, runs joined in float32), at N = 2.2e6 it holds 68 (more than 64: one
    pass per Gram with float64 joins).  Torus points, float32 factor; the
    eigenvalues match those of the float64-Gram form of the same factor to the
    split form's bar (4 x the float32 one, as above)."""
    torch, rp = gpu
    r, b, nev = 128, 64, 16
    X = torus_points(N, seed=8)
    eps = median_sq_distance(X, seed=8) / 64  # a narrow kernel: all 128 columns taken
    u = uniform_stream(2 * b * (r // b), seed=8)
    out = rp.rpchol_factor(torch.from_numpy(X).cuda(), eps, r, b, mode="sampled", gemm_dtype="f32",
                           factor_dtype="f32", uniforms=torch.from_numpy(u).cuda())
    assert rp.status_sync(out["status"]) == 0
    k = int(out["k"].item())
    deg = rp.bistoch_degrees(out["F"], out["k"])
    assert rp.status_sync(deg["status"]) == 0
    lam = {}
    for gram in ("f64", "split16"):
        e = rp.bistoch_eig(out["F"], out["k"], deg["d"], deg["q"], nev, gram_dtype=gram)
        assert rp.status_sync(e["status"]) == 0
        lam[gram] = e["lam"].cpu().numpy()
    le = np.abs(lam["split16"] / lam["f64"] - 1).max()
    print(f"N={N}, k={k}: eigenvalue error {le:.3g}")
    assert np.min(np.abs(lam["f64"] - 1.0)) < 1e-6
    assert le < 4e-6


def test_split16_rejects_float64_factor(gpu):
    torch, rp = gpu
    X, eps = _torus_case(seed=5)
    u = uniform_stream(2 * 8 * 4, seed=5)
    out, k, F, piv, rho = _run_factor(gpu, X, eps, 32, 8, "sampled", u=u)
    deg = rp.bistoch_degrees(out["F"], out["k"])
    with pytest.raises(rp.RpcError):
        rp.bistoch_eig(out["F"], out["k"], deg["d"], deg["q"], 4, gram_dtype="split16")


def test_subspace_iteration_path(gpu):
    """r > 96 takes the subspace-iteration eigensolver."""
    rng = np.random.default_rng(8)
    X = rng.standard_normal((3000, 6)).astype(np.float32)
    eps = median_sq_distance(X, seed=8)
    nev = 24
    ref, out, deg, eig, res = _eig_case(gpu, X, eps, 160, 32, nev, seed=24)
    lam = eig["lam"].cpu().numpy()
    assert np.abs(lam / res["lam"] - 1).max() < 1e-10
    m = _gap_index(res["lam_all"], nev)
    assert _angle(eig["U"].cpu().numpy()[:, :m], res["U"][:, :m]) < 1e-8


def test_nystrom_extension(gpu):
    torch, rp = gpu
    X, eps = _torus_case(seed=7)
    nev = 10
    ref, out, deg, eig, res = _eig_case(gpu, X, eps, 64, 8, nev, seed=25)
    Y = torus_points(500, seed=99)
    ph = rp.nystrom_extend(torch.from_numpy(Y).cuda(), torch.from_numpy(X).cuda(), eps, out["pivots"],
                           out["k"], out["F"], deg["c"], eig["E"])
    assert rp.status_sync(ph["status"]) == 0
    Phi = ph["Phi"].cpu().numpy()
    phi_ref = oracle.nystrom_extend(Y, X, ref["S"], ref["F"], res["c"], res["E"], eps)
    assert np.abs(Phi - phi_ref).max() / np.abs(phi_ref).max() < 1e-9
    # at training points the extension reproduces U
    rows = np.array([0, 5, 999, 1999])
    ph2 = rp.nystrom_extend(torch.from_numpy(X[rows]).cuda(), torch.from_numpy(X).cuda(), eps,
                            out["pivots"], out["k"], out["F"], deg["c"], eig["E"])
    U = eig["U"].cpu().numpy()
    assert np.abs(ph2["Phi"].cpu().numpy() - U[rows]).max() < 1e-9


def test_invalid_arguments_rejected(gpu):
    torch, rp = gpu
    X = torch.zeros((10, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(rp.RpcError):
        rp.rpchol_factor(X, 1.0, 11, 1, mode="greedy")  # r > N
    with pytest.raises(rp.RpcError):
        rp.rpchol_factor(X, 1.0, 4, 2, mode="greedy")  # greedy needs b = 1
    with pytest.raises(rp.RpcError):
        rp.rpchol_factor(X, -1.0, 4, 1, mode="greedy")  # eps <= 0


def test_nonfinite_input_flagged(gpu):
    torch, rp = gpu
    X = np.ones((64, 3), dtype=np.float32)
    X[5, 1] = np.nan
    out = rp.rpchol_factor(torch.from_numpy(X).cuda(), 1.0, 4, 1, mode="greedy")
    assert rp.status_sync(out["status"]) == rp.RPC_ENONFINITE


def test_repeat_runs_bitwise_identical(gpu):
    X, eps = _torus_case(seed=9)
    u = uniform_stream(2 * 16 * 4, seed=9)
    _, k1, F1, p1, r1 = _run_factor(gpu, X, eps, 64, 16, "sampled", u=u)
    _, k2, F2, p2, r2 = _run_factor(gpu, X, eps, 64, 16, "sampled", u=u)
    assert k1 == k2 and np.array_equal(p1, p2) and np.array_equal(F1, F2) and np.array_equal(r1, r2)


@pytest.mark.parametrize("gdt", ["bf16", "split16"])
def test_unfused_columns_and_schur_agree(gpu, gdt):
    """The two-kernel path (kernel columns, then the Schur update) and the fused
    kernel give the same factor to float32 rounding (the fp32 bar, 5e-5; the
    split form's fused Schur product is split, the separate one float32)."""
    torch, rp = gpu
    from synth import ks_points

    X = ks_points(6000, q=8, seed=21)
    eps = median_sq_distance(X, seed=21)
    u = uniform_stream(2 * 128, seed=21)
    Xd = torch.from_numpy(X).cuda()
    ud = torch.from_numpy(u).cuda()
    fused = rp.rpchol_factor(Xd, eps, 128, 32, uniforms=ud, gemm_dtype=gdt, factor_dtype="f32")
    assert rp.status_sync(fused["status"]) == 0
    k = int(fused["k"].item())
    rep = fused["pivots"][:k].clone()
    un = rp.rpchol_factor(Xd, eps, 128, 32, mode="replay", replay=rep, gemm_dtype=gdt,
                          factor_dtype="f32", unfused=True)
    fu = rp.rpchol_factor(Xd, eps, 128, 32, mode="replay", replay=rep, gemm_dtype=gdt,
                          factor_dtype="f32")
    assert rp.status_sync(un["status"]) == 0 and rp.status_sync(fu["status"]) == 0
    a = un["F"][:, :k].double().cpu().numpy()
    b = fu["F"][:, :k].double().cpu().numpy()
    print(f"{gdt}: unfused vs fused {np.abs(a - b).max() / np.abs(b).max():.3g}")
    assert np.abs(a - b).max() <= 5e-5 * np.abs(b).max()


@pytest.mark.parametrize("e", [20, -20])
def test_split16_distances_scale_free(gpu, e):
    """The split-fp16 distance form scales both operands by a power of two
    chosen from max |x|: points scaled by 2^e with eps scaled by 2^(2e) give
    the same kernel, and the same factor and pivots bit for bit (every scaling
    on the way is exact)."""
    torch, rp = gpu
    from synth import ks_points

    X = ks_points(3000, q=6, seed=31)
    eps = median_sq_distance(X, seed=31)
    u = uniform_stream(2 * 32 * 3, seed=31)
    ud = torch.from_numpy(u).cuda()
    outs = []
    for s in (0, e):
        Xs = (X.astype(np.float64) * 2.0 ** s).astype(np.float32)
        o = rp.rpchol_factor(torch.from_numpy(Xs).cuda(), eps * 4.0 ** s, 96, 32, uniforms=ud,
                             gemm_dtype="split16", factor_dtype="f32")
        assert rp.status_sync(o["status"]) == 0
        outs.append(o)
    a, b = outs
    assert a["k"].item() == b["k"].item()
    assert torch.equal(a["pivots"], b["pivots"]) and torch.equal(a["F"], b["F"])


def _sym_case(gpu, X, eps, r, b, nev, seed, gram="f64"):
    torch, rp = gpu
    u = uniform_stream(2 * b * (-(-r // b)), seed=seed)
    ref = oracle.arpc(X, eps, r=r, b=b, mode="sampled", uniforms=u)
    out, k, F, piv, rho = _run_factor(gpu, X, eps, r, b, "sampled", u=u)
    deg = rp.bistoch_degrees(out["F"], out["k"])
    eig = rp.bistoch_eig(out["F"], out["k"], deg["d"], None, nev, gram_dtype=gram,
                         normalization="symmetric")
    assert rp.status_sync(eig["status"]) == 0
    return ref, out, deg, eig, oracle.symmetric_eig(ref["F"], nev)


def test_symmetric_normalization_c1_f64(gpu):
    """L~ = D~^{-1/2} K~ D~^{-1/2}: eigenpairs against the oracle's QR route,
    and the exact leading pair (1, D~^{1/2} 1 / |D~^{1/2} 1|)."""
    X, eps = _torus_case(seed=3)
    nev = 16
    ref, out, deg, eig, res = _sym_case(gpu, X, eps, 64, 8, nev, seed=31)
    lam = eig["lam"].cpu().numpy()
    assert np.abs(lam / res["lam"] - 1).max() < 1e-10
    U = eig["U"].cpu().numpy()
    m = _gap_index(res["lam_all"], nev)
    assert _angle(U[:, :m], res["U"][:, :m]) < 1e-8
    assert abs(lam[0] - 1.0) < 1e-12
    sd = np.sqrt(deg["d"].cpu().numpy())
    assert np.abs(U[:, 0] - sd / np.linalg.norm(sd)).max() < 1e-10


def test_symmetric_normalization_subspace_path(gpu):
    rng = np.random.default_rng(9)
    X = rng.standard_normal((3000, 6)).astype(np.float32)
    eps = median_sq_distance(X, seed=9)
    nev = 24
    ref, out, deg, eig, res = _sym_case(gpu, X, eps, 160, 32, nev, seed=32)
    lam = eig["lam"].cpu().numpy()
    assert np.abs(lam / res["lam"] - 1).max() < 1e-10
    m = _gap_index(res["lam_all"], nev)
    assert _angle(eig["U"].cpu().numpy()[:, :m], res["U"][:, :m]) < 1e-8


def test_symmetric_extension(gpu):
    """nystrom_extend_symmetric: the eigenvectors of L~ at new points against
    the oracle's symmetric extension f(y)^T E / sqrt(c^T f(y)), and at
    training points the rows of U."""
    torch, rp = gpu
    X, eps = _torus_case(seed=8)
    nev = 10
    ref, out, deg, eig, res = _sym_case(gpu, X, eps, 64, 8, nev, seed=33)
    Y = torus_points(700, seed=101)
    rows = np.array([0, 5, 999, 1999, int(ref["S"][3])])
    Yall = np.concatenate([Y, X[rows]])
    ph = rp.nystrom_extend(torch.from_numpy(Yall).cuda(), torch.from_numpy(X).cuda(), eps, out["pivots"],
                           out["k"], out["F"], deg["c"], eig["E"], symmetric=True)
    assert rp.status_sync(ph["status"]) == 0
    P = ph["Phi"].cpu().numpy()
    # the oracle's extension with its own E, up to the last clear eigenvalue
    # gap, rotated by O = U_oracle^T U_gpu (eigenvectors of a degenerate
    # eigenvalue, e.g. the torus's symmetric pairs, are unique only up to an
    # orthogonal map of their block, and so is the extension)
    Po = oracle.symmetric_extend(Yall, X, ref["S"], ref["F"], res["c"], res["E"], eps)
    m = _gap_index(res["lam_all"], nev)
    O = res["U"][:, :m].T @ eig["U"].cpu().numpy()[:, :m]
    err = np.abs(P[:, :m] - Po[:, :m] @ O).max() / np.abs(Po[:, :m]).max()
    Ut = eig["U"].cpu().numpy()[rows]
    terr = np.abs(P[len(Y):] - Ut).max() / np.abs(Ut).max()
    print(f"symmetric extension: error {err:.3g} (new points), {terr:.3g} (training rows)")
    assert err < 1e-9 and terr < 1e-9


@pytest.mark.parametrize("gamma", [1e-6, 1e-3])
@pytest.mark.parametrize("r,b,nev", [(64, 8, 16), (160, 32, 24)])
def test_eig_gamma_regularised_qr(gpu, gamma, r, b, nev):
    """The regularised QR of the "Numerical experiments" section: gamma on the
    entries (i, i), i < k, of D~^{-1} F.  Float64 path against the oracle on
    the same pivots (bars of the float64 form), U orthonormal, and the
    extension identity U = B' E with B' the regularised matrix; r = 64 takes
    the Jacobi eigensolver, r = 160 the subspace iteration."""
    torch, rp = gpu
    X, eps = _torus_case(seed=31)
    u = uniform_stream(2 * b * (-(-r // b)), seed=31)
    ref = oracle.arpc(X, eps, r=r, b=b, mode="sampled", uniforms=u)
    out, k, F, piv, rho = _run_factor(gpu, X, eps, r, b, "sampled", u=u)
    assert k == ref["k"] and list(piv[:k]) == list(ref["S"])
    deg = rp.bistoch_degrees(out["F"], out["k"])
    eig = rp.bistoch_eig(out["F"], out["k"], deg["d"], deg["q"], nev, gamma=gamma)
    assert rp.status_sync(eig["status"]) == 0
    res = oracle.bistoch_eig(ref["F"], nev, gamma=gamma)
    lam = eig["lam"].cpu().numpy()
    U = eig["U"].cpu().numpy()
    assert np.abs(lam / res["lam"] - 1).max() < 1e-10
    m = _gap_index(res["lam_all"], nev)
    assert _angle(U[:, :m], res["U"][:, :m]) < 1e-8
    assert np.abs(U.T @ U - np.eye(nev)).max() < 1e-10
    d = deg["d"].cpu().numpy()
    Bp = F[:, :k] / d[:, None]
    Bp[np.arange(k), np.arange(k)] += gamma
    E = eig["E"].cpu().numpy()[:k]
    assert np.abs(Bp @ E - U).max() < 1e-8


@pytest.mark.parametrize("N,k,nev,kind", [(20_000, 128, 16, "halfnormal"), (20_000, 200, 64, "uniform"),
                                          (5_000, 256, 64, "uniform")])
def test_eig_clustered_spectrum(gpu, N, k, nev, kind):
    """Factors with random entries: P~ then has one eigenvalue 1 and a flat
    rest (the leading 100 eigenvalues within a factor of 2), where the
    block iteration alone converges too slowly at the edge of its block; the
    spectral-projector restart (Newton-Schulz sign of M - sigma I at the
    widest Ritz gap) must deliver the top nev to the float64 bars."""
    torch, rp = gpu
    rng = np.random.default_rng(5)
    F = rng.random((N, k)) if kind == "uniform" else np.abs(rng.standard_normal((N, k)))
    F[:, 1:] -= 0.5 * F[:, 1:].mean(0)  # column 0 keeps every degree positive
    res = oracle.bistoch_eig(F, nev)
    ld = (N + 7) // 8 * 8
    buf = torch.zeros((k, ld), dtype=torch.float64, device="cuda")
    buf[:, :N] = torch.from_numpy(F.T.copy()).cuda()
    Fd = buf[:, :N].t()
    kd = torch.tensor([k], dtype=torch.int32, device="cuda")
    print(f"clustered N={N} k={k} nev={nev}", flush=True)
    deg = rp.bistoch_degrees(Fd, kd)
    assert rp.status_sync(deg["status"]) == 0
    eig = rp.bistoch_eig(Fd, kd, deg["d"], deg["q"], nev)
    st = rp.status_sync(eig["status"])
    assert st == 0, rp.STATUS_NAMES.get(st, st)
    lam = eig["lam"].cpu().numpy()
    le = np.abs(lam / res["lam"] - 1).max()
    m = _gap_index(res["lam_all"], nev)
    ae = _angle(eig["U"].cpu().numpy()[:, :m], res["U"][:, :m])
    print(f"clustered: lam[1] / lam[{nev}] = {res['lam'][1] / res['lam'][-1]:.3g}, eigenvalue error "
          f"{le:.3g}, angle {ae:.3g} over {m}")
    assert le < 1e-10 and ae < 1e-8


@pytest.mark.parametrize("r,b,nev,gamma,norm", [(64, 8, 16, 0.0, "bistochastic"), (160, 32, 24, 0.0, "bistochastic"),
                                                (160, 32, 24, 1e-3, "bistochastic"),
                                                (64, 8, 12, 0.0, "symmetric")])
def test_eig_cholqr2(gpu, r, b, nev, gamma, norm):
    """Cholesky QR2 (Q1 = B R1^{-1} formed, its Gram factored again, R = R2
    R1): eigenpairs against the oracle's Householder QR route to the float64
    bars, U orthonormal, and the extension identity U = B' E."""
    torch, rp = gpu
    X, eps = _torus_case(seed=17)
    u = uniform_stream(2 * b * (-(-r // b)), seed=17)
    ref = oracle.arpc(X, eps, r=r, b=b, mode="sampled", uniforms=u)
    out, k, F, piv, rho = _run_factor(gpu, X, eps, r, b, "sampled", u=u)
    deg = rp.bistoch_degrees(out["F"], out["k"])
    eig = rp.bistoch_eig(out["F"], out["k"], deg["d"], deg["q"], nev, gamma=gamma, normalization=norm,
                         qr_mode="cholqr2")
    assert rp.status_sync(eig["status"]) == 0
    res = (oracle.bistoch_eig(ref["F"], nev, gamma=gamma) if norm == "bistochastic"
           else oracle.symmetric_eig(ref["F"], nev))
    lam = eig["lam"].cpu().numpy()
    U = eig["U"].cpu().numpy()
    m = _gap_index(res["lam_all"], nev)
    le, ae = np.abs(lam / res["lam"] - 1).max(), _angle(U[:, :m], res["U"][:, :m])
    orth = np.abs(U.T @ U - np.eye(nev)).max()
    print(f"cholqr2 r={r} gamma={gamma} {norm}: eigenvalues {le:.3g}, angle {ae:.3g}, orthonormality {orth:.3g}")
    assert le < 1e-10 and ae < 1e-8 and orth < 1e-12
    d = deg["d"].cpu().numpy()
    Bp = F[:, :k] / (d if norm == "bistochastic" else np.sqrt(d))[:, None]
    Bp[np.arange(k), np.arange(k)] += gamma
    assert np.abs(Bp @ eig["E"].cpu().numpy()[:k] - U).max() < 1e-8


@pytest.mark.parametrize("pdt", ["f64", "bf16"])
def test_point_dtypes(gpu, pdt):
    """Points stored as float64 (values float32 cannot hold) or bf16: the
    float64 path sees the stored values exactly, so pivots, F, the degrees and
    the eigenpairs match the oracle run on the same values, and the Nystrom
    extension of new points of the same type matches the oracle's."""
    torch, rp = gpu
    X32 = torus_points(1500, seed=17)
    if pdt == "f64":
        Xh = X32.astype(np.float64) + np.random.default_rng(17).normal(scale=1e-6, size=X32.shape)
        assert np.abs(Xh - Xh.astype(np.float32)).max() > 0
        Xd = torch.from_numpy(Xh).cuda()
    else:
        Xd = torch.from_numpy(X32).cuda().to(torch.bfloat16)
        Xh = Xd.double().cpu().numpy()
    eps = median_sq_distance(Xh, seed=17)
    r, b, nev = 64, 8, 12
    u = uniform_stream(2 * b * (r // b), seed=17)
    ref = oracle.arpc(Xh, eps, r=r, b=b, mode="sampled", uniforms=u)
    out = rp.rpchol_factor(Xd, eps, r, b, uniforms=torch.from_numpy(u).cuda())
    deg = rp.bistoch_degrees(out["F"], out["k"], status=out["status"])
    eig = rp.bistoch_eig(out["F"], out["k"], deg["d"], deg["q"], nev, status=out["status"])
    assert rp.status_sync(out["status"]) == 0
    k = int(out["k"].item())
    assert k == ref["k"] and list(out["pivots"][:k].cpu().numpy()) == list(ref["S"])
    F = out["F"][:, :k].cpu().numpy()
    assert np.abs(F - ref["F"]).max() < 1e-12 * np.abs(ref["F"]).max()
    res = oracle.bistoch_eig(ref["F"], nev)
    assert np.abs(eig["lam"].cpu().numpy() / res["lam"] - 1).max() < 1e-10
    assert _angle(eig["U"].cpu().numpy(), res["U"]) < 1e-8
    Y32 = torus_points(300, seed=18)
    Yd = torch.from_numpy(Y32.astype(np.float64)).cuda() if pdt == "f64" else \
        torch.from_numpy(Y32).cuda().to(torch.bfloat16)
    Yh = Yd.double().cpu().numpy()
    ext = rp.nystrom_extend(Yd, Xd, eps, out["pivots"], out["k"], out["F"], deg["c"], eig["E"])
    assert rp.status_sync(ext["status"]) == 0
    Phi_o = oracle.nystrom_extend(Yh, Xh, ref["S"], ref["F"], res["c"], res["E"], eps)
    Phi = ext["Phi"].cpu().numpy()
    assert np.abs(Phi - Phi_o).max() < 1e-9 * np.abs(Phi_o).max()
