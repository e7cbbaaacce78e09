"""Batched form: many decompositions overlapped over streams, and captured
into a HIP graph, against the same decompositions made one call at a time
(bit-identical: the same kernels on the same inputs) and against the oracle.
"""
import numpy as np
import pytest

import oracle
from synth import ks_points, median_sq_distance, torus_points, uniform_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_26574_amd as rp

    rp.load_library()
    return torch, rp


def _datasets(torch):
    """A few small problems of different shapes (torus d = 3, KS d = 32 / 128)."""
    out = []
    X = torus_points(1500, seed=1)
    out.append((torch.from_numpy(X).cuda(), median_sq_distance(X, seed=1)))
    X = ks_points(2500, q=1, seed=2)[:, :32].copy()
    out.append((torch.from_numpy(X).cuda(), median_sq_distance(X, seed=2)))
    X = ks_points(4000, q=2, seed=3)
    out.append((torch.from_numpy(X).cuda(), median_sq_distance(X, seed=3)))
    return out


def _jobs(torch, rp, data, dtypes=("f32", "f32", "f32", "f32")):
    g, f, gr, ud = dtypes
    jobs = []
    for i, (X, eps) in enumerate(data):
        for m, (r, b) in zip([0.5, 1.0, 4.0], [(64, 16), (96, 32), (128, 32)]):
            u = torch.from_numpy(uniform_stream(2 * r, seed=10 * i + int(m * 2))).cuda()
            jobs.append(rp.Job(X, m * eps, r, b, 8, uniforms=u, gemm_dtype=g, factor_dtype=f,
                               gram_dtype=gr, u_dtype=ud))
    return jobs


def _outputs(j):
    """The defined outputs (F and U without their leading-dimension padding)."""
    return [t.clone() for t in (j.F, j.pivots, j.rho, j.k, j.c, j.d, j.q, j.U, j.lam, j.Ebuf)]


def _single(rp, j):
    out = rp.rpchol_factor(j.X, j.rec.X.eps, j.rec.factor.r, j.rec.factor.b, uniforms=j.uniforms,
                           gemm_dtype="f32", factor_dtype="f32")
    deg = rp.bistoch_degrees(out["F"], out["k"], status=out["status"])
    eig = rp.bistoch_eig(out["F"], out["k"], deg["d"], deg["q"], j.rec.eig.nev, gram_dtype="f32",
                         u_dtype="f32", status=out["status"])
    assert rp.status_sync(out["status"]) == 0
    return out, deg, eig


def test_batched_equals_single_calls(gpu):
    torch, rp = gpu
    jobs = _jobs(torch, rp, _datasets(torch))
    rp.batched_run(jobs, n_streams=4)
    torch.cuda.synchronize()
    for j in jobs:
        assert int(j.status.item()) == 0
        out, deg, eig = _single(rp, j)
        N = j.X.shape[0]
        assert torch.equal(j.pivots, out["pivots"]) and torch.equal(j.k, out["k"])
        assert torch.equal(j.F, out["F"]) and torch.equal(j.rho, out["rho"])
        assert torch.equal(j.d, deg["d"]) and torch.equal(j.q, deg["q"])
        assert torch.equal(j.lam, eig["lam"]) and torch.equal(j.U[:, :8], eig["U"][:N])


def test_batched_graph_replays(gpu):
    torch, rp = gpu
    jobs = _jobs(torch, rp, _datasets(torch))
    rp.batched_run(jobs, n_streams=3)
    torch.cuda.synchronize()
    ref = [_outputs(j) for j in jobs]
    g = rp.BatchedGraph(jobs, n_streams=3)
    for rep in range(3):
        for j in jobs:  # wipe the outputs between replays (eager work on the device)
            for t in (j.Fbuf, j.pivots, j.rho, j.Ubuf, j.lam):
                t.fill_(-7)
        torch.cuda.synchronize()
        g.launch()
        g.synchronize()
        for j, r in zip(jobs, ref):
            assert int(j.status.item()) == 0
            for a, b in zip(_outputs(j), r):
                assert torch.equal(a, b), rep
    g.close()


def test_batched_job_matches_oracle(gpu):
    torch, rp = gpu
    X = torus_points(1200, seed=5)
    eps = median_sq_distance(X, seed=5)
    u = uniform_stream(2 * 48, seed=5)
    Xd = torch.from_numpy(X).cuda()
    jobs = [rp.Job(Xd, eps * m, 48, 8, 6, uniforms=torch.from_numpy(u).cuda(), gemm_dtype="f64",
                   factor_dtype="f64", gram_dtype="f64", u_dtype="f64") for m in (0.5, 2.0)]
    rp.batched_run(jobs, n_streams=2)
    torch.cuda.synchronize()
    for j, m in zip(jobs, (0.5, 2.0)):
        assert int(j.status.item()) == 0
        ref = oracle.arpc(X, eps * m, r=48, b=8, mode="sampled", uniforms=u)
        k = ref["k"]
        assert int(j.k.item()) == k
        assert np.array_equal(j.pivots.cpu().numpy()[:k], ref["S"])
        F = j.F.cpu().numpy()[:, :k]
        assert np.abs(F - ref["F"]).max() <= 1e-12 * np.abs(ref["F"]).max()
        res = oracle.bistoch_eig(ref["F"], 6)
        lam = j.lam.cpu().numpy()
        assert np.max(np.abs(lam - res["lam"]) / res["lam"]) < 1e-10


def test_autotune_block(gpu):
    torch, rp = gpu
    X = ks_points(3000, q=2, seed=4)
    eps = median_sq_distance(X, seed=4)
    u = torch.from_numpy(uniform_stream(2 * 128, seed=4)).cuda()
    j = rp.Job(torch.from_numpy(X).cuda(), eps, 128, 32, 8, uniforms=u)
    best, ms = rp.autotune_block(j, [16, 32, 64], reps=1)
    assert best in (16, 32, 64) and all(v > 0 for v in ms.values())
    assert ms[best] == min(ms.values())


def test_batched_rejects_bad_arguments(gpu):
    torch, rp = gpu
    data = _datasets(torch)[:1]
    jobs = _jobs(torch, rp, data)
    with pytest.raises(rp.RpcError):
        rp.batched_run(jobs, n_streams=33)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(rp.RpcError):
        rp.batched_run(jobs, n_streams=2, workspace=ws)


# ---- several bandwidths on shared points (rpchol_factor_group)

def _group_case(torch, n=2500, q=1, seed=7, d=32):
    X = ks_points(n, q=q, seed=seed)[:, :d].copy()
    return X, median_sq_distance(X, seed=seed)


@pytest.mark.parametrize("gdt", ["f32", "bf16"])
def test_group_equals_single_calls(gpu, gdt):
    """Each job of a group equals the same job factorised alone with the
    shared-points flag (the two-kernel column/Schur arithmetic), bit for bit."""
    torch, rp = gpu
    X, eps = _group_case(torch, n=2500, q=2, seed=8, d=64)
    Xd = torch.from_numpy(X).cuda()
    r, b = 96, 32
    mults = [0.5, 1.0, 2.0, 4.0]
    us = [torch.from_numpy(uniform_stream(2 * r, seed=40 + i)).cuda() for i in range(len(mults))]
    outs = rp.rpchol_factor_group(Xd, [m * eps for m in mults], r, b, us, gemm_dtype=gdt, factor_dtype="f32")
    for o, m, u in zip(outs, mults, us):
        assert rp.status_sync(o["status"]) == 0
        s = rp.rpchol_factor(Xd, m * eps, r, b, uniforms=u, gemm_dtype=gdt, factor_dtype="f32", shared_x=True)
        assert rp.status_sync(s["status"]) == 0
        assert torch.equal(o["k"], s["k"]) and torch.equal(o["pivots"], s["pivots"])
        assert torch.equal(o["F"], s["F"]) and torch.equal(o["rho"], s["rho"])
        assert torch.equal(o["round_accepted"], s["round_accepted"])


def test_group_matches_oracle(gpu):
    torch, rp = gpu
    X = torus_points(1300, seed=9)
    eps = median_sq_distance(X, seed=9)
    Xd = torch.from_numpy(X).cuda()
    r, b = 48, 8
    mults = [0.25, 1.0, 4.0]
    u = [uniform_stream(2 * r, seed=50 + i) for i in range(3)]
    outs = rp.rpchol_factor_group(Xd, [m * eps for m in mults], r, b, [torch.from_numpy(x).cuda() for x in u],
                                  gemm_dtype="f64", factor_dtype="f64")
    for o, m, ui in zip(outs, mults, u):
        assert rp.status_sync(o["status"]) == 0
        ref = oracle.arpc(X, m * eps, r=r, b=b, mode="sampled", uniforms=ui)
        k = ref["k"]
        assert int(o["k"].item()) == k
        assert np.array_equal(o["pivots"].cpu().numpy()[:k], ref["S"])
        F = o["F"].cpu().numpy()[:, :k]
        assert np.abs(F - ref["F"]).max() <= 1e-12 * np.abs(ref["F"]).max()
        assert not o["F"][:, k:].any().item()


def test_batched_shared_points(gpu):
    """Jobs on the same points at several bandwidths run as groups inside the
    batched form; each equals its single call with the shared-points flag,
    also after graph replays."""
    torch, rp = gpu
    data = _datasets(torch)
    jobs = []
    for i, (X, eps) in enumerate(data[:2]):
        for m in (0.5, 1.0, 2.0):
            u = torch.from_numpy(uniform_stream(2 * 96, seed=60 + 10 * i + int(4 * m))).cuda()
            jobs.append(rp.Job(X, m * eps, 96, 32, 8, uniforms=u, shared_x=True))
    # a job on other points and one without the flag stay on their own
    X2, eps2 = data[2]
    jobs.append(rp.Job(X2, eps2, 64, 16, 8, uniforms=torch.from_numpy(uniform_stream(128, seed=70)).cuda(),
                       shared_x=True))
    jobs.append(rp.Job(data[0][0], data[0][1], 64, 16, 8,
                       uniforms=torch.from_numpy(uniform_stream(128, seed=71)).cuda()))
    rp.batched_run(jobs, n_streams=3)
    torch.cuda.synchronize()
    ref = []
    for j in jobs:
        assert int(j.status.item()) == 0
        shared = bool(j.rec.factor.flags & rp.RPC_FACTOR_SHARED_X)
        out = rp.rpchol_factor(j.X, j.rec.X.eps, j.rec.factor.r, j.rec.factor.b, uniforms=j.uniforms,
                               gemm_dtype="f32", factor_dtype="f32", shared_x=shared)
        deg = rp.bistoch_degrees(out["F"], out["k"], status=out["status"])
        eig = rp.bistoch_eig(out["F"], out["k"], deg["d"], deg["q"], 8, gram_dtype="f32", u_dtype="f32",
                             status=out["status"])
        assert rp.status_sync(out["status"]) == 0
        assert torch.equal(j.pivots, out["pivots"]) and torch.equal(j.F, out["F"])
        assert torch.equal(j.lam, eig["lam"])
        ref.append(_outputs(j))
    g = rp.BatchedGraph(jobs, n_streams=3)
    for rep in range(2):
        for j in jobs:
            for t in (j.Fbuf, j.pivots, j.rho, j.Ubuf, j.lam):
                t.fill_(-7)
        torch.cuda.synchronize()
        g.launch()
        g.synchronize()
        for j, r0 in zip(jobs, ref):
            assert int(j.status.item()) == 0
            for a, b2 in zip(_outputs(j), r0):
                assert torch.equal(a, b2), rep
    g.close()
