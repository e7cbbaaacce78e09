"""Pins of the surrogate oracle against definitions it does not share code with.

* GELU against torch's exact-erf GELU and its derivative against central
  differences.
* Every gradient against central finite differences of the loss.
* AdamW against torch.optim.AdamW (a separate implementation of the same
  published update).
* A short training run against torch autograd + torch.optim.AdamW on an
  nn.Sequential of the same architecture.
* bfloat16 rounding against torch's float32 -> bfloat16 conversion.
"""
import numpy as np
import pytest
import torch

from oracle import surrogate as S
from synth import uniform_stream


def _problem(B=7, d=6, h=8, n_out=3, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, d)) * 2.0 + 0.5
    T = rng.normal(size=(B, n_out))
    shapes = S.param_shapes(d, h, n_out)
    n = sum(int(np.prod(s)) for s in shapes.values())
    P = S.init_params(d, h, n_out, uniform_stream(n, seed=seed))
    mu, rs = S.standardize_stats(X)
    return (X - mu) * rs, T, P


def test_gelu_matches_torch_and_derivative():
    x = np.linspace(-6, 6, 1001)
    ref = torch.nn.functional.gelu(torch.from_numpy(x), approximate="none").numpy()
    assert np.max(np.abs(S.gelu(x) - ref)) < 1e-15
    h = 1e-5
    fd = (S.gelu(x + h) - S.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(S.gelu_prime(x) - fd)) < 1e-9


def _fd_check(lossfn, P, keys, h=1e-6, tol=1e-7):
    _, G = lossfn(P)
    for k in keys:
        it = np.nditer(P[k], flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            Pp = {a: b.copy() for a, b in P.items()}
            Pm = {a: b.copy() for a, b in P.items()}
            Pp[k][i] += h
            Pm[k][i] -= h
            fd = (lossfn(Pp)[0] - lossfn(Pm)[0]) / (2 * h)
            assert abs(fd - G[k][i]) < tol * max(1.0, abs(fd)), (k, i, fd, G[k][i])


def test_mse_gradients_match_finite_differences():
    Xn, T, P = _problem()
    _fd_check(lambda Q: S.mse_loss_grads(Q, Xn, T), P, S.BACKBONE)
    _, G = S.mse_loss_grads(P, Xn, T)
    assert not np.any(G["Wr"]) and not np.any(G["br"])


def test_residual_head_gradients_match_finite_differences():
    Xn, _, P = _problem(seed=5)
    tgt = np.linspace(-3, -1, Xn.shape[0])
    _fd_check(lambda Q: S.residual_loss_grads(Q, Xn, tgt), P, S.HEAD)
    _, G = S.residual_loss_grads(P, Xn, tgt)
    assert all(not np.any(G[k]) for k in S.BACKBONE)


def test_adamw_matches_torch():
    rng = np.random.default_rng(0)
    P = {"W": rng.normal(size=(4, 3)), "b": rng.normal(size=(4,))}
    tp = [torch.tensor(P["W"], requires_grad=True), torch.tensor(P["b"], requires_grad=True)]
    opt = torch.optim.AdamW(tp, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01)
    st = S.adamw_init(P)
    for t in range(1, 6):
        G = {"W": rng.normal(size=(4, 3)) * 10.0 ** (-t), "b": rng.normal(size=(4,))}
        tp[0].grad = torch.tensor(G["W"])
        tp[1].grad = torch.tensor(G["b"])
        opt.step()
        P = S.adamw_step(P, G, st, t, ("W", "b"))
        assert np.max(np.abs(P["W"] - tp[0].detach().numpy())) < 1e-14
        assert np.max(np.abs(P["b"] - tp[1].detach().numpy())) < 1e-14


def test_training_matches_torch_autograd():
    Xn, T, P = _problem(B=32, d=10, h=16, n_out=4, seed=11)
    rng = np.random.default_rng(1)
    batches = [rng.permutation(32)[:8] for _ in range(6)]
    net = torch.nn.Sequential(
        torch.nn.Linear(10, 16), torch.nn.GELU(), torch.nn.Linear(16, 16), torch.nn.GELU(),
        torch.nn.Linear(16, 4)).double()
    with torch.no_grad():
        for lin, (w, b) in zip([net[0], net[2], net[4]], [("W1", "b1"), ("W2", "b2"), ("W3", "b3")]):
            lin.weight.copy_(torch.from_numpy(P[w]))
            lin.bias.copy_(torch.from_numpy(P[b]))
    opt = torch.optim.AdamW(net.parameters(), lr=1e-3, weight_decay=0.01)
    tl = []
    for idx in batches:
        opt.zero_grad()
        loss = torch.nn.functional.mse_loss(net(torch.from_numpy(Xn[idx])), torch.from_numpy(T[idx]))
        loss.backward()
        opt.step()
        tl.append(loss.item())
    P2, losses = S.train(P, Xn, T, batches)
    assert np.allclose(losses, tl, rtol=1e-13, atol=0)
    for lin, (w, b) in zip([net[0], net[2], net[4]], [("W1", "b1"), ("W2", "b2"), ("W3", "b3")]):
        assert np.max(np.abs(P2[w] - lin.weight.detach().numpy())) < 1e-14
        assert np.max(np.abs(P2[b] - lin.bias.detach().numpy())) < 1e-14


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-20, 20, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0, 3.4e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).double().numpy()
    got = S.bf16_round(x)
    assert np.array_equal(got, ref)


def test_init_bounds_and_order():
    d, h, n_out = 5, 7, 3
    shapes = S.param_shapes(d, h, n_out)
    n = sum(int(np.prod(s)) for s in shapes.values())
    u = uniform_stream(n, seed=9)
    P = S.init_params(d, h, n_out, u)
    assert P["W1"].shape == (h, d) and P["br"].shape == (1,)
    assert np.max(np.abs(P["W1"])) <= 1 / np.sqrt(d) and np.max(np.abs(P["W2"])) <= 1 / np.sqrt(h)
    # first entry of W1 comes from the first uniform, first entry of b1 follows W1
    assert P["W1"][0, 0] == (2 * u[0] - 1) / np.sqrt(d)
    assert P["b1"][0] == (2 * u[h * d] - 1) / np.sqrt(d)
    with pytest.raises(ValueError):
        S.init_params(d, h, n_out, u[:-1])


def test_standardize_and_residual_target():
    X = np.array([[1.0, 2.0, 5.0], [3.0, 2.0, 7.0]])
    mu, rs = S.standardize_stats(X)
    assert np.allclose(mu, [2, 2, 6]) and np.allclose(rs, [1, 1, 1])
    Xn = (X - mu) * rs
    assert np.allclose(Xn, [[-1, 0, -1], [1, 0, 1]])
    yh = np.array([[1.0, 1.0, 1.0, 1.0]])
    yr = np.array([[1.1, 0.9, 1.1, 0.9]])
    assert np.isclose(S.residual_target(yh, yr)[0], -1.0)
