"""Learned surrogate of the Nystrom extension (oracle; test infrastructure only).

The paper's Nystrom extension (Section "Nystrom method connection") maps a new
state y to the values of the approximate eigenvectors at y.  The surrogate is a
small multilayer perceptron trained to reproduce that map at the training
points (targets sqrt(N) U, i.e. eigenfunction values of order one), with a
second, scalar head that predicts the log10 RMS error of the first head so a
caller can fall back to the exact Nystrom formula where the network is
unreliable.

Definitions this module writes out in float64 (no blocking, no fusion):

* two hidden layers with the exact GELU, x Phi(x), Phi the standard normal
  CDF (Hendrycks & Gimpel, "Gaussian error linear units", 2016);
* linear output layer of width n_out and a linear residual head (one unit)
  on the last hidden layer;
* loss: mean squared error over the batch and the n_out outputs; residual
  head loss: mean squared error of the predicted log10 RMS error;
* AdamW with decoupled weight decay and bias-corrected moments (Loshchilov &
  Hutter, "Decoupled weight decay regularization", ICLR 2019); decay applies
  to every trained parameter, biases included;
* initialisation: every weight and bias uniform on +-1/sqrt(fan_in), drawn
  from a caller-supplied uniform stream in the order W1, b1, W2, b2, W3, b3,
  Wr, br (row-major within a matrix);
* inputs standardised per feature (population standard deviation; a constant
  feature keeps scale 1).

`quant` arguments take a rounding function applied wherever the reduced
precision form rounds a product operand (inputs, weights, hidden activations
and back-propagated errors rounded to bfloat16, everything else exact); the
default is exact float64.
"""
import numpy as np
from scipy.special import erf

SQRT2 = np.sqrt(2.0)
INV_SQRT_2PI = 1.0 / np.sqrt(2.0 * np.pi)


def _ident(x):
    return x


def bf16_round(x):
    """Round to bfloat16 (round to nearest even) after rounding to float32,
    returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def gelu(x):
    """Exact GELU: x Phi(x) = x (1 + erf(x / sqrt 2)) / 2."""
    return 0.5 * x * (1.0 + erf(x / SQRT2))


def gelu_prime(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / SQRT2)) + x * INV_SQRT_2PI * np.exp(-0.5 * x * x)


PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3", "Wr", "br")


def param_shapes(d, h, n_out):
    return {"W1": (h, d), "b1": (h,), "W2": (h, h), "b2": (h,), "W3": (n_out, h), "b3": (n_out,),
            "Wr": (1, h), "br": (1,)}


def init_params(d, h, n_out, uniforms):
    """Uniform(+-1/sqrt(fan_in)) initialisation from the uniform stream."""
    shapes = param_shapes(d, h, n_out)
    fan = {"W1": d, "b1": d, "W2": h, "b2": h, "W3": h, "b3": h, "Wr": h, "br": h}
    u = np.asarray(uniforms, dtype=np.float64)
    need = sum(int(np.prod(s)) for s in shapes.values())
    if u.size < need:
        raise ValueError(f"need {need} uniforms, got {u.size}")
    P, o = {}, 0
    for name in PARAM_ORDER:
        n = int(np.prod(shapes[name]))
        a = 1.0 / np.sqrt(fan[name])
        P[name] = ((2.0 * u[o:o + n] - 1.0) * a).reshape(shapes[name])
        o += n
    return P


def standardize_stats(X):
    """Per-feature mean and reciprocal population standard deviation."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    rs = np.where(sd > 0, 1.0 / np.where(sd > 0, sd, 1.0), 1.0)
    return mu, rs


def forward(P, Xn, quant=_ident):
    """Hidden pre-activations, activations, outputs and the residual head."""
    q = quant
    x = q(Xn)
    z1 = x @ q(P["W1"]).T + P["b1"]
    a1 = gelu(z1)
    z2 = q(a1) @ q(P["W2"]).T + P["b2"]
    a2 = gelu(z2)
    y = q(a2) @ q(P["W3"]).T + P["b3"]
    res = (q(a2) @ q(P["Wr"]).T + P["br"])[:, 0]
    return {"x": x, "z1": z1, "a1": a1, "z2": z2, "a2": a2, "y": y, "res": res}


def mse_loss_grads(P, Xn, T, quant=_ident):
    """Loss mean((y - T)^2) and its gradient for W1..b3 (residual head: zero)."""
    q = quant
    f = forward(P, Xn, quant)
    B, n_out = f["y"].shape
    diff = f["y"] - T
    loss = float(np.mean(diff * diff))
    gy = q(2.0 * diff / (B * n_out))
    G = {}
    G["W3"] = gy.T @ q(f["a2"])
    G["b3"] = gy.sum(axis=0)
    g2 = q((gy @ q(P["W3"])) * gelu_prime(f["z2"]))
    G["W2"] = g2.T @ q(f["a1"])
    G["b2"] = g2.sum(axis=0)
    g1 = q((g2 @ q(P["W2"])) * gelu_prime(f["z1"]))
    G["W1"] = g1.T @ f["x"]
    G["b1"] = g1.sum(axis=0)
    G["Wr"] = np.zeros_like(P["Wr"])
    G["br"] = np.zeros_like(P["br"])
    return loss, G


def residual_loss_grads(P, Xn, target, quant=_ident):
    """Residual-head loss mean((res - target)^2) and its gradient (head only;
    the backbone is held fixed)."""
    q = quant
    f = forward(P, Xn, quant)
    B = f["res"].shape[0]
    diff = f["res"] - target
    loss = float(np.mean(diff * diff))
    gr = q(2.0 * diff / B)
    G = {k: np.zeros_like(v) for k, v in P.items()}
    G["Wr"] = (gr @ q(f["a2"]))[None, :]
    G["br"] = np.array([gr.sum()])
    return loss, G


def residual_target(yhat, yref):
    """log10 of the per-point RMS difference over the outputs."""
    d = np.asarray(yhat, dtype=np.float64) - np.asarray(yref, dtype=np.float64)
    return np.log10(np.sqrt(np.mean(d * d, axis=1)))


def adamw_init(P):
    return {"m": {k: np.zeros_like(v) for k, v in P.items()},
            "v": {k: np.zeros_like(v) for k, v in P.items()}}


def adamw_step(P, G, state, t, keys, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.01):
    """One AdamW update (step number t >= 1) of the parameters named in keys."""
    Pn = dict(P)
    for k in keys:
        g = G[k]
        m = beta1 * state["m"][k] + (1.0 - beta1) * g
        v = beta2 * state["v"][k] + (1.0 - beta2) * g * g
        state["m"][k], state["v"][k] = m, v
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        Pn[k] = P[k] - lr * wd * P[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return Pn


BACKBONE = ("W1", "b1", "W2", "b2", "W3", "b3")
HEAD = ("Wr", "br")


def train(P, Xn, T, batches, quant=_ident, **hyper):
    """Train the backbone and output layer over the given list of batch index
    arrays (one AdamW step each).  Returns the parameters and the losses."""
    state = adamw_init(P)
    losses = []
    for t, idx in enumerate(batches, start=1):
        loss, G = mse_loss_grads(P, Xn[idx], T[idx], quant)
        P = adamw_step(P, G, state, t, BACKBONE, **hyper)
        losses.append(loss)
    return P, losses
