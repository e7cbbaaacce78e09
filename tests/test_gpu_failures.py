"""Device-side failure reports, forced from the host by the inputs.

Each case hands the library an input that violates one of the method's
conditions, so every kernel still runs to its normal end and only the status
word differs:
  * RPC_EDEGREE: a factor whose approximate degrees d~ = F F^T 1 are not all
    positive (the first assert of Algorithm 1);
  * RPC_EQDEGREE: d~ > 0 but q~ = F F^T D~^{-1} 1 not all positive (the
    second assert of Algorithm 1);
  * RPC_EBREAKDOWN: a replayed pivot list that repeats a point (its pivot
    block is singular), and a factor with a zero column inside the accepted
    rank (its Gram G_B is singular, so the Cholesky QR breaks down).
The oracle raises on the same degree inputs (checked here on the CPU too).
"""
import numpy as np
import pytest

import oracle
from oracle.bistoch import DegreeError
from synth import median_sq_distance, torus_points

pytestmark = pytest.mark.gpu

# d~ = (-1.5, 4.53, -0.69): negative degrees
F_BAD_D = [[1.0, 0.0], [-3.0, 0.1], [0.5, 0.2]]
# d~ > 0 everywhere, q~[0] = -0.065 (entries are multiples of 1/4: exact in float32)
F_BAD_Q = [[0.5, 1.0], [0.0, 0.75], [-0.5, 0.75], [-0.75, 0.75], [-0.25, 0.25], [-0.75, -0.25]]


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_26574_amd as rp

    rp.load_library()
    return torch, rp


def _colmajor(torch, F, dtype):
    F = np.asarray(F, dtype=np.float64)
    N, r = F.shape
    ld = (N + 7) // 8 * 8
    buf = torch.zeros((r, ld), dtype=dtype, device="cuda")
    buf[:, :N] = torch.from_numpy(F.T.copy()).to(dtype)
    return buf[:, :N].t()


@pytest.mark.parametrize("fdt", ["f64", "f32"])
@pytest.mark.parametrize("F,code", [(F_BAD_D, "RPC_EDEGREE"), (F_BAD_Q, "RPC_EQDEGREE")])
def test_degree_asserts(gpu, fdt, F, code):
    torch, rp = gpu
    with pytest.raises(DegreeError):
        oracle.bistoch_degrees(np.asarray(F))
    Fd = _colmajor(torch, F, torch.float64 if fdt == "f64" else torch.float32)
    k = torch.tensor([Fd.shape[1]], dtype=torch.int32, device="cuda")
    print(f"degrees {code} {fdt}", flush=True)
    deg = rp.bistoch_degrees(Fd, k)
    assert rp.STATUS_NAMES[rp.status_sync(deg["status"])] == code


def test_replayed_repeated_pivot_breaks_down(gpu):
    torch, rp = gpu
    X = torus_points(500, seed=3)
    eps = median_sq_distance(X, seed=3)
    rep = torch.tensor([17, 250, 17, 400], dtype=torch.int64, device="cuda")
    print("replay with a repeated pivot", flush=True)
    out = rp.rpchol_factor(torch.from_numpy(X).cuda(), eps, 8, 4, mode="replay", replay=rep)
    assert rp.STATUS_NAMES[rp.status_sync(out["status"])] == "RPC_EBREAKDOWN"


def test_singular_gram_breaks_down(gpu):
    torch, rp = gpu
    rng = np.random.default_rng(4)
    F = np.abs(rng.standard_normal((300, 8)))
    F[:, 3] = 0.0  # a zero column inside the accepted rank: G_B is singular
    Fd = _colmajor(torch, F, torch.float64)
    k = torch.tensor([8], dtype=torch.int32, device="cuda")
    deg = rp.bistoch_degrees(Fd, k)
    assert rp.status_sync(deg["status"]) == 0
    print("singular Gram", flush=True)
    eig = rp.bistoch_eig(Fd, k, deg["d"], deg["q"], 4)
    assert rp.STATUS_NAMES[rp.status_sync(eig["status"])] == "RPC_EBREAKDOWN"
