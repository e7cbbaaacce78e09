"""bistoch_degrees_noalloc (library-owned static scratch, no workspace)
against bistoch_degrees (caller workspace) through the C-ABI: bit for bit,
on two calls in a row, the second with a smaller input, both factor types."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_26574_amd as rp

    rp.load_library()
    return torch, rp


def _factor(torch, N, r, k, dtype, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    ld = (N + 7) // 8 * 8
    buf = torch.rand((r, ld), generator=g, dtype=torch.float64, device="cuda").to(dtype)
    buf[k:] = 0  # columns >= k are zero, as rpchol_factor leaves them
    return buf[:, :N].t(), torch.tensor([k], dtype=torch.int32, device="cuda")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_degrees_match_workspace_form(gpu, dtype):
    torch, rp = gpu
    tdt = torch.float64 if dtype == "f64" else torch.float32
    for N, r, k, seed in [(1_048_576, 1024, 1000, 1), (3001, 40, 37, 2)]:
        print(f"noalloc degrees {dtype} N={N} r={r} k={k}", flush=True)
        F, kd = _factor(torch, N, r, k, tdt, seed)
        ref = rp.bistoch_degrees(F, kd)
        assert rp.status_sync(ref["status"]) == 0
        c = torch.full((r,), float("nan"), dtype=torch.float64, device="cuda")
        d = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
        q = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        rp.bistoch_degrees_noalloc(F, kd, c, d, q, st)
        assert rp.status_sync(st) == 0
        assert torch.equal(c, ref["c"]) and torch.equal(d, ref["d"]) and torch.equal(q, ref["q"])


def test_noalloc_rejects_sizes_above_the_limit(gpu):
    torch, rp = gpu
    F, kd = _factor(torch, 16, 8, 8, torch.float64, 3)
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    lib = rp.load_library()
    s = rp._stream(torch, None)
    for N, r in [(1_048_577, 8), (2_000_000, 1025)]:
        rc = lib.bistoch_degrees_noalloc(rp._ptr(F), 0, N, N + 7, r, rp._ptr(kd), rp._ptr(one),
                                         rp._ptr(one), rp._ptr(one), rp._ptr(st), s)
        assert rc == rp.RPC_EWORKSPACE
