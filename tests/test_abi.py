"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/rpchol.h, and rejects bad arguments on the host."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpchol.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2510_26574_amd as rp

    if not os.path.exists(rp.LIB_PATH):
        pytest.skip("library not built")
    return rp.load_library()


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ["rpchol_factor", "bistoch_degrees", "bistoch_eig", "nystrom_extend"]:
        assert n in names and n + "_workspace_size" in names


def test_every_declared_symbol_is_exported(lib):
    for n in _declared():
        assert hasattr(lib, n), n


def test_version_string(lib):
    assert b"gfx950" in lib.rpc_version()


def test_host_side_validation(lib):
    import paper_2510_26574_amd as rp

    pts = rp.rpc_points(100, 3, 3, 0x1000, 1.0)
    opts = rp.rpc_factor_opts(8, 2, rp.MODES["sampled"], 0, 0, 0, 0.0, 0x2000, 64, 0, 0, 0)
    nb = ctypes.c_size_t(0)
    assert lib.rpchol_factor_workspace_size(ctypes.byref(pts), ctypes.byref(opts), ctypes.byref(nb)) == 0
    assert nb.value > 0
    bad = [
        dict(r=101),           # r > N
        dict(b=0),             # b < 1
        dict(b=129),           # b above the supported block
        dict(mode=1),          # greedy with b != 1
        dict(n_uniforms=10),   # too few uniforms
        dict(gemm_dtype=7),
        dict(factor_dtype=2),  # bf16 storage of F is not offered
    ]
    for kw in bad:
        o = rp.rpc_factor_opts(8, 2, rp.MODES["sampled"], 0, 0, 0, 0.0, 0x2000, 64, 0, 0, 0)
        for k, v in kw.items():
            setattr(o, k, v)
        assert lib.rpchol_factor_workspace_size(ctypes.byref(pts), ctypes.byref(o), ctypes.byref(nb)) == rp.RPC_EINVAL, kw
    p2 = rp.rpc_points(100, 3, 3, 0x1000, 0.0)  # eps <= 0
    assert lib.rpchol_factor_workspace_size(ctypes.byref(p2), ctypes.byref(opts), ctypes.byref(nb)) == rp.RPC_EINVAL
    eo = rp.rpc_eig_opts(200, 0, 0, 0, 0.0)  # nev > r
    assert lib.bistoch_eig_workspace_size(1000, 64, ctypes.byref(eo), ctypes.byref(nb)) == rp.RPC_EINVAL
    eo = rp.rpc_eig_opts(16, 0, 0, 0, 0.0)
    assert lib.bistoch_eig_workspace_size(1000, 64, ctypes.byref(eo), ctypes.byref(nb)) == 0
    assert lib.nystrom_extend_workspace_size(10, 3, 64, 65, ctypes.byref(nb)) == rp.RPC_EINVAL
