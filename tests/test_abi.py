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
        dict(flags=16),        # unknown option bit
        dict(flags=8),         # split solve: bf16 products with a float32 factor only
        dict(gemm_dtype=3),    # split-fp16 distances need a float32 factor
    ]
    for kw in bad:
        o = rp.rpc_factor_opts(8, 2, rp.MODES["sampled"], 0, 0, 0, 0.0, 0x2000, 64, 0, 0, 0)
        for k, v in kw.items():
            setattr(o, k, v)
        assert lib.rpchol_factor_workspace_size(ctypes.byref(pts), ctypes.byref(o), ctypes.byref(nb)) == rp.RPC_EINVAL, kw
    p3 = rp.rpc_points(100, 3, 3, 0x1000, 1.0, 3)  # points dtype: f32, f64 or bf16 only
    assert lib.rpchol_factor_workspace_size(ctypes.byref(p3), ctypes.byref(opts), ctypes.byref(nb)) == -1
    for dt in (0, 1, 2):
        p4 = rp.rpc_points(100, 3, 3, 0x1000, 1.0, dt)
        assert lib.rpchol_factor_workspace_size(ctypes.byref(p4), ctypes.byref(opts), ctypes.byref(nb)) == 0
    p2 = rp.rpc_points(100, 3, 3, 0x1000, 0.0)  # eps <= 0
    assert lib.rpchol_factor_workspace_size(ctypes.byref(p2), ctypes.byref(opts), ctypes.byref(nb)) == rp.RPC_EINVAL
    eo = rp.rpc_eig_opts(200, 0, 0, 0, 0, 0, 0.0)  # nev > r
    assert lib.bistoch_eig_workspace_size(1000, 64, ctypes.byref(eo), ctypes.byref(nb)) == rp.RPC_EINVAL
    eo = rp.rpc_eig_opts(16, 0, 0, 0, 0, 0, 0.0)
    assert lib.bistoch_eig_workspace_size(1000, 64, ctypes.byref(eo), ctypes.byref(nb)) == 0
    eo = rp.rpc_eig_opts(16, 0, rp.DTYPES["split16"], 1, 0, 0, 0.0)  # split-fp16 Gram
    assert lib.bistoch_eig_workspace_size(1000, 64, ctypes.byref(eo), ctypes.byref(nb)) == 0
    for bad in (dict(normalization=2), dict(normalization=1, fix_const=1), dict(qr_mode=2),
                dict(gram_dtype=4), dict(u_dtype=rp.DTYPES["split16"])):
        eo = rp.rpc_eig_opts(16, 0, 0, 0, 0, 0, 0.0)
        for kk, v in bad.items():
            setattr(eo, kk, v)
        assert lib.bistoch_eig_workspace_size(1000, 64, ctypes.byref(eo), ctypes.byref(nb)) == rp.RPC_EINVAL, bad
    assert lib.nystrom_extend_workspace_size(10, 3, 64, 65, ctypes.byref(nb)) == rp.RPC_EINVAL
    o = rp.rpc_factor_opts(8, 2, rp.MODES["sampled"], 0, 0, rp.RPC_FACTOR_UNFUSED, 0.0, 0x2000, 64, 0, 0, 0)
    assert lib.rpchol_factor_workspace_size(ctypes.byref(pts), ctypes.byref(o), ctypes.byref(nb)) == 0
    o = rp.rpc_factor_opts(8, 2, rp.MODES["sampled"], rp.DTYPES["split16"], rp.DTYPES["f32"], 0, 0.0,
                           0x2000, 64, 0, 0, 0)  # split-fp16 distances, float32 factor
    assert lib.rpchol_factor_workspace_size(ctypes.byref(pts), ctypes.byref(o), ctypes.byref(nb)) == 0
    o.flags = rp.RPC_FACTOR_SHARED_X  # not offered for a group on shared points
    assert lib.rpchol_factor_group_workspace_size(ctypes.byref(pts), ctypes.byref(o), 2,
                                                  ctypes.byref(nb)) == rp.RPC_EINVAL
    # low-memory form: float64 factor only, not on shared points; its workspace
    # holds two column blocks instead of the N x r factor
    o = rp.rpc_factor_opts(8, 2, rp.MODES["sampled"], rp.DTYPES["bf16"], rp.DTYPES["f64"],
                           rp.RPC_FACTOR_LOW_MEMORY, 0.0, 0x2000, 64, 0, 0, 0)
    assert lib.rpchol_factor_workspace_size(ctypes.byref(pts), ctypes.byref(o), ctypes.byref(nb)) == 0
    o.factor_dtype = rp.DTYPES["f32"]
    assert lib.rpchol_factor_workspace_size(ctypes.byref(pts), ctypes.byref(o), ctypes.byref(nb)) == rp.RPC_EINVAL
    o.factor_dtype = rp.DTYPES["f64"]
    o.flags = rp.RPC_FACTOR_LOW_MEMORY | rp.RPC_FACTOR_SHARED_X
    assert lib.rpchol_factor_workspace_size(ctypes.byref(pts), ctypes.byref(o), ctypes.byref(nb)) == rp.RPC_EINVAL
    big = rp.rpc_points(1_000_000, 512, 512, 0x1000, 1.0)
    full = rp.rpc_factor_opts(1024, 128, rp.MODES["sampled"], rp.DTYPES["bf16"], rp.DTYPES["f64"], 0,
                              0.0, 0x2000, 2048, 0, 0, 0)
    low = rp.rpc_factor_opts(1024, 128, rp.MODES["sampled"], rp.DTYPES["bf16"], rp.DTYPES["f64"],
                             rp.RPC_FACTOR_LOW_MEMORY, 0.0, 0x2000, 2048, 0, 0, 0)
    nf, nl = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.rpchol_factor_workspace_size(ctypes.byref(big), ctypes.byref(full), ctypes.byref(nf)) == 0
    assert lib.rpchol_factor_workspace_size(ctypes.byref(big), ctypes.byref(low), ctypes.byref(nl)) == 0
    # full form: workspace + the caller's N x r float64 factor (8.2 GB); low-memory
    # form: workspace + an r x r factor
    assert nl.value + 1024 * 1024 * 8 < nf.value + 1_000_000 * 1024 * 8 - 4 * 10**9
    # group of factorisations on shared points: sizes and option checks (host side only)
    og = rp.rpc_factor_opts(8, 2, rp.MODES["sampled"], 0, 0, rp.RPC_FACTOR_SHARED_X, 0.0, 0x2000, 64, 0, 0, 0)
    n1 = ctypes.c_size_t(0)
    assert lib.rpchol_factor_group_workspace_size(ctypes.byref(pts), ctypes.byref(og), 1, ctypes.byref(n1)) == 0
    n4 = ctypes.c_size_t(0)
    assert lib.rpchol_factor_group_workspace_size(ctypes.byref(pts), ctypes.byref(og), 4, ctypes.byref(n4)) == 0
    assert n1.value < n4.value < 4 * n1.value  # the converted points are shared
    for g in (0, 17):
        assert lib.rpchol_factor_group_workspace_size(ctypes.byref(pts), ctypes.byref(og), g,
                                                      ctypes.byref(n1)) == rp.RPC_EINVAL
    og2 = rp.rpc_factor_opts(16, 2, rp.MODES["sampled"], 0, 0, rp.RPC_FACTOR_SHARED_X, 0.0, 0x2000, 64, 0, 0, 0)
    og3 = rp.rpc_factor_opts(8, 2, rp.MODES["sampled"], 0, 0, 0, 0.0, 0x2000, 64, 0, 0, 0)
    eps2 = (ctypes.c_double * 2)(1.0, 2.0)
    fake = (ctypes.c_void_p * 2)(0x4000, 0x5000)
    for other in (og2, og3):  # different r; SHARED_X missing
        opts2 = (ctypes.c_void_p * 2)(ctypes.addressof(og), ctypes.addressof(other))
        rc = lib.rpchol_factor_group(ctypes.byref(pts), ctypes.cast(eps2, ctypes.c_void_p),
                                     ctypes.cast(opts2, ctypes.c_void_p), 2, ctypes.cast(fake, ctypes.c_void_p),
                                     104, ctypes.cast(fake, ctypes.c_void_p), ctypes.cast(fake, ctypes.c_void_p),
                                     ctypes.cast(fake, ctypes.c_void_p), ctypes.cast(fake, ctypes.c_void_p),
                                     None, 0, None)
        assert rc == rp.RPC_EINVAL


def test_noalloc_degrees_host_checks(lib):
    """The no-allocation degrees call refuses sizes beyond its static scratch
    (N > 2^20 or r > 1024) before touching a device, and bad arguments."""
    import paper_2510_26574_amd as rp

    fake = ctypes.c_void_p(0x1000)
    for N, r, rc in [(1_048_577, 8, rp.RPC_EWORKSPACE), (2_000_000, 1025, rp.RPC_EWORKSPACE),
                     (100, 101, rp.RPC_EINVAL), (100, 8, rp.RPC_EINVAL)]:
        fdt = 0 if N != 100 or r != 8 else 7  # the last case: unknown dtype
        assert lib.bistoch_degrees_noalloc(fake, fdt, N, N + 8, r, fake, fake, fake, fake, fake,
                                           None) == rc


def test_surrogate_and_batched_host_checks(lib):
    import paper_2510_26574_amd as rp

    lay = rp.surrogate_layout(512, 512, 64)
    assert lay["n3"] == 80 and lay["total"] % 64 == 0
    assert all(lay[k] % 64 == 0 for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    assert lay["b3"] + lay["n3"] <= lay["total"]
    assert rp.surrogate_init_uniforms(512, 512, 64) == 512 * 512 * 2 + 512 * 2 + 64 * 512 + 64 + 512 + 1
    sh = rp.sur_shape(512, 512, 64)
    nb = ctypes.c_size_t(0)
    assert lib.surrogate_train_workspace_size(ctypes.byref(sh), 4096, 0, ctypes.byref(nb)) == 0
    assert lib.surrogate_train_workspace_size(ctypes.byref(sh), 70000, 0, ctypes.byref(nb)) == rp.RPC_EINVAL
    assert lib.surrogate_train_workspace_size(ctypes.byref(sh), 4096, 65, ctypes.byref(nb)) == rp.RPC_EINVAL
    assert lib.surrogate_extend_workspace_size(ctypes.byref(sh), 1000, 512, 1024, 32, ctypes.byref(nb)) == rp.RPC_EINVAL
    assert lib.rpc_batched_workspace_size(None, 0, 4, ctypes.byref(nb)) == rp.RPC_EINVAL


def test_lowmem_alg1_host_checks(lib):
    """bistoch_lowmem accepts float64 Grams with Cholesky QR and block sizes
    that are multiples of 8192 (at least r), and nothing else."""
    import paper_2510_26574_amd as rp

    pts = rp.rpc_points(100000, 16, 16, 0x1000, 1.0)
    nb = ctypes.c_size_t(0)

    def size(r=256, nev=16, gram="f64", qr="cholqr", block=0, gamma=0.0):
        o = rp.rpc_eig_opts(nev, 0, rp.DTYPES[gram], rp.DTYPES["f64"], 0, rp.QR_MODES[qr], gamma)
        return lib.bistoch_lowmem_workspace_size(ctypes.byref(pts), r, ctypes.byref(o), block,
                                                 ctypes.byref(nb))

    assert size() == 0 and nb.value > 0
    small = nb.value
    assert size(block=8192) == 0 and nb.value < small  # smaller blocks, smaller workspace
    for bad in [dict(gram="f32"), dict(qr="cholqr2"), dict(block=1000), dict(block=-8192),
                dict(r=9000, block=8192), dict(nev=300), dict(gamma=-1.0)]:
        assert size(**bad) == rp.RPC_EINVAL, bad
    o = rp.rpc_eig_opts(16, 0, rp.DTYPES["f64"], rp.DTYPES["f64"], 0, 0, 0.0)
    fake = ctypes.c_void_p(0x1000)
    # null outputs and ldu below N are rejected before any launch
    assert lib.bistoch_lowmem(ctypes.byref(pts), fake, fake, fake, 256, 256, ctypes.byref(o), 0, fake,
                              fake, fake, None, 100008, fake, fake, fake, 1 << 30, fake,
                              None) == rp.RPC_EINVAL
    assert lib.bistoch_lowmem(ctypes.byref(pts), fake, fake, fake, 256, 256, ctypes.byref(o), 0, fake,
                              fake, fake, fake, 99992, fake, fake, fake, 1 << 30, fake,
                              None) == rp.RPC_EINVAL
