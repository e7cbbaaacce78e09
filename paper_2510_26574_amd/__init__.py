"""Python binding of librpchol (gfx950): argument marshalling only.

Every step of the method runs in the library's HIP kernels.  PyTorch supplies
device memory and the current stream; if the library cannot be loaded the
calls raise, there is no fallback.

The names follow the C-ABI in include/rpchol.h:
  rpchol_factor    accelerated randomly pivoted partial Cholesky (Algorithm 2
                   with the accept/reject check of Algorithm 3);
  bistoch_degrees  d~ = diag(F F^T 1), q~ = diag(F F^T D~^{-1} 1) (Algorithm 1);
  bistoch_eig      top eigenpairs of P~ = B C B^T (Algorithm 1);
  nystrom_extend   extension of the eigenvectors to new points.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpchol.so")

RPC_OK, RPC_EINVAL, RPC_EWORKSPACE, RPC_EHIP = 0, -1, -2, -3
RPC_EDEGREE, RPC_EQDEGREE, RPC_EBREAKDOWN, RPC_ENONFINITE, RPC_ENOCONV = -4, -5, -6, -7, -8
STATUS_NAMES = {
    0: "RPC_OK", -1: "RPC_EINVAL", -2: "RPC_EWORKSPACE", -3: "RPC_EHIP", -4: "RPC_EDEGREE",
    -5: "RPC_EQDEGREE", -6: "RPC_EBREAKDOWN", -7: "RPC_ENONFINITE", -8: "RPC_ENOCONV",
}
DTYPES = {"f64": 0, "f32": 1, "bf16": 2}
MODES = {"sampled": 0, "greedy": 1, "replay": 2}


class RpcError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}")


class rpc_points(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("d", ctypes.c_int64), ("ldx", ctypes.c_int64),
                ("X", ctypes.c_void_p), ("eps", ctypes.c_double)]


class rpc_factor_opts(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("b", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("gemm_dtype", ctypes.c_int32), ("factor_dtype", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("tau", ctypes.c_double),
                ("uniforms", ctypes.c_void_p), ("n_uniforms", ctypes.c_int64),
                ("replay", ctypes.c_void_p), ("n_replay", ctypes.c_int64),
                ("round_accepted", ctypes.c_void_p)]


class rpc_eig_opts(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int32), ("fix_const", ctypes.c_int32),
                ("gram_dtype", ctypes.c_int32), ("u_dtype", ctypes.c_int32),
                ("gamma", ctypes.c_double)]


_lib = None
_VP, _I64, _I32, _SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
_SIGS = {
    "rpchol_factor_workspace_size": [_VP, _VP, _VP],
    "rpchol_factor": [_VP, _VP, _VP, _I64, _VP, _VP, _VP, _VP, _SZ, _VP, _VP],
    "bistoch_degrees_workspace_size": [_I64, _I32, _VP],
    "bistoch_degrees": [_VP, _I32, _I64, _I64, _I32, _VP, _VP, _VP, _VP, _VP, _SZ, _VP, _VP],
    "bistoch_eig_workspace_size": [_I64, _I32, _VP, _VP],
    "bistoch_eig": [_VP, _I32, _I64, _I64, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _I64, _VP, _VP,
                    _VP, _SZ, _VP, _VP],
    "nystrom_extend_workspace_size": [_I64, _I64, _I32, _I32, _VP],
    "nystrom_extend": [_VP, _VP, _VP, _VP, _VP, _I32, _I64, _I32, _VP, _VP, _I32, _VP, _I64, _VP,
                       _SZ, _VP, _VP],
    "rpc_status_sync": [_VP, _VP],
    "rpc_version": [],
    "rpc_profile_enable": [ctypes.c_int],
    "rpc_profile_reset": [],
    "rpc_profile_read": [_I32, _VP, _VP],
}


def load_library(path=None):
    """Load librpchol.so (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"librpchol.so not built ({p}); run __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "rpc_version" else ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _check(rc, where):
    if rc != RPC_OK:
        raise RpcError(rc, where)


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("librpchol needs a GPU (torch.cuda is not available)")
    return torch


def _stream(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _ld(n):
    return (n + 7) // 8 * 8


def _points(X, eps):
    assert X.dtype.__str__() == "torch.float32" and X.is_cuda and X.dim() == 2 and X.stride(1) == 1
    return rpc_points(X.shape[0], X.shape[1], X.stride(0), X.data_ptr(), float(eps))


def _workspace(torch, nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def new_status(device="cuda"):
    torch = _torch()
    return torch.zeros(1, dtype=torch.int32, device=device)


def status_sync(status, stream=None):
    """Synchronise and return the device status code."""
    torch = _torch()
    return load_library().rpc_status_sync(_ptr(status), _stream(torch, stream))


def rpchol_factor(X, eps, r, b, mode="sampled", uniforms=None, replay=None, gemm_dtype="f64",
                  factor_dtype="f64", tau=0.0, status=None, stream=None):
    """Algorithm 2 on the Gaussian kernel of the rows of X (N x d float32, CUDA).

    Returns dict: F (N x r view, column-major storage), pivots (r int64),
    rho (N float64), k (1 int32, device), status (1 int32, device).
    """
    torch = _torch()
    lib = load_library()
    N = X.shape[0]
    dev = X.device
    fdt = torch.float64 if factor_dtype == "f64" else torch.float32
    ldf = _ld(N)
    Fbuf = torch.empty((r, ldf), dtype=fdt, device=dev)
    piv = torch.empty(r, dtype=torch.int64, device=dev)
    rho = torch.empty(N, dtype=torch.float64, device=dev)
    k = torch.zeros(1, dtype=torch.int32, device=dev)
    st = status if status is not None else torch.zeros(1, dtype=torch.int32, device=dev)
    pts = _points(X, eps)
    nrounds = -(-(r if mode != "replay" else replay.numel()) // b)
    racc = torch.zeros(nrounds, dtype=torch.int32, device=dev)
    opts = rpc_factor_opts(int(r), int(b), MODES[mode], DTYPES[gemm_dtype], DTYPES[factor_dtype], 0,
                           float(tau), 0, 0, 0, 0, racc.data_ptr())
    if mode == "sampled":
        assert uniforms is not None and uniforms.dtype == torch.float64 and uniforms.is_cuda
        opts.uniforms = uniforms.data_ptr()
        opts.n_uniforms = uniforms.numel()
    if mode == "replay":
        assert replay is not None and replay.dtype == torch.int64 and replay.is_cuda
        opts.replay = replay.data_ptr()
        opts.n_replay = replay.numel()
    nb = ctypes.c_size_t(0)
    _check(lib.rpchol_factor_workspace_size(ctypes.byref(pts), ctypes.byref(opts), ctypes.byref(nb)),
           "rpchol_factor_workspace_size")
    ws = _workspace(torch, nb.value, dev)
    _check(lib.rpchol_factor(ctypes.byref(pts), ctypes.byref(opts), _ptr(Fbuf), ldf, _ptr(piv),
                             _ptr(rho), _ptr(k), _ptr(ws), nb.value, _ptr(st), _stream(torch, stream)),
           "rpchol_factor")
    return {"F": Fbuf[:, :N].t(), "Fbuf": Fbuf, "ldf": ldf, "pivots": piv, "rho": rho, "k": k,
            "status": st, "round_accepted": racc, "workspace": ws}


def _factor_args(F):
    """(storage, dtype code, N, ldf, r) of an N x r column-major view."""
    import torch

    N, r = F.shape
    assert F.stride(0) == 1, "F must be column-major (stride(0) == 1)"
    ldf = F.stride(1) if r > 1 else _ld(N)
    code = DTYPES["f64"] if F.dtype == torch.float64 else DTYPES["f32"]
    return code, N, ldf, r


def bistoch_degrees(F, k, status=None, stream=None):
    """c = F^T 1, d~ = F c, q~ = F F^T (1/d~) (Algorithm 1); asserts on device."""
    torch = _torch()
    lib = load_library()
    code, N, ldf, r = _factor_args(F)
    dev = F.device
    c = torch.empty(r, dtype=torch.float64, device=dev)
    d = torch.empty(N, dtype=torch.float64, device=dev)
    q = torch.empty(N, dtype=torch.float64, device=dev)
    st = status if status is not None else torch.zeros(1, dtype=torch.int32, device=dev)
    nb = ctypes.c_size_t(0)
    _check(lib.bistoch_degrees_workspace_size(N, r, ctypes.byref(nb)), "bistoch_degrees_workspace_size")
    ws = _workspace(torch, nb.value, dev)
    _check(lib.bistoch_degrees(_ptr(F), code, N, ldf, r, _ptr(k), _ptr(c), _ptr(d), _ptr(q), _ptr(ws),
                               nb.value, _ptr(st), _stream(torch, stream)), "bistoch_degrees")
    return {"c": c, "d": d, "q": q, "status": st}


def bistoch_eig(F, k, d, q, nev, gamma=0.0, fix_const=False, gram_dtype="f64", u_dtype="f64",
                status=None, stream=None):
    """Top-nev eigenpairs of P~ (Algorithm 1). Returns U (N x nev view), lam, E."""
    torch = _torch()
    lib = load_library()
    code, N, ldf, r = _factor_args(F)
    dev = F.device
    udt = torch.float64 if u_dtype == "f64" else torch.float32
    ldu = _ld(N)
    Ubuf = torch.empty((nev, ldu), dtype=udt, device=dev)
    lam = torch.empty(nev, dtype=torch.float64, device=dev)
    E = torch.empty((nev, r), dtype=torch.float64, device=dev)
    st = status if status is not None else torch.zeros(1, dtype=torch.int32, device=dev)
    opts = rpc_eig_opts(int(nev), 1 if fix_const else 0, DTYPES[gram_dtype], DTYPES[u_dtype], float(gamma))
    nb = ctypes.c_size_t(0)
    _check(lib.bistoch_eig_workspace_size(N, r, ctypes.byref(opts), ctypes.byref(nb)),
           "bistoch_eig_workspace_size")
    ws = _workspace(torch, nb.value, dev)
    _check(lib.bistoch_eig(_ptr(F), code, N, ldf, r, _ptr(k), _ptr(d), _ptr(d), _ptr(q),
                           ctypes.byref(opts), _ptr(Ubuf), ldu, _ptr(lam), _ptr(E), _ptr(ws), nb.value,
                           _ptr(st), _stream(torch, stream)), "bistoch_eig")
    return {"U": Ubuf[:, :N].t(), "lam": lam, "E": E.t(), "status": st, "workspace": ws}


def nystrom_extend(Y, X, eps, pivots, k, F, c, E, status=None, stream=None):
    """Extended eigenvector values at the rows of Y (M x d float32). Returns Phi (M x nev)."""
    torch = _torch()
    lib = load_library()
    code, N, ldf, r = _factor_args(F)
    nev = E.shape[1]
    assert E.stride(0) == 1 and E.stride(1) == r, "E must be r x nev column-major"
    M = Y.shape[0]
    dev = Y.device
    Phib = torch.empty((nev, M), dtype=torch.float64, device=dev)
    st = status if status is not None else torch.zeros(1, dtype=torch.int32, device=dev)
    py, px = _points(Y, eps), _points(X, eps)
    nb = ctypes.c_size_t(0)
    _check(lib.nystrom_extend_workspace_size(M, Y.shape[1], r, nev, ctypes.byref(nb)),
           "nystrom_extend_workspace_size")
    ws = _workspace(torch, nb.value, dev)
    _check(lib.nystrom_extend(ctypes.byref(py), ctypes.byref(px), _ptr(pivots), _ptr(k), _ptr(F), code,
                              ldf, r, _ptr(c), _ptr(E), nev, _ptr(Phib), M, _ptr(ws), nb.value, _ptr(st),
                              _stream(torch, stream)), "nystrom_extend")
    return {"Phi": Phib.t(), "status": st}


def version():
    return load_library().rpc_version().decode()


PROFILE_KINDS = ["kernel_cols", "schur", "solve_downdate", "pivot", "accept_reject", "degrees", "gram",
                 "small", "form_u", "nystrom", "eig"]


def profile_enable(on=True):
    _check(load_library().rpc_profile_enable(1 if on else 0), "rpc_profile_enable")


def profile_reset():
    load_library().rpc_profile_reset()


def profile_read():
    """{kind: (total_ms, launches)} for the launches since the last reset."""
    lib = load_library()
    out = {}
    for i, name in enumerate(PROFILE_KINDS):
        ms, n = ctypes.c_double(0), ctypes.c_int64(0)
        _check(lib.rpc_profile_read(i, ctypes.byref(ms), ctypes.byref(n)), "rpc_profile_read")
        out[name] = (ms.value, n.value)
    return out
