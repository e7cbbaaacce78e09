"""Python binding of librpchol (gfx950): argument marshalling only.

Every step of the method runs in the library's HIP kernels.  PyTorch supplies
device memory and the current stream; if the library cannot be loaded the
calls raise, there is no fallback.

The names follow the C-ABI in include/rpchol.h:
  rpchol_factor    accelerated randomly pivoted partial Cholesky (Algorithm 2
                   with the accept/reject check of Algorithm 3);
  bistoch_degrees  d~ = diag(F F^T 1), q~ = diag(F F^T D~^{-1} 1) (Algorithm 1);
  bistoch_eig      top eigenpairs of P~ = B C B^T (Algorithm 1);
  nystrom_extend   extension of the eigenvectors to new points;
  surrogate_*      the learned surrogate of the extension (a perceptron
                   trained on the eigenvectors, with a per-point fallback to
                   nystrom_extend).
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
DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "split16": 3}  # split16: float32 products as split fp16 pairs
MODES = {"sampled": 0, "greedy": 1, "replay": 2}


class RpcError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}")


class rpc_points(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("d", ctypes.c_int64), ("ldx", ctypes.c_int64),
                ("X", ctypes.c_void_p), ("eps", ctypes.c_double), ("dtype", ctypes.c_int32)]

    def __init__(self, N=0, d=0, ldx=0, X=0, eps=0.0, dtype=1):
        # dtype defaults to RPC_F32, the points' usual storage
        super().__init__(N, d, ldx, X, eps, dtype)


class rpc_factor_opts(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("b", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("gemm_dtype", ctypes.c_int32), ("factor_dtype", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("tau", ctypes.c_double),
                ("uniforms", ctypes.c_void_p), ("n_uniforms", ctypes.c_int64),
                ("replay", ctypes.c_void_p), ("n_replay", ctypes.c_int64),
                ("round_accepted", ctypes.c_void_p), ("round_trace", ctypes.c_void_p)]


NORMALIZATIONS = {"bistochastic": 0, "symmetric": 1}


class rpc_eig_opts(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int32), ("fix_const", ctypes.c_int32),
                ("gram_dtype", ctypes.c_int32), ("u_dtype", ctypes.c_int32),
                ("normalization", ctypes.c_int32), ("qr_mode", ctypes.c_int32),
                ("gamma", ctypes.c_double)]


_lib = None
_VP, _I64, _I32, _SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
_SIGS = {
    "rpchol_factor_workspace_size": [_VP, _VP, _VP],
    "rpchol_factor": [_VP, _VP, _VP, _I64, _VP, _VP, _VP, _VP, _SZ, _VP, _VP],
    "bistoch_degrees_workspace_size": [_I64, _I32, _VP],
    "bistoch_degrees": [_VP, _I32, _I64, _I64, _I32, _VP, _VP, _VP, _VP, _VP, _SZ, _VP, _VP],
    "bistoch_degrees_noalloc": [_VP, _I32, _I64, _I64, _I32, _VP, _VP, _VP, _VP, _VP, _VP],
    "bistoch_eig_workspace_size": [_I64, _I32, _VP, _VP],
    "bistoch_eig": [_VP, _I32, _I64, _I64, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _I64, _VP, _VP,
                    _VP, _SZ, _VP, _VP],
    "nystrom_extend_workspace_size": [_I64, _I64, _I32, _I32, _VP],
    "nystrom_extend": [_VP, _VP, _VP, _VP, _VP, _I32, _I64, _I32, _VP, _VP, _I32, _VP, _I64, _VP,
                       _SZ, _VP, _VP],
    "nystrom_extend_symmetric": [_VP, _VP, _VP, _VP, _VP, _I32, _I64, _I32, _VP, _VP, _I32, _VP, _I64,
                                 _VP, _SZ, _VP, _VP],
    "surrogate_layout": [_VP, _VP],
    "surrogate_init_uniforms": [_VP, _VP],
    "surrogate_init": [_VP, _VP, _I64, _VP, _VP, _VP, _VP, _VP],
    "surrogate_standardize_workspace_size": [_I64, _I64, _VP],
    "surrogate_standardize": [_VP, _I64, _I64, _I64, _VP, _VP, _VP, _SZ, _VP],
    "surrogate_train_workspace_size": [_VP, _I64, _I32, _VP],
    "surrogate_train_step": [_VP, _VP, _VP, _I64, _I64, _VP, _VP, _VP, _I64, _VP, _I32, _I64,
                             ctypes.c_double, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP, _VP],
    "surrogate_train_epoch": [_VP, _VP, _VP, _I64, _I64, _VP, _VP, _VP, _I64, _I64, _VP, _I32, _I64,
                              ctypes.c_double, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP, _VP],
    "surrogate_infer_workspace_size": [_VP, _I64, _VP],
    "surrogate_infer": [_VP, _VP, _VP, _VP, _I64, _I64, _VP, _VP, _VP, _I64, _VP, _VP, _SZ, _VP,
                        _VP],
    "surrogate_residual_target": [_VP, _I64, _VP, _I64, ctypes.c_double, _I64, _I32, _VP, _VP],
    "surrogate_extend_workspace_size": [_VP, _I64, _I64, _I32, _I32, _VP],
    "surrogate_extend": [_VP, _VP, _VP, _VP, _VP, ctypes.c_double, _VP, _VP, _VP, _VP, _VP, _I32,
                         _I64, _I32, _VP, _VP, _I32, ctypes.c_double, _VP, _I64, _VP, _VP, _VP,
                         _SZ, _VP, _VP],
    "rpc_job_workspace_size": [_VP, _VP],
    "rpc_batched_workspace_size": [_VP, _I32, _I32, _VP],
    "rpc_batched_run": [_VP, _I32, _I32, _VP, _SZ, _VP],
    "rpc_batched_graph_create": [_VP, _I32, _I32, _VP, _SZ, _VP, _VP],
    "rpc_batched_graph_launch": [_VP, _VP],
    "rpc_batched_graph_destroy": [_VP],
    "rpc_autotune_block": [_VP, _VP, _I32, _I32, _VP, _SZ, _VP, _VP, _VP],
    "rpchol_factor_group_workspace_size": [_VP, _VP, _I32, _VP],
    "rpchol_factor_group": [_VP, _VP, _VP, _I32, _VP, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, _SZ,
                            _VP],
    "bistoch_lowmem_workspace_size": [_VP, _I32, _VP, _I64, _VP],
    "bistoch_lowmem": [_VP, _VP, _VP, _VP, _I64, _I32, _VP, _I64, _VP, _VP, _VP, _VP, _I64, _VP, _VP,
                       _VP, _SZ, _VP, _VP],
    "nystrom_extend_lowmem": [_VP, _VP, _VP, _VP, _VP, _I64, _I32, _VP, _VP, _I32, _I32, _VP, _I64,
                              _VP, _SZ, _VP, _VP],
    "surrogate_train_graph_create": [_VP, _VP, _VP, _I64, _I64, _VP, _VP, _VP, _I64, _I64, _VP, _I32,
                                     _I64, ctypes.c_double, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ,
                                     _VP, _VP, _VP],
    "rpc_graph_launch": [_VP, _VP],
    "rpc_graph_destroy": [_VP],
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


_POINT_DTYPES = {"torch.float32": 1, "torch.float64": 0, "torch.bfloat16": 2}


def _points(X, eps):
    """rpc_points of a row-major CUDA tensor (float32, float64 or bfloat16)."""
    code = _POINT_DTYPES.get(str(X.dtype))
    assert code is not None, f"points must be float32, float64 or bfloat16, not {X.dtype}"
    assert X.is_cuda and X.dim() == 2 and X.stride(1) == 1
    return rpc_points(X.shape[0], X.shape[1], X.stride(0), X.data_ptr(), float(eps), code)


def _workspace(torch, nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def new_status(device="cuda"):
    torch = _torch()
    return torch.zeros(1, dtype=torch.int32, device=device)


def status_sync(status, stream=None):
    """Synchronise and return the device status code."""
    torch = _torch()
    return load_library().rpc_status_sync(_ptr(status), _stream(torch, stream))


RPC_FACTOR_UNFUSED = 1
RPC_FACTOR_SHARED_X = 2
RPC_FACTOR_LOW_MEMORY = 4
RPC_FACTOR_SPLIT_SOLVE = 8


def rpchol_factor(X, eps, r, b, mode="sampled", uniforms=None, replay=None, gemm_dtype="f64",
                  factor_dtype="f64", tau=0.0, unfused=False, shared_x=False, low_memory=False,
                  split_solve=False, status=None, stream=None, ldf=None):
    """Algorithm 2 on the Gaussian kernel of the rows of X (N x d float32, CUDA).

    Returns dict: F (N x r view, column-major storage with leading dimension
    ldf, by default the row count rounded up to 8; with low_memory the r x r
    factor rows F(S, :) of the pivots in pivot order), pivots (r int64), rho
    (N float64), k (1 int32, device), status (1 int32, device).
    """
    torch = _torch()
    lib = load_library()
    N = X.shape[0]
    dev = X.device
    fdt = torch.float64 if factor_dtype == "f64" else torch.float32
    rows = r if low_memory else N
    ldf = _ld(rows) if ldf is None else int(ldf)
    Fbuf = torch.empty((r, ldf), dtype=fdt, device=dev)
    piv = torch.empty(r, dtype=torch.int64, device=dev)
    rho = torch.empty(N, dtype=torch.float64, device=dev)
    k = torch.zeros(1, dtype=torch.int32, device=dev)
    st = status if status is not None else torch.zeros(1, dtype=torch.int32, device=dev)
    pts = _points(X, eps)
    nrounds = -(-(r if mode != "replay" else replay.numel()) // b)
    racc = torch.zeros(nrounds, dtype=torch.int32, device=dev)
    rtrace = torch.zeros(nrounds, dtype=torch.float64, device=dev)
    opts = rpc_factor_opts(int(r), int(b), MODES[mode], DTYPES[gemm_dtype], DTYPES[factor_dtype],
                           (RPC_FACTOR_UNFUSED if unfused else 0) | (RPC_FACTOR_SHARED_X if shared_x else 0)
                           | (RPC_FACTOR_LOW_MEMORY if low_memory else 0)
                           | (RPC_FACTOR_SPLIT_SOLVE if split_solve else 0),
                           float(tau), 0, 0, 0, 0, racc.data_ptr(), rtrace.data_ptr())
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
    return {"F": Fbuf[:, :rows].t(), "Fbuf": Fbuf, "ldf": ldf, "pivots": piv, "rho": rho, "k": k,
            "status": st, "round_accepted": racc, "round_trace": rtrace, "workspace": ws}


def rpchol_factor_group(X, eps_list, r, b, uniforms_list, gemm_dtype="f32", factor_dtype="f32", tau=0.0,
                        mode="sampled", stream=None):
    """Algorithm 2 for several bandwidths of the same points in lockstep
    (rpchol_factor_group: one pass over X per round for the whole group).
    Returns one dict per bandwidth, as rpchol_factor does."""
    torch = _torch()
    lib = load_library()
    G = len(eps_list)
    N = X.shape[0]
    dev = X.device
    fdt = torch.float64 if factor_dtype == "f64" else torch.float32
    ldf = _ld(N)
    nrounds = -(-r // b)
    outs, opts = [], []
    for g in range(G):
        o = {"Fbuf": torch.empty((r, ldf), dtype=fdt, device=dev),
             "pivots": torch.empty(r, dtype=torch.int64, device=dev),
             "rho": torch.empty(N, dtype=torch.float64, device=dev),
             "k": torch.zeros(1, dtype=torch.int32, device=dev),
             "status": torch.zeros(1, dtype=torch.int32, device=dev),
             "round_accepted": torch.zeros(nrounds, dtype=torch.int32, device=dev), "ldf": ldf}
        o["F"] = o["Fbuf"][:, :N].t()
        fo = rpc_factor_opts(int(r), int(b), MODES[mode], DTYPES[gemm_dtype], DTYPES[factor_dtype],
                             RPC_FACTOR_SHARED_X, float(tau), 0, 0, 0, 0, o["round_accepted"].data_ptr())
        if mode == "sampled":
            u = uniforms_list[g]
            assert u.dtype == torch.float64 and u.is_cuda
            fo.uniforms, fo.n_uniforms = u.data_ptr(), u.numel()
        outs.append(o)
        opts.append(fo)
    pts = _points(X, eps_list[0])
    nb = ctypes.c_size_t(0)
    _check(lib.rpchol_factor_group_workspace_size(ctypes.byref(pts), ctypes.byref(opts[0]), G,
                                                  ctypes.byref(nb)), "rpchol_factor_group_workspace_size")
    ws = _workspace(torch, nb.value, dev)

    keep = []

    def arr(ctype, vals):
        a = (ctype * G)(*vals)
        keep.append(a)
        return ctypes.cast(a, ctypes.c_void_p)

    eps_a = arr(ctypes.c_double, [float(e) for e in eps_list])
    opt_a = arr(ctypes.c_void_p, [ctypes.addressof(o) for o in opts])
    F_a = arr(ctypes.c_void_p, [o["Fbuf"].data_ptr() for o in outs])
    p_a = arr(ctypes.c_void_p, [o["pivots"].data_ptr() for o in outs])
    r_a = arr(ctypes.c_void_p, [o["rho"].data_ptr() for o in outs])
    k_a = arr(ctypes.c_void_p, [o["k"].data_ptr() for o in outs])
    s_a = arr(ctypes.c_void_p, [o["status"].data_ptr() for o in outs])
    _check(lib.rpchol_factor_group(ctypes.byref(pts), eps_a, opt_a, G, F_a, ldf, p_a, r_a, k_a, s_a,
                                   _ptr(ws), nb.value, _stream(torch, stream)), "rpchol_factor_group")
    for o in outs:
        o["workspace"] = ws
    return outs


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


def bistoch_degrees_noalloc(F, k, c, d, q, status, stream=None):
    """bistoch_degrees into caller-given c (r), d, q (N) float64 buffers, with
    the library's static scratch instead of a workspace (no allocation)."""
    torch = _torch()
    code, N, ldf, r = _factor_args(F)
    _check(load_library().bistoch_degrees_noalloc(_ptr(F), code, N, ldf, r, _ptr(k), _ptr(c), _ptr(d),
                                                  _ptr(q), _ptr(status), _stream(torch, stream)),
           "bistoch_degrees_noalloc")


QR_MODES = {"cholqr": 0, "cholqr2": 1}


def bistoch_eig(F, k, d, q, nev, gamma=0.0, fix_const=False, gram_dtype="f64", u_dtype="f64",
                normalization="bistochastic", qr_mode="cholqr", status=None, stream=None):
    """Top-nev eigenpairs of P~ (Algorithm 1), or of L~ = D~^{-1/2} K~ D~^{-1/2}
    with normalization="symmetric" (q may then be None).  Returns U (N x nev
    view), lam, E."""
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
    opts = rpc_eig_opts(int(nev), 1 if fix_const else 0, DTYPES[gram_dtype], DTYPES[u_dtype],
                        NORMALIZATIONS[normalization], QR_MODES[qr_mode], float(gamma))
    nb = ctypes.c_size_t(0)
    _check(lib.bistoch_eig_workspace_size(N, r, ctypes.byref(opts), ctypes.byref(nb)),
           "bistoch_eig_workspace_size")
    ws = _workspace(torch, nb.value, dev)
    _check(lib.bistoch_eig(_ptr(F), code, N, ldf, r, _ptr(k), _ptr(None), _ptr(d), _ptr(q),
                           ctypes.byref(opts), _ptr(Ubuf), ldu, _ptr(lam), _ptr(E), _ptr(ws), nb.value,
                           _ptr(st), _stream(torch, stream)), "bistoch_eig")
    return {"U": Ubuf[:, :N].t(), "lam": lam, "E": E.t(), "status": st, "workspace": ws}


def nystrom_extend(Y, X, eps, pivots, k, F, c, E, status=None, stream=None, symmetric=False):
    """Extended eigenvector values at the rows of Y (M x d float32). Returns Phi
    (M x nev).  symmetric=True extends the eigenvectors of L~ (bistoch_eig with
    normalization="symmetric") through nystrom_extend_symmetric."""
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
    fn = lib.nystrom_extend_symmetric if symmetric else lib.nystrom_extend
    _check(fn(ctypes.byref(py), ctypes.byref(px), _ptr(pivots), _ptr(k), _ptr(F), code,
              ldf, r, _ptr(c), _ptr(E), nev, _ptr(Phib), M, _ptr(ws), nb.value, _ptr(st),
              _stream(torch, stream)), "nystrom_extend")
    return {"Phi": Phib.t(), "status": st}


def bistoch_lowmem(X, eps, pivots, k, FS, nev, gamma=0.0, fix_const=False, u_dtype="f64",
                   normalization="bistochastic", block_rows=0, status=None, stream=None):
    """Algorithm 1 from the low-memory factor: FS = F(S, :) (r x r, the F of
    rpchol_factor(..., low_memory=True)), the points X (N x d float32) and
    the pivots; factor rows recomputed block by block.  Returns c, d, q, U,
    lam, E as bistoch_degrees and bistoch_eig."""
    torch = _torch()
    lib = load_library()
    N = X.shape[0]
    r = FS.shape[1]
    assert FS.dtype == torch.float64 and FS.stride(0) == 1, "FS must be column-major float64"
    ldfs = FS.stride(1) if r > 1 else _ld(r)
    dev = X.device
    udt = torch.float64 if u_dtype == "f64" else torch.float32
    ldu = _ld(N)
    c = torch.empty(r, dtype=torch.float64, device=dev)
    d = torch.empty(N, dtype=torch.float64, device=dev)
    q = torch.empty(N, dtype=torch.float64, device=dev)
    Ubuf = torch.empty((nev, ldu), dtype=udt, device=dev)
    lam = torch.empty(nev, dtype=torch.float64, device=dev)
    E = torch.empty((nev, r), dtype=torch.float64, device=dev)
    st = status if status is not None else torch.zeros(1, dtype=torch.int32, device=dev)
    opts = rpc_eig_opts(int(nev), 1 if fix_const else 0, DTYPES["f64"], DTYPES[u_dtype],
                        NORMALIZATIONS[normalization], QR_MODES["cholqr"], float(gamma))
    pts = _points(X, eps)
    nb = ctypes.c_size_t(0)
    _check(lib.bistoch_lowmem_workspace_size(ctypes.byref(pts), r, ctypes.byref(opts), int(block_rows),
                                             ctypes.byref(nb)), "bistoch_lowmem_workspace_size")
    ws = _workspace(torch, nb.value, dev)
    _check(lib.bistoch_lowmem(ctypes.byref(pts), _ptr(pivots), _ptr(k), _ptr(FS), ldfs, r,
                              ctypes.byref(opts), int(block_rows), _ptr(c), _ptr(d), _ptr(q),
                              _ptr(Ubuf), ldu, _ptr(lam), _ptr(E), _ptr(ws), nb.value, _ptr(st),
                              _stream(torch, stream)), "bistoch_lowmem")
    return {"c": c, "d": d, "q": q, "U": Ubuf[:, :N].t(), "lam": lam, "E": E.t(), "status": st,
            "workspace": ws}


def nystrom_extend_lowmem(Y, X, eps, pivots, k, FS, c, E, symmetric=False, status=None, stream=None):
    """nystrom_extend with F(S, :) given directly (the low-memory factor)."""
    torch = _torch()
    lib = load_library()
    r = FS.shape[1]
    assert FS.dtype == torch.float64 and FS.stride(0) == 1
    ldfs = FS.stride(1) if r > 1 else _ld(r)
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
    _check(lib.nystrom_extend_lowmem(ctypes.byref(py), ctypes.byref(px), _ptr(pivots), _ptr(k),
                                     _ptr(FS), ldfs, r, _ptr(c), _ptr(E), nev,
                                     NORMALIZATIONS["symmetric" if symmetric else "bistochastic"],
                                     _ptr(Phib), M, _ptr(ws), nb.value, _ptr(st),
                                     _stream(torch, stream)), "nystrom_extend_lowmem")
    return {"Phi": Phib.t(), "status": st}


class rpc_job(ctypes.Structure):
    _fields_ = [("X", rpc_points), ("factor", rpc_factor_opts), ("eig", rpc_eig_opts),
                ("F", ctypes.c_void_p), ("ldf", ctypes.c_int64), ("pivots", ctypes.c_void_p),
                ("rho", ctypes.c_void_p), ("k", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("d_tilde", ctypes.c_void_p), ("q_tilde", ctypes.c_void_p), ("U", ctypes.c_void_p),
                ("ldu", ctypes.c_int64), ("lambda_", ctypes.c_void_p), ("ext_E", ctypes.c_void_p),
                ("dev_status", ctypes.c_void_p)]


class Job:
    """One decomposition of the batched form: its inputs, its output tensors
    (allocated here) and the C job record pointing at them."""

    def __init__(self, X, eps, r, b, nev, mode="sampled", uniforms=None, replay=None,
                 gemm_dtype="f32", factor_dtype="f32", gram_dtype="f32", u_dtype="f32", tau=0.0,
                 gamma=0.0, shared_x=False):
        torch = _torch()
        N = X.shape[0]
        dev = X.device
        self.X, self.uniforms, self.replay = X, uniforms, replay
        fdt = torch.float64 if factor_dtype == "f64" else torch.float32
        udt = torch.float64 if u_dtype == "f64" else torch.float32
        self.ldf = _ld(N)
        self.Fbuf = torch.empty((r, self.ldf), dtype=fdt, device=dev)
        self.pivots = torch.empty(r, dtype=torch.int64, device=dev)
        self.rho = torch.empty(N, dtype=torch.float64, device=dev)
        self.k = torch.zeros(1, dtype=torch.int32, device=dev)
        self.c = torch.empty(r, dtype=torch.float64, device=dev)
        self.d = torch.empty(N, dtype=torch.float64, device=dev)
        self.q = torch.empty(N, dtype=torch.float64, device=dev)
        self.Ubuf = torch.empty((nev, self.ldf), dtype=udt, device=dev)
        self.lam = torch.empty(nev, dtype=torch.float64, device=dev)
        self.Ebuf = torch.empty((nev, r), dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        fo = rpc_factor_opts(int(r), int(b), MODES[mode], DTYPES[gemm_dtype], DTYPES[factor_dtype],
                             RPC_FACTOR_SHARED_X if shared_x else 0, float(tau), 0, 0, 0, 0, 0)
        if mode == "sampled":
            assert uniforms is not None and uniforms.dtype == torch.float64 and uniforms.is_cuda
            fo.uniforms, fo.n_uniforms = uniforms.data_ptr(), uniforms.numel()
        if mode == "replay":
            assert replay is not None and replay.dtype == torch.int64 and replay.is_cuda
            fo.replay, fo.n_replay = replay.data_ptr(), replay.numel()
        eo = rpc_eig_opts(int(nev), 0, DTYPES[gram_dtype], DTYPES[u_dtype], 0, 0, float(gamma))
        self.rec = rpc_job(_points(X, eps), fo, eo, self.Fbuf.data_ptr(), self.ldf,
                           self.pivots.data_ptr(), self.rho.data_ptr(), self.k.data_ptr(),
                           self.c.data_ptr(), self.d.data_ptr(), self.q.data_ptr(), self.Ubuf.data_ptr(),
                           self.ldf, self.lam.data_ptr(), self.Ebuf.data_ptr(), self.status.data_ptr())

    @property
    def F(self):
        return self.Fbuf[:, :self.X.shape[0]].t()

    @property
    def U(self):
        return self.Ubuf[:, :self.X.shape[0]].t()

    @property
    def E(self):
        return self.Ebuf.t()


def _job_array(jobs):
    arr = (rpc_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = j.rec
    return arr


def batched_workspace(jobs, n_streams):
    torch = _torch()
    nb = ctypes.c_size_t(0)
    _check(load_library().rpc_batched_workspace_size(_job_array(jobs), len(jobs), int(n_streams),
                                                     ctypes.byref(nb)), "rpc_batched_workspace_size")
    return _workspace(torch, nb.value, jobs[0].X.device)


def batched_run(jobs, n_streams=4, workspace=None, stream=None):
    """Run every job's decomposition, overlapped over n_streams streams."""
    torch = _torch()
    ws = workspace if workspace is not None else batched_workspace(jobs, n_streams)
    _check(load_library().rpc_batched_run(_job_array(jobs), len(jobs), int(n_streams), _ptr(ws),
                                          ws.numel(), _stream(torch, stream)), "rpc_batched_run")
    return ws


class BatchedGraph:
    """The batched issue of `jobs` captured once into a HIP graph on a
    non-default stream; launch() replays it on that stream."""

    def __init__(self, jobs, n_streams=4, workspace=None, stream=None):
        torch = _torch()
        self.jobs = list(jobs)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.ws = workspace if workspace is not None else batched_workspace(self.jobs, n_streams)
        self._arr = _job_array(self.jobs)
        g = ctypes.c_void_p(0)
        self.stream.wait_stream(torch.cuda.current_stream())
        _check(load_library().rpc_batched_graph_create(self._arr, len(self.jobs), int(n_streams),
                                                       _ptr(self.ws), self.ws.numel(),
                                                       ctypes.c_void_p(self.stream.cuda_stream),
                                                       ctypes.byref(g)), "rpc_batched_graph_create")
        self._g = g

    def launch(self):
        _check(load_library().rpc_batched_graph_launch(self._g, ctypes.c_void_p(self.stream.cuda_stream)),
               "rpc_batched_graph_launch")

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if self._g:
            load_library().rpc_batched_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_block(job, candidates, reps=2, stream=None):
    """(best b, {b: mean ms}) over the candidate block sizes for this job."""
    torch = _torch()
    lib = load_library()
    need = 0
    for b in candidates:
        rec = rpc_job.from_buffer_copy(job.rec)
        rec.factor.b = int(b)
        nb = ctypes.c_size_t(0)
        _check(lib.rpc_job_workspace_size(ctypes.byref(rec), ctypes.byref(nb)), "rpc_job_workspace_size")
        need = max(need, nb.value)
    ws = _workspace(torch, need, job.X.device)
    cand = (ctypes.c_int32 * len(candidates))(*[int(b) for b in candidates])
    ms = (ctypes.c_double * len(candidates))()
    best = ctypes.c_int32(0)
    _check(lib.rpc_autotune_block(ctypes.byref(job.rec), cand, len(candidates), int(reps), _ptr(ws), need,
                                  _stream(torch, stream), ctypes.byref(best), ms), "rpc_autotune_block")
    return best.value, {int(b): ms[i] for i, b in enumerate(candidates)}


class sur_shape(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("h", ctypes.c_int32), ("n_out", ctypes.c_int32)]


class sur_layout(ctypes.Structure):
    _fields_ = [("W1", ctypes.c_int64), ("b1", ctypes.c_int64), ("W2", ctypes.c_int64),
                ("b2", ctypes.c_int64), ("W3", ctypes.c_int64), ("b3", ctypes.c_int64),
                ("total", ctypes.c_int64), ("n3", ctypes.c_int32)]


class sur_train_opts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("weight_decay", ctypes.c_double),
                ("step", ctypes.c_int64), ("phase", ctypes.c_int32), ("splits", ctypes.c_int32)]


def surrogate_layout(d, h, n_out):
    """Offsets of W1, b1, W2, b2, W3, b3 in the parameter vector, its length
    `total`, and n3 (rows of W3: outputs, residual head, zero pad)."""
    lib = load_library()
    lay = sur_layout()
    sh = sur_shape(int(d), int(h), int(n_out))
    _check(lib.surrogate_layout(ctypes.byref(sh), ctypes.byref(lay)), "surrogate_layout")
    return {f: getattr(lay, f) for f, _ in sur_layout._fields_}


def surrogate_init_uniforms(d, h, n_out):
    """Number of uniforms the initialisation draws."""
    n = ctypes.c_int64(0)
    sh = sur_shape(int(d), int(h), int(n_out))
    _check(load_library().surrogate_init_uniforms(ctypes.byref(sh), ctypes.byref(n)),
           "surrogate_init_uniforms")
    return n.value


class Surrogate:
    """Parameter vector, AdamW moments and bf16 copy of one surrogate, in
    device memory (float32 / bfloat16 torch tensors owned here)."""

    def __init__(self, d, h, n_out, init=None, uniforms=None, device="cuda", stream=None):
        """Either `init` (a full parameter vector in the layout) or `uniforms`
        (device float64, surrogate_init_uniforms(d, h, n_out) of them)."""
        torch = _torch()
        lib = load_library()
        self.shape = sur_shape(int(d), int(h), int(n_out))
        self.layout = surrogate_layout(d, h, n_out)
        tot = self.layout["total"]
        if init is not None:
            init = torch.as_tensor(init, dtype=torch.float32)
            assert init.numel() == tot, f"initial parameter vector must have {tot} entries"
            self.params = init.to(device).contiguous()
        else:
            assert uniforms is not None and uniforms.dtype == torch.float64 and uniforms.is_cuda
            self.params = torch.empty(tot, dtype=torch.float32, device=device)
        self.m = torch.empty(tot, dtype=torch.float32, device=device)
        self.v = torch.empty(tot, dtype=torch.float32, device=device)
        self.wbf16 = torch.empty(tot, dtype=torch.bfloat16, device=device)
        self.steps = {0: 0, 1: 0}  # AdamW step counters, one per phase
        nu = uniforms.numel() if init is None else 0
        _check(lib.surrogate_init(ctypes.byref(self.shape), _ptr(None if init is not None else uniforms),
                                  nu, _ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(self.wbf16),
                                  _stream(torch, stream)), "surrogate_init")
        self._ws = {}

    def _wsbuf(self, key, nbytes, device):
        torch = _torch()
        buf = self._ws.get(key)
        if buf is None or buf.numel() < nbytes:
            buf = _workspace(torch, nbytes, device)
            self._ws[key] = buf
        return buf

    def train_step(self, X, mean, rstd, idx, T, tscale=1.0, phase=0, step=None, lr=1e-3,
                   betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01, splits=0, grad=None,
                   loss=None, status=None, stream=None):
        """One AdamW step on rows idx of X against T (see surrogate_train_step)."""
        torch = _torch()
        lib = load_library()
        if step is None:
            self.steps[phase] += 1
            step = self.steps[phase]
        B = idx.numel()
        assert idx.dtype == torch.int64 and X.dtype == torch.float32 and X.stride(1) == 1
        if phase == 0:
            assert T.dim() == 2 and T.stride(0) == 1, "phase-0 targets must be column-major N x n_out"
            ldt = T.stride(1) if T.shape[1] > 1 else T.shape[0]
        else:
            assert T.dim() == 1
            ldt = T.shape[0]
        tcode = DTYPES["f64"] if T.dtype == torch.float64 else DTYPES["f32"]
        opts = sur_train_opts(float(lr), float(betas[0]), float(betas[1]), float(eps),
                              float(weight_decay), int(step), int(phase), int(splits))
        nb = ctypes.c_size_t(0)
        _check(lib.surrogate_train_workspace_size(ctypes.byref(self.shape), B, int(splits),
                                                  ctypes.byref(nb)), "surrogate_train_workspace_size")
        ws = self._wsbuf("train", nb.value, X.device)
        st = status if status is not None else torch.zeros(1, dtype=torch.int32, device=X.device)
        _check(lib.surrogate_train_step(ctypes.byref(self.shape), ctypes.byref(opts), _ptr(X),
                                        X.stride(0), X.shape[0], _ptr(mean), _ptr(rstd), _ptr(idx), B,
                                        _ptr(T), tcode, ldt, float(tscale), _ptr(self.params),
                                        _ptr(self.m), _ptr(self.v), _ptr(self.wbf16), _ptr(grad),
                                        _ptr(loss), _ptr(ws), nb.value, _ptr(st),
                                        _stream(torch, stream)), "surrogate_train_step")
        return st

    def train_epoch(self, X, mean, rstd, idx, T, batch, tscale=1.0, phase=0, lr=1e-3,
                    betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01, splits=0, loss=None,
                    status=None, stream=None):
        """ceil(len(idx) / batch) AdamW steps over consecutive slices of idx."""
        torch = _torch()
        lib = load_library()
        n = idx.numel()
        nsteps = -(-n // batch)
        assert idx.dtype == torch.int64 and X.dtype == torch.float32 and X.stride(1) == 1
        if phase == 0:
            assert T.dim() == 2 and T.stride(0) == 1, "phase-0 targets must be column-major N x n_out"
            ldt = T.stride(1) if T.shape[1] > 1 else T.shape[0]
        else:
            assert T.dim() == 1
            ldt = T.shape[0]
        if loss is not None:
            assert loss.dtype == torch.float64 and loss.numel() >= nsteps
        tcode = DTYPES["f64"] if T.dtype == torch.float64 else DTYPES["f32"]
        opts = sur_train_opts(float(lr), float(betas[0]), float(betas[1]), float(eps),
                              float(weight_decay), int(self.steps[phase] + 1), int(phase), int(splits))
        nb = ctypes.c_size_t(0)
        _check(lib.surrogate_train_workspace_size(ctypes.byref(self.shape), min(batch, n), int(splits),
                                                  ctypes.byref(nb)), "surrogate_train_workspace_size")
        ws = self._wsbuf("train", nb.value, X.device)
        st = status if status is not None else torch.zeros(1, dtype=torch.int32, device=X.device)
        _check(lib.surrogate_train_epoch(ctypes.byref(self.shape), ctypes.byref(opts), _ptr(X),
                                         X.stride(0), X.shape[0], _ptr(mean), _ptr(rstd), _ptr(idx), n,
                                         int(batch), _ptr(T), tcode, ldt, float(tscale),
                                         _ptr(self.params), _ptr(self.m), _ptr(self.v),
                                         _ptr(self.wbf16), _ptr(loss), _ptr(ws), nb.value, _ptr(st),
                                         _stream(torch, stream)), "surrogate_train_epoch")
        self.steps[phase] += nsteps
        return st

    def train_epochs(self, X, mean, rstd, perms, T, batch, tscale=1.0, phase=0, lr=1e-3,
                     betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01, splits=0, loss=None,
                     status=None, stream=None):
        """len(perms) epochs, each ceil(N / batch) AdamW steps over the slices of
        perms[e] (E x n int64, CUDA), from one captured epoch graph replayed per
        epoch (the permutation is copied into the graph's index buffer first).
        Equal bit for bit to calling train_epoch once per epoch.  loss (optional,
        float64, E * steps) receives every step's loss."""
        torch = _torch()
        lib = load_library()
        E, n = perms.shape
        nsteps = -(-n // batch)
        assert perms.dtype == torch.int64 and X.dtype == torch.float32 and X.stride(1) == 1
        if phase == 0:
            assert T.dim() == 2 and T.stride(0) == 1, "phase-0 targets must be column-major N x n_out"
            ldt = T.stride(1) if T.shape[1] > 1 else T.shape[0]
        else:
            assert T.dim() == 1
            ldt = T.shape[0]
        if loss is not None:
            assert loss.dtype == torch.float64 and loss.numel() >= E * nsteps
        tcode = DTYPES["f64"] if T.dtype == torch.float64 else DTYPES["f32"]
        opts = sur_train_opts(float(lr), float(betas[0]), float(betas[1]), float(eps),
                              float(weight_decay), 1, int(phase), int(splits))
        nb = ctypes.c_size_t(0)
        _check(lib.surrogate_train_workspace_size(ctypes.byref(self.shape), min(batch, n), int(splits),
                                                  ctypes.byref(nb)), "surrogate_train_workspace_size")
        dev = X.device
        ws = self._wsbuf("train", nb.value, dev)
        st = status if status is not None else torch.zeros(1, dtype=torch.int32, device=dev)
        idx = torch.empty(n, dtype=torch.int64, device=dev)
        lbuf = torch.zeros(nsteps, dtype=torch.float64, device=dev) if loss is not None else None
        counter = torch.full((1,), int(self.steps[phase]), dtype=torch.int64, device=dev)
        s = stream if stream is not None else torch.cuda.Stream(device=dev)
        s.wait_stream(torch.cuda.current_stream(dev))
        graph = ctypes.c_void_p(0)
        _check(lib.surrogate_train_graph_create(
            ctypes.byref(self.shape), ctypes.byref(opts), _ptr(X), X.stride(0), X.shape[0], _ptr(mean),
            _ptr(rstd), _ptr(idx), n, int(batch), _ptr(T), tcode, ldt, float(tscale), _ptr(self.params),
            _ptr(self.m), _ptr(self.v), _ptr(self.wbf16), _ptr(lbuf), _ptr(counter), _ptr(ws), nb.value,
            _ptr(st), ctypes.c_void_p(s.cuda_stream), ctypes.byref(graph)), "surrogate_train_graph_create")
        try:
            with torch.cuda.stream(s):
                for e in range(E):
                    idx.copy_(perms[e])
                    _check(lib.rpc_graph_launch(graph, ctypes.c_void_p(s.cuda_stream)), "rpc_graph_launch")
                    if loss is not None:
                        loss[e * nsteps:(e + 1) * nsteps].copy_(lbuf)
            torch.cuda.current_stream(dev).wait_stream(s)
            s.synchronize()
        finally:
            lib.rpc_graph_destroy(graph)
        self.steps[phase] += E * nsteps
        return st

    def infer(self, Y, mean, rstd, with_res=True, status=None, stream=None):
        """Phi (M x n_out float32 view of column-major storage) and the residual head."""
        torch = _torch()
        lib = load_library()
        M = Y.shape[0]
        n_out = self.shape.n_out
        Phib = torch.empty((n_out, max(M, 1)), dtype=torch.float32, device=Y.device)
        res = torch.empty(max(M, 1), dtype=torch.float32, device=Y.device) if with_res else None
        nb = ctypes.c_size_t(0)
        _check(lib.surrogate_infer_workspace_size(ctypes.byref(self.shape), M, ctypes.byref(nb)),
               "surrogate_infer_workspace_size")
        ws = self._wsbuf("infer", nb.value, Y.device)
        st = status if status is not None else torch.zeros(1, dtype=torch.int32, device=Y.device)
        _check(lib.surrogate_infer(ctypes.byref(self.shape), _ptr(self.params), _ptr(self.wbf16),
                                   _ptr(Y), Y.stride(0), M, _ptr(mean), _ptr(rstd), _ptr(Phib),
                                   max(M, 1), _ptr(res), _ptr(ws), nb.value, _ptr(st),
                                   _stream(torch, stream)), "surrogate_infer")
        return {"Phi": Phib[:, :M].t(), "res": res[:M] if res is not None else None, "status": st}

    def extend(self, Y, X, eps, pivots, k, F, c, E, mean, rstd, scale, log10_threshold=-2.0,
               status=None, stream=None):
        """Hybrid extension: surrogate everywhere, exact Nystrom (times scale)
        where the residual head exceeds the threshold.  Synchronises once."""
        torch = _torch()
        lib = load_library()
        code, N, ldf, r = _factor_args(F)
        nev = E.shape[1]
        assert E.stride(0) == 1 and E.stride(1) == r, "E must be r x nev column-major"
        M = Y.shape[0]
        n_out = self.shape.n_out
        Phib = torch.empty((n_out, max(M, 1)), dtype=torch.float32, device=Y.device)
        res = torch.empty(max(M, 1), dtype=torch.float32, device=Y.device)
        py, px = _points(Y, eps), _points(X, eps)
        nb = ctypes.c_size_t(0)
        _check(lib.surrogate_extend_workspace_size(ctypes.byref(self.shape), M, Y.shape[1], r, nev,
                                                   ctypes.byref(nb)), "surrogate_extend_workspace_size")
        ws = self._wsbuf("extend", nb.value, Y.device)
        st = status if status is not None else torch.zeros(1, dtype=torch.int32, device=Y.device)
        nf = ctypes.c_int64(0)
        _check(lib.surrogate_extend(ctypes.byref(self.shape), _ptr(self.params), _ptr(self.wbf16),
                                    _ptr(mean), _ptr(rstd), float(log10_threshold), ctypes.byref(py),
                                    ctypes.byref(px), _ptr(pivots), _ptr(k), _ptr(F), code, ldf, r,
                                    _ptr(c), _ptr(E), nev, float(scale), _ptr(Phib), max(M, 1),
                                    _ptr(res), ctypes.byref(nf), _ptr(ws), nb.value, _ptr(st),
                                    _stream(torch, stream)), "surrogate_extend")
        return {"Phi": Phib[:, :M].t(), "res": res[:M], "n_fallback": nf.value, "status": st}


def surrogate_standardize(X, stream=None):
    """Per-feature mean and 1/std (float64) of the rows of X (N x d float32)."""
    torch = _torch()
    lib = load_library()
    N, d = X.shape
    assert X.dtype == torch.float32 and X.stride(1) == 1
    mean = torch.empty(d, dtype=torch.float64, device=X.device)
    rstd = torch.empty(d, dtype=torch.float64, device=X.device)
    nb = ctypes.c_size_t(0)
    _check(lib.surrogate_standardize_workspace_size(N, d, ctypes.byref(nb)),
           "surrogate_standardize_workspace_size")
    ws = _workspace(torch, nb.value, X.device)
    _check(lib.surrogate_standardize(_ptr(X), N, d, X.stride(0), _ptr(mean), _ptr(rstd), _ptr(ws),
                                     nb.value, _stream(torch, stream)), "surrogate_standardize")
    return mean, rstd


def surrogate_residual_target(Phi_s, Phi_n, scale, stream=None):
    """log10 RMS over outputs of Phi_s - scale Phi_n (both M x n column-major views)."""
    torch = _torch()
    lib = load_library()
    M, n = Phi_s.shape
    assert Phi_s.stride(0) == 1 and Phi_n.stride(0) == 1 and Phi_n.shape[0] == M
    assert Phi_s.dtype == torch.float32 and Phi_n.dtype == torch.float64
    out = torch.empty(max(M, 1), dtype=torch.float64, device=Phi_s.device)
    lds = Phi_s.stride(1) if n > 1 else max(M, 1)
    ldn = Phi_n.stride(1) if Phi_n.shape[1] > 1 else max(M, 1)
    _check(lib.surrogate_residual_target(_ptr(Phi_s), lds, _ptr(Phi_n), ldn, float(scale), M, n,
                                         _ptr(out), _stream(torch, stream)), "surrogate_residual_target")
    return out[:M]


def version():
    return load_library().rpc_version().decode()


PROFILE_KINDS = ["kernel_cols", "schur", "solve_downdate", "pivot", "accept_reject", "degrees", "gram",
                 "small", "form_u", "nystrom", "eig", "sur_train", "sur_infer"]


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
