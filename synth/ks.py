"""Delay-embedded Kuramoto-Sivashinsky states (the paper-shaped workload).

The trajectory comes from the C integrator in ks_etdrk4.c (periodic domain
L = 22, 64 grid points, alias-free quadratic term, ETDRK4 with dt = 0.25),
started from 1e-2 * N(0, 1) on the 64 grid points (numpy default_rng(seed),
mean removed).  The first `spinup` steps are discarded and a 64-vector is
kept every `every` steps.

Delay embedding with q delays at the sample spacing: point n is
[s_{n+q-1}, s_{n+q-2}, ..., s_n] (newest first), so d = 64 q and
N = samples - q + 1.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_ks_etdrk4.so")
_lib = None


def build_ks(force=True):
    """Compile the integrator with the host C compiler (input data only)."""
    import subprocess

    src = os.path.join(_HERE, "ks_etdrk4.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-march=x86-64-v3", "-fPIC", "-shared", "-o", tmp, src, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_ks(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        for fn in (lib.ks_generate, lib.ks_generate64):
            fn.restype = ctypes.c_int
            fn.argtypes = [
                ctypes.c_long, ctypes.c_long, ctypes.c_long, ctypes.c_double, ctypes.c_double,
                ctypes.c_void_p, ctypes.c_void_p,
            ]
        _lib = lib
    return _lib


def ks_trajectory(n_samples, seed=0, spinup=10_000, every=4, dt=0.25, L=22.0, amp=1e-2, u0=None,
                  dtype=np.float32):
    """n_samples x 64 snapshots of the KS field (float32, or float64 on request)."""
    if u0 is None:
        rng = np.random.default_rng(seed)
        u0 = amp * rng.standard_normal(64)
        u0 = u0 - u0.mean()
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    out = np.empty((n_samples, 64), dtype=dtype)
    fn = _load().ks_generate64 if out.dtype == np.float64 else _load().ks_generate
    if out.dtype not in (np.float32, np.float64):
        raise ValueError("dtype must be float32 or float64")
    rc = fn(int(n_samples), int(spinup), int(every), float(dt), float(L), u0.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise RuntimeError("ks_generate failed")
    return out


def delay_embed(samples, q):
    """Rows [s_{n+q-1}, ..., s_n] for n = 0 .. len(samples)-q (float32, contiguous)."""
    s = np.asarray(samples)
    n = s.shape[0] - q + 1
    if n <= 0:
        raise ValueError("not enough samples for the delay window")
    out = np.empty((n, q * s.shape[1]), dtype=s.dtype)
    w = s.shape[1]
    for j in range(q):
        out[:, j * w:(j + 1) * w] = s[q - 1 - j: q - 1 - j + n]
    return out


def ks_points(N, q=8, seed=0, d=None, **kw):
    """N delay-embedded KS states of dimension 64 q (optionally the leading d)."""
    X = delay_embed(ks_trajectory(N + q - 1, seed=seed, **kw), q)
    if d is not None:
        X = np.ascontiguousarray(X[:, :d])
    return X
