"""Product-state points of the paper's vector-valued spectral analysis
workload (the "Numerical experiments" section).

A KS trajectory (L = 22, 64 grid points, ETDRK4, dt = 0.25) starts from the
field whose leading four Fourier modes k = 1..4 have coefficient 0.6 and all
others zero (reading: u0(x) = sum_k 0.6 (e^{2 pi i k x / L} + c.c.) =
1.2 sum_{k=1}^{4} cos(2 pi k x / L); the mean mode stays zero).  After
10 000 steps one 64-vector is kept every 4 steps (one time unit), S samples
in all.  With J delays there are N = S - J + 1 delay-embedded times, and each
pair (time n, grid point x) is one point in R^J:

    W(n, x) = (u_{n+J-1}(x), u_{n+J-2}(x), ..., u_n(x))   (newest first),

ordered time-major (index n * 64 + x).  The kernel of the section is
exp(-|W - W'|^2 / (eps J)), i.e. bandwidth eps * J in the exp(-d^2 / eps)
convention of the library; the paper uses eps = 32.
"""
import numpy as np

from .ks import ks_trajectory

GRID = 64
L_DOMAIN = 22.0


def vsa_initial_field():
    x = np.arange(GRID) * (L_DOMAIN / GRID)
    u0 = np.zeros(GRID)
    for k in range(1, 5):
        u0 += 1.2 * np.cos(2.0 * np.pi * k * x / L_DOMAIN)
    return u0


def vsa_points(n_time=512, J=64, spinup=10_000, every=4):
    """(n_time * 64) x J float32 product-state points."""
    S = n_time + J - 1
    s = ks_trajectory(S, spinup=spinup, every=every, u0=vsa_initial_field(), dtype=np.float64)
    out = np.empty((n_time, GRID, J), dtype=np.float32)
    for j in range(J):
        out[:, :, j] = s[J - 1 - j: J - 1 - j + n_time, :]
    return out.reshape(n_time * GRID, J)
