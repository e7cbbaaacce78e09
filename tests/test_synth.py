"""Checks of the seeded input generators (inputs only; no method arithmetic)."""
import os

import numpy as np
import pytest
from scipy.spatial.distance import pdist

from synth import delay_embed, ks_trajectory, median_sq_distance, philox4x32_10, torus_points, uniform_stream

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and not l.startswith("#")]
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox4x32_10(np.array([v[:4]], dtype=np.uint32), np.array(v[4:6], dtype=np.uint32))[0]
        assert [int(x) for x in out] == v[6:10]


def test_uniform_stream_properties():
    u = uniform_stream(100000, seed=3)
    assert u.min() >= 0 and u.max() < 1
    assert np.all(u * 2.0 ** 53 == np.floor(u * 2.0 ** 53))
    assert abs(u.mean() - 0.5) < 0.005
    # offsets address the same stream
    assert np.array_equal(uniform_stream(10, seed=3, offset=500), u[500:510])


def test_torus_on_surface_and_area_uniform():
    X = torus_points(20000, seed=0).astype(np.float64)
    rad = np.sqrt(X[:, 0] ** 2 + X[:, 1] ** 2)
    dist = np.sqrt((rad - 2.0) ** 2 + X[:, 2] ** 2)
    assert np.abs(dist - 1.0).max() < 0.08
    assert abs(np.std(dist - 1.0) - 0.01) < 0.003
    # poloidal angle density proportional to R + r cos(theta): E[cos theta] = r/(2R)
    theta = np.arctan2(X[:, 2], rad - 2.0)
    assert abs(np.cos(theta).mean() - 0.25) < 0.02
    assert np.array_equal(torus_points(100, seed=0), torus_points(100, seed=0))


def test_median_eps_matches_library():
    X = np.random.default_rng(0).standard_normal((800, 4)).astype(np.float32)
    rng = np.random.default_rng(5)
    idx = rng.choice(800, 500, replace=False)
    ref = np.median(pdist(X[idx].astype(np.float64), "sqeuclidean"))
    assert median_sq_distance(X, seed=5) == pytest.approx(ref, rel=1e-14)


def test_ks_integrator_converges_to_reference_solution():
    """The ETDRK4 trajectory converges to an independent high-accuracy solution
    of the same alias-free Fourier system (numpy FFTs + scipy DOP853), with
    high order in dt (ratio approaching 16 as dt shrinks)."""
    from scipy.integrate import solve_ivp

    L, M = 22.0, 64
    x = L * np.arange(M) / M
    u0 = np.cos(2 * np.pi * x / L) * (1 + np.sin(2 * np.pi * x / L))
    u0 = u0 - u0.mean()
    kk = np.fft.rfftfreq(M, 1.0 / M)
    q = 2 * np.pi * kk / L
    keep = (kk >= 1) & (kk <= 31)

    def rhs(t, y):
        v = np.zeros(33, complex)
        v[keep] = y[:31] + 1j * y[31:]
        vp = np.zeros(49, complex)
        vp[:32] = v[:32]
        u = np.fft.irfft(vp * 96, 96)
        w = np.fft.rfft(u * u) / 96
        dv = (q ** 2 - q ** 4) * v - 0.5j * q * w[:33]
        return np.concatenate([dv[keep].real, dv[keep].imag])

    v0 = np.fft.rfft(u0) / M
    sol = solve_ivp(rhs, (0, 4.0), np.concatenate([v0[keep].real, v0[keep].imag]),
                    method="DOP853", rtol=1e-13, atol=1e-15)
    v = np.zeros(33, complex)
    v[keep] = sol.y[:31, -1] + 1j * sol.y[31:, -1]
    uT = np.fft.irfft(v * M, M)
    errs = []
    for dt in [0.05, 0.025, 0.0125]:
        n = int(round(4.0 / dt))
        errs.append(np.abs(ks_trajectory(2, spinup=0, every=n, dt=dt, u0=u0, dtype=np.float64)[1] - uT).max())
    assert errs[-1] < 1e-8
    assert errs[0] / errs[1] > 7 and errs[1] / errs[2] > 9


def test_ks_mean_conserved_and_chaotic_range():
    s = ks_trajectory(3000, seed=1, spinup=2000)
    assert np.abs(s.mean(axis=1)).max() < 1e-5
    assert 0.8 < s.std() < 1.6 and np.abs(s).max() < 4.0


def test_delay_embedding_layout():
    s = np.arange(10 * 2, dtype=np.float32).reshape(10, 2)
    X = delay_embed(s, 3)
    assert X.shape == (8, 6)
    assert np.array_equal(X[0], np.concatenate([s[2], s[1], s[0]]))
    assert np.array_equal(X[7], np.concatenate([s[9], s[8], s[7]]))


def test_batch_specs_ranges_and_determinism():
    from synth import BANDWIDTH_MULTIPLIERS, batch_specs

    a, b = batch_specs(), batch_specs()
    assert a == b and len(a) == 64 and len(BANDWIDTH_MULTIPLIERS) == 8
    assert [s["seed"] for s in a] == list(range(1, 65))
    for s in a:
        assert 5000 <= s["N"] <= 200000
        assert (s["d"], s["q"]) in ((32, 1), (128, 2), (512, 8))
        assert s["r"] in (64, 128, 256, 512)
    assert batch_specs(seed=1) != a


def test_vsa_points_layout():
    from synth import ks_trajectory, vsa_initial_field, vsa_points

    u0 = vsa_initial_field()
    # leading four Fourier modes only, coefficient 0.6 (mean zero)
    c = np.fft.fft(u0) / len(u0)
    assert np.allclose(c[1:5].real, 0.6) and np.allclose(np.abs(c[5:-4]), 0, atol=1e-12)
    assert abs(c[0]) < 1e-12
    P = vsa_points(n_time=20, J=8, spinup=100, every=4)
    assert P.shape == (20 * 64, 8) and P.dtype == np.float32
    s = ks_trajectory(27, spinup=100, every=4, u0=u0, dtype=np.float64)
    n, x = 5, 17
    assert np.allclose(P[n * 64 + x], s[n:n + 8, x][::-1].astype(np.float32))
