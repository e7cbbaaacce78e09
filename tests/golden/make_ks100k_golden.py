"""Writes ks100k_r512_b64.npz: the float64 oracle's result on the plain-method
workload at paper shape (KS delay embedding, N = 100 000, d = 512, median
bandwidth, r = 512, b = 64, sampled pivots from the Philox stream of seed 0,
top 32 eigenpairs of P~).  Calls only `oracle/` and the shared input
generators in `synth/`; takes about two minutes on 8 cores.

Stored: sha256 of the float32 points, eps, the accepted pivots in order, the
per-round accepted counts and trace errors, the leading 40 eigenvalues, and
Z = R^{-1} V[:, :32] (k x 32) with R from the Householder QR of D~^{-1} F, so
that U = D~^{-1} F Z for the oracle's factor F (the parity test rebuilds U
from the device factor, which is checked separately against the closed form
F = K(:, S) chol(K(S, S))^{-T} at sampled rows).

    python tests/golden/make_ks100k_golden.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import ks_points, median_sq_distance, uniform_stream  # noqa: E402

N, Q, R, B, NEV, SEED = 100_000, 8, 512, 64, 32, 0
OUT = os.path.join(HERE, "ks100k_r512_b64.npz")


def main():
    X = ks_points(N, q=Q, seed=SEED)
    eps = median_sq_distance(X, seed=SEED)
    u = uniform_stream(2 * B * (-(-R // B)), seed=SEED)
    ref = oracle.arpc(X, eps, r=R, b=B, mode="sampled", uniforms=u)
    res = oracle.bistoch_eig(ref["F"], NEV)
    F = ref["F"]
    d = res["d"]
    # Z with U = D~^{-1} F Z, solved from the oracle's own U (least squares on
    # a full-column-rank B = D~^{-1} F is exact up to rounding)
    Z, *_ = np.linalg.lstsq(F / d[:, None], res["U"], rcond=None)
    np.savez_compressed(
        OUT,
        x_sha256=np.frombuffer(hashlib.sha256(X.tobytes()).digest(), dtype=np.uint8),
        eps=np.float64(eps),
        pivots=ref["S"],
        accepted=np.asarray(ref["accepted"], dtype=np.int64),
        trace_err=np.asarray(ref["trace_err"], dtype=np.float64),
        lam=res["lam_all"][:40],
        Z=Z,
    )
    print(f"wrote {OUT}: k = {ref['k']}, lam[:4] = {res['lam'][:4]}, "
          f"|D~^-1 F Z - U| = {np.abs((F / d[:, None]) @ Z - res['U']).max():.2e}")


if __name__ == "__main__":
    main()
