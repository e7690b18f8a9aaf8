"""Derivation of the binary32 coefficients of the oracle's simplified atan2.

atan(r) on r in [0, 1] is approximated as r * P(r^2) with P of degree 4.
The fit runs in float64: iteratively reweighted least squares (Lawson's
method) on a dense set of points clustered at both ends of the interval,
converging towards the minimax polynomial; the result is rounded to
binary32.  Prints the coefficients as C hex-float literals and the maximum
error of the binary32 Horner evaluation.

    python oracle/derive_phi16.py
"""

import numpy as np

DEGREE = 4


def fit(degree=DEGREE, iters=60):
    r = np.concatenate([np.cos(np.linspace(0, np.pi / 2, 20001)), np.linspace(0, 1, 20001)])
    s = r * r
    A = np.stack([r * s ** j for j in range(degree + 1)], axis=1)
    b = np.arctan(r)
    w = np.ones_like(r)
    for _ in range(iters):
        c, *_ = np.linalg.lstsq(A * np.sqrt(w)[:, None], b * np.sqrt(w), rcond=None)
        e = np.abs(A @ c - b)
        w = np.maximum(w * e / (w * e).sum(), 1e-30)
    return c.astype(np.float32)


def max_error(c32):
    r = np.linspace(0, 1, 2000001).astype(np.float32)
    s = (r * r).astype(np.float32)
    p = np.float32(c32[-1])
    for j in range(len(c32) - 2, -1, -1):
        p = (p * s).astype(np.float32) + c32[j]
        p = p.astype(np.float32)
    at = (r * p).astype(np.float32)
    return float(np.abs(at.astype(np.float64) - np.arctan(r.astype(np.float64))).max())


if __name__ == "__main__":
    c = fit()
    for j, v in enumerate(c):
        print(f"c{j} = {float(v).hex()}")
    err = max_error(c)
    print(f"max |error| = {err:.3e} rad = {err * 32768 / np.pi:.3f} phi16 units")
