"""Derive the minimax polynomial used for atan on [0, 1] by the kernels.

atan(t) ~= t * P(t^2) with P of degree ``n`` in x = t^2 on [0, 1], chosen by the
Remez exchange algorithm to minimise the maximum *relative* error
|t P(t^2) - atan t| / atan t (weight 1 / f with f(x) = atan(sqrt x) / sqrt x).
Relative error keeps small angles (far faces) proportionally accurate.

The kernels use degree 6 (the default here).

Run:  python gen_atan_poly.py [degree]  -> prints the coefficients (FP32-rounded,
highest degree first) and the max relative error of an FP32 Horner evaluation.
"""
import sys

import numpy as np


def f(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    nz = x > 0
    s = np.sqrt(x[nz])
    out[nz] = np.arctan(s) / s
    return out


def remez(n, iters=60):
    m = n + 2  # reference points
    k = np.arange(m)
    xs = 0.5 - 0.5 * np.cos(np.pi * k / (m - 1))  # Chebyshev extrema on [0, 1]
    dense = np.linspace(0.0, 1.0, 200001)
    for _ in range(iters):
        # solve P(x_i) + (-1)^i E f(x_i) = f(x_i)  (relative weighting)
        A = np.zeros((m, m))
        for i, x in enumerate(xs):
            A[i, :n + 1] = x ** np.arange(n + 1)
            A[i, n + 1] = (-1) ** i * f(np.array([x]))[0]
        c = np.linalg.solve(A, f(xs))
        p = c[:n + 1]
        err = (np.polyval(p[::-1], dense) - f(dense)) / f(dense)
        # new reference: extrema of err between sign changes
        sgn = np.sign(err)
        idx = [0]
        for i in range(1, len(dense)):
            if sgn[i] != sgn[idx[-1]]:
                idx.append(i)
            elif abs(err[i]) > abs(err[idx[-1]]):
                idx[-1] = i
        if len(idx) < m:
            break
        # keep m consecutive extrema containing the global maximum
        idx = np.array(idx)
        best = np.argmax(np.abs(err[idx]))
        start = min(max(0, best - m // 2), len(idx) - m)
        xs = dense[idx[start:start + m]]
    return p, np.max(np.abs(err))


def fp32_check(p):
    t = np.linspace(0, 1, 2_000_001).astype(np.float32)
    x = (t * t).astype(np.float32)
    acc = np.float32(p[-1])
    for c in p[-2::-1]:
        acc = (acc * x + np.float32(c)).astype(np.float32)
    a = (acc * t).astype(np.float32)
    ref = np.arctan(t.astype(np.float64))
    nz = ref > 0
    rel = np.abs(a[nz].astype(np.float64) - ref[nz]) / ref[nz]
    return rel.max(), np.abs(a.astype(np.float64) - ref).max()


if __name__ == "__main__":
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 6
    p, e = remez(n)
    p32 = [float(np.float32(c)) for c in p]
    rel, ab = fp32_check(p32)
    print(f"degree {n} in t^2: minimax rel err {e:.3e}; fp32 Horner max rel {rel:.3e} abs {ab:.3e}")
    for c in p32[::-1]:
        print(f"    {np.float32(c)!r:>16}f,".replace("np.float32(", "").replace(")", ""))
