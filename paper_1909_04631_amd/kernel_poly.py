"""Coefficients of the polynomial Q used by the HIP kernels for the sparse
kernel of Eq. (8), read in the continuous Melkumyan-Ramos form (the printed
equation is garbled: it puts (1 - r) on the cosine term only):

    f(r) = (2 + cos 2 pi r)(1 - r)/3 + sin(2 pi r)/(2 pi),   0 <= r < 1.

With s = 1 - r the Taylor series of f about r = 1 has only odd powers from s^5
on:  f(1 - s) = sum_{n >= 2} (-1)^n (2n - 2)(2 pi)^{2n} s^{2n+1} / (3 (2n+1)!),
so f(1 - s) = s^5 Q(s^2) with Q an entire function.  The kernels evaluate
s^5 Q(s^2) with a degree-6 polynomial fit of Q on u = s^2 in [0, 1], which
keeps f relatively accurate up to the support edge (where the direct formula
cancels).  This script derives the fit from the series (not from any other
code of the project) and prints the coefficients, highest degree first, in
the form used in csrc/smki_gather.h (kSmkiQ).

    python -m paper_1909_04631_amd.kernel_poly
"""
import math

import numpy as np

DEGREE = 6


def q_series(u, terms=40):
    """Q(u) from the series above, in double precision."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    for n in range(2, terms):
        c = (-1) ** n * (2 * n - 2) * (2 * math.pi) ** (2 * n) / (3 * math.factorial(2 * n + 1))
        out = out + c * u ** (n - 2)
    return out


def fit(degree=DEGREE, nodes=8000, rounds=30):
    """Relative least-squares fit on Chebyshev nodes of [0, 1], reweighted
    towards the minimax relative error (Lawson iterations)."""
    x = 0.5 * (1.0 - np.cos(np.pi * (np.arange(nodes) + 0.5) / nodes))
    y = q_series(x)
    w = 1.0 / np.abs(y)
    coef = np.polyfit(x, y, degree, w=w)
    for _ in range(rounds):
        coef = np.polyfit(x, y, degree, w=w)
        e = np.abs(np.polyval(coef, x) - y) / np.abs(y)
        w = w * np.sqrt(e / e.max() + 1e-3)
    return coef


def f32_horner_error(coef, samples=200001):
    """Largest relative error of Q evaluated in binary32 with fused multiply-add."""
    u = np.linspace(0.0, 1.0, samples)
    uf = u.astype(np.float32)
    c32 = np.asarray(coef, dtype=np.float32)
    acc = np.full_like(uf, c32[0])
    for c in c32[1:]:
        acc = (acc.astype(np.float64) * uf.astype(np.float64) + np.float64(c)).astype(np.float32)
    ref = q_series(u)
    return float(np.max(np.abs(acc.astype(np.float64) - ref) / np.abs(ref)))


if __name__ == "__main__":
    c = fit()
    u = np.linspace(0.0, 1.0, 200001)
    print("fit max relative error (double): %.3e" % np.max(np.abs(np.polyval(c, u) - q_series(u)) / np.abs(q_series(u))))
    print("binary32 FMA Horner max relative error: %.3e" % f32_horner_error(c))
    print("static constexpr double kSmkiQ[SMKI_POLY_N] = {" + ", ".join(repr(float(v)) for v in c) + "};")
