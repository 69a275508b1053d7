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

The adjoint of the differentiable form needs f'(r)/r (the gradient of f(|x|/l)
with respect to x is f'(r)/r times x/l^2).  Differentiating the series,
f'(1 - s) = sum_{n >= 2} (-1)^(n+1) (2n - 2)(2 pi)^{2n} s^{2n} / (3 (2n)!), so
f'(r)/r = s^4 P(s) with P(s) = [f'(1 - s) / s^4] / (1 - s), finite at s = 1
(r = 0, limit -4 pi^2 / 3).  P is fitted by a degree-10 polynomial in s on
[0, 1] (relative error about 2e-8); those are the coefficients kG of
csrc/loss.hip.

    python -m paper_1909_04631_amd.kernel_poly
"""
import math

import numpy as np

DEGREE = 6
DEGREE_G = 10


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


def p_reference(s):
    """P(s) = f'(r) / (r s^4), r = 1 - s, in double: the series of f'(1 - s)/s^4
    divided by r for s < 1/2; the closed form f'(r) = -(2 pi/3)(1 - r) sin(2 pi r)
    + (2/3)(cos(2 pi r) - 1) divided by r s^4 otherwise (its limit at r = 0)."""
    s = np.asarray(s, dtype=np.float64)
    r = 1.0 - s
    out = np.empty_like(s)
    lo = s < 0.5
    g = np.zeros_like(s[lo])
    for n in range(2, 40):
        c = (-1) ** (n + 1) * (2 * n - 2) * (2 * math.pi) ** (2 * n) / (3 * math.factorial(2 * n))
        g = g + c * s[lo] ** (2 * n - 4)
    out[lo] = g / r[lo]
    rr, ss = r[~lo], s[~lo]
    safe = np.where(rr > 1e-6, rr, 1.0)
    dfdr = -(2 * math.pi / 3) * (1 - safe) * np.sin(2 * math.pi * safe) + \
        (2.0 / 3.0) * (np.cos(2 * math.pi * safe) - 1.0)
    out[~lo] = np.where(rr > 1e-6, dfdr / safe, -4.0 * math.pi ** 2 / 3.0) / ss ** 4
    return out


def fit_dfdr(degree=DEGREE_G, nodes=8000, rounds=30):
    """The same relative fit (Chebyshev nodes, Lawson reweighting) of P on s in [0, 1]."""
    x = 0.5 * (1.0 - np.cos(np.pi * (np.arange(nodes) + 0.5) / nodes))
    y = p_reference(x)
    w = 1.0 / np.abs(y)
    coef = np.polyfit(x, y, degree, w=w)
    for _ in range(rounds):
        coef = np.polyfit(x, y, degree, w=w)
        e = np.abs(np.polyval(coef, x) - y) / np.abs(y)
        w = w * np.sqrt(e / e.max() + 1e-3)
    return coef


if __name__ == "__main__":
    g = fit_dfdr()
    s = np.linspace(0.0, 1.0, 200001)
    print("f'(r)/r fit max relative error (double): %.3e" %
          np.max(np.abs(np.polyval(g, s) - p_reference(s)) / np.abs(p_reference(s))))
    print("__constant__ float kG[11] = {" + ", ".join(repr(float(v)) + "f" for v in g) + "};")
    c = fit()
    u = np.linspace(0.0, 1.0, 200001)
    print("fit max relative error (double): %.3e" % np.max(np.abs(np.polyval(c, u) - q_series(u)) / np.abs(q_series(u))))
    print("binary32 FMA Horner max relative error: %.3e" % f32_horner_error(c))
    print("static constexpr double kSmkiQ[SMKI_POLY_N] = {" + ", ".join(repr(float(v)) for v in c) + "};")
