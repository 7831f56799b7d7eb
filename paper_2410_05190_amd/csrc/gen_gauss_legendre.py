"""Writes the Gauss-Legendre tables used by the distance integrals (pe_device.h): the positive
nodes of P_n on [-1, 1] and their weights (n = 16 for the likelihood's integral, n = 8 for the
time marginal's per-node integrals), from numpy's Golub-Welsch routine with a Newton polish on the
Legendre recurrence, printed to 17 significant digits (exact round trip)."""
import numpy as np


def legendre(n, x):
    p0, p1 = np.ones_like(x), x
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    dp = n * (x * p1 - p0) / (x * x - 1)
    return p1, dp


def table(n, suffix):
    x, _ = np.polynomial.legendre.leggauss(n)
    for _ in range(3):
        p, dp = legendre(n, x)
        x = x - p / dp
    _, dp = legendre(n, x)
    w = 2.0 / ((1 - x * x) * dp * dp)
    pos = x > 0
    xs, ws = x[pos][::-1], w[pos][::-1]
    print("constexpr double kGlX%s[%d] = {%s};" % (suffix, n // 2, ", ".join(repr(float(v)) for v in xs)))
    print("constexpr double kGlW%s[%d] = {%s};" % (suffix, n // 2, ", ".join(repr(float(v)) for v in ws)))
    assert abs(2 * ws.sum() - 2.0) < 1e-14


def main():
    table(16, "")
    table(8, "8")


if __name__ == "__main__":
    main()
