"""Writes the 16-point Gauss-Legendre table used by the distance integral (pe_device.h): the
positive nodes of P_16 on [-1, 1] and their weights, from numpy's Golub-Welsch routine with a
Newton polish on the Legendre recurrence, printed to 17 significant digits (exact round trip)."""
import numpy as np


def legendre(n, x):
    p0, p1 = np.ones_like(x), x
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    dp = n * (x * p1 - p0) / (x * x - 1)
    return p1, dp


def main(n=16):
    x, _ = np.polynomial.legendre.leggauss(n)
    for _ in range(3):
        p, dp = legendre(n, x)
        x = x - p / dp
    _, dp = legendre(n, x)
    w = 2.0 / ((1 - x * x) * dp * dp)
    pos = x > 0
    xs, ws = x[pos][::-1], w[pos][::-1]
    print("constexpr double kGlX[%d] = {%s};" % (n // 2, ", ".join(repr(float(v)) for v in xs)))
    print("constexpr double kGlW[%d] = {%s};" % (n // 2, ", ".join(repr(float(v)) for v in ws)))
    assert abs(2 * ws.sum() - 2.0) < 1e-14


if __name__ == "__main__":
    main()
