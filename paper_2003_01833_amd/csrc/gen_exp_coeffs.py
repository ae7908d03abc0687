"""Regenerates the polynomial coefficients of exp2_scaled in devmath.hpp.

The polynomial of degree 9 that interpolates 2^f at the 10 Chebyshev points of
the first kind on [-1/2, 1/2], in monomial form, computed in 60-digit arithmetic
and rounded to double. Prints the coefficients (hex) and the largest relative
error of the double-precision Horner evaluation (with fused multiply-adds) on a
dense grid.
"""
import mpmath as mp
import numpy as np


def main(degree: int = 9):
    mp.mp.dps = 60
    a = mp.mpf(1) / 2
    nodes = [a * mp.cos((2 * i + 1) * mp.pi / (2 * (degree + 1))) for i in range(degree + 1)]
    V = mp.matrix([[x ** j for j in range(degree + 1)] for x in nodes])
    c = mp.lu_solve(V, mp.matrix([mp.mpf(2) ** x for x in nodes]))
    coef = [float(c[j]) for j in range(degree + 1)]
    for j in range(degree, -1, -1):
        print(f"c{j} = {coef[j].hex()}")
    worst = 0.0
    for x in np.linspace(-0.5, 0.5, 4001):
        p = coef[degree]
        for j in range(degree - 1, -1, -1):
            p = float(mp.mpf(p) * mp.mpf(x) + mp.mpf(coef[j]))
        ex = mp.mpf(2) ** mp.mpf(x)
        worst = max(worst, float(abs((p - ex) / ex)))
    print(f"max relative error {worst:.3e} = {worst / 2 ** -53:.3f} ulp")


if __name__ == "__main__":
    main()
