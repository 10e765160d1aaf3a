"""Coefficients of tan_halfpi (csrc/device_common.hpp).

Lambert's continued fraction tan x = x / (1 - x^2 / (3 - x^2 / (5 - ...)))
cut after the term 2m + 1 is a rational function x N(x^2) / D(x^2) with
exact rational coefficients.  This script forms it with Fractions (m = 8),
normalises N(0) = D(0) = 1, prints the coefficients rounded to double, the
truncation error on [0, pi/4] against a much deeper cut, and the error in
ulp of a model of the device evaluation (Horner with fused multiply-adds,
two-part pi/2 reduction above pi/4) against the exact tangent of the same
double argument.

    python paper_1407_7595_amd/tan_coefficients.py
"""
import math
import random
from fractions import Fraction as Fr

PIO2_HI = 1.5707963267948966
PIO2_LO = 6.123233995736766e-17
# pi/2 to 53 digits, for the exact reference
PIO2 = Fr(157079632679489661923132169163975144209858469968755291, 10 ** 53)


def lambert(m):
    """(N, D) with tan x = x N(y) / D(y), y = x^2, cut after the term 2m + 1"""
    A, B = [Fr(2 * m + 1)], [Fr(1)]
    for k in range(m - 1, -1, -1):
        # (2k + 1) - y B / A = ((2k + 1) A - y B) / A
        n = max(len(A), len(B) + 1)
        nxt = [Fr(0)] * n
        for i, c in enumerate(A):
            nxt[i] += (2 * k + 1) * c
        for i, c in enumerate(B):
            nxt[i + 1] -= c
        A, B = nxt, A
    return B, A


def rational(N, D, x):
    y = x * x
    return x * sum(c * y ** i for i, c in enumerate(N)) / sum(c * y ** i for i, c in enumerate(D))


def fma(a, b, c):
    return float(Fr(a) * Fr(b) + Fr(c))


def device_model(theta, n, d):
    a = abs(theta)
    big = a > 0.78539816339744831
    x = float(Fr(float(Fr(PIO2_HI) - Fr(a))) + Fr(PIO2_LO)) if big else a
    y = float(Fr(x) * Fr(x))
    p = n[-1]
    for c in reversed(n[:-1]):
        p = fma(p, y, c)
    q = d[-1]
    for c in reversed(d[:-1]):
        q = fma(q, y, c)
    num = float(Fr(x) * Fr(p))
    t = float(Fr(q) / Fr(num)) if big else float(Fr(num) / Fr(q))
    return math.copysign(t, theta)


def main(m=8, samples=3000):
    N, D = lambert(m)
    n = [float(c / N[0]) for c in N]
    d = [float(c / D[0]) for c in D]
    print("N:", ", ".join(repr(c) for c in n))
    print("D:", ", ".join(repr(c) for c in d))
    Nr, Dr = lambert(m + 20)
    trunc = max(abs(float((rational(N, D, x) - rational(Nr, Dr, x)) / rational(Nr, Dr, x)))
                for x in (Fr(i, 400) * Fr(785398163397448, 10 ** 15) for i in range(1, 401)))
    print(f"truncation error on [0, pi/4]: {trunc:.3g} relative")
    rnd = random.Random(1)
    worst = 0.0
    for i in range(samples):
        th = rnd.uniform(-PIO2_HI, PIO2_HI)
        if i < 40:
            th = math.copysign(PIO2_HI - 10.0 ** (-1 - 0.3 * i), th)     # next to the pole
        a = abs(Fr(th))
        ref = 1 / rational(Nr, Dr, PIO2 - a) if a > PIO2 / 2 else rational(Nr, Dr, a)
        ref = ref if th >= 0 else -ref
        worst = max(worst, abs(float(Fr(device_model(th, n, d)) - ref)) / math.ulp(float(ref)))
    print(f"device model: worst error {worst:.2f} ulp over {samples} arguments")


if __name__ == "__main__":
    main()
