"""The FP64 tangent of the Breit-Wigner maps (tan_halfpi): its coefficients
are those of Lambert's continued fraction cut after the term 17, its
truncation error on [0, pi/4] is below 1e-18, and a model of its device
arithmetic stays within 3 ulp of the exact tangent, next to the pole
included (the exact reference is a much deeper cut of the same fraction)."""
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", "paper_1407_7595_amd"))
import tan_coefficients as tc  # noqa: E402


def test_coefficients_in_device_source():
    N, D = tc.lambert(8)
    n = [float(c / N[0]) for c in N]
    d = [float(c / D[0]) for c in D]
    src = open(os.path.join(HERE, "..", "paper_1407_7595_amd", "csrc", "device_common.hpp")).read()
    body = src[src.index("double tan_halfpi("):]
    body = body[:body.index("\n}\n")]
    got_n = [float(v) for v in re.findall(r"double n = ([-0-9.e+]+);", body)
             + re.findall(r"n = __fma_rn\(n, y, ([-0-9.e+]+)\);", body)]
    got_d = [float(v) for v in re.findall(r"double d = ([-0-9.e+]+);", body)
             + re.findall(r"d = __fma_rn\(d, y, ([-0-9.e+]+)\);", body)]
    assert got_n == n[::-1]
    assert got_d == d[::-1]


def test_lambert_is_tangent():
    from fractions import Fraction as Fr
    import math
    N, D = tc.lambert(8)
    # against the library tangent (0.5 ulp) across the reduced range
    for x in (1e-3, 0.1, 0.5, 0.785):
        assert abs(float(tc.rational(N, D, Fr(x))) - math.tan(x)) <= 2 * math.ulp(math.tan(x))


def test_device_model_within_3ulp(capsys):
    tc.main(samples=500)
    out = capsys.readouterr().out
    trunc = float(re.search(r"truncation error on \[0, pi/4\]: ([0-9.e+-]+)", out).group(1))
    worst = float(re.search(r"worst error ([0-9.]+) ulp", out).group(1))
    assert trunc < 1e-18
    assert worst < 3.0
