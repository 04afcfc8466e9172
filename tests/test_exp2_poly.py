"""The FP64 exponential of the pair kernels (exp2_fast<double> in
ssm_kernels.hpp) checked on the CPU: its 12 polynomial coefficients are read
from the kernel source and evaluated as the kernel does (Horner's scheme, one
rounding per fused multiply-add), against 2^x in 60-digit arithmetic."""
import math
import os
import random
import re

import mpmath as mp

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2105_09688_amd", "csrc", "ssm_kernels.hpp")


def _coefs():
    txt = open(SRC).read()
    body = re.search(r"exp2_poly_coef\(int k\)\s*\{\s*constexpr double c\[12\] = \{(.*?)\};", txt, re.S).group(1)
    c = [float.fromhex(t.strip()) for t in body.split(",")]
    assert len(c) == 12
    return c


def _fma(a, b, c):
    """a * b + c with one rounding to double (exact product and sum in mpmath)."""
    with mp.workdps(80):
        return float(mp.mpf(a) * mp.mpf(b) + mp.mpf(c))


def _exp2_kernel(x, c):
    """The kernel's steps: n = rint(x), r = x - n, Horner, ldexp by max(n, -1100)."""
    n = float(round(x)) if abs(x) < 2.0 ** 52 else x  # rint: ties to even, as Python's round
    r = x - n
    p = c[11]
    for k in range(10, -1, -1):
        p = _fma(p, r, c[k])
    return math.ldexp(p, int(max(n, -1100.0)))


def _ulps(got, x):
    with mp.workdps(60):
        ref = mp.power(2, mp.mpf(x))
        e = max(mp.floor(mp.log(ref, 2)), -1022) - 52
        return float(abs(mp.mpf(got) - ref) / mp.mpf(2) ** e)


def test_polynomial_interpolates_2_to_the_r_at_the_chebyshev_nodes():
    c = _coefs()
    with mp.workdps(60):
        for k in range(12):
            x = mp.mpf("0.5") * mp.cos((2 * k + 1) * mp.pi / 24)
            p = sum(mp.mpf(c[j]) * x ** j for j in range(12))
            assert abs(p / mp.power(2, x) - 1) < 2e-16  # only the coefficients' rounding


def test_within_one_ulp_on_the_reduced_range_and_beyond():
    c = _coefs()
    rng = random.Random(3)
    xs = [rng.uniform(-0.5, 0.5) for _ in range(1500)] + [rng.uniform(-60.0, 0.0) for _ in range(500)]
    xs += [0.0, -0.5, -1.5, -0.25, -1e-300, -2.0 ** -60, -1021.3, -1022.0]
    worst = max(_ulps(_exp2_kernel(x, c), x) for x in xs)
    assert worst <= 1.0, worst


def test_subnormal_results_and_underflow_to_zero():
    c = _coefs()
    for x in (-1023.5, -1040.25, -1073.0, -1074.0):
        assert _exp2_kernel(x, c) > 0.0 and _ulps(_exp2_kernel(x, c), x) <= 1.0, x
    for x in (-1076.0, -1100.0, -1e6, -4e30, -1e300):
        assert _exp2_kernel(x, c) == 0.0, x
    assert _exp2_kernel(-0.0, c) == 1.0
