"""The FP64 logarithm and sine/cosine of the Box-Muller transform
(log_unit and sincos_angle in ssm_device.hpp), checked on the CPU: their
constants are read from the kernel source and compared with the exact
values, and their steps, restated here with one rounding per fused
multiply-add, are compared with 60-digit values over the inputs the
transform can see.  The device code itself is held to the oracle's libm
normals by the GPU Brownian tests."""
import math
import os
import random
import re
from fractions import Fraction

import mpmath as mp

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2105_09688_amd", "csrc", "ssm_device.hpp")
TXT = open(SRC).read()


def _array(name):
    body = re.search(r"constexpr double " + name + r"\[\d+\] = \{(.*?)\};", TXT, re.S).group(1)
    return [float.fromhex(re.sub(r"//.*", "", t).strip()) for t in body.split(",") if t.strip()]


def _scalar(name):
    return float.fromhex(re.search(name + r" = (-?0x[0-9a-fp.+-]+)", TXT).group(1))


def _fma(a, b, c):
    with mp.workdps(80):
        return float(mp.mpf(a) * mp.mpf(b) + mp.mpf(c))


def _ulps(got, ref):
    with mp.workdps(60):
        ref = mp.mpf(ref)
        if ref == 0:
            return 0.0 if got == 0 else float("inf")
        return float(abs(mp.mpf(got) - ref) / mp.mpf(2) ** (mp.floor(mp.log(abs(ref), 2)) - 52))


def test_constants_are_the_rounded_exact_values():
    assert _array("inv_odd") == [float(Fraction(1, 2 * k + 1)) for k in range(1, 12)]
    assert _array("sin_c") == [float(Fraction((-1) ** k, math.factorial(2 * k + 1))) for k in range(1, 10)]
    assert _array("cos_c") == [float(Fraction((-1) ** k, math.factorial(2 * k))) for k in range(1, 10)]
    with mp.workdps(100):
        a, b, c = _scalar("pio2_a"), _scalar("pio2_b"), _scalar("pio2_c")
        assert abs(mp.mpf(a) + b + c - mp.pi / 2) < mp.mpf(2) ** -159
        hi, lo = _scalar("ln2_hi"), _scalar("ln2_lo")
        assert abs(mp.mpf(hi) + lo - mp.log(2)) < mp.mpf(2) ** -88
        assert (math.frexp(hi)[0] * 2 ** 33).is_integer()  # e * ln2_hi exact for |e| < 2^20


def _log_unit(u):
    inv_odd = _array("inv_odd")
    hi, lo = _scalar("ln2_hi"), _scalar("ln2_lo")
    m, e = math.frexp(u)
    if m < float.fromhex("0x1.6a09e667f3bcdp-1"):
        m, e = m * 2.0, e - 1
    s = (m - 1.0) / (m + 1.0)
    s2 = s * s
    p = inv_odd[10]
    for k in range(9, -1, -1):
        p = _fma(p, s2, inv_odd[k])
    at = _fma(s * s2, p, s)
    return _fma(float(e), hi, _fma(float(e), lo, 2.0 * at))


def _sincos_angle(x):
    sin_c, cos_c = _array("sin_c"), _array("cos_c")
    a, b, c = _scalar("pio2_a"), _scalar("pio2_b"), _scalar("pio2_c")
    k = float(round(x * float.fromhex("0x1.45f306dc9c883p-1")))
    r = _fma(-k, a, x)
    r = _fma(-k, b, r)
    r = _fma(-k, c, r)
    r2 = r * r
    ps, pc = sin_c[8], cos_c[8]
    for j in range(7, -1, -1):
        ps, pc = _fma(ps, r2, sin_c[j]), _fma(pc, r2, cos_c[j])
    sr, cr = _fma(r * r2, ps, r), _fma(r2, pc, 1.0)
    q = int(k) & 3
    aa, bb = (cr, sr) if q & 1 else (sr, cr)
    return (-aa if q & 2 else aa), (-bb if (q + 1) & 2 else bb)


def _unit_open(w):
    return ((w >> 11) + 0.5) * 2.0 ** -53


def test_log_within_one_and_a_half_ulp_on_unit_open_values():
    """Measured worst case 1.30 ulp (the rounded quotient s and the final sums)."""
    rng = random.Random(5)
    words = [rng.getrandbits(64) for _ in range(1500)] + [0, 2 ** 11, 2 ** 63, 2 ** 64 - 1, (2 ** 64 - 1) >> 1]
    words += [rng.getrandbits(64) >> rng.randrange(1, 60) for _ in range(300)]  # small u
    worst = 0.0
    for w in words:
        u = _unit_open(w)
        with mp.workdps(60):
            ref = mp.log(mp.mpf(u))
        worst = max(worst, _ulps(_log_unit(u), ref))
    assert worst <= 1.5, worst


def test_sincos_within_one_and_a_half_ulp_on_box_muller_angles():
    """Measured worst case 1.19 ulp, quadrant edges included."""
    rng = random.Random(6)
    two_pi = 6.283185307179586476925286766559
    us = [_unit_open(rng.getrandbits(64)) for _ in range(1500)]
    us += [k / 8 + d for k in range(9) for d in (-2.0 ** -40, 0.0, 2.0 ** -40)]  # near the quadrant edges
    us = [u for u in us if 0.0 < u < 1.0]
    worst = 0.0
    for u in us:
        x = two_pi * u
        s, c = _sincos_angle(x)
        with mp.workdps(60):
            worst = max(worst, _ulps(s, mp.sin(mp.mpf(x))), _ulps(c, mp.cos(mp.mpf(x))))
    assert worst <= 1.5, worst
