"""The sweep kernels divide by 6 without a division instruction:
q = RN(x * zh + RN(x * zl)) with zh = RN(1/6), zl = RN(1/6 - zh), one fused
multiply-add (Brisebarre, Muller, Raina, IEEE Trans. Computers 2004), and a
true division only for |x| below 2^-1000 (FP64) / 2^-100 (FP32).

These CPU checks evaluate that formula in exact rational arithmetic, rounding
where the hardware rounds, and compare it with IEEE division: the constants
are the rounded reciprocal and its remainder, the identity holds across
binades, signs, residues of the significand mod 3, binade edges and the
extremes of the range, and below the cut-off a tie exists that the formula
would round the wrong way (which is why the kernels divide there)."""
import math
import random
from fractions import Fraction as Fr

import numpy as np

ZH64 = float.fromhex("0x1.5555555555555p-3")
ZL64 = float.fromhex("0x1.5555555555555p-57")
ZH32 = float.fromhex("0x1.555556p-3")
ZL32 = float.fromhex("-0x1.555556p-28")


def rn32(q: Fr) -> float:
    """Round a rational to the nearest float32 (ties to even), subnormals included."""
    if q == 0:
        return 0.0
    s = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fr(2) ** e > a:
        e -= 1
    while Fr(2) ** (e + 1) <= a:
        e += 1
    ulp = Fr(2) ** (max(e, -126) - 23)
    n = a / ulp
    fl = n.numerator // n.denominator
    rem = n - fl
    if rem > Fr(1, 2) or (rem == Fr(1, 2) and fl % 2 == 1):
        fl += 1
    return s * float(fl * ulp)


def fused64(x: float) -> float:
    return float(Fr(x) * Fr(ZH64) + Fr(float(Fr(x) * Fr(ZL64))))


def fused32(x: float) -> float:
    return rn32(Fr(x) * Fr(ZH32) + Fr(rn32(Fr(x) * Fr(ZL32))))


def kernel64(x: float) -> float:
    """The kernels' div6 for FP64: the true quotient below the cut-off
    (zeros included, which keeps the sign of -0), else the fused form."""
    return x / 6.0 if abs(x) < 2.0 ** -1000 else fused64(x)


def kernel32(x: float) -> float:
    return float(np.float32(x) / np.float32(6.0)) if abs(x) < 2.0 ** -100 else fused32(x)


def test_constants_are_the_rounded_reciprocal_and_remainder():
    assert ZH64 == float(Fr(1, 6))
    assert ZL64 == float(Fr(1, 6) - Fr(ZH64))
    assert ZH32 == rn32(Fr(1, 6))
    assert ZL32 == rn32(Fr(1, 6) - Fr(ZH32))
    assert np.float32(ZH32) == ZH32 and np.float32(ZL32) == ZL32


def samples64(rng):
    xs = []
    for _ in range(4000):
        m = rng.getrandbits(52) | (1 << 52)
        e = rng.randint(-1000 - 52, 1023 - 53)
        xs.append(math.ldexp(m, e) * rng.choice((1, -1)))
    for r in range(3):  # significand residues mod 3, and binade edges around 6 * 2^k
        for k in (-900, -3, 0, 1, 5, 700):
            m = (1 << 52) + 3 * rng.getrandbits(40) + r
            xs.append(math.ldexp(m, k))
            xs.append(math.ldexp(6.0, k) * (1 + r * 2.0 ** -52))
            xs.append(math.ldexp(6.0, k) * (1 - (r + 1) * 2.0 ** -53))
    xs += [0.0, -0.0, 1.0, 6.0, 3.0, 1.0 / 3.0, np.finfo(np.float64).max, -np.finfo(np.float64).max,
           2.0 ** -1000, -(2.0 ** -1000), np.nextafter(2.0 ** -1000, 1.0)]
    return xs


def test_fp64_identity():
    rng = random.Random(61)
    for x in samples64(rng):
        want = x / 6.0
        got = kernel64(x)
        assert got == want and math.copysign(1, got) == math.copysign(1, want), x.hex()


def test_fp32_identity():
    rng = random.Random(62)
    xs = []
    for _ in range(4000):
        m = rng.getrandbits(23) | (1 << 23)
        e = rng.randint(-100 - 23, 104)
        xs.append(float(np.float32(math.ldexp(m, e) * rng.choice((1, -1)))))
    xs += [float(np.finfo(np.float32).max), 2.0 ** -100, 6.0, 1.0, 3.0, 0.0, -0.0]
    for x in xs:
        want = float(np.float32(x) / np.float32(6.0))
        got = kernel32(x)
        assert got == want and math.copysign(1, got) == math.copysign(1, want), float(x).hex()


def test_below_the_cutoff_a_tie_needs_the_division():
    # 9 * 2^-1074 / 6 = 1.5 * 2^-1074 is a tie on the subnormal grid: IEEE
    # rounds to 2 * 2^-1074 (even), the fused formula to 1 * 2^-1074
    x = 9 * 2.0 ** -1074
    assert x / 6.0 == 2 * 2.0 ** -1074
    assert fused64(x) == 2.0 ** -1074
    assert x < 2.0 ** -1000
