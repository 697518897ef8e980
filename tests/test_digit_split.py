"""CPU: the integer arithmetic of the INT8 digit form (Sec. 2, Eqs. (10)-(17) as reworked for
the matrix cores), emulated exactly in Python integers.

These pin the design the kernels rely on, not the oracle:
  * q = rint(u 2^(QB - S)) (round to nearest, ties to even) with |q| <= 2^QB, QB = 8M - 2,
    is recovered exactly from the FP64 steps the kernels use (xr = rint(x), hd =
    floor(xr 2^-32), lo = xr - hd 2^32 with 0 <= lo < 2^32: every step exact, every
    conversion in range) for every |x| < 2^62;
  * the bytes of q + sum_j 128 * 256^j, less 128, are M balanced digits d_j in [-128, 127]
    with sum_j 256^j d_j = q, and the bytes above M are exactly 128 (digit 0);
  * the INT32 pair sums C = 256 A d_hi + A d_lo of the integer matrices stay below 2^31,
    and the bf16 form's partial sums below 2^24, for the worst-case digits;
  * recombining the pair sums by Horner with factor 2^16 gives A q exactly (in integers).
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import element as el


def _int_matrices():
    Kl, Km = el.ovfem_reference_exact()
    AL = [[int(Fraction(x) * 256) for x in row] for row in Kl]
    AM = [[int(Fraction(x) * 128) for x in row] for row in Km]
    return AL, AM


def _q_two_steps(x):
    """The kernels' FP64 steps for q = rint(x) (x a double, |x| < 2^62): xr = rint(x) in the
    default rounding mode (Python's round() of a float also rounds ties to even); hd =
    floor(xr 2^-32), exact; lo = xr - hd 2^32, an integer in [0, 2^32) and so exact (Python's
    double subtraction is then the kernels' fma), converted to uint32 in range."""
    xr = float(round(x))
    assert xr == x or abs(xr - x) <= 0.5
    hd = math.floor(xr * 2.0 ** -32)
    lo = xr - hd * 2.0 ** 32
    assert 0 <= lo < 2 ** 32 and lo == int(lo)
    return int(hd) * 2 ** 32 + int(lo)


def _digits(q, M):
    bias = sum(128 * 256 ** j for j in range(8))
    b = (q + bias) % 2 ** 64
    d = [((b >> (8 * j)) & 0xFF) - 128 for j in range(8)]
    return d[:M], d[M:]


@pytest.mark.parametrize("M", [4, 5, 6, 7, 8])
def test_split_and_reconstruct_are_exact(M):
    QB = 8 * M - 2
    rng = random.Random(M)
    cases = [0.0, 0.5, -0.5, 1 - 2 ** -53, -(1 - 2 ** -53), 2 ** -60, -(2 ** -60), -(2.0 ** -300)]
    cases += [math.ldexp(k + 0.5, -QB) for k in (-3, -2, -1, 0, 1, 2)]  # ties
    if QB <= 51:  # values that round to q = +-2^QB, the largest magnitude
        cases += [math.ldexp(2.0 ** QB - 0.25, -QB), -math.ldexp(2.0 ** QB - 0.25, -QB)]
    cases += [rng.uniform(-1, 1) * 2.0 ** -rng.randrange(0, 70) for _ in range(4000)]
    for u in cases:  # u already scaled by 2^-S: |u| < 1 (the staging exponent makes it so)
        x = math.ldexp(u, QB)
        q = _q_two_steps(x) if M > 4 else int(round(x))
        assert q == round(Fraction(u) * 2 ** QB)
        assert abs(q) <= 2 ** QB
        if abs(u) < 2.0 ** (-QB - 1):
            assert q == 0  # tiny values round to zero, whatever their sign
        d, rest = _digits(q, M)
        assert all(-128 <= v <= 127 for v in d)
        assert all(v == 0 for v in rest)
        assert sum(v * 256 ** j for j, v in enumerate(d)) == q


def test_pair_sums_fit_int32_and_fp32():
    AL, AM = _int_matrices()
    rowabs = max(max(sum(abs(a) for a in row) for row in AL), max(sum(abs(a) for a in row) for row in AM))
    assert rowabs == 384
    # worst case over digits in [-128, 127]: every term at its largest magnitude
    worst_i32 = max(sum(abs(a) for a in row) * (128 * 256 + 128) for row in AL + AM)
    assert worst_i32 < 2 ** 31
    # bf16 form: A (256 d_hi) + A (d_lo + 128), partial sums below 2^24
    worst_f32 = max(sum(abs(a) for a in row) * (128 * 256 + 255) for row in AL + AM)
    assert worst_f32 < 2 ** 24


@pytest.mark.parametrize("M", [4, 6, 8])
def test_horner_over_pair_sums_is_the_integer_product(M):
    """C_p = 256 A d_{2p+1} + A d_{2p} per digit pair (top pair single when M is odd),
    then R = sum_p 2^(16 p) C_p equals A q exactly, row by row."""
    AL, AM = _int_matrices()
    rng = np.random.default_rng(M)
    QB = 8 * M - 2
    for trial in range(30):
        u = rng.uniform(-1, 1, 24) * 2.0 ** -rng.integers(0, 20, 24)
        q = [round(Fraction(float(v)) * 2 ** QB) for v in u]
        digits = [_digits(v, M)[0] for v in q]
        for A in (AL, AM):
            for row in A:
                exact = sum(a * v for a, v in zip(row, q))
                R = 0
                for p in reversed(range((M + 1) // 2)):
                    lo = sum(a * digits[k][2 * p] for k, a in enumerate(row))
                    hi = sum(a * digits[k][2 * p + 1] for k, a in enumerate(row)) if 2 * p + 1 < M else 0
                    C = 256 * hi + lo
                    assert abs(C) < 2 ** 31
                    R = R * 2 ** 16 + C
                assert R == exact
