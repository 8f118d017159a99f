"""Pin of the oracle's correctly rounded exp, log, sin and cos (used by its Monte-Carlo step)
against 60-digit decimal arithmetic: every result must be the nearest double."""
import math
import random
from decimal import Decimal, getcontext

import pytest

import oracle

getcontext().prec = 60


def _atan_inv(x):
    x = Decimal(x)
    s, t, n, sign, x2 = Decimal(0), 1 / x, 1, 1, x * x
    while True:
        term = t / n
        if abs(term) < Decimal(10) ** -58:
            return s
        s += sign * term
        t /= x2
        n += 2
        sign = -sign


PI = 16 * _atan_inv(5) - 4 * _atan_inv(239)   # Machin's formula


def _series(x, first, start):
    x = Decimal(x)
    r = x - (x / (2 * PI)).to_integral_value() * 2 * PI
    s, t, n = Decimal(0), first(r), start
    while abs(t) > Decimal(10) ** -58:
        s += t
        t = -t * r * r / ((n + 1) * (n + 2))
        n += 2
    return s


def _sin(x):
    return float(_series(x, lambda r: r, 1))


def _cos(x):
    return float(_series(x, lambda r: Decimal(1), 0))


@pytest.mark.parametrize("seed", [1, 2])
def test_correct_rounding_against_decimal(seed):
    rng = random.Random(seed)
    L = oracle.lib()
    for _ in range(1500):
        x = rng.uniform(-40.0, 5.0)
        assert L.oracle_cr_exp(x) == float(Decimal(x).exp())
        y = math.exp(rng.uniform(-40.0, 10.0))
        assert L.oracle_cr_log(y) == float(Decimal(y).ln())
        z = rng.uniform(-700.0, 700.0)
        assert L.oracle_cr_sin(z) == _sin(z)
        assert L.oracle_cr_cos(z) == _cos(z)


def test_special_values():
    L = oracle.lib()
    assert L.oracle_cr_exp(0.0) == 1.0
    assert L.oracle_cr_log(1.0) == 0.0
    assert L.oracle_cr_log(2.0) == math.log(2.0)
    assert L.oracle_cr_sin(0.0) == 0.0 and L.oracle_cr_cos(0.0) == 1.0
    # arguments near 1 and tiny logs keep full relative accuracy
    assert L.oracle_cr_log(1.0 + 2 ** -40) == float(Decimal(1.0 + 2 ** -40).ln())
