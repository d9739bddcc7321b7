"""Closed-form constants of the D1 stopping criterion (Sec. IV; test infrastructure only).

A sigma-flip pair applies h(x) = 2x^2 - x^4 (x^2 then 2x - x^2) or
h(x) = (2x - x^2)^2 (the other order).  Their derivatives factor as
h'(x) = 4x(1-x)(1+x) and h'(x) = 4x(1-x)(2-x), so |h'(x)| / |x - x^2| equals
4|1+x| or 4|2-x|.  On [-0.25, 1.25] the largest value is 9 (C_pt = 9).  If
every eigenvalue obeys |x - x^2| <= eps, x lies in
[(1 - sqrt(1+4 eps))/2, (1 + sqrt(1+4 eps))/2], which gives
C_pt(eps) = 6 + 4 sqrt(0.25 + eps).  The inflection points (h'' = 0) are
1 - 1/sqrt(3) for (2x - x^2)^2 and 1/sqrt(3) for 2x^2 - x^4.

Pins: tests/test_oracle_constants.py maximises the ratio and locates h'' sign
changes numerically on fine grids.
"""
import math


def h_sq_then_flip(x):
    """x -> x^2 then y -> 2y - y^2:  2x^2 - x^4."""
    return 2 * x * x - x ** 4


def h_flip_then_sq(x):
    """x -> 2x - x^2 then y -> y^2:  (2x - x^2)^2."""
    return (2 * x - x * x) ** 2


def dh_sq_then_flip(x):
    return 4 * x * (1 - x) * (1 + x)


def dh_flip_then_sq(x):
    return 4 * x * (1 - x) * (2 - x)


def c_pt(eps: float) -> float:
    """Smallest constant valid for all eigenvalues with |x - x^2| <= eps."""
    return 6.0 + 4.0 * math.sqrt(0.25 + eps)


C_PT_DEFAULT = 9.0
INFLECTION_FLIP_THEN_SQ = 1.0 - 1.0 / math.sqrt(3.0)
INFLECTION_SQ_THEN_FLIP = 1.0 / math.sqrt(3.0)
