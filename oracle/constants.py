"""Closed-form constants of the D1 stopping criterion (Sec. IV; test infrastructure only).

A sigma-flip pair applies h(x) = 2x^2 - x^4 (x^2 then 2x - x^2) or
h(x) = (2x - x^2)^2 (the other order).  Their derivatives factor as
h'(x) = 4x(1-x)(1+x) and h'(x) = 4x(1-x)(2-x), so |h'(x)| / |x - x^2| equals
4|1+x| or 4|2-x|.  On [-0.25, 1.25] the largest value is 9 (C_pt = 9).  If
every eigenvalue obeys |x - x^2| <= eps, x lies in
[(1 - sqrt(1+4 eps))/2, (1 + sqrt(1+4 eps))/2], which gives
C_pt(eps) = 6 + 4 sqrt(0.25 + eps).  The inflection points (h'' = 0) are
1 - 1/sqrt(3) for (2x - x^2)^2 and 1/sqrt(3) for 2x^2 - x^4.

The 4.5 factor of the D0 test (Alg. 2) is pinned the same way: after a
sigma flip the idempotency error contracts as IdErr_n <= 4.409 IdErr_{n-2}^2 in
exact arithmetic (D0_PAIR_BOUND below), so 4.5 sits just above the largest
noise-free ratio.

Pins: tests/test_oracle_constants.py maximises the ratios and locates h'' sign
changes numerically on fine grids, and checks the contraction bound on the
eigenvalue chains of the eigenbasis recursion.
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


# ---------------------------------------------------------------- the D0 factor (Alg. 2)
# IdErr_n = Tr(S_{n-1} - S_{n-1}^2) = sum_i (x_i - x_i^2) over the eigenvalues
# x_i in [0, 1] of S_{n-1}.  When sigma_{n-1} != sigma_{n-2}, S_{n-1} = h(S_{n-3})
# for one of the two flip-pair maps above, and
#   2x^2 - x^4:   h - h^2 = x^2 (2 - x^2) (1 - x^2)^2,
#                 (h - h^2) / (x - x^2)^2 = (2 - x^2)(1 + x)^2 =: r(x);
#   (2x - x^2)^2 = 1 - h_sq_then_flip(1 - x), so its ratio is r(1 - x).
# r'(x) = 2 (1 + x)(2 - x - 2x^2) vanishes on [0, 1] only at x* = (sqrt(17) - 1)/4,
# where r(x*) = (71 + 17 sqrt(17)) / 32 = 4.409...  Every term is non-negative,
# so sum (x - x^2)^2 <= (sum (x - x^2))^2 and, in exact arithmetic,
#   IdErr_n <= D0_PAIR_BOUND * IdErr_{n-2}^2    after a sigma flip.
# Alg. 2 declares convergence when IdErr_n exceeds 4.5 IdErr_{n-2}^2: with
# 4.5 above this bound the test cannot fire on a noise-free chain, only once
# rounding noise stops the quadratic decrease.


def pair_ratio_sq_then_flip(x):
    """(h - h^2) / (x - x^2)^2 for h = 2x^2 - x^4, simplified: (2 - x^2)(1 + x)^2."""
    return (2.0 - x * x) * (1.0 + x) ** 2


def pair_ratio_flip_then_sq(x):
    """The same ratio for h = (2x - x^2)^2: pair_ratio_sq_then_flip(1 - x)."""
    return pair_ratio_sq_then_flip(1.0 - x)


D0_PAIR_ARGMAX = (math.sqrt(17.0) - 1.0) / 4.0          # for 2x^2 - x^4; 1 - it for the other
D0_PAIR_BOUND = (71.0 + 17.0 * math.sqrt(17.0)) / 32.0  # = 4.40915...
