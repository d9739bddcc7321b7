"""Pins of the second-order oracle (P2, the lambda^2 coefficient of the density
matrix of H0 + lambda H1 + lambda^2 H2) against quantities fixed by mathematics:
second differences of the Newton-sign step (no eigensolver), first differences
of the first-order oracle, the explicit second-order Daleckii-Krein triple sum
with a generic divided difference, the 2x2 closed form, the second-order
blocks of D^2 = D and HD = DH, and the dense FP64 recursion."""
import numpy as np
import pytest

from oracle import exact, sp2pt
from workloads import dense_gapped_problem, sym_normal

from test_oracle_exact import p0_newton


def small(n=20, seed=11, gap=1.0):
    p = dense_gapped_problem(n, n // 2, gap, seed, h1="dense", k=1, h1_std=0.05)
    h2 = sym_normal(np.random.default_rng(seed + 100), n, 0.05)
    return p.H0, p.H1[0], h2, p.nocc


@pytest.mark.parametrize("with_h2", [False, True])
def test_p2_matches_second_difference_of_newton_p0(with_h2):
    h0, h1, h2, nocc = small()
    h2 = h2 if with_h2 else None
    _, _, p2 = exact.second_order_response(h0, h1, h2, nocc)
    h = 1e-3
    h2m = np.zeros_like(h0) if h2 is None else h2
    # P(h) - 2 P(0) + P(-h) = 2 h^2 P2 + O(h^4)
    d2 = (p0_newton(h0 + h * h1 + h * h * h2m, nocc) - 2 * p0_newton(h0, nocc)
          + p0_newton(h0 - h * h1 + h * h * h2m, nocc)) / (2 * h * h)
    assert np.abs(d2 - p2).max() < 1e-5 * max(1.0, np.abs(p2).max())


def test_p2_is_half_the_derivative_of_p1():
    """d/dh P1(H0 + h H1; H1) = D^2 P[H1, H1] = 2 P2 (no H2)."""
    h0, h1, _, nocc = small(seed=5)
    _, _, p2 = exact.second_order_response(h0, h1, None, nocc)
    h = 1e-4
    fd = (exact.density_response(h0 + h * h1, h1, nocc)
          - exact.density_response(h0 - h * h1, h1, nocc)) / (4 * h)
    assert np.abs(fd - p2).max() < 1e-7 * max(1.0, np.abs(p2).max())


def _theta_dd(x):
    """Divided difference of the step function (1 below the gap, 0 above) at
    distinct points, by the recursive definition."""
    if len(x) == 1:
        return 1.0 if x[0] < 0.0 else 0.0
    return (_theta_dd(x[:-1]) - _theta_dd(x[1:])) / (x[0] - x[-1])


def test_p2_matches_explicit_triple_sum():
    """Second-order Daleckii-Krein in the eigenbasis, summed term by term."""
    h0, h1, h2, nocc = small(n=8, seed=3)
    e, v = np.linalg.eigh(h0)
    t1, t2 = v.T @ h1 @ v, v.T @ h2 @ v
    n = len(e)
    pt = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            acc = 0.0
            for k in range(n):
                acc += _dd3(e[i], e[k], e[j]) * t1[i, k] * t1[k, j]
            acc += _dd2(e[i], e[j]) * t2[i, j]
            pt[i, j] = acc
    ref = v @ pt @ v.T
    _, _, p2 = exact.second_order_response(h0, h1, h2, nocc)
    assert np.abs(p2 - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def _dd2(x, y):
    # equal points: derivative of the step away from the gap is zero
    return 0.0 if x == y else _theta_dd([x, y])


def _dd3(x, y, z):
    pts = sorted([x, y, z])
    if pts[0] == pts[2]:
        return 0.0                            # second derivative, zero off the gap
    if pts[0] == pts[1]:
        a, b = pts[0], pts[2]                 # theta[a, a, b] = (theta'(a) - theta[a, b])/(a - b)
        return (0.0 - _theta_dd([a, b])) / (a - b)
    if pts[1] == pts[2]:
        a, b = pts[0], pts[1]                 # theta[a, b, b] = (theta[a, b] - theta'(b))/(a - b)
        return (_theta_dd([a, b]) - 0.0) / (a - b)
    return _theta_dd(pts)


def test_2x2_closed_form():
    """H(l) = [[-1, l b + l^2 c], [l b + l^2 c, 1]]: P = (I - H/r)/2 with
    r = sqrt(1 + (l b + l^2 c)^2), so P2 = diag(-b^2/4, b^2/4) - (c/2) offdiag."""
    b, c = 0.3, -0.7
    h0 = np.diag([-1.0, 1.0])
    h1 = np.array([[0.0, b], [b, 0.0]])
    h2 = np.array([[0.0, c], [c, 0.0]])
    _, _, p2 = exact.second_order_response(h0, h1, h2, 1)
    ref = np.array([[-b * b / 4, -c / 2], [-c / 2, b * b / 4]])
    assert np.abs(p2 - ref).max() < 1e-15


def test_second_order_invariants():
    h0, h1, h2, nocc = small(n=40, seed=9, gap=0.5)
    p0, p1, p2 = exact.second_order_response(h0, h1, h2, nocc)
    inv = exact.invariants2(h0, h1, h2, p0, p1, p2)
    scale = max(1.0, np.linalg.norm(p2))
    assert abs(inv["tr_p2"]) < 1e-12 * scale
    assert inv["idem2"] < 1e-12 * scale
    assert inv["comm2"] < 1e-11 * scale * np.abs(h0).max()


def test_dense_recursion_converges_to_p2():
    p = dense_gapped_problem(64, 32, 1.0, 7, h1="dense", k=1, h1_std=0.01)
    h2 = sym_normal(np.random.default_rng(3), 64, 0.01)
    for hh2 in (None, h2):
        _, (p1,), st = sp2pt.run(p.H0, p.H1, p.nocc, order2=True, h2=hh2)
        _, r1, r2 = exact.second_order_response(p.H0, p.H1[0], hh2, p.nocc)
        assert st["converged"]
        assert st["d2_layer"] >= st["d1_layer"][0] + 2
        assert exact.rel_fro(p1, r1) < 1e-9
        assert exact.rel_fro(st["p2"], r2) < 1e-9


def _mutant_oo_sign(e, v, h1, h2, nocc):
    p2 = exact.second_order_from_eigs(e, v, h1, h2, nocc)
    vo = v[:, :nocc]
    return p2 - 2 * vo @ (vo.T @ p2 @ vo) @ vo.T


def _mutant_no_h2(e, v, h1, h2, nocc):
    return exact.second_order_from_eigs(e, v, h1, None, nocc)


def _mutant_swap_blocks(e, v, h1, h2, nocc):
    p2 = exact.second_order_from_eigs(e, v, h1, h2, nocc)
    vo, vv = v[:, :nocc], v[:, nocc:]
    oo = vo @ (vo.T @ p2 @ vo) @ vo.T
    vvb = vv @ (vv.T @ p2 @ vv) @ vv.T
    return p2 - oo - vvb - 0.5 * (oo + vvb)


@pytest.mark.parametrize("mutant", [_mutant_oo_sign, _mutant_no_h2, _mutant_swap_blocks])
def test_pins_reject_mutants(mutant):
    h0, h1, h2, nocc = small(seed=13)
    e, v = np.linalg.eigh(h0)
    bad = mutant(e, v, h1, h2, nocc)
    h = 1e-3
    d2 = (p0_newton(h0 + h * h1 + h * h * h2, nocc) - 2 * p0_newton(h0, nocc)
          + p0_newton(h0 - h * h1 + h * h * h2, nocc)) / (2 * h * h)
    p0 = p0_newton(h0, nocc)
    p1 = exact.density_response(h0, h1, nocc)
    inv = exact.invariants2(h0, h1, h2, p0, p1, bad)
    fails_fd = np.abs(d2 - bad).max() > 1e-4 * max(1.0, np.abs(bad).max())
    fails_inv = inv["idem2"] > 1e-8 or inv["comm2"] > 1e-8
    assert fails_fd and fails_inv
