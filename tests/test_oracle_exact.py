"""Pins of the exact FP64 oracle against quantities fixed by mathematics, not by
the oracle itself: a Newton sign iteration (no eigh), brute-force finite
differences (Eqs. FnD_2/FnD_4), the 2x2 closed form, the diagonal case and the
block identities of Sec. III.B."""
import numpy as np
import pytest

from oracle import exact
from workloads import banded_gapped_problem, dense_gapped_problem


def newton_sign(a, tol=1e-15, maxit=100):
    """Matrix sign by Newton's iteration X <- (X + X^{-1})/2 (no eigensolver)."""
    x = a.copy()
    for _ in range(maxit):
        xn = 0.5 * (x + np.linalg.inv(x))
        if np.linalg.norm(xn - x) <= tol * np.linalg.norm(xn):
            return xn
        x = xn
    return x


def p0_newton(h, nocc):
    """theta(mu I - H) with mu = 0: the generators centre the gap on zero."""
    n = h.shape[0]
    return 0.5 * (np.eye(n) - newton_sign(h))


def small(n=24, seed=7, gap=1.0, h1="dense", k=1):
    return dense_gapped_problem(n, n // 2, gap, seed, h1=h1, k=k, h1_std=0.05)


def test_p0_matches_newton_sign():
    p = small()
    p0 = exact.density_matrix(p.H0, p.nocc)
    assert np.abs(p0 - p0_newton(p.H0, p.nocc)).max() < 1e-12


def test_p0_diagonal_is_indicator():
    e = np.array([3.0, -1.0, 2.0, -4.0, 0.5, -0.25])
    p0 = exact.density_matrix(np.diag(e), 3)
    assert np.array_equal(np.diag(p0).round(14), (e < 0).astype(float))
    assert np.abs(p0 - np.diag(np.diag(p0))).max() < 1e-15


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_p1_matches_two_point_fd_of_newton_p0(seed):
    p = small(seed=seed)
    p1 = exact.density_response(p.H0, p.H1[0], p.nocc)
    fd = exact.fd_response_2pt(p0_newton, p.H0, p.H1[0], p.nocc, 1e-4)
    assert exact.rel_fro(fd, p1) < 1e-7


def test_fd_orders_two_and_four_point():
    """The 4-point stencil is O(h^4), the 2-point one O(h^2) (Eqs. FnD_2, FnD_4)."""
    p = small(seed=11, gap=0.6)
    h1 = p.H1[0] * 20.0
    p1 = exact.density_response(p.H0, h1, p.nocc)
    e2 = [exact.rel_fro(exact.fd_response_2pt(exact.density_matrix, p.H0, h1, p.nocc, h), p1)
          for h in (0.02, 0.01)]
    e4 = [exact.rel_fro(exact.fd_response_4pt(exact.density_matrix, p.H0, h1, p.nocc, h), p1)
          for h in (0.02, 0.01)]
    assert 3.0 < e2[0] / e2[1] < 5.0        # halving h divides the error by ~4
    assert 12.0 < e4[0] / e4[1] < 20.0      # ... and by ~16
    assert e4[1] < e2[1]


def test_2x2_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(5):
        a, b, d = rng.normal(size=3)
        h = np.array([[a, b], [b, d]])
        h1 = rng.normal(size=(2, 2))
        h1 = h1 + h1.T
        r = np.sqrt(((a - d) / 2) ** 2 + b * b)
        k = h - 0.5 * (a + d) * np.eye(2)
        p0 = 0.5 * (np.eye(2) - k / r)
        dk = h1 - 0.5 * np.trace(h1) * np.eye(2)
        dr = np.trace(k @ dk) / (2 * r)
        p1 = -0.5 * (dk / r - k * dr / r ** 2)
        assert np.abs(exact.density_matrix(h, 1) - p0).max() < 1e-13
        assert np.abs(exact.density_response(h, h1, 1) - p1).max() < 1e-12


def test_diagonal_h0_response():
    rng = np.random.default_rng(5)
    e = np.concatenate([rng.uniform(-5, -0.5, 5), rng.uniform(0.5, 5, 4)])
    perm = rng.permutation(9)
    e = e[perm]
    h1 = rng.normal(size=(9, 9))
    h1 = h1 + h1.T
    p1 = exact.density_response(np.diag(e), h1, 5)
    occ = e < 0
    want = np.zeros((9, 9))
    for i in range(9):
        for a in range(9):
            if occ[i] and not occ[a]:
                want[i, a] = want[a, i] = h1[i, a] / (e[i] - e[a])
    assert np.abs(p1 - want).max() < 1e-14


def test_invariants_dense():
    p = dense_gapped_problem(96, 40, 0.5, 21, h1="dense", k=1)
    p0, (p1,) = exact.solve(p.H0, p.H1, p.nocc)
    inv = exact.invariants(p.H0, p.H1[0], p0, p1, p.nocc)
    for key, val in inv.items():
        assert abs(val) < 1e-11, (key, val)


def test_factored_solution_equals_eigh():
    p = banded_gapped_problem(256, 128, 0.2, 31, block=32, h1="dense", k=2)
    p0a, p1a = exact.solve(p.H0, p.H1, p.nocc)
    p0b, p1b = exact.solve_from_factors(p.basis.e, p.basis.dense_q(), p.H1, p.nocc)
    assert exact.rel_fro(p0b, p0a) < 1e-12
    for a, b in zip(p1a, p1b):
        assert exact.rel_fro(b, a) < 1e-10


def test_brickwall_factored_solution_equals_eigh():
    p = banded_gapped_problem(512, 256, 0.2, 41, block=64, h1="dense", k=1)
    p0a, p1a = exact.solve(p.H0, p.H1, p.nocc)
    p0b, p1b = exact.solve_from_brickwall(p.basis.e, p.basis.layers, p.basis.layer_offsets(),
                                          p.basis.block, p.H1, p.nocc)
    assert exact.rel_fro(p0b, p0a) < 1e-12
    assert exact.rel_fro(p1b[0], p1a[0]) < 1e-10


def test_gershgorin_encloses_spectrum():
    p = small(n=40, seed=9)
    e1, en = exact.gershgorin(p.H0)
    ev = np.linalg.eigvalsh(p.H0)
    assert e1 <= ev[0] and ev[-1] <= en
    d = np.array([1.0, -2.0, 3.0])
    assert exact.gershgorin(np.diag(d)) == (-2.0, 3.0)


def test_degenerate_gap_raises():
    with pytest.raises(exact.DegenerateGap):
        exact.density_matrix(np.diag([-1.0, 0.0, 0.0, 1.0]), 2)
    with pytest.raises(ValueError):
        exact.density_matrix(np.eye(3), 0)


# ---- the pins reject plausible mistakes planted in a copy of the oracle ----
def _mutant_sign(e, v, h1, nocc):
    vo, vv = v[:, :nocc], v[:, nocc:]
    c = (vv.T @ h1 @ vo) / (e[nocc:, None] - e[None, :nocc])
    m = vv @ c @ vo.T
    return m + m.T


def _mutant_no_transpose(e, v, h1, nocc):
    vo, vv = v[:, :nocc], v[:, nocc:]
    c = (vv.T @ h1 @ vo) / (e[None, :nocc] - e[nocc:, None])
    return 2 * vv @ c @ vo.T


def _mutant_index(e, v, h1, nocc):
    vo, vv = v[:, :nocc], v[:, nocc:]
    c = (vv.T @ h1 @ vo) / (e[None, nocc - 1::-1] - e[nocc:, None])
    m = vv @ c @ vo.T
    return m + m.T


@pytest.mark.parametrize("mutant", [_mutant_sign, _mutant_no_transpose, _mutant_index])
def test_pins_reject_mutants(mutant):
    p = small(seed=4)
    e, v = exact.eigensystem(p.H0)
    bad = mutant(e, v, p.H1[0], p.nocc)
    fd = exact.fd_response_2pt(p0_newton, p.H0, p.H1[0], p.nocc, 1e-4)
    p0 = exact.density_matrix(p.H0, p.nocc)
    idem = np.linalg.norm(p0 @ bad + bad @ p0 - bad)
    assert exact.rel_fro(fd, bad) > 1e-3 or idem > 1e-6


def test_step_divided_differences():
    """G_ij = theta[e_i, e_j]: the divided differences of a Fermi function so
    steep that it is 0/1 to 1e-16 on the spectrum, and the Daleckii-Krein form
    V (G o V^T H1 V) V^T equals the FD-pinned response of the Newton P0."""
    p = small(seed=5)
    e, v = exact.eigensystem(p.H0)
    g = exact.step_divided_differences(e, p.nocc)
    mu = 0.5 * (e[p.nocc - 1] + e[p.nocc])
    beta = 80.0 / (e[p.nocc] - e[p.nocc - 1])
    from scipy.special import expit
    f = expit(-beta * (e - mu))          # the Fermi function, without overflow
    assert np.abs(f - (e < mu)).max() < 1e-16
    de = e[:, None] - e[None, :]
    off = ~np.eye(len(e), dtype=bool)
    dd = np.zeros_like(de)
    dd[off] = (f[:, None] - f[None, :])[off] / de[off]
    assert np.abs(g - dd).max() < 1e-14
    p1 = v @ (g * (v.T @ p.H1[0] @ v)) @ v.T
    fd = exact.fd_response_2pt(p0_newton, p.H0, p.H1[0], p.nocc, 1e-4)
    assert exact.rel_fro(p1, fd) < 1e-7
