"""Pins of the reference gradients of L = Tr(P1 W): central finite differences
of L computed from the exact oracle P1, on random entries of H0 and H1."""
import numpy as np
import pytest

from oracle import adjoint, exact
from workloads import dense_gapped_problem, sym_normal


@pytest.fixture(scope="module")
def prob():
    p = dense_gapped_problem(40, 17, 0.6, 5, h1="dense", k=1, h1_std=0.05)
    w = sym_normal(np.random.default_rng(9), 40, 1.0)
    return p, w


def test_grad_h1_matches_fd(prob):
    p, w = prob
    g = adjoint.grad_h1(p.H0, [w], p.nocc)[0]
    rng = np.random.default_rng(1)
    for _ in range(6):
        i, j = sorted(rng.integers(0, p.N, 2))
        fd = adjoint.fd_entry(p.H0, p.H1, [w], p.nocc, i, j, "h1", h=1e-4)
        assert abs(fd - g[i, j]) <= 1e-6 * max(1.0, abs(g).max())


def test_grad_h0_matches_fd(prob):
    p, w = prob
    g = adjoint.grad_h0(p.H0, p.H1, [w], p.nocc)
    rng = np.random.default_rng(2)
    for _ in range(8):
        i, j = sorted(rng.integers(0, p.N, 2))
        fd = adjoint.fd_entry(p.H0, p.H1, [w], p.nocc, i, j, "h0", h=1e-5)
        assert abs(fd - g[i, j]) <= 1e-5 * max(1.0, abs(g).max()), (i, j, fd, g[i, j])
    d = 3
    fd = adjoint.fd_entry(p.H0, p.H1, [w], p.nocc, d, d, "h0", h=1e-5)
    assert abs(fd - g[d, d]) <= 1e-5 * max(1.0, abs(g).max())


def test_grad_h0_directional(prob):
    """<G, E> equals the derivative of L along a random symmetric direction E."""
    p, w = prob
    g = adjoint.grad_h0(p.H0, p.H1, [w], p.nocc)
    e = sym_normal(np.random.default_rng(3), p.N, 1.0)
    h = 1e-5
    dl = (adjoint.loss(p.H0 + h * e, p.H1, [w], p.nocc)
          - adjoint.loss(p.H0 - h * e, p.H1, [w], p.nocc)) / (2 * h)
    assert abs(np.sum(g * e) - dl) <= 1e-6 * max(1.0, abs(dl))


def test_grad_h1_is_self_adjoint_response(prob):
    """<DP[W], H1> = <DP[H1], W> (symmetry of the Frechet derivative)."""
    p, w = prob
    g = adjoint.grad_h1(p.H0, [w], p.nocc)[0]
    p1 = exact.density_response(p.H0, p.H1[0], p.nocc)
    assert abs(np.sum(g * p.H1[0]) - np.sum(p1 * w)) < 1e-12 * max(1.0, abs(np.sum(p1 * w)))


def test_mutant_wrong_sign_rejected(prob):
    p, w = prob
    g = adjoint.grad_h0(p.H0, p.H1, [w], p.nocc)
    e = sym_normal(np.random.default_rng(4), p.N, 1.0)
    h = 1e-5
    dl = (adjoint.loss(p.H0 + h * e, p.H1, [w], p.nocc)
          - adjoint.loss(p.H0 - h * e, p.H1, [w], p.nocc)) / (2 * h)
    # dropping the off-diagonal block, or flipping the occupied block, fails the check
    v = np.linalg.eigh(p.H0)[1]
    gt = v.T @ g @ v
    bad = gt.copy()
    bad[:p.nocc, :p.nocc] *= -1
    assert abs(np.sum((v @ bad @ v.T) * e) - dl) > 1e-4 * max(1.0, abs(dl))
    bad = gt.copy()
    bad[:p.nocc, p.nocc:] = 0
    bad[p.nocc:, :p.nocc] = 0
    assert abs(np.sum((v @ bad @ v.T) * e) - dl) > 1e-4 * max(1.0, abs(dl))


def _p0_newton(h):
    """theta(-H) by Newton's sign iteration (no eigensolver); the generators
    centre the gap on zero."""
    x = h.copy()
    for _ in range(100):
        xn = 0.5 * (x + np.linalg.inv(x))
        if np.linalg.norm(xn - x) <= 1e-15 * np.linalg.norm(xn):
            break
        x = xn
    return 0.5 * (np.eye(h.shape[0]) - xn)


def test_grad_h0_of_p0_term_matches_fd_of_newton_p0(prob):
    """d Tr(P0 W0)/dH0 = DP(H0)[W0]: central differences of Tr(P0 W0) with P0
    from the Newton sign iteration, along random entries and a direction."""
    p, w = prob
    w0 = sym_normal(np.random.default_rng(11), p.N, 1.0)
    g = adjoint.grad_h0(p.H0, [], [], p.nocc, w0=w0)
    h = 1e-5
    rng = np.random.default_rng(12)
    for _ in range(6):
        i, j = sorted(rng.integers(0, p.N, 2))
        e = np.zeros((p.N, p.N))
        e[i, j] = e[j, i] = 1.0
        fd = (np.sum(_p0_newton(p.H0 + h * e) * w0)
              - np.sum(_p0_newton(p.H0 - h * e) * w0)) / (2 * h) / (1.0 if i == j else 2.0)
        assert abs(fd - g[i, j]) <= 1e-6 * max(1.0, abs(g).max()), (i, j, fd, g[i, j])


def test_combined_loss_gradient(prob):
    """L = Tr(P0 W0) + Tr(P1 W): the two terms add, and H1 sees only the second."""
    p, w = prob
    w0 = sym_normal(np.random.default_rng(13), p.N, 1.0)
    g = adjoint.grad_h0(p.H0, p.H1, [w], p.nocc, w0=w0)
    e = sym_normal(np.random.default_rng(14), p.N, 1.0)
    h = 1e-5
    dl = (adjoint.loss(p.H0 + h * e, p.H1, [w], p.nocc, w0)
          - adjoint.loss(p.H0 - h * e, p.H1, [w], p.nocc, w0)) / (2 * h)
    assert abs(np.sum(g * e) - dl) <= 1e-6 * max(1.0, abs(dl))
    # a mutant that drops the zeroth-order term fails the same check
    g_bad = adjoint.grad_h0(p.H0, p.H1, [w], p.nocc)
    assert abs(np.sum(g_bad * e) - dl) > 1e-4 * max(1.0, abs(dl))
    fd1 = adjoint.fd_entry(p.H0, p.H1, [w], p.nocc, 2, 5, "h1", h=1e-4, w0=w0)
    assert abs(fd1 - adjoint.grad_h1(p.H0, [w], p.nocc)[0][2, 5]) <= 1e-6 * max(1.0, abs(fd1))
