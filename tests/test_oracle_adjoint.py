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
