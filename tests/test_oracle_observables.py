"""Pins of the contraction Pi_ab = Tr(H1_a P1_b) (the polarisability-type
observable of Sec. V.B): the band-energy identity d^2/dl^2 sum_occ e_i(H0 + l
H1) = Tr(H1 P1) checked by second differences of eigenvalues (no response
formula involved), symmetry, negative semidefiniteness, and agreement with
the trace of the oracle's P1."""
import numpy as np

from oracle import exact
from workloads import config2, dense_gapped_problem


def test_contraction_is_second_derivative_of_band_energy():
    p = dense_gapped_problem(30, 12, 0.8, 21, h1="dense", k=1, h1_std=0.05)
    pi = exact.contraction_matrix(p.H0, p.H1, p.nocc)
    h = 1e-3

    def band(lam):
        return float(np.sum(np.linalg.eigvalsh(p.H0 + lam * p.H1[0])[:p.nocc]))
    d2 = (band(h) - 2 * band(0.0) + band(-h)) / (h * h)
    assert abs(d2 - pi[0, 0]) < 1e-6 * max(1.0, abs(pi[0, 0]))


def test_contraction_matches_trace_of_response_and_is_negative_semidefinite():
    p = config2(n=48)
    pi = exact.contraction_matrix(p.H0, p.H1, p.nocc)
    _, p1s = exact.solve(p.H0, p.H1, p.nocc)
    direct = np.array([[np.trace(a @ b) for b in p1s] for a in p.H1])
    assert np.abs(pi - direct).max() < 1e-12 * np.abs(pi).max()
    assert np.abs(pi - pi.T).max() < 1e-12 * np.abs(pi).max()
    assert np.linalg.eigvalsh(pi).max() <= 1e-12 * np.abs(pi).max()


def test_mixed_second_derivative():
    """Off-diagonal entries: d^2/(dl dm) of the band energy of H0 + l A + m B."""
    p = dense_gapped_problem(24, 10, 1.0, 22, h1="dense", k=2, h1_std=0.05)
    a, b = p.H1
    pi = exact.contraction_matrix(p.H0, p.H1, p.nocc)
    h = 1e-3

    def band(x, y):
        return float(np.sum(np.linalg.eigvalsh(p.H0 + x * a + y * b)[:p.nocc]))
    d2 = (band(h, h) - band(h, -h) - band(-h, h) + band(-h, -h)) / (4 * h * h)
    assert abs(d2 - pi[0, 1]) < 1e-6 * max(1.0, abs(pi[0, 1]))
