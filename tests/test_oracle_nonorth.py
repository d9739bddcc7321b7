"""Pins of the non-orthogonal-basis oracle (Sec. II.A): the paper's inverse
factor recursion against O^{-1/2} from an eigendecomposition of O; the
generalised density matrix against the Newton-sign step of the Lowdin-
transformed Hamiltonian (no generalised eigensolver) and against the
metric forms of D^2 = D: D O D = D, Tr(D O) = Nocc, D1 O D + D O D1 = D1."""
import numpy as np

from oracle import exact
from workloads import nonorth_problem

from test_oracle_exact import newton_sign


def _lowdin(o):
    w, v = np.linalg.eigh(o)
    return (v / np.sqrt(w)[None, :]) @ v.T


def test_inverse_factor_recursion_converges_to_lowdin():
    p = nonorth_problem(40, 16, 0.8, 31)
    z, it, r = exact.inverse_factor(p.O)
    assert r < 1e-13 and it < 40
    assert np.abs(z - _lowdin(p.O)).max() < 1e-12
    assert np.abs(z - z.T).max() < 1e-13


def test_generalized_density_matrix_against_newton_step():
    p = nonorth_problem(30, 12, 0.8, 32)
    d0, (d1,) = exact.generalized_solve(p.H0, p.O, p.H1, p.nocc)
    z = _lowdin(p.O)

    def d_of(h):
        return z @ (0.5 * (np.eye(p.N) - newton_sign(z @ h @ z))) @ z
    assert np.abs(d0 - d_of(p.H0)).max() < 1e-11
    h = 1e-4
    fd = (d_of(p.H0 + h * p.H1[0]) - d_of(p.H0 - h * p.H1[0])) / (2 * h)
    assert np.abs(fd - d1).max() < 1e-6 * max(1.0, np.abs(d1).max())


def test_generalized_metric_identities():
    p = nonorth_problem(36, 14, 0.5, 33, k=2)
    d0, d1s = exact.generalized_solve(p.H0, p.O, p.H1, p.nocc)
    assert np.abs(d0 @ p.O @ d0 - d0).max() < 1e-11
    assert abs(np.trace(d0 @ p.O) - p.nocc) < 1e-10
    for d1 in d1s:
        assert np.abs(d1 @ p.O @ d0 + d0 @ p.O @ d1 - d1).max() < 1e-10 * max(1.0, np.abs(d1).max())


def test_orthogonal_route_equals_generalized():
    """D = Z D_perp Z with D_perp from the (pinned) orthogonal oracle."""
    p = nonorth_problem(32, 16, 1.0, 34)
    d0, (d1,) = exact.generalized_solve(p.H0, p.O, p.H1, p.nocc)
    z, _, _ = exact.inverse_factor(p.O)
    q0, (q1,) = exact.solve(z @ p.H0 @ z, [z @ p.H1[0] @ z], p.nocc)
    assert np.abs(z @ q0 @ z - d0).max() < 1e-11
    assert np.abs(z @ q1 @ z - d1).max() < 1e-10 * max(1.0, np.abs(d1).max())
