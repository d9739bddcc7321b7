"""Pin of the self-consistent response oracle for a linear induced field
G[P1] = c P1: the closed form against the fixed-point iteration
P1 <- DP[H1 + c P1] driven by the (pinned) first-order oracle, and against
the defining equation."""
import numpy as np

from oracle import exact
from workloads import dense_gapped_problem


def test_closed_form_equals_fixed_point_iteration():
    p = dense_gapped_problem(40, 16, 1.0, 41, h1="dense", k=1, h1_std=0.05)
    c = 0.3
    ref = exact.cpscf_linear(p.H0, p.H1[0], p.nocc, c)
    p1 = exact.density_response(p.H0, p.H1[0], p.nocc)
    for _ in range(200):
        nxt = exact.density_response(p.H0, p.H1[0] + c * p1, p.nocc)
        if np.abs(nxt - p1).max() < 1e-15:
            break
        p1 = nxt
    assert np.abs(p1 - ref).max() < 1e-12 * np.abs(ref).max()
    # the defining equation
    lhs = exact.density_response(p.H0, p.H1[0] + c * ref, p.nocc)
    assert np.abs(lhs - ref).max() < 1e-12 * np.abs(ref).max()
    # c = 0 is the plain response
    assert np.abs(exact.cpscf_linear(p.H0, p.H1[0], p.nocc, 0.0)
                  - exact.density_response(p.H0, p.H1[0], p.nocc)).max() < 1e-14
