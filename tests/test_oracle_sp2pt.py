"""Pins of the dense FP64 SP2-PT recursion and of the eigenbasis simulator:
each against the exact limit, and against each other layer by layer."""
import numpy as np
import pytest

from oracle import eigsim, exact, sp2pt
from workloads import config1, config2, dense_gapped_problem


@pytest.fixture(scope="module")
def c1_small():
    return config1(n=64)


def test_dense_recursion_converges_to_exact(c1_small):
    p = c1_small
    p0, (p1,), st = sp2pt.run(p.H0, p.H1, p.nocc)
    r0, (r1,) = exact.solve(p.H0, p.H1, p.nocc)
    assert st["converged"]
    assert exact.rel_fro(p0, r0) < 1e-12
    assert exact.rel_fro(p1, r1) < 1e-9
    # a few layers of first-order tail after D0 converged (Sec. IV: about 3-4)
    assert 2 <= st["d1_layer"][0] - st["d0_layer"] <= 5


def test_eigsim_converges_to_exact(c1_small):
    p = c1_small
    x, (y,), v, st = eigsim.run(p.H0, p.H1, p.nocc)
    p0, p1 = eigsim.to_dense(x, y, v)
    r0, (r1,) = exact.solve(p.H0, p.H1, p.nocc)
    assert st["converged"]
    assert exact.rel_fro(p0, r0) < 1e-12
    assert exact.rel_fro(p1, r1) < 1e-9


def test_per_layer_parity_dense_vs_eigenbasis(c1_small):
    p = c1_small
    _, _, sd = sp2pt.run(p.H0, p.H1, p.nocc, record=True)
    _, _, v, se = eigsim.run(p.H0, p.H1, p.nocc, record=True)
    d0 = sd["d0_layer"]
    assert sd["sigma"][:d0 - 1] == se["sigma"][:d0 - 1]
    for n in range(min(d0 - 1, len(se["history"]))):
        s0d, (s1d,) = sd["history"][n]
        x, (y,) = se["history"][n]
        s0e, s1e = eigsim.to_dense(x, y, v)
        assert np.abs(s0d - s0e).max() < 1e-11, n
        assert np.abs(s1d - s1e).max() < 1e-11 * max(1.0, np.abs(s1e).max() * 1e3), n


def test_three_diagonal_perturbations():
    p = config2(n=64)
    p0, p1s, st = sp2pt.run(p.H0, p.H1, p.nocc)
    r0, r1s = exact.solve(p.H0, p.H1, p.nocc)
    assert st["converged"] and len(p1s) == 3
    for a, b in zip(p1s, r1s):
        assert exact.rel_fro(a, b) < 1e-9


def test_noise_free_diagonal_input_terminates():
    rng = np.random.default_rng(2)
    e = np.concatenate([rng.uniform(-3, -0.5, 6), rng.uniform(0.5, 3, 6)])
    h1 = rng.normal(size=(12, 12)) * 0.01
    h1 = h1 + h1.T
    p0, (p1,), st = sp2pt.run(np.diag(e), [h1], 6)
    assert st["converged"]
    assert exact.rel_fro(p1, exact.density_response(np.diag(e), h1, 6)) < 1e-9


def test_layer_cap_reports_no_convergence(c1_small):
    p = c1_small
    _, _, st = sp2pt.run(p.H0, p.H1, p.nocc, max_layers=5)
    assert not st["converged"] and st["layers"] == 5


def test_gershgorin_normalisation_spectrum_in_unit_interval():
    p = dense_gapped_problem(48, 20, 0.5, 3)
    s0, _, (e1, en) = sp2pt.initial_layer(p.H0, p.H1)
    ev = np.linalg.eigvalsh(s0)
    assert ev.min() >= -1e-14 and ev.max() <= 1 + 1e-14
    # reverse order: the lowest level of H0 maps closest to 1
    e = np.linalg.eigvalsh(p.H0)
    assert abs(ev.max() - (en - e[0]) / (en - e1)) < 1e-13
