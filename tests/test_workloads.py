"""The seeded generators produce what their recipe states."""
import numpy as np

from workloads import (banded_gapped_problem, config1, config4, dense_gapped_problem,
                       gapped_spectrum, sym_normal)


def test_spectrum_has_exact_gap():
    rng = np.random.default_rng(0)
    e = gapped_spectrum(rng, 100, 37, 0.4)
    s = np.sort(e)
    assert s[36] == -0.2 and s[37] == 0.2
    assert s[0] >= -10 and s[-1] <= 10


def test_dense_problem_symmetric_and_gapped():
    p = dense_gapped_problem(128, 64, 0.5, 9)
    assert np.array_equal(p.H0, p.H0.T)
    assert np.array_equal(p.H1[0], p.H1[0].T)
    ev = np.linalg.eigvalsh(p.H0)
    assert abs(ev[64] - ev[63] - 0.5) < 1e-12
    assert np.allclose(np.sort(ev), np.sort(p.basis.e), atol=1e-12)


def test_deterministic():
    a = config1(n=64)
    b = config1(n=64)
    assert np.array_equal(a.H0, b.H0) and np.array_equal(a.H1[0], b.H1[0])


def test_banded_problem_structure():
    p = banded_gapped_problem(512, 256, 0.2, 3, block=64)
    assert np.array_equal(p.H0, p.H0.T)
    i, j = np.nonzero(p.H0)
    assert np.abs(i - j).max() < 3 * 64
    ev = np.linalg.eigvalsh(p.H0)
    assert abs(ev[256] - ev[255] - 0.2) < 1e-11
    q = p.basis.dense_q()
    assert np.abs(q.T @ q - np.eye(512)).max() < 1e-13
    assert np.abs((q * p.basis.e) @ q.T - p.H0).max() < 1e-12


def test_sym_normal_moments():
    rng = np.random.default_rng(4)
    a = sym_normal(rng, 600, 0.01)
    assert np.array_equal(a, a.T)
    up = a[np.triu_indices(600)]
    assert abs(up.std() - 0.01) < 2e-4 and abs(up.mean()) < 2e-4


def test_batch_sizes():
    ps = config4(count=12)
    for p in ps:
        assert p.N % 16 == 0 and 64 <= p.N <= 1024 and p.nocc == p.N // 2
        assert 1 <= p.k <= 3 and 0.3 <= p.gap <= 1.0
