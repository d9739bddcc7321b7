"""The stopping-criterion constants of Sec. IV, checked on fine grids."""
import numpy as np

from oracle import constants as c


def test_cpt_is_max_ratio_on_interval():
    x = np.linspace(-0.25, 1.25, 300001)
    mask = np.abs(x - x * x) > 1e-9
    for dh in (c.dh_sq_then_flip, c.dh_flip_then_sq):
        r = np.abs(dh(x[mask])) / np.abs(x[mask] - x[mask] ** 2)
        assert abs(r.max() - c.C_PT_DEFAULT) < 1e-4


def test_derivatives_match_finite_differences():
    x = np.linspace(-0.3, 1.3, 1001)
    h = 1e-6
    for f, df in ((c.h_sq_then_flip, c.dh_sq_then_flip), (c.h_flip_then_sq, c.dh_flip_then_sq)):
        fd = (f(x + h) - f(x - h)) / (2 * h)
        assert np.abs(fd - df(x)).max() < 1e-6


def test_cpt_of_eps():
    for eps in (0.0, 1e-3, 0.1, 0.5):
        lo = (1 - np.sqrt(1 + 4 * eps)) / 2
        hi = (1 + np.sqrt(1 + 4 * eps)) / 2
        x = np.linspace(lo, hi, 200001)
        x = x[np.abs(x - x * x) > 1e-9]
        r = max((np.abs(dh(x)) / np.abs(x - x * x)).max()
                for dh in (c.dh_sq_then_flip, c.dh_flip_then_sq))
        assert abs(r - c.c_pt(eps)) < 1e-3
    assert abs(c.c_pt(0.0) - 8.0) < 1e-15


def test_inflection_points():
    x = np.linspace(0, 1, 10001)
    h = 1e-3
    for f, want in ((c.h_flip_then_sq, c.INFLECTION_FLIP_THEN_SQ),
                    (c.h_sq_then_flip, c.INFLECTION_SQ_THEN_FLIP)):
        d2 = (f(x + h) - 2 * f(x) + f(x - h)) / (h * h)
        idx = np.where(np.diff(np.sign(d2)) != 0)[0]
        assert len(idx) == 1
        assert abs(x[idx[0]] - want) < 2e-4
    assert abs(c.INFLECTION_FLIP_THEN_SQ - 0.42265) < 1e-5
    assert abs(c.INFLECTION_SQ_THEN_FLIP - 0.57735) < 1e-5
