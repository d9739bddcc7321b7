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


# ------------------------------------------------------------------ the D0 factor of Alg. 2
def _pair_ratio_grid(h, x):
    """(h(x) - h(x)^2) / (x - x^2)^2 evaluated from the map itself (no simplification)."""
    y = h(x)
    return (y - y * y) / (x - x * x) ** 2


def test_flip_pair_contraction_bound_closed_form():
    x = np.linspace(0.0, 1.0, 2000001)[1:-1]
    for h, simple, arg in ((c.h_sq_then_flip, c.pair_ratio_sq_then_flip, c.D0_PAIR_ARGMAX),
                           (c.h_flip_then_sq, c.pair_ratio_flip_then_sq, 1 - c.D0_PAIR_ARGMAX)):
        r = _pair_ratio_grid(h, x)
        inner = (x > 1e-3) & (x < 1 - 1e-3)        # away from the cancellation at the ends
        assert np.allclose(r[inner], simple(x[inner]), rtol=1e-6, atol=0)
        assert abs(r.max() - c.D0_PAIR_BOUND) < 1e-9
        assert abs(x[r.argmax()] - arg) < 1e-5
    assert abs(c.D0_PAIR_BOUND - 4.409149863609382) < 1e-12


def test_d0_factor_lies_just_above_the_bound():
    from oracle.control import D0_FACTOR
    # no false stop in exact arithmetic, and the bound is tight (4.5 is not loose)
    assert c.D0_PAIR_BOUND < D0_FACTOR < 1.05 * c.D0_PAIR_BOUND


def test_bound_needs_the_sigma_flip():
    """Without the flip (a single layer, or two layers of the same branch) the
    ratio is unbounded: the quadratic contraction, and with it the factor's
    meaning, needs sigma_{n-1} != sigma_{n-2} as Alg. 2 requires."""
    x = np.linspace(0.0, 1.0, 200001)[1:-1]
    sq = lambda v: v * v                       # noqa: E731
    fl = lambda v: 2 * v - v * v               # noqa: E731
    for h in (sq, fl, lambda v: sq(sq(v)), lambda v: fl(fl(v))):
        assert _pair_ratio_grid(h, x).max() > 100 * c.D0_PAIR_BOUND


def test_contraction_on_noise_free_chains():
    """IdErr_n <= 4.409 IdErr_{n-2}^2 after every sigma flip of the eigenbasis
    chain, wherever the bound stands well above FP64 rounding; and the chain's
    D0 stop is the noise floor, not a quadratic stall: there the measured
    IdErr_n exceeds the bound only by rounding."""
    from oracle import eigsim
    from workloads import config1, dense_gapped_problem
    for p in (config1(n=128), dense_gapped_problem(96, 40, 0.3, seed=7, name="t")):
        _, _, _, st = eigsim.run(p.H0, p.H1, p.nocc)
        idr, sig = st["iderr"], st["sigma"]
        checked = 0
        for n in range(3, st["d0_layer"]):        # 1-based layers before D0
            a, b = idr[n - 1], idr[n - 3]
            if sig[n - 2] == sig[n - 3] or a is None or b is None:
                continue
            bound = c.D0_PAIR_BOUND * b * b
            if bound > 1e-8:
                assert a <= bound * (1 + 1e-9) + 1e-12, (n, a, bound)
                checked += 1
        assert checked >= 2
        assert 1 <= st["d0_layer"] - 1 <= len(idr)
        last = idr[st["d0_layer"] - 1]
        assert last <= 1e-10 * p.H0.shape[0] or last <= 0.0
