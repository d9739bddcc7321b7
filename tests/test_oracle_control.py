"""Decision rules of Algorithms 1-3 on scripted FP64 scalars."""
from oracle.control import C_PT, SP2PTControl


def test_sigma_rule_and_tie():
    c = SP2PTControl(nocc=5, n_s=6.0, k=1)
    c.begin_layer()
    # N_X = 5 hits Nocc exactly: |2*6-5-5| = 2 > |5-5| = 0 -> x^2 (sigma = +1)
    sig, upd = c.zeroth_order(5.0, lambda: 0.0)
    assert (sig, upd) == (1, True) and c.n_s == 5.0
    c.begin_layer()
    # tie |2*5 - 4 - 5| = 1 == |4 - 5| = 1 -> 2x - x^2 (sigma = -1)
    sig, upd = c.zeroth_order(4.0, lambda: 0.0)
    assert sig == -1 and upd
    assert c.n_s == 2 * 5.0 - 4.0


def test_d0_fires_on_nonpositive_iderr_and_flips_sigma():
    c = SP2PTControl(nocc=2, n_s=2.5, k=1)
    c.begin_layer()
    c.zeroth_order(2.2, lambda: 1.0)        # IdErr = 0.3
    c.begin_layer()
    sig, upd = c.zeroth_order(c.n_s + 1e-17, lambda: 0.125)   # IdErr <= 0
    assert c.d0 and c.d0_layer == 2 and not upd
    assert sig == -c.sigma[0] and c.fro0 == 0.125


def test_d0_quadratic_rule_needs_alternating_sigma():
    c = SP2PTControl(nocc=10, n_s=10.5, k=1)
    seq = [(10.3, 0.2)]
    c.begin_layer()
    c.zeroth_order(10.3, lambda: 0.0)        # sigma_1: |21-10.3-10|=0.7 > 0.3 -> +1
    assert c.sigma == [1]
    c.begin_layer()
    c.zeroth_order(c.n_s - 0.05, lambda: 0.0)  # IdErr_2 = 0.05; N_X=10.25 -> |20.6-10.25-10|=.35>.25 -> +1
    assert c.sigma == [1, 1]
    c.begin_layer()
    # IdErr_3 > 4.5 IdErr_1^2 but sigma_2 == sigma_1: no stop
    c.zeroth_order(c.n_s - 0.19, lambda: 0.0)
    assert not c.d0
    del seq


def test_d0_quadratic_rule_fires():
    c = SP2PTControl(nocc=10, n_s=10.0, k=1)
    c.sigma = [1, -1]
    c.iderr = [1e-3, 5e-4]
    c.n = 2
    c.begin_layer()
    c.n_s = 10.0 + 2e-6
    # IdErr_3 = 2e-6 > 4.5 * (1e-3)^2 = 4.5e-6 ? no -> continue
    c.zeroth_order(10.0, lambda: 7.0)
    assert not c.d0
    c2 = SP2PTControl(nocc=10, n_s=10.0, k=1)
    c2.sigma = [1, -1]
    c2.iderr = [1e-3, 5e-4]
    c2.n = 2
    c2.begin_layer()
    c2.n_s = 10.0 + 5e-6
    c2.zeroth_order(10.0, lambda: 7.0)        # 5e-6 > 4.5e-6 -> converged
    assert c2.d0 and c2.fro0 == 7.0 and c2.sigma[-1] == 1
    # the factor itself is pinned by the flip-pair contraction bound
    # (tests/test_oracle_constants.py)


def _converged_control(fro0=1e-3):
    c = SP2PTControl(nocc=1, n_s=1.0, k=1)
    c.sigma = [1]
    c.iderr = [0.1]
    c.n = 1
    c.begin_layer()
    c.zeroth_order(1.0, lambda: fro0)   # IdErr = 0 -> D0 at layer 2
    return c


def test_d1_test_waits_two_layers_then_uses_cpt():
    c = _converged_control(fro0=1e-3)
    assert c.first_order(0, lambda: 1.0)          # layer 2: record only
    c.begin_layer(); c.frozen_zeroth()
    assert c.first_order(0, lambda: 0.5)          # layer 3: no n-2 value yet
    c.begin_layer(); c.frozen_zeroth()
    # layer 4: 5e-3 <= 9 * 1e-3 * 1.0 = 9e-3 -> keep going
    assert c.first_order(0, lambda: 5e-3)
    c.begin_layer(); c.frozen_zeroth()
    # layer 5: 5e-3 > 9 * 1e-3 * 0.5 = 4.5e-3 -> converged, not updated
    assert not c.first_order(0, lambda: 5e-3)
    assert c.d1 == [True] and c.d1_layer == [5] and c.done()
    assert C_PT == 9.0
    assert c.sigma[-4:] == [-1, 1, -1, 1]


def test_d1_fires_on_exact_zero():
    c = _converged_control(fro0=0.0)
    c.first_order(0, lambda: 0.0)
    c.begin_layer(); c.frozen_zeroth()
    c.first_order(0, lambda: 0.0)
    c.begin_layer(); c.frozen_zeroth()
    assert not c.first_order(0, lambda: 0.0)
    assert c.done()
