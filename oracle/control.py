"""Decisions of the DNN-SP2-PT scheme on FP64 scalars (Algorithms 1-3).

Readings where the pseudocode is silent or garbled (listed in the design notes):
  * sigma rule (Alg. 1): sigma_n = +1 iff |2 N_S - N_X - Nocc| > |N_X - Nocc|
    (strict), else -1; a tie picks 2x - x^2.
  * the loop runs while some first-order response has not met its test, capped
    at ``max_layers``.
  * at the layer where the D0 test fires, X_n is discarded, S^(0) keeps its
    previous value, and sigma_n = -sigma_{n-1}, as in the frozen branch.
  * the D1 test needs FroErr^(1)_{n-2}, so it starts two layers after D0
    converged; it also fires when FroErr^(1)_n is exactly zero (otherwise a
    noise-free input would never stop).
  * when the D1 test fires at layer n, S^(1)_{n-1} is the result.
  * N_S <- sigma N_X + (1 - sigma) N_S, tracked as a scalar.
  * several perturbations share one S^(0) chain; each keeps its own FroErr^(1)
    history and stop flag; a stopped response is frozen.
  * second order (the paper gives stopping tests for first order only): the
    response S^(2) of the first perturbation is updated every layer until its
    own test fires.  The test is Alg. 3 applied to FroErr^(2)_n =
    ||S^(2)_{n-1} - X^(2)_n||_F, started two layers after the D1 layer of that
    perturbation: with S^(0) and S^(1) frozen, the S^(2) map has the same
    linear part as the S^(1) map with S^(0) frozen (Eq. S_n detailed with k = 2
    minus k = 1), so the same C_pt applies.  It also fires on an exact zero;
    the result is S^(2)_{n-1}.
Constants: C_pt = 9 (Sec. IV, valid on [-0.25, 1.25]); the 4.5 factor of the
D0 test (Alg. 2, taken from earlier work) lies just above the exact-arithmetic
contraction bound IdErr_n <= 4.409 IdErr_{n-2}^2 of a sigma-flip pair
(constants.D0_PAIR_BOUND), so the test fires only once rounding noise stops
the quadratic decrease.
"""
from __future__ import annotations

C_PT = 9.0
D0_FACTOR = 4.5


class SP2PTControl:
    def __init__(self, nocc: float, n_s: float, k: int, max_layers: int = 100,
                 order2: bool = False):
        self.nocc = float(nocc)
        self.n_s = float(n_s)
        self.k = int(k)
        self.max_layers = int(max_layers)
        self.n = 0
        self.sigma: list = []          # sigma[n-1] = sigma_n
        self.iderr: list = []          # iderr[n-1] = IdErr_n (zeroth-order layers only)
        self.d0 = False
        self.d0_layer = None
        self.fro0 = None
        self.fro1 = [dict() for _ in range(self.k)]
        self.d1 = [False] * self.k
        self.d1_layer = [None] * self.k
        self.order2 = bool(order2)
        self.fro2: dict = {}
        self.d2 = False
        self.d2_layer = None

    # ---------------------------------------------------------------- layers
    def begin_layer(self) -> int:
        self.n += 1
        return self.n

    def zeroth_order(self, n_x: float, fro0) -> tuple:
        """Alg. 1 sigma rule + Alg. 2.  ``fro0`` is a callable giving
        ||S_{n-1} - X_n||_F, evaluated only when the D0 test fires.
        Returns (sigma_n, update_S0)."""
        n = self.n
        n_x = float(n_x)
        iderr = self.n_s - n_x
        a = abs(2.0 * self.n_s - n_x - self.nocc)
        b = abs(n_x - self.nocc)
        sig = 1 if a > b else -1
        self.iderr.append(iderr)
        conv = iderr <= 0.0 or (
            n > 2 and self.sigma[n - 2] != self.sigma[n - 3]
            and iderr > D0_FACTOR * self.iderr[n - 3] ** 2)
        if conv:
            self.d0 = True
            self.d0_layer = n
            self.fro0 = float(fro0())
            if n > 1:
                sig = -self.sigma[n - 2]
            self.sigma.append(sig)
            return sig, False
        self.sigma.append(sig)
        self.n_s = sig * n_x + (1 - sig) * self.n_s
        return sig, True

    def frozen_zeroth(self) -> int:
        """Alg. 1 branch after D0 converged: S^(0) kept, sigma flipped."""
        sig = -self.sigma[-1]
        self.sigma.append(sig)
        self.iderr.append(None)
        return sig

    def first_order(self, j: int, fro1) -> bool:
        """Alg. 3 for response j.  ``fro1`` is a callable giving
        ||S1_{n-1} - X1_n||_F.  Returns whether S1_j is updated this layer."""
        if self.d1[j]:
            return False
        if self.d0:
            f = float(fro1())
            self.fro1[j][self.n] = f
            prev = self.fro1[j].get(self.n - 2)
            if prev is not None and (f > C_PT * self.fro0 * prev or f == 0.0):
                self.d1[j] = True
                self.d1_layer[j] = self.n
                return False
        return True

    def second_order(self, fro2) -> bool:
        """The second-order test (design reading above) for the response of
        the first perturbation.  ``fro2`` gives ||S2_{n-1} - X2_n||_F.
        Returns whether S2 is updated this layer."""
        if self.d2:
            return False
        if self.d0:
            f = float(fro2())
            self.fro2[self.n] = f
            if self.d1[0] and self.n - 2 >= self.d1_layer[0]:
                prev = self.fro2.get(self.n - 2)
                if prev is not None and (f > C_PT * self.fro0 * prev or f == 0.0):
                    self.d2 = True
                    self.d2_layer = self.n
                    return False
        return True

    def done(self) -> bool:
        return all(self.d1) and (self.d2 or not self.order2)

    def exhausted(self) -> bool:
        return self.n >= self.max_layers

    def stats(self) -> dict:
        return {
            "layers": self.n,
            "d0_layer": self.d0_layer,
            "d1_layer": list(self.d1_layer),
            "sigma": list(self.sigma),
            "iderr": list(self.iderr),
            "fro0": self.fro0,
            "fro1": [dict(f) for f in self.fro1],
            "d2_layer": self.d2_layer,
            "fro2": dict(self.fro2),
            "converged": self.done(),
        }
