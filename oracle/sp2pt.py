"""DNN-SP2-PT (Algorithms 1-3) run densely in FP64 on the CPU (test infrastructure only).

Normalisation layer (Sec. III.A, Algorithm 1): S0 = (eps_N I - H0)/(eps_N - eps_1),
S1_0 = -H1/(eps_N - eps_1), N_S = Tr S0, with Gershgorin bounds.
Deep layer n (Eq. S_n detailed with the bias of Eq. dB):
    X_n   = S_{n-1}^2,                       S_n   = sigma_n X_n   + (1 - sigma_n) S_{n-1}
    X1_n  = S_{n-1} S1_{n-1} + S1_{n-1} S_{n-1},
    S1_n  = sigma_n X1_n + (1 - sigma_n) S1_{n-1}
with sigma_n and the stopping tests from ``control``.  With ``order2`` the
second-order response of the first perturbation follows the k = 2 case of
Eq. S_n detailed,
    X2_n  = S_{n-1} S2_{n-1} + S1_{n-1} S1_{n-1} + S2_{n-1} S_{n-1},
    S2_n  = sigma_n X2_n + (1 - sigma_n) S2_{n-1},   S2_0 = -H2/(eps_N - eps_1).
Plain numpy matmuls, no symmetry tricks, no reordering.

Pins: its converged output equals ``exact`` to the FP64 level, and its
per-layer matrices equal those of ``eigsim`` (an independent eigenbasis
computation) -- tests/test_oracle_sp2pt.py.
"""
from __future__ import annotations

import numpy as np

from .control import SP2PTControl
from .exact import gershgorin


def initial_layer(h0, h1s):
    e1, en = gershgorin(h0)
    w = en - e1
    n = h0.shape[0]
    s0 = (en * np.eye(n) - h0) / w
    s1 = [-h / w for h in h1s]
    return s0, s1, (e1, en)


def run(h0: np.ndarray, h1s, nocc: int, max_layers: int = 100, record: bool = False,
        order2: bool = False, h2=None):
    """Returns (P0, [P1_k], stats), plus stats['p2'] with ``order2``.
    ``stats['converged']`` is False when the layer cap was reached first."""
    s0, s1, bounds = initial_layer(h0, h1s)
    ctl = SP2PTControl(nocc, float(np.trace(s0)), len(s1), max_layers, order2=order2)
    s2 = None
    if order2:
        s2 = np.zeros_like(h0) if h2 is None else -h2 / (bounds[1] - bounds[0])
    hist = [] if record else None
    while not ctl.done() and not ctl.exhausted():
        ctl.begin_layer()
        x1 = [None if ctl.d1[j] else s0 @ s + s @ s0 for j, s in enumerate(s1)]
        x2 = None if (s2 is None or ctl.d2) else s0 @ s2 + s1[0] @ s1[0] + s2 @ s0
        if not ctl.d0:
            x0 = s0 @ s0
            sig, upd = ctl.zeroth_order(np.trace(x0), lambda: np.linalg.norm(s0 - x0))
            s0_prev = s0
            if upd:
                s0 = sig * x0 + (1 - sig) * s0
        else:
            sig = ctl.frozen_zeroth()
            s0_prev = s0
        for j in range(len(s1)):
            if x1[j] is None:
                continue
            if ctl.first_order(j, lambda: np.linalg.norm(s1[j] - x1[j])):
                s1[j] = sig * x1[j] + (1 - sig) * s1[j]
        if x2 is not None and ctl.second_order(lambda: np.linalg.norm(s2 - x2)):
            s2 = sig * x2 + (1 - sig) * s2
        del s0_prev
        if record:   # (S_n, [S1_n]) and, with order2, S2_n
            hist.append((s0.copy(), [s.copy() for s in s1]) + ((s2.copy(),) if order2 else ()))
    st = ctl.stats()
    st["eps1"], st["epsN"] = bounds
    if order2:
        st["p2"] = s2
    if record:
        st["history"] = hist
    return s0, s1, st
