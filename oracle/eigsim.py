"""DNN-SP2-PT run in the eigenbasis of H0 (test infrastructure only).

Every layer matrix is a function of H0 (zeroth order) or its Frechet derivative
(first order).  With H0 = V diag(e) V^T the normalised S0 = V diag(x) V^T,
x = (eps_N - e)/(eps_N - eps_1), and S^(1) = V Y V^T.  Each layer then acts as
  x^2 branch:      x -> x^2,        Y_ij -> (x_i + x_j) Y_ij
  2x - x^2 branch: x -> 2x - x^2,   Y_ij -> (2 - x_i - x_j) Y_ij
which is the 2x2 block-function (Mathias) form of Sec. IV applied one layer at
a time.  Traces and Frobenius norms are exact in this basis by unitary
invariance: Tr S = sum x, Tr X = sum x^2, ||S - X||_F = ||x - x^2||_2,
||S1 - X1||_F = ||(1 - x_i - x_j) Y_ij||_F.

Pins: per-layer parity with the dense recursion in ``sp2pt`` and converged
limits equal to ``exact`` (tests/test_oracle_sp2pt.py).
"""
from __future__ import annotations

import numpy as np

from .control import SP2PTControl
from .exact import eigensystem, gershgorin


def run(h0: np.ndarray, h1s, nocc: int, max_layers: int = 100, record: bool = False):
    """Returns (x, [Y_k], V, stats); P0 = V diag(x) V^T, P1_k = V Y_k V^T."""
    e, v = eigensystem(h0)
    e1, en = gershgorin(h0)
    w = en - e1
    x = (en - e) / w
    ys = [-(v.T @ h @ v) / w for h in h1s]
    ctl = SP2PTControl(nocc, float(np.sum(x)), len(ys), max_layers)
    hist = [] if record else None
    while not ctl.done() and not ctl.exhausted():
        ctl.begin_layer()
        pair = x[:, None] + x[None, :]
        x1 = [None if ctl.d1[j] else pair * y for j, y in enumerate(ys)]
        if not ctl.d0:
            x0 = x * x
            sig, upd = ctl.zeroth_order(np.sum(x0), lambda: np.linalg.norm(x - x0))
            if upd:
                x = sig * x0 + (1 - sig) * x
        else:
            sig = ctl.frozen_zeroth()
        for j in range(len(ys)):
            if x1[j] is None:
                continue
            if ctl.first_order(j, lambda: np.linalg.norm(ys[j] - x1[j])):
                ys[j] = sig * x1[j] + (1 - sig) * ys[j]
        if record:
            hist.append((x.copy(), [y.copy() for y in ys]))
    st = ctl.stats()
    st["eps1"], st["epsN"] = e1, en
    if record:
        st["history"] = hist
    return x, ys, v, st


def to_dense(x: np.ndarray, y: np.ndarray, v: np.ndarray):
    return (v * x[None, :]) @ v.T, v @ y @ v.T
