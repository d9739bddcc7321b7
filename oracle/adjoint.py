"""Reference gradients of L = Tr(P0 W0) + sum_k Tr(P1_k W_k) in FP64 (test
infrastructure only).

P1 = DP(H0)[H1] is the first Frechet derivative of the step function
P(H) = theta(mu I - H) (Sec. IV).  In the eigenbasis of H0 (tildes: V^T . V,
levels ascending, o = occupied, v = virtual) with D_ia = 1/(e_i - e_a):

* dL/dH1 = DP(H0)[W]: the Frechet derivative of a spectral function is
  self-adjoint, so this is the P1 formula with W in place of H1.
* dL/dH0 = D^2 P(H0)[H1, .]^* W.  With the second divided differences
  theta[a, b, c] of the step (two occupied o1, o2 and one virtual v:
  -D_o1v D_o2v; one occupied o and two virtual v1, v2: +D_ov1 D_ov2; zero
  otherwise) and A = H1~_ov o D, B = W~_ov o D:
      G~_oo = -(A B^T + B A^T)
      G~_vv =  A^T B + B^T A
      G~_ov =  D o (A W~_vv + B H1~_vv - H1~_oo B - W~_oo A)
  and G = V G~ V^T.

* the zeroth-order term adds dTr(P0 W0)/dH0 = DP(H0)[W0] (W0 symmetrised):
  the same self-adjoint first derivative, with W0 in place of H1.  It does not
  reach H1.

The gradient is the symmetric matrix G with dL = <G, dH> for symmetric dH
(an off-diagonal entry perturbed together with its mirror changes L by
2 G_ij h).  Pins: central finite differences of L computed from the exact
oracle P1 (tests/test_oracle_adjoint.py).
"""
from __future__ import annotations

import numpy as np

from .exact import check_gap, eigensystem, response_from_eigs


def loss(h0, h1s, ws, nocc, w0=None) -> float:
    """L = Tr(P0 W0) + sum_k Tr(P1_k W_k) from the exact P0 and P1 (no W0 term
    when w0 is None)."""
    e, v = eigensystem(h0)
    check_gap(e, nocc)
    val = float(sum(np.sum(response_from_eigs(e, v, h1, nocc) * w) for h1, w in zip(h1s, ws)))
    if w0 is not None:
        vo = v[:, :nocc]
        val += float(np.sum((vo @ vo.T) * w0))
    return val


def grad_h1(h0, ws, nocc):
    """[dL/dH1_k] = [DP(H0)[W_k]]."""
    e, v = eigensystem(h0)
    check_gap(e, nocc)
    return [response_from_eigs(e, v, w, nocc) for w in ws]


def grad_h0(h0, h1s, ws, nocc, w0=None):
    """dL/dH0 from the second-order divided differences of the step function,
    plus DP(H0)[W0] for the zeroth-order term when w0 is given."""
    e, v = eigensystem(h0)
    check_gap(e, nocc)
    o = slice(0, nocc)
    u = slice(nocc, None)
    d = 1.0 / (e[o, None] - e[None, u])            # D_ia, i occupied, a virtual
    g = np.zeros_like(h0)
    for h1, w in zip(h1s, ws):
        ht = v.T @ h1 @ v
        wt = v.T @ w @ v
        a = ht[o, u] * d
        b = wt[o, u] * d
        gt = np.zeros_like(h0)
        gt[o, o] = -(a @ b.T + b @ a.T)
        gt[u, u] = a.T @ b + b.T @ a
        ov = d * (a @ wt[u, u] + b @ ht[u, u] - ht[o, o] @ b - wt[o, o] @ a)
        gt[o, u] = ov
        gt[u, o] = ov.T
        g += v @ gt @ v.T
    if w0 is not None:
        g += response_from_eigs(e, v, 0.5 * (w0 + w0.T), nocc)
    return 0.5 * (g + g.T)


def fd_entry(h0, h1s, ws, nocc, i, j, which: str, h: float = 1e-5, w0=None) -> float:
    """Central difference of L for the symmetric perturbation of entry (i, j)
    (and its mirror) of H0 (which='h0') or of H1_0 (which='h1').  Returns the
    matching gradient component: dL/dh divided by 2 off the diagonal."""
    e_ij = np.zeros_like(h0)
    e_ij[i, j] = 1.0
    e_ij[j, i] = 1.0
    def lval(s):
        if which == "h0":
            return loss(h0 + s * e_ij, h1s, ws, nocc, w0)
        return loss(h0, [h1s[0] + s * e_ij] + list(h1s[1:]), ws, nocc, w0)
    dl = (lval(h) - lval(-h)) / (2.0 * h)
    return dl / (1.0 if i == j else 2.0)
