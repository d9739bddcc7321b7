"""Exact zeroth- and first-order density matrices in FP64 (test infrastructure only).

P0 is the Heaviside step of the Hamiltonian at the chemical potential
(Sec. II.B, Eq. theta): with H0 = V diag(e) V^T (LAPACK dsyevd, ascending e),
P0 = V_o V_o^T over the Nocc lowest levels.

P1 is the Gateaux derivative of P along H1 (Sec. IV, definition of D^(1)).  By
the Daleckii-Krein theorem quoted in Sec. IV, P1 = V (G o V^T H1 V) V^T with G
the divided differences of the step function: G_ia = G_ai = 1/(e_i - e_a) for i
occupied and a virtual, zero inside the occupied and the virtual blocks.  This
is the sum-over-states form
    P1 = sum_{i occ, a virt} (v_i v_a^T + v_a v_i^T) (v_a^T H1 v_i)/(e_i - e_a).

P2 is the second-order coefficient of P(H0 + lambda H1 + lambda^2 H2) (Sec. III,
the lambda^2 term of the density-matrix expansion).  The second-order
Daleckii-Krein form in the eigenbasis (tilde = V^T . V) is
    P2~_ij = sum_k theta[e_i, e_k, e_j] H1~_ik H1~_kj + theta[e_i, e_j] H2~_ij
with the second divided differences of the step: theta[o, o', a] =
-1/((e_o - e_a)(e_o' - e_a)) and theta[o, a, b] = 1/((e_o - e_a)(e_o - e_b)) for
o, o' occupied and a, b virtual, zero when all three levels share a side.
With C = D o H1~_vo, D_ao = 1/(e_o - e_a) (so P1~_vo = C), the blocks are
    P2~_oo = -C^T C,   P2~_vv = C C^T,   P2~_vo = D o (H1~_vv C - C H1~_oo + H2~_vo).
Pins (tests/test_oracle_second.py): second differences of P(H0 + h H1 + h^2 H2)
with the Newton-sign P, first differences of P1, the explicit triple sum with a
generic divided difference on small inputs, the 2x2 closed form, and the
second-order blocks of D^2 = D and HD = DH.

Pins (tests/test_oracle_exact.py): brute-force finite differences of P(H0 +
lambda H1) (Eqs. FnD_2/FnD_4) with P computed by a Newton sign iteration that
never calls eigh; the 2x2 closed form; the diagonal-H0 case; the invariants
Tr P0 = Nocc, P0^2 = P0, Tr P1 = 0, P0 P1 + P1 P0 = P1 (first-order block of
D^2 = D, Sec. III.B) and [H0, P1] + [H1, P0] = 0 (first-order block of
HD = DH).
"""
from __future__ import annotations

import numpy as np


class DegenerateGap(ValueError):
    """HOMO-LUMO gap too small: the first-order response is undefined (Sec. III.A
    restricts the theory to non-degenerate systems)."""


def gershgorin(h: np.ndarray):
    """Gershgorin spectral bounds (eps_1, eps_N) used by the normalisation layer
    (Sec. II.B; Algorithm 1 inputs)."""
    d = np.diag(h)
    r = np.abs(h).sum(axis=1) - np.abs(d)
    return float(np.min(d - r)), float(np.max(d + r))


def eigensystem(h0: np.ndarray):
    """Ascending eigenvalues and orthonormal eigenvectors (LAPACK dsyevd)."""
    e, v = np.linalg.eigh(h0)
    return e, v


def check_gap(e: np.ndarray, nocc: int, rel_tol: float = 1e-8) -> float:
    n = e.shape[0]
    if not (0 < nocc < n):
        raise ValueError("need 0 < nocc < N")
    gap = float(e[nocc] - e[nocc - 1])
    if gap <= rel_tol * max(1.0, float(e[-1] - e[0])):
        raise DegenerateGap(f"HOMO-LUMO gap {gap:.3e} too small")
    return gap


def density_matrix(h0: np.ndarray, nocc: int) -> np.ndarray:
    """P0 = theta(mu I - H0) with Tr P0 = Nocc (Eq. theta)."""
    e, v = eigensystem(h0)
    check_gap(e, nocc)
    vo = v[:, :nocc]
    return vo @ vo.T


def step_divided_differences(e: np.ndarray, nocc: int) -> np.ndarray:
    """G_ij = theta[e_i, e_j] for the step function, e ascending (Sec. IV)."""
    n = e.shape[0]
    g = np.zeros((n, n))
    ov = 1.0 / (e[:nocc, None] - e[None, nocc:])
    g[:nocc, nocc:] = ov
    g[nocc:, :nocc] = ov.T
    return g


def response_from_eigs(e: np.ndarray, v: np.ndarray, h1: np.ndarray, nocc: int) -> np.ndarray:
    """P1 from eigenpairs sorted ascending: C_ai = (V_v^T H1 V_o)_ai / (e_i - e_a),
    P1 = V_v C V_o^T + transpose."""
    vo, vv = v[:, :nocc], v[:, nocc:]
    y = vv.T @ (h1 @ vo)
    c = y / (e[None, :nocc] - e[nocc:, None])
    m = vv @ (c @ vo.T)
    return m + m.T


def density_response(h0: np.ndarray, h1: np.ndarray, nocc: int) -> np.ndarray:
    """First-order density-matrix response D^(1) along H1."""
    e, v = eigensystem(h0)
    check_gap(e, nocc)
    return response_from_eigs(e, v, h1, nocc)


def solve(h0: np.ndarray, h1s, nocc: int):
    """(P0, [P1_k]) from one eigendecomposition."""
    e, v = eigensystem(h0)
    check_gap(e, nocc)
    vo = v[:, :nocc]
    return vo @ vo.T, [response_from_eigs(e, v, h, nocc) for h in h1s]


def solve_from_factors(e: np.ndarray, q: np.ndarray, h1s, nocc: int):
    """(P0, [P1_k]) when H0 = Q diag(e) Q^T is given in factored form (the
    eigenpairs are then known; they are only reordered ascending)."""
    order = np.argsort(e, kind="stable")
    es = e[order]
    check_gap(es, nocc)
    v = q[:, order]
    vo = v[:, :nocc]
    return vo @ vo.T, [response_from_eigs(es, v, h, nocc) for h in h1s]


def second_order_from_eigs(e: np.ndarray, v: np.ndarray, h1: np.ndarray, h2, nocc: int):
    """P2 from eigenpairs sorted ascending (h2 may be None: no second-order term
    in the Hamiltonian)."""
    vo, vv = v[:, :nocc], v[:, nocc:]
    d = 1.0 / (e[None, :nocc] - e[nocc:, None])          # D_ao = 1/(e_o - e_a)
    t_vo = vv.T @ (h1 @ vo)
    t_oo = vo.T @ (h1 @ vo)
    t_vv = vv.T @ (h1 @ vv)
    c = d * t_vo
    p_oo = -(c.T @ c)
    p_vv = c @ c.T
    inner = t_vv @ c - c @ t_oo
    if h2 is not None:
        inner = inner + vv.T @ (h2 @ vo)
    p_vo = d * inner
    m = vv @ (p_vo @ vo.T)
    return vo @ (p_oo @ vo.T) + vv @ (p_vv @ vv.T) + m + m.T


def second_order_response(h0: np.ndarray, h1: np.ndarray, h2, nocc: int):
    """(P0, P1, P2) of H(lambda) = H0 + lambda H1 + lambda^2 H2."""
    e, v = eigensystem(h0)
    check_gap(e, nocc)
    vo = v[:, :nocc]
    p1 = response_from_eigs(e, v, h1, nocc)   # H2 enters at second order only
    return vo @ vo.T, p1, second_order_from_eigs(e, v, h1, h2, nocc)


def invariants2(h0, h1, h2, p0, p1, p2) -> dict:
    """Second-order blocks of D^2 = D and HD = DH, and Tr P2 (= 0: the
    occupation does not depend on lambda)."""
    h2 = np.zeros_like(h0) if h2 is None else h2
    return {
        "tr_p2": float(np.trace(p2)),
        "idem2": float(np.linalg.norm(p0 @ p2 + p1 @ p1 + p2 @ p0 - p2)),
        "comm2": float(np.linalg.norm(h0 @ p2 - p2 @ h0 + h1 @ p1 - p1 @ h1 + h2 @ p0 - p0 @ h2)),
    }


def contraction_matrix(h0: np.ndarray, h1s, nocc: int) -> np.ndarray:
    """Pi_ab = Tr(H1_a P1_b), the observable behind the polarisability tables
    of Sec. V.B (isotropic value: the mean of the diagonal).  In the eigenbasis,
    Pi_ab = 2 sum_{i occ, c virt} (H1_a~)_ci (H1_b~)_ci / (e_i - e_c): symmetric
    and negative semidefinite."""
    e, v = eigensystem(h0)
    check_gap(e, nocc)
    vo, vv = v[:, :nocc], v[:, nocc:]
    d = 1.0 / (e[None, :nocc] - e[nocc:, None])
    t = [vv.T @ (h @ vo) for h in h1s]
    k = len(h1s)
    out = np.zeros((k, k))
    for a in range(k):
        for b in range(k):
            out[a, b] = 2.0 * float(np.sum(t[a] * t[b] * d))
    return out


def cpscf_linear(h0: np.ndarray, h1: np.ndarray, nocc: int, c: float) -> np.ndarray:
    """Self-consistent first-order response for the induced field G[P1] = c P1:
    P1 = DP[H1 + c P1] (the coupled-perturbed fixed point of Sec. V.B with a
    linear response kernel).  In the eigenbasis the fixed point is
    P1~_ai = H1~_ai / (e_i - e_a - c) on the virtual-occupied block."""
    e, v = eigensystem(h0)
    check_gap(e, nocc)
    vo, vv = v[:, :nocc], v[:, nocc:]
    y = vv.T @ (h1 @ vo)
    cm = y / (e[None, :nocc] - e[nocc:, None] - c)
    m = vv @ (cm @ vo.T)
    return m + m.T


def inverse_factor(o: np.ndarray, tol: float = 1e-14, max_iter: int = 200):
    """Z with Z^T O Z = I by the recursion of Sec. II.A: X_n = Z_n^T O Z_n,
    Z_{n+1} = Z_n (1.875 I - 1.25 X_n + 0.375 X_n^2), from Z_0 = I / sqrt(b) with
    b the Gershgorin bound of O.  Returns (Z, iterations, ||Z^T O Z - I||_F)."""
    n = o.shape[0]
    _, b = gershgorin(o)
    z = np.eye(n) / np.sqrt(b)
    eye = np.eye(n)
    for it in range(max_iter + 1):
        x = z.T @ o @ z
        r = float(np.linalg.norm(x - eye))
        if r < tol or it == max_iter:
            return z, it, r
        z = z @ (1.875 * eye - 1.25 * x + 0.375 * (x @ x))
    return z, max_iter, r


def generalized_solve(h0: np.ndarray, o: np.ndarray, h1s, nocc: int):
    """(D0, [D1_k]) in a non-orthogonal basis with overlap O (Sec. II.A:
    D = Z theta(mu I - Z^T H Z) Z^T): generalised eigenpairs H0 C = O C diag(e)
    with C^T O C = I (LAPACK sygvd), D0 = C_o C_o^T and D1 = C_v M C_o^T +
    transpose with M_ai = (C_v^T H1 C_o)_ai / (e_i - e_a)."""
    import scipy.linalg
    e, c = scipy.linalg.eigh(h0, o)
    check_gap(e, nocc)
    return c[:, :nocc] @ c[:, :nocc].T, [response_from_eigs(e, c, h, nocc) for h in h1s]


def _apply_layers(m, layers, offsets, block, transpose: bool):
    """In place: M <- Q M (Q = L_last ... L_0) or M <- Q^T M, for block-diagonal
    orthogonal layers L_l = blockdiag(I_offset_l, blocks..., I_rest)."""
    seq = list(zip(layers, offsets))
    # Q M = L1 (L0 M): L0 first.  Q^T M = L0^T (L1^T M): L1^T first.
    for blocks, off in (seq[::-1] if transpose else seq):
        for r in range(blocks.shape[0]):
            rows = slice(off + r * block, off + (r + 1) * block)
            o = blocks[r].T if transpose else blocks[r]
            m[rows] = o @ m[rows]


def _congruence(m, layers, offsets, block, transpose: bool):
    """Q M Q^T (transpose=False) or Q^T M Q (transpose=True) for symmetric M."""
    a = np.array(m, copy=True)
    _apply_layers(a, layers, offsets, block, transpose)
    a = np.ascontiguousarray(a.T)
    _apply_layers(a, layers, offsets, block, transpose)
    a += a.T
    a *= 0.5
    return a


def solve_from_brickwall(e: np.ndarray, layers, offsets, block: int, h1s, nocc: int):
    """(P0, [P1_k]) for H0 = Q diag(e) Q^T with Q a product of block-diagonal
    orthogonal layers (the factors as drawn).  The same Daleckii-Krein formula
    as ``response_from_eigs``; Q and Q^T are applied layer by layer, so the
    cost is O(N^2 b) per application instead of O(N^3)."""
    n = e.shape[0]
    order = np.argsort(e, kind="stable")
    check_gap(e[order], nocc)
    occ = np.zeros(n, dtype=bool)
    occ[order[:nocc]] = True
    p0 = _congruence(np.diag(occ.astype(float)), layers, offsets, block, transpose=False)
    p1s = []
    rows = 2048
    for h1 in h1s:
        y = _congruence(h1, layers, offsets, block, transpose=True)   # V^T H1 V
        for i0 in range(0, n, rows):
            i1 = min(n, i0 + rows)
            # G_ia = G_ai = 1/(e_i - e_a), i occupied, a virtual (symmetric)
            d = e[i0:i1, None] - e[None, :]
            inv = 1.0 / np.where(d == 0, 1.0, d)
            g = np.where(occ[i0:i1, None] & ~occ[None, :], inv, 0.0)
            g -= np.where(~occ[i0:i1, None] & occ[None, :], inv, 0.0)
            y[i0:i1] *= g
        p1s.append(_congruence(y, layers, offsets, block, transpose=False))
    return p0, p1s


def invariants(h0, h1, p0, p1, nocc: int) -> dict:
    """Residuals that vanish for the exact P0, P1 (Sec. III.B block identities)."""
    return {
        "trace_p0": float(np.trace(p0) - nocc),
        "idem_p0": float(np.linalg.norm(p0 @ p0 - p0)),
        "trace_p1": float(np.trace(p1)),
        "idem_p1": float(np.linalg.norm(p0 @ p1 + p1 @ p0 - p1)),
        "comm_p0": float(np.linalg.norm(h0 @ p0 - p0 @ h0)),
        "comm_p1": float(np.linalg.norm(h0 @ p1 - p1 @ h0 + h1 @ p0 - p0 @ h1)),
    }


def fd_response_2pt(pfun, h0, h1, nocc, h):
    """Central two-point difference (Eq. FnD_2)."""
    return (pfun(h0 + h * h1, nocc) - pfun(h0 - h * h1, nocc)) / (2.0 * h)


def fd_response_4pt(pfun, h0, h1, nocc, h):
    """Four-point stencil (Eq. FnD_4)."""
    return (-pfun(h0 + 2 * h * h1, nocc) + 8 * pfun(h0 + h * h1, nocc)
            - 8 * pfun(h0 - h * h1, nocc) + pfun(h0 - 2 * h * h1, nocc)) / (12.0 * h)


def rel_fro(a: np.ndarray, ref: np.ndarray) -> float:
    """||a - ref||_F / ||ref||_F."""
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(a - ref) / den) if den > 0 else float(np.linalg.norm(a))
