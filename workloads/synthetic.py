"""Seeded synthetic gapped Hamiltonians and perturbations.

The paper's own inputs (SCC-DFTB water boxes, Hartree-Fock water clusters;
Sec. V.A and V.B) are not available, so these generators stand in for them
with the sizes and half occupation of those workloads.  Every matrix is FP64,
row-major, exactly symmetric.

Construction (the same recipe the design notes list):

* A spectrum ``e`` with ``nocc`` occupied levels drawn U[-width, -gap/2] and
  ``N - nocc`` virtual levels drawn U[gap/2, width]; the highest occupied and
  lowest virtual levels are pinned to -gap/2 and +gap/2, so the HOMO-LUMO gap
  is exactly ``gap``.  Levels are placed in a random order.
* ``H0 = Q diag(e) Q^T`` with an orthogonal ``Q`` that is either dense Haar
  (QR of an N(0,1) matrix with diag(R) > 0) or a two-layer brick wall of
  Haar blocks (block ``b``, second layer offset by ``b/2``), which keeps H0
  banded with entries that fall off away from the diagonal.
* ``H1`` is either a dense symmetric matrix whose upper triangle and diagonal
  are i.i.d. N(0, std^2) and whose lower triangle mirrors it, or a diagonal
  matrix of U[-1, 1] "coordinates" (the form an electric-field perturbation
  takes in an orthonormal basis, Sec. V.A).

The factors (e, Q) are returned as drawn, so a checker may use them; they are
not derived from H0.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# seed = 1000 + configuration id
CONFIG_SEED = {1: 1001, 2: 1002, 3: 1003, 4: 1004, 5: 1005}


@dataclass
class Basis:
    """Construction factors of ``H0 = Q diag(e) Q^T``.

    kind == "dense":     ``Q`` is an N x N orthogonal matrix.
    kind == "brickwall": ``Q = L1 @ L0``; ``layers[0]`` holds the N/b blocks of
                         L0 (offset 0), ``layers[1]`` the N/b - 1 blocks of L1
                         (offset b/2); identity elsewhere.
    """
    e: np.ndarray
    kind: str
    Q: Optional[np.ndarray] = None
    block: int = 0
    layers: List[np.ndarray] = field(default_factory=list)

    def layer_offsets(self):
        return [0, self.block // 2][: len(self.layers)]

    def dense_q(self) -> np.ndarray:
        if self.kind == "dense":
            return self.Q
        n = self.e.shape[0]
        q = np.eye(n)
        for blocks, off in zip(self.layers, self.layer_offsets()):
            apply_blocks_left(q, blocks, off, self.block)
        return q


@dataclass
class Problem:
    name: str
    N: int
    nocc: int
    H0: np.ndarray
    H1: List[np.ndarray]
    gap: float
    basis: Basis
    seed: int
    W: Optional[np.ndarray] = None
    O: Optional[np.ndarray] = None     # overlap of a non-orthogonal basis (None: orthonormal)

    @property
    def k(self) -> int:
        return len(self.H1)


# ---------------------------------------------------------------- primitives
def haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of N(0,1) with diag(R) > 0."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def gapped_spectrum(rng: np.random.Generator, n: int, nocc: int, gap: float,
                    width: float = 10.0) -> np.ndarray:
    """Levels with exact HOMO-LUMO gap ``gap``, in random order."""
    if not (0 < nocc < n):
        raise ValueError("need 0 < nocc < n")
    occ = rng.uniform(-width, -gap / 2.0, nocc)
    vir = rng.uniform(gap / 2.0, width, n - nocc)
    occ[np.argmax(occ)] = -gap / 2.0
    vir[np.argmin(vir)] = gap / 2.0
    e = np.concatenate([occ, vir])
    return e[rng.permutation(n)]


def sym_normal(rng: np.random.Generator, n: int, std: float) -> np.ndarray:
    """Symmetric matrix: upper triangle + diagonal i.i.d. N(0, std^2), mirrored."""
    a = rng.standard_normal((n, n))
    a *= std
    blk = 1024
    for i0 in range(0, n, blk):
        i1 = min(n, i0 + blk)
        d = a[i0:i1, i0:i1]
        a[i0:i1, i0:i1] = np.triu(d) + np.triu(d, 1).T
        if i0:
            a[i0:i1, :i0] = a[:i0, i0:i1].T
    return a


def diag_coordinates(rng: np.random.Generator, n: int) -> np.ndarray:
    """Diagonal perturbation of U[-1, 1] coordinates."""
    return np.diag(rng.uniform(-1.0, 1.0, n))


def apply_blocks_left(m: np.ndarray, blocks: np.ndarray, offset: int, b: int) -> None:
    """In place: M <- L M for L = blockdiag(I_offset, blocks..., I_rest)."""
    for r in range(blocks.shape[0]):
        rows = slice(offset + r * b, offset + (r + 1) * b)
        m[rows] = blocks[r] @ m[rows]


def _symmetrize(h: np.ndarray) -> np.ndarray:
    h += h.T
    h *= 0.5
    return h


# ---------------------------------------------------------------- assemblies
def dense_gapped_problem(n: int, nocc: int, gap: float, seed: int, *, name: str = "",
                         h1: str = "dense", k: int = 1, h1_std: float = 0.01,
                         width: float = 10.0, with_w: bool = False) -> Problem:
    """H0 = Q diag(e) Q^T with dense Haar Q; ``k`` perturbations of type ``h1``."""
    rng = np.random.default_rng(seed)
    q = haar_orthogonal(rng, n)
    e = gapped_spectrum(rng, n, nocc, gap, width)
    h0 = _symmetrize((q * e[None, :]) @ q.T)
    h1s = _perturbations(rng, n, h1, k, h1_std)
    w = sym_normal(rng, n, 1.0) if with_w else None
    return Problem(name or f"dense_N{n}", n, nocc, h0, h1s, gap,
                   Basis(e=e, kind="dense", Q=q), seed, w)


def nonorth_problem(n: int, nocc: int, gap: float, seed: int, *, name: str = "", k: int = 1,
                    h1_std: float = 0.01, spread: float = 2.0, width: float = 10.0) -> Problem:
    """A non-orthogonal basis: B = Q_b diag(s) with Haar Q_b and s log-uniform in
    [1/sqrt(spread), sqrt(spread)], overlap O = B B^T (condition number up to
    spread^2), H0 = B H_perp B^T and H1 = B H1_perp B^T with (H_perp, H1_perp) the
    dense gapped recipe.  The generalised problem H0 c = e O c then has exactly
    the gapped spectrum of H_perp."""
    p = dense_gapped_problem(n, nocc, gap, seed, h1="dense", k=k, h1_std=h1_std, width=width)
    rng = np.random.default_rng(seed + 7919)
    qb = haar_orthogonal(rng, n)
    sc = np.exp(rng.uniform(-0.5, 0.5, n) * np.log(spread))
    b = qb * sc[None, :]
    o = _symmetrize(b @ b.T)
    h0 = _symmetrize(b @ p.H0 @ b.T)
    h1s = [_symmetrize(b @ h @ b.T) for h in p.H1]
    return Problem(name or f"nonorth_N{n}", n, nocc, h0, h1s, gap, p.basis, seed, None, o)


def banded_gapped_problem(n: int, nocc: int, gap: float, seed: int, *, block: int = 128,
                          name: str = "", h1: str = "dense", k: int = 1,
                          h1_std: float = 0.01, width: float = 10.0) -> Problem:
    """H0 = Q diag(e) Q^T with a two-layer brick wall Q of Haar blocks (banded H0)."""
    if n % block or block % 2:
        raise ValueError("n must be a multiple of an even block size")
    rng = np.random.default_rng(seed)
    nb = n // block
    l0 = np.stack([haar_orthogonal(rng, block) for _ in range(nb)])
    l1 = np.stack([haar_orthogonal(rng, block) for _ in range(nb - 1)])
    e = gapped_spectrum(rng, n, nocc, gap, width)
    # A = L0 diag(e) L0^T is block diagonal
    h0 = np.zeros((n, n))
    for r in range(nb):
        s = slice(r * block, (r + 1) * block)
        o = l0[r]
        h0[s, s] = (o * e[s][None, :]) @ o.T
    # H0 = L1 A L1^T
    apply_blocks_left(h0, l1, block // 2, block)
    ht = np.ascontiguousarray(h0.T)
    del h0
    apply_blocks_left(ht, l1, block // 2, block)
    h0 = _symmetrize(ht)
    h1s = _perturbations(rng, n, h1, k, h1_std)
    return Problem(name or f"banded_N{n}", n, nocc, h0, h1s, gap,
                   Basis(e=e, kind="brickwall", block=block, layers=[l0, l1]), seed)


def _perturbations(rng, n, kind, k, std):
    if kind == "dense":
        return [sym_normal(rng, n, std) for _ in range(k)]
    if kind == "diag":
        return [diag_coordinates(rng, n) for _ in range(k)]
    raise ValueError(kind)


# ---------------------------------------------------------------- named workloads
def config1(n: int = 256, nocc: Optional[int] = None, seed: int = CONFIG_SEED[1]) -> Problem:
    """N=256, Nocc=128, levels U[-10,-0.5] / U[0.5,10] (gap 1.0), one dense H1 N(0, 0.01^2)."""
    return dense_gapped_problem(n, nocc if nocc is not None else n // 2, 1.0, seed,
                                name=f"gap1.0_dense_N{n}", h1="dense", k=1)


def config2(n: int = 4096, nocc: Optional[int] = None, seed: int = CONFIG_SEED[2]) -> Problem:
    """N=4096, Nocc=2048, gap 0.5, three diagonal coordinate perturbations (x, y, z)."""
    return dense_gapped_problem(n, nocc if nocc is not None else n // 2, 0.5, seed,
                                name=f"gap0.5_xyz_N{n}", h1="diag", k=3)


def config3(n: int = 16384, nocc: Optional[int] = None, seed: int = CONFIG_SEED[3],
            block: int = 128) -> Problem:
    """N=16384, Nocc=8192, gap 0.2, banded H0, one dense H1 N(0, 0.01^2)."""
    return banded_gapped_problem(n, nocc if nocc is not None else n // 2, 0.2, seed,
                                 block=block, name=f"gap0.2_banded_N{n}", h1="dense", k=1)


def config4(count: int = 512, nmin: int = 64, nmax: int = 1024, step: int = 16,
            seed: int = CONFIG_SEED[4]) -> List[Problem]:
    """Many small problems: N uniform on {nmin, nmin+step, ..., nmax}, Nocc = N/2,
    gap U[0.3, 1.0], 1-3 diagonal perturbations each."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin // step, nmax // step + 1, count) * step
    gaps = rng.uniform(0.3, 1.0, count)
    ks = rng.integers(1, 4, count)
    seeds = rng.integers(0, 2**31 - 1, count)
    return [dense_gapped_problem(int(n), int(n) // 2, float(g), int(s),
                                 name=f"batch{i}_N{int(n)}", h1="diag", k=int(kk))
            for i, (n, g, kk, s) in enumerate(zip(sizes, gaps, ks, seeds))]


def config5(n: int = 4096, nocc: Optional[int] = None, seed: int = CONFIG_SEED[5]) -> Problem:
    """N=4096, Nocc=2048, gap 0.5, one dense H1 N(0, 0.01^2), loss weight W N(0,1) symmetric."""
    return dense_gapped_problem(n, nocc if nocc is not None else n // 2, 0.5, seed,
                                name=f"gap0.5_adjoint_N{n}", h1="dense", k=1, with_w=True)
