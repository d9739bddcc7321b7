"""Kernel-level parity of the HIP layer products, Gershgorin bounds and MFMA
lane layouts against plain FP64 numpy on the same seeded inputs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_2203_09621_amd as dm
    return dm


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_mfma_lane_layouts(dm):
    assert dm.dmpt_selftest_mfma() == 0


# data-sheet dense peak (TFLOP/s at 2.4 GHz) and flops per clock per SIMD
_MFMA_PEAK = {"split_fp16": (2516.6, 1024), "split_bf16": (2516.6, 1024),
              "fp32": (157.3, 64), "fp64": (78.6, 32)}


@pytest.mark.parametrize("precision", list(_MFMA_PEAK))
def test_mfma_rate_probe(dm, precision):
    """The probe's rate stays below the data-sheet dense peak and is consistent
    with its own clock reading: at most the per-clock rate of 4 SIMDs on each
    of 256 CUs."""
    peak, per_clock = _MFMA_PEAK[precision]
    tf, ghz = dm.dmpt_probe_mfma(precision)
    print(f"{precision} MFMA probe: {tf:.1f} TFLOP/s at {ghz:.3f} GHz", flush=True)
    assert 0.5 < ghz < 3.0
    assert 0.05 * peak < tf <= peak * 1.01
    assert tf <= per_clock * 4 * 256 * ghz * 1e-3 * 1.02


def test_mfma_rate_probe_rejects_unknown_precision(dm):
    from paper_2203_09621_amd import _native
    from ctypes import byref, c_double
    tf, ghz = c_double(0.0), c_double(0.0)
    assert _native.LIB.dmpt_probe_mfma(9, byref(tf), byref(ghz), None) == -1


@pytest.mark.parametrize("n", [37, 300, 1000])
def test_gershgorin_matches_numpy(dm, n):
    from oracle.exact import gershgorin
    from workloads import dense_gapped_problem
    p = dense_gapped_problem(n, n // 2, 0.5, 100 + n)
    e1, en = dm.dmpt_gershgorin(_cuda(p.H0))
    r1, rn = gershgorin(p.H0)
    assert abs(e1 - r1) <= 1e-12 * abs(r1) and abs(en - rn) <= 1e-12 * abs(rn)


def _normalised_pair(n, seed):
    """A symmetric S with spectrum in [0, 1] and a symmetric S1, as a layer sees them."""
    from workloads import dense_gapped_problem
    p = dense_gapped_problem(n, n // 2, 0.5, seed)
    ev = np.linalg.eigvalsh(p.H0)
    w = ev[-1] - ev[0]
    s = (ev[-1] * np.eye(n) - p.H0) / w
    s1 = -p.H1[0] / w
    return s, s1


TOL = {"fp64": 1e-13, "fp32": 2e-6, "split_fp16": 2e-6, "split_bf16": 5e-5}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "split_fp16", "split_bf16"])
@pytest.mark.parametrize("n", [200, 300, 600])
def test_layer_products(dm, precision, n):
    """X = S^2 and X1 = S S1 + S1 S, ragged N spanning several tiles."""
    s, s1 = _normalised_pair(n, 7 + n)
    x, x1 = dm.dmpt_layer_products(_cuda(s), _cuda(s1), precision)
    x, x1 = x.cpu().numpy(), x1.cpu().numpy()
    rx = s @ s
    rx1 = s @ s1 + s1 @ s
    ex = np.linalg.norm(x - rx) / np.linalg.norm(rx)
    ex1 = np.linalg.norm(x1 - rx1) / np.linalg.norm(rx1)
    assert ex < TOL[precision], ex
    assert ex1 < TOL[precision], ex1
    # mirrored tiles: the outputs are exactly symmetric
    assert np.array_equal(x, x.T) and np.array_equal(x1, x1.T)


def test_layer_products_deterministic(dm):
    s, s1 = _normalised_pair(520, 3)
    a = dm.dmpt_layer_products(_cuda(s), _cuda(s1), "split_fp16")
    b = dm.dmpt_layer_products(_cuda(s), _cuda(s1), "split_fp16")
    assert all(bool((u == v).all()) for u, v in zip(a, b))


@pytest.mark.parametrize("precision", ["split_fp16", "split_bf16"])
@pytest.mark.parametrize("n", [300, 1000])
def test_layer_trace_is_the_products_diagonal(dm, precision, n):
    """The split layers take N_X = Tr X before the products, from the diagonal
    fragments alone.  Each block sum must be the exactly rounded FP64 sum of
    the products' own X_ii (so every X_ii agrees bitwise; a 1-ulp difference
    in one of them changes the exact sum)."""
    import math
    s, _ = _normalised_pair(n, 11 + n)
    S = _cuda(s)
    part = dm.dmpt_layer_trace(S, precision).cpu().numpy()
    x, _ = dm.dmpt_layer_products(S, None, precision)
    d = np.diag(x.cpu().numpy())
    want = np.array([math.fsum(d[b:b + 32]) for b in range(0, n, 32)])
    assert len(part) == len(want)
    assert np.array_equal(part, want), np.abs(part - want).max()


def test_fp32_products_accumulate_in_blocks(dm):
    """The FP32 product kernel sums 64-wide k chunks from zero and adds each
    chunk to a running total (the FP32 MFMA rounds every product and every
    addition).  On an all-positive symmetric S at N = 4096 a single
    accumulator over k loses about sqrt(k) roundings at the size of the full
    sum: a CPU emulation of the MFMA's arithmetic gives relative Frobenius
    errors of X = S^2 of 3.0e-7, 4.2e-7 and 6.0e-7 at N = 512, 1024 and 2048
    (about 8e-7 here), the blocked sums 6.1e-8, 6.5e-8 and 8.0e-8."""
    rng = np.random.default_rng(41)
    n = 4096
    a = rng.random((n, n)).astype(np.float32)
    a = ((a + a.T) / 2).astype(np.float32).astype(np.float64)   # exact in FP32
    X, _ = dm.dmpt_layer_products(_cuda(a), None, precision="fp32")
    ref = a @ a
    err = np.linalg.norm(X.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"FP32 X = S^2 at N = {n}, positive S: rel err {err:.2e}", flush=True)
    assert err < 2.5e-7
