"""Edge cases and full-size parity of the HIP path against the FP64 oracle:
the smallest problem (N = 2, the 2x2 closed form), extreme occupations, a zero
perturbation, the maximum number of responses, empty inputs (refused), a
narrow gap, scale and shift invariances, and configurations 2 and 3 at their
full sizes (N = 4096 with three coordinate perturbations; N = 16384
banded against the exact factored oracle)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SPLIT_TOL = 1e-3
FP64_TOL = 1e-10


@pytest.fixture(scope="module")
def dm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_2203_09621_amd as dm
    return dm


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _solve(dm, h0, h1s, nocc, precision, **kw):
    P0, P1s, st = dm.solve(_cuda(h0), [_cuda(h) for h in h1s], nocc, precision=precision, **kw)
    return P0.cpu().numpy(), [q.cpu().numpy() for q in P1s], st


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("split_fp16", SPLIT_TOL),
                                           ("split_bf16", SPLIT_TOL)])
def test_two_by_two(dm, precision, tol):
    """H = [[-1, l b], [l b, 1]]: P0 = diag(1, 0), P1 = -(b/2) offdiag."""
    b = 0.3
    h0 = np.diag([-1.0, 1.0])
    h1 = np.array([[0.0, b], [b, 0.0]])
    P0, (P1,), st = _solve(dm, h0, [h1], 1, precision)
    assert st["converged"]
    assert np.abs(P0 - np.diag([1.0, 0.0])).max() < tol
    assert np.abs(P1 - np.array([[0.0, -b / 2], [-b / 2, 0.0]])).max() < tol * b


@pytest.mark.parametrize("nocc", [1, 199])
def test_extreme_occupations(dm, nocc):
    from oracle import exact
    from workloads import dense_gapped_problem
    p = dense_gapped_problem(200, nocc, 1.0, 1401 + nocc, h1="dense", k=1)
    P0, (P1,), st = _solve(dm, p.H0, p.H1, nocc, "split_fp16")
    r0, (r1,) = exact.solve(p.H0, p.H1, nocc)
    e0, e1 = exact.rel_fro(P0, r0), exact.rel_fro(P1, r1)
    print(f"Nocc={nocc}: layers {st['layers']} errors {e0:.2e} {e1:.2e}", flush=True)
    assert st["converged"] and e0 < SPLIT_TOL and e1 < SPLIT_TOL
    assert abs(st["trace_p0"] - nocc) < 1e-3 * nocc


@pytest.mark.parametrize("precision", ["fp64", "split_fp16"])
def test_zero_perturbation(dm, precision):
    """H1 = 0: P1 = 0 exactly, and the D1 test fires on FroErr = 0 (reading 5)."""
    from workloads import config1
    c1 = config1()
    P0, (P1,), st = _solve(dm, c1.H0, [np.zeros_like(c1.H0)], c1.nocc, precision)
    assert st["converged"]
    assert np.abs(P1).max() == 0.0
    assert st["d1_layer"][0] == st["d0_layer"] + 2


def test_maximum_number_of_responses(dm):
    from oracle import exact
    from workloads import dense_gapped_problem
    p = dense_gapped_problem(384, 192, 0.8, 1411, h1="dense", k=8)
    P0, P1s, st = _solve(dm, p.H0, p.H1, p.nocc, "split_fp16")
    r0, r1s = exact.solve(p.H0, p.H1, p.nocc)
    errs = [exact.rel_fro(a, b) for a, b in zip(P1s, r1s)]
    print(f"k=8: layers {st['layers']} d1 {st['d1_layer']} worst P1 error {max(errs):.2e}",
          flush=True)
    assert st["converged"] and len(P1s) == 8 and max(errs) < SPLIT_TOL


def test_full_size_configuration2(dm):
    """N = 4096, Nocc = 2048, gap 0.5, three coordinate perturbations, in every
    form: FP64 within 1e-10, the split forms and the FP32 form within 1e-3.
    The gap is 8e-4 of the Gershgorin width here, so early product errors in
    the occupied-virtual block are amplified; the FP32 form reaches 3.5e-5
    with its blocked accumulation (1.1e-3 with one accumulator over k)."""
    from oracle import exact
    from workloads import config2
    p = config2()
    r0, r1s = exact.solve(p.H0, p.H1, p.nocc)
    for precision, tol in (("fp64", FP64_TOL), ("fp32", SPLIT_TOL), ("split_fp16", SPLIT_TOL),
                           ("split_bf16", SPLIT_TOL)):
        P0, P1s, st = _solve(dm, p.H0, p.H1, p.nocc, precision)
        e = [exact.rel_fro(P0, r0)] + [exact.rel_fro(a, b) for a, b in zip(P1s, r1s)]
        print(f"configuration 2 {precision}: layers {st['layers']} errors {e}", flush=True)
        assert st["converged"] and max(e) < tol


def test_full_size_configuration3(dm):
    """N = 16384 banded, gap 0.2, split FP16, against the exact factored oracle."""
    from oracle import exact
    from workloads import config3
    p = config3()
    P0, (P1,), st = _solve(dm, p.H0, p.H1, p.nocc, "split_fp16")
    r0, (r1,) = exact.solve_from_brickwall(p.basis.e, p.basis.layers, p.basis.layer_offsets(),
                                           p.basis.block, p.H1, p.nocc)
    e0, e1 = exact.rel_fro(P0, r0), exact.rel_fro(P1, r1)
    print(f"configuration 3: layers {st['layers']} errors P0 {e0:.2e} P1 {e1:.2e}", flush=True)
    assert st["converged"] and e0 < SPLIT_TOL and e1 < SPLIT_TOL
    assert abs(st["trace_p0"] - p.nocc) < 1e-2


def test_empty_inputs_are_refused(dm):
    """Empty inputs return EINVAL before any device work: a 0 x 0 Hamiltonian,
    overlap, contraction operand or layer-product input, a batch of no
    problems, a batch holding an empty problem, and a contraction over no
    matrices."""
    import torch
    from ctypes import c_double, c_void_p
    from paper_2203_09621_amd import _native
    e = torch.empty((0, 0), dtype=torch.float64, device="cuda")
    a = _cuda(np.eye(4))
    calls = [
        lambda: dm.dmpt_init(e, 0),
        lambda: dm.dmpt_inverse_factor(e),
        lambda: dm.dmpt_contract([e], [e]),
        lambda: dm.dmpt_contract_noalloc([e], [e]),
        lambda: dm.dmpt_batch_init([], [], []),
        lambda: dm.dmpt_batch_init([0, 64], [0, 32], [1, 1]),
    ]
    for call in calls:
        with pytest.raises(dm.DmptError) as ei:
            call()
        assert ei.value.status == -1
    out = (c_double * 1)()
    one = (c_void_p * 1)(a.data_ptr())
    none = (c_void_p * 1)()
    for fn in (_native.LIB.dmpt_contract, _native.LIB.dmpt_contract_noalloc):
        assert fn(none, 0, one, 1, 4, out, None) == -1
        assert fn(one, 1, none, 0, 4, out, None) == -1
        assert fn(one, 1, one, 1, 0, out, None) == -1
    eps = (c_double * 2)()
    assert _native.LIB.dmpt_gershgorin(c_void_p(a.data_ptr()), 0, eps, None) == -1


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("split_fp16", SPLIT_TOL),
                                           ("fp32", SPLIT_TOL)])
def test_narrow_gap(dm, precision, tol):
    """A gap of 0.003 in a spectrum of width 10 (relative to the Gershgorin
    width: 1.3e-5) at N = 512: about 65 layers, and the forms with 22 or more
    operand bits stay within their bars (split BF16 does not at this gap:
    its 16 bits give P1 to about 8e-3)."""
    from oracle import exact
    from workloads import dense_gapped_problem
    p = dense_gapped_problem(512, 256, 0.003, 777, h1="dense", k=1)
    P0, (P1,), st = _solve(dm, p.H0, p.H1, p.nocc, precision)
    r0, (r1,) = exact.solve(p.H0, p.H1, p.nocc)
    e0, e1 = exact.rel_fro(P0, r0), exact.rel_fro(P1, r1)
    print(f"narrow gap {precision}: layers {st['layers']} err P0 {e0:.1e} P1 {e1:.1e}", flush=True)
    assert st["converged"] and st["layers"] >= 60
    assert e0 < tol and e1 < tol


@pytest.mark.parametrize("precision", ["split_fp16", "split_bf16"])
def test_perturbation_scale_is_carried_exactly(dm, precision):
    """P1 is linear in H1 and the split forms carry S1's magnitude in a
    power-of-two scale, so H1 scaled by 2^20 or 2^-27 gives P1 scaled by the
    same power of two, bitwise, with no overflow of the 16-bit splits."""
    from workloads import config1
    p = config1(n=300)
    _, (base,), st = _solve(dm, p.H0, p.H1, p.nocc, precision)
    for e in (20, -27):
        f = 2.0 ** e
        _, (P1,), s = _solve(dm, p.H0, [p.H1[0] * f], p.nocc, precision)
        assert s["layers"] == st["layers"] and s["d1_layer"] == st["d1_layer"]
        assert np.array_equal(P1, base * f), e


@pytest.mark.parametrize("precision", ["fp64", "split_fp16"])
def test_hamiltonian_scale_and_shift(dm, precision):
    """The normalisation layer (Sec. III.A) maps H0 and H1 scaled together by
    a power of two to the same S0 and S1 bitwise, so P0 and P1 are bitwise
    unchanged; a shift H0 + c I moves both Gershgorin bounds by c and leaves
    P0 and P1 unchanged up to the rounding of the shifted bounds."""
    from workloads import config1
    p = config1(n=300)
    P0, (P1,), st = _solve(dm, p.H0, p.H1, p.nocc, precision)
    f = 2.0 ** -9
    Q0, (Q1,), s = _solve(dm, p.H0 * f, [p.H1[0] * f], p.nocc, precision)
    assert s["layers"] == st["layers"]
    assert np.array_equal(Q0, P0) and np.array_equal(Q1, P1)
    tol = 1e-12 if precision == "fp64" else SPLIT_TOL
    R0, (R1,), _ = _solve(dm, p.H0 + 3.0 * np.eye(p.N), p.H1, p.nocc, precision)
    assert np.linalg.norm(R0 - P0) < tol * np.linalg.norm(P0)
    assert np.linalg.norm(R1 - P1) < tol * np.linalg.norm(P1)
