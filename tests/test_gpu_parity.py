"""End-to-end parity of the HIP DNN-SP2-PT path with the FP64 oracle.

Bars: the FP64 form within 1e-10 and the split / FP32 forms within 1e-3 in
relative Frobenius norm for P0 and every P1_k; the FP64 form also follows the
dense FP64 recursion's sigma sequence up to D0 convergence."""
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


def _solve(dm, p, precision, **kw):
    P0, P1s, st = dm.solve(_cuda(p.H0), [_cuda(h) for h in p.H1], p.nocc, precision=precision, **kw)
    return P0.cpu().numpy(), [q.cpu().numpy() for q in P1s], st


def _errors(p, P0, P1s):
    from oracle import exact
    r0, r1s = exact.solve(p.H0, p.H1, p.nocc)
    return exact.rel_fro(P0, r0), [exact.rel_fro(a, b) for a, b in zip(P1s, r1s)]


@pytest.fixture(scope="module")
def c1():
    from workloads import config1
    return config1()


def test_config1_fp64_parity_and_sigma(dm, c1):
    from oracle import sp2pt
    P0, P1s, st = _solve(dm, c1, "fp64")
    e0, e1 = _errors(c1, P0, P1s)
    print(f"config1 fp64: layers={st['layers']} d0={st['d0_layer']} d1={st['d1_layer']} "
          f"err P0={e0:.2e} P1={e1[0]:.2e}", flush=True)
    assert st["converged"]
    assert e0 < FP64_TOL and e1[0] < FP64_TOL
    _, _, ref = sp2pt.run(c1.H0, c1.H1, c1.nocc)
    d0 = min(ref["d0_layer"], st["d0_layer"])
    assert st["sigma"][:d0 - 1] == ref["sigma"][:d0 - 1]
    assert abs(st["d0_layer"] - ref["d0_layer"]) <= 1
    assert abs(st["trace_p0"] - c1.nocc) < 1e-9 and abs(st["trace_p1"][0]) < 1e-9


@pytest.mark.parametrize("n", [256, 300])
def test_fp64_every_layer_matches_eigenbasis_recursion(dm, n):
    """Layer by layer, the FP64 form's S_m and S1_m equal the recursion run
    in the eigenbasis of H0 (the 2x2 block-function form of Sec. IV, one layer
    at a time), which has no rounding in its traces or norms.  A context
    capped at m layers stops with ENOCONV and returns S_m and S1_m.  Every
    layer up to the earlier D1 layer is compared, the zeroth-order chain
    frozen after D0 included; the dense FP64 recursion stays within about
    2e-14 of the eigenbasis run over the same layers.  N = 300 leaves a ragged
    44-row tail on the 128-row tiles."""
    import torch
    from oracle import eigsim, exact
    from workloads import config1
    p = config1(n=n)
    _, _, v, se = eigsim.run(p.H0, p.H1, p.nocc, record=True)
    _, _, full = _solve(dm, p, "fp64")
    assert full["converged"]
    assert full["d0_layer"] == se["d0_layer"]
    d0 = se["d0_layer"]
    last = min(full["d1_layer"][0], se["d1_layer"][0]) - 1
    assert full["sigma"][:d0 - 1] == se["sigma"][:d0 - 1]
    h0, h1 = _cuda(p.H0), _cuda(p.H1[0])
    worst = [0.0, 0.0]
    for m in range(1, last + 1):
        S0 = torch.full_like(h0, float("nan"))
        S1 = torch.full_like(h0, float("nan"))
        ctx = dm.dmpt_init(h0, p.nocc, k_max=1, precision="fp64", max_layers=m)
        try:
            with pytest.raises(dm.DmptError) as ei:
                dm.dmpt_response(ctx, [h1], P0=S0, P1s=[S1])
        finally:
            dm.dmpt_destroy(ctx)
        assert ei.value.status == -4 and ei.value.stats["layers"] == m
        x, (y,) = se["history"][m - 1]
        s0e, s1e = eigsim.to_dense(x, y, v)
        e0 = exact.rel_fro(S0.cpu().numpy(), s0e)
        e1 = exact.rel_fro(S1.cpu().numpy(), s1e)
        worst = [max(worst[0], e0), max(worst[1], e1)]
        assert e0 < 1e-12 and e1 < 1e-12, (m, e0, e1)
    print(f"N={n}: layers 1..{last} (D0 at {d0}) worst S0 {worst[0]:.2e} S1 {worst[1]:.2e}",
          flush=True)


@pytest.mark.parametrize("precision", ["split_fp16", "split_bf16", "fp32"])
def test_reduced_precision_every_layer_within_the_bar(dm, precision):
    """The split and FP32 forms layer by layer against the eigenbasis
    recursion at N = 300: every S_m and S1_m before D0, while both runs take
    the same sigma, within the end-to-end bar of 1e-3.  Each form picks sigma
    (Alg. 1) and fires Alg. 2's noise-floor test on its own traces; near
    convergence the two sigma candidates differ by less than the form's
    rounding, so a reduced form may take the other branch a few layers
    before D0 (split BF16 here at layer 31 of 37), and D0 may move by one."""
    import torch
    from oracle import eigsim, exact
    from workloads import config1
    p = config1(n=300)
    _, _, v, se = eigsim.run(p.H0, p.H1, p.nocc, record=True)
    _, _, full = _solve(dm, p, precision)
    assert full["converged"]
    last = min(full["d0_layer"], se["d0_layer"]) - 1
    last = next((i for i in range(last) if full["sigma"][i] != se["sigma"][i]), last)
    assert last >= 25
    h0, h1 = _cuda(p.H0), _cuda(p.H1[0])
    worst = [0.0, 0.0]
    for m in range(1, last + 1):
        S0 = torch.full_like(h0, float("nan"))
        S1 = torch.full_like(h0, float("nan"))
        ctx = dm.dmpt_init(h0, p.nocc, k_max=1, precision=precision, max_layers=m)
        try:
            with pytest.raises(dm.DmptError) as ei:
                dm.dmpt_response(ctx, [h1], P0=S0, P1s=[S1])
        finally:
            dm.dmpt_destroy(ctx)
        assert ei.value.status == -4 and ei.value.stats["layers"] == m
        x, (y,) = se["history"][m - 1]
        s0e, s1e = eigsim.to_dense(x, y, v)
        e0 = exact.rel_fro(S0.cpu().numpy(), s0e)
        e1 = exact.rel_fro(S1.cpu().numpy(), s1e)
        worst = [max(worst[0], e0), max(worst[1], e1)]
        assert e0 < SPLIT_TOL and e1 < SPLIT_TOL, (m, e0, e1)
    print(f"{precision} N=300: layers 1..{last} worst S0 {worst[0]:.2e} S1 {worst[1]:.2e}",
          flush=True)


@pytest.mark.parametrize("precision", ["fp32", "split_fp16", "split_bf16"])
def test_config1_reduced_precision(dm, c1, precision):
    P0, P1s, st = _solve(dm, c1, precision)
    e0, e1 = _errors(c1, P0, P1s)
    print(f"config1 {precision}: layers={st['layers']} d0={st['d0_layer']} d1={st['d1_layer']} "
          f"err P0={e0:.2e} P1={e1[0]:.2e}", flush=True)
    assert st["converged"]
    assert e0 < SPLIT_TOL and e1[0] < SPLIT_TOL


@pytest.mark.parametrize("precision", ["fp64", "split_fp16", "split_bf16", "fp32"])
def test_ragged_three_diagonal_perturbations(dm, precision):
    """N = 1000 (not a tile multiple), three coordinate perturbations (config 2 shape)."""
    from workloads import config2
    p = config2(n=1000)
    P0, P1s, st = _solve(dm, p, precision)
    e0, e1 = _errors(p, P0, P1s)
    print(f"N=1000 k=3 {precision}: layers={st['layers']} d0={st['d0_layer']} "
          f"d1={st['d1_layer']} err P0={e0:.2e} P1={[f'{x:.2e}' for x in e1]}", flush=True)
    tol = FP64_TOL if precision == "fp64" else SPLIT_TOL
    assert st["converged"]
    assert e0 < tol and max(e1) < tol


def test_banded_small(dm):
    """Banded H0 (config 3 construction) at N = 768, split FP16."""
    from workloads import banded_gapped_problem
    p = banded_gapped_problem(768, 384, 0.2, 77, block=64)
    P0, P1s, st = _solve(dm, p, "split_fp16")
    e0, e1 = _errors(p, P0, P1s)
    print(f"banded N=768: layers={st['layers']} err P0={e0:.2e} P1={e1[0]:.2e}", flush=True)
    assert st["converged"] and e0 < SPLIT_TOL and e1[0] < SPLIT_TOL


def test_repeat_is_bitwise_deterministic(dm, c1):
    a = _solve(dm, c1, "split_fp16")
    b = _solve(dm, c1, "split_fp16")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1][0], b[1][0])
    assert a[2]["sigma"] == b[2]["sigma"]


def test_context_reuse_two_responses(dm):
    """One dmpt_init, two dmpt_response calls with different k."""
    from oracle import exact
    from workloads import config2
    p = config2(n=300)
    ctx = dm.dmpt_init(_cuda(p.H0), p.nocc, k_max=3, precision="split_fp16")
    try:
        _, P1a, _ = dm.dmpt_response(ctx, [_cuda(p.H1[0])])
        _, P1b, _ = dm.dmpt_response(ctx, [_cuda(h) for h in p.H1])
    finally:
        dm.dmpt_destroy(ctx)
    r0, r1s = exact.solve(p.H0, p.H1, p.nocc)
    assert exact.rel_fro(P1a[0].cpu().numpy(), r1s[0]) < SPLIT_TOL
    for a, b in zip(P1b, r1s):
        assert exact.rel_fro(a.cpu().numpy(), b) < SPLIT_TOL


# ------------------------------------------------------------------ error paths
def test_invalid_arguments(dm, c1):
    import torch
    h0 = _cuda(c1.H0)
    for nocc in (0, c1.N, -3):
        with pytest.raises(dm.DmptError) as ei:
            dm.dmpt_init(h0, nocc)
        assert ei.value.status == -1
    with pytest.raises(dm.DmptError) as ei:
        dm.dmpt_init(h0, 10, k_max=9)
    assert ei.value.status == -1
    with pytest.raises(TypeError):
        dm.dmpt_init(h0.float(), 10)
    del torch


def test_asymmetric_input_rejected(dm, c1):
    h = c1.H0.copy()
    h[3, 5] += 1e-9
    with pytest.raises(dm.DmptError) as ei:
        dm.solve(_cuda(h), [_cuda(c1.H1[0])], c1.nocc, check_symmetry=True)
    assert ei.value.status == -6


def test_nonfinite_perturbation(dm, c1):
    h1 = c1.H1[0].copy()
    h1[2, 2] = np.nan
    with pytest.raises(dm.DmptError) as ei:
        dm.solve(_cuda(c1.H0), [_cuda(h1)], c1.nocc, precision="split_fp16")
    assert ei.value.status == -5


def test_layer_cap(dm, c1):
    with pytest.raises(dm.DmptError) as ei:
        dm.solve(_cuda(c1.H0), [_cuda(c1.H1[0])], c1.nocc, precision="fp64", max_layers=5)
    assert ei.value.status == -4
    assert ei.value.stats["layers"] == 5 and not ei.value.stats["converged"]


def test_diagonal_h0_terminates(dm):
    """Noise-free FP64 input: the D1 test must still stop (exact-zero rule)."""
    from oracle import exact
    rng = np.random.default_rng(2)
    n = 130
    e = np.concatenate([rng.uniform(-3, -0.5, 60), rng.uniform(0.5, 3, 70)])
    h1 = rng.normal(size=(n, n)) * 0.01
    h1 = np.triu(h1) + np.triu(h1, 1).T
    P0, P1s, st = dm.solve(_cuda(np.diag(e)), [_cuda(h1)], 60, precision="fp64")
    assert st["converged"]
    assert exact.rel_fro(P1s[0].cpu().numpy(), exact.density_response(np.diag(e), h1, 60)) < 1e-9


@pytest.mark.parametrize("precision", ["split_fp16", "fp64"])
def test_padded_row_stride(dm, precision, monkeypatch):
    """Workspace rows longer than Np (pad columns must stay zero)."""
    from workloads import config2
    monkeypatch.setenv("DMPT_LD_PAD", "72")
    p = config2(n=520)
    P0, P1s, st = _solve(dm, p, precision)
    e0, e1 = _errors(p, P0, P1s)
    tol = FP64_TOL if precision == "fp64" else SPLIT_TOL
    assert st["converged"] and e0 < tol and max(e1) < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32", "split_fp16", "split_bf16"])
def test_reported_idempotency_residuals(dm, precision):
    """stats idem0 = ||P0 - P0^2||_F (Alg. 2, at the D0 layer) and idem1 =
    ||P1 - (P0 P1 + P1 P0)||_F (Alg. 3, at the D1 layer) as the layers formed
    them.  They equal the same residuals built from the returned P0, P1 with
    the library's layer products (the products of those layers), and they
    differ from the oracle's FP64 invariants on the returned matrices by at
    most the error of those products (triangle inequality)."""
    from oracle import exact
    from workloads import dense_gapped_problem
    p = dense_gapped_problem(300, 150, 0.5, 3001, h1="dense", k=1, h1_std=0.01)
    P0, P1s, st = _solve(dm, p, precision)
    P1 = P1s[0]
    x, x1 = dm.dmpt_layer_products(_cuda(P0), _cuda(P1), precision)
    x, x1 = x.cpu().numpy(), x1.cpu().numpy()
    lay0 = float(np.linalg.norm(P0 - x))
    lay1 = float(np.linalg.norm(P1 - x1))
    idem0, idem1 = st["idem0"], st["idem1"][0]
    print(f"{precision}: idem0 {idem0:.3e} (products {lay0:.3e}), idem1 {idem1:.3e} "
          f"(products {lay1:.3e})", flush=True)
    assert abs(idem0 - lay0) <= 1e-9 * lay0 + 1e-300
    assert abs(idem1 - lay1) <= 1e-9 * lay1 + 1e-300
    inv = exact.invariants(p.H0, p.H1[0], P0, P1, p.nocc)
    err0 = float(np.linalg.norm(x - P0 @ P0))
    err1 = float(np.linalg.norm(x1 - (P0 @ P1 + P1 @ P0)))
    assert abs(idem0 - inv["idem_p0"]) <= err0 * (1 + 1e-9) + 1e-14
    assert abs(idem1 - inv["idem_p1"]) <= err1 * (1 + 1e-9) + 1e-14


@pytest.mark.parametrize("n", [2048, 700])
def test_tile_choice_does_not_change_results(dm, n):
    """Small contexts run the fused layer on 128-row tiles, contexts that keep
    adjoint checkpoints on 256-row tiles.  Every output element takes the same
    operands, k order and MFMA sequence either way, so P0, P1 and the layer
    counts agree bitwise."""
    import torch
    from workloads import dense_gapped_problem
    p = dense_gapped_problem(n, n // 2, 0.5, 3100 + n, h1="dense", k=1)
    H0, H1 = _cuda(p.H0), _cuda(p.H1[0])
    outs = []
    for ckpt in (0, 8):
        ctx = dm.dmpt_init(H0, p.nocc, k_max=1, precision="split_bf16", ckpt_every=ckpt)
        try:
            P0, (P1,), st = dm.dmpt_response(ctx, [H1])
            torch.cuda.synchronize()
            outs.append((P0.cpu().numpy(), P1.cpu().numpy(), st["layers"], st["d0_layer"]))
        finally:
            dm.dmpt_destroy(ctx)
    (a0, a1, la, da), (b0, b1, lb, db) = outs
    assert (la, da) == (lb, db)
    assert np.array_equal(a0, b0) and np.array_equal(a1, b1)


def test_two_contexts_on_two_threads(dm):
    """Two contexts, each with its own stream and host thread, solving at the
    same time (the binding releases the interpreter during library calls):
    every result is bitwise the one the same problem gives alone, so the
    contexts share no state."""
    import threading
    import torch
    from workloads import config1, config2
    probs = [config1(n=300), config2(n=520)]
    inputs = [(_cuda(p.H0), [_cuda(h) for h in p.H1]) for p in probs]
    torch.cuda.synchronize()

    def solve_three(i, stream):
        p, (h0, h1s) = probs[i], inputs[i]
        ctx = dm.dmpt_init(h0, p.nocc, k_max=len(h1s), precision="split_fp16", stream=stream)
        try:
            res = []
            for _ in range(3):
                P0, P1s, _ = dm.dmpt_response(ctx, h1s)
                res.append((P0.cpu().numpy(), [q.cpu().numpy() for q in P1s]))
            return res
        finally:
            dm.dmpt_destroy(ctx)

    alone = [solve_three(i, None) for i in range(2)]
    out, errors = [None, None], []

    def worker(i):
        try:
            out[i] = solve_three(i, torch.cuda.Stream())
        except Exception as exc:        # reported in the main thread
            errors.append(exc)

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors, errors
    for i in range(2):
        for (a0, a1s), (b0, b1s) in zip(out[i], alone[i]):
            assert np.array_equal(a0, b0)
            assert all(np.array_equal(x, y) for x, y in zip(a1s, b1s))


@pytest.mark.parametrize("precision", ["fp64", "split_fp16"])
def test_set_hamiltonian_equals_fresh_context(dm, precision):
    """dmpt_set_hamiltonian reuses the workspace: after it, a response is
    bitwise the one of a fresh context for the new H0, and going back to the
    first H0 gives bitwise the first results again."""
    from workloads import config1
    pa, pb = config1(n=300), config1(n=300, seed=91)
    fresh = [_solve(dm, p, precision) for p in (pa, pb)]
    ctx = dm.dmpt_init(_cuda(pa.H0), pa.nocc, k_max=1, precision=precision)
    try:
        got = []
        for p in (pa, pb, pa):
            dm.dmpt_set_hamiltonian(ctx, _cuda(p.H0))
            P0, P1s, st = dm.dmpt_response(ctx, [_cuda(p.H1[0])])
            got.append((P0.cpu().numpy(), P1s[0].cpu().numpy(), st["layers"]))
    finally:
        dm.dmpt_destroy(ctx)
    for (P0, P1, layers), (F0, F1s, fst) in zip(got, [fresh[0], fresh[1], fresh[0]]):
        assert layers == fst["layers"]
        assert np.array_equal(P0, F0) and np.array_equal(P1, F1s[0])


@pytest.mark.parametrize("precision", ["fp64", "split_fp16"])
def test_outputs_may_overwrite_the_inputs(dm, c1, precision):
    """dmpt_response reads every H1 before it writes an output, and the
    context holds its own copy of H0: P0 written over the H0 tensor and P1
    over the H1 tensor give bitwise the results of separate outputs."""
    P0r, (P1r,), _ = _solve(dm, c1, precision)
    h0, h1 = _cuda(c1.H0), _cuda(c1.H1[0])
    ctx = dm.dmpt_init(h0, c1.nocc, k_max=1, precision=precision)
    try:
        dm.dmpt_response(ctx, [h1], P0=h0, P1s=[h1])
    finally:
        dm.dmpt_destroy(ctx)
    assert np.array_equal(h0.cpu().numpy(), P0r) and np.array_equal(h1.cpu().numpy(), P1r)


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
@pytest.mark.parametrize("precision", ["fp64", "split_fp16"])
def test_nonfinite_hamiltonian(dm, c1, bad, precision):
    h = c1.H0.copy()
    h[3, 3] = bad
    with pytest.raises(dm.DmptError) as ei:
        dm.solve(_cuda(h), [_cuda(c1.H1[0])], c1.nocc, precision=precision)
    assert ei.value.status == -5
