"""Second-order response (dmpt_response2) against the FP64 oracle: the closed
form P2 (second-order Daleckii-Krein) and the dense FP64 recursion with the
same stopping tests.  Bars as for first order: 1e-10 for the FP64 form, 1e-3
relative Frobenius for the split and FP32 forms."""
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


def _problem(n, seed, gap=1.0, with_h2=True):
    from workloads import dense_gapped_problem, sym_normal
    p = dense_gapped_problem(n, n // 2, gap, seed, h1="dense", k=1, h1_std=0.01)
    h2 = sym_normal(np.random.default_rng(seed + 7), n, 0.01) if with_h2 else None
    return p, h2


def _run(dm, p, h2, precision):
    ctx = dm.dmpt_init(_cuda(p.H0), p.nocc, k_max=2, precision=precision)
    try:
        P0, P1, P2, st = dm.dmpt_response2(ctx, _cuda(p.H1[0]),
                                           None if h2 is None else _cuda(h2))
        return P0.cpu().numpy(), P1.cpu().numpy(), P2.cpu().numpy(), st
    finally:
        dm.dmpt_destroy(ctx)


def _errors(p, h2, P0, P1, P2):
    from oracle import exact
    r0, r1, r2 = exact.second_order_response(p.H0, p.H1[0], h2, p.nocc)
    return exact.rel_fro(P0, r0), exact.rel_fro(P1, r1), exact.rel_fro(P2, r2)


@pytest.mark.parametrize("with_h2", [False, True])
def test_fp64_second_order_parity_and_layers(dm, with_h2):
    from oracle import sp2pt
    p, h2 = _problem(256, 1001, with_h2=with_h2)
    P0, P1, P2, st = _run(dm, p, h2, "fp64")
    e = _errors(p, h2, P0, P1, P2)
    print(f"fp64 second order (H2 {'on' if with_h2 else 'off'}): layers {st['layers']} "
          f"d0 {st['d0_layer']} d1/d2 {st['d1_layer']} errors {e}", flush=True)
    assert st["converged"]
    assert max(e) < FP64_TOL
    _, _, ref = sp2pt.run(p.H0, p.H1, p.nocc, order2=True, h2=h2)
    # the tests follow the dense FP64 recursion (readings of Alg. 2-3); the
    # D0 layer may move by one with the rounding of the traces
    assert abs(st["d0_layer"] - ref["d0_layer"]) <= 1
    assert st["d1_layer"][0] - st["d0_layer"] == ref["d1_layer"][0] - ref["d0_layer"]
    assert st["d1_layer"][1] - st["d1_layer"][0] == ref["d2_layer"] - ref["d1_layer"][0]
    assert abs(st["trace_p1"][1]) < 1e-9


def test_fp64_second_order_every_layer(dm):
    """Layer by layer, the FP64 form's S_m, S1_m and S2_m (three-product X2
    items) equal the dense FP64 recursion of Sec. III with k = 2 within 1e-12:
    a context capped at m layers stops with ENOCONV and returns them.  Layers
    up to the first D test that the two runs do not pass together."""
    import torch
    from oracle import exact, sp2pt
    p, h2 = _problem(256, 1001, with_h2=True)
    _, _, ref = sp2pt.run(p.H0, p.H1, p.nocc, order2=True, h2=h2, record=True)
    _, _, _, full = _run(dm, p, h2, "fp64")
    assert full["converged"]
    last = min(full["d0_layer"], ref["d0_layer"]) - 1
    if full["d0_layer"] == ref["d0_layer"]:
        last = min(full["d1_layer"][0], ref["d1_layer"][0]) - 1
    assert last >= 20
    assert full["sigma"][:last] == ref["sigma"][:last]
    h0, h1, hh2 = _cuda(p.H0), _cuda(p.H1[0]), _cuda(h2)
    worst = [0.0, 0.0, 0.0]
    for m in range(1, last + 1):
        outs = [torch.full_like(h0, float("nan")) for _ in range(3)]
        ctx = dm.dmpt_init(h0, p.nocc, k_max=2, precision="fp64", max_layers=m)
        try:
            with pytest.raises(dm.DmptError) as ei:
                dm.dmpt_response2(ctx, h1, hh2, P0=outs[0], P1=outs[1], P2=outs[2])
        finally:
            dm.dmpt_destroy(ctx)
        assert ei.value.status == -4 and ei.value.stats["layers"] == m
        s0, (s1,), s2 = ref["history"][m - 1]
        errs = [exact.rel_fro(o.cpu().numpy(), r) for o, r in zip(outs, (s0, s1, s2))]
        worst = [max(w, e) for w, e in zip(worst, errs)]
        assert max(errs) < 1e-12, (m, errs)
    print(f"second order fp64: layers 1..{last} worst S {worst[0]:.2e} S1 {worst[1]:.2e} "
          f"S2 {worst[2]:.2e}", flush=True)


@pytest.mark.parametrize("precision", ["fp32", "split_fp16", "split_bf16"])
def test_reduced_precision_second_order(dm, precision):
    p, h2 = _problem(256, 1001)
    P0, P1, P2, st = _run(dm, p, h2, precision)
    e = _errors(p, h2, P0, P1, P2)
    print(f"{precision} second order: layers {st['layers']} d1/d2 {st['d1_layer']} "
          f"errors {e}", flush=True)
    assert st["converged"]
    assert max(e) < SPLIT_TOL
    assert st["d1_layer"][1] >= st["d1_layer"][0] + 2


def test_ragged_second_order_split(dm):
    """N = 1000: several tiles and a ragged edge, gap 0.5."""
    p, h2 = _problem(1000, 1003, gap=0.5)
    P0, P1, P2, st = _run(dm, p, h2, "split_fp16")
    e = _errors(p, h2, P0, P1, P2)
    print(f"N=1000 split_fp16 second order: layers {st['layers']} errors {e}", flush=True)
    assert st["converged"] and max(e) < SPLIT_TOL


def test_second_order_matches_first_order_response(dm):
    """P0 and P1 of dmpt_response2 equal those of dmpt_response (same kernels,
    same decisions up to the D1 layer)."""
    p, h2 = _problem(512, 1005)
    ctx = dm.dmpt_init(_cuda(p.H0), p.nocc, k_max=2, precision="split_fp16")
    try:
        A0, (A1,), sa = dm.dmpt_response(ctx, [_cuda(p.H1[0])])
        B0, B1, _, sb = dm.dmpt_response2(ctx, _cuda(p.H1[0]), _cuda(h2))
    finally:
        dm.dmpt_destroy(ctx)
    assert sa["d1_layer"][0] == sb["d1_layer"][0]
    assert np.array_equal(A0.cpu().numpy(), B0.cpu().numpy())
    assert np.array_equal(A1.cpu().numpy(), B1.cpu().numpy())


def test_second_order_needs_two_slots(dm):
    p, _ = _problem(128, 1007)
    ctx = dm.dmpt_init(_cuda(p.H0), p.nocc, k_max=1, precision="split_fp16")
    try:
        with pytest.raises(dm.DmptError) as ei:
            dm.dmpt_response2(ctx, _cuda(p.H1[0]))
        assert ei.value.status == -1
    finally:
        dm.dmpt_destroy(ctx)


def test_adjoint_refuses_after_second_order(dm):
    p, h2 = _problem(128, 1009)
    ctx = dm.dmpt_init(_cuda(p.H0), p.nocc, k_max=2, precision="fp32", ckpt_every=4)
    try:
        dm.dmpt_response2(ctx, _cuda(p.H1[0]), _cuda(h2))
        with pytest.raises(dm.DmptError) as ei:
            dm.dmpt_adjoint(ctx, [_cuda(h2)])
        assert ei.value.status == -1
    finally:
        dm.dmpt_destroy(ctx)
