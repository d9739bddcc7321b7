"""Non-orthogonal bases on the GPU: the inverse factor recursion and the
congruences (dmpt_inverse_factor, dmpt_congruence) against the FP64 oracle,
and the response in a non-orthogonal basis against the generalised
eigenproblem."""
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


@pytest.fixture(scope="module")
def prob():
    from workloads import nonorth_problem
    return nonorth_problem(300, 120, 0.8, 1201)


def test_inverse_factor_fp64(dm, prob):
    from oracle import exact
    Z, it, err = dm.dmpt_inverse_factor(_cuda(prob.O), precision="fp64", tol=1e-12)
    z_ref, it_ref, _ = exact.inverse_factor(prob.O, tol=1e-12)
    Zh = Z.cpu().numpy()
    print(f"inverse factor fp64: {it} updates (oracle {it_ref}), residual {err:.2e}", flush=True)
    assert err < 1e-12 and abs(it - it_ref) <= 1
    assert np.abs(Zh - z_ref).max() < 1e-10 * np.abs(z_ref).max()
    assert np.array_equal(Zh, Zh.T)


def test_inverse_factor_every_iterate_fp64(dm, prob):
    """Each iterate Z_m of the Sec. II.A recursion (a call capped at m updates
    stops with ENOCONV and returns Z_m and the residual of Z_m) equals the
    oracle's iterate within 1e-12, relative to its largest entry."""
    import torch
    from oracle import exact
    _, it_total, _ = exact.inverse_factor(prob.O, tol=1e-12)
    assert it_total >= 5
    O = _cuda(prob.O)
    worst = 0.0
    for m in range(1, it_total):
        Zt = torch.full_like(O, float("nan"))
        with pytest.raises(dm.DmptError) as ei:
            dm.dmpt_inverse_factor(O, precision="fp64", max_iter=m, tol=1e-300, Z=Zt)
        assert ei.value.status == -4 and ei.value.stats["iters"] == m
        z_ref, it_ref, r_ref = exact.inverse_factor(prob.O, tol=0.0, max_iter=m)
        assert it_ref == m
        d = float(np.abs(Zt.cpu().numpy() - z_ref).max() / np.abs(z_ref).max())
        worst = max(worst, d)
        assert d < 1e-12, (m, d)
        assert abs(ei.value.stats["err"] - r_ref) <= 1e-9 * max(r_ref, 1e-3), (m, r_ref)
    print(f"inverse factor fp64: iterates 1..{it_total - 1} within {worst:.2e}", flush=True)


def test_inverse_factor_fp32(dm, prob):
    Z, it, err = dm.dmpt_inverse_factor(_cuda(prob.O), precision="fp32", tol=1e-4)
    Zh = Z.cpu().numpy()
    r = np.linalg.norm(Zh @ prob.O @ Zh - np.eye(prob.N))
    print(f"inverse factor fp32: {it} updates, residual {err:.2e} (FP64 check {r:.2e})", flush=True)
    assert err < 1e-4 and r < 1e-3


def test_congruence_fp64(dm, prob):
    from workloads import sym_normal
    rng = np.random.default_rng(5)
    z = sym_normal(rng, prob.N, 1.0)
    a = sym_normal(rng, prob.N, 1.0)
    out = dm.dmpt_congruence(_cuda(z), _cuda(a), precision="fp64").cpu().numpy()
    ref = z @ a @ z
    assert np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.array_equal(out, out.T)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("split_fp16", 1e-3)])
def test_response_in_nonorthogonal_basis(dm, prob, precision, tol):
    from oracle import exact
    P0, P1s, st = dm.solve_nonorth(_cuda(prob.H0), _cuda(prob.O), [_cuda(h) for h in prob.H1],
                                   prob.nocc, precision=precision)
    r0, r1s = exact.generalized_solve(prob.H0, prob.O, prob.H1, prob.nocc)
    e0 = exact.rel_fro(P0.cpu().numpy(), r0)
    e1 = exact.rel_fro(P1s[0].cpu().numpy(), r1s[0])
    print(f"non-orthogonal {precision}: layers {st['layers']} errors P0 {e0:.2e} P1 {e1:.2e}",
          flush=True)
    assert st["converged"] and e0 < tol and e1 < tol


def test_indefinite_overlap_is_reported(dm):
    import torch
    o = -torch.eye(64, dtype=torch.float64, device="cuda")
    with pytest.raises(dm.DmptError) as ei:
        dm.dmpt_inverse_factor(o)
    assert ei.value.status == -5
