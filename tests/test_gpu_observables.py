"""The contraction Tr(A_a B_b) on the GPU (dmpt_contract): against FP64 numpy
sums on random symmetric matrices, and end to end as Pi_ab = Tr(H1_a P1_b)
from the split-precision responses against the oracle's closed form."""
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


@pytest.mark.parametrize("n", [1, 7, 1000])
def test_contract_matches_fp64_sums(dm, n):
    from workloads import sym_normal
    rng = np.random.default_rng(n)
    As = [sym_normal(rng, n, 1.0) for _ in range(2)]
    Bs = [sym_normal(rng, n, 1.0) for _ in range(3)]
    got = dm.dmpt_contract([_cuda(a) for a in As], [_cuda(b) for b in Bs])
    ref = np.array([[np.trace(a @ b) for b in Bs] for a in As])
    assert got.shape == (2, 3)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_polarisability_contraction_end_to_end(dm):
    """Three coordinate perturbations (configuration 2 recipe at N = 768)."""
    from oracle import exact
    from workloads import config2
    p = config2(n=768)
    P0, P1s, st = dm.solve(_cuda(p.H0), [_cuda(h) for h in p.H1], p.nocc, precision="split_fp16")
    H1s = [_cuda(h) for h in p.H1]
    pi = dm.dmpt_contract(H1s, P1s)
    ref = exact.contraction_matrix(p.H0, p.H1, p.nocc)
    err = np.abs(pi - ref).max() / np.abs(ref).max()
    iso, iso_ref = np.trace(pi) / 3, np.trace(ref) / 3
    print(f"Pi (isotropic) {iso:.8f} vs oracle {iso_ref:.8f}; max rel err {err:.2e}", flush=True)
    assert err < 1e-3
    assert abs(iso - iso_ref) < 1e-4 * abs(iso_ref)


def test_contract_rejects_bad_arguments(dm):
    import torch
    buf = torch.zeros(65, dtype=torch.float64, device="cuda")
    a = buf[:64].view(8, 8)
    shifted = buf[1:65].view(8, 8)          # 8 bytes off a 16-byte boundary
    with pytest.raises(dm.DmptError) as ei:
        dm.dmpt_contract([shifted], [a])
    assert ei.value.status == -1
