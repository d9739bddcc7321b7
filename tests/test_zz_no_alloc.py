"""dmpt_contract_noalloc (the contraction with its partial sums in the
library's fixed device scratch) against dmpt_contract, the entry point it
varies, and against FP64 numpy sums: two calls in a row, the second smaller,
so that a stale scratch or a wrong offset shows; the pair limit is refused on
the host."""
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


def _case(seed, n, na, nb):
    from workloads import sym_normal
    rng = np.random.default_rng(seed)
    As = [sym_normal(rng, n, 1.0) for _ in range(na)]
    Bs = [sym_normal(rng, n, 1.0) for _ in range(nb)]
    ref = np.array([[np.sum(a * b) for b in Bs] for a in As])
    return As, Bs, ref


def test_noalloc_matches_contract_two_calls(dm):
    # first call: 32 pairs at N = 1000; second: 6 pairs at N = 77, then the
    # 64-pair limit at N = 33
    for seed, n, na, nb in ((7, 1000, 4, 8), (8, 77, 2, 3), (9, 33, 8, 8)):
        print(f"contract_noalloc seed={seed} N={n} na={na} nb={nb}", flush=True)
        As, Bs, ref = _case(seed, n, na, nb)
        dA, dB = [_cuda(a) for a in As], [_cuda(b) for b in Bs]
        got = dm.dmpt_contract_noalloc(dA, dB)
        base = dm.dmpt_contract(dA, dB)
        assert got.shape == (na, nb)
        assert np.array_equal(got, base), np.abs(got - base).max()
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_noalloc_refuses_more_pairs_than_the_scratch_holds(dm):
    import torch
    a = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(dm.DmptError) as ei:
        dm.dmpt_contract_noalloc([a] * 5, [a] * 13)     # 65 pairs
    assert ei.value.status == -1
    assert "64" in str(ei.value)
