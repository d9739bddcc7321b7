"""Host logic of the persistent product launches: the dealing plan of tile
items over workgroup slots (dmpt_plan_rounds, no GPU involved).  Position q of
a plan runs on slot q % grid; -1 is a placeholder the kernel skips."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def dm():
    import paper_2203_09621_amd as dm
    return dm


def slot_loads(order, cost, grid):
    loads = np.zeros(grid, dtype=np.int64)
    for q, i in enumerate(order):
        if i >= 0:
            loads[q % grid] += cost[i]
    return loads


def plain_loads(cost, grid):
    return slot_loads(np.arange(len(cost)), cost, grid)


def check_plan(order, cost, grid):
    """Every item once, in list order; each slot within one item of the mean."""
    items = order[order >= 0]
    assert np.array_equal(items, np.arange(len(cost)))
    assert len(order) == 0 or order[-1] >= 0                     # no trailing placeholders
    loads = slot_loads(order, cost, grid)
    bound = -(-int(cost.sum()) // grid) + int(cost.max())
    assert loads.max() <= bound
    return loads


def test_few_items_keep_the_plain_order(dm):
    cost = np.array([3, 1, 2], dtype=np.int64)
    assert np.array_equal(dm.dmpt_plan_rounds(cost, 8), np.arange(3))


@pytest.mark.parametrize("grid", [7, 64, 256])
@pytest.mark.parametrize("seed", [0, 1])
def test_random_costs(dm, grid, seed):
    rng = np.random.default_rng(seed)
    cost = rng.integers(1, 40, size=5 * grid + 3).astype(np.int64)
    check_plan(dm.dmpt_plan_rounds(cost, grid), cost, grid)


def test_layer_items_balance(dm):
    """One layer at N = 16384 with 256-row tiles: 2080 response tiles (two
    products each) then 2080 tiles of X, over 256 CUs.  Dealt in plain order
    the busiest slot carries 6.7% more than the mean; the plan cuts that to
    within one item (2.6%)."""
    T, grid = 64, 256
    n_up = T * (T + 1) // 2
    cost = np.array([2] * n_up + [1] * n_up, dtype=np.int64)
    loads = check_plan(dm.dmpt_plan_rounds(cost, grid), cost, grid)
    mean = cost.sum() / grid
    assert plain_loads(cost, grid).max() / mean > 1.06
    assert loads.max() / mean < 1.03


def test_heavy_tail_batch_costs(dm):
    """Batch-like costs (problems sorted by decreasing cost, items of one
    problem contiguous): the plan never does worse than the plain deal."""
    rng = np.random.default_rng(7)
    sizes = np.sort(rng.integers(1, 33, size=300))[::-1]
    cost = np.concatenate([np.full(s * (s + 1) // 2, 3 * s) for s in sizes]).astype(np.int64)
    grid = 512
    loads = check_plan(dm.dmpt_plan_rounds(cost, grid), cost, grid)
    assert loads.max() <= plain_loads(cost, grid).max()


def test_cap_falls_back_to_plain_order(dm):
    cost = np.array([5] + [1] * 40, dtype=np.int64)
    order = dm.dmpt_plan_rounds(cost, 4, cap=len(cost))
    assert np.array_equal(order, np.arange(len(cost)))


@pytest.mark.parametrize("args", [
    (np.array([1, 0, 2], dtype=np.int64), 2, None),     # a cost below 1
    (np.array([1, 2, 3], dtype=np.int64), 0, None),     # no slots
    (np.array([1, 2, 3], dtype=np.int64), 2, 2),        # capacity below n
])
def test_bad_arguments(dm, args):
    cost, grid, cap = args
    with pytest.raises(dm.DmptError) as ei:
        dm.dmpt_plan_rounds(cost, grid, cap=cap)
    assert ei.value.status == -1


def test_partial_slots_cover_every_response_count(dm):
    """The fused launch writes one FP64 partial per item position.  Balanced
    rounds add placeholders, so the plan's length is not monotonic in k (e.g.
    T = 10, k = 6 has more positions than k = 7); a context sized for k_max
    must hold the plan of every k <= k_max.  Grid 256 (one workgroup per CU),
    every tile count T up to 128."""
    nonmono = 0
    for T in range(1, 129):
        npos = [dm.dmpt_plan_layer(T, k, 8)[0] for k in range(1, 9)]
        nonmono += any(npos[i] > npos[i + 1] for i in range(7))
        for k_max in range(1, 9):
            cap = dm.dmpt_plan_layer(T, 1, k_max)[1]
            assert max(npos[:k_max]) <= cap, (T, k_max, npos[:k_max], cap)
    assert nonmono > 0        # the case the capacity must cover does occur


def test_plan_layer_matches_plan_rounds(dm):
    """dmpt_plan_layer counts the positions of dmpt_plan_rounds over the fused
    item costs: k response outputs of T (T + 1) / 2 tiles at cost 2, then X at
    cost 1."""
    for T, k in ((10, 6), (17, 2), (64, 1), (33, 3)):
        tiles = T * (T + 1) // 2
        cost = np.array([2] * (k * tiles) + [1] * tiles, dtype=np.int64)
        order = dm.dmpt_plan_rounds(cost, 256, cap=2 * len(cost))
        assert dm.dmpt_plan_layer(T, k, k)[0] == len(order)
