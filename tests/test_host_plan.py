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


# ---------------------------------------------------------------------------
# Host model of the index arithmetic of the fused split product launch
# (256 x 256 tiles, 32-wide k-tiles, 2 x 2 waves, two LDS stages): every
# workgroup of the persistent grid, every item it takes, and every address
# the kernel forms, checked against the buffers the context allocates.  The
# formulas restate the kernel's, so a change on one side that the other does
# not follow shows here before it reaches a GPU.
BM, BK, WGM, WGN, SWZ = 256, 32, 2, 2, 2
NT = WGM * WGN * 64
CH = BK // 8                      # 16-byte chunks per row of a k-tile
ROWS = 4 * BM                     # A_hi | A_lo | B_hi | B_lo
STAGE = ROWS * CH                 # chunks per stage
RPW, RPL = 64 // CH, NT // CH
LOADS = ROWS // RPL
PANEL_ROWS, PANEL_K = 256, 32
WTM, WTN = BM // WGM, BM // WGN
FM, FN = WTM // 32, WTN // 32
LDS_CHUNKS = 2 * STAGE            # dynamic LDS of the launch, in 16-byte chunks


def xcd_remap(b, g):
    q, r = divmod(g, 8)
    x, i = b % 8, b // 8
    return x * (q + 1) + i if x < r else r * (q + 1) + (x - r) * q + i


def layer_items(T, k):
    """(out, ti, tj) of one fused layer: responses 1..k, then X; bands of 8
    tile rows, each walked column by column over the upper triangle."""
    v = []
    for out in list(range(1, k + 1)) + [0]:
        for g0 in range(0, T, 8):
            g1 = min(T, g0 + 8)
            for tj in range(g0, T):
                for ti in range(g0, min(g1, tj + 1)):
                    v.append((out, ti, tj))
    return v


def _load_model():
    """Item-independent parts of the global->LDS loads: per (round i, thread)
    the element offset inside a 256 x 32 panel block and the LDS chunk the
    lane writes; and the chunk each lane reads for (row R, chunk c)."""
    tid = np.arange(NT)
    lane, wave = tid % 64, tid // 64
    lrow, lsl = tid // CH, tid % CH
    csrc = lsl ^ ((lrow >> SWZ) & (CH - 1))
    voff = lrow * PANEL_K + csrc * 8
    local, dst, rows, chunks = [], [], [], []
    for i in range(LOADS):
        arr = (i * RPL) // BM
        local.append((arr, (i * RPL - arr * BM) * PANEL_K + voff))
        d = (i * RPL + wave * RPW) * CH + lane
        dst.append(d)
        # the chunk that lands in slot d: row i RPL + lrow, chunk csrc
        rows.append(i * RPL + lrow)
        chunks.append(csrc)
    return local, np.concatenate(dst), np.concatenate(rows), np.concatenate(chunks)


def test_load_and_read_addressing_is_a_consistent_permutation():
    local, dst, rows, chunks = _load_model()
    # one stage: every 16-byte slot written exactly once per k-tile
    assert dst.min() == 0 and dst.max() == STAGE - 1 and len(np.unique(dst)) == STAGE
    # slot d holds (row, chunk); the reader of (R, c) looks in slot R CH + (c ^ swz(R))
    held = {int(d): (int(r), int(c)) for d, r, c in zip(dst, rows, chunks)}
    for R in range(ROWS):
        for c in range(CH):
            slot = R * CH + (c ^ ((R >> SWZ) & (CH - 1)))
            assert held[slot] == (R, c)
    # panel-block offsets of one round stay inside one 256 x 32 block
    for arr, off in local:
        assert 0 <= arr < 4
        assert off.min() >= 0 and off.max() + 8 <= PANEL_ROWS * PANEL_K
    # fragment reads: lane rows of a wave's A or B fragment, hi or lo
    lane = np.arange(64)
    for wm in range(WGM):
        for wn in range(WGN):
            for g in range(2 * (FM + FN)):
                a_side = g < 2 * FM
                idx = g % FM if a_side else (g - 2 * FM) % FN
                lo = (g >= FM) if a_side else (g >= 2 * FM + FN)
                R = (wm * WTM + idx * 32 if a_side else 2 * BM + wn * WTN + idx * 32) + lane % 32
                for kk in range(2):
                    c = kk * 2 + lane // 32
                    q = (R + (BM if lo else 0)) * CH + (c ^ ((R >> SWZ) & (CH - 1)))
                    assert q.min() >= 0 and q.max() < STAGE


def test_epilogue_staging_and_stores_in_bounds():
    SR, PT = 32 * WGM, BM + 4
    ITER = SR * BM // (4 * NT)
    # parked fragments
    lane = np.arange(64)
    for wm in range(WGM):
        for wn in range(WGN):
            for r in range(16):
                row = wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)
                col = wn * WTN + (FN - 1) * 32 + lane % 32
                assert row.max() < SR and (row * PT + col).max() < LDS_CHUNKS * 4
    tid = np.arange(NT)
    for m in range(FM):
        lrs = []
        for g in range(ITER):
            e = (tid + g * NT) * 4
            tr, lc = e // BM, e % BM
            lr = (tr >> 5) * WTM + m * 32 + (tr & 31)
            assert tr.max() < SR and (tr * PT + lc + 3).max() < LDS_CHUNKS * 4
            assert lr.max() < BM and lc.max() + 3 < BM and np.all(lc % 4 == 0)
            lrs.append(lr * BM + lc)
        # the direct block of round m covers rows m*32 + {0..31} of both wave rows, once
        cov = np.concatenate(lrs)
        assert len(np.unique(cov)) == len(cov) == SR * BM // 4
        e = np.arange(BM * (SR // 4))
        qd, lc = e % (SR // 4), e // (SR // 4)
        tr = 4 * qd
        lr = (tr >> 5) * WTM + m * 32 + (tr & 31)
        assert (tr + 3).max() < SR and np.all(lr % 4 == 0) and lr.max() + 3 < BM


@pytest.mark.parametrize("N,k,k_max", [(256, 1, 1), (300, 2, 3), (2560, 6, 7), (4608, 2, 3),
                                       (4096, 3, 3), (16384, 1, 1), (16384, 1, 8)])
def test_persistent_loop_model(dm, N, k, k_max):
    """Every workgroup of the launch the context makes for N, k (k_max slots):
    the slot remap is a bijection, the workgroups together take every item
    position once, each real item is a valid upper-triangle tile of an
    existing output, its partial slot lies inside the context's capacity, and
    every operand fetch and epilogue store lies inside its buffer."""
    Np = -(-N // BM) * BM
    T, ld = Np // BM, Np + 128
    items = layer_items(T, k)
    cost = np.array([1 if o == 0 else 2 for o, _, _ in items], dtype=np.int64)
    order = dm.dmpt_plan_rounds(cost, 256, cap=2 * len(cost))
    n_pos, cap = dm.dmpt_plan_layer(T, k, k_max)
    assert len(order) == n_pos <= cap
    grid = min(n_pos, 256)
    slots = [xcd_remap(b, grid) for b in range(grid)]
    assert sorted(slots) == list(range(grid))
    taken = np.zeros(n_pos, dtype=np.int64)
    for s in slots:
        taken[s::grid] += 1
    assert np.all(taken == 1)
    # real items: every tile of every output once, in the list's order
    real = order[order >= 0]
    assert np.array_equal(real, np.arange(len(items)))
    kblocks = Np // PANEL_K                   # panel blocks per row panel (pdim)
    kt_per = -(-N // PANEL_K)                 # k-tiles of one product (kdim = N rounded to 32)
    assert kt_per <= kblocks
    local, _, _, _ = _load_model()
    max_local = max(int(off.max()) for _, off in local) + 8
    for pos, idx in enumerate(order):
        assert pos < cap                      # part_f / part_m slot (slot_base 0)
        if idx < 0:
            continue
        out, ti, tj = items[idx]
        assert 0 <= out <= k and 0 <= ti <= tj < T
        nprod = 1 if out == 0 else 2
        for t in (0, nprod * kt_per - 1):
            p = int(t >= kt_per) + int(t >= 2 * kt_per)
            assert p < nprod
            kofs = (t - p * kt_per) * PANEL_ROWS * PANEL_K
            for row0 in (ti * BM, tj * BM):
                off = (row0 // PANEL_ROWS) * kblocks * PANEL_ROWS * PANEL_K + \
                      (row0 % PANEL_ROWS) * PANEL_K
                assert off + kofs >= 0 and off + kofs + max_local <= Np * Np
        # epilogue: last row/column of the tile and its mirror
        for grow, gcol in ((ti * BM + BM - 1, tj * BM + BM - 4), (tj * BM + BM - 1, ti * BM + BM - 4)):
            assert grow * ld + gcol + 4 <= Np * ld
            pi = ((grow // PANEL_ROWS) * (Np // PANEL_K) + gcol // PANEL_K) * PANEL_ROWS * PANEL_K \
                + (grow % PANEL_ROWS) * PANEL_K + gcol % PANEL_K
            assert gcol % PANEL_K + 4 <= PANEL_K and pi + 4 <= Np * Np


@pytest.mark.parametrize("N,k,k_max", [(300, 1, 1), (2048, 1, 1), (4096, 2, 2), (3000, 3, 3),
                                       (4096, 1, 8)])
def test_persistent_loop_model_128(dm, N, k, k_max):
    """The same walk for the 128-row fused launch that small single-problem
    contexts use: 2 x 2 waves of 64 x 64, 32 KB stages, two
    workgroups per CU (grid 512), tiles of 128 rows inside the 256-row panel
    blocks, the k loop over N rounded up to 32, partial slots sized for the
    128-row tiling."""
    bm, grid = 128, 512
    nt, ch = 256, 4
    rows = 4 * bm
    stage = rows * ch
    rpl = nt // ch
    loads = rows // rpl
    Np = -(-N // 256) * 256
    T, ld = -(-N // bm), Np + 128
    items = layer_items(T, k)
    cost = np.array([1 if o == 0 else 2 for o, _, _ in items], dtype=np.int64)
    order = dm.dmpt_plan_rounds(cost, grid, cap=2 * len(cost))
    n_pos, cap = dm.dmpt_plan_layer(T, k, k_max, grid)
    assert len(order) == n_pos <= cap
    g = min(n_pos, grid)
    slots = [xcd_remap(b, g) for b in range(g)]
    assert sorted(slots) == list(range(g))
    real = order[order >= 0]
    assert np.array_equal(real, np.arange(len(items)))
    kblocks, kt = Np // 32, -(-N // 32)
    tid = np.arange(nt)
    lane, wave = tid % 64, tid // 64
    lrow, lsl = tid // ch, tid % ch
    csrc = lsl ^ ((lrow >> 2) & (ch - 1))
    voff = lrow * 32 + csrc * 8
    for i in range(loads):
        arr = (i * rpl) // bm
        assert arr < 4
        dst = (i * rpl + wave * (64 // ch)) * ch + lane
        assert dst.max() < stage
        local = (i * rpl - arr * bm) * 32 + voff
        assert local.max() + 8 <= 256 * 32          # inside one panel block
    for idx in real:
        out, ti, tj = items[idx]
        for row0 in (ti * bm, tj * bm):
            off = (row0 // 256) * kblocks * 8192 + (row0 % 256) * 32
            assert off + (kt - 1) * 8192 + (bm - 1) * 32 + 32 <= Np * Np
        assert tj * bm + bm <= Np and (tj * bm + bm - 1) * ld + tj * bm + bm <= Np * ld
    # epilogue staging of the 128-row tile inside the launch's 2 x 32 KB
    sr, pt = 64, bm + 4
    assert sr * pt * 4 <= 2 * stage * 16


# ---------------------------------------------------------------------------
# Host model of the batch's pair launch (k_products_pair): items of two
# 128 x 128 tiles that share a row band (ti2 == ti: the A panels) or a column
# band (tj2 == tj: the B panels), 2 x 4 waves of 64 x 64, six load arrays of
# 128 rows (X_hi, X_lo: the shared panel; Y0_hi, Y0_lo, Y1_hi, Y1_lo: each
# tile's other panel) per 48 KB stage, three stages (k-tile t in stage t % 3),
# one workgroup per CU.
P_BM, P_NT, P_CH, P_NARR, P_STAGES = 128, 512, 4, 6, 3
P_STAGE = P_NARR * P_BM * P_CH                 # chunks per stage
P_RPW, P_RPL = 64 // P_CH, P_NT // P_CH
P_WGM, P_WGN, P_WT = 2, 4, 64


def pair_items(T, k):
    """(out, ti, tj, ti2, tj2) as the batch builds them: responses, then X;
    per row band the tiles from the diagonal two by two, the odd last ones
    (all in column band T - 1) two by two, a last odd one alone."""
    v = []
    for out in list(range(1, k + 1)) + [0]:
        rest = []
        for ti in range(T):
            tj = ti
            while tj + 1 < T:
                v.append((out, ti, tj, ti, tj + 1))
                tj += 2
            if tj < T:
                rest.append(ti)
        for i in range(0, len(rest), 2):
            if i + 1 < len(rest):
                v.append((out, rest[i], T - 1, rest[i + 1], T - 1))
            else:
                v.append((out, rest[i], T - 1, -1, -1))
    return v


@pytest.mark.parametrize("T", [1, 2, 3, 4, 5, 7, 8, 9])
def test_pair_items_cover_every_tile_once(T):
    for k in (1, 3):
        seen = {}
        alone = 0
        for out, ti, tj, ti2, tj2 in pair_items(T, k):
            assert 0 <= ti <= tj < T
            if ti2 < 0:
                assert tj2 < 0
                alone += 1
            else:
                assert ti2 <= tj2 < T and (ti2 == ti) != (tj2 == tj)   # one shared band
            for t in ((ti, tj), (ti2, tj2)):
                if t[0] >= 0:
                    seen[(out,) + t] = seen.get((out,) + t, 0) + 1
        want = {(o, i, j) for o in range(k + 1) for i in range(T) for j in range(i, T)}
        assert set(seen) == want and all(n == 1 for n in seen.values())
        assert alone <= k + 1                           # at most one lone tile per output


def _pair_reads(colp):
    """LDS slot each lane reads for every (wave, fragment, k step)."""
    out = []
    for wm in range(P_WGM):
        for wn in range(P_WGN):
            half = wn >> 1
            row_a = (2 + 2 * half) * P_BM if colp else 0
            row_b = 0 if colp else (2 + 2 * half) * P_BM
            for g in range(8):
                a_side = g < 4
                idx = g % 2 if a_side else (g - 4) % 2
                lo = (g >= 2) if a_side else (g >= 6)
                rin = (wm * P_WT if a_side else (wn & 1) * P_WT) + idx * 32 + np.arange(64) % 32
                R = (row_a if a_side else row_b) + (P_BM if lo else 0) + rin
                want_arr = ((1 if lo else 0) if a_side != colp else 2 + 2 * half + (1 if lo else 0))
                assert np.all(R // P_BM == want_arr) and np.all(R % P_BM == rin)
                for kk in range(2):
                    c = kk * 2 + np.arange(64) // 32
                    slot = R * P_CH + (c ^ ((rin >> 2) & (P_CH - 1)))
                    out.append((R, c, slot))
    return out


def test_pair_launch_lds_layout():
    # LDS: three stages plus the kernel's static partial arrays within one CU
    assert P_STAGES * P_STAGE * 16 + 8 * 8 + 8 * 4 <= 160 * 1024
    tid = np.arange(P_NT)
    lane, wave = tid % 64, tid // 64
    lrow, lsl = tid // P_CH, tid % P_CH
    csrc = lsl ^ ((lrow >> 2) & (P_CH - 1))
    voff = lrow * 32 + csrc * 8
    assert voff.min() >= 0 and voff.max() + 8 <= 256 * 32 and lrow.max() < P_BM
    held = {}
    for i in range(P_NARR):
        dst = (i * P_RPL + wave * P_RPW) * P_CH + lane
        for d, r, c in zip(dst, i * P_RPL + lrow, csrc):
            assert int(d) not in held
            held[int(d)] = (int(r), int(c))
    assert sorted(held) == list(range(P_STAGE))
    # fragment reads, row pairs (A shared) and column pairs (B shared): the
    # slot a lane reads holds the row and chunk it wants
    for colp in (False, True):
        for R, c, slot in _pair_reads(colp):
            assert slot.max() < P_STAGE
            for s_, r_, c_ in zip(slot, R, c):
                assert held[int(s_)] == (int(r_), int(c_))
    # epilogue staging: 64 rows of 256 + 4 floats inside the three stages
    SR, PT, BN = 64, 260, 256
    assert SR * PT * 4 <= P_STAGES * P_STAGE * 16
    ITER = SR * BN // (4 * P_NT)
    for m in range(2):
        cov = []
        for g in range(ITER):
            e = (tid + g * P_NT) * 4
            tr, lc = e // BN, e % BN
            assert np.array_equal(lc, (tid * 4) % BN)        # a thread keeps its column
            lr = (tr >> 5) * P_WT + m * 32 + (tr & 31)
            assert tr.max() < SR and lr.max() < P_BM and lc.max() + 3 < BN
            cov.append(lr * BN + lc)
        cov = np.concatenate(cov)
        assert len(np.unique(cov)) == len(cov) == SR * BN // 4
        e = np.arange(BN * (SR // 4))
        qd, lc = e % (SR // 4), e // (SR // 4)
        lr = ((4 * qd) >> 5) * P_WT + m * 32 + ((4 * qd) & 31)
        assert lc.max() < BN and np.all(lr % 4 == 0) and lr.max() + 3 < P_BM


@pytest.mark.parametrize("N,k", [(2, 1), (37, 1), (100, 2), (129, 3), (300, 2), (513, 1),
                                 (1024, 3)])
def test_pair_launch_fetches_and_stores_in_bounds(N, k):
    """Per item: the six panel-block offsets of the first and last k-tile of
    each product, and the epilogue's extreme master and panel addresses of
    both tiles and their mirrors, inside the problem's buffers (panel layout
    padded to 256, masters of row stride Np, k loop over N rounded to 32)."""
    Np = -(-N // 256) * 256
    T, ld = -(-N // P_BM), Np
    kblocks, kt_per = Np // 32, -(-N // 32)
    assert kt_per <= kblocks and T * P_BM <= Np
    blk = 256 * 32
    for out, ti, tj, ti2, tj2 in pair_items(T, k):
        nprod = 1 if out == 0 else 2
        colp = ti2 >= 0 and ti2 != ti
        x = tj if colp else ti
        y0 = ti if colp else tj
        y1 = tj if ti2 < 0 else (ti2 if colp else tj2)
        for t in (0, nprod * kt_per - 1):
            p = int(t >= kt_per)
            kofs = (t - p * kt_per) * blk
            for band in (x, y0, y1):
                r0 = band * P_BM
                off = (r0 // 256) * kblocks * blk + (r0 % 256) * 32
                assert (r0 % 256) + P_BM <= 256             # a tile stays in one panel block
                assert off + kofs >= 0 and off + kofs + (P_BM - 1) * 32 + 32 <= Np * Np
        tiles = [(ti, tj)] + ([(ti2, tj2)] if ti2 >= 0 else [])
        for r, c in tiles:
            for grow, gcol in ((r * P_BM + P_BM - 1, c * P_BM + P_BM - 4),
                               (c * P_BM + P_BM - 1, r * P_BM + P_BM - 4)):
                assert grow * ld + gcol + 4 <= Np * ld
                pi = ((grow // 256) * kblocks + gcol // 32) * blk + (grow % 256) * 32 + gcol % 32
                assert gcol % 32 + 4 <= 32 and pi + 4 <= Np * Np


def _pair_epilogue_stores(r0, c0, kd):
    """The pair epilogue's stores for one tile at (r0, c0) (the first tile of
    an item, h = 0), as the kernel's index arithmetic forms them: a map
    (row, col) -> number of split stores, the set of master stores, and
    whether every staged entry the mirror pass reads was written as a split by
    the direct pass of the same round."""
    BN, SR, NT = 2 * P_BM, 32 * P_WGM, P_NT
    ITER = SR * BN // (4 * NT)
    diag = r0 == c0
    split, master, reads_ok = {}, set(), True
    for m in range(P_BM // P_WT):
        staged = set()
        for g in range(ITER):
            e = (np.arange(NT) + g * NT) * 4
            tr, lc = e // BN, e % BN
            for t_r, l_c in zip(tr, lc):
                h, lcl = l_c // P_BM, l_c % P_BM
                if h:
                    continue
                lr = (t_r >> 5) * P_WT + m * 32 + (t_r & 31)
                grow, gcol = r0 + lr, c0 + lcl
                if grow >= kd or gcol >= kd:
                    continue
                staged.update((t_r, l_c + q) for q in range(4))
                for q in range(4):
                    if not diag or lr <= lcl + q:
                        split[(grow, gcol + q)] = split.get((grow, gcol + q), 0) + 1
                        master.add((grow, gcol + q))
        for e in range(BN * (SR // 4)):
            qd, lc = e % (SR // 4), e // (SR // 4)
            h, lcl = lc // P_BM, lc % P_BM
            if h:
                continue
            tr = 4 * qd
            lr = (tr >> 5) * P_WT + m * 32 + (tr & 31)
            if diag and lr >= lcl:
                continue
            grow, gcol = c0 + lcl, r0 + lr
            if grow >= kd or gcol >= kd:
                continue
            reads_ok &= all((tr + q, lc) in staged for q in range(4))
            for q in range(4):
                if not diag or lr + q < lcl:
                    split[(grow, gcol + q)] = split.get((grow, gcol + q), 0) + 1
    return split, master, reads_ok


@pytest.mark.parametrize("N,ti,tj", [(37, 0, 0), (300, 2, 2), (300, 0, 2), (300, 1, 2),
                                     (256, 0, 1), (200, 1, 1)])
def test_pair_epilogue_skips_only_the_zero_padding(N, ti, tj):
    """The pair epilogue leaves out rows and columns from kd = N rounded up to
    32 on (zero in every buffer).  Inside [0, kd)^2 the tile and its mirror
    still get every split exactly once and the masters every element of the
    upper side; the mirror pass reads only staged splits of the same round."""
    kd = -(-N // 32) * 32
    r0, c0 = ti * P_BM, tj * P_BM
    split, master, reads_ok = _pair_epilogue_stores(r0, c0, kd)
    assert reads_ok
    rows = range(r0, min(r0 + P_BM, kd))
    cols = range(c0, min(c0 + P_BM, kd))
    want = {(i, j) for i in rows for j in cols if r0 != c0 or i <= j}
    assert master == want
    want_split = want | {(j, i) for (i, j) in want}
    assert set(split) == want_split and set(split.values()) <= {1}
    assert all(i < kd and j < kd for (i, j) in split)


def _trace_walk(kb, U=8):
    """The trace kernel's batch loop over kb panel blocks: (fetched block
    indices, blocks multiplied in order)."""
    nb = -(-kb // U)
    fetched, used = [], []
    bufs = [None, None]

    def fetch(slot, i):
        blocks = [min(i * U + u, kb - 1) for u in range(U)]
        fetched.extend(blocks)
        bufs[slot] = (i, blocks)

    def consume(slot, i):
        j, blocks = bufs[slot]
        assert j == i                                   # the buffer holds batch i
        cnt = min(U, kb - i * U)
        used.extend(blocks[:cnt])

    fetch(0, 0)
    for q in range(0, nb, 2):
        fetch(1, q + 1 if q + 1 < nb else q)
        consume(0, q)
        fetch(0, q + 2 if q + 2 < nb else q)
        if q + 1 < nb:
            consume(1, q + 1)
    return fetched, used


@pytest.mark.parametrize("kb", list(range(1, 40)) + [512, 513])
def test_trace_batches_cover_every_block_once_in_order(kb):
    """Every fetch stays inside [0, kb) and the MFMAs take blocks 0 .. kb - 1
    exactly once, in k order (the product's sequence, so the diagonal stays
    bitwise the product's)."""
    fetched, used = _trace_walk(kb)
    assert min(fetched) >= 0 and max(fetched) <= kb - 1
    assert used == list(range(kb))
