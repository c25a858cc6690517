"""Pins of the per-layer mesh adaptation written out for the tests
(oracle/layers.py, Section 4.1): invariants checked on a finest-cell grid (a
formulation independent of the leaf lists), and hand-worked cases of
coarsening and its threshold."""
import numpy as np
import pytest

from oracle import layers as LY


def _grid(leaves, max_level, n0, top):
    """level of the leaf covering each finest cell; -1 uncovered; counts"""
    nfx, nfy = n0[0] << max_level, n0[1] << max_level
    lev = -np.ones((top, nfy, nfx), dtype=np.int64)
    cnt = np.zeros((top, nfy, nfx), dtype=np.int64)
    for l, x, y, z in leaves:
        s = 1 << (max_level - l)
        assert x % s == 0 and y % s == 0 and z % s == 0
        assert z + s <= top, "leaf above the active top"
        lev[z:z + s, y:y + s, x:x + s] = l
        cnt[z:z + s, y:y + s, x:x + s] += 1
    return lev, cnt


def _check_mesh(leaves, max_level, n0, top, d_haz):
    lev, cnt = _grid(leaves, max_level, n0, top)
    assert (cnt == 1).all(), "leaves must tile the active part exactly once"
    # 2:1 across faces, edges and vertices: neighbouring finest cells
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                a = lev[max(0, dz):top + min(0, dz), max(0, dy):lev.shape[1] + min(0, dy),
                        max(0, dx):lev.shape[2] + min(0, dx)]
                b = lev[max(0, -dz):top + min(0, -dz), max(0, -dy):lev.shape[1] + min(0, -dy),
                        max(0, -dx):lev.shape[2] + min(0, -dx)]
                assert np.abs(a - b).max() <= 1
    # the current layer and the HAZ at the finest level
    assert (lev[max(0, top - 1 - d_haz):top] == max_level).all()
    return lev


@pytest.mark.parametrize("n0,ml", [((2, 1), 2), ((1, 2), 3)])
def test_layer_sequence_invariants(n0, ml):
    rng = np.random.default_rng(7)
    d_haz = 4
    top = 1 << ml
    lv = LY.initial_leaves(n0, ml, top, d_haz)
    old_lev = _check_mesh(lv, ml, n0, top, d_haz)
    for layer in range(12):
        rc = rng.choice([0.3, 0.95, 1.0], size=len(lv), p=[0.1, 0.3, 0.6])
        new = LY.adapt(lv, rc, ml, n0, top, top + 1, d_haz, 0.9)
        lev = _check_mesh(new, ml, n0, top + 1, d_haz)
        # wherever a cell got coarser, every old leaf inside its new leaf was
        # above the threshold and the new leaf lies farther than d_HAZ below
        # the current layer; coarsening goes one level at a time
        rcg = np.full(old_lev.shape, np.nan)
        for (l, x, y, z), r in zip(lv, rc):
            s = 1 << (ml - l)
            rcg[z:z + s, y:y + s, x:x + s] = r
        for l, x, y, z in new:
            s = 1 << (ml - l)
            if z + s > top:
                continue
            old = old_lev[z:z + s, y:y + s, x:x + s]
            if (old > l).any():
                assert (old == l + 1).all()
                assert (rcg[z:z + s, y:y + s, x:x + s] > 0.9).all()
                assert (top + 1 - 1) - (z + s) > d_haz
        lv, top, old_lev = new, top + 1, lev


def test_coarsening_threshold_hand_case():
    """One coarse column (max level 1: coarse cells are two layers tall).  After
    the layers have risen far enough, the octets at the bottom are farther than
    d_HAZ = 4 layers below the current layer and coarsen when their
    consolidated fraction exceeds 0.9 everywhere, not when one leaf holds 0.5;
    coarsening one octet of a 2x1 coarse row cannot unbalance the mesh."""
    n0, ml, d = (2, 1), 1, 4
    lv = LY.initial_leaves(n0, ml, 2, d)  # z in [0, 2): every cell at level 1
    assert len(lv) == 2 * 8
    top = 2
    for _ in range(5):  # layers up to z = 7
        lv = LY.adapt(lv, np.ones(len(lv)), ml, n0, top, top + 1, d, 0.9)
        top += 1
    # current layer [6, 7): cells with z_max > 6 - 4 = 2 stay fine; the octets
    # with z in [0, 2) (z_max = 2, distance 4, not greater than d_HAZ) stay
    assert all(l == 1 for l, *_ in lv)
    lv8 = LY.adapt(lv, np.ones(len(lv)), ml, n0, top, top + 1, d, 0.9)
    # current layer [7, 8): the two bottom octets are at distance 5 > 4
    coarse = sorted(tuple(r[1:]) for r in lv8 if r[0] == 0)
    assert coarse == [(0, 0, 0), (2, 0, 0)]
    rc = np.ones(len(lv))
    i = next(i for i, r in enumerate(lv) if tuple(r) == (1, 1, 1, 1))
    rc[i] = 0.5  # an unfused point in the first octet keeps it refined
    lv8b = LY.adapt(lv, rc, ml, n0, top, top + 1, d, 0.9)
    coarse = sorted(tuple(r[1:]) for r in lv8b if r[0] == 0)
    assert coarse == [(2, 0, 0)]
    rc[i] = 0.9  # the threshold itself is not above it
    assert sorted(tuple(r[1:]) for r in LY.adapt(lv, rc, ml, n0, top, top + 1, d, 0.9) if r[0] == 0) == [(2, 0, 0)]


def test_balance_splits_the_coarser_neighbour():
    """A finest leaf next to a coarse cell two levels coarser forces the coarse
    cell to split once (face, edge and vertex contact alike)."""
    ml = 2
    lv = [(0, 4, 0, 0)] + [(1, x, y, z) for z in (0, 2) for y in (0, 2) for x in (0, 2)
                           if (x, y, z) != (0, 0, 0)] + \
         [(2, x, y, z) for z in (0, 1) for y in (0, 1) for x in (0, 1)]
    out = LY.balance(lv, ml)
    # the level-2 leaves at x = 1 touch only level-1 leaves within the first
    # coarse cell; the coarse cell at x = 4 touches level-1 leaves only
    assert (0, 4, 0, 0) in set(map(tuple, out.tolist()))
    lv2 = [(0, 4, 0, 0)] + [(1, x, y, z) for z in (0, 2) for y in (0, 2) for x in (0, 2)
                            if (x, y, z) != (2, 0, 0)] + \
          [(2, x, y, z) for z in (0, 1) for y in (0, 1) for x in (2, 3)]
    out2 = set(map(tuple, LY.balance(lv2, ml).tolist()))
    assert (0, 4, 0, 0) not in out2  # a level-2 leaf at x = 3 touches it: split
    assert {(1, 4, 0, 0), (1, 6, 2, 2)} <= out2
