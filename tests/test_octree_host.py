"""CPU checks of the library's octree host code (no GPU): dof map and hanging
nodes against the oracle's brute-force construction, and rejection of invalid
leaf sets."""
import ctypes as C

import numpy as np
import pytest

import pbf_workloads as W
from oracle import OctOracle


def _ctx():
    from paper_2302_05164_amd import pbftherm
    L = pbftherm.load_library()
    ctx = C.c_void_p()
    assert L.pbf_create(C.byref(ctx)) == 0
    return L, ctx


def _mesh(L, ctx, p, leaves):
    lv = np.ascontiguousarray(leaves, dtype=np.int32)
    return L.pbf_mesh_octree(ctx, p.degree, p.nx, p.ny, p.nz, *map(float, p.L), p.max_level, len(lv),
                             lv.ctypes.data_as(C.POINTER(C.c_int32)))


def _key(x, h):
    return set(map(tuple, np.round(x / h).astype(np.int64)))


@pytest.mark.parametrize("deg,ml,ahead", [(1, 2, 60e-6), (2, 2, 60e-6), (2, 3, 100e-6)])
def test_dof_map_matches_oracle(deg, ml, ahead):
    p = W.small_octree(degree=deg, max_level=ml, ahead=ahead)
    L, ctx = _ctx()
    try:
        assert _mesh(L, ctx, p, p.leaves) == 0
        nd = C.c_int64()
        assert L.pbf_mesh_info(ctx, C.byref(nd), None, None, None, None, None) == 0
        nl, nh, mx = C.c_int64(), C.c_int64(), C.c_int()
        assert L.pbf_octree_info(ctx, C.byref(nl), C.byref(nh), C.byref(mx)) == 0
        O = OctOracle(p)
        assert nd.value == O.N and nh.value == O.n_hanging and nl.value == len(p.leaves) and mx.value == ml
        x = np.zeros((nd.value, 3))
        assert L.pbf_dof_coords(ctx, x.ctypes.data_as(C.POINTER(C.c_double))) == 0
        h = p.L[0] / p.nx / 2 ** ml / deg
        assert _key(x, h) == _key(O.dof_coords(), h)
    finally:
        L.pbf_destroy(ctx)


def test_invalid_leaf_sets_are_rejected():
    p = W.small_octree(degree=2, max_level=2)
    L, ctx = _ctx()
    try:
        lv = p.leaves.copy()
        assert _mesh(L, ctx, p, lv[1:]) == -3  # a gap
        assert b"cover" in L.pbf_last_error(ctx)
        assert _mesh(L, ctx, p, np.concatenate([lv, lv[:1]])) == -3  # duplicate
        bad = lv.copy()
        bad[0, 1] += 1  # misaligned origin
        assert _mesh(L, ctx, p, bad) == -3
        # a coarse cell next to cells two levels finer
        q = p.replace(nx=2, ny=1, nz=1, L=(2.5e-4, 1.25e-4, 1.25e-4), max_level=2)
        fine = [[2, i, j, k] for k in range(4) for j in range(4) for i in range(4)]
        assert _mesh(L, ctx, q, np.array([[0, 4, 0, 0]] + fine)) == -3
        assert b"balanced" in L.pbf_last_error(ctx)
        assert _mesh(L, ctx, p, lv) == 0
    finally:
        L.pbf_destroy(ctx)


def test_surface_loss_parameters_validated():
    """pbf_set_surface_loss rejects negative or non-finite constants (no GPU)."""
    from paper_2302_05164_amd import pbftherm
    L, ctx = _ctx()
    try:
        S = pbftherm._SurfaceLoss
        ok = S(0.7, 293.0, 1, 3000.0, 54e3, 5e4, 1e-3, 6e6, 663.0, 1000.0)
        assert L.pbf_set_surface_loss(ctx, C.byref(ok)) == 0
        assert L.pbf_set_surface_loss(ctx, None) == 0  # off
        for bad in (S(-0.1, 293.0, 0, 0, 0, 0, 0, 0, 0, 0), S(float("nan"), 293.0, 0, 0, 0, 0, 0, 0, 0, 0),
                    S(0.7, 293.0, 1, 3000.0, 54e3, 5e4, 0.0, 6e6, 663.0, 1000.0),
                    S(0.7, 293.0, 1, 3000.0, 54e3, 5e4, 1e-3, 6e6, 663.0, -5.0)):
            assert L.pbf_set_surface_loss(ctx, C.byref(bad)) != 0
            assert L.pbf_last_error(ctx)
    finally:
        L.pbf_destroy(ctx)
