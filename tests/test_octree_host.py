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


@pytest.mark.parametrize("case", ["small_l2", "small_l3", "cfg3_start", "cfg3_window"])
def test_library_path_leaves_equal_the_input_generator(case):
    """pbf_octree_path_leaves (the library's leaf generator, used by the octree
    schedule for its remeshes) gives exactly the leaves of the seeded input
    generator, in the same Morton order, and they form a valid 2:1 mesh."""
    from paper_2302_05164_amd import pbftherm
    if case == "small_l2":
        p, lo, hi = W.small_octree(), 0.0, 60e-6
    elif case == "small_l3":
        p, lo, hi = W.small_octree(max_level=3, radius=30e-6), 0.0, 150e-6
    elif case == "cfg3_start":
        p, lo, hi = W.cfg3(), 0.0, 50e-6
    else:
        p, lo, hi = W.cfg3(), 1.9e-3, 2.4e-3
    ref = W.octree_leaves(p, hi, lo)
    got = pbftherm.octree_path_leaves(p.nx, p.ny, p.nz, p.L, p.max_level, p.refine_radius, p.tracks, lo, hi)
    assert got.dtype == np.int32 and got.shape == ref.shape
    assert np.array_equal(got, ref)
    L, ctx = _ctx()
    try:
        assert _mesh(L, ctx, p, got) == 0  # tiles the box, 2:1 balanced
    finally:
        L.pbf_destroy(ctx)


def test_path_leaves_capacity_and_arguments():
    from paper_2302_05164_amd import pbftherm
    L = pbftherm.load_library()
    p = W.small_octree()
    arr, nt = pbftherm._track_array(p.tracks)
    n = C.c_int64()
    args = (None, p.nx, p.ny, p.nz, *map(float, p.L), p.max_level, p.refine_radius, nt, arr, 0.0, 60e-6)
    assert L.pbf_octree_path_leaves(*args, None, 0, C.byref(n)) == 0 and n.value == 145
    small = np.zeros((10, 4), dtype=np.int32)
    assert L.pbf_octree_path_leaves(*args, small.ctypes.data_as(C.POINTER(C.c_int32)), 10, C.byref(n)) == -2
    bad = (None, p.nx, p.ny, p.nz, *map(float, p.L), 16, p.refine_radius, nt, arr, 0.0, 60e-6)
    assert L.pbf_octree_path_leaves(*bad, None, 0, C.byref(n)) == -1


@pytest.mark.parametrize("n0,ml", [((2, 1), 2), ((1, 2), 3), ((3, 2), 2)])
def test_library_layer_leaves_equal_the_oracle(n0, ml):
    """pbf_octree_layer_leaves (Section 4.1 adaptation in the library) gives the
    leaves of the oracle's plain implementation over a sequence of layer
    activations with seeded per-leaf consolidated fractions; the library
    accepts each as a growing mesh with the new top."""
    from oracle import layers as LY
    from paper_2302_05164_amd import pbftherm
    rng = np.random.default_rng(11)
    d_haz = 4
    top = 1 << ml
    h0 = 0.25e-3
    L_box = (n0[0] * h0, n0[1] * h0, 4 * h0)
    lv = LY.initial_leaves(n0, ml, top, d_haz)
    lib = pbftherm.load_library()
    for layer in range(10):
        ctx = C.c_void_p()
        assert lib.pbf_create(C.byref(ctx)) == 0
        try:
            lv32 = np.ascontiguousarray(lv, dtype=np.int32)
            assert lib.pbf_mesh_octree_growing(ctx, 2, n0[0], n0[1], 4, *L_box, ml, top, len(lv32),
                                               lv32.ctypes.data_as(C.POINTER(C.c_int32))) == 0
            rc = rng.choice([0.3, 0.95, 1.0], size=len(lv), p=[0.1, 0.3, 0.6])
            n = C.c_int64()
            rcp = np.ascontiguousarray(rc).ctypes.data_as(C.POINTER(C.c_double))
            assert lib.pbf_octree_layer_leaves(ctx, rcp, top + 1, d_haz, 0.9, None, 0, C.byref(n)) == 0
            got = np.zeros((n.value, 4), dtype=np.int32)
            assert lib.pbf_octree_layer_leaves(ctx, rcp, top + 1, d_haz, 0.9,
                                               got.ctypes.data_as(C.POINTER(C.c_int32)), n.value, C.byref(n)) == 0
        finally:
            lib.pbf_destroy(ctx)
        ref = LY.adapt(lv, rc, ml, n0, top, top + 1, d_haz, 0.9)
        assert np.array_equal(got, ref), f"layer {layer}"
        lv, top = ref, top + 1


def test_growing_mesh_dofs_match_the_oracle():
    """A growing octree (active part below the top) has the oracle's dofs,
    hanging nodes and Dirichlet nodes on z = top for face z+."""
    from oracle import layers as LY
    from paper_2302_05164_amd import pbftherm
    p = W.cfg3_reduced(max_level=2).replace(dirichlet_mask=W.FACE_ZM | W.FACE_ZP)
    top = 6
    lv = LY.initial_leaves((p.nx, p.ny), p.max_level, 4, 4)
    lv = LY.adapt(lv, None, p.max_level, (p.nx, p.ny), 4, top, 4, 0.9)
    O = OctOracle(p.replace(leaves=lv), top=top)
    lib = pbftherm.load_library()
    ctx = C.c_void_p()
    assert lib.pbf_create(C.byref(ctx)) == 0
    try:
        lv32 = np.ascontiguousarray(lv, dtype=np.int32)
        assert lib.pbf_mesh_octree_growing(ctx, 2, p.nx, p.ny, p.nz, *map(float, p.L), p.max_level, top,
                                           len(lv32), lv32.ctypes.data_as(C.POINTER(C.c_int32))) == 0
        nd = C.c_int64()
        assert lib.pbf_mesh_info(ctx, C.byref(nd), None, None, None, None, None) == 0
        nl, nh, mx = C.c_int64(), C.c_int64(), C.c_int()
        assert lib.pbf_octree_info(ctx, C.byref(nl), C.byref(nh), C.byref(mx)) == 0
        assert nd.value == O.N and nh.value == O.n_hanging
        x = np.zeros((nd.value, 3))
        assert lib.pbf_dof_coords(ctx, x.ctypes.data_as(C.POINTER(C.c_double))) == 0
        h = p.L[0] / p.nx / 2 ** p.max_level / 2
        assert _key(x, h) == _key(O.dof_coords(), h)
        ztop = top * p.L[2] / p.nz / 2 ** p.max_level
        assert abs(x[:, 2].max() - ztop) < 1e-15 and O.dirichlet_mask().sum() == \
            np.sum(np.isclose(O.dof_coords()[:, 2], 0.0) | np.isclose(O.dof_coords()[:, 2], ztop))
        # leaves above the top are refused
        bad = np.vstack([lv32, [[p.max_level, 0, 0, top]]]).astype(np.int32)
        assert lib.pbf_mesh_octree_growing(ctx, 2, p.nx, p.ny, p.nz, *map(float, p.L), p.max_level, top,
                                           len(bad), bad.ctypes.data_as(C.POINTER(C.c_int32))) == -3
    finally:
        lib.pbf_destroy(ctx)
