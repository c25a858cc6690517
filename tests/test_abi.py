"""CPU checks of the C ABI library: it loads, exports every declared symbol,
and validates arguments on the host (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pbftherm.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:pbf_status|void|const char \*)\s*(pbf_\w+)\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2302_05164_amd import pbftherm
    L = pbftherm.load_library()
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    # the binding declares argument types for every exported entry point
    assert set(names) == set(pbftherm.SIGNATURES)


def _ctx():
    from paper_2302_05164_amd import pbftherm
    L = pbftherm.load_library()
    ctx = C.c_void_p()
    assert L.pbf_create(C.byref(ctx)) == 0
    return L, ctx


def test_host_validation_errors():
    from paper_2302_05164_amd import pbftherm
    L, ctx = _ctx()
    try:
        assert L.pbf_mesh_box(ctx, 3, 4, 4, 4, 1.0, 1.0, 1.0) == -3  # EMESH
        assert b"degree" in L.pbf_last_error(ctx)
        assert L.pbf_mesh_box(ctx, 2, 0, 4, 4, 1.0, 1.0, 1.0) == -1
        assert L.pbf_mesh_box(ctx, 2, 4, 4, 4, 1.0, -1.0, 1.0) == -1
        # stepping before binding
        assert L.pbf_mesh_box(ctx, 2, 4, 4, 4, 1.0, 1.0, 1.0) == 0
        assert L.pbf_explicit_steps(ctx, None, None, None, 0.0, 1e-3, 1, 64, None) == -7
        dt = C.c_double()
        assert L.pbf_stability_dt(ctx, None, 10, C.byref(dt), None, None) == -7  # material not set
        assert L.pbf_stability_dt(ctx, None, 10, None, None, None) == -1  # no output
        assert L.pbf_laplace_apply(ctx, None, None, None) == -7
        assert L.pbf_set_dirichlet(ctx, 64, 293.0) == -1
        assert L.pbf_set_newton_forcing(ctx, 7) == -1
        assert b"Eisenstat" in L.pbf_last_error(ctx)
        assert L.pbf_set_newton_forcing(ctx, 1) == 0 and L.pbf_set_newton_forcing(ctx, 0) == 0
        assert L.pbf_set_newton_forcing(None, 0) == -1
        # unsorted breakpoints
        import numpy as np
        T = np.array([300.0, 200.0])
        k = np.array([1.0, 1.0])
        dp = C.POINTER(C.c_double)
        m = pbftherm._Material(2, T.ctypes.data_as(dp), k.ctypes.data_as(dp), k.ctypes.data_as(dp),
                               7900.0, 1500.0, 1600.0, 0.0, 0.01, 0.0)
        assert L.pbf_set_material(ctx, C.byref(m)) == -1
        assert b"increasing" in L.pbf_last_error(ctx)
        m.T_bp = np.array([200.0, 300.0]).ctypes.data_as(dp)
        m.T_s, m.T_l = 1600.0, 1500.0
        assert L.pbf_set_material(ctx, C.byref(m)) == -1
        nb = C.c_size_t()
        assert L.pbf_workspace_bytes(ctx, C.byref(nb)) == 0 and nb.value > 0
        # misaligned / too small workspace is rejected before any device work
        assert L.pbf_bind_device(ctx, C.c_void_p(256), 16, None) == -2
        assert L.pbf_bind_device(ctx, C.c_void_p(257), nb.value, None) == -1
    finally:
        L.pbf_destroy(ctx)


def test_mesh_info_and_history_layers():
    import pbf_workloads as W
    from paper_2302_05164_amd import pbftherm
    L, ctx = _ctx()
    try:
        p = W.cfg2()
        assert L.pbf_mesh_box(ctx, 2, p.nx, p.ny, p.nz, *p.L) == 0
        import numpy as np
        dp = C.POINTER(C.c_double)
        arrs = [np.ascontiguousarray(a) for a in (p.T_bp, p.k_bp, p.cp_bp)]
        m = pbftherm._Material(8, *[a.ctypes.data_as(dp) for a in arrs], p.rho, p.T_s, p.T_l,
                               p.latent, p.powder_k_factor, p.powder_depth)
        assert L.pbf_set_material(ctx, C.byref(m)) == 0
        v = [C.c_int64() for _ in range(6)]
        assert L.pbf_mesh_info(ctx, *[C.byref(x) for x in v]) == 0
        nd, nc, nq, nhl, nhc, nhq = (x.value for x in v)
        assert nd == 8_520_321 and nc == 1_048_576 and nq == 27 * nc
        # 40 um of powder on 31.25 um cells: the top layer and the lowest Gauss
        # level of the second layer start as powder
        assert nhl == 2 and nhc == 2 * 128 * 128 and nhq == 27 * nhc
    finally:
        L.pbf_destroy(ctx)


def test_workspace_sizes_face_slots_and_rejects_oversized_boxes():
    """The parity-slot storage holds one entry per column-face node (8 parities),
    not one per node, and a box whose face nodes exceed the 32-bit index range of
    the face kernels is rejected at workspace sizing with a message."""
    L, ctx = _ctx()
    try:
        b = C.c_size_t()
        assert L.pbf_mesh_box(ctx, 2, 128, 128, 64, 4e-3, 4e-3, 2e-3) == 0
        assert L.pbf_workspace_bytes(ctx, C.byref(b)) == 0
        n = 257 * 257 * 129
        # 11 vectors of n doubles plus slots far below 8 n doubles (cfg2: ~0.93 M face nodes)
        assert 11 * 8 * n < b.value < 11 * 8 * n + 8 * 8 * 1_000_000 + 2 * 2**30
        assert L.pbf_mesh_box(ctx, 2, 4096, 4096, 4096, 1.0, 1.0, 1.0) == 0
        assert L.pbf_workspace_bytes(ctx, C.byref(b)) != 0
        assert b"too large" in L.pbf_last_error(ctx)
    finally:
        L.pbf_destroy(ctx)


def test_noalloc_steps_host_refusals():
    """pbf_explicit_steps_noalloc refuses on the host, before any device call:
    no material, octree meshes, and boxes whose scratch exceeds the 32 MiB
    static array (reporting the bytes the mesh needs)."""
    import numpy as np
    from paper_2302_05164_amd import pbftherm
    L, ctx = _ctx()
    need = C.c_size_t(0)
    try:
        assert L.pbf_mesh_box(ctx, 2, 128, 128, 64, 4e-3, 4e-3, 2e-3) == 0
        assert L.pbf_explicit_steps_noalloc(ctx, None, None, None, 0.0, 1e-6, 1, 64, C.byref(need), None) == -7
        T = np.array([293.0, 3000.0])
        k = np.array([20.0, 30.0])
        dp = C.POINTER(C.c_double)
        m = pbftherm._Material(2, T.ctypes.data_as(dp), k.ctypes.data_as(dp), k.ctypes.data_as(dp),
                               7900.0, 1563.0, 1623.0, 0.0, 0.01, 0.0)
        assert L.pbf_set_material(ctx, C.byref(m)) == 0
        assert L.pbf_explicit_steps_noalloc(ctx, None, None, None, 0.0, 1e-6, 1, 64, C.byref(need), None) == -2
        assert need.value > 32 << 20
        assert b"static scratch" in L.pbf_last_error(ctx)
        lv = np.array([0, 0, 0, 0], dtype=np.int32)
        assert L.pbf_mesh_octree(ctx, 2, 1, 1, 1, 1e-3, 1e-3, 1e-3, 0, 1,
                                 lv.ctypes.data_as(C.POINTER(C.c_int32))) == 0
        assert L.pbf_explicit_steps_noalloc(ctx, None, None, None, 0.0, 1e-6, 1, 64, None, None) == -3
    finally:
        L.pbf_destroy(ctx)
