"""Pins of the octree oracle (hanging-node constraints) against what the
mathematics fixes: a uniformly refined octree is the box mesh, the constrained
space reproduces polynomials of the element degree, linear fields are steady
states away from the boundary, the diffusion operator is symmetric and
conservative, and transfer to a refined mesh is exact.  CPU only."""
import numpy as np
import pytest

import pbf_workloads as W
from oracle import OctOracle, Oracle


def _const_law(p):
    return p.replace(T_bp=np.array([0.0, 1e4]), k_bp=np.array([25.0, 25.0]), cp_bp=np.array([600.0, 600.0]),
                     latent=0.0, powder_k_factor=1.0, powder_depth=0.0, laser_kind=W.LASER_OFF)


def _uniform_leaves(nx, ny, nz, level):
    s = 2 ** 0  # leaves at the finest level have size 1 in finest units
    g = np.stack(np.meshgrid(np.arange(nx * 2 ** level), np.arange(ny * 2 ** level),
                             np.arange(nz * 2 ** level), indexing="ij"), -1).reshape(-1, 3) * s
    return np.concatenate([np.full((len(g), 1), level), g], 1).astype(np.int64)


@pytest.mark.parametrize("deg", [1, 2])
def test_dof_and_hanging_counts_one_refined_cell(deg):
    """Two coarse cells, one refined once: the refined cell has (2p+1)^3 nodes,
    the coarse one (p+1)^3 of which (p+1)^2 lie on the shared face; of the
    (2p+1)^2 fine nodes on that face the (p+1)^2 coarse ones are regular and the
    others hang."""
    p = W.small_octree(degree=deg).replace(nx=2, ny=1, nz=1, L=(2e-4, 1e-4, 1e-4), max_level=1)
    leaves = [[0, 2, 0, 0]] + [[1, i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)]
    O = OctOracle(p, leaves=np.array(leaves))
    n_fine, n_face_fine, n_face_coarse = (2 * deg + 1) ** 3, (2 * deg + 1) ** 2, (deg + 1) ** 2
    nodes = n_fine + (deg + 1) ** 3 - n_face_coarse
    assert O.n_hanging == n_face_fine - n_face_coarse
    assert O.N == nodes - O.n_hanging


@pytest.mark.parametrize("deg", [1, 2])
def test_uniform_octree_equals_box(deg):
    """All leaves on one level: the box mesh (same dof order), so the octree
    oracle must give the box oracle's vectors and steps."""
    p = W.small_nonlinear(nx=4, ny=4, nz=2, steps=0, h=62.5e-6, n_tracks=2, track_length=0.15e-3,
                          hatch=60e-6).replace(degree=deg)
    box = Oracle(p)
    po = p.replace(nx=2, ny=2, nz=1, max_level=1)
    O = OctOracle(po, leaves=_uniform_leaves(2, 2, 1, 1))
    assert O.N == box.N and O.n_hanging == 0
    T = box.init_T() + 900.0 * (1.0 + W.seeded_vector(box.N, 3))
    rb = box.init_history()
    f1, C1, v1 = box.assemble(T, rb.copy(), 2e-5)
    f2, C2, v2 = O.assemble(T, O.init_history(), 2e-5)
    for a, b in ((f1, f2), (C1, C2), (v1, v2)):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    dt = 2e-7
    Tb = box.init_T()
    To = O.init_T()
    box.explicit_steps(Tb, rb, 0.0, dt, 30)
    O.explicit_steps(To, O.init_history(), 0.0, dt, 30)
    assert np.abs(Tb - To).max() <= 1e-12 * Tb.max()
    lb = box.stability_lambda(W.seeded_vector(box.N, 1), 40)
    lo = O.stability_lambda(W.seeded_vector(box.N, 1), 40)
    assert abs(lb - lo) <= 1e-12 * lb
    Ti_b, ib = box.implicit_step(Tb, box.init_history(), 0.0, 1e-4, cg_rtol=1e-12)
    Ti_o, io = O.implicit_step(To, O.init_history(), 0.0, 1e-4, cg_rtol=1e-12)
    assert ib["status"] == io["status"] == 0 and ib["cg_iters"] == io["cg_iters"]
    assert np.abs(Ti_b - Ti_o).max() <= 1e-10 * Ti_b.max()


def _poly(x, deg):
    X, Y, Z = (x[:, 0] / 1e-4, x[:, 1] / 1e-4, x[:, 2] / 1e-4)
    v = 300.0 + 11.0 * X - 7.0 * Y + 5.0 * Z
    if deg == 2:
        v = v + 3.0 * X * X - 2.0 * X * Y + 4.0 * Y * Z + 1.5 * Z * Z - Y * Y + 2.5 * X * Z
    return v


@pytest.mark.parametrize("deg", [1, 2])
def test_constrained_space_reproduces_polynomials(deg):
    """Dof values of a polynomial of degree p give exactly that polynomial
    everywhere, including in cells with hanging nodes."""
    p = W.small_octree(degree=deg)
    O = OctOracle(p)
    assert O.n_hanging > 0
    T = _poly(O.dof_coords(), deg)
    rng = np.random.default_rng(5)
    pts = rng.uniform(0, 1, (400, 3)) * np.array(p.L)
    np.testing.assert_allclose(O.probe(T, pts), _poly(pts, deg), rtol=1e-12, atol=0)


@pytest.mark.parametrize("deg", [1, 2])
def test_linear_field_is_steady_inside(deg):
    """Constant k, no source: for T linear, f_i = -k int grad N_i . grad T is a
    boundary integral, zero for every dof off the box boundary."""
    p = _const_law(W.small_octree(degree=deg))
    O = OctOracle(p)
    x = O.dof_coords()
    T = _poly(x, 1)
    f, _, _ = O.assemble(T, O.init_history(), 0.0)
    inner = np.all((x > 1e-12) & (x < np.array(p.L) - 1e-12), axis=1)
    assert inner.sum() > 30
    scale = 25.0 * np.abs(T).max() * 1e-4  # k |grad T| h^2 / h
    assert np.abs(f[inner]).max() <= 1e-11 * scale


@pytest.mark.parametrize("deg", [1, 2])
def test_diffusion_symmetric_and_conservative(deg):
    p = _const_law(W.small_octree(degree=deg))
    O = OctOracle(p)
    rc = O.init_history()
    v, w = W.seeded_vector(O.N, 1), W.seeded_vector(O.N, 2)
    fv, _, _ = O.assemble(v, rc, 0.0)
    fw, _, _ = O.assemble(w, rc, 0.0)
    assert abs(np.dot(v, fw) - np.dot(w, fv)) <= 1e-12 * np.abs(v).sum() * np.abs(fw).max()
    # the nonlinear law with history: rows still sum to zero
    q = W.small_octree(degree=deg).replace(laser_kind=W.LASER_OFF)
    Oq = OctOracle(q)
    T = Oq.init_T() + 900.0 * (1.0 + W.seeded_vector(Oq.N, 4))
    f, _, _ = Oq.assemble(T, Oq.init_history(), 0.0)
    assert abs(f.sum()) <= 1e-12 * np.abs(f).sum()


@pytest.mark.parametrize("deg", [1, 2])
def test_lumped_mass_sums_to_volume(deg):
    p = _const_law(W.small_octree(degree=deg))
    O = OctOracle(p)
    _, C, _ = O.assemble(O.init_T(), O.init_history(), 0.0)
    assert C.min() > 0
    np.testing.assert_allclose(C.sum() / (p.rho * 600.0), np.prod(p.L), rtol=1e-12)


def test_transfer_to_refined_mesh_is_exact():
    """Refining the mesh (the old space is a subspace of the new one): the field
    is reproduced exactly, and the history is copied from the old points."""
    p = W.small_octree(degree=2, ahead=30e-6)
    old = OctOracle(p)
    new = OctOracle(p, leaves=W.octree_leaves(p, 150e-6))
    assert new.N > old.N
    T = old.init_T() + 500.0 * (1.0 + W.seeded_vector(old.N, 9))
    rc = old.init_history()
    rc[::3] = 0.7
    Tn, rn = old.transfer(T, rc, new)
    rng = np.random.default_rng(3)
    pts = rng.uniform(0, 1, (300, 3)) * np.array(p.L)
    np.testing.assert_allclose(new.probe(Tn, pts), old.probe(T, pts), rtol=1e-12, atol=0)
    assert set(np.unique(rn)) <= {0.0, 0.7, 1.0}


def test_generated_octrees_are_balanced():
    """2:1 balance across faces, edges and vertices, and the leaves tile the box."""
    for p in (W.small_octree(max_level=3, ahead=100e-6), W.small_octree(max_level=2)):
        lv = p.leaves
        n0 = np.array([p.nx, p.ny, p.nz]) * 2 ** p.max_level
        size = 2 ** (p.max_level - lv[:, 0])
        assert (size.astype(np.int64) ** 3).sum() == np.prod(n0)
        lo = lv[:, 1:]
        hi = lo + size[:, None]
        touch = np.all((lo[:, None, :] <= hi[None, :, :]) & (lo[None, :, :] <= hi[:, None, :]), axis=2)
        overlap = np.all((lo[:, None, :] < hi[None, :, :]) & (lo[None, :, :] < hi[:, None, :]), axis=2)
        np.fill_diagonal(overlap, False)
        assert not overlap.any()
        dl = np.abs(lv[:, None, 0] - lv[None, :, 0])
        assert dl[touch].max() <= 1
