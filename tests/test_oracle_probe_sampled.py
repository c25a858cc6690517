"""Pins of two oracle functions that the GPU parity tests lean on.

- Finite element probe T_h(x) = sum_a N_a(xi) T_a (Section 3.1, eq.
  bubnov_galerkin) on boxes: it must reproduce every field of degree <= p per
  variable exactly, and for an arbitrary nodal field it must equal the unique
  tensor-product polynomial through the nodes of a cell that contains the point
  (fitted here with numpy's Vandermonde matrices, not with the oracle's basis),
  at random interior points, on shared faces, edges and vertices, and on the
  domain boundary.  A wrong local node index, a transposed axis or a cell that
  does not contain the point fails these checks.
- The explicit step evaluated at listed nodes only (Section 3.2, eq.
  forward_euler), which is the reference for the full-size GPU checks: at every
  node of a small ragged box stepped into melting it must equal the full step.
"""
import itertools

import numpy as np
import pytest
from numpy.polynomial import polynomial as npoly

import pbf_workloads as W
from oracle import Oracle


def _box(deg):
    # ragged, non-cubic cells: hx != hy != hz
    p = W.small_nonlinear(nx=5, ny=4, nz=3, steps=0).replace(degree=deg)
    return p.replace(L=(5 * 31.25e-6, 4 * 40e-6, 3 * 27e-6))


def _nodes_of_cell(prob, c):
    p = prob.degree
    NX, NY, _ = prob.nodes_per_dim
    idx = []
    for az, ay, ax in itertools.product(range(p + 1), repeat=3):
        idx.append((p * c[0] + ax) + NX * ((p * c[1] + ay) + NY * (p * c[2] + az)))
    # (az, ay, ax) order of the loop: local coordinates
    loc = np.array([(ax / p, ay / p, az / p) for az, ay, ax in itertools.product(range(p + 1), repeat=3)])
    return np.array(idx), loc


def _fit_value(prob, T, c, xi):
    """Value at reference point xi of the tensor-product polynomial of degree p
    through the nodal values of cell c (Vandermonde solve)."""
    idx, loc = _nodes_of_cell(prob, c)
    p = prob.degree
    V = npoly.polyvander3d(loc[:, 0], loc[:, 1], loc[:, 2], [p, p, p])
    coef = np.linalg.solve(V, T[idx])
    return float(npoly.polyvander3d(np.array([xi[0]]), np.array([xi[1]]), np.array([xi[2]]), [p, p, p])[0] @ coef)


def _containing_cells(prob, x):
    """Every cell whose closed box contains x (test's own rule), with the
    reference coordinates of x in it."""
    n = (prob.nx, prob.ny, prob.nz)
    h = [prob.L[d] / n[d] for d in range(3)]
    per_dim = []
    for d in range(3):
        s = x[d] / h[d]
        cand = []
        for c in range(n[d]):
            t = s - c
            if -1e-12 <= t <= 1 + 1e-12:
                cand.append((c, min(max(t, 0.0), 1.0)))
        assert cand, x
        per_dim.append(cand)
    out = []
    for (cx, tx), (cy, ty), (cz, tz) in itertools.product(*per_dim):
        out.append(((cx, cy, cz), (tx, ty, tz)))
    return out


def _points(prob, rng):
    n = (prob.nx, prob.ny, prob.nz)
    h = np.array([prob.L[d] / n[d] for d in range(3)])
    L = np.array(prob.L)
    pts = [rng.uniform(0, 1, 3) * L for _ in range(40)]  # interior (almost surely)
    for _ in range(30):  # on shared faces, edges and vertices
        q = rng.uniform(0, 1, 3) * L
        k = rng.integers(1, 4)
        for d in rng.choice(3, size=k, replace=False):
            q[d] = rng.integers(1, n[d]) * h[d]
        pts.append(q)
    for corner in itertools.product(*[(0.0, L[d]) for d in range(3)]):  # box corners
        pts.append(np.array(corner))
    for d in range(3):  # boundary faces
        for side in (0.0, L[d]):
            q = rng.uniform(0, 1, 3) * L
            q[d] = side
            pts.append(q)
    # nodes
    NX, NY, NZ = prob.nodes_per_dim
    for _ in range(10):
        i, j, k = rng.integers(0, NX), rng.integers(0, NY), rng.integers(0, NZ)
        pts.append(np.array([i, j, k]) * h / prob.degree)
    return np.array(pts)


@pytest.mark.parametrize("deg", [1, 2])
def test_probe_reproduces_tensor_polynomials(deg):
    prob = _box(deg)
    o = Oracle(prob)
    NX, NY, NZ = prob.nodes_per_dim
    L = np.array(prob.L)
    k, j, i = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")
    X = (i / (NX - 1) * L[0]).ravel() / L[0]
    Y = (j / (NY - 1) * L[1]).ravel() / L[1]
    Z = (k / (NZ - 1) * L[2]).ravel() / L[2]
    rng = np.random.default_rng(deg)
    coef = rng.uniform(-1, 1, (deg + 1, deg + 1, deg + 1))
    T = npoly.polyval3d(X, Y, Z, coef)
    pts = _points(prob, rng)
    vals = o.probe(T, pts)
    exact = npoly.polyval3d(pts[:, 0] / L[0], pts[:, 1] / L[1], pts[:, 2] / L[2], coef)
    np.testing.assert_allclose(vals, exact, rtol=0, atol=1e-13 * np.abs(T).max())


@pytest.mark.parametrize("deg", [1, 2])
def test_probe_equals_cellwise_interpolant_of_random_field(deg):
    prob = _box(deg)
    o = Oracle(prob)
    rng = np.random.default_rng(10 + deg)
    T = 300.0 + 1000.0 * rng.random(o.N)
    pts = _points(prob, rng)
    vals = o.probe(T, pts)
    for x, v in zip(pts, vals):
        refs = [_fit_value(prob, T, c, xi) for c, xi in _containing_cells(prob, x)]
        # continuity: every containing cell gives the same value
        assert max(refs) - min(refs) <= 1e-10 * 1300.0
        assert abs(v - refs[0]) <= 1e-10 * 1300.0, (x, v, refs)


@pytest.mark.parametrize("deg", [1, 2])
def test_sampled_step_equals_full_step_at_every_node(deg):
    """From a hot state with melting and partly consolidated powder (oracle
    steps), one step evaluated node by node equals the assembled step."""
    prob = W.small_nonlinear(nx=7, ny=5, nz=4, steps=0, track_length=0.15e-3, n_tracks=2,
                             hatch=50e-6).replace(degree=deg)
    o = Oracle(prob)
    dt = 2.5e-6 if deg == 2 else 1.0e-5
    T, rc = o.init_T(), o.init_history()
    n0 = 40
    o.explicit_steps(T, rc, 0.0, dt, n0)
    assert T.max() > prob.T_l and np.any((rc > 0) & (rc < 1))
    full = T.copy()
    o.explicit_steps(full, rc.copy(), n0 * dt, dt, 1)
    sampled = o.explicit_step_sampled(T, rc, n0 * dt, dt, np.arange(o.N))
    np.testing.assert_allclose(sampled, full, rtol=0, atol=1e-14 * np.abs(full).max())
    # a subset in arbitrary order gives the same values
    sel = np.random.default_rng(3).permutation(o.N)[:50]
    np.testing.assert_array_equal(o.explicit_step_sampled(T, rc, n0 * dt, dt, sel), sampled[sel])
