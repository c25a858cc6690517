"""Pins of the oracle's layer activation (Section 4.1; initial condition of
Section 2, eq. consolidated_fraction): new nodes start at T0, new Gauss points
within the powder depth of the new top start as powder, older cells keep their
history, and the activated layer couples conservatively to the old part (the
diffusion rows of the grown box still sum to zero)."""
import numpy as np
import pytest

import pbf_workloads as W
from oracle import Oracle


def _box(deg=2):
    return W.small_nonlinear(nx=6, ny=5, nz=6, steps=0).replace(degree=deg)


@pytest.mark.parametrize("deg", [1, 2])
def test_activation_sets_new_nodes_and_powder(deg):
    p = _box(deg)
    O = Oracle(p)
    NX, NY, NZ = p.nodes_per_dim
    T = np.full(O.N, 1234.0)
    rc = np.full(O.NQ, 0.5)
    O.activate_layers(4, 6, 293.0, T, rc)
    planes = T.reshape(NZ, NY, NX)
    assert np.all(planes[: deg * 4 + 1] == 1234.0) and np.all(planes[deg * 4 + 1:] == 293.0)
    nq = (deg + 1) ** 3
    r = rc.reshape(p.nz, p.ny, p.nx, nq)
    assert np.all(r[:4] == 0.5)  # older cells keep their history
    hz = p.L[2] / p.nz
    xg = np.polynomial.legendre.leggauss(deg + 1)[0] * 0.5 + 0.5
    for cz in (4, 5):
        for q in range(nq):
            z = (cz + xg[q // (deg + 1) ** 2]) * hz
            expect = 0.0 if 6 * hz - z <= p.powder_depth else 1.0
            assert np.all(r[cz, :, :, q] == expect)
    # the new top holds powder, the layer below the powder depth is solid
    assert r[5].min() == 0.0 and (hz < p.powder_depth or r[4].max() == 1.0)


def test_grown_box_couples_conservatively():
    """Hot old part, cold new layer, laser off, no Dirichlet face: the first step's
    stored-energy change is zero (heat only moves into the new layer)."""
    p = _box(2).replace(laser_kind=W.LASER_OFF, dirichlet_mask=0)
    full = Oracle(p)
    T = np.zeros(full.N)
    rc = np.ones(full.NQ)
    act = Oracle(W.active_part(p, 4))
    rng = np.random.default_rng(2)
    T[: act.N] = rng.uniform(800.0, 1500.0, act.N)
    full.activate_layers(4, 6, 293.0, T, rc)
    grown = Oracle(W.active_part(p, 6))
    f, Cl, _ = grown.assemble(T, rc.copy(), 0.0)
    assert abs(f.sum()) <= 1e-10 * np.abs(f).sum()
    NX, NY, NZ = p.nodes_per_dim
    new = np.zeros(full.N, dtype=bool).reshape(NZ, NY, NX)
    new[2 * 4 + 1:] = True
    assert f[new.reshape(-1)].sum() > 0  # heat flows into the activated layer
