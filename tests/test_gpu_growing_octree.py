"""A growing build on an octree (Section 4.1, mesh adaptivity and layer
activation) on the GPU against the oracle: per layer, explicit steps of one
scan track, then the activation of the next layer with the library's
adaptation (refine the new layer and the HAZ, coarsen octets with r_c > 0.9
farther than d_HAZ = 4 layers, 2:1 balance) and transfer.  The oracle runs the
same schedule with its own adaptation (oracle/layers.py) and transfer.  Bars:
identical leaves after every activation, T to 1e-12 relative, the history to
1e-10 (a derived quantity: r = max(r, g) with g = (T - T_s)/(T_l - T_s)
turns a temperature difference into a history difference 1/(T_l - T_s) =
1/60 K^-1 larger, and the melt pool reaches 6000 K, so the T bar of 1e-12
relative allows 1e-10 in r)."""
import numpy as np
import pytest
import torch

import oracle
import pbf_workloads as W
from oracle import layers as LY
from tests.gpu_util import need_gpu, rel_errors

pytestmark = pytest.mark.gpu


def _to_lib(sim, O, p):
    xl = sim.dof_coords()
    h = p.L[0] / p.nx / 2 ** p.max_level / p.degree
    kl = {tuple(k): i for i, k in enumerate(np.round(xl / h).astype(np.int64))}
    return np.array([kl[tuple(k)] for k in np.round(O.dof_coords() / h).astype(np.int64)])


def test_growing_octree_build_vs_oracle():
    need_gpu()
    from paper_2302_05164_amd import pbftherm
    p = W.growing_octree_build()
    ml, n0, d_haz = p.max_level, (p.nx, p.ny), 4
    top = 1 << ml  # one coarse layer of substrate
    lv = LY.initial_leaves(n0, ml, top, d_haz)
    sim = pbftherm.from_problem(p, leaves=lv, top=top)
    O = oracle.OctOracle(p.replace(leaves=lv), top=top)
    dt = p.dt_factor * 2.0 / O.stability_lambda(W.seeded_vector(O.N, 1), 100)
    T, rc = sim.init_state(p.T0)
    To, ro = O.init_T(), O.init_history()
    nq = (p.degree + 1) ** 3
    track_t0 = np.concatenate([[0.0], np.cumsum(np.linalg.norm(p.tracks[:, 3:6] - p.tracks[:, 0:3], axis=1)
                                                / p.tracks[:, 6])])
    coarsened = 0
    for layer in range(len(p.tracks)):
        t0 = track_t0[layer]
        sim.explicit_steps(T, rc, t0, dt, p.steps)
        O.explicit_steps(To, ro, t0, dt, p.steps)
        torch.cuda.synchronize()
        m = _to_lib(sim, O, p.replace(leaves=lv))
        mx, l2 = rel_errors(T.cpu().numpy()[m], To)
        nh = len(lv)
        rg = rc.cpu().numpy()[:nq * nh].reshape(nq, nh).T.reshape(-1)  # point-major -> leaf-major
        print(f"layer {layer}: top {top}, leaves {len(lv)}, dofs {O.N}, T max {To.max():.0f} K, "
              f"max rel {mx:.2e}, history {np.abs(rg - ro).max():.1e}")
        assert mx <= 1e-12 and l2 <= 1e-12
        assert np.abs(rg - ro).max() <= 1e-10
        # activate the next layer: adaptation and transfer on both sides
        rmin_g = sim.history_min(rc)
        rmin_o = LY.rc_min_per_leaf(ro, len(lv), nq)
        assert np.abs(rmin_g - rmin_o).max() <= 1e-12
        new_g = sim.layer_leaves(rmin_g, top + 1, d_haz, 0.9)
        new_o = LY.adapt(lv, rmin_o, ml, n0, top, top + 1, d_haz, 0.9)
        assert np.array_equal(new_g, new_o)
        coarsened += int((new_o[:, 0] < ml).sum() > (np.asarray(lv)[:, 0] < ml).sum())
        T, rc = sim.grow(new_g, top + 1, T, rc)
        On = oracle.OctOracle(p.replace(leaves=new_o), top=top + 1)
        To, ro = O.transfer_growing(To, ro, On, p.T0)
        O, lv, top = On, new_o, top + 1
        torch.cuda.synchronize()
        m = _to_lib(sim, O, p.replace(leaves=lv))
        mx, _ = rel_errors(T.cpu().numpy()[m], To)
        assert mx <= 1e-12
        x = O.dof_coords()
        assert np.all(To[x[:, 2] > (top - 1) * p.L[2] / p.nz / 2 ** ml + 1e-12] == p.T0)  # activated at T0
    assert coarsened >= 1  # octets far below the current layer were coarsened
