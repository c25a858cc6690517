"""The octree schedule (explicit steps on an octree that follows the beam,
remeshed every few steps, then a backward-Euler cool-down with the laser off)
on the GPU against the same schedule run by the octree oracle: leaves from the
seeded input generator on the oracle side and from the library's generator on
the GPU side (equal, pinned on the CPU), the remesh transfer and the steps of
each side's own implementation.  Bars: 1e-12 relative after the explicit phase,
1e-10 after the implicit steps (CG to 1e-10); the history after the explicit
phase to 1e-12."""
import numpy as np
import pytest
import torch

import oracle
import pbf_workloads as W
from tests.gpu_util import need_gpu, rel_errors

pytestmark = pytest.mark.gpu


def _oracle_schedule(p, dt, n_explicit, n_implicit):
    from paper_2302_05164_amd import octree_schedule as S
    t0 = S.time_at_arc_length(p, p.scan_start)

    def mesh(s):
        lo, hi = S.window(p, s)
        return p.replace(leaves=W.octree_leaves(p, hi, lo))

    pm = mesh(p.scan_start)
    O = oracle.OctOracle(pm)
    T, rc = O.init_T(), O.init_history()
    n, remeshes = 0, 0
    while n < n_explicit:
        k = min(p.remesh_every, n_explicit - n)
        O.explicit_steps(T, rc, t0 + n * dt, dt, k)
        n += k
        if n < n_explicit:
            pn = mesh(S.arc_length_at(p, t0 + n * dt))
            On = oracle.OctOracle(pn)
            T, rc = O.transfer(T, rc, On)
            O, pm = On, pn
            remeshes += 1
    t = t0 + n_explicit * dt
    if n_implicit:
        Off = oracle.OctOracle(pm.replace(laser_kind=W.LASER_OFF))  # same leaves: same dof numbering
        for _ in range(n_implicit):
            T, info = Off.implicit_step(T, rc, t, p.implicit_dt)
            assert info["status"] == 0
            t += p.implicit_dt
    return T, rc, O, pm, remeshes


def _to_lib(sim, O, p):
    xl = sim.dof_coords()
    h = p.L[0] / p.nx / 2 ** p.max_level / p.degree
    kl = {tuple(k): i for i, k in enumerate(np.round(xl / h).astype(np.int64))}
    return np.array([kl[tuple(k)] for k in np.round(O.dof_coords() / h).astype(np.int64)])


@pytest.mark.parametrize("ml", [2, 3])
def test_schedule_vs_oracle(ml):
    need_gpu()
    from paper_2302_05164_amd import octree_schedule as S
    p = W.cfg3_reduced(max_level=ml)
    O0 = oracle.OctOracle(p.replace(leaves=S.window_leaves(p, p.scan_start)))
    dt = p.dt_factor * 2.0 / O0.stability_lambda(W.seeded_vector(O0.N, 1), 100)
    # explicit phase alone
    Tg, rg, sim, rec = S.run(p, dt=dt, n_implicit=0)
    To, ro, O, pm, nre = _oracle_schedule(p, dt, p.steps, 0)
    torch.cuda.synchronize()
    assert nre == len(rec["blocks"]) - 1 >= 3
    dofs = [b["dofs"] for b in rec["blocks"]]
    m = _to_lib(sim, O, pm)
    mx, l2 = rel_errors(Tg.cpu().numpy()[m], To)
    print(f"level {ml}: dofs per block {dofs}, T max {To.max():.0f} K, explicit phase max rel {mx:.2e} "
          f"rel-L2 {l2:.2e}")
    assert To.max() > p.T0 + 100.0 and len(set(dofs)) > 1
    assert mx <= 1e-12 and l2 <= 1e-12
    from tests.test_gpu_octree import _hist_map
    oi, li, nh = _hist_map(pm, O)
    assert np.abs(rg.cpu().numpy()[:nh][li] - ro[oi]).max() <= 1e-12
    # with the cool-down
    Tg, rg, sim, rec = S.run(p, dt=dt)
    To, ro, O, pm, _ = _oracle_schedule(p, dt, p.steps, p.implicit_steps)
    torch.cuda.synchronize()
    m = _to_lib(sim, O, pm)
    mx, l2 = rel_errors(Tg.cpu().numpy()[m], To)
    its = [(r["picard"], r["cg"]) for r in rec["implicit"]]
    print(f"level {ml}: after {p.implicit_steps} implicit steps (Picard, CG) {its}: max rel {mx:.2e} rel-L2 {l2:.2e}")
    assert mx <= 1e-10 and l2 <= 1e-10
