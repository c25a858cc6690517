"""The multigrid preconditioner of the implicit steps (geometric V-cycle with
Chebyshev smoothing on boxes) against the oracle's implicit steps (plain
Jacobi-CG Picard and Jacobi-GMRES Newton): the preconditioner changes the
iteration, not the root, so both sides agree to the solver tolerance (1e-10
on T), and the Krylov iteration counts fall well below the Jacobi ones."""
import numpy as np
import pytest
import torch

import oracle
import pbf_workloads as W
from tests.gpu_util import full_to_history, history_to_full, need_gpu, oracle_dt, rel_errors, sim_for

pytestmark = pytest.mark.gpu


def _hot(prob, steps=60):
    o = oracle.Oracle(prob)
    dt_ex = oracle_dt(prob)
    T, rc = o.init_T(), o.init_history()
    o.explicit_steps(T, rc, 0.0, dt_ex, steps)
    return T, rc, steps * dt_ex


def _gpu(prob, T, rc, t, dt, newton=False, kind="multigrid", forcing="fixed", **kw):
    sim = sim_for(prob)
    sim.set_preconditioner(kind)
    sim.set_newton_forcing(forcing)
    info = sim.info()
    hist = full_to_history(prob, rc, info["n_hist_layers"])
    rd = torch.tensor(hist if hist.size else np.zeros(1), device="cuda")
    Td = torch.tensor(T, device="cuda")
    if newton:
        Tg, gi = sim.implicit_step_newton(Td, rd, t, dt, **kw)
    else:
        Tg, gi = sim.implicit_step(Td, rd, t, dt, **kw)
    torch.cuda.synchronize()
    return Tg.cpu().numpy(), gi, history_to_full(prob, rd.cpu().numpy(), info["n_hist_layers"])


@pytest.mark.parametrize("degree,dims,dt", [(2, (24, 24, 12), 1e-4), (2, (20, 18, 9), 2e-4), (1, (32, 24, 16), 1e-3)])
def test_multigrid_picard_cg_vs_oracle(degree, dims, dt):
    need_gpu()
    nx, ny, nz = dims
    prob = W.small_nonlinear(nx=nx, ny=ny, nz=nz, steps=0, track_length=0.5 * nx * 31.25e-6).replace(degree=degree)
    T, rc, t = _hot(prob)
    assert T.max() > prob.T_l
    cool = prob.replace(laser_kind=W.LASER_OFF)
    kw = dict(cg_rtol=1e-12, picard_tol=1e-9, picard_max_it=60)
    To, oi = oracle.Oracle(cool).implicit_step(T, rc.copy(), t, dt, **kw)
    assert oi["status"] == 0
    Tg, gi, rg = _gpu(cool, T, rc, t, dt, **kw)
    Tj, gj, _ = _gpu(cool, T, rc, t, dt, kind="jacobi", **kw)
    mx, l2 = rel_errors(Tg, To)
    print(f"Q{degree} {dims} dt {dt:g}: multigrid {gi} jacobi {gj} oracle {oi} max rel {mx:.2e} rel-L2 {l2:.2e}")
    assert mx <= 1e-10 and l2 <= 1e-10
    assert abs(gi["picard_iters"] - oi["picard_iters"]) <= 1
    assert gi["cg_iters"] * 2 <= gj["cg_iters"]
    ro = rc.copy()
    oracle.Oracle(cool).assemble(To, ro, t + dt)  # history commit as in the step
    assert np.abs(rg - ro).max() <= 1e-9


@pytest.mark.parametrize("degree,dims", [(2, (16, 16, 8)), (2, (20, 18, 10))])
def test_multigrid_newton_gmres_vs_oracle(degree, dims):
    need_gpu()
    nx, ny, nz = dims
    prob = W.small_nonlinear(nx=nx, ny=ny, nz=nz, steps=0, track_length=0.5 * nx * 31.25e-6).replace(degree=degree)
    T, rc, t = _hot(prob)
    cool = prob.replace(laser_kind=W.LASER_OFF)
    kw = dict(lin_rtol=1e-12, restart=30, lin_max_it=20000, newton_tol=1e-9, newton_max_it=30)
    To, oi = oracle.Oracle(cool).implicit_step_newton(T, rc.copy(), t, 2e-4, **kw)
    assert oi["status"] == 0
    Tg, gi, _ = _gpu(cool, T, rc, t, 2e-4, newton=True, **kw)
    Tj, gj, _ = _gpu(cool, T, rc, t, 2e-4, newton=True, kind="jacobi", **kw)
    mx, l2 = rel_errors(Tg, To)
    print(f"Q{degree} {dims} newton: multigrid {gi} jacobi {gj} oracle {oi} max rel {mx:.2e} rel-L2 {l2:.2e}")
    assert mx <= 1e-10 and l2 <= 1e-10
    assert abs(gi["newton_iters"] - oi["newton_iters"]) <= 1
    assert gi["lin_iters"] * 2 <= gj["lin_iters"]


@pytest.mark.parametrize("degree,dims", [(2, (16, 16, 8)), (2, (20, 18, 10))])
def test_eisenstat_walker_newton_same_root(degree, dims):
    """Inexact Newton (loose early linear solves, Eisenstat-Walker forcing) converges
    to the same root as the oracle's Newton with every system solved to lin_rtol,
    in fewer Krylov iterations than the fixed forcing."""
    need_gpu()
    nx, ny, nz = dims
    prob = W.small_nonlinear(nx=nx, ny=ny, nz=nz, steps=0, track_length=0.5 * nx * 31.25e-6).replace(degree=degree)
    T, rc, t = _hot(prob)
    cool = prob.replace(laser_kind=W.LASER_OFF)
    kw = dict(lin_rtol=1e-12, restart=30, lin_max_it=20000, newton_tol=1e-9, newton_max_it=40)
    To, oi = oracle.Oracle(cool).implicit_step_newton(T, rc.copy(), t, 2e-4, **kw)
    assert oi["status"] == 0
    Tg, gi, _ = _gpu(cool, T, rc, t, 2e-4, newton=True, forcing="eisenstat-walker", **kw)
    Tf, gf, _ = _gpu(cool, T, rc, t, 2e-4, newton=True, **kw)
    mx, l2 = rel_errors(Tg, To)
    print(f"Q{degree} {dims} newton EW: {gi} fixed {gf} oracle {oi} max rel {mx:.2e} rel-L2 {l2:.2e}")
    assert mx <= 1e-10 and l2 <= 1e-10
    assert gi["lin_iters"] < gf["lin_iters"]


def test_multigrid_refused_where_unsupported():
    need_gpu()
    from paper_2302_05164_amd import pbftherm
    p = W.small_octree()
    sim = sim_for(p)
    with pytest.raises(pbftherm.PbfError, match="box"):
        sim.set_preconditioner("multigrid")
