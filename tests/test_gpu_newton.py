"""GPU parity of the implicit step by Newton's method (Section 3.2, eqs.
Newton_1, Newton_2: full Jacobian with the nonsymmetric term, restarted GMRES
with Jacobi on the right) against the oracle's Newton step, plus the agreement
of the Newton and Picard roots on the GPU.  FP64, tolerance 1e-10 on T (the
linear solves stop at a relative residual, so both sides agree to the
Newton tolerance, not to rounding)."""
import numpy as np
import pytest
import torch

import oracle
import pbf_workloads as W
from tests.gpu_util import full_to_history, history_to_full, need_gpu, oracle_dt, rel_errors, sim_for

pytestmark = pytest.mark.gpu


def _hot_state(prob, steps=60):
    o = oracle.Oracle(prob)
    dt_ex = oracle_dt(prob)
    T, rc = o.init_T(), o.init_history()
    o.explicit_steps(T, rc, 0.0, dt_ex, steps)
    return T, rc, steps * dt_ex


def _gpu_newton(prob, T, rc, t, dt, **kw):
    sim = sim_for(prob)
    info = sim.info()
    hist = full_to_history(prob, rc, info["n_hist_layers"])
    rd = torch.tensor(hist if hist.size else np.zeros(1), device="cuda")
    Tg, gi = sim.implicit_step_newton(torch.tensor(T, device="cuda"), rd, t, dt, **kw)
    torch.cuda.synchronize()
    return Tg.cpu().numpy(), gi, history_to_full(prob, rd.cpu().numpy(), info["n_hist_layers"]), sim


@pytest.mark.parametrize("degree,dims", [(2, (20, 18, 10)), (1, (20, 18, 10)), (2, (9, 9, 5))])
def test_newton_step_vs_oracle(degree, dims):
    need_gpu()
    nx, ny, nz = dims
    prob = W.small_nonlinear(nx=nx, ny=ny, nz=nz, steps=0, track_length=0.8 * nx * 31.25e-6).replace(degree=degree)
    T, rc, t = _hot_state(prob)
    assert T.max() > prob.T_l
    cool = prob.replace(laser_kind=W.LASER_OFF)
    kw = dict(lin_rtol=1e-13, restart=30, lin_max_it=20000, newton_tol=1e-10, newton_max_it=30)
    To, oi = oracle.Oracle(cool).implicit_step_newton(T, rc.copy(), t, 2e-4, **kw)
    assert oi["status"] == 0
    Tg, gi, rg, _ = _gpu_newton(cool, T, rc, t, 2e-4, **kw)
    mx, l2 = rel_errors(Tg, To)
    print(f"CHECK Q{degree} {dims} newton: gpu {gi} oracle {oi} max rel {mx:.2e} rel-L2 {l2:.2e}")
    assert mx <= 1e-10 and l2 <= 1e-10
    assert abs(gi["newton_iters"] - oi["newton_iters"]) <= 1
    assert abs(gi["lin_iters"] - oi["lin_iters"]) <= max(3, 0.03 * oi["lin_iters"])
    ro = rc.copy()
    oracle.Oracle(cool).assemble(To, ro, t + 2e-4)  # history commit as in the step
    assert np.abs(rg - ro).max() <= 1e-9


def test_first_newton_iteration_vs_oracle():
    """One Newton iteration only: isolates the first GMRES solve of J dT = -R."""
    need_gpu()
    prob = W.small_nonlinear(nx=12, ny=10, nz=6, steps=0).replace(degree=2)
    T, rc, t = _hot_state(prob, 40)
    cool = prob.replace(laser_kind=W.LASER_OFF)
    kw = dict(lin_rtol=1e-12, restart=20, lin_max_it=20000, newton_tol=1e-12, newton_max_it=1)
    To, oi = oracle.Oracle(cool).implicit_step_newton(T, rc.copy(), t, 1e-3, **kw)
    Tg, gi, _, _ = _gpu_newton(cool, T, rc, t, 1e-3, check=False, **kw)
    mx, l2 = rel_errors(Tg - T, To - T)
    print(f"CHECK first Newton iteration: gpu {gi} oracle {oi} max rel (of the update) {mx:.2e}")
    assert oi["newton_iters"] == gi["newton_iters"] == 1
    assert mx <= 1e-9


def test_newton_and_picard_roots_agree_on_gpu():
    need_gpu()
    prob = W.small_nonlinear(nx=20, ny=18, nz=10, steps=0)
    T, rc, t = _hot_state(prob)
    cool = prob.replace(laser_kind=W.LASER_OFF)
    Tn_, gi, _, sim = _gpu_newton(cool, T, rc, t, 2e-4, lin_rtol=1e-13, newton_tol=1e-11)
    hist = full_to_history(cool, rc, sim.info()["n_hist_layers"])
    rd = torch.tensor(hist if hist.size else np.zeros(1), device="cuda")
    Tp, pi = sim.implicit_step(torch.tensor(T, device="cuda"), rd, t, 2e-4, cg_rtol=1e-13, picard_tol=1e-11,
                               picard_max_it=100)
    d = np.abs(Tp.cpu().numpy() - Tn_).max() / np.abs(Tn_).max()
    print(f"CHECK newton {gi} picard {pi} root difference {d:.2e}")
    assert d <= 1e-10
    assert gi["newton_iters"] * 3 < pi["picard_iters"]


def test_newton_with_source_and_surface_losses_vs_oracle():
    need_gpu()
    prob = W.with_surface_losses(W.small_nonlinear(nx=20, ny=18, nz=10, steps=0, track_length=0.5e-3))
    T, rc, t = _hot_state(prob, 80)
    kw = dict(lin_rtol=1e-13, restart=30, lin_max_it=20000, newton_tol=1e-10, newton_max_it=40)
    To, oi = oracle.Oracle(prob).implicit_step_newton(T, rc.copy(), t, 1e-5, **kw)  # beam on at t + dt
    assert oi["status"] == 0
    Tg, gi, _, _ = _gpu_newton(prob, T, rc, t, 1e-5, **kw)
    mx, l2 = rel_errors(Tg, To)
    print(f"CHECK newton with source and losses: gpu {gi} oracle {oi} max rel {mx:.2e}")
    assert mx <= 1e-10 and l2 <= 1e-10


def test_newton_refused_on_octree():
    need_gpu()
    from paper_2302_05164_amd import pbftherm
    p = W.small_octree(degree=2)
    sim = pbftherm.from_problem(p, device="cuda:0")
    T, rc = sim.init_state(p.T0)
    with pytest.raises(pbftherm.PbfError, match="box mesh"):
        sim.implicit_step_newton(T, rc, 0.0, 1e-4, restart=5)
