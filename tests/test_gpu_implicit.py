"""GPU parity of the implicit backward-Euler step (Picard + matrix-free
Jacobi-PCG) against the oracle and the backward-Euler closed form.

Both sides run the same algorithm (residual, Jacobi diagonal, CG from zero,
Picard update) in double precision with different summation orders, so they
agree to about the CG tolerance times the conditioning; the tests use tight
tolerances (CG 1e-13) and compare to 1e-10 relative."""
import math

import numpy as np
import pytest
import torch

import oracle
import pbf_workloads as W
from tests.gpu_util import full_to_history, history_to_full, need_gpu, oracle_dt, rel_errors, sim_for

pytestmark = pytest.mark.gpu


def _sine_field(deg, n):
    x = np.linspace(0.0, 1.0, deg * n + 1)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return (np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)).ravel()


def test_backward_euler_sine_mode_q1_closed_form():
    need_gpu()
    n, k, rho, cp = 6, 20.0, 7900.0, 500.0
    alpha = k / (rho * cp)
    prob = W.sine_mode(1, n, k=k, rho=rho, cp=cp)
    sim = sim_for(prob)
    h = 1.0 / n
    a = 2.0 / h ** 2 * (1.0 - math.cos(math.pi * h))
    b = (2.0 + math.cos(math.pi * h)) / 3.0
    lam = 3.0 * a / b
    dt = 50.0 * 2.0 / (alpha * 4.0 / h ** 2)
    s = _sine_field(1, n)
    A = 120.0
    T = torch.tensor(prob.T_D + A * s, device="cuda")
    rc = torch.zeros(1, device="cuda", dtype=torch.float64)
    for step in range(3):
        T, info = sim.implicit_step(T, rc, step * dt, dt, cg_rtol=1e-14, picard_tol=1e-10)
    torch.cuda.synchronize()
    np.testing.assert_allclose(T.cpu().numpy(), prob.T_D + A * s * (1.0 + dt * alpha * lam) ** -3,
                               rtol=0, atol=1e-11 * A)


def _compare(prob, Tn, rc_full, t, dt, cg_rtol=1e-13, picard_tol=1e-10, tol=1e-10):
    sim = sim_for(prob)
    info = sim.info()
    hist = full_to_history(prob, rc_full, info["n_hist_layers"])
    Td = torch.tensor(Tn, device="cuda")
    rd = torch.tensor(hist if hist.size else np.zeros(1), device="cuda")
    Tg, gi = sim.implicit_step(Td, rd, t, dt, cg_rtol=cg_rtol, picard_tol=picard_tol, picard_max_it=60)
    torch.cuda.synchronize()
    o = oracle.Oracle(prob)
    ro = rc_full.copy()
    To, oi = o.implicit_step(Tn, ro, t, dt, cg_rtol=cg_rtol, picard_tol=picard_tol, picard_max_it=60)
    assert oi["status"] == 0
    mx, l2 = rel_errors(Tg.cpu().numpy(), To)
    print(f"{prob.name}: gpu {gi} oracle {oi} max rel {mx:.2e} rel-L2 {l2:.2e}")
    assert mx <= tol and l2 <= tol
    assert abs(gi["picard_iters"] - oi["picard_iters"]) <= 1
    assert abs(gi["cg_iters"] - oi["cg_iters"]) <= max(2, 0.02 * oi["cg_iters"])
    rg = history_to_full(prob, rd.cpu().numpy(), info["n_hist_layers"])
    np.testing.assert_array_equal(rg > 0, ro > 0)
    assert np.abs(rg - ro).max() <= 1e-9
    return Tg, To


@pytest.mark.parametrize("dims", [(3, 2, 2), (17, 6, 5)])
def test_constant_coefficient_q2_vs_oracle(dims):
    need_gpu()
    p = W.sine_mode(2, 1)
    prob = p.replace(nx=dims[0], ny=dims[1], nz=dims[2], L=(0.3, 0.2, 0.2), dirichlet_mask=W.FACE_ZM)
    o = oracle.Oracle(prob)
    Tn = prob.T_D + 100.0 * (1.0 + W.seeded_vector(o.N, 4))
    Tn[o.dirichlet_mask()] = prob.T_D
    _compare(prob, Tn, o.init_history(), 0.0, 1e3)


@pytest.mark.parametrize("degree", [1, 2])
def test_nonlinear_cooldown_step_vs_oracle(degree):
    """Hot state with a melt pool and partly consolidated powder (after explicit
    steps of the oracle), then one implicit cool-down step with the laser off."""
    need_gpu()
    prob = W.small_nonlinear(nx=20, ny=18, nz=10, steps=0).replace(degree=degree)
    o = oracle.Oracle(prob)
    dt_ex = oracle_dt(prob)
    T = o.init_T()
    rc = o.init_history()
    o.explicit_steps(T, rc, 0.0, dt_ex, 60)
    assert T.max() > prob.T_l
    cool = prob.replace(laser_kind=W.LASER_OFF)
    _compare(cool, T, rc, 60 * dt_ex, 1e-4)


def test_implicit_step_with_source_vs_oracle():
    """Laser on during the implicit step (source at t + dt)."""
    need_gpu()
    prob = W.small_nonlinear(nx=12, ny=10, nz=6, steps=0)
    o = oracle.Oracle(prob)
    T = o.init_T()
    _compare(prob, T, o.init_history(), 0.0, 2e-5)


def test_cg_nonconvergence_reported():
    need_gpu()
    from paper_2302_05164_amd import pbftherm
    prob = W.small_nonlinear(nx=12, ny=10, nz=6, steps=0)
    sim = sim_for(prob)
    T, rc = sim.init_state(prob.T0)
    Tout, info = sim.implicit_step(T, rc, 0.0, 2e-5, cg_rtol=1e-14, cg_max_it=2, check=False)
    assert info["status"] == -5 and info["cg_iters"] >= 2
    with pytest.raises(pbftherm.PbfError):
        sim.implicit_step(T, rc, 0.0, 2e-5, cg_rtol=1e-14, cg_max_it=2)
