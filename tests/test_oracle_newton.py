"""Pins of the oracle's Newton step for the implicit scheme (Section 3.2, eqs.
backward_euler_nonlinear, Newton_1, Newton_2) with restarted GMRES:

- the Jacobian action against central differences of the residual on a smooth
  law (the linear k(T) has no kinks in the range, the capacity, history and
  surface losses are lagged), which fixes the nonsymmetric L term's sign and
  operands;
- Newton and Picard iterations converge to the same root of the residual, the
  Newton one in a handful of iterations;
- with constant coefficients the problem is linear and symmetric: one Newton
  step whose GMRES solution equals the CG solution of the Picard step.
"""
import numpy as np
import pytest

import pbf_workloads as W
from oracle import Oracle


def _smooth_problem(deg):
    p = W.small_nonlinear(nx=5, ny=4, nz=3, steps=0).replace(degree=deg, laser_kind=W.LASER_OFF)
    return p.replace(T_bp=np.array([293.0, 3000.0]), k_bp=np.array([15.0, 45.0]), cp_bp=np.array([500.0, 700.0]),
                     latent=0.0)


def _hot_state(O, p, lo, hi, seed=4):
    rng = np.random.default_rng(seed)
    T = rng.uniform(lo, hi, O.N)
    T[O.dirichlet_mask()] = p.T_D
    return T


@pytest.mark.parametrize("deg", [1, 2])
def test_jacobian_matches_central_differences(deg):
    p = _smooth_problem(deg)
    O = Oracle(p)
    Tn = _hot_state(O, p, 500.0, 2500.0, 1)
    Ti = _hot_state(O, p, 500.0, 2500.0, 2)
    rc = np.random.default_rng(3).uniform(0.0, 1.0, O.NQ)  # partly consolidated
    dt = 1e-3
    x = np.random.default_rng(5).uniform(-1.0, 1.0, O.N)
    x[O.dirichlet_mask()] = 0.0
    Jx = O.jacobian_apply(Tn, Ti, rc, dt, x)
    h = 1e-2
    fd = (O.implicit_residual(Tn, Ti + h * x, rc, 0.0, dt) - O.implicit_residual(Tn, Ti - h * x, rc, 0.0, dt)) / (2 * h)
    err = np.abs(Jx - fd).max() / np.abs(Jx).max()
    # the residual is quadratic in T along x (k linear in T): central differences are exact up to rounding
    assert err <= 1e-9
    # the nonsymmetric term matters: the Picard matrix alone misses it
    Ax = O.picard_apply(Tn, Ti, rc, dt, x)
    assert np.abs(Ax - fd).max() / np.abs(fd).max() > 1e-3
    # and J = A + L with L nonsymmetric: <y, L x> != <x, L y>
    y = np.random.default_rng(6).uniform(-1.0, 1.0, O.N)
    y[O.dirichlet_mask()] = 0.0
    Lx, Ly = Jx - Ax, O.jacobian_apply(Tn, Ti, rc, dt, y) - O.picard_apply(Tn, Ti, rc, dt, y)
    assert abs(y @ Lx - x @ Ly) > 1e-3 * abs(y @ Lx)
    assert abs(y @ Ax - x @ O.picard_apply(Tn, Ti, rc, dt, y)) <= 1e-12 * np.abs(Ax).sum()


def test_newton_and_picard_reach_the_same_root():
    p = W.small_nonlinear(nx=8, ny=7, nz=4, steps=0)
    O = Oracle(p)
    dt_ex = 0.5 * 2.0 / O.stability_lambda(W.seeded_vector(O.N, 1), 60)
    T, rc = O.init_T(), O.init_history()
    O.explicit_steps(T, rc, 0.0, dt_ex, 60)
    assert T.max() > p.T_l
    cool = Oracle(p.replace(laser_kind=W.LASER_OFF))
    t = 60 * dt_ex
    Tp, ip = cool.implicit_step(T, rc.copy(), t, 2e-4, cg_rtol=1e-13, picard_tol=1e-11, picard_max_it=100)
    Tn_, inw = cool.implicit_step_newton(T, rc.copy(), t, 2e-4, lin_rtol=1e-13, restart=30, lin_max_it=20000,
                                         newton_tol=1e-11, newton_max_it=30)
    assert ip["status"] == 0 and inw["status"] == 0
    assert inw["newton_iters"] <= 8 and 3 * inw["newton_iters"] < ip["picard_iters"]
    assert inw["lin_iters"] < ip["cg_iters"]
    assert np.abs(Tp - Tn_).max() <= 1e-8 * np.abs(Tp).max()
    r = cool.implicit_residual(T, Tn_, rc, t, 2e-4)
    Cx = cool.capacity_apply(T, Tn_ - T) / 2e-4
    assert np.abs(r).max() <= 1e-9 * np.abs(Cx).max()


def test_linear_problem_one_newton_step_equals_cg():
    p = W.sine_mode(2, 1).replace(nx=4, ny=3, nz=3, L=(0.3, 0.2, 0.2), dirichlet_mask=W.FACE_ZM)
    O = Oracle(p)
    Tn = p.T_D + 100.0 * (1.0 + W.seeded_vector(O.N, 4))
    Tn[O.dirichlet_mask()] = p.T_D
    rc = O.init_history()
    Tc, ic = O.implicit_step(Tn, rc.copy(), 0.0, 1e3, cg_rtol=1e-14, picard_tol=1e-9)
    Tg, ig = O.implicit_step_newton(Tn, rc.copy(), 0.0, 1e3, lin_rtol=1e-14, restart=20, lin_max_it=5000,
                                    newton_tol=1e-9)
    assert ig["status"] == 0 and ig["newton_iters"] <= 2
    assert np.abs(Tg - Tc).max() <= 1e-10 * np.abs(Tc).max()
