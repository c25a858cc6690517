"""Pins of the CPU oracle against what mathematics and the paper fix.

Each test checks the oracle against something other than itself: closed-form
quadrature rules, exact 1D element matrices (Kronecker assembly), the discrete
eigenmode of the heat operator, the explicit stability limit (closed form and
dense eigensolver), the critical step the paper prints for its bridge example,
energy conservation, the Gaussian source normalization, and hand-computed
values of the material law.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sl

import pbf_workloads as W
from oracle import Oracle, gauss_legendre, lagrange, lagrange_deriv
from tests.fem1d import global_1d, global_3d
from tests.sine_modes import q1_explicit, q2_explicit, sine_field

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# reference element
# --------------------------------------------------------------------------
def test_gauss_rules_closed_form_and_exactness():
    x, w = gauss_legendre(2)
    np.testing.assert_allclose(x, [0.5 - 0.5 / math.sqrt(3), 0.5 + 0.5 / math.sqrt(3)], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [0.5, 0.5], atol=1e-15)
    x, w = gauss_legendre(3)
    np.testing.assert_allclose(x, [0.5 - math.sqrt(15) / 10, 0.5, 0.5 + math.sqrt(15) / 10], atol=1e-15)
    np.testing.assert_allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-15)
    for n in (1, 2, 3, 4):
        x, w = gauss_legendre(n)
        for k in range(2 * n):
            assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) < 1e-14
        # not exact one degree higher
        assert abs(np.dot(w, x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-6


@pytest.mark.parametrize("p", [1, 2, 3])
def test_lagrange_basis(p):
    nodes = [a / p for a in range(p + 1)]
    for a in range(p + 1):
        for b in range(p + 1):
            assert abs(lagrange(p, a, nodes[b]) - (1.0 if a == b else 0.0)) < 1e-14
    for x in np.linspace(0, 1, 7):
        assert abs(sum(lagrange(p, a, x) for a in range(p + 1)) - 1.0) < 1e-14
        # derivatives reproduce d/dx x^m for m <= p
        for m in range(p + 1):
            d = sum(lagrange_deriv(p, a, x) * nodes[a] ** m for a in range(p + 1))
            exact = m * x ** (m - 1) if m > 0 else 0.0
            assert abs(d - exact) < 1e-12


# --------------------------------------------------------------------------
# operator = assembled matrix (Section 4.2 remark: apply to unit vectors)
# --------------------------------------------------------------------------
def _const_problem(deg, nx, ny, nz, L, mask=0, k=20.0, rho=7900.0, cp=500.0):
    p = W.sine_mode(deg, 1, k=k, rho=rho, cp=cp)
    return p.replace(nx=nx, ny=ny, nz=nz, L=L, dirichlet_mask=mask)


@pytest.mark.parametrize("deg", [1, 2])
def test_matrix_free_equals_kronecker_assembly(deg):
    L = (0.3, 0.5, 0.4)
    nx, ny, nz = 2, 3, 2
    k, rho, cp = 17.0, 7000.0, 600.0
    prob = _const_problem(deg, nx, ny, nz, L, k=k, rho=rho, cp=cp)
    o = Oracle(prob)
    K3, M3 = global_3d(deg, nx, ny, nz, L)
    N = o.N
    assert K3.shape == (N, N)
    rc = o.init_history()
    cols = np.zeros((N, N))
    Cl = None
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        f, Cl, fv = o.assemble(e, rc.copy(), 0.0)
        cols[:, j] = -f
    np.testing.assert_allclose(cols, k * K3, rtol=0, atol=1e-11 * np.abs(k * K3).max())
    # lumped capacity = row sums of the consistent capacity matrix
    np.testing.assert_allclose(Cl, rho * cp * M3.sum(axis=1), rtol=1e-13)
    # partition of unity: total capacity = rho c |Omega|
    assert abs(Cl.sum() - rho * cp * L[0] * L[1] * L[2]) < 1e-12 * rho * cp
    # consistent capacity apply
    x = W.seeded_vector(N, 3)
    y = o.capacity_apply(np.full(N, 300.0), x)
    np.testing.assert_allclose(y, rho * cp * M3 @ x, rtol=0, atol=1e-12 * np.abs(rho * cp * M3).sum())


def test_operator_symmetric_and_annihilates_constants_nonlinear():
    """For any state, sum_i f_diff,i = 0 (the gradients of the shape functions sum
    to zero), and the Jacobian-free diffusion part K(T) is symmetric in its
    argument when k is frozen."""
    prob = W.small_nonlinear(nx=4, ny=3, nz=3, steps=0)
    prob = prob.replace(laser_kind=W.LASER_OFF)
    o = Oracle(prob)
    rng = np.random.default_rng(0)
    T = 293.0 + 2500.0 * rng.random(o.N)
    rc = o.init_history()
    f, Cl, fv = o.assemble(T, rc, 0.0)
    assert abs(f.sum()) < 1e-12 * np.abs(f).sum()
    assert np.all(fv == 0.0)


# --------------------------------------------------------------------------
# decaying eigenmode sin(pi x) sin(pi y) sin(pi z)
# --------------------------------------------------------------------------
_sine_field = sine_field


@pytest.mark.parametrize("n", [5, 8])
def test_sine_mode_q1_discrete_closed_form(n):
    """Q1, uniform h: the nodal sine is an eigenvector of C~^{-1}K with eigenvalue
    alpha * 3 a b^2, a = 2(1-cos(pi h))/h^2, b = (2+cos(pi h))/3, so forward Euler
    multiplies it by (1 - dt alpha lambda) per step (eq. forward_euler)."""
    k, rho, cp = 20.0, 7900.0, 500.0
    prob = W.sine_mode(1, n, k=k, rho=rho, cp=cp)
    o = Oracle(prob)
    alpha = k / (rho * cp)
    h = 1.0 / n
    dt = 0.4 * 2.0 / (alpha * 4.0 / h ** 2)
    A = 150.0
    T = prob.T_D + A * _sine_field(1, n)
    rc = o.init_history()
    nsteps = 7
    o.explicit_steps(T, rc, 0.0, dt, nsteps)
    expect = prob.T_D + A * q1_explicit(n, alpha, dt, nsteps)
    np.testing.assert_allclose(T, expect, rtol=0, atol=1e-12 * A)


@pytest.mark.parametrize("n", [4, 6])
def test_sine_mode_q2_invariant_subspace(n):
    """Q2: the sine sampled at vertices and at edge midpoints spans a 2D subspace
    invariant under the 1D operators C~^{-1}K and C~^{-1}M (found from the exact
    1D matrices); in 3D the evolution is an 8x8 matrix power, exact to round-off."""
    k, rho, cp = 20.0, 7900.0, 500.0
    alpha = k / (rho * cp)
    prob = W.sine_mode(2, n, k=k, rho=rho, cp=cp)
    o = Oracle(prob)
    h = 1.0 / n
    dt = 0.4 * 2.0 / (alpha * 36.0 / h ** 2)
    nsteps = 6
    A0 = 80.0
    T = prob.T_D + A0 * _sine_field(2, n)
    rc = o.init_history()
    o.explicit_steps(T, rc, 0.0, dt, nsteps)
    np.testing.assert_allclose(T, prob.T_D + A0 * q2_explicit(n, alpha, dt, nsteps), rtol=0, atol=1e-11 * A0)


@pytest.mark.parametrize("deg", [1, 2])
def test_sine_mode_converges_to_continuous_decay(deg):
    """As h, dt -> 0 the discrete decay tends to exp(-3 alpha pi^2 t)."""
    k, rho, cp = 20.0, 7900.0, 500.0
    alpha = k / (rho * cp)
    t_end = 0.02 / alpha / (3 * math.pi ** 2)  # decay of about 2%
    errs = []
    for n in (4, 8, 16):
        prob = W.sine_mode(deg, n, k=k, rho=rho, cp=cp)
        o = Oracle(prob)
        h = 1.0 / n
        lam_max = (4.0 if deg == 1 else 36.0) / h ** 2
        nsteps = max(4, int(math.ceil(t_end / (0.5 * 2.0 / (alpha * lam_max)))))
        dt = t_end / nsteps
        T = prob.T_D + _sine_field(deg, n)
        rc = o.init_history()
        o.explicit_steps(T, rc, 0.0, dt, nsteps)
        mid = (deg * n + 1) ** 3 // 2
        errs.append(abs((T[mid] - prob.T_D) - math.exp(-3 * alpha * math.pi ** 2 * t_end)))
    # second order in h (dt is refined with h^2): each halving cuts the error ~4x
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3
    assert errs[2] < (5e-4 if deg == 1 else 1e-4)


# --------------------------------------------------------------------------
# explicit stability limit (eq. explicit_time_step)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("deg,closed", [(1, 4.0), (2, 36.0)])
def test_stability_lambda_closed_form_neumann(deg, closed):
    n = 4
    k, rho, cp = 20.0, 7900.0, 500.0
    prob = _const_problem(deg, n, n, n, (1.0, 1.0, 1.0), mask=0, k=k, rho=rho, cp=cp)
    o = Oracle(prob)
    alpha = k / (rho * cp)
    h = 1.0 / n
    lam = o.stability_lambda(W.seeded_vector(o.N, 11), 4000)
    K3, M3 = global_3d(deg, n, n, n, (1.0, 1.0, 1.0))
    dense = sl.eigh(K3, np.diag(M3.sum(1)), eigvals_only=True).max() * alpha
    assert abs(dense - closed * alpha / h ** 2) < 1e-9 * dense
    assert lam <= dense * (1 + 1e-12)
    assert abs(lam - dense) < 2e-3 * dense


def test_stability_lambda_dirichlet_matches_dense():
    prob = _const_problem(2, 3, 3, 2, (0.3, 0.3, 0.2), mask=W.FACE_ZM)
    o = Oracle(prob)
    K3, M3 = global_3d(2, 3, 3, 2, (0.3, 0.3, 0.2))
    free = ~o.dirichlet_mask()
    Kf = K3[np.ix_(free, free)]
    Mf = np.diag(M3.sum(1)[free])
    alpha = prob.k_bp[0] / (prob.rho * prob.cp_bp[0])
    dense = sl.eigh(Kf, Mf, eigvals_only=True).max() * alpha
    lam = o.stability_lambda(W.seeded_vector(o.N, 5), 3000)
    assert abs(lam - dense) < 1e-3 * dense


def test_stability_uses_critical_breakpoint():
    """The critical parameters are those of the breakpoint with the largest k/c_p."""
    prob = W.small_nonlinear(nx=3, ny=3, nz=2, steps=0)
    o = Oracle(prob)
    ratio = prob.k_bp / prob.cp_bp
    i = int(np.argmax(ratio))
    const = _const_problem(2, 3, 3, 2, prob.L, mask=prob.dirichlet_mask, k=prob.k_bp[i],
                           rho=prob.rho, cp=prob.cp_bp[i])
    oc = Oracle(const)
    v0 = W.seeded_vector(o.N, 2)
    assert abs(o.stability_lambda(v0, 300) - oc.stability_lambda(v0, 300)) < 1e-12 * oc.stability_lambda(v0, 300)


def test_bridge_critical_time_step_pin():
    g = json.load(open(os.path.join(GOLD, "bridge_critical_dt.json")))
    h = g["h"]
    n = 6
    prob = _const_problem(g["degree"], n, n, n, (n * h, n * h, n * h), mask=0, k=g["k"],
                          rho=g["rho"], cp=g["c"])
    o = Oracle(prob)
    lam = o.stability_lambda(W.seeded_vector(o.N, 7), 3000)
    dt_crit = 2.0 / lam
    assert float(f"{dt_crit:.{g['printed_digits']}g}") == g["dt_crit_printed"]


def test_explicit_growth_above_and_decay_below_limit():
    prob = _const_problem(1, 4, 4, 4, (1.0, 1.0, 1.0), mask=W.FACE_ZM)
    o = Oracle(prob)
    K3, M3 = global_3d(1, 4, 4, 4, (1.0, 1.0, 1.0))
    free = ~o.dirichlet_mask()
    alpha = prob.k_bp[0] / (prob.rho * prob.cp_bp[0])
    lam = sl.eigh(K3[np.ix_(free, free)], np.diag(M3.sum(1)[free]), eigvals_only=True).max() * alpha
    dt_crit = 2.0 / lam
    out = {}
    for fac in (0.99, 1.01):
        T = prob.T_D + W.seeded_vector(o.N, 9)
        T[~free] = prob.T_D
        rc = o.init_history()
        o.explicit_steps(T, rc, 0.0, fac * dt_crit, 800)
        out[fac] = np.abs(T - prob.T_D).max()
    assert out[0.99] < 1.0
    assert out[1.01] > 100.0


# --------------------------------------------------------------------------
# energy and source normalization
# --------------------------------------------------------------------------
def test_source_integrates_to_effective_power():
    """eq. heat_soruce_cylindrical integrates to W_eff over the layer when the beam
    is resolved and inside the domain."""
    R = 50e-6
    h = 5e-6
    n = 60
    prob = W.small_nonlinear(nx=n, ny=n, nz=8, h=h, steps=0)
    tr = np.array([[0.5 * n * h, 0.5 * n * h, 8 * h, 0.5 * n * h + 1e-6, 0.5 * n * h, 8 * h, 0.8, 150.0]])
    prob = prob.replace(tracks=tr, h_powder=40e-6)
    o = Oracle(prob)
    T = o.init_T()
    rc = o.init_history()
    f, Cl, fv = o.assemble(T, rc, 0.0)
    Weff = prob.absorptivity * 150.0
    assert abs(fv.sum() - Weff) < 2e-3 * Weff
    # f_diff sums to zero, so the total right-hand side is the absorbed power
    assert abs(f.sum() - fv.sum()) < 1e-9 * Weff


def test_adiabatic_energy_balance_exact():
    """Insulated box, constant c: sum_i C~_i (T_N - T_0)_i equals the absorbed
    energy sum_n dt sum_i f_vol,i to round-off (Sections 2 and 3.2)."""
    prob = W.small_nonlinear(nx=6, ny=5, nz=4, steps=0, h=20e-6)
    prob = prob.replace(dirichlet_mask=0, T_bp=np.array([0.0, 1e4]), k_bp=np.array([20.0, 20.0]),
                        cp_bp=np.array([500.0, 500.0]), latent=0.0, powder_k_factor=1.0,
                        powder_depth=0.0)
    o = Oracle(prob)
    T = o.init_T()
    T0 = T.copy()
    rc = o.init_history()
    dt = 2e-7
    absorbed = 0.0
    for n in range(40):
        f, Cl, fv = o.assemble(T, rc.copy(), n * dt)
        absorbed += dt * fv.sum()
        o.explicit_steps(T, rc, n * dt, dt, 1)
    stored = np.dot(Cl, T - T0)
    assert absorbed > 0
    assert abs(stored - absorbed) < 1e-10 * absorbed


def test_surface_flux_integrates_to_effective_power():
    prob = W.cfg1()
    h = 5e-6
    n = 60
    tr = np.array([[0.5 * n * h, 0.5 * n * h, 4 * h, 0.5 * n * h + 1e-6, 0.5 * n * h, 4 * h, 0.8, 200.0]])
    prob = prob.replace(nx=n, ny=n, nz=4, L=(n * h, n * h, 4 * h), tracks=tr)
    o = Oracle(prob)
    f, Cl, fv = o.assemble(o.init_T(), o.init_history(), 0.0)
    Weff = 0.35 * 200.0
    assert abs(fv.sum() - Weff) < 2e-3 * Weff


# --------------------------------------------------------------------------
# material law, laser path and history
# --------------------------------------------------------------------------
def _law(T_bp, k_bp, cp_bp, **kw):
    p = W.small_nonlinear(nx=1, ny=1, nz=1, steps=0)
    return Oracle(p.replace(T_bp=np.array(T_bp), k_bp=np.array(k_bp), cp_bp=np.array(cp_bp), **kw))


def test_material_law_hand_values():
    o = _law([300.0, 500.0, 2000.0], [10.0, 30.0, 40.0], [400.0, 600.0, 800.0],
             T_s=1500.0, T_l=1600.0, latent=2.0e5, powder_k_factor=0.01)
    # eq. liquid_fraction
    assert o.liquid_fraction(1499.0) == 0.0
    assert o.liquid_fraction(1500.0) == 0.0
    assert abs(o.liquid_fraction(1550.0) - 0.5) < 1e-15
    assert o.liquid_fraction(1600.0) == 1.0
    assert o.liquid_fraction(1700.0) == 1.0
    # consolidated material: k = k(T); table interpolation and constant extrapolation
    assert abs(o.conductivity(400.0, 1.0) - 20.0) < 1e-13
    assert abs(o.conductivity(250.0, 1.0) - 10.0) < 1e-13
    assert abs(o.conductivity(2500.0, 1.0) - 40.0) < 1e-13
    assert abs(o.conductivity(1250.0, 1.0) - 35.0) < 1e-13
    # powder (r_c = 0) below solidus: k = 0.01 k(T)
    assert abs(o.conductivity(400.0, 0.0) - 0.2) < 1e-15
    # half-consolidated, half-melted at 1550: r_p = 0.5 (powder), r_m = 0.5, r_s = 0
    kT = 30.0 + (1550.0 - 500.0) * 10.0 / 1500.0
    assert abs(o.conductivity(1550.0, 0.5) - (0.5 * 0.01 * kT + 0.5 * kT)) < 1e-12
    # apparent capacity: latent heat spread over [T_s, T_l]
    assert abs(o.capacity(400.0) - 500.0) < 1e-12
    cp1550 = 600.0 + (1550.0 - 500.0) * 200.0 / 1500.0
    assert abs(o.capacity(1550.0) - (cp1550 + 2.0e5 / 100.0)) < 1e-10
    assert abs(o.capacity(1500.0) - (600.0 + 1000.0 * 200.0 / 1500.0 + 2000.0)) < 1e-10
    assert abs(o.capacity(1601.0) - (600.0 + 1101.0 * 200.0 / 1500.0)) < 1e-10


def test_beam_path_zigzag():
    prob = W.cfg2()
    o = Oracle(prob)
    tr = prob.tracks
    L0 = np.linalg.norm(tr[0, 3:6] - tr[0, 0:3])
    v = tr[0, 6]
    on, xb, yb, Wb, k = o.beam(0.0)
    assert on and k == 0 and abs(xb - tr[0, 0]) < 1e-15 and abs(yb - tr[0, 1]) < 1e-15
    assert abs(Wb - 0.35 * 200.0) < 1e-12
    on, xb, yb, Wb, k = o.beam(0.25 * L0 / v)
    assert on and k == 0 and abs(xb - (tr[0, 0] + 0.25 * (tr[0, 3] - tr[0, 0]))) < 1e-12
    on, xb, yb, Wb, k = o.beam(1.5 * L0 / v)
    assert on and k == 1 and abs(yb - tr[1, 1]) < 1e-15
    assert abs(xb - 0.5 * (tr[1, 0] + tr[1, 3])) < 1e-12
    # zigzag: track 1 starts where track 0 ended (in x), one hatch over
    assert abs(tr[1, 0] - tr[0, 3]) < 1e-15 and abs(abs(tr[1, 1] - tr[0, 1]) - 100e-6) < 1e-15
    on, *_ = o.beam(10 * L0 / v + 1e-9)
    assert not on


def test_history_initial_state_and_monotone_update():
    prob = W.small_nonlinear(nx=6, ny=6, nz=4, steps=0)
    o = Oracle(prob)
    rc = o.init_history()
    rc3 = rc.reshape(prob.nz, prob.ny, prob.nx, 3, 3, 3)
    # h = 31.25 um: the top cell layer is powder, plus the lowest qp level of the second
    assert np.all(rc3[-1] == 0.0)
    depth_q = prob.L[2] - (prob.nz - 2 + np.array([0.5 - math.sqrt(15) / 10, 0.5, 0.5 + math.sqrt(15) / 10])) * 31.25e-6
    for lev in range(3):
        expect = 0.0 if depth_q[lev] <= 40e-6 else 1.0
        assert np.all(rc3[-2][:, :, lev] == expect)
    assert np.all(rc3[:-2] == 1.0)
    # heat the top: r only grows, stays in [0,1], and g <= r (so r_s >= 0)
    T = o.init_T()
    T[-(2 * prob.nx + 1) * (2 * prob.ny + 1) * 3:] = 1600.0  # whole top cell layer
    rc_before = rc.copy()
    f, Cl, fv = o.assemble(T, rc, 0.0)
    assert np.all(rc >= rc_before) and np.all(rc <= 1.0) and np.all(rc >= 0.0)
    assert np.any(rc > rc_before)


# --------------------------------------------------------------------------
# implicit backward Euler (eq. backward_euler_nonlinear)
# --------------------------------------------------------------------------
def test_backward_euler_sine_mode_q1_closed_form():
    """Consistent capacity: the nodal sine is a generalized eigenvector of (K, M)
    with eigenvalue alpha * 3a/b, so each backward Euler step divides it by
    (1 + dt alpha 3a/b)."""
    n = 6
    k, rho, cp = 20.0, 7900.0, 500.0
    alpha = k / (rho * cp)
    prob = W.sine_mode(1, n, k=k, rho=rho, cp=cp)
    o = Oracle(prob)
    h = 1.0 / n
    a = 2.0 / h ** 2 * (1.0 - math.cos(math.pi * h))
    b = (2.0 + math.cos(math.pi * h)) / 3.0
    lam = 3.0 * a / b
    dt = 50.0 * 2.0 / (alpha * 4.0 / h ** 2)  # far beyond the explicit limit
    s = _sine_field(1, n)
    A = 120.0
    T = prob.T_D + A * s
    rc = o.init_history()
    for step in range(3):
        T, info = o.implicit_step(T, rc, step * dt, dt, cg_rtol=1e-14, picard_tol=1e-10)
        assert info["status"] == 0
    np.testing.assert_allclose(T, prob.T_D + A * s * (1.0 + dt * alpha * lam) ** -3, rtol=0,
                               atol=1e-11 * A)


def test_backward_euler_q2_matches_direct_solve():
    """Constant coefficients: the Picard/PCG step equals a dense direct solve of
    (M/dt + K) T_{n+1} = M T_n / dt with Dirichlet rows eliminated."""
    prob = _const_problem(2, 3, 2, 2, (0.3, 0.2, 0.2), mask=W.FACE_ZM)
    o = Oracle(prob)
    K3, M3 = global_3d(2, 3, 2, 2, (0.3, 0.2, 0.2))
    kk, rc_ = prob.k_bp[0], prob.rho * prob.cp_bp[0]
    free = ~o.dirichlet_mask()
    Tn = prob.T_D + 100.0 * (1.0 + W.seeded_vector(o.N, 4))
    Tn[~free] = prob.T_D
    dt = 1e3
    A = rc_ * M3 / dt + kk * K3
    rhs = rc_ * M3 @ Tn / dt
    T = Tn.copy()
    T[~free] = prob.T_D
    # move the known Dirichlet values to the right-hand side
    rhs_f = rhs[free] - A[np.ix_(free, ~free)] @ T[~free]
    T[free] = np.linalg.solve(A[np.ix_(free, free)], rhs_f)
    out, info = o.implicit_step(Tn, o.init_history(), 0.0, dt, cg_rtol=1e-14, picard_tol=1e-10)
    np.testing.assert_allclose(out, T, rtol=0, atol=1e-10 * np.abs(T).max())


def test_backward_euler_nonlinear_residual_vanishes():
    """With the nonlinear law, the converged step satisfies the discrete equation
    C(T_n)(T - T_n)/dt = f(T; r_n) at free nodes (f assembled by the element loop
    with the history held at the start of the step), and the history is then
    committed as max(r_n, g(T))."""
    prob = W.small_nonlinear(nx=4, ny=4, nz=3, steps=0).replace(laser_kind=W.LASER_OFF)
    o = Oracle(prob)
    rng = np.random.default_rng(1)
    Tn = 293.0 + 1800.0 * rng.random(o.N)
    Tn[o.dirichlet_mask()] = prob.T_D
    rc = o.init_history()
    dt = 1e-3
    rc_out = rc.copy()
    T, info = o.implicit_step(Tn, rc_out, 0.0, dt, cg_rtol=1e-13, picard_tol=1e-10, picard_max_it=60)
    assert info["status"] == 0
    f, Cl, fv = o.assemble_lagged(T, rc, dt)
    rc_commit = rc.copy()
    o.assemble(T, rc_commit, dt)
    np.testing.assert_array_equal(rc_out, rc_commit)
    assert np.any(rc_out > rc)
    r = o.capacity_apply(Tn, T - Tn) / dt - f
    free = ~o.dirichlet_mask()
    assert np.abs(r[free]).max() < 1e-7 * np.abs(f[free]).max()


# --------------------------------------------------------------------------
# discrete adjoint
# --------------------------------------------------------------------------
def _adjoint_case(kind):
    prob = W.small_nonlinear(nx=8, ny=6, nz=4, steps=0, n_tracks=3, track_length=0.06e-3,
                             hatch=50e-6)
    if kind == "linear":
        prob = prob.replace(T_bp=np.array([0.0, 1e4]), k_bp=np.array([25.0, 25.0]),
                            cp_bp=np.array([600.0, 600.0]), latent=0.0, powder_k_factor=1.0,
                            powder_depth=0.0)
    elif kind == "no_latent":
        prob = prob.replace(latent=0.0)
    prob = W.with_probes(prob, 6, seed=3, t_hi=900.0)
    return prob


# (case, relative FD step, tolerance).  The apparent capacity jumps by
# L/(T_l - T_s) at T_s and T_l, so the step map is discontinuous where a
# quadrature point crosses them; central differences with a 1e-4 step straddle
# such jumps, and the full law is checked with steps small enough not to.
@pytest.mark.parametrize("kind,rel,tol", [("linear", 1e-4, 1e-7), ("no_latent", 1e-4, 5e-4),
                                          ("full", 1e-8, 1e-6)])
def test_adjoint_matches_central_differences(kind, rel, tol):
    prob = _adjoint_case(kind)
    P0 = prob.tracks[:, 7].copy() * (1.0 + 0.1 * np.arange(len(prob.tracks)))
    o = Oracle(prob, track_power=P0)
    T0 = o.init_T()
    dt, n = 2.5e-6, 100
    J, dW, TN = o.adjoint(T0, 0.0, dt, n, prob.probes, prob.targets)
    A = prob.absorptivity
    assert np.all(dW != 0.0)  # every track is scanned within the run
    if kind != "linear":
        assert TN.max() > prob.T_l  # the law's nonlinear branches are exercised
    for k in range(len(P0)):
        eps = rel * P0[k]
        Js = []
        for sgn in (1, -1):
            P = P0.copy()
            P[k] += sgn * eps
            Js.append(Oracle(prob, track_power=P).adjoint(T0, 0.0, dt, n, prob.probes, prob.targets)[0])
        fd = (Js[0] - Js[1]) / (2 * eps)
        # dJ/dP_k = A dJ/dW_k
        assert abs(A * dW[k] - fd) <= tol * abs(fd)


# (case, FD step in K, tolerance): J is quadratic in T_0 for constant
# coefficients, so central differences are exact up to round-off there.
@pytest.mark.parametrize("kind,eps,tol", [("linear", 1.0, 1e-8), ("full", 1e-5, 1e-5)])
def test_adjoint_initial_state_gradient_matches_central_differences(kind, eps, tol):
    """<dJ/dT_0, v> from the adjoint against central differences of J along
    seeded directions v over all nodes (Dirichlet nodes included: the first
    step reads them before they are reset)."""
    prob = _adjoint_case(kind)
    o = Oracle(prob)
    T0 = o.init_T() + 50.0 * W.seeded_vector(o.N, 11)
    dt, n = 2.5e-6, 60
    J, dW, TN, lam0 = o.adjoint(T0, 0.0, dt, n, prob.probes, prob.targets, with_lam0=True)
    if kind != "linear":
        assert TN.max() > prob.T_l
    for seed in (21, 22):
        v = W.seeded_vector(o.N, seed)
        Jp = o.adjoint(T0 + eps * v, 0.0, dt, n, prob.probes, prob.targets)[0]
        Jm = o.adjoint(T0 - eps * v, 0.0, dt, n, prob.probes, prob.targets)[0]
        fd = (Jp - Jm) / (2 * eps)
        assert abs(np.dot(lam0, v) - fd) <= tol * abs(fd)


def test_adjoint_linear_case_exact_response():
    """Constant coefficients: T_N is affine in the track powers, so
    dJ/dW_k = 2 sum_p (T_p - T*_p) R_pk with R_pk the probe response to a unit
    change of W_k (obtained from two forward runs, exact up to round-off)."""
    prob = _adjoint_case("linear")
    P0 = prob.tracks[:, 7].copy()
    o = Oracle(prob, track_power=P0)
    T0 = o.init_T()
    dt, n = 2.5e-6, 100
    J, dW, TN = o.adjoint(T0, 0.0, dt, n, prob.probes, prob.targets)
    Tp = o.probe(TN, prob.probes)
    A = prob.absorptivity
    for k in range(len(P0)):
        P = P0.copy()
        P[k] += 1.0 / A  # unit change of W_k
        TN1 = Oracle(prob, track_power=P).adjoint(T0, 0.0, dt, n, prob.probes, prob.targets)[2]
        R = o.probe(TN1, prob.probes) - Tp
        expect = 2.0 * np.dot(Tp - prob.targets, R)
        assert abs(dW[k] - expect) <= 1e-6 * max(abs(expect), 1e-6)


# --------------------------------------------------------------------------
# lumped capacity with a temperature-dependent c
# --------------------------------------------------------------------------
@pytest.mark.parametrize("deg", [1, 2])
def test_diffusion_rows_sum_to_zero(deg):
    """Sum over all nodes of f_diff = -sum_e sum_q W k grad(sum_a N_a) . grad T = 0
    for any T and history (the basis sums to one), so the heat leaving the free
    nodes is the reaction at the Dirichlet nodes."""
    prob = W.small_nonlinear(nx=5, ny=4, nz=3, steps=0).replace(degree=deg)
    o = Oracle(prob)
    T = o.init_T() + 900.0 * (1.0 + W.seeded_vector(o.N, 4))
    rc = o.init_history()
    f, Cl, fv = o.assemble(T, rc, 1e-5)
    fd = f - fv
    assert abs(fd.sum()) <= 1e-12 * np.abs(fd).sum()


@pytest.mark.parametrize("deg", [1, 2])
def test_lumped_capacity_nodal_form(deg):
    """C~_i = rho c(T_i) M~_i with M~ the row sums of the exact mass matrix
    (Kronecker assembly), for a field spanning every segment of the law."""
    prob = W.small_nonlinear(nx=3, ny=2, nz=2, steps=0).replace(degree=deg, laser_kind=W.LASER_OFF)
    o = Oracle(prob)
    K3, M3 = global_3d(deg, 3, 2, 2, prob.L)
    T = 250.0 + 2900.0 * np.random.default_rng(2).random(o.N)
    f, Cl, fv = o.assemble(T, o.init_history(), 0.0)
    c = np.array([o.capacity(t) for t in T])
    np.testing.assert_allclose(Cl, prob.rho * c * M3.sum(axis=1), rtol=1e-13)
    assert np.all(Cl > 0)


def test_q2_nonlinear_scheme_does_not_amplify_rounding():
    """With the nodal lumped capacity the explicit Q2 scheme at half the
    stability limit keeps a 1e-15 relative perturbation at rounding level through
    melting, while the row sum of the consistent C(T) turns negative on Q2."""
    prob = W.small_nonlinear(nx=10, ny=9, nz=5, steps=0, track_length=0.25e-3)
    o = Oracle(prob)
    lam = o.stability_lambda(W.seeded_vector(o.N, 1), 100)
    dt = 0.5 * 2.0 / lam
    T1, r1 = o.init_T(), o.init_history()
    T2 = T1 * (1.0 + 1e-15 * np.random.default_rng(0).standard_normal(o.N))
    r2 = r1.copy()
    o.explicit_steps(T1, r1, 0.0, dt, 80)
    o.explicit_steps(T2, r2, 0.0, dt, 80)
    assert T1.max() > prob.T_l
    assert np.abs(T1 - T2).max() < 1e-10 * T1.max()
