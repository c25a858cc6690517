"""Pins of the oracle's radiation and evaporation terms on the free top surface
(Section 2, eqs. bc_rad_evap, bc_radiation, bc_evaporation; lagging in the
implicit scheme, Section 3.2, eq. backward_euler_nonlinear).

What fixes them independently of the oracle's own code:
- the Stefan-Boltzmann form: q_rad vanishes at the ambient temperature and
  q_rad(2 T_inf) = 15 eps sigma T_inf^4;
- the evaporation law: zero up to the boiling point, clamped above
  T_v + dT_max, and ln(mdot sqrt(T)) linear in 1/T with slope -C_T (the
  Arrhenius-type exponent) and intercept ln(0.82 C_P sqrt(C_M)) + C_T/T_v;
- the face integral: a uniform temperature gives sum_a f_a = -q(T) Lx Ly
  (partition of unity, Gauss exact for constants), on boxes and octrees;
- a brute-force numpy face quadrature with its own Lagrange basis on a tiny mesh;
- energy balance of an explicit step on a box with no Dirichlet face:
  sum_i C~_i (T_{n+1} - T_n)_i = dt sum_i f_RE,i;
- the implicit residual takes f_RE at T_n (not at T_{n+1}).
"""
import numpy as np
import pytest

import pbf_workloads as W
from oracle import Oracle, OctOracle

SIGMA = 5.670374419e-8


def _box(deg, nx=3, ny=2, nz=2, emissivity=0.7, evap=True, mask=W.FACE_ZM):
    p = W.small_nonlinear(nx=nx, ny=ny, nz=nz, steps=1)
    return W.with_surface_losses(p, emissivity=emissivity, evap=evap).replace(
        degree=deg, dirichlet_mask=mask, laser_kind=W.LASER_OFF)


def test_radiation_law():
    p = _box(2, evap=False)
    O = Oracle(p)
    Tinf = p.ambient
    assert O.surface_loss(Tinf) == 0.0
    assert O.surface_loss(2 * Tinf) == pytest.approx(15 * 0.7 * SIGMA * Tinf ** 4, rel=1e-14)
    assert O.surface_loss(0.5 * Tinf) < 0  # a colder surface gains heat


def test_evaporation_law_threshold_clamp_and_arrhenius_form():
    p = _box(2, emissivity=0.0)
    O = Oracle(p)
    assert O.surface_loss(p.T_v) == 0.0 and O.surface_loss(p.T_v - 1.0) == 0.0
    Tmax = p.T_v + p.dT_max
    assert O.surface_loss(Tmax + 500.0) == O.surface_loss(Tmax)
    assert O.surface_loss(p.T_v + 1e-9) > 0.0
    # above the last breakpoint the specific heat is the last table value
    cp = float(p.cp_bp[-1])
    T = np.linspace(p.T_v + 50.0, Tmax - 50.0, 9)
    mdot = np.array([O.surface_loss(t) for t in T]) / (p.h_v + cp * (T - p.T_h0))
    y = np.log(mdot * np.sqrt(T))
    slope, icpt = np.polyfit(1.0 / T, y, 1)
    assert slope == pytest.approx(-p.C_T, rel=1e-9)
    assert icpt == pytest.approx(np.log(0.82 * p.C_P * np.sqrt(p.C_M)) + p.C_T / p.T_v, rel=1e-9)


@pytest.mark.parametrize("deg", [1, 2])
@pytest.mark.parametrize("Tu", [1200.0, 3400.0, 4500.0])
def test_uniform_temperature_total_flux(deg, Tu):
    p = _box(deg)
    O = Oracle(p)
    f = O.surface_loss_vector(np.full(O.N, Tu))
    assert f.sum() == pytest.approx(-O.surface_loss(Tu) * p.L[0] * p.L[1], rel=1e-12)
    NX, NY, NZ = p.nodes_per_dim
    assert np.all(f.reshape(NZ, NY, NX)[:-1] == 0.0)  # top face only


def test_uniform_temperature_total_flux_octree():
    p = W.with_surface_losses(W.small_octree(degree=2, max_level=2)).replace(laser_kind=W.LASER_OFF)
    O = OctOracle(p)
    Tu = 3600.0
    f = np.zeros(O.N)
    T = np.full(O.N, Tu)
    rc = np.ones(O.NQ)
    f_re, _, _ = O.assemble(T, rc.copy(), 0.0)
    p0 = p.replace(emissivity=0.0, evap_on=False)
    f0, _, _ = OctOracle(p0).assemble(T, rc.copy(), 0.0)
    f = f_re - f0
    assert f.sum() == pytest.approx(-O.base.surface_loss(Tu) * p.L[0] * p.L[1], rel=1e-10)


def _lagrange_1d(p, a, x):
    nodes = np.arange(p + 1) / p
    v = np.ones_like(x)
    for b in range(p + 1):
        if b != a:
            v = v * (x - nodes[b]) / (nodes[a] - nodes[b])
    return v


@pytest.mark.parametrize("deg", [1, 2])
def test_face_quadrature_brute_force(deg):
    """numpy face quadrature with its own basis against the oracle's assembly."""
    p = _box(deg, nx=2, ny=3, nz=1)
    O = Oracle(p)
    NX, NY, NZ = p.nodes_per_dim
    rng = np.random.default_rng(11)
    T = rng.uniform(2500.0, 4200.0, O.N)
    xg, wg = np.polynomial.legendre.leggauss(deg + 1)
    xg, wg = 0.5 * (xg + 1.0), 0.5 * wg
    hx, hy = p.L[0] / p.nx, p.L[1] / p.ny
    f = np.zeros(O.N)
    k = NZ - 1
    for cy in range(p.ny):
        for cx in range(p.nx):
            for j in range(deg + 1):
                for i in range(deg + 1):
                    Ns, idx = [], []
                    for ay in range(deg + 1):
                        for ax in range(deg + 1):
                            Ns.append(_lagrange_1d(deg, ax, np.array(xg[i])) * _lagrange_1d(deg, ay, np.array(xg[j])))
                            idx.append((deg * cx + ax) + NX * ((deg * cy + ay) + NY * k))
                    Ns = np.array(Ns, dtype=float).reshape(-1)
                    Ts = float(Ns @ T[idx])
                    q = O.surface_loss(Ts)
                    f[idx] -= wg[i] * wg[j] * hx * hy * Ns * q
    g = O.surface_loss_vector(T)
    assert np.max(np.abs(g - f)) <= 1e-12 * np.max(np.abs(f))
    # the assembly of the explicit operator carries the same term
    rc = np.ones(O.NQ)
    fa, _, _ = O.assemble(T, rc.copy(), 0.0)
    f0, _, _ = Oracle(p.replace(emissivity=0.0, evap_on=False)).assemble(T, rc.copy(), 0.0)
    assert np.max(np.abs((fa - f0) - g)) <= 1e-9 * np.max(np.abs(fa))


@pytest.mark.parametrize("deg", [1, 2])
def test_explicit_step_energy_balance(deg):
    """No Dirichlet face, laser off: the stored-energy change of one step is dt
    times the assembled surface loss (the diffusion rows sum to zero)."""
    p = _box(deg, mask=0)
    O = Oracle(p)
    rng = np.random.default_rng(5)
    T0 = rng.uniform(2800.0, 4000.0, O.N)
    rc = np.ones(O.NQ)
    f, Cl, _ = O.assemble(T0, rc.copy(), 0.0)
    dt = 1e-7
    T1 = T0.copy()
    O.explicit_steps(T1, rc.copy(), 0.0, dt, 1)
    dE = float(np.sum(Cl * (T1 - T0)))
    Q = float(O.surface_loss_vector(T0).sum())
    assert Q < 0
    assert dE == pytest.approx(dt * Q, rel=1e-9)


def test_implicit_residual_uses_surface_loss_at_step_start():
    p = _box(2, nx=3, ny=3, nz=2)
    O = Oracle(p)
    rng = np.random.default_rng(3)
    Tn = O.init_T()
    NX, NY, NZ = p.nodes_per_dim
    Tn = Tn.reshape(NZ, NY, NX)
    Tn[-1] += rng.uniform(2500.0, 3800.0, Tn[-1].shape)  # hot top layer
    Tn = Tn.reshape(-1)
    rc = np.ones(O.NQ)
    dt = 1e-4
    T1, info = O.implicit_step(Tn, rc.copy(), 0.0, dt, cg_rtol=1e-13, picard_tol=1e-10)
    f, _, _ = O.assemble_lagged(T1, rc, dt)
    Cx = O.capacity_apply(Tn, T1 - Tn)
    free = ~O.dirichlet_mask()
    r_lag = (Cx / dt - f - O.surface_loss_vector(Tn))[free]
    r_new = (Cx / dt - f - O.surface_loss_vector(T1))[free]
    scale = np.max(np.abs(Cx[free] / dt))
    assert np.max(np.abs(r_lag)) < 1e-8 * scale
    assert np.max(np.abs(r_new)) > 1e3 * np.max(np.abs(r_lag))


def test_adjoint_rejects_surface_losses():
    p = _box(2)
    O = Oracle(p)
    with pytest.raises(ValueError):
        O.adjoint(O.init_T(), 0.0, 1e-6, 2, np.zeros((1, 3)) + 1e-5, np.zeros(1))
