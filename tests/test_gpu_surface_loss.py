"""GPU parity of the radiation and evaporation terms on the free top surface
(Section 2, eqs. bc_rad_evap, bc_radiation, bc_evaporation) against the oracle:
explicit runs hot enough for evaporation (Q1, Q2, FP64 and the FP32 operator),
the assembled vector, the implicit step with the terms lagged at T_n, octree
meshes, the energy identity, and the adjoint's refusal.

FP64 bar 1e-12 relative (1e-10 for implicit steps), FP32 operator 1e-4."""
import numpy as np
import pytest
import torch

import oracle
import pbf_workloads as W
from tests.gpu_util import full_to_history, history_to_full, need_gpu, oracle_dt, rel_errors, sim_for

pytestmark = pytest.mark.gpu


def _hot_problem(degree, dims=(20, 18, 10)):
    nx, ny, nz = dims
    p = W.small_nonlinear(nx=nx, ny=ny, nz=nz, steps=0, track_length=0.8 * nx * 31.25e-6)
    return W.with_surface_losses(p.replace(degree=degree))


@pytest.mark.parametrize("degree,steps,dims", [(2, 120, (20, 18, 10)), (1, 60, (20, 18, 10)),
                                               (2, 80, (9, 9, 5))])
def test_explicit_run_with_surface_losses(degree, steps, dims):
    need_gpu()
    prob = _hot_problem(degree, dims)
    dt = oracle_dt(prob)
    sim = sim_for(prob)
    info = sim.info()
    T, rc = sim.init_state(prob.T0)
    sim.explicit_steps(T, rc, 0.0, dt, steps)
    torch.cuda.synchronize()
    o = oracle.Oracle(prob)
    To, ro = o.init_T(), o.init_history()
    o.explicit_steps(To, ro, 0.0, dt, steps)
    o0 = oracle.Oracle(prob.replace(emissivity=0.0, evap_on=False))
    T0, r0 = o0.init_T(), o0.init_history()
    o0.explicit_steps(T0, r0, 0.0, dt, steps)
    Tg = T.cpu().numpy()
    mx, l2 = rel_errors(Tg, To)
    effect = np.abs(To - T0).max()
    print(f"CHECK Q{degree} {dims}: max rel {mx:.2e} rel-L2 {l2:.2e} Tmax {To.max():.0f} "
          f"(without losses {T0.max():.0f}), max effect {effect:.2f} K")
    assert To.max() > prob.T_v or degree == 1  # evaporation active on the Q2 runs
    assert effect > 1.0
    assert mx <= 1e-12 and l2 <= 1e-12
    rg = history_to_full(prob, rc.cpu().numpy(), info["n_hist_layers"])
    assert np.abs(rg - ro).max() <= 1e-9


@pytest.mark.parametrize("degree", [1, 2])
def test_assemble_hot_surface(degree):
    need_gpu()
    prob = _hot_problem(degree, (7, 5, 3))
    o = oracle.Oracle(prob)
    NX, NY, NZ = prob.nodes_per_dim
    T = 293.0 + 600.0 * (1.0 + W.seeded_vector(o.N, 9))
    T = T.reshape(NZ, NY, NX)
    T[-1] = 2600.0 + 1000.0 * (1.0 + W.seeded_vector(NX * NY, 10).reshape(NY, NX))  # 1600..4600 K
    T = T.reshape(-1)
    T[o.dirichlet_mask()] = prob.T_D
    rc = np.ones(o.NQ)
    f, Cl, _ = o.assemble(T, rc.copy(), 0.0)
    sim = sim_for(prob)
    info = sim.info()
    hist = full_to_history(prob, rc, info["n_hist_layers"])
    rd = torch.tensor(hist if hist.size else np.zeros(1), device="cuda")
    fg, Cg = sim.assemble(torch.tensor(T, device="cuda"), rd, 0.0)
    err = np.abs(fg.cpu().numpy() - f).max() / np.abs(f).max()
    print(f"CHECK Q{degree} assemble f: {err:.2e}, top-face share {np.abs(o.surface_loss_vector(T)).max() / np.abs(f).max():.2e}")
    assert err <= 1e-12
    assert np.abs(Cg.cpu().numpy() - Cl).max() <= 1e-13 * np.abs(Cl).max()


def test_fp32_operator_with_surface_losses():
    need_gpu()
    prob = _hot_problem(2)
    dt = oracle_dt(prob)
    sim = sim_for(prob)
    T, rc = sim.init_state(prob.T0)
    sim.explicit_steps(T, rc, 0.0, dt, 120, precision=32)
    torch.cuda.synchronize()
    o = oracle.Oracle(prob)
    To, ro = o.init_T(), o.init_history()
    o.explicit_steps(To, ro, 0.0, dt, 120)
    mx, l2 = rel_errors(T.cpu().numpy(), To)
    print(f"CHECK fp32 op with losses: max rel {mx:.2e} rel-L2 {l2:.2e}")
    assert mx <= 1e-4 and l2 <= 1e-4


def test_implicit_step_surface_losses_lagged():
    need_gpu()
    prob = _hot_problem(2)
    o = oracle.Oracle(prob)
    dt_ex = oracle_dt(prob)
    T, rc = o.init_T(), o.init_history()
    o.explicit_steps(T, rc, 0.0, dt_ex, 100)
    assert T.max() > prob.T_v
    cool = prob.replace(laser_kind=W.LASER_OFF)
    oc = oracle.Oracle(cool)
    To, oi = oc.implicit_step(T, rc.copy(), 100 * dt_ex, 1e-4, cg_rtol=1e-13, picard_tol=1e-10, picard_max_it=60)
    assert oi["status"] == 0
    sim = sim_for(cool)
    info = sim.info()
    hist = full_to_history(cool, rc, info["n_hist_layers"])
    rd = torch.tensor(hist if hist.size else np.zeros(1), device="cuda")
    Tg, gi = sim.implicit_step(torch.tensor(T, device="cuda"), rd, 100 * dt_ex, 1e-4, cg_rtol=1e-13,
                               picard_tol=1e-10, picard_max_it=60)
    torch.cuda.synchronize()
    mx, l2 = rel_errors(Tg.cpu().numpy(), To)
    print(f"CHECK implicit with losses: gpu {gi} oracle {oi} max rel {mx:.2e} rel-L2 {l2:.2e}")
    assert mx <= 1e-10 and l2 <= 1e-10
    assert abs(gi["cg_iters"] - oi["cg_iters"]) <= max(2, 0.02 * oi["cg_iters"])


def test_energy_identity_with_surface_losses():
    need_gpu()
    prob = _hot_problem(2)
    o = oracle.Oracle(prob)
    dt = oracle_dt(prob)
    T, rc = o.init_T(), o.init_history()
    o.explicit_steps(T, rc, 0.0, dt, 100)
    t = 100 * dt
    f, Cl, fv = o.assemble(T, rc.copy(), t)
    fre = o.surface_loss_vector(T)
    free = ~o.dirichlet_mask()
    sim = sim_for(prob)
    info = sim.info()
    hist = full_to_history(prob, rc, info["n_hist_layers"])
    rd = torch.tensor(hist if hist.size else np.zeros(1), device="cuda")
    Tp = torch.tensor(T, device="cuda")
    Tn = Tp.clone()
    sim.explicit_steps(Tn, rd, t, dt, 1)
    e = sim.energy(Tp, Tn, rd, t, dt)
    ext = np.sum(fv[free]) + np.sum(fre[free])  # source minus surface losses
    print(f"CHECK energy with losses: gpu {e}, oracle external power {ext:.6e}, losses {np.sum(fre):.3e}")
    assert np.sum(fre) < 0
    assert abs(e[1] - ext) <= 1e-10 * abs(np.sum(fv[free]))
    assert abs(e[3]) <= 1e-11 * dt * (abs(e[1]) + abs(e[2]))


def test_adjoint_refuses_surface_losses():
    need_gpu()
    from paper_2302_05164_amd import pbftherm
    prob = _hot_problem(2, (6, 6, 3))
    sim = sim_for(prob)
    pts = np.array([[0.5 * prob.L[0], 0.5 * prob.L[1], prob.L[2]]])
    sim.set_probes(pts, np.array([1000.0]))
    work = sim.gradient_work(2)
    T, rc = sim.init_state(prob.T0)
    with pytest.raises(pbftherm.PbfError, match="surface losses"):
        sim.gradient_forward(T, rc, 0.0, 1e-7, 3, work)


def _oct_setup(p):
    from paper_2302_05164_amd import pbftherm
    sim = pbftherm.from_problem(p, device="cuda:0")
    O = oracle.OctOracle(p)
    xl = sim.dof_coords()
    h = p.L[0] / p.nx / 2 ** p.max_level / p.degree
    kl = {tuple(k): i for i, k in enumerate(np.round(xl / h).astype(np.int64))}
    ko = np.round(O.dof_coords() / h).astype(np.int64)
    return sim, O, np.array([kl[tuple(k)] for k in ko], dtype=np.int64)


@pytest.mark.parametrize("deg", [1, 2])
def test_octree_explicit_and_implicit_with_surface_losses(deg):
    need_gpu()
    p = W.with_surface_losses(W.small_octree(degree=deg))
    sim, O, to_lib = _oct_setup(p)
    lam = O.stability_lambda(W.seeded_vector(O.N, 1), 60)
    dt = 0.5 * 2.0 / lam
    n = 80 if deg == 2 else 12
    T, ro = O.init_T(), O.init_history()
    O.explicit_steps(T, ro, 0.0, dt, n)
    Tl, rl = sim.init_state(p.T0)
    sim.explicit_steps(Tl, rl, 0.0, dt, n)
    torch.cuda.synchronize()
    err = np.abs(Tl.cpu().numpy()[to_lib] - T).max() / np.abs(T).max()
    print(f"CHECK octree Q{deg} explicit with losses: {err:.2e}, Tmax {T.max():.0f}")
    assert err <= 1e-12
    if deg == 1:
        return
    cool = p.replace(laser_kind=W.LASER_OFF)
    sim_c, Oc, _ = _oct_setup(cool)
    To, io = Oc.implicit_step(T, ro.copy(), n * dt, 1e-4, cg_rtol=1e-13, picard_tol=1e-10, picard_max_it=60)
    assert io["status"] == 0
    rl_h = rl.clone()
    Tg, ig = sim_c.implicit_step(Tl, rl_h, n * dt, 1e-4, cg_rtol=1e-13, picard_tol=1e-10, picard_max_it=60)
    torch.cuda.synchronize()
    err = np.abs(Tg.cpu().numpy()[to_lib] - To).max() / np.abs(To).max()
    print(f"CHECK octree implicit with losses: {err:.2e} gpu {ig} oracle {io}")
    assert err <= 1e-10
