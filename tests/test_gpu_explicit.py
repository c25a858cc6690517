"""GPU parity of the explicit scheme: the HIP library against the CPU oracle on
the same seeded inputs, element by element.

FP64 bar: max-relative and relative-L2 error <= 1e-12 (relative to max|T| and
||T||).  Cases cover Q1 and Q2, meshes smaller than one GPU tile, exact tile
multiples and ragged tails, the surface and the volume source, the powder
history, the assembled vectors f and C~, the stability estimate, Dirichlet
conditions on every face, the sine eigenmode against its discrete closed form,
and steps at the full benchmark sizes (whole field and sampled nodes)."""
import numpy as np
import pytest
import torch

import oracle
import pbf_workloads as W
from tests.gpu_util import history_to_full, need_gpu, oracle_dt, rel_errors, sim_for

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def _run_pair(prob, steps, dt, precision=64):
    sim = sim_for(prob)
    info = sim.info()
    T, rc = sim.init_state(prob.T0)
    sim.explicit_steps(T, rc, 0.0, dt, steps, precision=precision)
    torch.cuda.synchronize()
    o = oracle.Oracle(prob)
    To, ro = o.init_T(), o.init_history()
    o.explicit_steps(To, ro, 0.0, dt, steps)
    Tg = T.cpu().numpy()
    rg = history_to_full(prob, rc.cpu().numpy(), info["n_hist_layers"])
    return Tg, rg, To, ro, info


def test_cfg1_q1_surface_flux_full_run():
    need_gpu()
    prob = W.cfg1()
    dt = oracle_dt(prob)
    Tg, rg, To, ro, info = _run_pair(prob, prob.steps, dt)
    mx, l2 = rel_errors(Tg, To)
    print(f"cfg1: dt={dt:.4e} max rel {mx:.2e} rel-L2 {l2:.2e} Tmax {To.max():.1f}")
    assert To.max() > prob.T0 + 10.0  # the beam heated the box
    assert mx <= TOL64 and l2 <= TOL64


@pytest.mark.parametrize("dims", [(20, 18, 10), (16, 16, 8), (3, 2, 1), (1, 1, 1), (9, 9, 5)])
def test_q2_nonlinear_run(dims):
    need_gpu()
    nx, ny, nz = dims
    prob = W.small_nonlinear(nx=nx, ny=ny, nz=nz, steps=120, track_length=0.8 * nx * 31.25e-6)
    dt = oracle_dt(prob)
    Tg, rg, To, ro, info = _run_pair(prob, prob.steps, dt)
    mx, l2 = rel_errors(Tg, To)
    print(f"{dims}: dt={dt:.3e} max rel {mx:.2e} rel-L2 {l2:.2e} Tmax {To.max():.0f} "
          f"melted points {(ro > 0).sum() - (ro == 1).sum()}")
    assert mx <= TOL64 and l2 <= TOL64
    assert np.abs(rg - ro).max() <= 1e-9


@pytest.mark.parametrize("degree", [1, 2])
def test_anisotropic_spacing_run(degree):
    """Unequal cell sizes in x, y and z (the cell kernel then forms the three
    flux factors separately instead of one common factor per point)."""
    need_gpu()
    nx, ny, nz = 21, 17, 9
    base = W.small_nonlinear(nx=nx, ny=ny, nz=nz, steps=100, track_length=0.8 * nx * 31.25e-6)
    prob = base.replace(degree=degree, L=(nx * 31.25e-6, ny * 26.0e-6, nz * 37.5e-6))
    dt = oracle_dt(prob)
    Tg, rg, To, ro, info = _run_pair(prob, prob.steps, dt)
    mx, l2 = rel_errors(Tg, To)
    print(f"Q{degree} anisotropic: dt={dt:.3e} max rel {mx:.2e} rel-L2 {l2:.2e} Tmax {To.max():.0f}")
    assert To.max() > prob.T0 + 100.0
    assert mx <= TOL64 and l2 <= TOL64
    assert np.abs(rg - ro).max() <= 1e-9


def test_q2_run_reaches_melting_and_history():
    """The small case must exercise every branch of the law: melting, latent heat,
    powder consolidation, several breakpoints."""
    need_gpu()
    prob = W.small_nonlinear(nx=20, ny=18, nz=10, steps=200)
    dt = oracle_dt(prob)
    Tg, rg, To, ro, info = _run_pair(prob, prob.steps, dt)
    assert To.max() > prob.T_l
    assert np.any((ro > 0) & (ro < 1))  # partially consolidated powder
    assert np.any(ro == 1.0) and info["n_hist_layers"] == 2
    mx, l2 = rel_errors(Tg, To)
    assert mx <= TOL64 and l2 <= TOL64
    assert np.abs(rg - ro).max() <= 1e-9


def test_q2_many_columns_segmented_run():
    """A box with enough columns that the explicit kernel splits each column into
    z-segments of several layers (a short top segment over longer ones) with ragged
    x and y tails, run through melting: full-field parity with the oracle."""
    need_gpu()
    prob = W.small_nonlinear(nx=33, ny=33, nz=57, steps=20, track_length=0.5e-3, n_tracks=2)
    Tg, rg, To, ro, info = _run_pair(prob, prob.steps, 2.5e-6)
    mx, l2 = rel_errors(Tg, To)
    print(f"33x33x57: max rel {mx:.2e} rel-L2 {l2:.2e} Tmax {To.max():.0f}")
    assert To.max() > prob.T_l
    assert mx <= TOL64 and l2 <= TOL64
    assert np.abs(rg - ro).max() <= 1e-9


@pytest.mark.parametrize("degree", [1, 2])
def test_q1_q2_volume_source_run(degree):
    need_gpu()
    prob = W.small_nonlinear(nx=12, ny=10, nz=6, steps=80)
    if degree == 1:
        prob = prob.replace(degree=1)
    dt = oracle_dt(prob)
    Tg, rg, To, ro, info = _run_pair(prob, prob.steps, dt)
    mx, l2 = rel_errors(Tg, To)
    assert mx <= TOL64 and l2 <= TOL64


@pytest.mark.parametrize("degree", [1, 2])
def test_assemble_random_field(degree):
    """f(T) and C~(T) for a random temperature field spanning all material
    segments, on a mesh with ragged tiles."""
    need_gpu()
    prob = W.small_nonlinear(nx=19, ny=10, nz=9, steps=0).replace(degree=degree)
    sim = sim_for(prob)
    info = sim.info()
    o = oracle.Oracle(prob)
    rng = np.random.default_rng(5)
    T = 250.0 + 2900.0 * rng.random(o.N)
    rc_full = o.init_history()
    rc_full[rc_full == 0.0] = rng.random((rc_full == 0.0).sum()) * 0.8
    from tests.gpu_util import full_to_history
    hist = full_to_history(prob, rc_full, info["n_hist_layers"])
    t = 1.3e-4
    Td = torch.tensor(T, device="cuda")
    rd = torch.tensor(hist if hist.size else np.zeros(1), device="cuda")
    f, Cl = sim.assemble(Td, rd, t)
    torch.cuda.synchronize()
    fo, Co, fvo = o.assemble(T, rc_full, t)
    assert np.abs(f.cpu().numpy() - fo).max() <= TOL64 * np.abs(fo).max()
    assert np.abs(Cl.cpu().numpy() - Co).max() <= TOL64 * np.abs(Co).max()
    rg = history_to_full(prob, rd.cpu().numpy(), info["n_hist_layers"])
    assert np.abs(rg - rc_full).max() <= 1e-12


@pytest.mark.parametrize("degree,dims,mask", [(1, (5, 4, 3), W.FACE_ZM), (2, (7, 5, 4), W.FACE_ZM),
                                               (2, (4, 4, 4), 0)])
def test_stability_lambda_matches_oracle(degree, dims, mask):
    need_gpu()
    prob = W.small_nonlinear(nx=dims[0], ny=dims[1], nz=dims[2], steps=0).replace(
        degree=degree, dirichlet_mask=mask)
    o = oracle.Oracle(prob)
    v0 = W.seeded_vector(o.N, 3)
    lam_o = o.stability_lambda(v0, 150)
    sim = sim_for(prob)
    lam_g = sim.stability_lambda(torch.tensor(v0, device="cuda"), 150)
    assert abs(lam_g - lam_o) <= 1e-10 * lam_o


def _sampled_nodes(prob, rng, T, n_random=160):
    NX, NY, NZ = prob.nodes_per_dim
    nodes = set(rng.integers(0, prob.n_dofs, n_random).tolist())
    # hottest nodes (melt pool) and their neighbourhood
    hot = np.argsort(T)[-48:]
    nodes.update(hot.tolist())
    # whole node columns through every z-segment end: under the beam, and on an
    # x and a y column face next to it
    hi = int(hot[-1])
    bi, bj = hi % NX, (hi // NX) % NY
    fi, fj = (bi // 32) * 32 or 32, (bj // 32) * 32 or 32
    for ci, cj in [(bi, bj), (fi, bj), (bi, fj), (fi, fj)]:
        nodes.update(ci + NX * (cj + NY * k) for k in range(NZ))
    # tile faces, corners, the Dirichlet bottom and the last node
    for gi, gj, gk in [(16, 16, 8), (16, 5, 3), (5, 16, 3), (5, 5, 8), (0, 0, 0), (NX - 1, NY - 1, NZ - 1),
                       (NX - 1, 3, NZ - 1), (32, 32, 16), (NX // 2, NY // 2, NZ - 1)]:
        if gi < NX and gj < NY and gk < NZ:
            nodes.add(gi + NX * (gj + NY * gk))
    return np.array(sorted(nodes), dtype=np.int64)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("cfg", ["cfg2", "cfg4"])
def test_full_size_steps_vs_oracle(cfg):
    """At the benchmark sizes and launch configuration: from a seeded state with a
    melt pool under the beam and partly consolidated powder, two GPU steps
    against two oracle steps over the whole field, then a third GPU step against
    the oracle's step evaluated at sampled nodes (melt pool, tile faces,
    segment ends, boundaries, random) from the oracle's own state."""
    need_gpu()
    prob = W.CONFIGS[cfg]()
    o = oracle.Oracle(prob)
    T0, t0 = W.hot_spot_state(prob, seed=17)
    rc_full = o.init_history()
    rng = np.random.default_rng(23)
    powder = rc_full == 0.0
    rc_full[powder] = np.where(rng.random(powder.sum()) < 0.3, rng.random(powder.sum()), 0.0)
    dt = 2.5e-6
    sim = sim_for(prob)
    info = sim.info()
    from tests.gpu_util import full_to_history
    T = torch.tensor(T0, device="cuda")
    rc = torch.tensor(full_to_history(prob, rc_full, info["n_hist_layers"]), device="cuda")
    sim.explicit_steps(T, rc, t0, dt, 2)
    torch.cuda.synchronize()
    Tg2 = T.cpu().numpy()
    rg2 = history_to_full(prob, rc.cpu().numpy(), info["n_hist_layers"])
    To, ro = T0.copy(), rc_full.copy()
    o.explicit_steps(To, ro, t0, dt, 2)
    assert To.max() > prob.T_l
    mx, l2 = rel_errors(Tg2, To)
    print(f"{cfg}: 2 steps full field max rel {mx:.2e} rel-L2 {l2:.2e} Tmax {To.max():.0f}")
    assert mx <= TOL64 and l2 <= TOL64
    assert np.abs(rg2 - ro).max() <= 1e-12
    sim.explicit_steps(T, rc, t0 + 2 * dt, dt, 1)
    torch.cuda.synchronize()
    Tg3 = T.cpu().numpy()
    nodes = _sampled_nodes(prob, rng, To)
    ref = o.explicit_step_sampled(To, ro, t0 + 2 * dt, dt, nodes)
    err = np.abs(Tg3[nodes] - ref).max() / np.abs(ref).max()
    print(f"{cfg}: third step, {len(nodes)} sampled nodes, max rel err {err:.2e}")
    assert err <= TOL64


@pytest.mark.parametrize("degree,n", [(1, 40), (2, 20)])
def test_explicit_sine_mode_closed_form(degree, n):
    """Every face Dirichlet, constant coefficients: the GPU's forward-Euler steps
    of sin(pi x) sin(pi y) sin(pi z) equal the discrete closed form (Q1: scalar
    decay factor; Q2: 8x8 matrix power on the invariant subspace).  n cells per
    direction span two column tiles with a ragged tail and several z-segments."""
    need_gpu()
    from tests.sine_modes import q1_explicit, q2_explicit, sine_field
    k, rho, cp = 20.0, 7900.0, 500.0
    alpha = k / (rho * cp)
    prob = W.sine_mode(degree, n, k=k, rho=rho, cp=cp)
    h = 1.0 / n
    dt = 0.4 * 2.0 / (alpha * (4.0 if degree == 1 else 36.0) / h ** 2)
    A, nsteps = 120.0, 30
    sim = sim_for(prob)
    T = torch.tensor(prob.T_D + A * sine_field(degree, n), device="cuda")
    rc = torch.zeros(1, dtype=torch.float64, device="cuda")
    sim.explicit_steps(T, rc, 0.0, dt, nsteps)
    torch.cuda.synchronize()
    expect = prob.T_D + A * (q1_explicit if degree == 1 else q2_explicit)(n, alpha, dt, nsteps)
    err = np.abs(T.cpu().numpy() - expect).max() / A
    print(f"Q{degree} n={n}: max |T - closed form| / A = {err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("mask", [W.ALL_FACES, W.ALL_FACES & ~W.FACE_ZP, W.FACE_XP | W.FACE_YM | W.FACE_ZM])
def test_dirichlet_faces_nonlinear_vs_oracle(mask):
    """Dirichlet on side and top faces (x/y column-face nodes, ragged far faces,
    segment ends) on a ragged multi-column box run through the beam."""
    need_gpu()
    prob = W.small_nonlinear(nx=21, ny=18, nz=11, steps=100, track_length=0.5e-3).replace(dirichlet_mask=mask)
    dt = oracle_dt(prob)
    Tg, rg, To, ro, info = _run_pair(prob, prob.steps, dt)
    mx, l2 = rel_errors(Tg, To)
    print(f"mask {mask}: max rel {mx:.2e} rel-L2 {l2:.2e} Tmax {To.max():.0f}")
    assert To.max() > prob.T0 + 500.0
    assert mx <= TOL64 and l2 <= TOL64
    assert np.abs(rg - ro).max() <= 1e-9
    d = oracle.Oracle(prob).dirichlet_mask()
    assert np.all(Tg[d] == prob.T_D)


def test_fp32_operator_error_vs_fp64_oracle():
    """Operator in FP32 on T - T_ref, state and update in FP64: errors against the
    FP64 oracle are reported and bounded (no exact FP32 result exists)."""
    need_gpu()
    prob = W.small_nonlinear(nx=20, ny=18, nz=10, steps=200)
    dt = oracle_dt(prob)
    Tg, rg, To, ro, info = _run_pair(prob, prob.steps, dt, precision=32)
    mx, l2 = rel_errors(Tg, To)
    rise = To - prob.T0
    mx_rise = np.abs(Tg - To).max() / np.abs(rise).max()
    melt = To >= prob.T_s
    mp = np.abs(Tg[melt] - To[melt]).max() / np.abs(To[melt]).max() if melt.any() else 0.0
    print(f"fp32 op: max rel {mx:.2e} rel-L2 {l2:.2e} max/rise {mx_rise:.2e} melt pool max rel {mp:.2e}")
    assert mx <= 1e-4 and l2 <= 1e-4


@pytest.mark.parametrize("degree,dims", [(2, (21, 18, 11)), (1, (37, 17, 9)), (2, (3, 2, 1))])
def test_laplace_reference_operator_vs_oracle(degree, dims):
    """The unit-conductivity reference operator y = K x equals minus the
    oracle's diffusion vector for a constant law k = 1 (laser off, no powder)
    at every node, on ragged multi-column boxes."""
    need_gpu()
    nx, ny, nz = dims
    base = W.small_nonlinear(nx=nx, ny=ny, nz=nz, steps=0).replace(degree=degree)
    prob = base.replace(T_bp=np.array([0.0, 1e9]), k_bp=np.array([1.0, 1.0]), cp_bp=np.array([500.0, 500.0]),
                        latent=0.0, powder_k_factor=1.0, powder_depth=0.0, laser_kind=W.LASER_OFF)
    o = oracle.Oracle(prob)
    x = W.seeded_vector(o.N, 31) * 100.0 + 500.0
    f, _, _ = o.assemble(x, o.init_history(), 0.0)
    sim = sim_for(base)  # the reference operator ignores the law, history and laser
    y = sim.laplace_apply(torch.tensor(x, device="cuda"))
    torch.cuda.synchronize()
    err = np.abs(y.cpu().numpy() + f).max() / np.abs(f).max()
    print(f"Laplace Q{degree} {dims}: max rel {err:.2e}")
    assert err <= TOL64

