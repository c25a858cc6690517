"""GPU parity of the explicit scheme: the HIP library against the CPU oracle on
the same seeded inputs, element by element.

FP64 bar: max-relative and relative-L2 error <= 1e-12 (relative to max|T| and
||T||).  Cases cover Q1 and Q2, meshes smaller than one GPU tile, exact tile
multiples and ragged tails, the surface and the volume source, the powder
history, the assembled vectors f and C~, the stability estimate, and one step at
the full benchmark sizes checked on sampled nodes."""
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


@pytest.mark.parametrize("cfg", ["cfg2", "cfg4"])
def test_full_size_step_on_sampled_nodes(cfg):
    """At the benchmark sizes: advance the GPU state 150 steps, then check one
    more GPU step against the oracle's step from the same state at sampled nodes
    (melt pool, tile faces, boundaries, random)."""
    need_gpu()
    prob = W.CONFIGS[cfg]()
    sim = sim_for(prob)
    info = sim.info()
    T, rc = sim.init_state(prob.T0)
    dt = 2.5e-6
    n0 = 150
    sim.explicit_steps(T, rc, 0.0, dt, n0)
    torch.cuda.synchronize()
    Tn = T.cpu().numpy()
    rn = rc.cpu().numpy()
    sim.explicit_steps(T, rc, n0 * dt, dt, 1)
    torch.cuda.synchronize()
    Tn1 = T.cpu().numpy()
    assert Tn.max() > prob.T_l  # a melt pool exists
    o = oracle.Oracle(prob)
    rng = np.random.default_rng(11)
    nodes = _sampled_nodes(prob, rng, Tn)
    rc_full = history_to_full(prob, rn, info["n_hist_layers"])
    ref = o.explicit_step_sampled(Tn, rc_full, n0 * dt, dt, nodes)
    err = np.abs(Tn1[nodes] - ref).max() / np.abs(ref).max()
    print(f"{cfg}: {len(nodes)} sampled nodes, max rel err {err:.2e}, Tmax {Tn.max():.0f}")
    assert err <= TOL64


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
