"""Temporal convergence of the combined explicit/implicit scheme with layer
activation (the paper's appendix on temporal convergence).

Two layers of a growing box with one track each: explicit steps while the beam
scans layer 1, a cool-down whose first part stays explicit and whose rest is
taken with implicit (backward Euler) steps, activation of layer 2 at T_0, and
explicit steps while the beam scans layer 2.  The temperature at an observation
point (top of layer 1, middle of the track) is recorded after every step.  The
sequence runs on the GPU through the library for step sizes dt_ref / 2^k in both
phases, and the differences between successive levels at common times give the
observed order of the scheme (one for forward and backward Euler).
"""
from __future__ import annotations

import math

import numpy as np


def schedule(prob, dt_crit, level, n_cool_explicit=50, t_cool=0.06, dt_imp_ref=2e-2, dt_ex_max=2e-5):
    """The step plan of one level: scan and cool-down lengths and step sizes.
    The explicit reference step is the paper's 2e-5 s or half the stability
    limit if that is smaller, rounded so that the scan takes a whole number of
    steps; every level halves both steps (2^level times as many)."""
    tr1 = np.asarray(prob.tracks[0])
    t_scan = float(np.linalg.norm(tr1[3:6] - tr1[0:3]) / tr1[6])
    n_ref = math.ceil(t_scan / min(dt_ex_max, 0.5 * dt_crit))
    f = 2 ** level
    dt_ex = t_scan / (n_ref * f)
    t_ce = n_cool_explicit * t_scan / n_ref  # explicit part of the cool-down (same at all levels)
    n_imp_ref = max(1, round((t_cool - t_ce) / dt_imp_ref))
    dt_imp = (t_cool - t_ce) / (n_imp_ref * f)
    return {"t_scan": t_scan, "dt_ex": dt_ex, "n_scan": n_ref * f, "n_cool_explicit": n_cool_explicit * f,
            "dt_imp": dt_imp, "n_implicit": n_imp_ref * f, "t_cool": t_cool, "factor": f}


def run(prob, plan, obs, layer_cells=1, device="cuda:0", newton=False):
    """One run of the two-layer sequence on the GPU.  prob: a box whose top
    2 * layer_cells cell layers are the two powder layers (e.g.
    pbf_workloads.convergence_box()); returns the times, the observation-point
    temperatures after every step and the phase of every step."""
    import torch

    from . import pbftherm

    tr = np.asarray(prob.tracks, dtype=np.float64)
    p1 = prob.replace(tracks=tr[:1], t_start=0.0)
    nz1 = prob.nz - layer_cells
    sim = pbftherm.from_problem(p1, device=device, active_layers=nz1)
    sim.set_probes(np.asarray([obs], dtype=np.float64), None)
    T, rc = sim.init_state(prob.T0)
    T_tmp = torch.empty_like(T)
    ts, vals, phases = [], [], []

    def record(t, phase):
        ts.append(t)
        vals.append(float(sim.probe(T).item()))
        phases.append(phase)

    t = 0.0
    record(t, "start")
    for _ in range(plan["n_scan"]):  # scan of layer 1
        sim.explicit_steps(T, rc, t, plan["dt_ex"], 1, T_tmp=T_tmp)
        t += plan["dt_ex"]
        record(t, "scan1")
    for _ in range(plan["n_cool_explicit"]):  # dynamic start of the cool-down
        sim.explicit_steps(T, rc, t, plan["dt_ex"], 1, T_tmp=T_tmp)
        t += plan["dt_ex"]
        record(t, "cool_explicit")
    work = sim.newton_work(30) if newton else None
    for _ in range(plan["n_implicit"]):  # rest of the cool-down, implicit
        if newton:
            Tn, _ = sim.implicit_step_newton(T, rc, t, plan["dt_imp"], lin_rtol=1e-11, newton_tol=1e-8, work=work,
                                             T_out=T_tmp)
        else:
            Tn, _ = sim.implicit_step(T, rc, t, plan["dt_imp"], cg_rtol=1e-11, picard_tol=1e-8, T_out=T_tmp)
        T.copy_(Tn)
        t += plan["dt_imp"]
        record(t, "cool_implicit")
    t2 = plan["t_scan"] + plan["n_cool_explicit"] * plan["dt_ex"] + plan["n_implicit"] * plan["dt_imp"]
    t = t2
    sim.activate_layers(prob.nz, prob.T0, T, rc)  # layer 2
    sim.set_laser(prob.laser_kind, prob.radius, prob.absorptivity, prob.h_powder, t2, tr[1:2])
    for _ in range(plan["n_scan"]):  # scan of layer 2
        sim.explicit_steps(T, rc, t, plan["dt_ex"], 1, T_tmp=T_tmp)
        t += plan["dt_ex"]
        record(t, "scan2")
    return {"t": np.array(ts), "T_obs": np.array(vals), "phase": np.array(phases), "t2": t2}


def temporal_convergence(prob, levels=3, obs=(0.5e-3, 0.0, 0.24e-3), layer_cells=1, device="cuda:0",
                         newton=False, dt_crit=None):
    """Runs levels 0..levels-1 and compares successive levels at the times of the
    coarser one, per phase: max |T_k - T_{k+1}| and the observed order
    log2(d_k / d_{k+1})."""
    import torch

    from . import pbftherm

    if dt_crit is None:
        s = pbftherm.from_problem(prob, device=device)
        v0 = torch.tensor(np.random.default_rng(1).uniform(-1, 1, s.info()["n_dofs"]), device=device)
        dt_crit = s.stability_dt(v0, 100)
        del s
    runs = []
    for k in range(levels):
        plan = schedule(prob, dt_crit, k)
        runs.append((plan, run(prob, plan, obs, layer_cells, device, newton)))
    out = {"dt_crit": dt_crit, "levels": [], "diff": {}, "order": {}, "diff_end": {}, "order_end": {}}
    for plan, r in runs:
        out["levels"].append({"dt_ex": plan["dt_ex"], "dt_imp": plan["dt_imp"], "T_obs_max": float(r["T_obs"].max()),
                              "T_obs_end": float(r["T_obs"][-1])})
    for ph in ("scan1", "cool_explicit", "cool_implicit", "scan2"):
        d = []
        for k in range(levels - 1):
            a, b = runs[k][1], runs[k + 1][1]
            ia = np.nonzero(a["phase"] == ph)[0]
            ib = np.nonzero(b["phase"] == ph)[0][1::2]  # the finer run's steps at the coarse times
            d.append(float(np.abs(a["T_obs"][ia] - b["T_obs"][ib]).max()))
        out["diff"][ph] = d
        out["order"][ph] = [math.log2(d[k] / d[k + 1]) if d[k + 1] > 0 else float("inf") for k in range(len(d) - 1)]
        # at the end of the phase only (the implicit cool-down starts with steps far
        # from the asymptotic regime of backward Euler: lambda dt >> 1 for the melt
        # pool's decay modes)
        e = []
        for k in range(levels - 1):
            a, b = runs[k][1], runs[k + 1][1]
            e.append(float(abs(a["T_obs"][np.nonzero(a["phase"] == ph)[0][-1]] -
                               b["T_obs"][np.nonzero(b["phase"] == ph)[0][-1]])))
        out["diff_end"][ph] = e
        out["order_end"][ph] = [math.log2(e[k] / e[k + 1]) if e[k + 1] > 0 else float("inf")
                                for k in range(len(e) - 1)]
    out["runs"] = runs
    return out
