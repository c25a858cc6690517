"""Scan phase on an octree that follows the beam, then a backward-Euler cool-down.

The octree workload (not a method of the paper, which remeshes per layer,
Section 4.1): Q_p leaves at max_level within refine_radius of the window
[s(t) - refine_trail, s(t) + refine_ahead] of the scan path around the beam's
arc length s(t); every `remesh_every` explicit steps the library builds the
leaves of the moved window (pbf_octree_path_leaves) and moves the state onto
them (pbf_octree_remesh: T interpolated, history taken from the nearest old
Gauss point).  Then backward-Euler steps with the laser off (Section 3.2),
Picard iterations with Jacobi-preconditioned CG.

Orchestration only: the leaves, the remesh transfer, every step and every
solve run in the library; this module sequences the calls and times them.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import pbftherm


def window(prob, s):
    """Arc-length window of the refinement around beam arc length s."""
    return max(0.0, s - prob.refine_trail), s + prob.refine_ahead


def window_leaves(prob, s):
    lo, hi = window(prob, s)
    return pbftherm.octree_path_leaves(prob.nx, prob.ny, prob.nz, prob.L, prob.max_level, prob.refine_radius,
                                       prob.tracks, lo, hi)


def time_at_arc_length(prob, s):
    """Time at which the beam reaches arc length s (tracks scanned in order,
    back to back, from prob.t_start)."""
    t = prob.t_start
    s0 = 0.0
    for tr in prob.tracks:
        length = float(np.linalg.norm(np.asarray(tr[3:6]) - np.asarray(tr[0:3])))
        if s <= s0 + length:
            return t + (s - s0) / tr[6]
        s0 += length
        t += length / tr[6]
    return t


def arc_length_at(prob, t):
    s, tk = 0.0, prob.t_start
    for tr in prob.tracks:
        length = float(np.linalg.norm(np.asarray(tr[3:6]) - np.asarray(tr[0:3])))
        dur = length / tr[6]
        if t < tk + dur:
            return s + max(0.0, t - tk) * tr[6]
        s += length
        tk += dur
    return s


def _timed(fn):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    out = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), out


def run(prob, n_explicit=None, n_implicit=None, dt=None, dt_implicit=None, remesh_every=None, cg_rtol=1e-10,
        picard_tol=1e-8, picard_max_it=30, cg_max_it=100000, leaves_fn=None, device="cuda:0", log=None):
    """Run the schedule from the beam at arc length prob.scan_start.

    Returns (T, rc, sim, record): record holds the explicit dt, per block of
    explicit steps (t, dofs, leaves, hanging nodes, ms on the GPU, host
    remesh ms) and per implicit step (ms, Picard and CG iterations, final
    relative residual).  leaves_fn(prob, s) gives the leaves at beam arc
    length s (default: the library's window leaves)."""
    leaves_fn = leaves_fn or window_leaves
    n_explicit = prob.steps if n_explicit is None else n_explicit
    n_implicit = prob.implicit_steps if n_implicit is None else n_implicit
    dt_implicit = prob.implicit_dt if dt_implicit is None else dt_implicit
    every = prob.remesh_every if remesh_every is None else remesh_every
    t0 = time_at_arc_length(prob, prob.scan_start)
    th = time.perf_counter()
    sim = pbftherm.from_problem(prob, device=device, leaves=leaves_fn(prob, prob.scan_start))
    rec = {"setup_host_ms": (time.perf_counter() - th) * 1e3, "t0": t0, "blocks": [], "implicit": []}
    if dt is None:
        from pbf_workloads import seeded_vector
        v0 = torch.tensor(seeded_vector(sim.info()["n_dofs"], 1), device=device)
        dt = prob.dt_factor * sim.stability_dt(v0, 50)
    rec["dt"] = dt
    T, rc = sim.init_state(prob.T0)
    T_tmp = torch.empty_like(T)
    n = 0
    while n < n_explicit:
        k = min(every, n_explicit - n) if every > 0 else n_explicit - n
        oi = sim.octree_info()
        nd = sim.info()["n_dofs"]
        ms, _ = _timed(lambda: sim.explicit_steps(T, rc, t0 + n * dt, dt, k, T_tmp=T_tmp))
        n += k
        blk = {"step": n, "t": t0 + n * dt, "dofs": nd, "leaves": oi["n_leaves"], "hanging": oi["n_hanging"],
               "steps": k, "ms": ms, "ms_per_step": ms / k}
        if every > 0 and n < n_explicit:
            th = time.perf_counter()
            lv = leaves_fn(prob, arc_length_at(prob, t0 + n * dt))
            T, rc = sim.remesh(lv, T, rc)
            torch.cuda.synchronize()
            T_tmp = torch.empty_like(T)
            blk["remesh_host_ms"] = (time.perf_counter() - th) * 1e3
        rec["blocks"].append(blk)
        if log:
            log(blk)
    t = t0 + n_explicit * dt
    if n_implicit:
        sim.set_laser(-1, prob.radius, prob.absorptivity, prob.h_powder, prob.t_start, prob.tracks)  # cool-down
    for i in range(n_implicit):
        ms, (Tn, info) = _timed(lambda: sim.implicit_step(T, rc, t, dt_implicit, cg_rtol=cg_rtol, cg_max_it=cg_max_it,
                                                          picard_tol=picard_tol, picard_max_it=picard_max_it))
        T = Tn
        t += dt_implicit
        it = {"step": i, "t": t, "ms": ms, "picard": info["picard_iters"], "cg": info["cg_iters"],
              "rel_res": info["rel_res"]}
        rec["implicit"].append(it)
        if log:
            log(it)
    return T, rc, sim, rec
