"""Benchmark: explicit-step throughput of the matrix-free PBF thermal operator.

One "step" is one forward-Euler step of the whole hot path (sum-factorized
operator, material law, laser source, lumped-mass update, tile-face completion)
over the full mesh.  The default workload is the 160x160x80 Q2 box
(16,589,601 DoFs, 4x4x2 mm) with the seeded nonlinear law and the 10-track
zigzag scan; the value is whole-job DoF-updates/s in FP64, inputs resident in
HBM.  The FP32-operator variant is timed on the same workload and reported
beside it, with its error against the FP64 run after 5000 steps.

Prints one JSON line.  --gpus N with N > 1 exits: the build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TIMING_EVERY = 10  # kernel events on every 10th timed step

# peaks of one MI355X (public figures)
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def algorithmic_counts(prob, info):
    """Per-step algorithmic bytes and flops of the explicit step:
    bytes: read T_n and write T_{n+1} (8 B each per DoF) plus one read of the
    powder history (8 B per stored quadrature point);
    flops: the sum-factorized Q2 cell operator, 1755 flop per cell (interpolation
    270, collocation gradients 405, flux and one law hinge 324, collocation
    transpose 486, integration 270), plus 12 flop per node for the lumped
    capacity and the update.  Q1: 8 x the 1D work of 2-point lines."""
    n = info["n_dofs"]
    bytes_step = 16.0 * n + 8.0 * info["n_hist_qp"]
    if prob.degree == 2:
        per_cell = 1755.0
    else:
        # Q1: 3 sweeps x 4 lines x 2 outputs x 3 flop, gradients 3 x 4 x 2 x 3,
        # flux 8 x 12, transpose 3 x 8 x 2 x 2, integration 3 x 4 x 2 x 3
        per_cell = 72 + 72 + 96 + 96 + 72
    flops_step = per_cell * info["n_cells"] + 12.0 * n
    return bytes_step, flops_step


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, dt, steps=5):
    """The oracle (plain serial C, one thread) timed on a bounded sample of the
    workload: `steps` explicit steps of the full mesh at the benchmark's dt from
    a seeded hot state (a melt pool under the beam, so the nonlinear law, the
    latent heat and the source are all active)."""
    import oracle
    import pbf_workloads as W

    o = oracle.Oracle(prob)
    T, t0 = W.hot_spot_state(prob, seed=17)
    rc = o.init_history()
    t = time.perf_counter()
    o.explicit_steps(T, rc, t0, dt, steps)
    el = time.perf_counter() - t
    return {"value": o.N * steps / el, "unit": "DoF-updates/s", "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{steps} explicit steps of {prob.name} ({o.N} DoFs, full mesh) at dt = {dt:.4e} s from "
                      f"a seeded melt-pool state, serial C on one thread, {el:.2f} s"}


# every source file the explicit cell kernel is compiled from
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2302_05164_amd", "csrc", f)
                  for f in ("cells.h", "cells_q2_f64.hip", "cellkit.h", "pbf_internal.h")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def pmc_summary(fetch_dir, write_dir, out_path, workload, kernel="k_cells<2, double, 0"):
    """Summarize two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of
    `bench.py --calib-copy`: per-dispatch KiB of the cell kernel, scaled by the
    counter/true-bytes ratio of the 1 GiB device copy of the same run."""
    import csv
    import glob

    def read(d, name):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += [r for r in csv.DictReader(open(f)) if r["Counter_Name"] == name]
        return rows

    run = (f"python3 <repo>/bench.py --workload {workload} --steps 30 --warmup 5 --no-cpu --no-fp32 --no-adjoint "
           "--no-implicit --no-octree --no-laplace --calib-copy")
    res = {"workload": workload, "kernel": kernel, "kernel_source_sha256_16": kernel_source_hash(),
           "commands": ["cd /tmp && export TMPDIR=/tmp",
                        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/fetch -o run -- {run}",
                        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/write -o run -- {run}",
                        f"python3 <repo>/bench.py --pmc-summary <out>/fetch <out>/write {os.path.basename(out_path)}"]}
    for d, name in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        rows = read(d, name)
        copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        calib_kib = max(copy)  # the 1 GiB copy is the largest copy dispatch
        scale = (1 << 20) / calib_kib  # true KiB per counted KiB
        kv = [float(r["Counter_Value"]) for r in rows if kernel in r["Kernel_Name"]]
        res[name] = {"kib_per_dispatch": sum(kv) / len(kv), "dispatches": len(kv),
                     "copy_1GiB_counter_kib": calib_kib, "scale": scale,
                     "bytes_per_dispatch": sum(kv) / len(kv) * scale * 1024.0}
    res["traffic_bytes_per_dispatch"] = (res["FETCH_SIZE"]["bytes_per_dispatch"] +
                                         res["WRITE_SIZE"]["bytes_per_dispatch"])
    json.dump(res, open(out_path, "w"), indent=1)
    print(json.dumps(res))


def sq_summary(dirs, out_path, workload, kernel="k_cells<2, double, 0"):
    """Summarize rocprofv3 --pmc runs of SQ counters (one directory per run) of
    `bench.py --workload W --steps 30 --warmup 5` with every other leg off: the
    per-dispatch mean of each counter over the cell kernel's launches, and the
    instruction mix per wavefront."""
    import csv
    import glob

    per = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if kernel in r["Kernel_Name"]:
                    per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    mean = {k: sum(v) / len(v) for k, v in per.items()}
    res = {"workload": workload, "kernel": kernel, "kernel_source_sha256_16": kernel_source_hash(),
           "dispatches": {k: len(v) for k, v in per.items()}, "per_dispatch": mean}
    w = mean.get("SQ_WAVES")
    if w:
        res["per_wave"] = {k: v / w for k, v in mean.items() if k.startswith("SQ_INSTS") or k.startswith("SQ_WAIT")}
    valu = mean.get("SQ_INSTS_VALU")
    if valu:
        fma, mul, add = (mean.get("SQ_INSTS_VALU_%s_F64" % k, 0.0) for k in ("FMA", "MUL", "ADD"))
        res["fp64_share_of_valu"] = (fma + mul + add) / valu
        res["fp64_flop_per_valu"] = (2 * fma + mul + add) / valu
        res["int_share_of_valu"] = (mean.get("SQ_INSTS_VALU_INT32", 0.0) + mean.get("SQ_INSTS_VALU_INT64", 0.0)) / valu
    if mean.get("SQ_WAVE_CYCLES"):
        res["wait_any_over_wave_cycles"] = mean.get("SQ_WAIT_ANY", 0.0) / mean["SQ_WAVE_CYCLES"]
    json.dump(res, open(out_path, "w"), indent=1)
    print(json.dumps(res))


def measured_traffic(workload):
    """Counter-based HBM bytes per cell-kernel launch from the committed
    summary, if it was taken on the current kernel source, else None."""
    path = os.path.join(ROOT, "profiles", f"k_cells_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d["traffic_bytes_per_dispatch"]


def copy_calibration(nbytes=1 << 30, reps=3):
    """Plain device copy of known size, for scaling HBM counters (FETCH_SIZE,
    WRITE_SIZE) of a profiled run."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return nbytes


def fp32_errors(sim, prob, dt, steps):
    """Error of the FP32-operator run against the FP64 run after `steps` steps
    from the initial state (the FP64 path is the one checked against the oracle
    step by step, at these sizes on the whole field): max and relative-L2 error
    over the whole field and over the melt pool {T_fp64 >= T_s}."""
    import torch

    out = {}
    for prec in (64, 32):
        T, rc = sim.init_state(prob.T0)
        sim.explicit_steps(T, rc, 0.0, dt, steps, precision=prec)
        out[prec] = T
    torch.cuda.synchronize()
    a, b = out[32], out[64]
    d = a - b
    pool = b >= prob.T_s
    res = {"steps": steps, "dt": dt, "reference": "fp64 run of the same steps",
           "max_abs_K": d.abs().max().item(),
           "max_rel": (d.abs().max() / b.abs().max()).item(),
           "rel_l2": (torch.linalg.norm(d) / torch.linalg.norm(b)).item(),
           "max_rel_to_rise": (d.abs().max() / (b - prob.T0).abs().max()).item(),
           "melt_pool_nodes": int(pool.sum().item())}
    if res["melt_pool_nodes"]:
        dp, bp = d[pool], b[pool]
        res["melt_pool_max_abs_K"] = dp.abs().max().item()
        res["melt_pool_max_rel"] = (dp.abs().max() / bp.abs().max()).item()
        res["melt_pool_rel_l2"] = (torch.linalg.norm(dp) / torch.linalg.norm(bp)).item()
    res["T_max_fp64"] = b.max().item()
    # sensitivity of the model itself: the FP64 run from the same initial state
    # perturbed by seeded +-1e-9 K (3e-12 relative, the FP64 parity scale); the
    # apparent capacity jumps at T_s and T_l, so a node crossing them one step
    # earlier or later changes its increment by a finite amount
    import pbf_workloads as W
    T, rc = sim.init_state(prob.T0)
    T += torch.tensor(1e-9 * W.seeded_vector(T.numel(), 41), device=T.device)
    sim.explicit_steps(T, rc, 0.0, dt, steps, precision=64)
    torch.cuda.synchronize()
    dq = T - b
    res["fp64_perturbed_1e-9K"] = {"max_abs_K": dq.abs().max().item(),
                                   "rel_l2": (torch.linalg.norm(dq) / torch.linalg.norm(b)).item()}
    # one step of each operator from the same (FP64) state
    one = {}
    for prec in (64, 32):
        T1, r1 = b.clone(), rc.clone()
        sim.explicit_steps(T1, r1, steps * dt, dt, 1, precision=prec)
        one[prec] = T1
    torch.cuda.synchronize()
    d1 = one[32] - one[64]
    inc = one[64] - b
    res["one_step"] = {"max_abs_K": d1.abs().max().item(),
                       "max_rel": (d1.abs().max() / one[64].abs().max()).item(),
                       "max_rel_to_increment": (d1.abs().max() / inc.abs().max()).item()}
    return res


def adjoint_timing(reps=1):
    """Adjoint/forward time ratio on the differentiation workload: the 48x48x24 Q2
    box with the seeded nonlinear law, 3000 explicit steps, 64 probes, gradients
    with respect to 10 track powers and the absorptivity, 30 checkpoint slots.
    Times (HIP events on the library's stream): the forward sweep (steps,
    snapshots, objective), the backward sweep (replays and adjoint steps), and
    3000 plain explicit steps."""
    import torch

    import pbf_workloads as W
    from paper_2302_05164_amd import pbftherm

    prob = W.cfg5()
    sim = pbftherm.from_problem(prob, device="cuda:0")
    info = sim.info()
    v0 = torch.tensor(W.seeded_vector(info["n_dofs"], 1), device="cuda")
    dt = prob.dt_factor * sim.stability_dt(v0, 100)
    sim.set_probes(prob.probes, prob.targets)
    n, s = prob.steps, 30
    work = sim.gradient_work(s)

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        out = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), out

    res = []
    for it in range(reps + 1):  # first repetition is warm-up
        T0, rc0 = sim.init_state(prob.T0)
        t_fwd, (TN, J) = timed(lambda: sim.gradient_forward(T0, rc0, 0.0, dt, n, work))
        t_bwd, g = timed(lambda: sim.gradient_backward(0.0, dt, n, work))
        T, rc = sim.init_state(prob.T0)
        T_tmp = torch.empty_like(T)
        t_plain, _ = timed(lambda: sim.explicit_steps(T, rc, 0.0, dt, n, T_tmp=T_tmp))
        if it > 0:
            res.append((t_fwd, t_bwd, t_plain, J.item(), g))
    t_fwd, t_bwd, t_plain, J, g = res[-1]
    return {"workload": prob.name, "n_dofs": info["n_dofs"], "steps": n, "checkpoint_slots": s,
            "parameters": len(prob.tracks) + 1, "forward_ms": t_fwd, "backward_ms": t_bwd,
            "plain_forward_ms": t_plain, "adjoint_forward_ratio": t_bwd / t_fwd,
            "total_over_plain_forward": (t_fwd + t_bwd) / t_plain,
            "forward_steps_total": g["n_advances"], "work_bytes": work["bytes"], "J": J,
            "dJdA": g["dJdA"].item(), "dJdP_norm": float(torch.linalg.norm(g["dJdP"]).item())}


def implicit_timing(sim, T, rc, t, dt=1e-4):
    """One backward-Euler step of dt from the end state of the explicit run,
    solved by Picard iterations with CG and by Newton's method with restarted
    GMRES(30) (relative residual 1e-10 per linear system, 1e-8 K on the
    update), each with the Jacobi preconditioner and with the geometric
    multigrid V-cycle, and Newton with multigrid and Eisenstat-Walker forcing
    (inexact Newton); wall time on the library's stream, iteration counts."""
    import torch

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        out = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), out

    res = {"dt": dt}
    roots = {}
    for kind in ("jacobi", "multigrid"):
        sim.set_preconditioner(kind)
        work = sim.newton_work(30)
        r1 = rc.clone()
        ms, (Tp, ip) = timed(lambda: sim.implicit_step(T, r1, t, dt, cg_rtol=1e-10, picard_tol=1e-8,
                                                       picard_max_it=60))
        res[f"picard_cg_{kind}"] = {"ms": ms, "outer": ip["picard_iters"], "krylov": ip["cg_iters"],
                                    "ms_per_krylov": ms / max(1, ip["cg_iters"])}
        r2 = rc.clone()
        ms, (Tn, inw) = timed(lambda: sim.implicit_step_newton(T, r2, t, dt, lin_rtol=1e-10, restart=30,
                                                               newton_tol=1e-8, newton_max_it=60, work=work))
        res[f"newton_gmres_{kind}"] = {"ms": ms, "outer": inw["newton_iters"], "krylov": inw["lin_iters"],
                                       "ms_per_krylov": ms / max(1, inw["lin_iters"]), "work_bytes": work["bytes"]}
        roots[kind] = (Tp, Tn)
        if kind == "multigrid":
            sim.set_newton_forcing("eisenstat-walker")
            r3 = rc.clone()
            ms, (Te, ie) = timed(lambda: sim.implicit_step_newton(T, r3, t, dt, lin_rtol=1e-10, restart=30,
                                                                   newton_tol=1e-8, newton_max_it=60, work=work))
            sim.set_newton_forcing("fixed")
            res["newton_gmres_multigrid_ew"] = {"ms": ms, "outer": ie["newton_iters"], "krylov": ie["lin_iters"],
                                                "ms_per_krylov": ms / max(1, ie["lin_iters"])}
            roots["ew"] = Te
        del work
    sim.set_preconditioner("jacobi")
    res["max_abs_diff_K"] = {
        "picard_vs_newton": float((roots["jacobi"][0] - roots["jacobi"][1]).abs().max().item()),
        "multigrid_vs_jacobi_picard": float((roots["multigrid"][0] - roots["jacobi"][0]).abs().max().item()),
        "multigrid_vs_jacobi_newton": float((roots["multigrid"][1] - roots["jacobi"][1]).abs().max().item()),
        "multigrid_ew_vs_jacobi_newton": float((roots["ew"] - roots["jacobi"][1]).abs().max().item())}
    j, m = res["picard_cg_jacobi"], res["newton_gmres_multigrid_ew"]
    res["best_over_jacobi_picard"] = {"krylov": j["krylov"] / max(1, m["krylov"]), "time": j["ms"] / m["ms"]}
    return res


def laplace_timing(sim, info, prob, steps, warmup, step_ms, step_cell_ms):
    """The constant-coefficient reference operator y = K x (unit conductivity,
    no law, history, source, capacity or update) on the same mesh with the same
    column kernels, timed like the explicit step; the explicit step's
    throughput as a fraction of it (Section 5.1 reports 44% on CPUs)."""
    import torch

    x = torch.rand(info["n_dofs"], dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(warmup):
        sim.laplace_apply(x, y)
    torch.cuda.synchronize()
    sim.timing_begin(steps, every=TIMING_EVERY)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        sim.laplace_apply(x, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    cell_ms, face_ms, _ = sim.timing_end()
    n = info["n_dofs"]
    return {"operator": "y = K x, unit conductivity, Q%d" % prob.degree, "ms_per_apply": ms,
            "value": n / (ms / 1e3), "unit": "DoF/s", "kernel_ms": cell_ms, "face_kernel_ms": face_ms,
            "explicit_step_fraction_of_laplace": ms / step_ms,
            "explicit_kernel_fraction_of_laplace_kernel": cell_ms / step_cell_ms}


def octree_timing(n_explicit=200, n_implicit=1):
    """The octree schedule on the octree workload (Q2 over a 10x10x5 mm part,
    coarse 20x20x10 cells refined to level 6 within 200 um of the window
    [s - 8 mm, s + 100 um] of the scan path around the beam's arc length s,
    about 5.2M dofs): a bounded sample of the stated 2000 explicit steps with a
    remesh every 100 and 50 backward-Euler steps of 1 ms (Jacobi-CG to 1e-10),
    namely the first n_explicit steps (with their remeshes) and the first
    n_implicit implicit steps.  GPU times from HIP events on the library's
    stream; remesh times are host wall time (mesh build and transfer)."""
    import pbf_workloads as W
    from paper_2302_05164_amd import octree_schedule as S

    prob = W.cfg3()
    T, rc, sim, rec = S.run(prob, n_explicit=n_explicit, n_implicit=n_implicit)
    blocks, imp = rec["blocks"], rec["implicit"]
    ms_expl = sum(b["ms"] for b in blocks) / n_explicit
    dofs = [b["dofs"] for b in blocks]
    out = {"workload": prob.name, "dt": rec["dt"], "explicit_steps": n_explicit,
           "remesh_every": prob.remesh_every, "dofs_per_block": dofs,
           "leaves_per_block": [b["leaves"] for b in blocks],
           "hanging_per_block": [b["hanging"] for b in blocks],
           "ms_per_explicit_step": ms_expl,
           "value": sum(b["dofs"] * b["steps"] for b in blocks) / (sum(b["ms"] for b in blocks) / 1e3),
           "unit": "DoF-updates/s",
           "remesh_host_ms": [round(b["remesh_host_ms"], 1) for b in blocks if "remesh_host_ms" in b],
           "setup_host_ms": rec["setup_host_ms"],
           "finite": bool(torch_isfinite(T)), "T_max": float(T.max().item())}
    if imp:
        ms_imp = sum(r["ms"] for r in imp) / len(imp)
        out["implicit"] = {"dt": prob.implicit_dt, "steps": len(imp), "ms_per_step": ms_imp,
                           "picard_iters": [r["picard"] for r in imp], "cg_iters": [r["cg"] for r in imp],
                           "ms_per_cg_iter": sum(r["ms"] for r in imp) / max(1, sum(r["cg"] for r in imp)),
                           "implicit_over_explicit_step": ms_imp / ms_expl}
    return out


def torch_isfinite(T):
    import torch
    return torch.isfinite(T).all().item()


def progress(msg):
    """One progress line on stderr (the JSON result is the only stdout line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="cfg4", choices=["cfg2", "cfg4", "cfg5", "cfg1"])
    ap.add_argument("--fp32-error-steps", type=int, default=5000,
                    help="steps of the FP32-operator vs FP64 error statement (0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-operator timing")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward timing")
    ap.add_argument("--no-implicit", action="store_true", help="skip the implicit-step timing")
    ap.add_argument("--no-octree", action="store_true", help="skip the octree-mesh timing")
    ap.add_argument("--no-laplace", action="store_true", help="skip the Laplace reference operator timing")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 1 GiB device copy first (HBM counter calibration)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON"),
                    help="summarize rocprofv3 FETCH_SIZE/WRITE_SIZE runs and exit")
    ap.add_argument("--sq-summary", nargs="+", metavar="DIR_OR_OUT",
                    help="summarize rocprofv3 SQ counter runs (directories, then the output JSON) and exit")
    args = ap.parse_args()
    if args.pmc_summary:
        prob_name = {"cfg1": "cfg1", "cfg2": "cfg2", "cfg4": "cfg4", "cfg5": "cfg5"}[args.workload]
        pmc_summary(*args.pmc_summary, workload=prob_name)
        return
    if args.sq_summary:
        sq_summary(args.sq_summary[:-1], args.sq_summary[-1], workload=args.workload)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (the library has no multi-GPU path); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import pbf_workloads as W
    from paper_2302_05164_amd import pbftherm

    if args.calib_copy:
        copy_calibration()

    prob = W.CONFIGS[args.workload]()
    sim = pbftherm.from_problem(prob, device="cuda:0")
    info = sim.info()
    # time step: half the explicit stability limit (power iteration on the GPU)
    v0 = torch.tensor(W.seeded_vector(info["n_dofs"], 1), device="cuda")
    dt = prob.dt_factor * sim.stability_dt(v0, 100)
    del v0

    results = {}
    for prec in ([64] if args.no_fp32 else [64, 32]):
        T, rc = sim.init_state(prob.T0)
        T_tmp = torch.empty_like(T)
        sim.explicit_steps(T, rc, 0.0, dt, args.warmup, precision=prec, T_tmp=T_tmp)
        torch.cuda.synchronize()
        # timed region: K steps; the library records HIP events on its stream
        # around the kernels of every 10th step (events on every step would add
        # ~20 us per step of launch gaps to the timed region)
        sim.timing_begin(args.steps, every=TIMING_EVERY)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        sim.explicit_steps(T, rc, args.warmup * dt, dt, args.steps, precision=prec, T_tmp=T_tmp)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        cell_ms, face_ms, nt = sim.timing_end()
        finite = bool(torch.isfinite(T).all().item())
        results[prec] = dict(ms=ms, cell_ms=cell_ms, face_ms=face_ms, n=nt, finite=finite,
                             Tmax=float(T.max().item()))
        progress(f"fp{prec} operator: {ms / args.steps:.4f} ms per step")
        if prec == 64:
            end_state = (T.clone(), rc.clone())
        del T, rc, T_tmp

    n = info["n_dofs"]
    r64 = results[64]
    ms_step = r64["ms"] / args.steps
    value = n * args.steps / (r64["ms"] / 1e3)
    bytes_step, flops_step = algorithmic_counts(prob, info)
    cell_s = r64["cell_ms"] / 1e3
    hbm_gbs = bytes_step / cell_s / 1e9
    tflops = flops_step / cell_s / 1e12
    frac_hbm = hbm_gbs / HBM_PEAK_GBS
    frac_alu = tflops / FP64_PEAK_TFLOPS
    if frac_alu >= frac_hbm:
        roof = {"bound": "alu", "achieved": round(tflops, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(frac_alu, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(frac_hbm, 4)}
    roof["traffic"] = measured_traffic(args.workload)
    roof["kernel"] = "k_cells<2,double,0>" if prob.degree == 2 else "k_cells<1,double,0>"
    roof["kernel_ms"] = round(r64["cell_ms"], 5)
    roof["face_kernel_ms"] = round(r64["face_ms"], 5)
    roof["algorithmic_bytes_per_launch"] = bytes_step
    roof["algorithmic_flops_per_launch"] = flops_step
    roof["hbm_frac_algorithmic"] = round(frac_hbm, 4)
    roof["fp64_frac_algorithmic"] = round(frac_alu, 4)

    out = {
        "metric": "DoF-updates/s per explicit step (Q2, FP64 vs FP32-op); adjoint/forward time ratio",
        "value": value,
        "unit": "DoF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": prob.name, "degree": prob.degree,
                   "cells": [prob.nx, prob.ny, prob.nz], "n_dofs": n, "dt": dt,
                   "operator_precision": "fp64", "finite": r64["finite"],
                   "T_max": r64["Tmax"]},
        "roofline": roof,
    }
    if 32 in results:
        r32 = results[32]
        v32 = n * args.steps / (r32["ms"] / 1e3)
        out["fp32_operator"] = {"value": v32, "unit": "DoF-updates/s",
                                "ms_per_step": r32["ms"] / args.steps,
                                "speedup_vs_fp64": v32 / value,
                                "kernel_ms": r32["cell_ms"], "finite": r32["finite"]}
        if args.fp32_error_steps > 0:
            out["fp32_operator"]["error_vs_fp64"] = fp32_errors(sim, prob, dt, args.fp32_error_steps)
            progress("fp32 error statement done")
    if not args.no_laplace:
        out["laplace_reference"] = laplace_timing(sim, info, prob, args.steps, args.warmup, ms_step,
                                                  r64["cell_ms"])
        progress("laplace reference done")
    if not args.no_implicit:
        out["implicit"] = implicit_timing(sim, *end_state, (args.warmup + args.steps) * dt)
        progress("implicit step done")
    del end_state
    if not args.no_adjoint:
        out["adjoint"] = adjoint_timing()
        progress("adjoint done")
    if not args.no_octree:
        out["octree"] = octree_timing()
        progress("octree done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, dt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
