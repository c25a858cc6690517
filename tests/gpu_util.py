"""Helpers shared by the GPU parity tests: run a problem through the HIP library
and through the oracle on the same seeded inputs, and convert between the
library's compressed history and the oracle's per-point history."""
import numpy as np
import torch

import oracle
import pbf_workloads as W


def need_gpu():
    import pytest
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def sim_for(prob):
    from paper_2302_05164_amd import pbftherm
    return pbftherm.from_problem(prob, device="cuda:0")


def oracle_dt(prob, iters=100, seed=1):
    o = oracle.Oracle(prob)
    lam = o.stability_lambda(W.seeded_vector(o.N, seed), iters)
    return prob.dt_factor * 2.0 / lam


def history_to_full(prob, hist, n_hist_layers):
    """library history (point-major over the top layers) -> oracle rc (cell-major, all cells)"""
    nq = prob.n_qp_per_cell
    full = np.ones((prob.nz, prob.ny, prob.nx, nq))
    if n_hist_layers:
        h = np.asarray(hist[: nq * n_hist_layers * prob.ny * prob.nx]).reshape(
            nq, n_hist_layers, prob.ny, prob.nx)
        full[prob.nz - n_hist_layers:] = h.transpose(1, 2, 3, 0)
    return full.reshape(-1)


def full_to_history(prob, rc_full, n_hist_layers):
    nq = prob.n_qp_per_cell
    f = rc_full.reshape(prob.nz, prob.ny, prob.nx, nq)[prob.nz - n_hist_layers:]
    return np.ascontiguousarray(f.transpose(3, 0, 1, 2)).reshape(-1)


def rel_errors(a, ref):
    """(max |a - ref| / max |ref|, ||a - ref||_2 / ||ref||_2, same two against the rise ref - T0)"""
    d = a - ref
    return (np.abs(d).max() / np.abs(ref).max(), np.linalg.norm(d) / np.linalg.norm(ref))
