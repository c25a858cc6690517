"""GPU checks of the diagnostics: per-step energy terms against the oracle's
assembled vectors, the per-step energy identity, and the finite-value check."""
import numpy as np
import pytest
import torch

import oracle
import pbf_workloads as W
from tests.gpu_util import full_to_history, need_gpu, oracle_dt, sim_for

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("degree", [1, 2])
def test_energy_terms_vs_oracle(degree):
    need_gpu()
    prob = W.small_nonlinear(nx=20, ny=18, nz=10, steps=0).replace(degree=degree)
    o = oracle.Oracle(prob)
    dt = oracle_dt(prob)
    T = o.init_T()
    rc = o.init_history()
    o.explicit_steps(T, rc, 0.0, dt, 40)  # melt pool and consolidated powder present
    t = 40 * dt
    # oracle: f, C~, f_vol at the step start (history updated as in the step)
    ro = rc.copy()
    f, Cl, fv = o.assemble(T, ro, t)
    T1 = T.copy()
    o.explicit_steps(T1, rc.copy(), t, dt, 1)
    free = ~o.dirichlet_mask()
    ref = (np.sum(Cl[free] * (T1 - T)[free]), np.sum(fv[free]), -np.sum((f - fv)[free]))
    # GPU: one step from the same state, then the energy terms
    sim = sim_for(prob)
    info = sim.info()
    Tp = torch.tensor(T, device="cuda")
    hist = full_to_history(prob, rc, info["n_hist_layers"])
    rd = torch.tensor(hist if hist.size else np.zeros(1), device="cuda")
    Tn = Tp.clone()
    sim.explicit_steps(Tn, rd, t, dt, 1)
    e = sim.energy(Tp, Tn, rd, t, dt)
    print(f"Q{degree}: gpu {e} oracle {ref}")
    assert ref[1] > 0 and ref[2] != 0
    for k in range(3):
        assert abs(e[k] - ref[k]) <= 1e-10 * max(abs(ref[k]), abs(dt * ref[1]))
    assert abs(e[3]) <= 1e-11 * dt * (abs(e[1]) + abs(e[2]))
    # the diffusion rows sum to zero: the Dirichlet heat flow is the reaction there
    assert abs(ref[2] - np.sum((f - fv)[~free])) <= 1e-12 * np.abs(f - fv).sum()


def test_check_finite():
    need_gpu()
    prob = W.small_nonlinear(nx=12, ny=10, nz=6, steps=0)
    sim = sim_for(prob)
    T, rc = sim.init_state(prob.T0)
    ok, mx = sim.check_finite(T)
    assert ok and mx == prob.T0
    T[17] = float("nan")
    T[23] = -5000.0
    ok, mx = sim.check_finite(T)
    assert not ok and mx == 5000.0
