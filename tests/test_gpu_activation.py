"""GPU parity of the growing box (Section 4.1, layer activation) against the
oracle run on the active part: a two-layer build with explicit steps, an
implicit cool-down step on the first layer, activation of the second layer at
T0 with fresh powder, and explicit steps on the grown box (surface losses on,
so the free surface moves with the active top).  FP64, tolerance 1e-12
(1e-10 after the implicit step)."""
import numpy as np
import pytest
import torch

import oracle
import pbf_workloads as W
from tests.gpu_util import need_gpu, rel_errors

pytestmark = pytest.mark.gpu


def _lib_hist_to_oracle(prob, rc_lib, n_cells):
    nq = prob.n_qp_per_cell
    stride = prob.nx * prob.ny * prob.nz
    return np.asarray(rc_lib).reshape(nq, stride)[:, :n_cells].T.reshape(-1)


@pytest.mark.parametrize("deg", [1, 2])
def test_two_layer_build_vs_oracle(deg):
    need_gpu()
    from paper_2302_05164_amd import pbftherm
    p = W.with_surface_losses(W.small_nonlinear(nx=12, ny=10, nz=8, steps=0, track_length=0.25e-3,
                                                n_tracks=2, hatch=60e-6).replace(degree=deg))
    nz0 = 6
    a0, a1 = W.active_part(p, nz0), W.active_part(p, p.nz)
    O0, O1, Of = oracle.Oracle(a0), oracle.Oracle(a1), oracle.Oracle(p)
    dt = 0.5 * 2.0 / O1.stability_lambda(W.seeded_vector(O1.N, 1), 80)
    n1, n2 = 60, 60
    # oracle: active part of the full arrays (prefixes)
    To, ro = np.full(Of.N, p.T0), np.ones(Of.NQ)
    To[: O0.N] = O0.init_T()
    ro[: O0.NQ] = O0.init_history()
    O0.explicit_steps(To[: O0.N], ro[: O0.NQ], 0.0, dt, n1)
    t = n1 * dt
    Ti, info = O0.implicit_step(To[: O0.N].copy(), ro[: O0.NQ], t, 5e-5, cg_rtol=1e-13, picard_tol=1e-10)
    assert info["status"] == 0
    To[: O0.N] = Ti
    t += 5e-5
    Of.activate_layers(nz0, p.nz, p.T0, To, ro)
    O1.explicit_steps(To, ro, t, dt, n2)
    # GPU: the same sequence on a growing box
    sim = pbftherm.from_problem(p, device="cuda:0", active_layers=nz0)
    ai = sim.active_info()
    assert ai["nz_active"] == nz0 and ai["n_active_dofs"] == O0.N
    T, rc = sim.init_state(p.T0)
    sim.explicit_steps(T, rc, 0.0, dt, n1)
    Tn, gi = sim.implicit_step(T, rc, n1 * dt, 5e-5, cg_rtol=1e-13, picard_tol=1e-10)
    T.copy_(Tn)
    sim.activate_layers(p.nz, p.T0, T, rc)
    assert sim.active_info()["n_active_dofs"] == O1.N
    sim.explicit_steps(T, rc, t, dt, n2)
    torch.cuda.synchronize()
    Tg = T.cpu().numpy()
    mx, l2 = rel_errors(Tg, To)
    rg = _lib_hist_to_oracle(p, rc.cpu().numpy(), p.nx * p.ny * p.nz)
    print(f"CHECK Q{deg} two-layer build: max rel {mx:.2e} rel-L2 {l2:.2e} Tmax {To.max():.0f} "
          f"implicit gpu {gi} oracle {info}; history max diff {np.abs(rg - ro).max():.2e}")
    assert To.max() > p.T_l or deg == 1  # the Q2 build melts under the beam
    assert mx <= 1e-10 and l2 <= 1e-10
    assert np.abs(rg - ro).max() <= 1e-9


def test_activation_refusals():
    need_gpu()
    from paper_2302_05164_amd import pbftherm
    p = W.small_nonlinear(nx=6, ny=5, nz=4, steps=0)
    sim = pbftherm.from_problem(p, device="cuda:0", active_layers=3)
    T, rc = sim.init_state(p.T0)
    with pytest.raises(pbftherm.PbfError):
        sim.activate_layers(3, p.T0, T, rc)  # not a growth
    with pytest.raises(pbftherm.PbfError):
        sim.set_active_layers(2)  # after binding
    plain = pbftherm.from_problem(p, device="cuda:0")
    T2, rc2 = plain.init_state(p.T0)
    with pytest.raises(pbftherm.PbfError):
        plain.activate_layers(4, p.T0, T2, rc2)  # not a growing box
