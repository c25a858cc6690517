"""pbf_explicit_steps_noalloc (the explicit steps for callers that cannot
allocate device memory, scratch in the library's static device array) against
pbf_explicit_steps on the same seeded inputs, through the C ABI: two calls in a
row on one GPU, the second on a smaller mesh (the array keeps the first call's
contents), each within the FP64 parity bar (1e-12 relative) of the
workspace-bound steps, which run the same kernels."""
import numpy as np
import pytest
import torch

import pbf_workloads as W
from paper_2302_05164_amd import pbftherm
from tests.gpu_util import need_gpu, oracle_dt, rel_errors, sim_for

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _compare(prob, steps, precision):
    dt = oracle_dt(prob)
    ref = sim_for(prob)
    T, rc = ref.init_state(prob.T0)
    T_na, rc_na = T.clone(), rc.clone()
    ref.explicit_steps(T, rc, 0.0, dt, steps, precision=precision)
    na = pbftherm.from_problem(prob, device="cuda:0", bind=False)
    T0_na, _ = na.init_state(prob.T0)  # no workspace needed on boxes; sets the FP32 reference
    assert torch.equal(T0_na, T_na)
    need = na.explicit_steps_noalloc(T_na, rc_na, 0.0, dt, steps, torch.empty_like(T_na), precision=precision)
    torch.cuda.synchronize()
    a, b = T_na.cpu().numpy(), T.cpu().numpy()
    mx, l2 = rel_errors(a, b)
    print(f"{prob.name} {prob.nx}x{prob.ny}x{prob.nz} Q{prob.degree} fp{precision}: {steps} steps, "
          f"scratch {need} B, max rel {mx:.2e} rel-L2 {l2:.2e}, bitwise {np.array_equal(a, b)}, "
          f"T max {b.max():.1f} K", flush=True)
    assert b.max() > prob.T0 + 50.0  # the beam heated the box
    assert mx <= TOL and l2 <= TOL
    if rc.numel():
        assert np.abs(rc_na.cpu().numpy() - rc.cpu().numpy()).max() <= TOL
    return need


def test_noalloc_steps_match_bound_steps_twice_second_smaller():
    need_gpu()
    big = W.small_nonlinear(nx=20, ny=18, nz=10, steps=0, track_length=0.5e-3)
    small = W.small_nonlinear(nx=9, ny=7, nz=4, steps=0, track_length=0.2e-3)
    n_big = _compare(big, 80, 64)
    n_small = _compare(small, 60, 64)
    assert n_small < n_big
    _compare(small, 60, 32)  # FP32 operator: the FP32 law copy lives in the array too


def test_noalloc_refusals_leave_the_bound_path_intact():
    need_gpu()
    prob = W.small_nonlinear(nx=9, ny=7, nz=4, steps=0, track_length=0.2e-3)
    sim = sim_for(prob)  # bound workspace
    T, rc = sim.init_state(prob.T0)
    T2, rc2 = T.clone(), rc.clone()
    dt = oracle_dt(prob)
    sim.explicit_steps_noalloc(T2, rc2, 0.0, dt, 30, torch.empty_like(T2))
    sim.explicit_steps(T, rc, 0.0, dt, 30)  # the bound workspace's laws are still in place
    torch.cuda.synchronize()
    assert np.array_equal(T.cpu().numpy(), T2.cpu().numpy())
    with pytest.raises(pbftherm.PbfError, match="T_tmp"):
        sim.explicit_steps_noalloc(T, rc, 0.0, dt, 1, T)
