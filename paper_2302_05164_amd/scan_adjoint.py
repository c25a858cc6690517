"""torch.autograd interface to the checkpointed discrete adjoint.

J(P, A) = sum_p (T_h(x_p, t_N) - T*_p)^2 after n_steps explicit FP64 steps of
the scan with track powers P_k and absorptivity A (W_eff,k = A P_k).  The
forward pass runs the library's forward sweep (binomial checkpoints in a device
buffer), the backward pass its reversal; both are single library calls, the
gradient arithmetic runs in the library's kernels.  Only the product with the
incoming gradient dL/dJ is done here, as autograd's chain rule.
"""
from __future__ import annotations

import torch


class ScanAdjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, powers, absorptivity, sim, T0, rc0, t0, dt, n_steps, n_snaps):
        sim.set_track_powers(powers.detach().double().cpu().numpy(),
                             float(torch.as_tensor(absorptivity).item()))
        work = sim.gradient_work(n_snaps)
        _, J = sim.gradient_forward(T0, rc0, t0, dt, n_steps, work)
        ctx.sim, ctx.work, ctx.args = sim, work, (t0, dt, n_steps)
        ctx.p_meta = (powers.device, powers.dtype)
        a = torch.as_tensor(absorptivity)
        ctx.a_meta = (a.device, a.dtype)
        return J[0].to(powers.dtype)

    @staticmethod
    def backward(ctx, gJ):
        g = ctx.sim.gradient_backward(*ctx.args, ctx.work)
        ctx.work = None
        gJ = gJ.to(g["dJdP"].device, torch.float64)
        dP = (gJ * g["dJdP"]).to(*ctx.p_meta)
        dA = (gJ * g["dJdA"][0]).to(*ctx.a_meta)
        return dP, dA, None, None, None, None, None, None, None


def scan_objective(powers, absorptivity, sim, T0, rc0, t0, dt, n_steps, n_snaps=30):
    """J as a differentiable function of the track powers and the absorptivity."""
    return ScanAdjoint.apply(powers, absorptivity, sim, T0, rc0, t0, dt, n_steps, n_snaps)
