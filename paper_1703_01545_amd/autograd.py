"""dE/dlambda of the mixed energy behind torch.autograd (argument marshalling
only; the forward window and the reverse pass run in libafqmc)."""
from __future__ import annotations

import torch


class AfqmcEnergy(torch.autograd.Function):
    """E(lambda): mixed energy after a window of walker steps for the one-body
    perturbation h -> h + lambda V, evaluated at lambda = 0 (the system's own
    h; build the system with h + lambda0 V to differentiate elsewhere).

    AfqmcEnergy.apply(lam, system, V, n_steps, seed, checkpoint_every,
    precision) advances `system` n_steps; backward returns dE/dlambda from the
    library's reverse pass (snapshots every checkpoint_every steps)."""

    @staticmethod
    def forward(ctx, lam, system, V, n_steps, seed=0, checkpoint_every=10, precision="fp64"):
        if float(lam) != 0.0:
            raise ValueError("AfqmcEnergy differentiates at lambda = 0: build the system on "
                             "h + lambda0 V to move the expansion point")
        e = system.adjoint_forward(V, n_steps, seed=seed, checkpoint_every=checkpoint_every,
                                   precision=precision)
        ctx.system = system
        return torch.tensor(e, dtype=torch.float64, device=lam.device)

    @staticmethod
    def backward(ctx, grad):
        d = ctx.system.adjoint_backward()
        return grad * d, None, None, None, None, None, None
