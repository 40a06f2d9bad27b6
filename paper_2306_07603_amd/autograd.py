"""torch.autograd.Function over the library's discrete adjoint: the kinetic
energy of a cavity (Eq. 5.1) after a fixed number of steps as a
differentiable function of the top angle theta (radians), the power-law index
n and the lid speed U."""
from __future__ import annotations

import math

import torch

from . import ifdlbm as _m


def _cavity(theta, n, u_lid, n_xi, n_eta, re):
    return _m.Cavity(int(n_xi), int(n_eta), float(re), float(n), math.degrees(float(theta)), float(u_lid))


class CavityKineticEnergy(torch.autograd.Function):
    """J = E(theta, n, U) after `steps` steps.  When any input needs a gradient,
    forward runs ifdlbm_adjoint (forward sweep with a checkpoint every
    `checkpoint_every` steps, then the reverse sweep) and keeps dJ/d(theta, n, U)
    for backward; method="tangent" takes the tangent-linear sweep instead.
    Otherwise only the forward steps run.  All arithmetic is on the GPU."""

    @staticmethod
    def forward(ctx, theta, n, u_lid, n_xi: int, n_eta: int, re: float, steps: int, options=None,
                checkpoint_every: int = 500, method: str = "adjoint"):
        cav = _cavity(theta, n, u_lid, n_xi, n_eta, re)
        if any(ctx.needs_input_grad[:3]):
            if method == "adjoint":
                J, grad = _m.ifdlbm_adjoint(cav, options, int(steps), int(checkpoint_every))
            elif method == "tangent":
                J, grad = _m.ifdlbm_gradient(cav, options, int(steps))
            else:
                raise ValueError("method must be 'adjoint' or 'tangent'")
            ctx.save_for_backward(torch.tensor(grad, dtype=torch.float64))
            return torch.tensor(J, dtype=torch.float64)
        h = _m.ifdlbm_create([cav], options)
        try:
            _m.ifdlbm_step(h, int(steps))
            J = _m.ifdlbm_kinetic_energy(h, 0)
        finally:
            h.close()
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        gJ = gJ.to(torch.float64)
        return gJ * g[0], gJ * g[1], gJ * g[2], None, None, None, None, None, None, None


def cavity_kinetic_energy(theta, n, u_lid, n_xi: int, n_eta: int, re: float, steps: int, options=None,
                          checkpoint_every: int = 500, method: str = "adjoint"):
    return CavityKineticEnergy.apply(theta, n, u_lid, n_xi, n_eta, re, steps, options, checkpoint_every, method)
