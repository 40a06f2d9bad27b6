"""torch.autograd.Function over ifdlbm_gradient: the kinetic energy of a cavity
after a fixed number of steps as a differentiable function of the top angle
theta (radians), the power-law index n and the lid speed U."""
from __future__ import annotations

import math

import torch

from . import ifdlbm as _m


class CavityKineticEnergy(torch.autograd.Function):
    """J = E(theta, n, U) of Eq. (5.1) after `steps` steps; backward returns dJ/d(theta, n, U)
    from the tangent-linear sweep of the library (no CPU arithmetic)."""

    @staticmethod
    def forward(ctx, theta, n, u_lid, n_xi: int, n_eta: int, re: float, steps: int, options=None):
        cav = _m.Cavity(int(n_xi), int(n_eta), float(re), float(n), math.degrees(float(theta)), float(u_lid))
        J, grad = _m.ifdlbm_gradient(cav, options, int(steps))
        ctx.save_for_backward(torch.tensor(grad, dtype=torch.float64))
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        gJ = gJ.to(torch.float64)
        return gJ * g[0], gJ * g[1], gJ * g[2], None, None, None, None, None


def cavity_kinetic_energy(theta, n, u_lid, n_xi: int, n_eta: int, re: float, steps: int, options=None):
    return CavityKineticEnergy.apply(theta, n, u_lid, n_xi, n_eta, re, steps, options)
