"""torch.autograd interface to the field-driven dynamics of the library.

dipole_after_pulse(A, ...) returns D(A) = <psi_N|mu|psi_N> / <psi_N|psi_N> after N RK4 steps
under H(t) = H0 + A f(t) M as a differentiable scalar: backward() calls the library's adjoint
of the discrete RK4 map (tdmps_pulse_backward).  Only argument marshalling happens here; the
propagation, the adjoint and every contraction run in the library.
"""
from __future__ import annotations

import torch

from . import tdmps as T


class _DipoleAfterPulse(torch.autograd.Function):
    @staticmethod
    def forward(ctx, amplitude, H0, h0, m, mu, psi0, omega, t_center, width, dt, nsteps, checkpoint_every, params):
        traj = T.Trajectory(H0, h0, m, mu, psi0, float(amplitude.item()), omega, t_center, width, dt, nsteps,
                            checkpoint_every, params)
        ctx.traj = traj
        return torch.tensor(traj.value, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.traj.backward()
        ctx.traj = None
        return (grad_out * g,) + (None,) * 12


def dipole_after_pulse(amplitude: torch.Tensor, H0, h0, m, mu, psi0, omega, t_center, width, dt, nsteps,
                       checkpoint_every=20, params=None) -> torch.Tensor:
    """D(amplitude) as a torch scalar (float64) with a backward through the library's adjoint."""
    return _DipoleAfterPulse.apply(amplitude, H0, h0, m, mu, psi0, omega, t_center, width, dt, nsteps,
                                   checkpoint_every, params)
