"""The oracle's own discrete adjoint (test infrastructure only).

The paper has no adjoint; the hot path adds one.  Here it is obtained by
reverse-mode automatic differentiation (torch.autograd) of the oracle's
residual and SSP-RK3 step, so it is independent of the hand-written HIP
reverse pass.  Non-smooth points follow torch's conventions: the derivative
of max(a, b) is split 1/2, 1/2 at ties and that of |x| is 0 at x = 0.

The surface-tension coefficient enters the residual linearly through the CSF
source, so its cotangent is <R_bar, dR/dsigma>.
"""

import dataclasses

import torch

from .residual import rhs
from .stepper import rk_step


def _with_sigma(prm, sigma):
    return dataclasses.replace(prm, sigma=sigma)


def rhs_vjp(U, R_bar, mesh, prm):
    """(U_bar, sigma_bar) of R(U) for the cotangent R_bar."""
    Ux = U.detach().clone().requires_grad_(True)
    sig = torch.tensor(float(prm.sigma), dtype=torch.float64, requires_grad=True)
    R = rhs(Ux, mesh, _with_sigma(prm, sig))
    Ub, sb = torch.autograd.grad(R, (Ux, sig), R_bar, allow_unused=True)
    return Ub, (0.0 if sb is None else float(sb))


def rk_step_vjp(U, dt, U1_bar, mesh, prm):
    """(U_bar, sigma_bar) of one SSP-RK3 step with fixed dt."""
    Ux = U.detach().clone().requires_grad_(True)
    sig = torch.tensor(float(prm.sigma), dtype=torch.float64, requires_grad=True)
    U1 = rk_step(Ux, dt, mesh, _with_sigma(prm, sig))
    Ub, sb = torch.autograd.grad(U1, (Ux, sig), U1_bar, allow_unused=True)
    return Ub, (0.0 if sb is None else float(sb))
