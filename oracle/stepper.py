"""Time-step rule, SSP-RK3 and monitors (test infrastructure only).

The paper integrates explicitly (classical RK4 in its results) and gives no
time-step rule.  The hot path advances with the three-stage Shu-Osher
strong-stability-preserving Runge-Kutta scheme; the step size follows the
reading

    dt = CFL * h_min / ( max_nodes(sum_k |u_k| + d c)
                         + (p+1)^2 d nu_max / h_min ),
    nu_max = max(Gamma eps, max_nodes mu / rho),

i.e. dt = CFL / rate with rate = (...) / h_min.

Monitors: the integral of every field (sum_j W_j q_j, from the diagonal GLL
mass matrix; the mass-conservation error of the Rider-Kothe study in the
Results section is built from the integral of phi), the range of alpha
(boundedness claimed in the abstract and conclusions), the deviation of P and
u from reference values (the interface equilibrium condition of the water
droplet study), and the count of nodes with no valid closure.
"""

import torch

from .physics import primitives, nonphysical_mask
from .residual import rhs


def max_rate(U, mesh, prm):
    """Largest stable-rate estimate max_nodes(...)/h_min of the time-step rule."""
    d = mesh.d
    pr = primitives(U, d, prm)
    wave = torch.abs(pr["u"]).sum(0) + d * pr["c"]
    hmin = min(mesh.h)
    nu = prm.Gamma * prm.eps
    if prm.viscous:
        alpha = U[3 + d]
        mu = prm.mu[0] * alpha + prm.mu[1] * (1.0 - alpha)
        nu = max(nu, float((mu / pr["rho"]).max()))
    return (float(wave.max()) + (mesh.p + 1) ** 2 * d * nu / hmin) / hmin


def max_dt(U, mesh, prm, cfl=0.1):
    return cfl / max_rate(U, mesh, prm)


def rk_step(U, dt, mesh, prm, rhs_fn=None):
    """One Shu-Osher SSP-RK3 step:
    U1 = U + dt R(U); U2 = 3/4 U + 1/4 (U1 + dt R(U1));
    U+ = 1/3 U + 2/3 (U2 + dt R(U2)).
    ``rhs_fn`` replaces the DG residual (used to pin the scheme on y' = z y)."""
    R = (lambda V: rhs(V, mesh, prm)) if rhs_fn is None else rhs_fn
    U1 = U + dt * R(U)
    U2 = 0.75 * U + 0.25 * (U1 + dt * R(U1))
    return (1.0 / 3.0) * U + (2.0 / 3.0) * (U2 + dt * R(U2))


def monitors(U, mesh, prm, p_ref=None, u_ref=None):
    d = mesh.d
    W = mesh.node_weights()
    integral = (U * W).sum(dim=(1, 2))
    pr = primitives(U, d, prm)
    alpha = U[3 + d]
    out = dict(integral=integral,
               min_alpha=float(alpha.min()), max_alpha=float(alpha.max()),
               nonphys=int(nonphysical_mask(pr).sum()),
               max_rate=max_rate(U, mesh, prm))
    if p_ref is not None:
        out["dev_p"] = float(torch.abs(pr["P"] - p_ref).max())
    if u_ref is not None:
        ur = torch.as_tensor(u_ref, dtype=torch.float64).view(d, 1, 1)
        out["dev_u"] = float(torch.abs(pr["u"] - ur).max())
    return out
