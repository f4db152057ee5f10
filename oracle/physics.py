"""Stiffened-gas closure, mixture rules and the initial-condition map
(test infrastructure only).

Follows Section "Five equation model": the stiffened-gas pressure written
with the volume fraction (the equation right after the system), the phase
sound speed and enthalpy, and the mixture rules for 1/(gamma-1) and
P_inf gamma/(gamma-1) that close it.

Field order of a state vector (d = space dimension, N_f = d + 5):
  0: alpha_1 rho_1, 1: alpha_2 rho_2, 2..d+1: rho u_j, d+2: rho E,
  d+3: alpha (= phi_1, the advected volume fraction), d+4: psi (level set)
"""

from dataclasses import dataclass

import torch


@dataclass
class Params:
    gamma: tuple = (1.4, 4.4)
    pinf: tuple = (0.0, 0.6)
    rho0: tuple = (1.0, 10.0)      # reference densities rho_l^(0) in R_l = rho_l^(0) a_l
    Gamma: float = 1.0             # Allen-Cahn velocity scale
    eps: float = 1e-2              # Allen-Cahn interface thickness
    mu: tuple = (0.0, 0.0)         # phase viscosities
    sigma: float = 0.0             # surface tension coefficient
    g: tuple = (0.0, 0.0, 0.0)     # gravity
    c_ip: float = 1.0              # interior-penalty constant
    grad_reg: float = 1e-12        # regulariser of |grad psi| and |grad alpha|

    @property
    def viscous(self):
        return self.mu[0] != 0.0 or self.mu[1] != 0.0


def mixture_xi_pi(alpha, prm):
    """xi = 1/(gamma-1) and Pi = P_inf gamma/(gamma-1) of the mixture
    (mixture rules of Section "Five equation model", phi_2 = 1 - phi_1)."""
    g1, g2 = prm.gamma
    p1, p2 = prm.pinf
    xi = alpha / (g1 - 1.0) + (1.0 - alpha) / (g2 - 1.0)
    pi = alpha * (g1 * p1 / (g1 - 1.0)) + (1.0 - alpha) * (g2 * p2 / (g2 - 1.0))
    return xi, pi


def primitives(Q, d, prm):
    """Primitive variables from conserved fields Q (leading axis = field).

    rho = sum of partial densities, u = (rho u)/rho, P from the stiffened-gas
    law P = (rho e - Pi) / xi, mixture sound speed c^2 = ((1+xi) P + Pi)/(xi rho)
    (frozen mixture stiffened gas: c^2 = gamma (P + P_inf)/rho with the mixture
    gamma and P_inf), and rho_l H_l = gamma_l (P + P_inf_l)/(gamma_l - 1).
    """
    q1, q2 = Q[0], Q[1]
    rho = q1 + q2
    u = torch.stack([Q[2 + j] / rho for j in range(d)])
    kin = 0.5 * (u * u).sum(0)
    rhoE = Q[2 + d]
    alpha = Q[3 + d]
    rhoe = rhoE - rho * kin
    xi, pi = mixture_xi_pi(alpha, prm)
    P = (rhoe - pi) / xi
    c = torch.sqrt(((1.0 + xi) * P + pi) / (xi * rho))
    g1, g2 = prm.gamma
    p1, p2 = prm.pinf
    rH1 = g1 * (P + p1) / (g1 - 1.0)
    rH2 = g2 * (P + p2) / (g2 - 1.0)
    return dict(rho=rho, u=u, kin=kin, P=P, c=c, rH1=rH1, rH2=rH2,
                alpha=alpha, xi=xi, pi=pi)


def prim_to_cons(alpha, psi, rho1, rho2, u, P, prm):
    """Initial-condition map: primitives -> conserved state (leading axis = field).

    alpha_1 rho_1 = alpha rho_1, alpha_2 rho_2 = (1-alpha) rho_2, rho u,
    rho E = xi P + Pi + rho |u|^2 / 2 (the stiffened-gas law solved for rho e).
    ``u`` has a leading axis of length d.
    """
    d = u.shape[0]
    q1 = alpha * rho1
    q2 = (1.0 - alpha) * rho2
    rho = q1 + q2
    xi, pi = mixture_xi_pi(alpha, prm)
    kin = 0.5 * (u * u).sum(0)
    rhoE = xi * P + pi + rho * kin
    return torch.stack([q1, q2] + [rho * u[j] for j in range(d)]
                       + [rhoE, alpha, psi])


def nonphysical_mask(prim):
    """Nodes whose state has no valid closure: rho <= 0, xi rho <= 0,
    (1+xi) P + Pi <= 0, or anything non-finite."""
    rho, xi, P, pi = prim["rho"], prim["xi"], prim["P"], prim["pi"]
    bad = (rho <= 0) | (xi * rho <= 0) | ((1.0 + xi) * P + pi <= 0)
    bad = bad | ~torch.isfinite(P) | ~torch.isfinite(prim["c"])
    return bad
