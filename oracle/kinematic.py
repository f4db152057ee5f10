"""Kinematic mode: phase field and level set under a prescribed velocity
(test infrastructure only).

Paper passages followed (Tonicello & Ihme, arXiv 2306.05002):
  * Results, "Kinematic tests": the velocity is a given analytic function
    and only the phase-field and level-set equations are advanced, which
    isolates the interface-capturing technique;
  * the Allen-Cahn and level-set weak forms of the Section "Discontinuous
    Galerkin discretisation": transport u.grad phi as a volume term plus the
    hat/tilde face fluxes, the Allen-Cahn flux a_1 = Gamma (eps grad phi -
    phi (1-phi) n) with n from the level set, symmetric interior penalty for
    the a_1 fluxes;
  * Rider-Kothe vortex: u = (sin^2(pi x) sin(2 pi y), -sin(2 pi x)
    sin^2(pi y)) cos(pi t / T), T = 4, droplet R = 0.15; classical RK4;
  * the L1 error and the relative mass error
    E_m = int (phi(t) - phi(0)) / int phi(0) of the same study.

The discretisation of the phi and psi equations is the one of the full
residual (``residual.py``) with the prescribed nodal velocity in place of
rho u / rho.  Readings (listed in the design notes):
  * face speed: with no sound speed, lambda = max(|u.m| inside, |u.m|
    outside), i.e. the hat/tilde correction 1/2 (lambda - u.m)(phi_e -
    phi_i) is the upwind flux;
  * velocity u(x, t) = u0(x) s(t) with s = cos(pi t / T) (T > 0) or s = 1;
  * L1 = sum_j W_j |phi_j(T) - phi_j(0)| (GLL quadrature of the area
    integral), E_m from the same quadrature;
  * time step: the rule of the full path without the sound speed,
    dt = CFL h_min / (max sum_k |u0_k| + (p+1)^2 d Gamma eps / h_min).

State layout: Phi[0] = phi, Phi[1] = psi, each [element, node]; velocity
u[k, element, node].  Periodic meshes only.
"""

import math

import torch

from .residual import _dk, _trace, _place


class KinParams:
    def __init__(self, Gamma=1.0, eps=0.01, c_ip=1.0, grad_reg=1e-12, period=0.0):
        self.Gamma = float(Gamma)
        self.eps = float(eps)
        self.c_ip = float(c_ip)
        self.grad_reg = float(grad_reg)
        self.period = float(period)


def time_factor(t, kp):
    """s(t) of u(x, t) = u0(x) s(t)."""
    return math.cos(math.pi * t / kp.period) if kp.period > 0.0 else 1.0


def rider_kothe_velocity(X):
    """Single-vortex velocity field at time 0 (Rider-Kothe), X = coordinates [2, ...]."""
    x, y = X[0], X[1]
    pi = math.pi
    return torch.stack([torch.sin(pi * x) ** 2 * torch.sin(2 * pi * y),
                        -torch.sin(2 * pi * x) * torch.sin(pi * y) ** 2])


def _flux_a(phi, gphi, gpsi, kp):
    """a_1 = Gamma (eps grad phi - phi (1 - phi) n), n = g / sqrt(g.g + delta^2)."""
    delta = kp.grad_reg
    nrm = torch.sqrt((gpsi * gpsi).sum(0) + delta * delta)
    return kp.Gamma * (kp.eps * gphi - (phi * (1.0 - phi)) * (gpsi / nrm))


def _batch(Phi, u, mesh, kp):
    """Local data of every element: nodal phi, psi, u and element-local gradients."""
    d, n = mesh.d, mesh.n
    shp = (Phi.shape[1],) + (n,) * d
    phi = Phi[0].reshape(shp)
    psi = Phi[1].reshape(shp)
    uu = u.reshape((d,) + shp)
    gphi = torch.stack([_dk(phi, k, mesh) for k in range(d)])
    gpsi = torch.stack([_dk(psi, k, mesh) for k in range(d)])
    a = _flux_a(phi, gphi, gpsi, kp)
    return dict(phi=phi, psi=psi, u=uu, gphi=gphi, gpsi=gpsi, a=a)


def kin_rhs(Phi, u, mesh, kp):
    """R = dPhi/dt of the phase field and level set for the nodal velocity u
    (already multiplied by the time factor).  Strong form, equal to the weak
    form under GLL collocation as for the full residual."""
    d, n, p = mesh.d, mesh.n, mesh.p
    if any(mesh.bc[k][s] != "periodic" for k in range(d) for s in (0, 1)):
        raise ValueError("kinematic mode: periodic meshes only")
    E = Phi.shape[1]
    B = _batch(Phi, u, mesh, kp)
    # volume: transport as a source, divergence of a for phi
    Rphi = -(B["u"] * B["gphi"]).sum(0) + sum(_dk(B["a"][k], k, mesh) for k in range(d))
    Rpsi = -(B["u"] * B["gpsi"]).sum(0)
    R = torch.stack([Rphi, Rpsi])
    el = torch.arange(E)
    for k in range(d):
        h = mesh.h[k]
        L = 1.0 / (float(mesh.w[0]) * mesh.J[k])
        eta = kp.c_ip * kp.Gamma * kp.eps * (p + 1) ** 2 / h
        for side in (0, 1):
            sm = -1.0 if side == 0 else 1.0
            nb, _ = mesh.neighbour(el, k, side)
            Bn = _batch(Phi[:, nb], u[:, nb], mesh, kp)
            iI = 0 if side == 0 else n - 1
            iE = n - 1 if side == 0 else 0
            phiI, phiE = _trace(B["phi"], k, iI), _trace(Bn["phi"], k, iE)
            psiI, psiE = _trace(B["psi"], k, iI), _trace(Bn["psi"], k, iE)
            umI = sm * _trace(B["u"][k], k, iI)
            umE = sm * _trace(Bn["u"][k], k, iE)
            amI = sm * _trace(B["a"][k], k, iI)
            amE = sm * _trace(Bn["a"][k], k, iE)
            lam = torch.maximum(torch.abs(umI), torch.abs(umE))
            ahat = 0.5 * (amI + amE) - eta * (phiI - phiE)
            cphi = L * (0.5 * (lam - umI) * (phiE - phiI) + (ahat - amI))
            cpsi = L * (0.5 * (lam - umI) * (psiE - psiI))
            onehot = torch.zeros(n, dtype=torch.float64)
            onehot[iI] = 1.0
            R = R + _place(torch.stack([cphi, cpsi]), k, onehot)
            # SIPG symmetric term along the normal line through each face node
            wts = torch.stack([mesh.D[iI, a] / (2.0 * mesh.w[a] * mesh.J[k] ** 2) for a in range(n)])
            sym = sm * kp.Gamma * kp.eps * (phiI - phiE)
            R = R + _place(torch.stack([sym, torch.zeros_like(sym)]), k, wts)
    return R.reshape(2, E, n ** d)


def velocity(u0, t, kp):
    return u0 * time_factor(t, kp)


def velocity_from_stream(S, mesh):
    """2D velocity amplitude u0 = (dS/dy, -dS/dx) from a nodal stream
    function S [element, node], with the broken (element-local) derivatives:
    one representation on the mesh of the divergence-free prescribed field of
    the Rider-Kothe study.  Its discrete divergence vanishes node by node and
    its normal component is continuous across faces."""
    n = mesh.n
    F = S.reshape(S.shape[0], n, n)
    ux = _dk(F, 1, mesh)
    uy = -_dk(F, 0, mesh)
    return torch.stack([ux.reshape(S.shape), uy.reshape(S.shape)])


def rk4_step(Phi, t, dt, u0, mesh, kp, rhs_fn=None):
    """Classical fourth-order Runge-Kutta step from time t.
    ``rhs_fn(Phi, t)`` replaces the DG residual (used to pin the scheme)."""
    R = (lambda V, s: kin_rhs(V, velocity(u0, s, kp), mesh, kp)) if rhs_fn is None else rhs_fn
    k1 = R(Phi, t)
    k2 = R(Phi + 0.5 * dt * k1, t + 0.5 * dt)
    k3 = R(Phi + 0.5 * dt * k2, t + 0.5 * dt)
    k4 = R(Phi + dt * k3, t + dt)
    return Phi + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def max_dt(u0, mesh, kp, cfl=0.1):
    """Time-step rule of the kinematic mode (the full path's rule without the
    sound speed), from the velocity amplitude u0."""
    d = mesh.d
    hmin = min(mesh.h)
    wave = float(torch.abs(u0).sum(0).max())
    rate = (wave + (mesh.p + 1) ** 2 * d * kp.Gamma * kp.eps / hmin) / hmin
    return cfl / rate


def l1_error(phi, phi0, mesh):
    """sum_j W_j |phi_j - phi0_j| (GLL quadrature of int |phi - phi0|)."""
    return float((torch.abs(phi - phi0) * mesh.node_weights()).sum())


def mass_error(phi, phi0, mesh):
    """E_m = int (phi - phi0) / int phi0 with the GLL quadrature."""
    W = mesh.node_weights()
    return float(((phi - phi0) * W).sum() / (phi0 * W).sum())


# ---- level-set re-initialisation (Section "Discontinuous Galerkin
# discretisation", closing paragraphs) --------------------------------------------
# Pseudo-time Eikonal iteration from psi0 = phi - 1/2 with the smeared sign
# sgn = tanh(psi0 / (2 eps |grad psi0|)), a vanishing viscosity nu_h (SIPG
# diffusive flux) and the sign term as a source.  Readings (design notes):
#   * sign convention of Sussman, Smereka and Osher: d psi / d tau =
#     sgn (1 - |grad psi|) + div(nu_h grad psi), which relaxes |grad psi|
#     towards 1 (the printed form has the opposite sign of the source, which
#     would steepen the profile);
#   * |grad psi0| regularised as sqrt(g.g + delta^2), the same delta as n;
#   * nu_h = h / (p+1) (one nodal spacing), pseudo step
#     dtau = 0.1 h_min / (1 + (p+1)^2 d nu_h / h_min), classical RK4
#     iterations (50 every 2000 physical steps in the paper's runs).

def reinit_start(phi, mesh, kp):
    """psi0 = phi - 1/2 and the smeared sign tanh(psi0 / (2 eps |grad psi0|))."""
    d, n = mesh.d, mesh.n
    shp = (phi.shape[0],) + (n,) * d
    psi0 = (phi - 0.5).reshape(shp)
    g = torch.stack([_dk(psi0, k, mesh) for k in range(d)])
    nrm = torch.sqrt((g * g).sum(0) + kp.grad_reg * kp.grad_reg)
    sgn = torch.tanh(psi0 / (2.0 * kp.eps * nrm))
    return psi0.reshape(phi.shape), sgn.reshape(phi.shape)


def reinit_rhs(psi, sgn, mesh, nu, c_ip):
    """sgn (1 - |grad psi|) + div(nu grad psi), the diffusive flux with
    symmetric interior penalty (the a-flux discretisation with a = nu grad psi).
    psi, sgn: [element, node]."""
    d, n, p = mesh.d, mesh.n, mesh.p
    E = psi.shape[0]
    shp = (E,) + (n,) * d

    def local(f):
        F = f.reshape(shp)
        g = torch.stack([_dk(F, k, mesh) for k in range(d)])
        return F, g

    P, g = local(psi)
    mag = torch.sqrt((g * g).sum(0))
    R = sgn.reshape(shp) * (1.0 - mag) + sum(_dk(nu * g[k], k, mesh) for k in range(d))
    el = torch.arange(E)
    for k in range(d):
        L = 1.0 / (float(mesh.w[0]) * mesh.J[k])
        eta = c_ip * nu * (p + 1) ** 2 / mesh.h[k]
        for side in (0, 1):
            sm = -1.0 if side == 0 else 1.0
            nb, _ = mesh.neighbour(el, k, side)
            Pn, gn = local(psi[nb])
            iI = 0 if side == 0 else n - 1
            iE = n - 1 if side == 0 else 0
            pI, pE = _trace(P, k, iI), _trace(Pn, k, iE)
            amI = sm * nu * _trace(g[k], k, iI)
            amE = sm * nu * _trace(gn[k], k, iE)
            ahat = 0.5 * (amI + amE) - eta * (pI - pE)
            onehot = torch.zeros(n, dtype=torch.float64)
            onehot[iI] = 1.0
            R = R + _place(L * (ahat - amI), k, onehot)
            wts = torch.stack([mesh.D[iI, a] / (2.0 * mesh.w[a] * mesh.J[k] ** 2) for a in range(n)])
            R = R + _place(sm * nu * (pI - pE), k, wts)
    return R.reshape(E, n ** d)


def reinit_params(mesh, cfl=0.1):
    """(nu_h, dtau) of the re-initialisation readings."""
    hmin = min(mesh.h)
    nu = hmin / (mesh.p + 1)
    return nu, cfl * hmin / (1.0 + (mesh.p + 1) ** 2 * mesh.d * nu / hmin)


def reinit(phi, mesh, kp, n_iter, nu, dtau):
    """Level set re-initialised from phi: n_iter classical RK4 pseudo-time
    steps of reinit_rhs from psi0 = phi - 1/2."""
    psi, sgn = reinit_start(phi, mesh, kp)
    R = lambda v: reinit_rhs(v, sgn, mesh, nu, kp.c_ip)
    for _ in range(n_iter):
        k1 = R(psi)
        k2 = R(psi + 0.5 * dtau * k1)
        k3 = R(psi + 0.5 * dtau * k2)
        k4 = R(psi + dtau * k3)
        psi = psi + (dtau / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return psi
