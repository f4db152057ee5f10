"""Seeded synthetic workloads: mesh descriptions, parameters and primitive
initial fields of the five benchmark configurations.

This module is the only code shared by the HIP path and the test oracle.  It
holds none of the method's arithmetic: it evaluates analytic initial
conditions (signed distances, logistic profiles, a smeared planar shock from
the textbook Rankine-Hugoniot relations, a hydrostatic column) at node
coordinates that the caller supplies, and returns *primitive* fields
(alpha, psi, phase densities, velocity, pressure).  Each side turns them
into conserved state with its own stiffened-gas map.  Everything is numpy
float64 and deterministic (fixed seeds).

Configurations (all p = 3, i.e. four GLL nodes per direction):
  drop1d     1D periodic air/water slab on [0,1], 100 elements, u = 1, P = 1
  drop2d     2D periodic water droplet (R 0.15) in air, 128 x 128, u = (1, 0.5)
  shock2d    2D shock (pressure ratio 10 in air) onto a water cylinder,
             512 x 256 on [0,2] x [0,1]; Dirichlet inflow, outflow, periodic y
  rt3d       3D heavy-over-light box, 96^3, gravity, viscosity, surface tension,
             slip walls in z
  adjoint2d  drop2d plus viscosity 1e-3 and surface tension 1e-2
  waterair2d the paper's water droplet (R 25/89) in air, 24 x 24, density
             ratio 1000 (rho 1e-3 / 1), P_inf 0 / 6000, u = (5, 5), P = 1,
             Gamma 5, five advection periods (t = 1)
  bubble2d   the paper's rising bubble: R 0.25 at (0, 0.5) in [-0.5, 0.5] x
             [0, 2], 20 x 40, rho_1/rho_2 = mu_1/mu_2 = 10, Re 35, Eo 10;
             no-slip bottom, Riemann-invariant top (zero velocity, P 1000),
             slip side walls
  rt2d       the paper's 2D Rayleigh-Taylor case: [0, 1] x [0, 4], 20 x 80,
             interface y = 2 + 0.1 cos(2 pi x), At 0.5, Re 3000, g = -e_y;
             boundaries as bubble2d (Riemann top at P 100)
Phase 1 is air (gamma 1.4, P_inf 0), phase 2 water-like (gamma 4.4,
P_inf 0.6), except in bubble2d where phase 1 is the heavy surrounding
liquid; alpha is the volume fraction of phase 1 and psi increases towards
phase 1, alpha = 1 / (1 + exp(-psi / eps)).
"""

import math

import numpy as np

ORDER = 3
NAMES = ("drop1d", "drop2d", "shock2d", "rt3d", "adjoint2d", "waterair2d", "bubble2d", "rt2d")
FULL_ELEMS = {
    "drop1d": (100,),
    "drop2d": (128, 128),
    "shock2d": (512, 256),
    "rt3d": (96, 96, 96),
    "adjoint2d": (128, 128),
    "waterair2d": (24, 24),
    "bubble2d": (20, 40),
    "rt2d": (20, 80),
}


def _sigmoid(z):
    out = np.empty_like(z)
    pos = z >= 0
    out[pos] = 1.0 / (1.0 + np.exp(-z[pos]))
    ez = np.exp(z[~pos])
    out[~pos] = ez / (1.0 + ez)
    return out


def _softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def shock_states(pressure_ratio=10.0, gamma=1.4, rho_pre=1.0, p_pre=1.0):
    """Post-shock density and velocity of a normal shock moving into gas at
    rest (textbook Rankine-Hugoniot relations for a calorically perfect gas)."""
    pi_ = pressure_ratio
    rho_ratio = ((gamma + 1) * pi_ + (gamma - 1)) / ((gamma - 1) * pi_ + (gamma + 1))
    ms = math.sqrt(1.0 + (gamma + 1) * (pi_ - 1) / (2 * gamma))
    w = ms * math.sqrt(gamma * p_pre / rho_pre)
    rho_post = rho_pre * rho_ratio
    u_post = w * (1.0 - rho_pre / rho_post)
    return rho_post, u_post, p_pre * pi_


def config(name, n_elem=None, order=ORDER):
    """Mesh description and physical parameters of a configuration.

    ``n_elem`` overrides the element counts (reduced sizes for parity tests);
    ``order`` the polynomial degree (3; 4 for the 2D configurations, the
    degree of the paper's Rayleigh-Taylor and rising-bubble runs); eps follows
    the rule eps = h / (2 (p+1)) of the configuration's own grid (waterair2d,
    bubble2d, rt2d: eps = h / 2).
    """
    if name not in NAMES:
        raise KeyError(name)
    n_elem = tuple(n_elem) if n_elem is not None else FULL_ELEMS[name]
    p = int(order)
    base = dict(gamma=(1.4, 4.4), pinf=(0.0, 0.6), rho0=(1.0, 10.0), Gamma=1.0,
                mu=(0.0, 0.0), sigma=0.0, g=(0.0, 0.0, 0.0), c_ip=1.0,
                grad_reg=1e-12)
    cfg = dict(name=name, order=p, n_elem=n_elem, cfl=0.1, freeze_dt=False)
    if name == "drop1d":
        cfg.update(dim=1, lo=(0.0,), hi=(1.0,), bc=[("periodic", "periodic")],
                   steps=4200)
    elif name in ("drop2d", "adjoint2d"):
        cfg.update(dim=2, lo=(0.0, 0.0), hi=(1.0, 1.0),
                   bc=[("periodic", "periodic")] * 2, steps=20)
        if name == "adjoint2d":
            base.update(mu=(1e-3, 1e-3), sigma=1e-2)
            cfg.update(steps=400, freeze_dt=True, checkpoint_every=20)
    elif name == "shock2d":
        cfg.update(dim=2, lo=(0.0, 0.0), hi=(2.0, 1.0),
                   bc=[("dirichlet", "extrapolate"), ("periodic", "periodic")],
                   steps=200, shock_x=0.34, shock_width=3.0)
        rho_post, u_post, p_post = shock_states()
        cfg["bc_prim"] = {(0, 0): dict(alpha=1.0, psi=0.0, rho1=rho_post,
                                       rho2=base["rho0"][1], u=(u_post, 0.0),
                                       P=p_post)}
    elif name == "waterair2d":
        # the paper's water droplet in air: density ratio 1000, P_inf of
        # water 6000, u = (5, 5), five advection periods
        cfg.update(dim=2, lo=(0.0, 0.0), hi=(1.0, 1.0),
                   bc=[("periodic", "periodic")] * 2, t_end=1.0)
        base.update(rho0=(1e-3, 1.0), pinf=(0.0, 6.0e3), Gamma=5.0)
        cfg.update(steps=200)
    elif name == "bubble2d":
        # Re = rho_1 d^(3/2) |g|^(1/2) / mu_1 = 35 and Eo = 4 rho_1 |g| R^2 / sigma
        # = 10 with rho_1 = 1000, |g| = 0.98, d = 2R = 0.5; stiffened gases with
        # a Mach number below 0.1 at the rise velocity
        cfg.update(dim=2, lo=(-0.5, 0.0), hi=(0.5, 2.0),
                   bc=[("slip_wall", "slip_wall"), ("no_slip", "riemann")],
                   t_end=3.0, steps=200, p_top=1000.0, radius=0.25, centre=(0.0, 0.5))
        base.update(gamma=(4.4, 1.4), pinf=(6.0e4, 0.0), rho0=(1000.0, 100.0),
                    mu=(10.0, 1.0), sigma=24.5, g=(0.0, -0.98, 0.0))
        cfg["bc_state"] = {(1, 1): [cfg["p_top"]]}
    elif name == "rt2d":
        # At = (rho_h - rho_l)/(rho_h + rho_l) = 0.5, Re = rho_h d^(3/2) |g|^(1/2)
        # / mu = 3000 with d = 1, |g| = 1; light phase 1 below, heavy phase 2
        # above; ideal gases at a Mach number near 0.1
        cfg.update(dim=2, lo=(0.0, 0.0), hi=(1.0, 4.0),
                   bc=[("slip_wall", "slip_wall"), ("no_slip", "riemann")],
                   t_end=3.0 * math.sqrt(2.0), steps=200, p_top=100.0)
        base.update(gamma=(1.4, 1.4), pinf=(0.0, 0.0), rho0=(1.0, 3.0),
                    mu=(1e-3, 1e-3), g=(0.0, -1.0, 0.0))
        cfg["bc_state"] = {(1, 1): [cfg["p_top"]]}
    elif name == "rt3d":
        cfg.update(dim=3, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                   bc=[("periodic", "periodic")] * 2 + [("slip_wall", "slip_wall")],
                   steps=100)
        base.update(rho0=(1.0, 3.0), mu=(1e-3, 1e-3), sigma=1e-3, g=(0.0, 0.0, -1.0))
    d = cfg["dim"]
    if len(n_elem) != d:
        raise ValueError("n_elem has the wrong length")
    h = min((cfg["hi"][k] - cfg["lo"][k]) / n_elem[k] for k in range(d))
    # eps: half a nodal spacing; the water droplet in air (air density 1e-3,
    # where an overshoot of alpha by 1e-3 empties the air) and the two
    # wall-bounded cases (bubble2d, rt2d: their interfaces stay in bounds only
    # so) h / 2
    wide = name in ("waterair2d", "bubble2d", "rt2d")
    base["eps"] = (0.5 * h) if wide else 0.5 * h / (p + 1)
    cfg["params"] = base
    cfg.setdefault("bc_prim", {})
    cfg.setdefault("bc_state", {})
    return cfg


def _rt_interface_noise(x, y, scaled=True):
    """Seeded 1e-3 perturbation of the Rayleigh-Taylor interface: 4 x 4 Fourier
    modes with N(0,1) amplitudes (seed 3), scaled to max |zeta| = 1 on a 256^2
    grid.  Separable form: cos/sin of 2 pi (m x + n y) from the per-axis
    harmonics (8 transcendental evaluations per axis instead of 32 per point)."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 4))
    B = rng.standard_normal((4, 4))

    def zeta(xx, yy):
        cx = [np.cos(2.0 * math.pi * m * xx) for m in range(1, 5)]
        sx = [np.sin(2.0 * math.pi * m * xx) for m in range(1, 5)]
        cy = [np.cos(2.0 * math.pi * n * yy) for n in range(1, 5)]
        sy = [np.sin(2.0 * math.pi * n * yy) for n in range(1, 5)]
        z = np.zeros(np.broadcast(xx, yy).shape)
        for m in range(4):
            for n in range(4):
                c = cx[m] * cy[n] - sx[m] * sy[n]      # cos 2 pi (m x + n y)
                s_ = sx[m] * cy[n] + cx[m] * sy[n]     # sin 2 pi (m x + n y)
                z += A[m, n] * c + B[m, n] * s_
        return z

    if not scaled:
        return zeta(x, y)
    g = (np.arange(256) + 0.5) / 256.0
    gx, gy = np.meshgrid(g, g, indexing="ij")
    scale = np.abs(zeta(gx, gy)).max()
    return zeta(x, y) / scale


def _rt3d_fields(X, eps, r1, r2, d, shp):
    """rt3d: interface z = eta(x, y) = 0.5 + 0.02 cos 2 pi x cos 2 pi y + 1e-3 zeta,
    psi = eta - z, hydrostatic P for g = -e_z with P(z = 1) = 1:
    P = 1 + int_z^1 rho dz' with rho = rho2 + (rho1 - rho2) alpha."""
    import torch
    x, y, z = (torch.from_numpy(np.ascontiguousarray(X[k])) for k in range(3))
    eta = (0.5 + 0.02 * torch.cos(2 * math.pi * x) * torch.cos(2 * math.pi * y)
           + 1e-3 * torch.from_numpy(_rt_interface_noise_t(x, y)))
    psi = eta - z
    def sp(t):  # softplus log(1 + e^t) without torch's large-argument cut-off
        return torch.clamp(t, min=0.0) + torch.log1p(torch.exp(-torch.abs(t)))

    P = 1.0 + r2 * (1.0 - z) + (r1 - r2) * eps * (sp((eta - z) / eps) - sp((eta - 1.0) / eps))
    alpha = torch.sigmoid(psi / eps)
    return dict(alpha=alpha.numpy(), psi=psi.numpy(), rho1=np.full(shp, r1), rho2=np.full(shp, r2),
                P=P.numpy(), u=np.zeros((d,) + shp))


def _rt_interface_noise_t(x, y):
    """_rt_interface_noise on torch CPU tensors (same modes and scale)."""
    import torch
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 4))
    B = rng.standard_normal((4, 4))
    g = (np.arange(256) + 0.5) / 256.0
    gx, gy = np.meshgrid(g, g, indexing="ij")
    scale = np.abs(_rt_interface_noise(gx, gy, scaled=False)).max()
    cx = [torch.cos(2.0 * math.pi * m * x) for m in range(1, 5)]
    sx = [torch.sin(2.0 * math.pi * m * x) for m in range(1, 5)]
    cy = [torch.cos(2.0 * math.pi * n * y) for n in range(1, 5)]
    sy = [torch.sin(2.0 * math.pi * n * y) for n in range(1, 5)]
    zt = torch.zeros_like(x)
    for m in range(4):
        # sum_n A_mn cos 2 pi (m x + n y) + B_mn sin 2 pi (m x + n y)
        cm = sum(float(A[m, n]) * cy[n] + float(B[m, n]) * sy[n] for n in range(4))
        sm = sum(float(B[m, n]) * cy[n] - float(A[m, n]) * sy[n] for n in range(4))
        zt += cx[m] * cm + sx[m] * sm
    return (zt / scale).numpy()


def primitive_fields(cfg, coords, variant=None):
    """Primitive initial fields at the given node coordinates.

    coords: float64 array of shape (d, ...) (usually (d, E, nn)).
    Returns dict(alpha, psi, rho1, rho2, P, u) with u of shape (d, ...).
    ``variant="noisy_u"`` (drop1d only) adds 1e-3 N(0,1) noise per node to u
    (seed 0).
    """
    name = cfg["name"]
    d = cfg["dim"]
    prm = cfg["params"]
    eps = prm["eps"]
    X = np.asarray(coords, dtype=np.float64)
    shp = X.shape[1:]
    r1, r2 = prm["rho0"]
    rho1 = np.full(shp, r1)
    rho2 = np.full(shp, r2)
    u = np.zeros((d,) + shp)
    P = np.ones(shp)
    if name == "drop1d":
        psi = np.abs(X[0] - 0.5) - 0.25
        u[0] = 1.0
        if variant == "noisy_u":
            rng = np.random.default_rng(0)
            u[0] = 1.0 + 1e-3 * rng.standard_normal(shp)
    elif name in ("drop2d", "adjoint2d"):
        psi = np.sqrt((X[0] - 0.5) ** 2 + (X[1] - 0.5) ** 2) - 0.15
        u[0] = 1.0
        u[1] = 0.5
    elif name == "waterair2d":
        psi = np.sqrt((X[0] - 0.5) ** 2 + (X[1] - 0.5) ** 2) - 25.0 / 89.0
        u[0] = 5.0
        u[1] = 5.0
    elif name == "shock2d":
        psi = np.sqrt((X[0] - 0.5) ** 2 + (X[1] - 0.5) ** 2) - 0.1
        h = (cfg["hi"][0] - cfg["lo"][0]) / cfg["n_elem"][0]
        w = _sigmoid(-(X[0] - cfg["shock_x"]) / (cfg["shock_width"] * h))
        rho_post, u_post, p_post = shock_states()
        rho1 = w * rho_post + (1.0 - w) * 1.0
        u[0] = w * u_post
        P = w * p_post + (1.0 - w) * 1.0
    elif name == "bubble2d":
        cx, cy = cfg["centre"]
        psi = np.sqrt((X[0] - cx) ** 2 + (X[1] - cy) ** 2) - cfg["radius"]
        # heavy-liquid column under P_top, plus the Laplace jump sigma / R inside
        # the bubble
        inside = 1.0 - _sigmoid(psi / eps)
        P = (cfg["p_top"] + r1 * (-prm["g"][1]) * (cfg["hi"][1] - X[1])
             + prm["sigma"] / cfg["radius"] * inside)
    elif name == "rt2d":
        x, y = X[0], X[1]
        eta = 2.0 + 0.1 * np.cos(2.0 * math.pi * x)
        psi = eta - y
        top = cfg["hi"][1]
        # hydrostatic column for g = -e_y under P_top:
        # P = P_top + int_y^top rho dy' with rho = rho2 + (rho1 - rho2) alpha
        P = (cfg["p_top"] + r2 * (top - y)
             + (r1 - r2) * eps * (_softplus((eta - y) / eps) - _softplus((eta - top) / eps)))
    elif name == "rt3d":
        # evaluated with torch's multithreaded CPU kernels (the 96^3 box has
        # 56.6 M nodes); the formulas are those of the other cases
        return _rt3d_fields(X, eps, r1, r2, d, shp)
    else:
        raise KeyError(name)
    alpha = _sigmoid(psi / eps)
    return dict(alpha=alpha, psi=psi, rho1=rho1, rho2=rho2, P=P, u=u)


def adjoint_target_perturbation(coords):
    """Smooth seeded perturbation (2 Fourier modes per velocity component,
    amplitudes N(0,1) with seed 4) used to build the adjoint target run."""
    X = np.asarray(coords, dtype=np.float64)
    d = X.shape[0]
    rng = np.random.default_rng(4)
    amp = rng.standard_normal((d, 2, 2))
    out = np.zeros_like(X)
    for j in range(d):
        for m in range(2):
            arg = 2.0 * math.pi * (m + 1) * (X[0] + (m + 1) * X[d - 1])
            out[j] += amp[j, m, 0] * np.cos(arg) + amp[j, m, 1] * np.sin(arg)
    return out


def fd_direction(shape_u, k):
    """Seeded finite-difference direction k: nodal N(0,1) velocity components
    and one N(0,1) surface-tension component (seed 1000 + k), not yet
    normalised."""
    rng = np.random.default_rng(1000 + k)
    du = rng.standard_normal(shape_u)
    ds = float(rng.standard_normal())
    return du, ds


# ---- kinematic mode (phase field and level set under a prescribed velocity) ----------
KIN_NAMES = ("rk2d", "adv2d")
KIN_FULL_ELEMS = {"rk2d": (16, 16), "adv2d": (16, 16)}


def kinematic_config(name, n_elem=None, order=ORDER, psi="cone", eps=None):
    """Kinematic test cases of the Results section, p = 3 (or 1) on [0,1]^2,
    periodic.

    rk2d   Rider-Kothe single vortex: droplet R = 0.15 at (0.5, 0.75),
           u = (sin^2(pi x) sin(2 pi y), -sin(2 pi x) sin^2(pi y)) cos(pi t / 4),
           one period T = 4, Gamma = 1, eps = 2 h / (p + 1): two nodal
           spacings (h / 2 at p = 3, the element size h at p = 1)
    adv2d  linear advection of a droplet R = 0.15 at (0.5, 0.5) by u = (1, 0)
           for one period, fixed eps = 0.05, Gamma = 1

    psi "cone": the level set is the signed distance R - r (the paper's
    choice; its gradient has a cone tip at the centre); "smooth": (R^2 - r^2)
    / (2R), the same zero level and the same normal direction away from the
    centre, polynomial (so its nodal gradient is exact for p >= 2).  eps
    overrides the interface thickness.
    """
    if name not in KIN_NAMES:
        raise KeyError(name)
    n_elem = tuple(n_elem) if n_elem is not None else KIN_FULL_ELEMS[name]
    h = 1.0 / n_elem[0]
    if psi not in ("cone", "smooth"):
        raise ValueError("psi must be 'cone' or 'smooth'")
    cfg = dict(name=name, dim=2, order=order, n_elem=n_elem, lo=(0.0, 0.0), hi=(1.0, 1.0),
               bc=[("periodic", "periodic")] * 2, cfl=0.1, psi=psi)
    if name == "rk2d":
        cfg.update(kin=dict(Gamma=1.0, eps=2.0 * h / (order + 1), c_ip=1.0, grad_reg=1e-12, period=4.0),
                   t_end=4.0, centre=(0.5, 0.75))
    else:
        cfg.update(kin=dict(Gamma=1.0, eps=0.05, c_ip=1.0, grad_reg=1e-12, period=0.0),
                   t_end=1.0, centre=(0.5, 0.5))
    if eps is not None:
        cfg["kin"]["eps"] = float(eps)
    return cfg


def kinematic_fields(cfg, X):
    """(phi, psi, u0) at node coordinates X [2, ...]: phi = 1/(1 + exp(-psi/eps))
    with psi = R - r the signed distance to the droplet rim (positive inside)."""
    x, y = X[0], X[1]
    cx, cy = cfg["centre"]
    eps = cfg["kin"]["eps"]
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    phi = _sigmoid((0.15 - r) / eps)
    psi = 0.15 - r if cfg.get("psi", "cone") == "cone" else (0.15 ** 2 - r ** 2) / (2 * 0.15)
    if cfg["name"] == "rk2d":
        u0 = np.stack([np.sin(math.pi * x) ** 2 * np.sin(2 * math.pi * y),
                       -np.sin(2 * math.pi * x) * np.sin(math.pi * y) ** 2])
    else:
        u0 = np.stack([np.ones_like(x), np.zeros_like(x)])
    return phi, psi, u0


def kinematic_stream(cfg, X):
    """Nodal stream function S of the prescribed field, u0 = (dS/dy, -dS/dx):
    S = sin^2(pi x) sin^2(pi y) / pi for rk2d, S = y for adv2d."""
    x, y = X[0], X[1]
    if cfg["name"] == "rk2d":
        return np.sin(math.pi * x) ** 2 * np.sin(math.pi * y) ** 2 / math.pi
    return np.array(y, dtype=np.float64, copy=True)
