"""Pins of the oracle's wall and Riemann-invariant boundaries (no GPU).

The no-slip wall and the Riemann-invariant far field are the boundaries of
the paper's Rayleigh-Taylor and rising-bubble cases (Sections
"Rayleigh-Taylor instability" and "Rising bubble"); the paper names them
without formulas, so each is pinned to what its definition fixes:
  * the Riemann ghost carries the interior's outgoing invariant and the far
    field's incoming one, and is transparent to a state at the far-field
    pressure at rest;
  * wall ghosts make the discrete operator conserve both partial masses and
    the total energy;
  * a uniform stream along a no-slip wall feels exactly the drag of the
    Lax-Friedrichs and viscous-penalty fluxes against a ghost at -u, and
    none along a slip wall.
"""

import math

import pytest
import torch

import oracle
from oracle import residual
from oracle.physics import primitives

torch.set_default_dtype(torch.float64)


def _prm(**kw):
    base = dict(gamma=(4.4, 1.4), pinf=(6.0e4, 0.0), rho0=(1000.0, 100.0), Gamma=1.0, eps=0.01,
                mu=(0.0, 0.0), sigma=0.0, g=(0.0, 0.0, 0.0))
    base.update(kw)
    return oracle.Params(**base)


def _state(alpha, psi, rho1, rho2, u, P, prm):
    T = lambda v: torch.as_tensor(v, dtype=torch.float64)
    return oracle.prim_to_cons(T(alpha), T(psi), T(rho1), T(rho2), T(u), T(P), prm)


@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("k", [0, 1])
def test_riemann_ghost_carries_the_two_invariants(k, side):
    prm = _prm()
    gen = torch.Generator().manual_seed(11)
    n = 64
    alpha = torch.rand(n, generator=gen)
    u = 0.3 * torch.randn(2, n, generator=gen)
    P = 1500.0 + 500.0 * torch.rand(n, generator=gen)
    Q = _state(alpha, torch.randn(n, generator=gen), 1000.0 + torch.rand(n, generator=gen),
               100.0 + torch.rand(n, generator=gen), u, P, prm)
    P_b = 1200.0
    G = residual._riemann_ghost(Q, k, side, 2, P_b, prm)
    pi, pg = primitives(Q, 2, prm), primitives(G, 2, prm)
    sm = 1.0 if side == 1 else -1.0
    # the far field: the interior composition and density at rest under P_b,
    # through the initial-condition map and the closure
    rho1 = Q[0] / alpha
    rho2 = Q[1] / (1.0 - alpha)
    far = primitives(_state(alpha, Q[6], rho1, rho2, torch.zeros(2, n), torch.full((n,), P_b), prm), 2, prm)
    xi = pi["xi"]
    j_out_i = sm * pi["u"][k] + 2.0 * xi * pi["c"]
    j_out_g = sm * pg["u"][k] + 2.0 * xi * pg["c"]
    j_in_g = sm * pg["u"][k] - 2.0 * xi * pg["c"]
    j_in_far = -2.0 * xi * far["c"]
    scale = float((2.0 * xi * pi["c"]).max())
    assert float((j_out_g - j_out_i).abs().max()) <= 1e-12 * scale
    assert float((j_in_g - j_in_far).abs().max()) <= 1e-12 * scale
    t = 1 - k
    assert float((pg["u"][t] - pi["u"][t]).abs().max()) <= 1e-13
    for f in (0, 1, 5, 6):       # partial densities, alpha, psi
        assert torch.equal(G[f], Q[f])


def _uniform(om, prm, alpha, u, P, psi_slope=(0.3, -0.2)):
    X = om.node_coords()
    psi = psi_slope[0] * X[0] + psi_slope[1] * X[1]
    shp = X.shape[1:]
    return _state(torch.full(shp, alpha), psi, torch.full(shp, prm.rho0[0]), torch.full(shp, prm.rho0[1]),
                  torch.stack([torch.full(shp, u[0]), torch.full(shp, u[1])]), torch.full(shp, P), prm)


@pytest.mark.parametrize("bc", [
    [("slip_wall", "slip_wall"), ("no_slip", "riemann")],
    [("riemann", "riemann"), ("no_slip", "no_slip")],
])
def test_rest_state_at_far_field_pressure_is_steady(bc):
    """alpha uniform, u = 0, P = P_b: every ghost equals the interior trace, so
    R vanishes to round-off (viscous on, no gravity)."""
    prm = _prm(mu=(10.0, 1.0))
    P_b = 1300.0
    om = oracle.OracleMesh(2, 3, (3, 4), (-0.5, 0.0), (0.5, 2.0), bc,
                           {(k, s): torch.tensor([P_b]) for k in range(2) for s in range(2)})
    U = _uniform(om, prm, 1.0, (0.0, 0.0), P_b)
    R = oracle.rhs(U, om, prm)
    c = float(primitives(U, 2, prm)["c"].max())
    for f in range(7):
        # zero fields (q2 of a pure phase, momentum at rest) take the mass scale
        scale = max(float(U[f].abs().max()), float(U[0].abs().max())) * c / min(om.h)
        assert float(R[f].abs().max()) <= 1e-11 * scale, (f, float(R[f].abs().max()))


def _integral(R, om):
    w = torch.outer(om.w, om.w).reshape(-1) * (om.J[0] * om.J[1])   # node index = a_x + 4 a_y
    return (R * w).sum(dim=(1, 2))


@pytest.mark.parametrize("kind", ["no_slip", "slip_wall"])
def test_walls_conserve_mass_and_energy(kind):
    """A smooth two-phase state with velocity in a box walled on all four
    sides (viscous, no gravity, no surface tension): the integrals of the
    partial-density and energy residuals vanish."""
    prm = _prm(mu=(10.0, 1.0), eps=0.05)
    om = oracle.OracleMesh(2, 3, (4, 5), (-0.5, 0.0), (0.5, 2.0), [(kind, kind)] * 2)
    X = om.node_coords()
    psi = torch.sqrt(X[0] ** 2 + (X[1] - 0.8) ** 2) - 0.3
    alpha = 1.0 / (1.0 + torch.exp(-psi / prm.eps))
    u = torch.stack([0.2 * torch.sin(3.0 * X[1]) + 0.1, 0.15 * torch.cos(2.0 * X[0]) - 0.05])
    P = 2000.0 + 300.0 * X[1]
    U = _state(alpha, psi, torch.full_like(psi, 1000.0), torch.full_like(psi, 100.0), u, P, prm)
    R = oracle.rhs(U, om, prm)
    I = _integral(R, om)
    Iabs = _integral(R.abs(), om)
    for f in (0, 1, 4):
        assert abs(float(I[f])) <= 1e-12 * float(Iabs[f]), (f, float(I[f]), float(Iabs[f]))


@pytest.mark.parametrize("kind", ["no_slip", "slip_wall"])
def test_uniform_stream_along_a_wall(kind):
    """u = (0, v0) uniform, walls at x = -0.5, 0.5, periodic in y, single phase:
    no-slip walls take tangential momentum at the rate
    Ly v0 (lambda rho + 2 eta_v) per wall (Lax-Friedrichs dissipation with
    lambda = c, and the viscous penalty eta_v = c_ip mu (p+1)^2 / h_x against
    the ghost velocity -v0); slip walls take none."""
    prm = _prm(mu=(10.0, 1.0))
    v0 = 0.2
    om = oracle.OracleMesh(2, 3, (3, 2), (-0.5, 0.0), (0.5, 2.0), [(kind, kind), ("periodic", "periodic")])
    U = _uniform(om, prm, 1.0, (0.0, v0), 1500.0, psi_slope=(0.0, 0.0))
    R = oracle.rhs(U, om, prm)
    I = _integral(R, om)
    pr = primitives(U, 2, prm)
    rho, c = float(pr["rho"].mean()), float(pr["c"].mean())
    Ly = om.hi[1] - om.lo[1]
    eta = prm.c_ip * prm.mu[0] * (om.p + 1) ** 2 / om.h[0]
    want = -2.0 * Ly * v0 * (c * rho + 2.0 * eta) if kind == "no_slip" else 0.0
    scale = 2.0 * Ly * v0 * (c * rho + 2.0 * eta)
    assert abs(float(I[3]) - want) <= 1e-12 * scale, (float(I[3]), want)
    assert abs(float(I[2])) <= 1e-12 * scale        # no normal force from a uniform pressure
    for f in (0, 1):
        assert abs(float(I[f])) <= 1e-12 * scale
