"""Pins of the oracle's kinematic mode (phase field and level set under a
prescribed velocity) against closed forms, textbook DG properties and the
oracle's full residual.  CPU only."""

import math

import pytest
import torch

import oracle
from oracle import kinematic as K

torch.set_default_dtype(torch.float64)


def _mesh(d, N, p=3):
    return oracle.OracleMesh(d, p, (N,) * d, (0.0,) * d, (1.0,) * d)


@pytest.mark.parametrize("p", [3, 1])
def test_upwind_energy_identity(p):
    """Gamma = 0, constant u: the upwind DG transport operator dissipates
    exactly sum_faces |u.m| [[phi]]^2 / 2 per unit face measure (GLL/SBP
    identity), i.e. sum_j W_j phi_j R_j = -1/2 sum_faces |u.m| |f| (jump)^2.
    Fails on a wrong sign of the hat/tilde correction, of the volume term, or
    on a wrong lift factor."""
    torch.manual_seed(0)
    for d, N in ((1, 7), (2, 3)):
        mesh = _mesh(d, N, p)
        kp = K.KinParams(Gamma=0.0)
        u = torch.tensor([0.7, -0.4][:d]).view(d, 1, 1).expand(d, mesh.E, mesh.nn).clone()
        Phi = torch.randn(2, mesh.E, mesh.nn)
        R = K.kin_rhs(Phi, u, mesh, kp)
        W = mesh.node_weights()
        lhs = (Phi * R * W).sum(dim=(1, 2))
        # face dissipation: every face once, with the face-node quadrature weights
        n = mesh.n
        w = mesh.w
        want = torch.zeros(2)
        el = torch.arange(mesh.E)
        shp = (2, mesh.E) + (n,) * d
        P = Phi.reshape(shp)
        for k in range(d):
            nb, _ = mesh.neighbour(el, k, 1)
            right = P.select(P.dim() - 1 - k, n - 1)
            left_of_nb = P[:, nb].select(P.dim() - 1 - k, 0)
            jump2 = (right - left_of_nb) ** 2
            fw = torch.ones(())
            for kk in range(d):
                if kk != k:
                    fw = fw * mesh.J[kk]
            if d == 2:
                jw = jump2 * w.view(1, 1, n) * fw
            else:
                jw = jump2 * fw
            want += -0.5 * abs(float(u[k, 0, 0])) * jw.reshape(2, -1).sum(1)
        assert torch.allclose(lhs, want, rtol=1e-12, atol=1e-12), (lhs, want)


def test_upwind_lift_closed_form_1d():
    """Gamma = 0, u = 1, phi constant per element: only the inflow node of
    each element changes, R = (phi_{e-1} - phi_e) / (w_0 J) = 12/h (...)."""
    N = 5
    mesh = _mesh(1, N)
    kp = K.KinParams(Gamma=0.0)
    vals = torch.tensor([0.3, -1.0, 2.0, 0.5, 4.0])
    Phi = torch.stack([vals[:, None].expand(N, 4), -vals[:, None].expand(N, 4)]).clone()
    u = torch.ones(1, N, 4)
    R = K.kin_rhs(Phi, u, mesh, kp)
    h = 1.0 / N
    want = torch.zeros(2, N, 4)
    want[0, :, 0] = (12.0 / h) * (vals.roll(1) - vals)
    want[1, :, 0] = -(12.0 / h) * (vals.roll(1) - vals)
    assert torch.allclose(R, want, rtol=1e-13, atol=1e-11)


def test_upwind_lift_closed_form_1d_p1():
    """The same at p = 1 (two nodes, w_0 = 1): R = (phi_{e-1} - phi_e) / J
    = 2/h (...) at the inflow node, zero at the other."""
    N = 5
    mesh = _mesh(1, N, 1)
    kp = K.KinParams(Gamma=0.0)
    vals = torch.tensor([0.3, -1.0, 2.0, 0.5, 4.0])
    Phi = torch.stack([vals[:, None].expand(N, 2), -vals[:, None].expand(N, 2)]).clone()
    R = K.kin_rhs(Phi, torch.ones(1, N, 2), mesh, kp)
    h = 1.0 / N
    want = torch.zeros(2, N, 2)
    want[0, :, 0] = (2.0 / h) * (vals.roll(1) - vals)
    want[1, :, 0] = -(2.0 / h) * (vals.roll(1) - vals)
    assert torch.allclose(R, want, rtol=1e-13, atol=1e-11)


@pytest.mark.parametrize("p", [3, 1])
def test_sipg_block_symmetric_nsd_and_conservative(p):
    """u = 0, psi = 0 (exactly zero gradient, so n = 0): the phi operator is
    the linear SIPG Laplacian Gamma eps div grad; W A is symmetric, negative
    semidefinite with the constants as its only null space (fails on a wrong
    sign or weight of the symmetric term or the penalty), and
    sum_j W_j R_j = 0."""
    mesh = _mesh(2, 3 if p == 3 else 5, p)
    kp = K.KinParams(Gamma=1.3, eps=0.05)
    u = torch.zeros(2, mesh.E, mesh.nn)
    psi = torch.zeros(mesh.E, mesh.nn)

    def rphi(v):
        return K.kin_rhs(torch.stack([v.reshape(mesh.E, mesh.nn), psi]), u, mesh, kp)[0].reshape(-1)

    x0 = torch.rand(mesh.E * mesh.nn)
    Jm = torch.autograd.functional.jacobian(rphi, x0)
    W = mesh.node_weights().repeat(mesh.E)
    A = W[:, None] * Jm
    scale = float(torch.abs(A).max())
    assert float(torch.abs(A - A.T).max()) < 1e-10 * scale
    ev = torch.linalg.eigvalsh(0.5 * (A + A.T))
    assert float(ev.max()) < 1e-9 * scale
    assert int((torch.abs(ev) < 1e-9 * scale).sum()) == 1
    assert abs(float((W * rphi(x0)).sum())) < 1e-11 * scale


def test_matches_full_residual_on_continuous_fields():
    """Globally continuous phi and psi (no face jumps) and a uniform velocity:
    the kinematic residual equals the alpha and psi rows of the full
    two-phase residual with that velocity and uniform pressure (the two share
    the volume terms and the a-flux faces; only jump-weighted terms, zero
    here, differ)."""
    mesh = _mesh(2, 4)
    X = mesh.node_coords()
    prm = oracle.Params(eps=0.04, Gamma=1.1)
    kp = K.KinParams(Gamma=1.1, eps=0.04)
    psi = 0.3 * torch.sin(2 * math.pi * X[0]) * torch.cos(2 * math.pi * X[1]) + 0.05
    phi = torch.sigmoid(psi / 0.04)
    uvec = torch.stack([torch.full_like(phi, 0.8), torch.full_like(phi, -0.3)])
    one = torch.ones_like(phi)
    U = oracle.prim_to_cons(phi, psi, one, 10 * one, uvec, one, prm)
    Rf = oracle.rhs(U, mesh, prm)
    Rk = K.kin_rhs(torch.stack([phi, psi]), uvec, mesh, kp)
    scale = float(torch.abs(Rk).max())
    assert float(torch.abs(Rk[0] - Rf[5]).max()) < 1e-12 * scale
    assert float(torch.abs(Rk[1] - Rf[6]).max()) < 1e-12 * scale


def test_rk4_taylor_on_linear_operator():
    """Gamma = 0, constant u: the operator is linear, and one classical RK4
    step is exactly the degree-4 Taylor polynomial of exp(dt L)."""
    mesh = _mesh(1, 6)
    kp = K.KinParams(Gamma=0.0)
    u0 = torch.ones(1, mesh.E, mesh.nn)
    torch.manual_seed(1)
    Phi = torch.randn(2, mesh.E, mesh.nn)
    dt = 0.013
    Lop = lambda V: K.kin_rhs(V, u0, mesh, kp)
    terms = [Phi]
    for k in range(1, 5):
        terms.append(Lop(terms[-1]) * (dt / k))
    want = sum(terms)
    got = K.rk4_step(Phi, 0.0, dt, u0, mesh, kp)
    assert torch.allclose(got, want, rtol=1e-12, atol=1e-12)


def test_rk4_fourth_order_with_time_dependent_rate():
    """y' = cos(t) y (exact exp(sin t)): the global error over [0, 2] falls by
    2^4 per halving of dt (fails on wrong stage times or weights)."""
    errs = []
    for ns in (20, 40, 80):
        dt = 2.0 / ns
        y = torch.tensor([1.0])
        t = 0.0
        for _ in range(ns):
            y = K.rk4_step(y, t, dt, None, None, None, rhs_fn=lambda v, s: math.cos(s) * v)
            t += dt
        errs.append(abs(float(y) - math.exp(math.sin(2.0))))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 3.8, (errs, orders)


def test_time_factor_and_rider_kothe_field():
    """s(t) = cos(pi t / T) reverses the flow at T/2; the single-vortex field
    is divergence free (checked with the exact derivatives) and has zero
    normal velocity on the boundary of the unit square."""
    kp = K.KinParams(period=4.0)
    assert abs(K.time_factor(2.0, kp)) < 1e-15 and abs(K.time_factor(4.0, kp) + 1.0) < 1e-15
    x = torch.rand(200)
    y = torch.rand(200)
    pi = math.pi
    div = (2 * pi * torch.sin(pi * x) * torch.cos(pi * x) * torch.sin(2 * pi * y)
           - torch.sin(2 * pi * x) * 2 * pi * torch.sin(pi * y) * torch.cos(pi * y))
    assert float(torch.abs(div).max()) < 1e-12
    edge = torch.linspace(0, 1, 11)
    u = K.rider_kothe_velocity(torch.stack([torch.zeros(11), edge]))
    v = K.rider_kothe_velocity(torch.stack([edge, torch.zeros(11)]))
    assert float(torch.abs(u[0]).max()) < 1e-15 and float(torch.abs(v[1]).max()) < 1e-15


@pytest.mark.parametrize("p", [3, 1])
def test_time_step_rule(p):
    mesh = _mesh(2, 8, p)
    kp = K.KinParams(Gamma=2.0, eps=0.01)
    u0 = torch.zeros(2, mesh.E, mesh.nn)
    u0[0] = 0.5
    u0[1, 3, 3] = -1.5
    h = 1.0 / 8
    rate = (2.0 + (16 if p == 3 else 4) * 2 * 2.0 * 0.01 / h) / h
    assert abs(K.max_dt(u0, mesh, kp, cfl=0.2) - 0.2 / rate) < 1e-15


@pytest.mark.parametrize("p", [3, 1])
def test_profile_advection_converges_at_p_plus_1(p):
    """The paper's linear-advection check in one dimension: an equilibrium
    slab profile (fixed eps = 0.02) carried by u = 1 keeps its shape, and the
    L1 error against the translated profile falls at the optimal rate
    p + 1 = 4, with and without the Allen-Cahn terms.  (The periodic distance
    of a 2D droplet has kinks where phi ~ e^(-(0.5 - R)/eps); with the
    paper's eps = 0.05 those cap every DG scheme near order 3.)"""
    T, eps = 0.05, 0.02
    for G in (1.0, 0.0):
        errs = []
        for N in ((16, 32, 64) if p == 3 else (64, 128, 256)):
            mesh = _mesh(1, N, p)
            X = mesh.node_coords()
            kp = K.KinParams(Gamma=G, eps=eps)

            def fields(s):
                psi = torch.abs((X[0] - s) % 1.0 - 0.5) - 0.25
                return torch.sigmoid(psi / eps), psi

            phi0, psi0 = fields(0.0)
            u0 = torch.ones(1, mesh.E, mesh.nn)
            ns = int(math.ceil(T / K.max_dt(u0, mesh, kp, cfl=0.1)))
            dt = T / ns
            Phi = torch.stack([phi0, psi0])
            t = 0.0
            for _ in range(ns):
                Phi = K.rk4_step(Phi, t, dt, u0, mesh, kp)
                t += dt
            errs.append(K.l1_error(Phi[0], fields(T)[0], mesh))
        orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert orders[-1] > (3.7 if p == 3 else 1.8), (G, errs, orders)


# ---- level-set re-initialisation ------------------------------------------------
def test_reinit_diffusion_block_symmetric_nsd():
    """sgn = 0: the re-initialisation operator is the SIPG Laplacian with the
    vanishing viscosity nu_h; W A is symmetric, negative semidefinite with the
    constants as its only null space, and conservative."""
    mesh = _mesh(2, 3)
    nu, _ = K.reinit_params(mesh)
    sgn = torch.zeros(mesh.E, mesh.nn)

    def r(v):
        return K.reinit_rhs(v.reshape(mesh.E, mesh.nn), sgn, mesh, nu, 1.0).reshape(-1)

    x0 = torch.rand(mesh.E * mesh.nn)
    Jm = torch.autograd.functional.jacobian(r, x0)
    W = mesh.node_weights().repeat(mesh.E)
    A = W[:, None] * Jm
    scale = float(torch.abs(A).max())
    assert float(torch.abs(A - A.T).max()) < 1e-10 * scale
    ev = torch.linalg.eigvalsh(0.5 * (A + A.T))
    assert float(ev.max()) < 1e-9 * scale
    assert int((torch.abs(ev) < 1e-9 * scale).sum()) == 1
    assert abs(float((W * r(x0)).sum())) < 1e-11 * scale


def test_reinit_source_relaxes_slope():
    """psi = 2 (x - 1/2), sgn = sign(psi): away from the periodic seam the
    diffusion of a linear field vanishes and R = sgn (1 - |grad psi|) = -sgn,
    i.e. the iteration lowers |psi| where the slope exceeds 1 (the standard
    Eikonal relaxation; fails on a flipped source sign)."""
    mesh = _mesh(1, 8)
    X = mesh.node_coords()[0]
    psi = 2.0 * (X - 0.5)
    sgn = torch.sign(psi)
    nu, _ = K.reinit_params(mesh)
    R = K.reinit_rhs(psi, sgn, mesh, nu, 1.0)
    inner = slice(1, 7)  # elements not touching the seam at x = 0 = 1
    assert float(torch.abs(R[inner] + sgn[inner]).max()) < 1e-12


def test_reinit_converges_to_distance_near_interface():
    """Slab phi = sigmoid((|x - 1/2| - 1/4) / eps): the iteration from
    psi0 = phi - 1/2 keeps the zero level at x = 1/4, 3/4 and turns the
    slope there into 1 (a signed distance near the interface)."""
    N = 32
    mesh = _mesh(1, N)
    X = mesh.node_coords()[0]
    eps = 0.5 / N
    kp = K.KinParams(eps=eps)
    phi = torch.sigmoid((torch.abs(X - 0.5) - 0.25) / eps)
    nu, dtau = K.reinit_params(mesh)
    psi = K.reinit(phi, mesh, kp, 800, nu, dtau)
    g = K._dk(psi.reshape(N, 4), 0, mesh).reshape(-1)
    xs, ps = X.reshape(-1), psi.reshape(-1)
    near = (torch.abs(xs - 0.25) < 0.02) | (torch.abs(xs - 0.75) < 0.02)
    assert float(torch.abs(g[near].abs() - 1.0).max()) < 1e-3
    for x0 in (0.25, 0.75):
        i = int(torch.argmin(torch.abs(xs - x0)))
        assert abs(float(ps[i])) < 1e-6


# ---- velocity representation and the mass balance ---------------------------------

@pytest.mark.parametrize("p", [3, 1])
def test_velocity_from_stream_differentiates_polynomials_exactly(p):
    """A stream function of degree <= p per axis is interpolated exactly, so
    u0 = (dS/dy, -dS/dx) is exact at the nodes (fails on swapped axes, a
    wrong sign or a wrong Jacobian)."""
    mesh = oracle.OracleMesh(2, p, (3, 4), (0.0, -1.0), (1.5, 1.0))
    x, y = mesh.node_coords()
    if p == 3:
        S = x ** 3 * y ** 2 + 2 * x * y ** 3 - y
        want = torch.stack([2 * x ** 3 * y + 6 * x * y ** 2 - 1, -(3 * x ** 2 * y ** 2 + 2 * y ** 3)])
    else:
        S = x * y + 3 * x - 2 * y
        want = torch.stack([x - 2, -(y + 3)])
    u0 = K.velocity_from_stream(S, mesh)
    assert float((u0 - want).abs().max()) < 1e-11


@pytest.mark.parametrize("p", [3, 1])
def test_mass_balance_is_the_discrete_divergence_of_the_velocity(p):
    """Random phi and psi, Gamma > 0, a nodally interpolated velocity field
    (continuous at the shared face nodes): sum_j W_j R_phi_j equals
    sum_j W_j phi_j (div_h u)_j to rounding (the upwind face terms, the
    SIPG a-flux and its symmetric term all cancel in the sum), and is zero to
    rounding for the stream-function velocity, whose div_h u vanishes.  Fails
    on a wrong upwind sign, an unpaired face term or a lift factor that does
    not match the face quadrature."""
    torch.manual_seed(3)
    N = 6 if p == 3 else 9
    mesh = oracle.OracleMesh(2, p, (N, N - 1), (0.0, 0.0), (1.0, 1.0))
    x, y = mesh.node_coords()
    kp = K.KinParams(Gamma=0.7, eps=0.04)
    Phi = torch.stack([torch.rand(mesh.E, mesh.nn), torch.randn(mesh.E, mesh.nn)])
    W = mesh.node_weights()
    u_nodal = K.rider_kothe_velocity(torch.stack([x, y]))
    n = mesh.n
    div = (K._dk(u_nodal[0].reshape(-1, n, n), 0, mesh) + K._dk(u_nodal[1].reshape(-1, n, n), 1, mesh)).reshape(
        mesh.E, mesh.nn)
    R = K.kin_rhs(Phi, u_nodal, mesh, kp)
    got = float((W * R[0]).sum())
    want = float((W * Phi[0] * div).sum())
    scale = float((W * (R[0].abs() + (Phi[0] * div).abs())).sum())
    assert abs(got - want) < 1e-13 * scale, (got, want)
    assert abs(want) > 1e-6 * scale            # the nodal field is not discretely divergence free
    S = torch.sin(math.pi * x) ** 2 * torch.sin(math.pi * y) ** 2 / math.pi
    Rs = K.kin_rhs(Phi, K.velocity_from_stream(S, mesh), mesh, kp)
    assert abs(float((W * Rs[0]).sum())) < 1e-13 * float((W * Rs[0].abs()).sum())
