"""Quadrilaterals of degree 4 (the paper's order for the Rayleigh-Taylor and
rising-bubble runs) on the GPU through the C ABI, against the FP64 oracle at
p = 4: residuals under every boundary kind with the viscous, surface-tension
and gravity terms, RK steps and the device time step, the monitors, and
dg2p_advance / dg2p_advance_monitored bit for bit against dg2p_rk_step.  Metric and bar as in
test_gpu_parity.py (1e-12 per field)."""

import pytest
import torch

import oracle
from helpers import oracle_setup
from test_gpu_parity import TOL, res_errors, state_errors

pytestmark = pytest.mark.gpu


def _dg():
    from paper_2306_05002_amd import dg2p
    return dg2p


def case(name, ne, bc=None, **over):
    cfg, om, prm, U0 = oracle_setup(name, n_elem=ne, bc=bc, order=4, **over)
    dg = _dg()
    P = dg.make_params(cfg["params"])
    mesh = dg.mesh_from_config(cfg, P)
    assert mesh.nn == 25 and om.nn == 25
    return cfg, om, prm, U0, mesh, P


RHS = [
    ("drop2d", (5, 4), None),                 # periodic, inviscid
    ("drop2d", (1, 1), None),                 # one element, its own periodic neighbour
    ("drop2d", (3, 3), None),
    ("drop2d", (3, 2), None),                 # odd element count: the last wave's second half is empty
    ("bubble2d", (4, 6), None),               # no-slip bottom, Riemann top, slip sides; viscous, CSF, gravity
    ("rt2d", (3, 8), None),                   # viscous + gravity, walls
    ("shock2d", (6, 3), None),                # Dirichlet inflow, extrapolation outflow
    ("drop2d", (4, 5), [("no_slip", "no_slip"), ("no_slip", "no_slip")]),
]


@pytest.mark.parametrize("name,ne,bc", RHS)
def test_p4_rhs_parity(name, ne, bc):
    cfg, om, prm, U0, mesh, P = case(name, ne, bc)
    torch.manual_seed(5)
    # an asymmetric perturbation, so that every derivative and face term is
    # exercised; the level set too: at p = 4 a GLL node can sit exactly on the
    # tip of the droplets' cone psi = r - R, where grad psi is a cancellation
    # (~1e-17) and n = grad psi / |grad psi| an ill-conditioned direction
    U = U0.clone()
    U[2:2 + om.d] += 1e-2 * torch.randn(U[2:2 + om.d].shape, dtype=torch.float64) * U0[0].abs().max()
    U[3 + om.d + 1] += 1e-3 * torch.randn(U[0].shape, dtype=torch.float64)
    Ro = oracle.rhs(U, om, prm)
    Rg = _dg().rhs(mesh, P, U.cuda().contiguous()).cpu()
    rate = oracle.max_rate(U, om, prm)
    errs = res_errors(Rg, Ro, U, rate, prm, om.d)
    print(name, ne, ["%.1e" % e for e in errs])
    assert max(errs) <= TOL, errs


# (grids whose GLL nodes miss the droplets' cone tips; see test_p4_rhs_parity)
@pytest.mark.parametrize("name,ne", [("bubble2d", (3, 5)), ("rt2d", (2, 6)), ("shock2d", (5, 4))])
def test_p4_rk_step_and_dt_parity(name, ne):
    cfg, om, prm, U0, mesh, P = case(name, ne)
    dg = _dg()
    Ud = U0.cuda().contiguous()
    dt = dg.max_dt(mesh, P, Ud, cfl=0.1)
    dto = oracle.max_dt(U0, om, prm, cfl=0.1)
    assert abs(float(dt.cpu()) - dto) <= TOL * dto
    dg.rk_step(mesh, P, Ud, dt)
    U1 = oracle.rk_step(U0, float(dt.cpu()), om, prm)
    errs = state_errors(Ud.cpu(), U1, prm, om.d)
    assert max(errs) <= TOL, errs


@pytest.mark.parametrize("name,ne", [("rt2d", (3, 7)), ("bubble2d", (4, 5))])
def test_p4_advance_and_monitors(name, ne):
    """Three steps of dg2p_advance (device dt, carried face ingredients) equal
    max_dt + rk_step bit for bit and match the oracle; the monitors match the
    oracle's."""
    cfg, om, prm, U0, mesh, P = case(name, ne)
    dg = _dg()
    A = U0.cuda().contiguous()
    B = A.clone()
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dg.advance(mesh, P, A, 3, cfl=0.1, t=t)
    Uo = U0
    for _ in range(3):
        dt = dg.max_dt(mesh, P, B, cfl=0.1)
        dg.rk_step(mesh, P, B, dt)
        Uo = oracle.rk_step(Uo, float(dt.cpu()), om, prm)
    assert torch.equal(A, B)
    assert max(state_errors(A.cpu(), Uo, prm, om.d)) <= 1e-11
    mg = dg.monitors(mesh, P, A, p_ref=1.0)
    mo = oracle.monitors(Uo, om, prm, p_ref=1.0, u_ref=[0.0, 0.0])
    scales = [float((Uo[f].abs() * om.node_weights()).sum()) for f in range(om.nf)]
    for f in range(om.nf):
        # momentum starts at rest (its integral is a cancellation of ~1e-6
        # values): a floor of 1e-13 of the largest field's scale
        tol = 1e-11 * scales[f] + 1e-13 * max(scales)
        assert abs(mg["integral"][f] - float(mo["integral"][f])) <= tol, f
    assert abs(mg["min_alpha"] - mo["min_alpha"]) <= 1e-11 and abs(mg["max_alpha"] - mo["max_alpha"]) <= 1e-11
    assert mg["nonphys"] == mo["nonphys"] == 0
    assert abs(mg["max_rate"] - mo["max_rate"]) <= 1e-11 * mo["max_rate"]


@pytest.mark.parametrize("name,ne", [("bubble2d", (16, 32)), ("rt2d", (16, 64))])
def test_p4_bench_grid_step_against_the_oracle(name, ne):
    """The grids the benchmark runs at p = 4 (rising bubble 16 x 32, RT
    16 x 64, at CFL 0.05), in its launch configuration: one dg2p_advance step
    (device dt) against the oracle's step from the same state, dt to 1e-14
    and every field to 1e-12.  The level set is perturbed as in the residual
    tests (the bubble's cone tip sits on a GLL node of this grid)."""
    cfg, om, prm, U0, mesh, P = case(name, ne)
    dg = _dg()
    torch.manual_seed(11)
    U = U0.clone()
    U[3 + om.d + 1] += 1e-3 * torch.randn(U[0].shape, dtype=torch.float64)
    dto = oracle.max_dt(U, om, prm, cfl=0.05)
    Uo = oracle.rk_step(U, dto, om, prm)
    A = U.cuda().contiguous()
    last = torch.zeros(1, dtype=torch.float64, device="cuda")
    dg.advance(mesh, P, A, 1, cfl=0.05, dt_last=last)
    assert abs(float(last.cpu()) - dto) <= 1e-14 * dto
    errs = state_errors(A.cpu(), Uo, prm, om.d)
    print(name, ["%.1e" % e for e in errs])
    assert max(errs) <= TOL, errs


# one-wave workgroups of two quads: bubble2d 6x5 (15 workgroups) and 16x32
# (256, the largest grid whose first stage reduces the records itself) take
# the fused reduction of dt and the monitors; rt2d 3x7 (11) fuses dt only,
# 16x64 (512) neither
@pytest.mark.parametrize("name,ne", [("bubble2d", (6, 5)), ("bubble2d", (16, 32)), ("rt2d", (3, 7)),
                                     ("rt2d", (16, 64))])
def test_p4_advance_monitored_every_step(name, ne):
    """dg2p_advance_monitored at p = 4: the same states and time as
    dg2p_advance bit for bit, and every step's monitors equal to the
    stand-alone monitors of that step's state (alpha range and non-physical
    count exactly, rate and dt to rounding, integrals up to the summation
    order)."""
    cfg, om, prm, U0, mesh, P = case(name, ne)
    dg = _dg()
    steps = 3
    A = U0.cuda().contiguous()
    B = A.clone()
    ms = torch.zeros(steps, dg.MONITOR_DOUBLES, dtype=torch.float64, device="cuda")
    tA = torch.zeros(1, dtype=torch.float64, device="cuda")
    tB = torch.zeros(1, dtype=torch.float64, device="cuda")
    dg.advance_monitored(mesh, P, A, steps, ms, cfl=0.05, t=tA)
    dg.advance(mesh, P, B, steps, cfl=0.05, t=tB)
    assert torch.equal(A, B) and torch.equal(tA, tB)
    rows = dg.decode_monitors(ms, mesh.nf)
    C = U0.cuda().contiguous()
    for i in range(steps):
        dt = dg.max_dt(mesh, P, C, cfl=0.05)
        dg.rk_step(mesh, P, C, dt)
        ref = dg.monitors(mesh, P, C)
        got = rows[i]
        assert got["min_alpha"] == ref["min_alpha"] and got["max_alpha"] == ref["max_alpha"]
        assert got["nonphys"] == ref["nonphys"] == 0
        assert abs(got["max_rate"] - ref["max_rate"]) <= 1e-14 * ref["max_rate"]
        dtr = float(dg.max_dt(mesh, P, C, cfl=0.05).cpu())
        assert abs(got["dt"] - dtr) <= 1e-14 * dtr
        for f in range(mesh.nf):
            scale = float(torch.abs(C[f]).max()) * sum(mesh.node_weights()) * mesh.E + 1e-300
            assert abs(got["integral"][f] - ref["integral"][f]) <= 1e-14 * scale, (i, f)
    assert torch.equal(A, C)


def test_p4_rejects_what_it_does_not_run():
    """p = 4: FP64 two-phase path only (no mixed forms, adjoint or kinematic
    mode), and quadrilaterals only."""
    dg = _dg()
    cfg = oracle_setup("drop2d", n_elem=(2, 2), order=4)[0]
    mesh = dg.mesh_from_config(cfg)
    U = torch.zeros(mesh.nf, mesh.E, mesh.nn, dtype=torch.float64, device="cuda")
    with pytest.raises(dg.Dg2pError) as ei:
        dg.rhs(mesh, dg.make_params(cfg["params"], precision="fp32"), U)
    assert ei.value.status == dg.EUNSUPPORTED
    with pytest.raises(dg.Dg2pError) as ei:
        dg.rhs_vjp(mesh, dg.make_params(cfg["params"]), U, U.clone())
    assert ei.value.status == dg.EUNSUPPORTED
    Phi = torch.zeros(2, mesh.E, mesh.nn, dtype=torch.float64, device="cuda")
    with pytest.raises(dg.Dg2pError) as ei:
        dg.kin_rhs(mesh, dg.make_kin_params(), Phi, Phi.clone(), 0.0)
    assert ei.value.status == dg.EUNSUPPORTED
    with pytest.raises(dg.Dg2pError) as ei:
        dg.Mesh(3, (2, 2, 2), (0.0,) * 3, (1.0,) * 3, order=4)
    assert ei.value.status == dg.EUNSUPPORTED
