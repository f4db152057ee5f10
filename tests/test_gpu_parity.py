"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Metric (per field f): e_f = max|X_gpu - X_oracle| / max(max|X_oracle|, S_f)
with S_f = M_f * rate for residuals (rate = the time-step rule's largest
rate, i.e. the size of R that a state of that magnitude can produce) and
S_f = M_f for states, where M_f = max|U_f| except for momentum components,
M_f = max rho (|u| + c) (a momentum component may vanish identically while
its residual carries pressure round-off).  Bar: e_f <= 1e-12 for FP64.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from helpers import oracle_setup, field_scales
from paper_2306_05002_amd import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _dg():
    from paper_2306_05002_amd import dg2p
    return dg2p


def gpu_case(name, n_elem=None, variant=None, bc=None, bc_state=None, **over):
    order = over.pop("order", 3)
    cfg, om, prm, U0 = oracle_setup(name, n_elem=n_elem, variant=variant, bc=bc, bc_state=bc_state, order=order,
                                    **over)
    dg = _dg()
    P = dg.make_params({**cfg["params"], **over})
    mesh = dg.mesh_from_config(dict(cfg, params={**cfg["params"], **over}), P)
    return cfg, om, prm, U0, mesh, P


def res_errors(Rg, Ro, U, rate, prm, d):
    out = []
    M = field_scales(U, d, prm)
    for f in range(U.shape[0]):
        den = max(float(Ro[f].abs().max()), M[f] * rate)
        out.append(float((Rg[f] - Ro[f]).abs().max()) / den)
    return out


def state_errors(Ug, Uo, prm, d):
    M = field_scales(Uo, d, prm)
    return [float((Ug[f] - Uo[f]).abs().max()) / max(float(Uo[f].abs().max()), M[f], 1e-300)
            for f in range(Uo.shape[0])]


SMALL = [
    ("drop1d", None, None),
    ("drop1d", None, "noisy_u"),
    ("drop1d", (37,), "noisy_u"),      # ragged: 37 elements, 16 per wave
    ("drop1d", (1,), None),            # single element, its own periodic neighbour
    ("drop2d", (12, 10), None),
    ("drop2d", (7, 5), None),          # ragged: 35 elements, 4 per wave
    ("drop2d", (1, 1), None),
    ("shock2d", (16, 8), None),        # Dirichlet inflow, extrapolated outflow
    ("shock2d", (13, 7), None),
    ("adjoint2d", (10, 9), None),      # viscous + CSF
    ("rt3d", (5, 4, 6), None),         # viscous + CSF + gravity + slip walls
    ("rt3d", (1, 1, 2), None),
    ("waterair2d", (6, 5), None),      # density ratio 1000, P_inf 6000
    ("bubble2d", (4, 8), None),        # no-slip bottom, Riemann top, slip sides; viscous + CSF + gravity
    ("bubble2d", (5, 7), None),        # ragged: 35 elements
    ("rt2d", (3, 8), None),            # viscous + gravity, same boundaries, no surface tension
]


@pytest.mark.parametrize("name,ne,variant", SMALL)
def test_rhs_parity(name, ne, variant):
    cfg, om, prm, U0, mesh, P = gpu_case(name, ne, variant)
    dg = _dg()
    Ro = oracle.rhs(U0, om, prm)
    Rg = dg.rhs(mesh, P, U0.cuda().contiguous()).cpu()
    rate = oracle.max_rate(U0, om, prm)
    errs = res_errors(Rg, Ro, U0, rate, prm, om.d)
    print(name, ne, variant, ["%.1e" % e for e in errs])
    assert max(errs) <= TOL, errs


WALL_KINDS = [
    # 3D: no-slip in x, Riemann top (the column's own top pressure) over a no-slip bottom in z
    ("rt3d", (2, 3, 3), [("no_slip", "no_slip"), ("periodic", "periodic"), ("no_slip", "riemann")],
     {(2, 1): [1.0]}),
    # 3D: walls across y (the y-face jobs of each z-layer meet the boundary), periodic z
    ("rt3d", (3, 2, 2), [("periodic", "periodic"), ("no_slip", "riemann"), ("periodic", "periodic")],
     {(1, 1): [1.0]}),
    # 1D: Riemann inflow side (u = 1 enters) against a no-slip wall
    ("drop1d", (13,), [("riemann", "no_slip")], {(0, 0): [1.0]}),
    # 1D: pressure below the state's at the Riemann side (outflow expansion)
    ("drop1d", (9,), [("no_slip", "riemann")], {(0, 1): [0.8]}),
    # 2D periodic droplet boxed by no-slip walls (every face of the corner elements a wall)
    ("drop2d", (5, 4), [("no_slip", "no_slip"), ("no_slip", "no_slip")], None),
]


@pytest.mark.parametrize("name,ne,bc,bcs", WALL_KINDS)
def test_rhs_parity_wall_kinds(name, ne, bc, bcs):
    """The no-slip and Riemann-invariant ghosts in 1D (the loop form of the
    face pass), on x-, y- and z-sides of hexahedra (x and y faces in the
    remapped pass, z faces in the loop) and on every side of a 2D box."""
    cfg, om, prm, U0, mesh, P = gpu_case(name, ne, bc=bc, bc_state=bcs)
    Ro = oracle.rhs(U0, om, prm)
    Rg = _dg().rhs(mesh, P, U0.cuda().contiguous()).cpu()
    errs = res_errors(Rg, Ro, U0, oracle.max_rate(U0, om, prm), prm, om.d)
    print(name, ne, bc, ["%.1e" % e for e in errs])
    assert max(errs) <= TOL, errs


@pytest.mark.parametrize("name,ne,steps", [("drop1d", None, 100), ("drop2d", (8, 8), 30),
                                           ("rt3d", (4, 4, 4), 10), ("adjoint2d", (8, 8), 20),
                                           ("bubble2d", (4, 8), 20)])
def test_rhs_parity_evolved_state(name, ne, steps):
    """Parity on a state the oracle has advanced (not an initial condition)."""
    cfg, om, prm, U0, mesh, P = gpu_case(name, ne, "noisy_u" if name == "drop1d" else None)
    dt = oracle.max_dt(U0, om, prm)
    U = U0
    for _ in range(steps):
        U = oracle.rk_step(U, dt, om, prm)
    Ro = oracle.rhs(U, om, prm)
    Rg = _dg().rhs(mesh, P, U.cuda().contiguous()).cpu()
    errs = res_errors(Rg, Ro, U, oracle.max_rate(U, om, prm), prm, om.d)
    assert max(errs) <= TOL, errs


@pytest.mark.parametrize("name,ne", [("drop1d", (37,)), ("drop2d", (7, 5)), ("shock2d", (13, 7)),
                                     ("adjoint2d", (6, 5)), ("rt3d", (3, 4, 5)), ("bubble2d", (5, 9)),
                                     # hexahedra in more than one 16 x 16 traversal
                                     # tile per layer, the last cut short in x and y
                                     ("rt3d", (19, 17, 2))])
def test_rk_step_and_dt_parity(name, ne):
    cfg, om, prm, U0, mesh, P = gpu_case(name, ne)
    dg = _dg()
    Ud = U0.cuda().contiguous()
    dt = dg.max_dt(mesh, P, Ud, cfl=0.1)
    dto = oracle.max_dt(U0, om, prm, cfl=0.1)
    assert abs(float(dt.cpu()) - dto) <= TOL * dto
    dg.rk_step(mesh, P, Ud, dt)
    U1 = oracle.rk_step(U0, float(dt.cpu()), om, prm)
    errs = state_errors(Ud.cpu(), U1, prm, om.d)
    assert max(errs) <= TOL, errs


@pytest.mark.parametrize("name,ne", [("drop2d", (9, 6)), ("rt3d", (3, 3, 4)), ("shock2d", (10, 5))])
def test_monitors_parity(name, ne):
    cfg, om, prm, U0, mesh, P = gpu_case(name, ne)
    d = cfg["dim"]
    u_ref = [1.0, 0.5, 0.0][:d]
    mg = _dg().monitors(mesh, P, U0.cuda().contiguous(), p_ref=1.0, u_ref=u_ref)
    mo = oracle.monitors(U0, om, prm, p_ref=1.0, u_ref=u_ref)
    for f in range(om.nf):
        a, b = mg["integral"][f], float(mo["integral"][f])
        scale = float((U0[f].abs() * om.node_weights()).sum()) + 1e-300
        assert abs(a - b) <= TOL * scale, (f, a, b)
    assert mg["min_alpha"] == mo["min_alpha"] and mg["max_alpha"] == mo["max_alpha"]
    assert mg["nonphys"] == mo["nonphys"]
    assert abs(mg["max_rate"] - mo["max_rate"]) <= TOL * mo["max_rate"]
    assert abs(mg["dev_p"] - mo["dev_p"]) <= 1e-12 * max(1.0, mo["dev_p"])
    assert abs(mg["dev_u"] - mo["dev_u"]) <= 1e-12 * max(1.0, mo["dev_u"])


def test_monitors_count_nonphysical_nodes():
    """Injected bad nodes (NaN, negative density, P + Pinf < 0) are counted."""
    cfg, om, prm, U0, mesh, P = gpu_case("drop2d", (4, 4))
    U = U0.clone()
    U[0, 3, 5] = float("nan")
    U[0, 7, 1] = -5.0
    U[1, 7, 1] = 0.0
    U[4, 9, 9] = -50.0            # energy far below the stiffened-gas floor
    mg = _dg().monitors(mesh, P, U.cuda().contiguous())
    mo = oracle.monitors(U, om, prm)
    assert mg["nonphys"] == mo["nonphys"] == 3


@pytest.mark.parametrize("name,ne", [("drop1d", (23,)), ("drop2d", (5, 6)), ("rt3d", (2, 3, 2))])
def test_prim_to_cons_parity(name, ne):
    cfg = workloads.config(name, n_elem=ne)
    dg = _dg()
    P = dg.make_params(cfg["params"])
    mesh = dg.mesh_from_config(cfg, P)
    om = oracle.OracleMesh(cfg["dim"], 3, ne, cfg["lo"], cfg["hi"], cfg["bc"])
    X = om.node_coords().numpy()
    pf = workloads.primitive_fields(cfg, X)
    prm = oracle.Params(**cfg["params"])
    from helpers import cons_from_prim
    Uo = cons_from_prim(pf, prm)
    Ug = dg.prim_to_cons(mesh, P, dg.prim_tensor(pf, cfg["dim"])).cpu()
    assert max(state_errors(Ug, Uo, prm, cfg["dim"])) <= 1e-15


def test_determinism_bitwise():
    cfg, om, prm, U0, mesh, P = gpu_case("rt3d", (4, 3, 4))
    dg = _dg()
    Ud = U0.cuda().contiguous()
    R1 = dg.rhs(mesh, P, Ud).clone()
    R2 = dg.rhs(mesh, P, Ud).clone()
    assert torch.equal(R1, R2)
    A, B = Ud.clone(), Ud.clone()
    dt = dg.max_dt(mesh, P, Ud)
    dg.rk_step(mesh, P, A, dt)
    dg.rk_step(mesh, P, B, dt)
    assert torch.equal(A, B)


def test_water_air_interface_equilibrium():
    """The paper's water droplet in air (density ratio 1000, stiffened water
    with P_inf = 6000, u = (5, 5)): 400 FP64 steps keep P and u uniform to the
    round-off floor of P = (rho e - Pi)/xi (Pi ~ 8e3), the state physical, and
    match the oracle after 20 steps."""
    cfg, om, prm, U0, mesh, P = gpu_case("waterair2d", (12, 12))
    dg = _dg()
    U = U0.cuda().contiguous()
    dt = dg.max_dt(mesh, P, U)
    Uo = U0
    for _ in range(20):
        Uo = oracle.rk_step(Uo, float(dt.cpu()), om, prm)
    dg.advance(mesh, P, U, 20, dt_fixed=dt)
    assert max(state_errors(U.cpu(), Uo, prm, om.d)) <= 1e-11
    dg.advance(mesh, P, U, 380, dt_fixed=dt)
    m = dg.monitors(mesh, P, U, p_ref=1.0, u_ref=[5.0, 5.0])
    print("water-air after 400 steps", m["dev_p"], m["dev_u"], m["min_alpha"], m["max_alpha"])
    assert m["nonphys"] == 0
    assert m["dev_p"] < 1e-7 and m["dev_u"] < 1e-7
    # boundedness of the phase field (Introduction and Conclusions: it holds
    # for suitable Gamma and eps, which this case has: eps = h/2, Gamma = |u|)
    assert -1e-8 <= m["min_alpha"] and m["max_alpha"] <= 1.0 + 1e-8


def test_interface_equilibrium_on_gpu():
    """50 GPU SSP-RK3 steps of the droplet keep P and u uniform to round-off
    and conserve both phase masses, momentum and energy."""
    cfg, om, prm, U0, mesh, P = gpu_case("drop2d", (16, 16))
    dg = _dg()
    U = U0.cuda().contiguous()
    m0 = dg.monitors(mesh, P, U, p_ref=1.0, u_ref=[1.0, 0.5])
    for _ in range(50):
        dt = dg.max_dt(mesh, P, U)
        dg.rk_step(mesh, P, U, dt)
    m1 = dg.monitors(mesh, P, U, p_ref=1.0, u_ref=[1.0, 0.5])
    assert m1["dev_p"] < 1e-12 and m1["dev_u"] < 1e-12, m1
    assert m1["nonphys"] == 0
    for f in range(5):
        assert abs(m1["integral"][f] - m0["integral"][f]) <= 1e-13 * abs(m0["integral"][f]) + 1e-15


@pytest.mark.parametrize("name,ne,steps", [("drop2d", (9, 7), 4), ("rt3d", (3, 3, 4), 3),
                                           ("shock2d", (10, 6), 3), ("drop1d", (21,), 5),
                                           ("bubble2d", (5, 9), 4)])
def test_advance_matches_rk_steps(name, ne, steps):
    """dg2p_advance (device dt, carried face ingredients, fused records) gives
    the same states as dg2p_max_dt + dg2p_rk_step repeated, bit for bit, and
    matches the oracle; its monitors match dg2p_compute_monitors."""
    cfg, om, prm, U0, mesh, P = gpu_case(name, ne)
    dg = _dg()
    A = U0.cuda().contiguous()
    B = A.clone()
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    mon = torch.zeros(dg.MONITOR_DOUBLES, dtype=torch.float64, device="cuda")
    dg.advance(mesh, P, A, steps, cfl=0.1, t=t, mon=mon, p_ref=1.0)
    tsum = 0.0
    Uo = U0
    for _ in range(steps):
        dt = dg.max_dt(mesh, P, B, cfl=0.1)
        dg.rk_step(mesh, P, B, dt)
        tsum += float(dt.cpu())
        Uo = oracle.rk_step(Uo, float(dt.cpu()), om, prm)
    assert torch.equal(A, B)
    assert abs(float(t.cpu()) - tsum) <= 1e-15 * tsum
    errs = state_errors(A.cpu(), Uo, prm, om.d)
    assert max(errs) <= 1e-11, errs
    m1 = dg.decode_monitors(mon, mesh.nf)
    m2 = dg.monitors(mesh, P, A, p_ref=1.0)
    for k in ("min_alpha", "max_alpha", "nonphys"):
        assert m1[k] == m2[k], k
    assert abs(m1["max_rate"] - m2["max_rate"]) <= 1e-15 * m2["max_rate"]
    for f in range(mesh.nf):
        assert abs(m1["integral"][f] - m2["integral"][f]) <= 1e-13 * (abs(m2["integral"][f]) + 1e-300)


def _advance_vs_rk_steps(name, ne, steps=3):
    cfg, om, prm, U0, mesh, P = gpu_case(name, ne)
    dg = _dg()
    A = U0.cuda().contiguous()
    B = A.clone()
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    last = torch.zeros(1, dtype=torch.float64, device="cuda")
    dg.advance(mesh, P, A, steps, cfl=0.1, t=t, dt_last=last)
    tsum = 0.0
    for _ in range(steps):
        dt = dg.max_dt(mesh, P, B, cfl=0.1)
        dg.rk_step(mesh, P, B, dt)
        tsum += float(dt.cpu())
    assert torch.equal(A, B)
    assert float(t.cpu()) == tsum or abs(float(t.cpu()) - tsum) <= 1e-15 * tsum
    assert float(last.cpu()) == float(dt.cpu())


@pytest.mark.parametrize("name,ne", [("drop2d", (136, 136)), ("rt3d", (20, 20, 12))])
def test_advance_two_level_dt(name, ne):
    """Grids with more than 1024 rate records reduce each step's dt in two
    small kernels instead of inside the first stage: still the same states,
    bit for bit, as dg2p_max_dt + dg2p_rk_step, and the same elapsed time."""
    _advance_vs_rk_steps(name, ne)


@pytest.mark.parametrize("ne", [(128, 128), (125, 128)])
def test_advance_fused_dt_at_record_limit(ne):
    """The first stage's own reduction at its limit: 1024 rate records (four
    per thread, all taken) and 1000 (the last four-record share partly
    empty) give the same states and dt, bit for bit, as dg2p_max_dt +
    dg2p_rk_step."""
    _advance_vs_rk_steps("drop2d", ne)


def test_advance_fixed_dt():
    cfg, om, prm, U0, mesh, P = gpu_case("adjoint2d", (6, 6))
    dg = _dg()
    A = U0.cuda().contiguous()
    dt = torch.tensor([1e-4], dtype=torch.float64, device="cuda")
    dg.advance(mesh, P, A, 3, dt_fixed=dt)
    Uo = U0
    for _ in range(3):
        Uo = oracle.rk_step(Uo, 1e-4, om, prm)
    assert max(state_errors(A.cpu(), Uo, prm, om.d)) <= 1e-12


@pytest.mark.parametrize("name,ne", [("drop2d", (6, 5)), ("rt3d", (3, 2, 4))])
def test_advance_zero_steps(name, ne):
    """n_steps = 0 is the degenerate run: the state and the time stay as
    they were, a monitored call writes no step row, and the final monitors
    are those of the unchanged state (equal to the stand-alone monitors)."""
    cfg, om, prm, U0, mesh, P = gpu_case(name, ne)
    dg = _dg()
    A = U0.cuda().contiguous()
    t = torch.full((1,), 0.25, dtype=torch.float64, device="cuda")
    mon = torch.zeros(dg.MONITOR_DOUBLES, dtype=torch.float64, device="cuda")
    dg.advance(mesh, P, A, 0, cfl=0.1, t=t, mon=mon)
    assert torch.equal(A.cpu(), U0) and float(t.cpu()) == 0.25
    got = dg.decode_monitors(mon.view(1, -1), mesh.nf)[0]
    ref = dg.monitors(mesh, P, A)
    assert got["min_alpha"] == ref["min_alpha"] and got["max_alpha"] == ref["max_alpha"]
    assert got["integral"] == ref["integral"] and got["max_rate"] == ref["max_rate"]
    rows = torch.full((2, dg.MONITOR_DOUBLES), -7.0, dtype=torch.float64, device="cuda")
    dg.advance_monitored(mesh, P, A, 0, rows, cfl=0.1, t=t)
    assert torch.equal(A.cpu(), U0) and float(t.cpu()) == 0.25
    assert bool((rows == -7.0).all())


@pytest.mark.parametrize("ne", [(128, 128), (136, 136)])
def test_full_grid_step_against_the_oracle(ne):
    """One step of dg2p_advance on the full 128 x 128 droplet (1024 rate
    records: dt reduced inside the first stage) and on 136 x 136 (1156
    records: two-level reduction), and one dg2p_rk_step with dg2p_max_dt,
    against the oracle's step from the same state: dt to 1e-14, every field
    to 1e-12."""
    cfg, om, prm, U0, mesh, P = gpu_case("drop2d", ne)
    dg = _dg()
    dto = oracle.max_dt(U0, om, prm)
    Uo = oracle.rk_step(U0, dto, om, prm)
    A = U0.cuda().contiguous()
    last = torch.zeros(1, dtype=torch.float64, device="cuda")
    dg.advance(mesh, P, A, 1, cfl=0.1, dt_last=last)
    assert abs(float(last.cpu()) - dto) <= 1e-14 * dto
    errs = state_errors(A.cpu(), Uo, prm, om.d)
    assert max(errs) <= 1e-12, errs
    B = U0.cuda().contiguous()
    dtg = dg.max_dt(mesh, P, B, cfl=0.1)
    dg.rk_step(mesh, P, B, dtg)
    errs = state_errors(B.cpu(), Uo, prm, om.d)
    assert max(errs) <= 1e-12, errs


# ---- mixed precision: error vs the FP64 oracle, stated per field -------------------
# The per-node a-priori rounding bound of the contractions is tested where it
# applies exactly (tests/test_gpu_mixed.py).  On the full workloads the
# interface flux, the normal and the curvature are themselves contracted
# fields, so errors compound; the bars below are the largest measured normwise
# field errors of one residual (FP32 1.3e-7, BF16 1.3e-2) with a margin of 8x.
MIXED = [("drop2d", (9, 7)), ("shock2d", (12, 6)), ("adjoint2d", (8, 7)), ("rt3d", (3, 4, 3)),
         ("drop1d", (19,))]


@pytest.mark.parametrize("prec,bar", [("fp32", 1e-6), ("bf16", 0.1)])
@pytest.mark.parametrize("name,ne", MIXED)
def test_mixed_precision_rhs_error(name, ne, prec, bar):
    cfg, om, prm, U0, mesh, P = gpu_case(name, ne)
    dg = _dg()
    Pm = dg.make_params(cfg["params"], precision=prec)
    Ro = oracle.rhs(U0, om, prm)
    Rm = dg.rhs(mesh, Pm, U0.cuda().contiguous()).cpu()
    errs = res_errors(Rm, Ro, U0, oracle.max_rate(U0, om, prm), prm, om.d)
    print(name, prec, ["%.2e" % e for e in errs])
    assert max(errs) <= bar, errs
    if prec == "fp32":
        assert max(errs) > 0.0   # it really is a different (lower) precision path


def test_mixed_precision_interface_equilibrium():
    """Uniform P and u contract to exactly zero in the fluctuation form; the
    remaining drift comes from FP32 rounding of the varying fluxes."""
    cfg, om, prm, U0, mesh, P = gpu_case("drop2d", (16, 16))
    dg = _dg()
    Pm = dg.make_params(cfg["params"], precision="fp32")
    U = U0.cuda().contiguous()
    dg.advance(mesh, Pm, U, 50)
    m = dg.monitors(mesh, Pm, U, p_ref=1.0, u_ref=[1.0, 0.5])
    print("fp32 IEC after 50 steps", m["dev_p"], m["dev_u"])
    assert m["dev_p"] < 1e-5 and m["dev_u"] < 1e-5 and m["nonphys"] == 0


# ---- hand-written adjoint vs the oracle's autograd adjoint ---------------------------
PERIODIC3 = [("periodic", "periodic")] * 3
# (name, elements, boundary override, parameter overrides, tolerance).  The CSF
# delta function |grad alpha| is differentiated through grad alpha / |grad alpha|;
# where alpha is within ~1e-11 of 0 or 1, grad alpha comes out of a
# cancellation (relative rounding ~1e-7 on each side), so with the thin
# interface of the workloads the surface-tension part of the alpha cotangent
# is conditioned at ~1e-9: those cases carry 1e-8.  The same physics with a
# thick interface (eps = 0.05, no cancellation) must agree to round-off.
VJP_CASES = [("drop1d", (13,), None, {}, 1e-11), ("drop2d", (6, 5), None, {}, 1e-11),
             ("adjoint2d", (6, 5), None, {"eps": 0.05}, 1e-11),
             ("adjoint2d", (5, 3), None, {"eps": 0.05}, 1e-11),
             ("adjoint2d", (6, 5), None, {}, 1e-8),
             ("rt3d", (3, 2, 4), PERIODIC3, {"eps": 0.05}, 1e-11),
             ("rt3d", (3, 2, 4), PERIODIC3, {}, 1e-8),
             # boundary ghosts reversed into the boundary elements: slip walls
             # in z (rt3d's own), no-slip / Riemann / slip (rising bubble,
             # RT), Dirichlet inflow and extrapolation (shock), no-slip and
             # slip walls all round (viscous + CSF)
             ("rt3d", (3, 2, 4), None, {"eps": 0.05}, 1e-11),
             ("bubble2d", (4, 6), None, {"eps": 0.08}, 1e-11),
             ("rt2d", (3, 8), None, {"eps": 0.1}, 1e-11),
             ("shock2d", (6, 3), None, {}, 1e-11),
             ("adjoint2d", (5, 4), [("no_slip", "no_slip"), ("no_slip", "no_slip")], {"eps": 0.05}, 1e-11),
             ("adjoint2d", (5, 4), [("slip_wall", "slip_wall"), ("slip_wall", "slip_wall")], {"eps": 0.05}, 1e-11)]


def vjp_errors(Ug, Uo):
    """Per-field max error relative to that field's own largest cotangent
    (every field of these cases carries at least 2 % of the largest one; the
    1e-12 floor only guards an identically zero field)."""
    top = float(Uo.abs().max())
    return [float((Ug[f] - Uo[f]).abs().max()) / max(float(Uo[f].abs().max()), 1e-12 * top)
            for f in range(Uo.shape[0])]


@pytest.mark.parametrize("name,ne,bc,over,tol", VJP_CASES)
def test_rhs_vjp_parity(name, ne, bc, over, tol):
    cfg, om, prm, U0, mesh, P = gpu_case(name, ne, bc=bc, **over)
    dg = _dg()
    w = torch.randn(U0.shape, generator=torch.Generator().manual_seed(11), dtype=torch.float64)
    Ubo, sbo = oracle.adjoint.rhs_vjp(U0, w, om, prm)
    pbar = torch.zeros(1, dtype=torch.float64, device="cuda")
    Ubg = dg.rhs_vjp(mesh, P, U0.cuda().contiguous(), w.cuda().contiguous(), param_bar=pbar).cpu()
    errs = vjp_errors(Ubg, Ubo)
    print(name, ne, over, ["%.1e" % x for x in errs], float(pbar.cpu()), sbo)
    assert max(errs) <= tol, errs
    # R is affine in sigma: dR/dsigma = R(sigma=1) - R(sigma=0) exactly; the sigma
    # cotangent is compared against the absolute size of its terms (in 1D the
    # curvature of a +-1 normal is round-off, so sigma_bar itself is noise there)
    import dataclasses
    dR = oracle.rhs(U0, om, dataclasses.replace(prm, sigma=1.0)) - oracle.rhs(U0, om, dataclasses.replace(prm, sigma=0.0))
    scale = float((w.abs() * dR.abs()).sum())
    if om.d >= 2:
        assert abs(float(pbar.cpu()) - sbo) <= 1e-12 * scale


@pytest.mark.parametrize("name,ne,bc,over,tol", [("adjoint2d", (5, 4), None, {"eps": 0.05}, 1e-11),
                                                 ("adjoint2d", (5, 4), None, {}, 1e-8),
                                                 ("rt3d", (2, 2, 3), PERIODIC3, {"eps": 0.05}, 1e-11),
                                                 ("drop1d", (11,), None, {}, 1e-11),
                                                 ("bubble2d", (4, 6), None, {"eps": 0.08}, 1e-11),
                                                 ("shock2d", (5, 3), None, {}, 1e-11),
                                                 ("rt3d", (2, 2, 3), None, {"eps": 0.05}, 1e-11)])
def test_rk_step_vjp_parity(name, ne, bc, over, tol):
    """The VJP of a step reverses the residual at the two intermediate stage
    states, which each side computes itself (they agree to rounding).  The
    residual is not differentiable where two wave speeds of a face tie
    (d max = 1/2, 1/2 there): a uniform region (the shock's pre-shock state,
    a hydrostatic column) ties exactly on one side and by a rounding on the
    other, so the state is perturbed by 1e-6 (relative, seeded) to move every
    face off the ties."""
    cfg, om, prm, U0, mesh, P = gpu_case(name, ne, bc=bc, **over)
    dg = _dg()
    U0 = U0 * (1.0 + 1e-6 * torch.randn(U0.shape, generator=torch.Generator().manual_seed(7), dtype=torch.float64))
    dt = oracle.max_dt(U0, om, prm)
    w = torch.randn(U0.shape, generator=torch.Generator().manual_seed(12), dtype=torch.float64)
    Ubo, sbo = oracle.adjoint.rk_step_vjp(U0, dt, w, om, prm)
    pbar = torch.zeros(1, dtype=torch.float64, device="cuda")
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
    Ubg = dg.rk_step_vjp(mesh, P, U0.cuda().contiguous(), dtd, w.cuda().contiguous(), param_bar=pbar).cpu()
    errs = vjp_errors(Ubg, Ubo)
    print(name, over, ["%.1e" % x for x in errs], float(pbar.cpu()), sbo)
    assert max(errs) <= tol, errs
    if om.d >= 2:   # in 1D the curvature is round-off (see the residual test)
        assert abs(float(pbar.cpu()) - sbo) <= 1e-10 * abs(sbo)


def test_rhs_vjp_dot_product_gpu():
    """<J v, w> from central differences of the GPU residual equals <v, J^T w>
    (resolved interface, so the residual is smooth at the difference step)."""
    cfg, om, prm, U0, mesh, P = gpu_case("adjoint2d", (8, 8), eps=0.05)
    dg = _dg()
    g = torch.Generator().manual_seed(3)
    scale = U0.abs().amax(dim=(1, 2), keepdim=True)
    v = (torch.randn(U0.shape, generator=g, dtype=torch.float64) * scale * 1e-3).cuda()
    w = torch.randn(U0.shape, generator=g, dtype=torch.float64).cuda()
    U = U0.cuda().contiguous()
    h = 1e-6
    Jv = (dg.rhs(mesh, P, (U + h * v).contiguous()) - dg.rhs(mesh, P, (U - h * v).contiguous())) / (2 * h)
    Ub = dg.rhs_vjp(mesh, P, U, w.contiguous())
    lhs, rhs_ = float((Jv * w).sum()), float((v * Ub).sum())
    assert abs(lhs - rhs_) <= 1e-6 * max(abs(lhs), abs(rhs_))


def test_vjp_rejects_unsupported():
    """The adjoint is FP64 only (and p = 3, tested with the p = 4 kernels)."""
    cfg, om, prm, U0, mesh, P = gpu_case("shock2d", (4, 3))
    dg = _dg()
    U = U0.cuda().contiguous()
    with pytest.raises(dg.Dg2pError) as ei:
        dg.rhs_vjp(mesh, dg.make_params(cfg["params"], precision="fp32"), U, U.clone())
    assert ei.value.status == dg.EUNSUPPORTED


FULL = ["drop2d", "shock2d", "adjoint2d", "rt3d", "bubble2d", "rt2d", "waterair2d"]


def _sample_elements(cfg, n=48, seed=0):
    """Sampled element indices: corners and boundary layers plus random ones."""
    N = cfg["n_elem"]
    E = int(np.prod(N))
    rng = np.random.default_rng(seed)
    picks = set(rng.integers(0, E, n).tolist())
    d = len(N)
    for corner in range(2 ** d):
        c = [(N[k] - 1) if (corner >> k) & 1 else 0 for k in range(d)]
        e = 0
        stride = 1
        for k in range(d):
            e += c[k] * stride
            stride *= N[k]
        picks.add(e)
    return torch.tensor(sorted(picks), dtype=torch.long)


@pytest.mark.parametrize("name", FULL)
def test_full_size_sampled_parity(name):
    """Full-size grid, the launch shapes the benchmark times: GPU residual on
    every element, oracle on sampled elements (one by one)."""
    cfg, om, prm, U0, mesh, P = gpu_case(name)
    dg = _dg()
    Ud = U0.cuda().contiguous()
    Rg = dg.rhs(mesh, P, Ud)
    el = _sample_elements(cfg)
    Ro = oracle.rhs(U0, om, prm, elems=el)
    Rs = Rg[:, el.cuda()].cpu()
    rate = oracle.max_rate(U0, om, prm)
    errs = res_errors(Rs, Ro, U0, rate, prm, om.d)
    print(name, ["%.1e" % e for e in errs])
    assert max(errs) <= TOL, errs
    dt = dg.max_dt(mesh, P, Ud)
    assert abs(float(dt.cpu()) - 0.1 / rate) <= TOL * 0.1 / rate
    del Rg, Ud
    torch.cuda.empty_cache()


def test_rising_bubble_rises():
    """The paper's rising bubble (no-slip bottom, Riemann-invariant top, slip
    sides; 20 x 40, p = 3) over t = 0.5: no non-physical state, the bubble's
    centre of gravity moves up and its mean vertical velocity is positive
    (a qualitative check: the paper's reference curves are not reproduced)."""
    cfg = workloads.config("bubble2d")
    dg = _dg()
    P = dg.make_params(cfg["params"])
    mesh = dg.mesh_from_config(cfg, P)
    X = mesh.node_coords()
    U = dg.prim_to_cons(mesh, P, dg.prim_tensor(workloads.primitive_fields(cfg, X), 2))
    W = torch.tensor(mesh.node_weights(), device="cuda")     # tensor-product GLL weights per node
    y = torch.tensor(X[1], device="cuda")

    def centre(U):
        b = (1.0 - U[5]) * W          # bubble (phase 2) volume fraction, quadrature weights
        rho = U[0] + U[1]
        return float((b * y).sum() / b.sum()), float((b * U[3] / rho).sum() / b.sum())

    y0, v0 = centre(U)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    mon = torch.zeros(dg.MONITOR_DOUBLES, dtype=torch.float64, device="cuda")
    while float(t.cpu()) < 0.5:
        dg.advance(mesh, P, U, 200, cfl=0.1, t=t, mon=mon)
        m = dg.decode_monitors(mon, mesh.nf)
        assert m["nonphys"] == 0
        assert -1e-8 <= m["min_alpha"] and m["max_alpha"] <= 1.0 + 1e-8     # bounded phase field
    y1, v1 = centre(U)
    print("t", float(t.cpu()), "y_c", y0, "->", y1, "v_c", v0, "->", v1)
    assert y1 > y0 + 0.02 and v1 > 0.05


def test_checkpoint_resume_is_bitwise(tmp_path):
    """40 steps of dg2p_advance against 20 steps, a checkpoint written and read
    back, and 20 more: the same state and time, bit for bit."""
    from paper_2306_05002_amd import checkpoint
    cfg, om, prm, U0, mesh, P = gpu_case("rt3d", (3, 3, 4))
    dg = _dg()
    A = U0.cuda().contiguous()
    ta = torch.zeros(1, dtype=torch.float64, device="cuda")
    dg.advance(mesh, P, A, 40, cfl=0.1, t=ta)
    B = U0.cuda().contiguous()
    tb = torch.zeros(1, dtype=torch.float64, device="cuda")
    dg.advance(mesh, P, B, 20, cfl=0.1, t=tb)
    path = tmp_path / "run.npz"
    checkpoint.save(path, B, tb, 20, cfg["params"], {"n_elem": list(cfg["n_elem"]), "bc": cfg["bc"]})
    del B, tb
    ck = checkpoint.load(path)
    assert ck["step"] == 20 and ck["params"] == json_round(cfg["params"])
    P2 = dg.make_params(ck["params"])
    dg.advance(mesh, P2, ck["U"], 20, cfl=0.1, t=ck["t"])
    assert torch.equal(ck["U"], A)
    assert torch.equal(ck["t"], ta)


def json_round(d):
    import json
    return json.loads(json.dumps(d, sort_keys=True))


def test_require_physical_raises_on_injected_nodes():
    """The sync helper turns counted non-physical nodes into DG2P_ENONPHYS."""
    cfg, om, prm, U0, mesh, P = gpu_case("drop2d", (4, 4))
    dg = _dg()
    good = dg.monitors(mesh, P, U0.cuda().contiguous())
    assert dg.require_physical(good) is good
    U = U0.clone()
    U[0, 2, 3] = float("inf")
    with pytest.raises(dg.Dg2pError) as ei:
        dg.require_physical(dg.monitors(mesh, P, U.cuda().contiguous()))
    assert ei.value.status == dg.ENONPHYS


def test_residual_beyond_32bit_offsets():
    """A 2D droplet grid of 4400 x 4400 quads (7 x 19.36 M x 16 = 2.17e9 state
    entries, past 2^31): the library's residual on every element against the
    oracle on sampled elements.  The state is built on the GPU (the droplet
    fields of the benchmark workload with this grid's interface width); the
    oracle's copy holds only the sampled elements and their neighbours."""
    dg = _dg()
    N = 4400
    cfg = workloads.config("drop2d", n_elem=(N, N))
    prm = oracle.Params(**cfg["params"])
    P = dg.make_params(cfg["params"])
    mesh = dg.mesh_from_config(cfg, P)
    E, nn, nf = mesh.E, mesh.nn, mesh.nf
    assert nf * E * nn > 2 ** 31
    ref = torch.tensor(dg.Mesh(2, (1, 1), (0, 0), (1, 1)).node_coords()[:, 0, :], device="cuda")  # nodes on [0,1]^2
    h = 1.0 / N
    e = torch.arange(E, device="cuda")
    x = ((e % N).to(torch.float64)[:, None] + ref[0][None, :]) * h
    y = ((e // N).to(torch.float64)[:, None] + ref[1][None, :]) * h
    psi = torch.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2) - 0.15
    del x, y, e
    alpha = torch.sigmoid(psi / cfg["params"]["eps"])
    one = torch.ones_like(psi)
    prim = torch.stack([alpha, psi, prm.rho0[0] * one, prm.rho0[1] * one, one, 0.5 * one, one])
    del alpha, psi, one
    U = dg.prim_to_cons(mesh, P, prim)
    del prim
    torch.cuda.empty_cache()
    R = dg.rhs(mesh, P, U)
    dt = float(dg.max_dt(mesh, P, U).cpu())
    om = oracle.OracleMesh(2, 3, (N, N), cfg["lo"], cfg["hi"], cfg["bc"])
    el = _sample_elements(cfg, n=32, seed=1)
    # plus two elements on the droplet rim (r = 0.15 around (0.5, 0.5))
    el = torch.cat([el, torch.tensor([2200 * N + 2860, 2860 * N + 2200], dtype=torch.long)])
    need = [el]
    for k in range(2):
        for side in (0, 1):
            need.append(om.neighbour(el, k, side)[0])
    need = torch.unique(torch.cat(need))
    Uc = torch.empty((nf, E, nn), dtype=torch.float64)        # pages touched only where filled
    Uc[:, need] = U[:, need.cuda()].cpu()
    Ro = oracle.rhs(Uc, om, prm, elems=el)
    Rs = R[:, el.cuda()].cpu()
    rate = 0.1 / dt
    errs = res_errors(Rs, Ro, Uc[:, el], rate, prm, 2)
    print("4400^2", ["%.1e" % v for v in errs])
    assert max(errs) <= TOL, errs
    del U, R
    torch.cuda.empty_cache()
