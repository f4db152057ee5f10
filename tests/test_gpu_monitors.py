"""Per-step monitors on the stepping path (dg2p_advance_monitored) and NaN
propagation of the time-step and monitor reductions, against the library's
stand-alone monitor pass and the FP64 oracle."""

import math

import pytest
import torch

import oracle
from helpers import oracle_setup

pytestmark = pytest.mark.gpu


def _dg():
    from paper_2306_05002_amd import dg2p
    return dg2p


def _case(name, ne):
    cfg, om, prm, U0 = oracle_setup(name, n_elem=ne)
    dg = _dg()
    P = dg.make_params(cfg["params"])
    mesh = dg.mesh_from_config(cfg, P)
    return cfg, om, prm, U0, mesh, P


# Grids of fewer than 13 workgroups reduce each step's records in separate
# kernels, larger ones (up to 1024 workgroups) in the next step's first stage:
# drop2d 12x10 (8 workgroups of 16 quads), 16x13 (13, the smallest fused),
# 16x16 (16), 128x128 (1024); shock2d 16x8 (8); rt3d 3x4x3 (36 one-hexahedron
# workgroups, fused); drop1d 37 (1).
@pytest.mark.parametrize("name,ne", [("drop2d", (12, 10)), ("drop2d", (16, 13)), ("drop2d", (16, 16)),
                                     ("drop2d", (128, 128)), ("shock2d", (16, 8)),
                                     ("rt3d", (3, 4, 3)), ("drop1d", (37,))])
def test_advance_monitored_every_step(name, ne):
    """Same states as dg2p_advance, bit for bit; row i of the per-step
    monitors equals the stand-alone monitors of the state after step i + 1
    (alpha range and non-physical count exactly; deviations, rate and dt to
    rounding; integrals up to the summation order) and the oracle's monitors
    of its own run with the same dt (1e-12)."""
    cfg, om, prm, U0, mesh, P = _case(name, ne)
    dg = _dg()
    d = cfg["dim"]
    steps = 4
    u_ref = [float(v) for v in oracle.primitives(U0[:, :1, :1], d, prm)["u"].flatten()]
    A = U0.cuda().contiguous()
    B = A.clone()
    ms = torch.zeros(steps, dg.MONITOR_DOUBLES, dtype=torch.float64, device="cuda")
    tA = torch.zeros(1, dtype=torch.float64, device="cuda")
    tB = torch.zeros(1, dtype=torch.float64, device="cuda")
    dg.advance_monitored(mesh, P, A, steps, ms, cfl=0.1, t=tA, p_ref=1.0, u_ref=u_ref)
    dg.advance(mesh, P, B, steps, cfl=0.1, t=tB)
    assert torch.equal(A, B)
    assert torch.equal(tA, tB)
    rows = dg.decode_monitors(ms, mesh.nf)
    C = U0.cuda().contiguous()
    Uo = U0
    for i in range(steps):
        dt = dg.max_dt(mesh, P, C, cfl=0.1)
        dg.rk_step(mesh, P, C, dt)
        Uo = oracle.rk_step(Uo, float(dt.cpu()), om, prm)
        ref = dg.monitors(mesh, P, C, p_ref=1.0, u_ref=u_ref)
        got = rows[i]
        for k in ("min_alpha", "max_alpha", "nonphys"):
            assert got[k] == ref[k], (i, k, got[k], ref[k])
        # derived from the closure, whose multiply-adds the compiler may
        # contract differently in the two kernels: equal to rounding
        assert abs(got["dev_p"] - ref["dev_p"]) <= 1e-13 * max(1.0, ref["dev_p"])
        assert abs(got["dev_u"] - ref["dev_u"]) <= 1e-13 * max(1.0, ref["dev_u"])
        assert abs(got["max_rate"] - ref["max_rate"]) <= 1e-14 * ref["max_rate"]
        dtr = float(dg.max_dt(mesh, P, C, cfl=0.1).cpu())
        assert abs(got["dt"] - dtr) <= 1e-14 * dtr
        for f in range(mesh.nf):
            scale = float(torch.abs(C[f]).max()) * sum(mesh.node_weights()) * mesh.E + 1e-300
            assert abs(got["integral"][f] - ref["integral"][f]) <= 1e-14 * scale, (i, f)
        mo = oracle.monitors(Uo, om, prm, p_ref=1.0, u_ref=u_ref)
        assert abs(got["min_alpha"] - mo["min_alpha"]) <= 1e-12
        assert abs(got["max_alpha"] - mo["max_alpha"]) <= 1e-12
        assert got["nonphys"] == mo["nonphys"] == 0
        assert abs(got["max_rate"] - mo["max_rate"]) <= 1e-12 * mo["max_rate"]
        for f in range(mesh.nf):
            scale = float(torch.abs(Uo[f]).max()) * float(om.node_weights().sum()) * om.E + 1e-300
            assert abs(got["integral"][f] - float(mo["integral"][f])) <= 1e-12 * scale, (i, f)
    assert torch.equal(A, C)


@pytest.mark.parametrize("ne", [(4, 4), (16, 16)])
def test_failed_closure_makes_dt_nan_like_the_oracle(ne):
    """A node whose squared sound speed is negative (energy below the
    stiffened-gas floor) has a NaN wave speed: the reduced rate and dt are
    NaN on both sides (the reductions propagate NaN instead of skipping the
    node), and a step taken from that state reports it in its monitors
    (one workgroup: separate reduction; sixteen: fused into the stage)."""
    cfg, om, prm, U0, mesh, P = _case("drop2d", ne)
    dg = _dg()
    U = U0.clone()
    U[4, 9, 9] = -50.0
    assert math.isnan(oracle.max_rate(U, om, prm))
    Ud = U.cuda().contiguous()
    dt = dg.max_dt(mesh, P, Ud, cfl=0.1)
    assert math.isnan(float(dt.cpu()))
    m = dg.monitors(mesh, P, Ud)
    assert math.isnan(m["max_rate"]) and m["nonphys"] == 1
    ms = torch.zeros(1, dg.MONITOR_DOUBLES, dtype=torch.float64, device="cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dg.advance_monitored(mesh, P, Ud, 1, ms, cfl=0.1, t=t)
    assert math.isnan(float(t.cpu()))
    row = dg.decode_monitors(ms, mesh.nf)[0]
    assert row["nonphys"] > 0 and math.isnan(row["dt"])


@pytest.mark.parametrize("ne", [(12, 10), (16, 16)])
def test_advance_monitored_fixed_dt(ne):
    """With a prescribed dt the per-step monitors still carry the state's
    rate (equal to the stand-alone monitors') and report dt = dt_fixed; the
    states equal dg2p_advance's with the same dt bit for bit."""
    cfg, om, prm, U0, mesh, P = _case("drop2d", ne)
    dg = _dg()
    steps = 3
    dtf = torch.tensor([0.3 * float(dg.max_dt(mesh, P, U0.cuda().contiguous(), cfl=0.1).cpu())],
                       dtype=torch.float64, device="cuda")
    A = U0.cuda().contiguous()
    B = A.clone()
    ms = torch.zeros(steps, dg.MONITOR_DOUBLES, dtype=torch.float64, device="cuda")
    dg.advance_monitored(mesh, P, A, steps, ms, cfl=0.1, dt_fixed=dtf)
    dg.advance(mesh, P, B, steps, cfl=0.1, dt_fixed=dtf)
    assert torch.equal(A, B)
    rows = dg.decode_monitors(ms, mesh.nf)
    C = U0.cuda().contiguous()
    for i in range(steps):
        dg.rk_step(mesh, P, C, dtf)
        ref = dg.monitors(mesh, P, C, p_ref=1.0)
        assert rows[i]["dt"] == float(dtf.cpu())
        assert abs(rows[i]["max_rate"] - ref["max_rate"]) <= 1e-14 * ref["max_rate"]
        assert rows[i]["min_alpha"] == ref["min_alpha"] and rows[i]["max_alpha"] == ref["max_alpha"]
    assert torch.equal(A, C)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_advance_monitored_mixed_precision_fused(precision):
    """The mixed contraction forms on a grid whose monitors are reduced in
    the next first stage (16 workgroups): states equal dg2p_advance's bit for
    bit, and each row equals the stand-alone monitors of the same state
    (integrals to rounding)."""
    cfg, om, prm, U0, mesh, _ = _case("drop2d", (16, 16))
    dg = _dg()
    P = dg.make_params(cfg["params"], precision=precision)
    steps = 3
    A = U0.cuda().contiguous()
    B = A.clone()
    ms = torch.zeros(steps, dg.MONITOR_DOUBLES, dtype=torch.float64, device="cuda")
    dg.advance_monitored(mesh, P, A, steps, ms, cfl=0.1)
    dg.advance(mesh, P, B, steps, cfl=0.1)
    assert torch.equal(A, B)
    rows = dg.decode_monitors(ms, mesh.nf)
    C = U0.cuda().contiguous()
    for i in range(steps):
        dt = dg.max_dt(mesh, P, C, cfl=0.1)
        dg.rk_step(mesh, P, C, dt)
        ref = dg.monitors(mesh, P, C)
        assert rows[i]["min_alpha"] == ref["min_alpha"] and rows[i]["max_alpha"] == ref["max_alpha"]
        assert rows[i]["nonphys"] == ref["nonphys"]
        assert abs(rows[i]["max_rate"] - ref["max_rate"]) <= 1e-14 * ref["max_rate"]
        for f in range(mesh.nf):
            scale = float(torch.abs(C[f]).max()) * sum(mesh.node_weights()) * mesh.E + 1e-300
            assert abs(rows[i]["integral"][f] - ref["integral"][f]) <= 1e-14 * scale
    assert torch.equal(A, C)
