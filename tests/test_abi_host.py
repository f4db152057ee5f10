"""Host-side checks of the C-ABI library (no GPU): it loads, exports every
function include/dg2p.h declares, validates descriptors and parameters, and
its node coordinates and workspace arithmetic agree with the oracle's grid."""

import ctypes
import os
import re

import numpy as np
import pytest
import torch

import oracle
from paper_2306_05002_amd import dg2p, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dg2p.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg2p_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(dg2p.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_status_strings():
    assert "gfx950" in dg2p.version()
    assert dg2p._lib.dg2p_status_string(-1).decode() == "DG2P_EINVAL"


def test_fma_calibration_rejects_null_output():
    """Argument checks come before any device call."""
    assert dg2p._lib.dg2p_calibrate_fp64_fma(None, None) == dg2p.EINVAL


def test_library_links_the_roctx_ranges():
    """The entry points open roctx ranges (rocprofv3 --marker-trace): the
    library depends on the ROCm roctx library."""
    import subprocess
    out = subprocess.run(["readelf", "-d", dg2p.LIB_PATH], capture_output=True, text=True).stdout
    assert "librocprofiler-sdk-roctx" in out


@pytest.mark.parametrize("bad", ["dim", "order", "n_elem", "box", "bc", "periodic_pair", "riemann_pressure",
                                 "elem_count"])
def test_create_mesh_rejects_bad_descriptors(bad):
    kw = dict(dim=2, n_elem=(4, 4), lo=(0, 0), hi=(1, 1), bc=None, order=3)
    if bad == "dim":
        kw["dim"] = 4
    elif bad == "order":
        kw["order"] = 2
    elif bad == "n_elem":
        kw["n_elem"] = (0, 4)
    elif bad == "box":
        kw["hi"] = (1, -1)
    elif bad == "bc":
        kw["bc"] = [(0, 0), (7, 7)]
    elif bad == "elem_count":          # element indices are 32-bit inside the kernels
        kw["n_elem"] = (1 << 16, 1 << 15)
    elif bad == "riemann_pressure":    # a Riemann side needs its far-field pressure
        kw["bc"] = [("slip_wall", "slip_wall"), ("no_slip", "riemann")]
    else:
        kw["bc"] = [("periodic", "slip_wall"), ("periodic", "periodic")]
    with pytest.raises(dg2p.Dg2pError) as ei:
        dg2p.Mesh(kw["dim"], kw["n_elem"], kw["lo"], kw["hi"], kw["bc"], order=kw["order"])
    want = dg2p.EUNSUPPORTED if bad == "order" else dg2p.EINVAL
    assert ei.value.status == want


def test_create_mesh_accepts_largest_element_count():
    m = dg2p.Mesh(2, ((1 << 16) - 1, 1 << 15), (0, 0), (1, 1))
    assert m.E == (1 << 31) - (1 << 15)


def test_create_mesh_accepts_wall_and_riemann_kinds():
    m = dg2p.Mesh(2, (4, 8), (-0.5, 0), (0.5, 2), [("slip_wall", "slip_wall"), ("no_slip", "riemann")],
                  bc_state={(1, 1): [1000.0]})
    assert m.E == 32


def test_params_validation():
    m = dg2p.Mesh(1, (4,), (0,), (1,))
    p = dg2p.make_params(workloads.config("drop1d")["params"])
    assert m.workspace_bytes(p, dg2p.OP_RHS) > 0
    p.gamma[0] = 1.0
    with pytest.raises(dg2p.Dg2pError):
        m.workspace_bytes(p, dg2p.OP_RHS)
    p = dg2p.make_params(workloads.config("drop1d")["params"])
    p.eps = 0.0
    with pytest.raises(dg2p.Dg2pError):
        m.workspace_bytes(p, dg2p.OP_RHS)


@pytest.mark.parametrize("name,ne", [("drop1d", (7,)), ("shock2d", (6, 5)), ("rt3d", (3, 2, 4))])
def test_node_coords_match_oracle(name, ne):
    cfg = workloads.config(name, n_elem=ne)
    m = dg2p.Mesh(cfg["dim"], ne, cfg["lo"], cfg["hi"], cfg["bc"])
    om = oracle.OracleMesh(cfg["dim"], 3, ne, cfg["lo"], cfg["hi"], cfg["bc"])
    assert (m.nf, m.E, m.nn) == (om.nf, om.E, om.nn)
    assert np.abs(m.node_coords() - om.node_coords().numpy()).max() < 1e-14


def test_workspace_sizes():
    cfg = workloads.config("rt3d", n_elem=(4, 4, 4))
    m = dg2p.Mesh(3, (4, 4, 4), cfg["lo"], cfg["hi"], cfg["bc"])
    p = dg2p.make_params(cfg["params"])
    state = 8 * 64 * 64 * 8
    g = 6 * 4 * 64 * 16 * 8          # viscous: a and tau.e_k per face node
    assert m.workspace_bytes(p, dg2p.OP_RHS) >= g
    assert m.workspace_bytes(p, dg2p.OP_RK_STEP) >= g + 2 * state


def _header_enum(prefix):
    src = open(os.path.join(ROOT, "include", "dg2p.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return {m.group(1).lower(): int(m.group(2)) for m in re.finditer(prefix + r"([A-Z0-9_]+)\s*=\s*(-?\d+)", src)}


def test_binding_enums_match_header():
    """Boundary kinds, precisions, operation codes and struct sizes of the
    binding agree with the header."""
    assert _header_enum("DG2P_BC_") == dg2p.BC
    prec = {k.replace("mixed_", ""): v for k, v in _header_enum("DG2P_").items()
            if k in ("fp64", "mixed_fp32", "mixed_bf16")}
    assert prec == dg2p.PRECISION
    ops = {k: v for k, v in _header_enum("DG2P_OP_").items()}
    assert ops["rhs"] == dg2p.OP_RHS and ops["advance"] == dg2p.OP_ADVANCE
    assert ops["kin_rhs"] == dg2p.OP_KIN_RHS and ops["kin_aux"] == dg2p.OP_KIN_AUX
    assert ctypes.sizeof(dg2p.MeshDesc) == 4 * 2 + 4 * 3 + 8 * 6 + 4 * 6 + 4 + 8 * 48   # incl. 4 padding bytes
    assert ctypes.sizeof(dg2p.Monitors) == 8 * 15


def test_noalloc_step_refuses_oversized_mesh_before_any_device_call():
    """dg2p_rk_step_noalloc checks the mesh's workspace against its static
    scratch (64 MiB) on the host and returns DG2P_EWORKSPACE without touching
    the device (the pointers below are never dereferenced)."""
    assert dg2p.noalloc_scratch_bytes() == 64 << 20
    P = dg2p.make_params(workloads.config("drop2d")["params"])
    mesh = dg2p.Mesh(2, (512, 256), (0.0, 0.0), (2.0, 1.0))      # two 117 MB stage states
    assert mesh.workspace_bytes(P, dg2p.OP_RK_STEP) > dg2p.noalloc_scratch_bytes()
    fake = ctypes.c_void_p(1 << 20)
    st = dg2p._lib.dg2p_rk_step_noalloc(mesh.handle, ctypes.byref(P), fake, fake, None)
    assert st == dg2p.EWORKSPACE
    assert "static scratch" in dg2p._lib.dg2p_last_error().decode()
    st = dg2p._lib.dg2p_rk_step_noalloc(mesh.handle, ctypes.byref(P), None, fake, None)
    assert st == dg2p.EINVAL


@pytest.mark.parametrize("n_elem,hi", [((16, 16), (1.0, 1.0)), ((8, 12), (2.0, 1.0))])
def test_kin_reinit_params_match_the_oracle_reading(n_elem, hi):
    """dg2p_kin_reinit_params (host arithmetic in the library) and the
    oracle's reinit_params implement the same reading independently:
    nu = h_min / (p+1), dtau = 0.1 h_min / (1 + (p+1)^2 d nu / h_min)."""
    from oracle import kinematic as K
    mesh = dg2p.Mesh(2, n_elem, (0.0, 0.0), hi)
    om = oracle.OracleMesh(2, 3, n_elem, (0.0, 0.0), hi)
    nu, dtau = dg2p.kin_reinit_params(mesh)
    onu, odtau = K.reinit_params(om)
    assert abs(nu - onu) <= 1e-15 * onu and abs(dtau - odtau) <= 1e-15 * odtau


def test_order_one_meshes_and_their_host_checks():
    """p = 1 meshes (kinematic mode): four nodes per 2D element at the
    corners, weights J_x J_y; the two-phase entry points and the
    re-initialisation refuse them on the host, and the stream-function
    velocity refuses non-2D meshes and aliasing before any device call."""
    m1 = dg2p.Mesh(2, (5, 4), (0.0, 0.0), (1.0, 1.0), order=1)
    assert (m1.nf, m1.E, m1.nn) == (7, 20, 4)
    om = oracle.OracleMesh(2, 1, (5, 4), (0.0, 0.0), (1.0, 1.0))
    assert np.array_equal(m1.node_coords(), om.node_coords().numpy())
    W = m1.node_weights()
    assert np.allclose(np.asarray(W), om.node_weights().numpy(), rtol=0, atol=1e-17)
    fake = ctypes.c_void_p(1 << 20)
    P = dg2p.make_params(workloads.config("drop2d")["params"])
    st = dg2p._lib.dg2p_rhs(m1.handle, ctypes.byref(P), fake, ctypes.c_void_p(2 << 20), fake, None)
    assert st == dg2p.EUNSUPPORTED
    kp = dg2p.make_kin_params()
    st = dg2p._lib.dg2p_kin_reinit(m1.handle, ctypes.byref(kp), fake, 2, ctypes.c_double(0.1),
                                   ctypes.c_double(0.01), fake, None)
    assert st == dg2p.EUNSUPPORTED
    m3 = dg2p.Mesh(3, (2, 2, 2), (0.0,) * 3, (1.0,) * 3)
    assert dg2p._lib.dg2p_kin_velocity_from_stream(m3.handle, fake, ctypes.c_void_p(2 << 20), None) \
        == dg2p.EUNSUPPORTED
    assert dg2p._lib.dg2p_kin_velocity_from_stream(m1.handle, fake, fake, None) == dg2p.EINVAL
    assert dg2p._lib.dg2p_kin_velocity_from_stream(m1.handle, None, fake, None) == dg2p.EINVAL


def test_order_four_quadrilaterals():
    """p = 4 on quadrilaterals (the paper's order for the wall-bounded runs):
    25 nodes per element at the GLL points of degree 4, weights W_j =
    w_a w_b J_x J_y, the face-ingredient buffer sized for 5 nodes per face;
    hexahedra of order 4 are refused."""
    m = dg2p.Mesh(2, (3, 2), (0.0, 0.0), (1.5, 1.0), order=4)
    assert (m.nf, m.E, m.nn) == (7, 6, 25)
    om = oracle.OracleMesh(2, 4, (3, 2), (0.0, 0.0), (1.5, 1.0))
    assert np.abs(m.node_coords() - om.node_coords().numpy()).max() < 1e-15
    assert np.abs(np.asarray(m.node_weights()) - om.node_weights().numpy()).max() < 1e-16
    with pytest.raises(dg2p.Dg2pError) as ei:
        dg2p.Mesh(3, (2, 2, 2), (0.0,) * 3, (1.0,) * 3, order=4)
    assert ei.value.status == dg2p.EUNSUPPORTED
    P = dg2p.make_params(workloads.config("drop2d")["params"])
    m3 = dg2p.Mesh(2, (3, 2), (0.0, 0.0), (1.0, 1.0), order=3)
    assert m.workspace_bytes(P, dg2p.OP_RHS) > m3.workspace_bytes(P, dg2p.OP_RHS)
