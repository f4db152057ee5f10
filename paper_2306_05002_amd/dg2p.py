"""Thin ctypes binding of libdg2p (the C ABI of include/dg2p.h).

Argument marshalling only: every step of the residual, the RK stages, the
time-step reduction, the monitors and the initial-condition map runs in the
library's HIP kernels.  Torch provides device memory (tensors), streams and
the workspace buffers.  Importing this module loads ``libdg2p.so`` from the
package directory (or the file named by the environment variable
DG2P_LIBRARY, for comparing two builds) and raises ImportError if it is
missing: there is no fallback path.
"""

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DG2P_LIBRARY") or os.path.join(_HERE, "libdg2p.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libdg2p.so not found at {LIB_PATH}; run __graft_entry__.build()")
_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, EHIP, ENONPHYS, EUNSUPPORTED, EWORKSPACE = 0, -1, -2, -3, -4, -5
BC = {"periodic": 0, "slip_wall": 1, "dirichlet": 2, "extrapolate": 3, "no_slip": 4, "riemann": 5}
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2}
OP_RHS, OP_RK_STEP, OP_MAX_DT, OP_MONITORS, OP_RHS_VJP, OP_RK_STEP_VJP, OP_ADVANCE = range(7)
OP_KIN_RHS, OP_KIN_RK4, OP_KIN_AUX = 7, 8, 9


class MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("order", ctypes.c_int),
                ("n_elem", ctypes.c_int * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("bc", (ctypes.c_int * 2) * 3),
                ("bc_state", ((ctypes.c_double * 8) * 2) * 3)]


class KinParams(ctypes.Structure):
    _fields_ = [("Gamma", ctypes.c_double), ("eps", ctypes.c_double), ("c_ip", ctypes.c_double),
                ("grad_reg", ctypes.c_double), ("period", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double * 2), ("pinf", ctypes.c_double * 2),
                ("rho0", ctypes.c_double * 2), ("Gamma", ctypes.c_double),
                ("eps", ctypes.c_double), ("mu", ctypes.c_double * 2),
                ("sigma", ctypes.c_double), ("g", ctypes.c_double * 3),
                ("c_ip", ctypes.c_double), ("grad_reg", ctypes.c_double),
                ("precision", ctypes.c_int)]


class Monitors(ctypes.Structure):
    _fields_ = [("max_rate", ctypes.c_double), ("dt", ctypes.c_double),
                ("min_alpha", ctypes.c_double), ("max_alpha", ctypes.c_double),
                ("integral", ctypes.c_double * 8), ("dev_p", ctypes.c_double),
                ("dev_u", ctypes.c_double), ("nonphys", ctypes.c_longlong)]


MONITOR_DOUBLES = ctypes.sizeof(Monitors) // 8

_vp, _dp, _i, _d = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
_SIG = {
    "dg2p_version": ([], ctypes.c_char_p),
    "dg2p_status_string": ([_i], ctypes.c_char_p),
    "dg2p_last_error": ([], ctypes.c_char_p),
    "dg2p_create_mesh": ([ctypes.POINTER(MeshDesc), ctypes.POINTER(ctypes.c_void_p)], _i),
    "dg2p_destroy_mesh": ([_vp], _i),
    "dg2p_layout": ([_vp, ctypes.POINTER(_i), ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(_i)], _i),
    "dg2p_node_coords": ([_vp, _dp], _i),
    "dg2p_workspace_size": ([_vp, ctypes.POINTER(Params), _i, ctypes.POINTER(ctypes.c_size_t)], _i),
    "dg2p_prim_to_cons": ([_vp, ctypes.POINTER(Params), _dp, _dp, _vp], _i),
    "dg2p_rhs": ([_vp, ctypes.POINTER(Params), _dp, _dp, _vp, _vp], _i),
    "dg2p_max_dt": ([_vp, ctypes.POINTER(Params), _dp, _d, _dp, _vp, _vp, _vp], _i),
    "dg2p_rk_step": ([_vp, ctypes.POINTER(Params), _dp, _dp, _vp, _vp], _i),
    "dg2p_rk_step_noalloc": ([_vp, ctypes.POINTER(Params), _dp, _dp, _vp], _i),
    "dg2p_kin_reinit_params": ([_vp, _d, ctypes.POINTER(_d), ctypes.POINTER(_d)], _i),
    "dg2p_noalloc_scratch_bytes": ([], ctypes.c_size_t),
    "dg2p_compute_monitors": ([_vp, ctypes.POINTER(Params), _dp, _d, _dp, _vp, _vp, _vp], _i),
    "dg2p_advance": ([_vp, ctypes.POINTER(Params), _dp, _i, _d, _dp, _dp, _dp, _vp, _d, _vp, _vp, _vp], _i),
    "dg2p_advance_monitored": ([_vp, ctypes.POINTER(Params), _dp, _i, _d, _dp, _dp, _dp, _vp, _d, _vp, _vp,
                                _vp], _i),
    "dg2p_rhs_vjp": ([_vp, ctypes.POINTER(Params), _dp, _dp, _dp, _dp, _vp, _vp], _i),
    "dg2p_rk_step_vjp": ([_vp, ctypes.POINTER(Params), _dp, _dp, _dp, _dp, _dp, _vp, _vp], _i),
    "dg2p_prim_to_cons_vjp": ([_vp, ctypes.POINTER(Params), _dp, _dp, _dp, _vp], _i),
    "dg2p_node_weights": ([_vp, _dp], _i),
    "dg2p_kin_workspace_size": ([_vp, _i, ctypes.POINTER(ctypes.c_size_t)], _i),
    "dg2p_kin_rhs": ([_vp, ctypes.POINTER(KinParams), _dp, _dp, _d, _dp, _vp, _vp], _i),
    "dg2p_kin_rk4": ([_vp, ctypes.POINTER(KinParams), _dp, _dp, _i, _d, _d, _vp, _vp], _i),
    "dg2p_kin_max_dt": ([_vp, ctypes.POINTER(KinParams), _dp, _d, _dp, _vp, _vp], _i),
    "dg2p_kin_reinit": ([_vp, ctypes.POINTER(KinParams), _dp, _i, _d, _d, _vp, _vp], _i),
    "dg2p_kin_errors": ([_vp, _dp, _dp, _dp, _vp, _vp], _i),
    "dg2p_kin_velocity_from_stream": ([_vp, _dp, _dp, _vp], _i),
    "dg2p_calibrate_fp64_fma": ([ctypes.POINTER(_d), _vp], _i),
    "dg2p_timing_enable": ([_i], _i),
    "dg2p_timing_read": ([_i, ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_longlong)], _i),
}
K_INGREDIENTS, K_STAGE, K_RATE, K_RATE_FINAL, K_MONITOR, K_PRIM, K_VJP_LOCAL, K_VJP_GATHER, K_KIN_STAGE = range(9)
for _name, (_args, _res) in _SIG.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


class Dg2pError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        detail = _lib.dg2p_last_error().decode()
        name = _lib.dg2p_status_string(status).decode()
        super().__init__(f"{what}: {name} ({detail})")


def _check(status, what):
    if status != OK:
        raise Dg2pError(status, what)


def version():
    return _lib.dg2p_version().decode()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_params(p, precision="fp64"):
    """dg2p_params from a dict with keys gamma, pinf, rho0, Gamma, eps, mu,
    sigma, g, c_ip, grad_reg (the workloads module's parameter dict)."""
    P = Params()
    P.gamma[:] = list(p["gamma"])
    P.pinf[:] = list(p["pinf"])
    P.rho0[:] = list(p["rho0"])
    P.Gamma = p["Gamma"]
    P.eps = p["eps"]
    P.mu[:] = list(p.get("mu", (0.0, 0.0)))
    P.sigma = p.get("sigma", 0.0)
    g = list(p.get("g", (0.0, 0.0, 0.0))) + [0.0, 0.0, 0.0]
    P.g[:] = g[:3]
    P.c_ip = p.get("c_ip", 1.0)
    P.grad_reg = p.get("grad_reg", 1e-12)
    P.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    return P


class Mesh:
    """Owning wrapper of a dg2p_mesh handle plus cached workspaces."""

    def __init__(self, dim, n_elem, lo, hi, bc=None, bc_state=None, order=3):
        d = MeshDesc()
        d.dim = dim
        d.order = order
        for k in range(3):
            have = k < min(dim, len(n_elem))
            d.n_elem[k] = int(n_elem[k]) if have else 1
            d.lo[k] = float(lo[k]) if have else 0.0
            d.hi[k] = float(hi[k]) if have else 1.0
            for s in range(2):
                kind = bc[k][s] if (bc is not None and k < min(dim, len(bc))) else "periodic"
                d.bc[k][s] = BC[kind] if isinstance(kind, str) else int(kind)
                vals = (bc_state or {}).get((k, s))
                if vals is not None:
                    for f, v in enumerate(list(vals)[:8]):
                        d.bc_state[k][s][f] = float(v)
        h = ctypes.c_void_p()
        _check(_lib.dg2p_create_mesh(ctypes.byref(d), ctypes.byref(h)), "dg2p_create_mesh")
        self._h = h
        self.desc = d
        self.dim = dim
        nf, E, nn = ctypes.c_int(), ctypes.c_longlong(), ctypes.c_int()
        _check(_lib.dg2p_layout(h, ctypes.byref(nf), ctypes.byref(E), ctypes.byref(nn)), "dg2p_layout")
        self.nf, self.E, self.nn = nf.value, E.value, nn.value
        self._ws = {}

    @property
    def handle(self):
        return self._h

    def __del__(self, _destroy=_lib.dg2p_destroy_mesh):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _destroy(h)
            self._h = None

    def state_shape(self):
        return (self.nf, self.E, self.nn)

    def node_coords(self):
        out = np.empty((self.dim, self.E, self.nn), dtype=np.float64)
        _check(_lib.dg2p_node_coords(self._h, out.ctypes.data_as(ctypes.c_void_p)), "dg2p_node_coords")
        return out

    def node_weights(self):
        out = np.empty(self.nn, dtype=np.float64)
        _check(_lib.dg2p_node_weights(self._h, out.ctypes.data_as(ctypes.c_void_p)), "dg2p_node_weights")
        return out

    def workspace_bytes(self, params, op):
        n = ctypes.c_size_t()
        _check(_lib.dg2p_workspace_size(self._h, ctypes.byref(params), op, ctypes.byref(n)),
               "dg2p_workspace_size")
        return n.value

    def workspace(self, params, op, device):
        """Device workspace for an operation (cached per op, grown on demand)."""
        if op >= OP_KIN_RHS:
            n = ctypes.c_size_t()
            _check(_lib.dg2p_kin_workspace_size(self._h, op, ctypes.byref(n)), "dg2p_kin_workspace_size")
            need = n.value
        else:
            need = self.workspace_bytes(params, op)
        key = (op, str(device))
        buf = self._ws.get(key)
        if buf is None or buf.numel() < need + 256:
            buf = torch.empty(max(need + 256, 256), dtype=torch.uint8, device=device)
            self._ws[key] = buf
        off = (-buf.data_ptr()) % 256
        return ctypes.c_void_p(buf.data_ptr() + off) if need else None


def _as_state(mesh, U):
    if U.dtype != torch.float64 or not U.is_cuda or not U.is_contiguous():
        raise ValueError("state must be a contiguous float64 CUDA tensor")
    if tuple(U.shape) != mesh.state_shape():
        raise ValueError(f"state shape {tuple(U.shape)} != {mesh.state_shape()}")
    return U


def prim_to_cons(mesh, params, prim, stream=None):
    prim = _as_state(mesh, prim)
    U = torch.empty_like(prim)
    _check(_lib.dg2p_prim_to_cons(mesh.handle, ctypes.byref(params), _ptr(prim), _ptr(U),
                                  _stream(stream)), "dg2p_prim_to_cons")
    return U


def prim_to_cons_vjp(mesh, params, prim, U_bar, stream=None):
    prim = _as_state(mesh, prim)
    U_bar = _as_state(mesh, U_bar)
    out = torch.empty_like(prim)
    _check(_lib.dg2p_prim_to_cons_vjp(mesh.handle, ctypes.byref(params), _ptr(prim), _ptr(U_bar), _ptr(out),
                                      _stream(stream)), "dg2p_prim_to_cons_vjp")
    return out


def rhs(mesh, params, U, out=None, stream=None):
    U = _as_state(mesh, U)
    R = torch.empty_like(U) if out is None else out
    ws = mesh.workspace(params, OP_RHS, U.device)
    _check(_lib.dg2p_rhs(mesh.handle, ctypes.byref(params), _ptr(U), _ptr(R), ws, _stream(stream)),
           "dg2p_rhs")
    return R


def max_dt(mesh, params, U, cfl=0.1, dt=None, stream=None):
    """Device scalar dt = cfl / max_rate (no host synchronisation)."""
    U = _as_state(mesh, U)
    if dt is None:
        dt = torch.empty(1, dtype=torch.float64, device=U.device)
    ws = mesh.workspace(params, OP_MAX_DT, U.device)
    _check(_lib.dg2p_max_dt(mesh.handle, ctypes.byref(params), _ptr(U), float(cfl), _ptr(dt), None, ws,
                            _stream(stream)), "dg2p_max_dt")
    return dt


def rk_step(mesh, params, U, dt, stream=None):
    """One SSP-RK3 step, in place on U; dt is a 1-element float64 device tensor."""
    U = _as_state(mesh, U)
    ws = mesh.workspace(params, OP_RK_STEP, U.device)
    _check(_lib.dg2p_rk_step(mesh.handle, ctypes.byref(params), _ptr(U), _ptr(dt), ws, _stream(stream)),
           "dg2p_rk_step")
    return U


def rk_step_noalloc(mesh, params, U, dt, stream=None):
    """dg2p_rk_step_noalloc: the step of rk_step with the library's static
    device scratch instead of a workspace (no device allocation anywhere on
    the call path).  Raises Dg2pError (DG2P_EWORKSPACE) for meshes whose
    workspace exceeds noalloc_scratch_bytes()."""
    U = _as_state(mesh, U)
    _check(_lib.dg2p_rk_step_noalloc(mesh.handle, ctypes.byref(params), _ptr(U), _ptr(dt), _stream(stream)),
           "dg2p_rk_step_noalloc")
    return U


def noalloc_scratch_bytes():
    """Bytes of the static device scratch behind rk_step_noalloc."""
    return int(_lib.dg2p_noalloc_scratch_bytes())


def advance(mesh, params, U, n_steps, cfl=0.1, dt_fixed=None, t=None, dt_last=None, mon=None,
            p_ref=0.0, u_ref=None, stream=None):
    """n_steps SSP-RK3 steps in place with device-side dt (no host sync).
    dt_fixed / t / dt_last: 1-element float64 device tensors (optional);
    mon: float64 device tensor of MONITOR_DOUBLES (optional)."""
    U = _as_state(mesh, U)
    ws = mesh.workspace(params, OP_ADVANCE, U.device)
    ur = (ctypes.c_double * 3)(*([0.0, 0.0, 0.0] if u_ref is None else (list(u_ref) + [0.0] * 3)[:3]))
    _check(_lib.dg2p_advance(mesh.handle, ctypes.byref(params), _ptr(U), int(n_steps), float(cfl),
                             _ptr(dt_fixed), _ptr(t), _ptr(dt_last), _ptr(mon), float(p_ref),
                             ctypes.cast(ur, ctypes.c_void_p), ws, _stream(stream)), "dg2p_advance")
    return U


def advance_monitored(mesh, params, U, n_steps, mon_steps, cfl=0.1, dt_fixed=None, t=None, dt_last=None,
                      p_ref=0.0, u_ref=None, stream=None):
    """advance() with the monitors of every step: mon_steps is a float64
    device tensor of shape (n_steps, MONITOR_DOUBLES); row i receives the
    monitors of the state after step i + 1 (decode with decode_monitors)."""
    U = _as_state(mesh, U)
    if (mon_steps.dtype != torch.float64 or not mon_steps.is_cuda or not mon_steps.is_contiguous()
            or mon_steps.numel() < int(n_steps) * MONITOR_DOUBLES):
        raise ValueError("mon_steps must be a contiguous float64 CUDA tensor of n_steps x MONITOR_DOUBLES")
    ws = mesh.workspace(params, OP_ADVANCE, U.device)
    ur = (ctypes.c_double * 3)(*([0.0, 0.0, 0.0] if u_ref is None else (list(u_ref) + [0.0] * 3)[:3]))
    _check(_lib.dg2p_advance_monitored(mesh.handle, ctypes.byref(params), _ptr(U), int(n_steps), float(cfl),
                                       _ptr(dt_fixed), _ptr(t), _ptr(dt_last), _ptr(mon_steps), float(p_ref),
                                       ctypes.cast(ur, ctypes.c_void_p), ws, _stream(stream)),
           "dg2p_advance_monitored")
    return U


def rhs_vjp(mesh, params, U, R_bar, param_bar=None, stream=None):
    """U_bar = (dR/dU)^T R_bar; param_bar (1-element device tensor) += sigma cotangent."""
    U = _as_state(mesh, U)
    R_bar = _as_state(mesh, R_bar)
    Ub = torch.empty_like(U)
    ws = mesh.workspace(params, OP_RHS_VJP, U.device)
    _check(_lib.dg2p_rhs_vjp(mesh.handle, ctypes.byref(params), _ptr(U), _ptr(R_bar), _ptr(Ub),
                             _ptr(param_bar), ws, _stream(stream)), "dg2p_rhs_vjp")
    return Ub


def rk_step_vjp(mesh, params, U_n, dt, U_np1_bar, param_bar=None, out=None, stream=None):
    """U_n_bar = (dU_{n+1}/dU_n)^T U_np1_bar for one SSP-RK3 step with device dt."""
    U_n = _as_state(mesh, U_n)
    U_np1_bar = _as_state(mesh, U_np1_bar)
    Ub = torch.empty_like(U_n) if out is None else out
    ws = mesh.workspace(params, OP_RK_STEP_VJP, U_n.device)
    _check(_lib.dg2p_rk_step_vjp(mesh.handle, ctypes.byref(params), _ptr(U_n), _ptr(dt), _ptr(U_np1_bar),
                                 _ptr(Ub), _ptr(param_bar), ws, _stream(stream)), "dg2p_rk_step_vjp")
    return Ub


def decode_monitors(buf, nf):
    """Monitors from a device or host buffer of MONITOR_DOUBLES float64 (a
    dg2p_monitors struct); for a (n, MONITOR_DOUBLES) buffer, a list of n."""
    raw = buf.detach().cpu().numpy()
    if raw.ndim == 2:
        return [decode_monitors(torch.from_numpy(r.copy()), nf) for r in raw]
    m = Monitors.from_buffer_copy(raw.tobytes())
    return dict(max_rate=m.max_rate, dt=m.dt, min_alpha=m.min_alpha, max_alpha=m.max_alpha,
                integral=list(m.integral)[:nf], dev_p=m.dev_p, dev_u=m.dev_u,
                nonphys=int(m.nonphys))


def monitors(mesh, params, U, p_ref=0.0, u_ref=None, stream=None, sync=True):
    U = _as_state(mesh, U)
    buf = torch.zeros(MONITOR_DOUBLES, dtype=torch.float64, device=U.device)
    ur = (ctypes.c_double * 3)(*([0.0, 0.0, 0.0] if u_ref is None else (list(u_ref) + [0.0] * 3)[:3]))
    ws = mesh.workspace(params, OP_MONITORS, U.device)
    _check(_lib.dg2p_compute_monitors(mesh.handle, ctypes.byref(params), _ptr(U), float(p_ref),
                                      ctypes.cast(ur, ctypes.c_void_p), _ptr(buf), ws, _stream(stream)),
           "dg2p_compute_monitors")
    if not sync:
        return buf
    return decode_monitors(buf, mesh.nf)


def require_physical(mon, what="state"):
    """Raise Dg2pError(DG2P_ENONPHYS) when decoded monitors count
    non-physical nodes (partial densities summing to <= 0, (1+xi) P + Pi <= 0,
    or a NaN / Inf); returns the monitors otherwise."""
    if mon["nonphys"] > 0:
        raise Dg2pError(ENONPHYS, f"{what}: {mon['nonphys']} non-physical nodes")
    return mon


def calibrate_fp64_fma(stream=None):
    """Measured FP64 vector FMA rate of the device in TFLOP/s (host blocking)."""
    v = ctypes.c_double()
    _check(_lib.dg2p_calibrate_fp64_fma(ctypes.byref(v), _stream(stream)), "dg2p_calibrate_fp64_fma")
    return v.value


def timing_enable(on=True):
    """Bracket every library kernel launch with hipEvents (benchmarks only)."""
    _check(_lib.dg2p_timing_enable(1 if on else 0), "dg2p_timing_enable")


def timing_read(kind):
    """(mean ms, count) of the recorded launches of one kernel kind."""
    ms, n = ctypes.c_double(), ctypes.c_longlong()
    _check(_lib.dg2p_timing_read(kind, ctypes.byref(ms), ctypes.byref(n)), "dg2p_timing_read")
    return ms.value, n.value


def mesh_from_config(cfg, params=None):
    """Mesh for a workloads configuration; Dirichlet states are mapped to
    conserved variables with the library's own initial-condition kernel."""
    d = cfg["dim"]
    bc_state = {key: list(v) for key, v in cfg.get("bc_state", {}).items()}
    if cfg.get("bc_prim"):
        P = make_params(cfg["params"]) if params is None else params
        probe = Mesh(d, (1,) * d, (0.0,) * d, (1.0,) * d)
        for key, bp in cfg["bc_prim"].items():
            vals = [bp["alpha"], bp["psi"], bp["rho1"], bp["rho2"]] + list(bp["u"][:d]) + [bp["P"]]
            prim = torch.tensor(vals, dtype=torch.float64, device="cuda")[:, None, None]
            prim = prim.expand(probe.nf, 1, probe.nn).contiguous()
            Uc = prim_to_cons(probe, P, prim)
            bc_state[key] = Uc[:, 0, 0].cpu().tolist()
    return Mesh(d, cfg["n_elem"], cfg["lo"], cfg["hi"], cfg["bc"], bc_state, order=cfg["order"])


def prim_tensor(pf, d, device="cuda"):
    """Stack the workloads primitive dict into the library's primitive layout."""
    arrs = [pf["alpha"], pf["psi"], pf["rho1"], pf["rho2"]] + [pf["u"][j] for j in range(d)] + [pf["P"]]
    host = np.stack([np.ascontiguousarray(a, dtype=np.float64) for a in arrs])
    return torch.from_numpy(host).to(device)


# ---- kinematic mode: phi and psi under a prescribed velocity u0(x) s(t) -------------
def make_kin_params(Gamma=1.0, eps=0.01, c_ip=1.0, grad_reg=1e-12, period=0.0):
    return KinParams(float(Gamma), float(eps), float(c_ip), float(grad_reg), float(period))


def _as_kin(mesh, t, rows, what):
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous float64 CUDA tensor")
    if tuple(t.shape) != (rows, mesh.E, mesh.nn):
        raise ValueError(f"{what} shape {tuple(t.shape)} != {(rows, mesh.E, mesh.nn)}")
    return t


def kin_rhs(mesh, kp, Phi, u0, t, out=None, stream=None):
    """R = dPhi/dt at time t; Phi [2, E, nn] (phi, psi), u0 [d, E, nn]."""
    Phi = _as_kin(mesh, Phi, 2, "Phi")
    u0 = _as_kin(mesh, u0, mesh.dim, "u0")
    R = torch.empty_like(Phi) if out is None else out
    ws = mesh.workspace(None, OP_KIN_RHS, Phi.device)
    _check(_lib.dg2p_kin_rhs(mesh.handle, ctypes.byref(kp), _ptr(Phi), _ptr(u0), float(t), _ptr(R), ws,
                             _stream(stream)), "dg2p_kin_rhs")
    return R


def kin_rk4(mesh, kp, Phi, u0, n_steps, t0, dt, stream=None):
    """n_steps classical RK4 steps in place from t0 with fixed dt (host scalars)."""
    Phi = _as_kin(mesh, Phi, 2, "Phi")
    u0 = _as_kin(mesh, u0, mesh.dim, "u0")
    ws = mesh.workspace(None, OP_KIN_RK4, Phi.device)
    _check(_lib.dg2p_kin_rk4(mesh.handle, ctypes.byref(kp), _ptr(Phi), _ptr(u0), int(n_steps), float(t0),
                             float(dt), ws, _stream(stream)), "dg2p_kin_rk4")
    return Phi


def kin_max_dt(mesh, kp, u0, cfl=0.1, stream=None):
    """Device scalar dt of the kinematic time-step rule."""
    u0 = _as_kin(mesh, u0, mesh.dim, "u0")
    dt = torch.empty(1, dtype=torch.float64, device=u0.device)
    ws = mesh.workspace(None, OP_KIN_AUX, u0.device)
    _check(_lib.dg2p_kin_max_dt(mesh.handle, ctypes.byref(kp), _ptr(u0), float(cfl), _ptr(dt), ws,
                                _stream(stream)), "dg2p_kin_max_dt")
    return dt


def kin_errors(mesh, phi, phi0, stream=None):
    """(int |phi - phi0|, int (phi - phi0), int phi0) as a device tensor of 3."""
    for t, w in ((phi, "phi"), (phi0, "phi0")):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or \
                tuple(t.shape) != (mesh.E, mesh.nn):
            raise ValueError(f"{w} must be a contiguous float64 CUDA tensor of shape (E, nn)")
    out = torch.empty(3, dtype=torch.float64, device=phi.device)
    ws = mesh.workspace(None, OP_KIN_AUX, phi.device)
    _check(_lib.dg2p_kin_errors(mesh.handle, _ptr(phi), _ptr(phi0), _ptr(out), ws, _stream(stream)),
           "dg2p_kin_errors")
    return out


def kin_velocity_from_stream(mesh, S, stream=None):
    """Velocity amplitude u0 = (dS/dy, -dS/dx) [2, E, nn] of a nodal stream
    function S [E, nn] (2D; element-local derivatives)."""
    if S.dtype != torch.float64 or not S.is_cuda or not S.is_contiguous() or tuple(S.shape) != (mesh.E, mesh.nn):
        raise ValueError("S must be a contiguous float64 CUDA tensor of shape (E, nn)")
    u0 = torch.empty(2, mesh.E, mesh.nn, dtype=torch.float64, device=S.device)
    _check(_lib.dg2p_kin_velocity_from_stream(mesh.handle, _ptr(S), _ptr(u0), _stream(stream)),
           "dg2p_kin_velocity_from_stream")
    return u0


def kin_reinit(mesh, kp, Phi, n_iter, nu, dtau, stream=None):
    """Re-initialise Phi[1] (psi) from Phi[0] (phi) in place: n_iter RK4
    pseudo-time steps of the Eikonal relaxation with viscosity nu."""
    Phi = _as_kin(mesh, Phi, 2, "Phi")
    ws = mesh.workspace(None, OP_KIN_RK4, Phi.device)
    _check(_lib.dg2p_kin_reinit(mesh.handle, ctypes.byref(kp), _ptr(Phi), int(n_iter), float(nu), float(dtau), ws,
                                _stream(stream)), "dg2p_kin_reinit")
    return Phi


def kin_reinit_params(mesh, cfl=0.1):
    """(nu_h, dtau) of dg2p_kin_reinit_params."""
    nu, dtau = ctypes.c_double(), ctypes.c_double()
    _check(_lib.dg2p_kin_reinit_params(mesh.handle, float(cfl), ctypes.byref(nu), ctypes.byref(dtau)),
           "dg2p_kin_reinit_params")
    return nu.value, dtau.value
