"""Glue between the seeded workloads and the oracle, used by the tests."""

import numpy as np
import torch

import oracle
from paper_2306_05002_amd import workloads


def oracle_setup(name, n_elem=None, variant=None, bc=None, bc_state=None, order=3, **param_over):
    """(cfg, mesh, params, U0) for a configuration, built on the oracle side.
    ``bc`` overrides the boundary kinds (e.g. all periodic), ``bc_state`` the
    raw per-side boundary values (e.g. a Riemann far-field pressure), ``order``
    the polynomial degree."""
    cfg = workloads.config(name, n_elem=n_elem, order=order)
    if bc is not None:
        cfg["bc"] = bc
        cfg["bc_prim"] = {}
    if bc_state is not None:
        cfg["bc_state"] = dict(bc_state)
    cfg["params"] = {**cfg["params"], **param_over}   # overrides reach the initial state too
    prm = oracle.Params(**cfg["params"])
    d = cfg["dim"]
    bc_state = {key: torch.tensor(v, dtype=torch.float64) for key, v in cfg.get("bc_state", {}).items()}
    for key, bp in cfg.get("bc_prim", {}).items():
        t = lambda v: torch.tensor([float(v)], dtype=torch.float64)
        Qb = oracle.prim_to_cons(t(bp["alpha"]), t(bp["psi"]), t(bp["rho1"]),
                                 t(bp["rho2"]),
                                 torch.tensor(bp["u"][:d], dtype=torch.float64)[:, None],
                                 t(bp["P"]), prm)
        bc_state[key] = Qb[:, 0]
    mesh = oracle.OracleMesh(d, cfg["order"], cfg["n_elem"], cfg["lo"], cfg["hi"],
                             cfg["bc"], bc_state)
    X = mesh.node_coords().numpy()
    pf = workloads.primitive_fields(cfg, X, variant=variant)
    U0 = cons_from_prim(pf, prm)
    return cfg, mesh, prm, U0


def cons_from_prim(pf, prm):
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)
    return oracle.prim_to_cons(T(pf["alpha"]), T(pf["psi"]), T(pf["rho1"]),
                               T(pf["rho2"]), T(pf["u"]), T(pf["P"]), prm)


def field_scales(U, d, prm):
    """Magnitude of each field for the parity metric: max|U_f|, except the
    momentum components, which use the momentum-flux scale max rho (|u| + c)
    (a momentum component can be identically zero, e.g. the transverse one of
    a planar shock, while its residual carries pressure round-off)."""
    pr = oracle.primitives(U, d, prm)
    speed = torch.sqrt((pr["u"] ** 2).sum(0)) + pr["c"]
    mom = float((pr["rho"] * speed).max())
    out = []
    for f in range(U.shape[0]):
        out.append(mom if 2 <= f < 2 + d else float(U[f].abs().max()))
    return out


def rel_err_fields(X, Y, scale):
    """Per-field normwise error max|X - Y| / max(max|Y|, scale_f)."""
    out = []
    for f in range(X.shape[0]):
        num = float(torch.abs(X[f] - Y[f]).max())
        den = max(float(torch.abs(Y[f]).max()), float(scale[f]))
        out.append(num / den if den > 0 else num)
    return out
