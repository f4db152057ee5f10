"""Writes rk2d_16x16_p3.json (and, with --reinit, rk2d_16x16_p3_reinit.json;
with --p1, rk2d_32x32_p1.json): the oracle's Rider-Kothe run (16 x 16
elements, p = 3, i.e. 64^2 nodes, eps = h/2; or 32 x 32 elements at p = 1,
eps = h; Gamma = 1, T = 4, classical RK4 with the kinematic time-step rule at
CFL 0.1, one full period; with --reinit the level set is re-initialised from
phi for 50 pseudo-time iterations every 2000 steps): the L1 error and the
relative mass error of phi.  Calls the oracle only.  Takes about 20 minutes
on 4 CPU threads.

    python tests/golden/make_kinematic_golden.py [--reinit | --p1]
"""

import json
import math
import os
import sys

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import kinematic as K  # noqa: E402
from paper_2306_05002_amd import workloads  # noqa: E402


def main():
    torch.set_num_threads(4)
    order, N = (1, 32) if "--p1" in sys.argv else (3, 16)
    cfg = workloads.kinematic_config("rk2d", n_elem=(N, N), order=order)
    mesh = oracle.OracleMesh(2, order, cfg["n_elem"], cfg["lo"], cfg["hi"], cfg["bc"])
    X = mesh.node_coords().numpy()
    phi, psi, u0 = workloads.kinematic_fields(cfg, X)
    T = lambda a: torch.as_tensor(a, dtype=torch.float64)
    kp = K.KinParams(**cfg["kin"])
    Phi0 = torch.stack([T(phi), T(psi)])
    U0 = T(u0)
    dt0 = K.max_dt(U0, mesh, kp, cfg["cfl"])
    ns = int(math.ceil(cfg["t_end"] / dt0))
    dt = cfg["t_end"] / ns
    reinit = "--reinit" in sys.argv
    nu, dtau = K.reinit_params(mesh)
    Phi = Phi0
    n_reinit = 0
    for s in range(ns):
        Phi = K.rk4_step(Phi, s * dt, dt, U0, mesh, kp)
        if reinit and (s + 1) % 2000 == 0 and s + 1 < ns:
            Phi = torch.stack([Phi[0], K.reinit(Phi[0], mesh, kp, 50, nu, dtau)])
            n_reinit += 1
    out = dict(case="rk2d", n_elem=[N, N], order=order, eps=cfg["kin"]["eps"], steps=ns, dt=dt, reinit=n_reinit,
               l1=K.l1_error(Phi[0], Phi0[0], mesh), mass_error=K.mass_error(Phi[0], Phi0[0], mesh),
               phi_min=float(Phi[0].min()), phi_max=float(Phi[0].max()))
    name = "rk2d_%dx%d_p%d%s.json" % (N, N, order, "_reinit" if reinit else "")
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
