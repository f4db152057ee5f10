"""Kinematic test runs on the library's kinematic mode (phase field and level
set under a prescribed velocity; Results, "Kinematic tests").

``rider_kothe`` runs the single-vortex case for one period with classical
RK4 at the kinematic time-step rule and, optionally, the level-set
re-initialisation of the paper's runs (50 pseudo-time iterations every 2000
physical steps); ``advected_droplet`` runs the linear advection of a droplet
for one period (the convergence study of the same section).  Every step runs
in the library's kernels; this module only sequences the calls.
"""

import math

import numpy as np
import torch

from . import dg2p, workloads


def rider_kothe(N, reinit_every=0, reinit_iters=50, time_it=False, order=3, velocity="nodal"):
    """One Rider-Kothe period on N x N elements (see ``run``)."""
    return run("rk2d", N, reinit_every, reinit_iters, time_it, order, velocity)


def advected_droplet(N, order=3, time_it=False, psi="cone", eps=None):
    """One period of the droplet carried by u = (1, 0) on N x N elements
    (fixed eps = 0.05 unless given, Gamma = 1; level set `psi` as in
    workloads.kinematic_config): the L1 error against the initial field and
    the relative mass error."""
    return run("adv2d", N, 0, 0, time_it, order, "nodal", psi, eps)


def run(name, N, reinit_every=0, reinit_iters=50, time_it=False, order=3, velocity="nodal", psi="cone",
        eps=None):
    """One period of the kinematic case `name` (workloads.KIN_NAMES) on N x N
    elements of degree `order` (3 or 1; the re-initialisation, every
    `reinit_every` steps, is p = 3 only).  velocity "nodal": the analytic field
    at the nodes; "stream": the field from the nodal stream function
    (dg2p_kin_velocity_from_stream, discretely divergence free).  Returns a
    dict with the L1 error, the relative mass error, the step count and
    (time_it) the elapsed milliseconds of the whole run."""
    cfg = workloads.kinematic_config(name, n_elem=(N, N), order=order, psi=psi, eps=eps)
    mesh = dg2p.Mesh(2, (N, N), cfg["lo"], cfg["hi"], order=order)
    phi, psi, u0 = workloads.kinematic_fields(cfg, mesh.node_coords())
    kp = dg2p.make_kin_params(**cfg["kin"])
    P = torch.from_numpy(np.ascontiguousarray(np.stack([phi, psi]))).cuda()
    P0 = P[0].clone()
    if velocity == "stream":
        S = torch.from_numpy(np.ascontiguousarray(workloads.kinematic_stream(cfg, mesh.node_coords()))).cuda()
        u0d = dg2p.kin_velocity_from_stream(mesh, S)
    elif velocity == "nodal":
        u0d = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
    else:
        raise ValueError("velocity must be 'nodal' or 'stream'")
    dt0 = float(dg2p.kin_max_dt(mesh, kp, u0d, cfl=cfg["cfl"]).cpu())
    ns = int(math.ceil(cfg["t_end"] / dt0))
    dt = cfg["t_end"] / ns
    nu, dtau = dg2p.kin_reinit_params(mesh) if reinit_every > 0 else (0.0, 0.0)
    e0 = e1 = None
    if time_it:
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
    done = 0
    n_reinit = 0
    while done < ns:
        n = min(reinit_every, ns - done) if reinit_every > 0 else ns
        dg2p.kin_rk4(mesh, kp, P, u0d, n, done * dt, dt)
        done += n
        if reinit_every > 0 and done < ns:
            dg2p.kin_reinit(mesh, kp, P, reinit_iters, nu, dtau)
            n_reinit += 1
    if time_it:
        e1.record()
        torch.cuda.synchronize()
    e = dg2p.kin_errors(mesh, P[0].contiguous(), P0).cpu().tolist()
    out = dict(elements=[N, N], steps=ns, dt=dt, reinit=n_reinit, l1=e[0], mass_error=e[1] / e[2],
               phi_range=[float(P[0].min()), float(P[0].max())])
    if time_it:
        out["ms"] = e0.elapsed_time(e1)
        out["dof"] = 2 * mesh.E * mesh.nn
    return out
