#!/usr/bin/env python3
"""Benchmark: DOF-updates/s of the DG SSP-RK3 stage on one MI355X.

Headline workload: the 3D heavy-over-light box, 96^3 hexahedra, p = 3,
viscous + CSF + gravity, FP64 (the largest configuration; 3.6 GB per state,
so every stage streams its arrays through HBM).  One step = one pass of the
whole hot path: SSP-RK3's three residual + stage-combine passes, the
time-step reduction and the per-step monitors (alpha range, field integrals,
non-physical count, P/u deviations), run by dg2p_advance_monitored with the
state resident in HBM and no host synchronisation inside the timed region.
value = 3 * N_nodes * N_fields / (seconds per step).

The JSON line also carries
  roofline:     algorithmic bytes of the stage kernel per launch (21.33 B per
                DOF per stage, averaged over the three stages: stage 1 reads
                U^n and writes U^1, stages 2 and 3 read U^n and U^s and write
                U^{s+1}) divided by its mean launch duration, measured with
                hipEvents the library records around its own launches on the
                launch stream during the timed region; HBM peak 8 TB/s.
                `traffic` is the counter-measured HBM traffic per launch
                recorded under profiles/ for the current kernel sources (null
                if the sources changed since).  Beside it: the bandwidth of a
                plain device copy and the FP64 vector FMA rate, both measured
                in the same run (dg2p_calibrate_fp64_fma).
  mixed_precision: FP32 and BF16 contraction forms on the 512 x 256 shock
                (200 steps) and the 96^3 box (100 steps): per-field L2 / Linf
                error against the FP64 path and speed.
  cache_resident_2d: the 128^2 droplet (its ~60 MB working set stays in the
                256 MB Infinity Cache, so its fraction is fabric bandwidth,
                not HBM).
  cpu_baseline: the FP64 CPU oracle's residual on a bounded sample of the
                headline workload, with one thread and with every core of the
                host (core count from os.sched_getaffinity).

--gpus N with N > 1 is refused: this build runs on one GPU.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD_DESC = {
    "drop1d": "1D periodic air/water slab, 100 elements, p=3, FP64",
    "drop2d": "2D periodic water droplet in air, 128x128 quads, p=3, FP64",
    "shock2d": "2D shock onto water cylinder, 512x256 quads, p=3, FP64",
    "rt3d": "3D heavy-over-light box, 96^3 hexahedra, p=3, viscous + CSF + gravity, FP64",
    "adjoint2d": "2D droplet 128x128 p=3, viscous + CSF, FP64 forward",
    "waterair2d": "2D water droplet in air (density ratio 1000, P_inf 6000), 24x24 quads, p=3, FP64",
    "bubble2d": "2D rising bubble, 20x40 quads, p=3, rho/mu ratio 10, Re 35, Eo 10, no-slip bottom, "
                "Riemann top, slip sides, FP64",
    "rt2d": "2D Rayleigh-Taylor, 20x80 quads, p=3, At 0.5, Re 3000, no-slip bottom, Riemann top, slip sides, FP64",
}

# default timed steps per workload: about 50 ms of GPU time on one MI355X, long
# enough for the clocks to settle and the event timing to be stable
DEFAULT_STEPS = {"drop1d": 2000, "drop2d": 1000, "shock2d": 200, "rt3d": 20, "adjoint2d": 1000,
                 "waterair2d": 2000, "bubble2d": 2000, "rt2d": 1000}
HEADLINE = "rt3d"
# the 2D wall-bounded workloads at p = 4: grids of the p = 3 grids' node count
P4_GRIDS = {"bubble2d": (16, 32), "rt2d": (16, 64)}
# workloads whose working set exceeds the 256 MB Infinity Cache (HBM-bound)
HBM_RESIDENT = {"shock2d", "rt3d"}


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2306_05002_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded(workload, what, key, src_hash):
    """A figure from a committed counter summary profiles/k_stage_<workload>_<what>.md,
    if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"k_stage_{workload}_{what}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != src_hash:
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


# a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles; 1024 SIMDs at 2.4 GHz
VALU_ISSUE_PER_S = 1024 * 2.4e9 / 4
# FP64 vector FMA at that issue rate: 1024 SIMDs x 16 lanes x 2 flop x 2.4 GHz
FP64_VFMA_NOMINAL_TFLOPS = 1024 * 16 * 2 * 2.4e9 / 1e12


def oracle_state(cfg, pf):
    """The oracle's mesh, parameters and initial state from the primitive
    fields (the oracle's own initial-condition map)."""
    import numpy as np
    import torch
    import oracle

    prm = oracle.Params(**cfg["params"])
    d = cfg["dim"]
    bc_state = {}
    for key, bp in cfg.get("bc_prim", {}).items():
        t = lambda v: torch.tensor([float(v)], dtype=torch.float64)
        Qb = oracle.prim_to_cons(t(bp["alpha"]), t(bp["psi"]), t(bp["rho1"]), t(bp["rho2"]),
                                 torch.tensor(bp["u"][:d], dtype=torch.float64)[:, None],
                                 t(bp["P"]), prm)
        bc_state[key] = Qb[:, 0]
    om = oracle.OracleMesh(d, cfg["order"], cfg["n_elem"], cfg["lo"], cfg["hi"], cfg["bc"], bc_state)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)
    U = oracle.prim_to_cons(T(pf["alpha"]), T(pf["psi"]), T(pf["rho1"]), T(pf["rho2"]),
                            T(pf["u"]), T(pf["P"]), prm)
    return om, prm, U


def cpu_baseline(cfg, pf, seconds):
    """FP64 oracle residual evaluations on the host over a bounded sample of
    the workload (at most 4096 consecutive elements from the middle of the
    grid, whose faces reach into the rest of it), about `seconds` per thread
    count, with one thread and with every core the process may run on."""
    import torch
    import oracle

    om, prm, U = oracle_state(cfg, pf)
    n_s = min(om.E, 4096)
    lo = (om.E - n_s) // 2
    el = torch.arange(lo, lo + n_s)
    cores = len(os.sched_getaffinity(0))
    dof = n_s * om.nn * om.nf
    rates = {}
    for nt in (1, cores):
        torch.set_num_threads(nt)
        oracle.rhs(U, om, prm, elems=el)
        reps, t0 = 0, time.perf_counter()
        while True:
            oracle.rhs(U, om, prm, elems=el)
            reps += 1
            el_t = time.perf_counter() - t0
            if el_t >= seconds or reps >= 200:
                break
        rates[nt] = (dof * reps / el_t, reps, el_t)
    sample = (f"oracle residual (one RK stage's work) on elements {lo}..{lo + n_s - 1} of {om.E}; "
              f"{rates[cores][1]} evaluations in {rates[cores][2]:.1f} s with {cores} threads, "
              f"{rates[1][1]} in {rates[1][2]:.1f} s with 1 thread")
    return dict(value=rates[cores][0], unit="DOF-updates/s", cores=cores, kind="oracle", sample=sample,
                value_1_thread=rates[1][0], threads=[1, cores])


# L1 errors of the paper's Rider-Kothe table (quadrilateral mesh, p = 3) at
# 64^2, 128^2, 256^2 degrees of freedom, i.e. 16^2, 32^2, 64^2 elements
PAPER_RK_L1_P3 = {16: 1.75e-2, 32: 4.83e-3, 64: 1.23e-3}
PAPER_RK_L1_P1 = {32: 2.22e-2, 64: 8.71e-3, 128: 3.31e-3}


def kinematic_section():
    """Rider-Kothe single vortex, one full period, classical RK4, on the
    library's kinematic mode at the paper's six cells (64^2, 128^2, 256^2
    nodes at p = 3 and p = 1): L1 error and relative mass error with the
    nodal analytic velocity, the same with the stream-function velocity
    (discretely divergence free), at p = 3 also with the level-set
    re-initialisation (50 pseudo-time iterations every 2000 steps), and the
    kinematic stage throughput."""
    from paper_2306_05002_amd import kinematic
    rows = []
    for order, table in ((3, PAPER_RK_L1_P3), (1, PAPER_RK_L1_P1)):
        for N in sorted(table):
            r0 = kinematic.rider_kothe(N, time_it=True, order=order)
            rs = kinematic.rider_kothe(N, order=order, velocity="stream")
            row = {"order": order, "elements": [N, N], "dof": f"{(order + 1) * N}^2", "steps": r0["steps"],
                   "l1": r0["l1"], "l1_paper": table[N], "mass_error": r0["mass_error"],
                   "l1_stream_velocity": rs["l1"], "mass_error_stream_velocity": rs["mass_error"]}
            if order == 3:
                r1 = kinematic.rider_kothe(N, reinit_every=2000, order=order)
                row.update(l1_reinit=r1["l1"], mass_error_reinit=r1["mass_error"], reinit_calls=r1["reinit"])
            row.update(ms_per_step=r0["ms"] / r0["steps"], value=4.0 * r0["dof"] * r0["steps"] / (r0["ms"] * 1e-3))
            rows.append(row)
    adv = {}
    for psi, eps in (("cone", 0.05), ("smooth", 0.025)):
        for order, Ns in ((3, (8, 16, 32, 64)), (1, (16, 32, 64, 128))):
            errs = [kinematic.advected_droplet(N, order=order, psi=psi, eps=eps) for N in Ns]
            l1 = [r["l1"] for r in errs]
            adv[f"p{order}_{psi}_psi_eps{eps}"] = {
                "elements": list(Ns), "l1": l1, "mass_error": [r["mass_error"] for r in errs],
                "order": [math.log2(l1[i] / l1[i + 1]) for i in range(len(l1) - 1)]}
    return {"workload": "rk2d: Rider-Kothe vortex, [0,1]^2 periodic, p=3 and p=1, eps=2h/(p+1), Gamma=1, T=4, "
                        "RK4, CFL 0.1",
            "unit": "DOF-updates/s", "runs": rows,
            "linear_advection": {"workload": "adv2d: droplet R=0.15 carried by u=(1,0) for one period, [0,1]^2 "
                                             "periodic, Gamma=1, RK4, CFL 0.1; the paper's set-up (level set "
                                             "psi = R - r, eps = 0.05 fixed) and a smooth level set "
                                             "(R^2 - r^2)/(2R) with eps = 0.025",
                                 "runs": adv}}


def waterair_section():
    """The paper's water droplet in air (24 x 24, p = 3, density ratio 1000,
    P_inf 6000, u = (5, 5)) for five advection periods with a fixed step, in
    FP64 and the two mixed forms: interface equilibrium (max |P - 1|,
    max |u - (5, 5)|), the droplet's shape (L1 of alpha against the initial
    field, which it should return to) and throughput."""
    import torch
    from paper_2306_05002_amd import dg2p, workloads
    cfg = workloads.config("waterair2d")
    P64 = dg2p.make_params(cfg["params"])
    mesh = dg2p.mesh_from_config(cfg, P64)
    U0 = dg2p.prim_to_cons(mesh, P64, dg2p.prim_tensor(
        workloads.primitive_fields(cfg, mesh.node_coords()), cfg["dim"]))
    dt0 = float(dg2p.max_dt(mesh, P64, U0, cfl=0.1).cpu())
    ns = int(math.ceil(cfg["t_end"] / dt0))
    dtf = torch.tensor([cfg["t_end"] / ns], dtype=torch.float64, device="cuda")
    a0 = U0[3 + cfg["dim"]].contiguous()
    dof = mesh.E * mesh.nn * mesh.nf
    runs = {}
    for prec in ("fp64", "fp32", "bf16"):
        Pm = dg2p.make_params(cfg["params"], precision=prec)
        U = U0.clone()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        dg2p.advance(mesh, Pm, U, ns, dt_fixed=dtf)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        m = dg2p.monitors(mesh, P64, U, p_ref=1.0, u_ref=[5.0, 5.0])
        e = dg2p.kin_errors(mesh, U[3 + cfg["dim"]].contiguous(), a0).cpu().tolist()
        runs[prec] = {"dev_p": m["dev_p"], "dev_u": m["dev_u"], "nonphys": m["nonphys"],
                      "alpha_range": [m["min_alpha"], m["max_alpha"]],
                      "alpha_l1_vs_initial": e[0], "alpha_mass_error": e[1] / e[2],
                      "ms_per_step": ms / ns, "value": 3.0 * dof * ns / (ms * 1e-3)}
    return {"workload": "waterair2d: water droplet R=25/89 in air, 24x24 p=3, rho 1e-3/1, P_inf 0/6000, "
                        "u=(5,5), eps=h/2, Gamma=5, five periods (t=1), fixed dt",
            "steps": ns, "unit": "DOF-updates/s", "runs": runs}


def walls_section():
    """The paper's two wall-bounded cases with the no-slip bottom, the
    Riemann-invariant top (zero velocity, constant pressure) and slip sides,
    run to their final times in FP64 with the device time step (qualitative:
    the comparison curves are not reproduced here).  Rising bubble: centre of
    gravity and mean rise velocity of the bubble; Rayleigh-Taylor: the highest
    point of the light fluid and the lowest of the heavy fluid (nodal
    alpha = 1/2 crossings), against t* = t / sqrt(d / (|g| At))."""
    import torch
    from paper_2306_05002_amd import dg2p, workloads
    out = {}
    # (name, degree, elements, CFL): the p = 3 grids and p = 4 grids of the
    # same node count; at p = 4 the time-step rule needs CFL 0.05 (at 0.1 the
    # diffusive part of the p = 4 operator outgrows the (p+1)^2 factor of the
    # rule and the run diverges)
    for name, order, ne, cfl in (("bubble2d", 3, None, 0.1), ("rt2d", 3, None, 0.1),
                                 ("bubble2d", 4, (16, 32), 0.05), ("rt2d", 4, (16, 64), 0.05)):
        cfg = workloads.config(name, n_elem=ne, order=order)
        P = dg2p.make_params(cfg["params"])
        mesh = dg2p.mesh_from_config(cfg, P)
        X = mesh.node_coords()
        U = dg2p.prim_to_cons(mesh, P, dg2p.prim_tensor(workloads.primitive_fields(cfg, X), 2))
        W = torch.tensor(mesh.node_weights(), device="cuda")
        y = torch.tensor(X[1], device="cuda")
        dof = mesh.E * mesh.nn * mesh.nf
        t = torch.zeros(1, dtype=torch.float64, device="cuda")
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        mon = torch.zeros(dg2p.MONITOR_DOUBLES, dtype=torch.float64, device="cuda")
        t_scale = 1.0 if name == "bubble2d" else math.sqrt(2.0)     # t* = t / sqrt(d / (|g| At))
        dt0 = None
        marks = [0.5 * i for i in range(1, 7)]
        rows, steps, ms = [], 0, 0.0
        chunk = 250
        while float(t.cpu()) < cfg["t_end"] * (1.0 - 1e-12):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            dg2p.advance(mesh, P, U, chunk, cfl=cfl, t=t, dt_last=dt, mon=mon)
            e1.record()
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
            steps += chunk
            tn = float(t.cpu())
            dtn = float(dt.cpu())
            dt0 = dtn if dt0 is None else dt0
            if (steps >= 200000 or not math.isfinite(tn) or not dtn > 1e-2 * dt0
                    or dg2p.decode_monitors(mon, mesh.nf)["nonphys"]):
                # the time step collapsed or a state left the physical domain
                rows.append({"stopped_at_t": tn, "steps": steps, "dt": dtn, "dt_initial": dt0})
                break
            if not marks or tn / t_scale < marks[0]:
                continue
            while marks and tn / t_scale >= marks[0]:
                marks.pop(0)
            m = dg2p.decode_monitors(mon, mesh.nf)
            a = U[5]
            if name == "bubble2d":
                b = (1.0 - a) * W
                rho = U[0] + U[1]
                rows.append({"t": tn, "y_c": float((b * y).sum() / b.sum()),
                             "v_c": float((b * U[3] / rho).sum() / b.sum()), "nonphys": m["nonphys"]})
            else:
                light = a > 0.5
                rows.append({"t_star": tn / t_scale, "top": float(y[light].max()),
                             "bottom": float(y[~light].min()), "nonphys": m["nonphys"],
                             "min_partial_density": [float(U[0].min()), float(U[1].min())]})
        key = name if order == 3 else f"{name}_p{order}"
        desc = WORKLOAD_DESC[name] if order == 3 else (
            f"{name} at p=4 on {cfg['n_elem'][0]}x{cfg['n_elem'][1]} quads (the p=3 grid's node count), "
            f"eps=h/2, CFL {cfl}")
        out[key] = {"workload": f"{name}: {desc}", "steps": steps, "series": rows,
                    "ms_per_step": ms / steps, "value": 3.0 * dof * steps / (ms * 1e-3),
                    "unit": "DOF-updates/s"}
    return out


# steps after which the mixed-precision forms' field errors are stated
ERROR_STEPS = {"shock2d": 200, "rt3d": 100}


def field_errors(Ua, Ub, Wn, d, n_steps):
    """Per-field relative errors of state Ua against Ub (fields in state order):
    W-weighted L2, sqrt(sum W (a-b)^2 / sum W b^2), and Linf, max|a-b| / max|b|,
    where for the momentum components b stands for the whole momentum vector
    (sum over components in L2, largest component in Linf): a transverse
    momentum may vanish identically."""
    import torch
    W = Wn.reshape(1, 1, -1)
    diff = (Ua - Ub)
    den = (Ub * Ub * W).sum(dim=(1, 2))
    den[2:2 + d] = den[2:2 + d].sum()
    l2 = torch.sqrt((diff * diff * W).sum(dim=(1, 2)) / den.clamp_min(1e-300))
    amax = Ub.abs().amax(dim=(1, 2))
    mom = float(amax[2:2 + d].max())
    scale = amax.clone()
    scale[2:2 + d] = mom
    linf = diff.abs().amax(dim=(1, 2)) / scale.clamp_min(1e-300)
    return {"after_steps": n_steps, "l2_rel": [float(x) for x in l2], "linf_rel": [float(x) for x in linf]}


def copy_bandwidth(gib=2.0, reps=10):
    """Achieved HBM bandwidth of a plain device copy (torch's copy kernel,
    `gib` GiB read and written per launch, well beyond the 256 MB Infinity
    Cache): bytes moved / mean launch time, HIP events on the current
    stream.  Context for the roofline fraction: what a streaming kernel with
    no arithmetic reaches on this GPU."""
    import torch
    n = int(gib * (1 << 30) / 8)
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return 2.0 * n * 8 / (ms * 1e-3) / 1e9


def calibrate_copy(gib=2.0, reps=10):
    """Plain copy kernel of known size (reads and writes `gib` GiB) for
    scaling the HBM counters of the profiler."""
    import torch
    n = int(gib * (1 << 30) / 8)
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": n * 8, "bytes_written": n * 8, "launches": reps}))


def initial_state(cfg, mesh, P):
    """Primitive fields of the workload at the mesh's nodes (host) and the
    conserved initial state on the GPU (the library's initial-condition map)."""
    from paper_2306_05002_amd import dg2p, workloads
    pf = workloads.primitive_fields(cfg, mesh.node_coords())
    U0 = dg2p.prim_to_cons(mesh, P, dg2p.prim_tensor(pf, cfg["dim"]))
    return pf, U0


def stage_timing(dg2p, n_steps, ms_step):
    """Per-launch means of the kernel kinds recorded by the library while its
    timing was enabled, and the stage kernel's mean."""
    k_ms = {}
    for name, kind in (("stage", dg2p.K_STAGE), ("ingredients", dg2p.K_INGREDIENTS),
                       ("rate", dg2p.K_RATE), ("rate_final", dg2p.K_RATE_FINAL)):
        k_ms[name] = dg2p.timing_read(kind)
    # the step less the other kernels' share, over its three stage launches
    other = sum(k_ms[k][0] * k_ms[k][1] for k in ("ingredients", "rate", "rate_final")) / n_steps
    return k_ms, (ms_step - other) / 3.0


def timed_steps(mesh, P, U, steps, warmup, cfl, monitored=True, events=False):
    """warmup untimed steps, then `steps` timed steps (CUDA events around the
    batch on the current stream; with events=True the library also records
    its per-launch hipEvents during the timed batch).  Returns ms per step,
    the per-step monitors of the timed steps (or None) and the wall time."""
    import torch
    from paper_2306_05002_amd import dg2p
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    ms = torch.zeros(max(steps, warmup, 1), dg2p.MONITOR_DOUBLES, dtype=torch.float64, device="cuda")

    def run(n):
        if monitored:
            dg2p.advance_monitored(mesh, P, U, n, ms, cfl=cfl, t=t, dt_last=dt, p_ref=1.0)
        else:
            dg2p.advance(mesh, P, U, n, cfl=cfl, t=t, dt_last=dt)

    run(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    if events:
        dg2p.timing_enable(True)
    t0 = time.perf_counter()
    e0.record(stream)
    run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if events:
        dg2p.timing_enable(False)
    mon = dg2p.decode_monitors(ms[:steps], mesh.nf) if monitored else None
    return e0.elapsed_time(e1) / steps, mon, wall


def roofline(workload, dof, stage_ms, event_ms, src):
    alg_bytes = (64.0 / 3.0) * dof          # per stage launch, averaged over the 3 stages
    achieved = alg_bytes / (event_ms * 1e-3) / 1e9
    traffic = recorded(workload, "traffic", "traffic_bytes_per_launch", src)
    valu = recorded(workload, "valu", "valu_insts_per_launch", src)
    return {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "kernel": "k_stage (residual + stage combine)",
        "kernel_mean_ms": event_ms,
        "kernel_mean_ms_from_step": stage_ms,
        "valu_issue": None if valu is None else {
            "insts_per_launch": valu,
            "issue_ms": valu / VALU_ISSUE_PER_S * 1e3,
            "frac": valu / VALU_ISSUE_PER_S * 1e3 / event_ms},
        "algorithmic_bytes_per_launch": alg_bytes,
    }


def mixed_section(name, U0=None, mesh=None, steps=20, warmup=5, cfl=0.1):
    """FP32 and BF16 contraction forms of one workload: per-field error
    against the FP64 path after the workload's error horizon (same initial
    state, same fixed dt: that of the initial state) and speed."""
    import torch
    from paper_2306_05002_amd import dg2p, workloads
    cfg = workloads.config(name)
    P64 = dg2p.make_params(cfg["params"])
    if mesh is None:
        mesh = dg2p.mesh_from_config(cfg, P64)
        U0 = initial_state(cfg, mesh, P64)[1]
    dof = mesh.E * mesh.nn * mesh.nf
    n_err = ERROR_STEPS[name]
    dt0 = dg2p.max_dt(mesh, P64, U0, cfl=cfl)
    Uref = U0.clone()
    dg2p.advance(mesh, P64, Uref, n_err, dt_fixed=dt0)
    Wn = torch.from_numpy(mesh.node_weights()).cuda()
    out = {"workload": f"{name}: {WORKLOAD_DESC[name]}", "error_steps": n_err,
           "error_reference": "FP64 GPU path (itself within 1e-12 of the oracle), same fixed dt"}
    U = U0.clone()
    ms64, _, _ = timed_steps(mesh, P64, U, steps, warmup, cfl, monitored=True)
    out["fp64"] = {"value": 3.0 * dof / (ms64 * 1e-3), "ms_per_step": ms64}
    for prec in ("fp32", "bf16"):
        Pm = dg2p.make_params(cfg["params"], precision=prec)
        Ue = U0.clone()
        dg2p.advance(mesh, Pm, Ue, n_err, dt_fixed=dt0)
        err = field_errors(Ue, Uref, Wn, cfg["dim"], n_err)
        m = dg2p.monitors(mesh, P64, Ue)
        del Ue
        U = U0.clone()
        msm, _, _ = timed_steps(mesh, Pm, U, steps, warmup, cfl, monitored=True)
        out[prec] = {"error_vs_fp64": err, "nonphys_after": m["nonphys"],
                     "value": 3.0 * dof / (msm * 1e-3), "ms_per_step": msm, "speedup_vs_fp64": ms64 / msm,
                     "contractions": prec, "closure_and_rk": "fp64"}
    del Uref, U
    return out


def cache_resident_section(src, cfl=0.1):
    """The 128 x 128 droplet (FP64): its ~60 MB working set stays in the
    Infinity Cache, so the bandwidth figure is fabric traffic, not HBM."""
    from paper_2306_05002_amd import dg2p, workloads
    name = "drop2d"
    cfg = workloads.config(name)
    P = dg2p.make_params(cfg["params"])
    mesh = dg2p.mesh_from_config(cfg, P)
    U = initial_state(cfg, mesh, P)[1]
    dof = mesh.E * mesh.nn * mesh.nf
    steps = DEFAULT_STEPS[name]
    msd, _, _ = timed_steps(mesh, P, U, steps, steps // 4, cfl, monitored=False)
    ms_mon, _, _ = timed_steps(mesh, P, U, steps, steps // 4, cfl, monitored=True)
    # the per-launch event pairs cost microseconds per launch, a large share
    # of a step this short: a separate run records them for the kernel figures
    ms_ev, _, _ = timed_steps(mesh, P, U, steps, steps // 4, cfl, monitored=True, events=True)
    k_ms, stage_ms = stage_timing(dg2p, steps, ms_ev)
    rl = roofline(name, dof, stage_ms, stage_ms, src)
    rl["bound"] = "infinity-cache resident (fabric, not HBM)"
    return {"workload": f"{name}: {WORKLOAD_DESC[name]}", "value": 3.0 * dof / (msd * 1e-3),
            "ms_per_step": msd, "step": "dg2p_advance (dt fused into the first stage, no per-step monitors)",
            "value_with_step_monitors": 3.0 * dof / (ms_mon * 1e-3), "ms_per_step_with_step_monitors": ms_mon,
            "step_with_step_monitors": "dg2p_advance_monitored (dt and the monitors reduced in the next "
                                       "step's first stage)",
            "ms_per_step_with_step_monitors_and_launch_events": ms_ev,
            "roofline_cache": rl}


def adjoint_section(steps):
    """VJP of one SSP-RK3 step on the adjoint workload (viscous + CSF droplet,
    128 x 128, frozen dt), and central-difference agreement of the gradient
    of the 400-step rollout."""
    import torch
    from paper_2306_05002_amd import dg2p
    from paper_2306_05002_amd import adjoint as adj
    prob = adj.AdjointProblem()
    Ua = dg2p.prim_to_cons(prob.mesh, prob.P, prob.prim0)
    Wb = torch.randn(Ua.shape, dtype=torch.float64, device="cuda",
                     generator=torch.Generator(device="cuda").manual_seed(0))
    Ub = torch.empty_like(Ua)
    sb = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        dg2p.rk_step_vjp(prob.mesh, prob.P, Ua, prob.dt, Wb, param_bar=sb, out=Ub)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    n_adj = max(5, min(steps, 50))
    e0.record(stream)
    for _ in range(n_adj):
        dg2p.rk_step_vjp(prob.mesh, prob.P, Ua, prob.dt, Wb, param_bar=sb, out=Ub)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_vjp = e0.elapsed_time(e1) / n_adj
    dof_a = prob.mesh.E * prob.mesh.nn * prob.mesh.nf
    L0, gu, gs = prob.gradient()
    worst = 0.0
    h = 1e-6
    for k in range(16):
        du, ds = prob.fd_directions(k)
        with torch.no_grad():
            Lp = float(prob.loss(prob.u0 + h * du, prob.sigma0 + h * ds))
            Lm = float(prob.loss(prob.u0 - h * du, prob.sigma0 - h * ds))
        fd = (Lp - Lm) / (2 * h)
        ad = float((gu * du).sum()) + gs * ds
        worst = max(worst, abs(fd - ad) / max(abs(fd), abs(ad), 1e-300))
    return {"workload": "adjoint2d: droplet 128x128 p=3, viscous + CSF, 400 steps, checkpoint every 20",
            "value": 3.0 * dof_a / (ms_vjp * 1e-3), "unit": "DOF-updates/s",
            "ms_per_step_vjp": ms_vjp,
            "step_vjp": "recompute 2 stages + 3 residual VJPs (local + gather)",
            "fd_directions": 16, "fd_step": h, "fd_max_rel_err": worst,
            "dL_dsigma": gs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: about 50 ms of GPU time for the workload, 20 on the 96^3 box)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps before the timed region (default: a quarter of --steps, at least 10)")
    ap.add_argument("--workload", default=HEADLINE, choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--order", type=int, default=3, choices=(3, 4),
                    help="polynomial degree; 4: the 2D wall-bounded workloads on their p = 4 grids")
    ap.add_argument("--cfl", type=float, default=None, help="CFL number (default 0.1; 0.05 at p = 4)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="oracle timing per thread count (one thread, then every core)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the mixed-precision, cache-resident, adjoint, kinematic, water-air and "
                         "wall-bounded measurements")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = DEFAULT_STEPS[args.workload]
    if args.warmup is None:
        args.warmup = max(10, args.steps // 4)
    if args.order == 4 and args.workload not in P4_GRIDS:
        print("bench.py: --order 4 runs the 2D wall-bounded workloads only (%s)" % ", ".join(sorted(P4_GRIDS)),
              file=sys.stderr)
        sys.exit(2)
    if args.cfl is None:
        args.cfl = 0.05 if args.order == 4 else 0.1

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); no multi-GPU path exists",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return

    import torch
    from paper_2306_05002_amd import dg2p, workloads

    if args.order == 4:
        cfg = workloads.config(args.workload, n_elem=P4_GRIDS[args.workload], order=4)
        desc = "%s at p=4 on %dx%d quads, eps=h/2, CFL %g" % (args.workload, *cfg["n_elem"], args.cfl)
    else:
        cfg = workloads.config(args.workload)
        desc = WORKLOAD_DESC[args.workload]
    P = dg2p.make_params(cfg["params"])
    mesh = dg2p.mesh_from_config(cfg, P)
    pf, U0 = initial_state(cfg, mesh, P)
    U = U0.clone()
    n_nodes = mesh.E * mesh.nn
    dof = n_nodes * mesh.nf
    src = source_hash()

    # headline: the whole step (three stages, dt reduction, per-step monitors),
    # the library's per-launch events recorded on its launch stream.  On the
    # small grids an event pair is a large share of a launch: there the step
    # is timed without them and a second run records them for the kernel
    # figures.
    ms_step, mon_rows, wall = timed_steps(mesh, P, U, args.steps, args.warmup, args.cfl,
                                          monitored=True, events=args.workload in HBM_RESIDENT)
    ms_ev = ms_step
    if args.workload not in HBM_RESIDENT:
        ms_ev = timed_steps(mesh, P, U, args.steps, args.warmup, args.cfl, monitored=True, events=True)[0]
    value = 3.0 * dof / (ms_step * 1e-3)
    k_ms, stage_ms = stage_timing(dg2p, args.steps, ms_ev)
    # (counter summaries under profiles/ are keyed by workload, and degree when not 3)
    prof_key = args.workload if args.order == 3 else "%s_p%d" % (args.workload, args.order)
    rl = roofline(prof_key, dof, stage_ms, k_ms["stage"][0], src)
    if args.workload not in HBM_RESIDENT:
        rl["bound"] = "infinity-cache resident (fabric, not HBM)"
        rl["ms_per_step_with_launch_events"] = ms_ev
    else:
        cbw = copy_bandwidth()
        rl["copy_kernel_gbs"] = cbw
        rl["frac_of_copy_kernel"] = rl["achieved"] / cbw
        if rl["traffic"] is not None:
            rl["traffic_gbs"] = rl["traffic"] / (rl["kernel_mean_ms"] * 1e-3) / 1e9
    # the FP64 FMA rate this GPU sustains (the VALU issue fraction assumes the
    # nominal 2.4 GHz; a lower measured rate means a lower sustained clock)
    fma = dg2p.calibrate_fp64_fma()
    rl["fp64_vfma_tflops_measured"] = fma
    if rl["valu_issue"] is not None:
        rl["valu_issue"]["frac_at_measured_fma_rate"] = rl["valu_issue"]["frac"] * FP64_VFMA_NOMINAL_TFLOPS / fma
    last = mon_rows[-1]
    monitors = {"per_step": True, "steps_with_nonphys": sum(1 for r in mon_rows if r["nonphys"]),
                "last_step": {"nonphys": last["nonphys"], "min_alpha": last["min_alpha"],
                              "max_alpha": last["max_alpha"], "dt": last["dt"], "dev_p": last["dev_p"],
                              "integral": last["integral"]}}
    del U

    variants = {}
    extra = {}
    if not args.no_variants:
        for name in ("shock2d", "rt3d"):
            if name == args.workload:
                variants[name] = mixed_section(name, U0=U0, mesh=mesh, steps=args.steps, warmup=args.warmup,
                                               cfl=args.cfl)
            else:
                variants[name] = mixed_section(name, steps=DEFAULT_STEPS[name], warmup=DEFAULT_STEPS[name] // 4,
                                               cfl=args.cfl)
            torch.cuda.empty_cache()
    del U0
    torch.cuda.empty_cache()
    if not args.no_variants:
        extra["cache_resident_2d"] = cache_resident_section(src, args.cfl)
        extra["adjoint"] = adjoint_section(args.steps)
        extra["kinematic"] = kinematic_section()
        extra["water_air_droplet"] = waterair_section()
        extra["wall_bounded"] = walls_section()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, pf, args.cpu_seconds)
    del pf

    out = {
        "metric": "DOF-updates/s of DG RK stage, FP64 vs mixed vs adjoint, at stated error",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {desc}",
            "n_elem": list(cfg["n_elem"]),
            "order": cfg["order"],
            "nodes": n_nodes,
            "fields": mesh.nf,
            "dof": dof,
            "precision": "fp64",
            "step": "SSP-RK3 (3 stages) + device dt reduction + per-step monitors, dg2p_advance_monitored",
        },
        "roofline": rl,
        "kernels_mean_ms": {k: v[0] for k, v in k_ms.items()},
        "monitors": monitors,
        "mixed_precision": variants,
        **extra,
        "cpu_baseline": cpu,
        "wall_s_timed": wall,
        "source_sha256_16": src,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
