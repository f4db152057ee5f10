"""Build step of libdg2p.so (hipcc, gfx950), in-tree next to the binding.

The library is linked from several objects compiled in parallel: the host
entry points (dg2p.hip), the stage and ingredient kernels once per
(dimension, contraction precision) pair (dg2p_stage_inst.hip with
-DDG2P_DIM / -DDG2P_PR), the kernels of quadrilaterals of degree 4
(dg2p_stage_gen.hip) and the residual VJP kernels once per dimension
(dg2p_vjp_inst.hip).
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
OUT = os.path.join(HERE, "libdg2p.so")
OBJDIR = os.path.join(HERE, "_build")

COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
NOISE = "is not a recognized feature for this target"


def units():
    """(object name, source, extra defines) of every translation unit."""
    u = [("dg2p_host", "dg2p.hip", []), ("stage_gen", "dg2p_stage_gen.hip", [])]
    for d in (1, 2, 3):
        for p in (0, 1, 2):
            u.append((f"stage_d{d}_p{p}", "dg2p_stage_inst.hip", [f"-DDG2P_DIM={d}", f"-DDG2P_PR={p}"]))
        u.append((f"vjp_d{d}", "dg2p_vjp_inst.hip", [f"-DDG2P_DIM={d}"]))
    return u


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if NOISE not in l)
    return res.returncode, err


def _jobs():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 4
    return max(1, min(n, 16))


def build(verbose=False, extra=()):
    """Compile libdg2p.so (always recompiles every object)."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = []
    for name, src, defs in units():
        obj = os.path.join(OBJDIR, name + ".o")
        jobs.append((obj, [HIPCC] + COMMON + list(extra) + defs + ["-c", "-o", obj, os.path.join(CSRC, src)]))
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(lambda j: _run(j[1]), jobs))
    for (obj, cmd), (rc, err) in zip(jobs, results):
        if rc != 0:
            raise RuntimeError(f"hipcc failed ({rc}) on {os.path.basename(obj)}:\n{err}")
        if verbose and err.strip():
            print(err, file=sys.stderr)
    tmp = OUT + ".tmp"
    rc, err = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [j[0] for j in jobs] +
                   ["-lrocprofiler-sdk-roctx"])
    if rc != 0:
        raise RuntimeError(f"link failed ({rc}):\n{err}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
