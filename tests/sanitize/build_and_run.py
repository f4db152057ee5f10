"""Host-sanitised build of libdg2p and its C-ABI host check.

The library's host code (the entry points, mesh and workspace logic in
dg2p.hip) is compiled with AddressSanitizer and UndefinedBehaviorSanitizer
(host pass only, `-Xarch_host` before each flag; its device code as in the
product build); the other translation units as in the product build.  The
C driver abi_host_check.c is compiled and linked with the same sanitizers
(clang from the ROCm toolchain, whose runtime the library's instrumented code
expects) and run; it needs no GPU.  Returns the driver's exit status.

    python tests/sanitize/build_and_run.py [outdir]
"""

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, os.path.join(ROOT, "paper_2306_05002_amd"))
import build  # noqa: E402  (the library's own list of translation units)

HIPCC = build.HIPCC
CLANG = os.environ.get("DG2P_SAN_CLANG", "/opt/rocm/llvm/bin/clang")
CLANGXX = os.environ.get("DG2P_SAN_CLANGXX", "/opt/rocm/llvm/bin/clang++")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def run(cmd, env=None):
    res = subprocess.run(cmd, capture_output=True, text=True, env=env)
    if res.returncode != 0:
        err = "\n".join(l for l in res.stderr.splitlines() if build.NOISE not in l)
        raise RuntimeError(f"{' '.join(cmd[:3])} ... failed ({res.returncode}):\n{err}\n{res.stdout}")
    return res


def build_and_run(outdir):
    from concurrent.futures import ThreadPoolExecutor
    jobs = []
    for name, src, defs in build.units():
        obj = os.path.join(outdir, name + ".o")
        extra = SAN + ["-g"] if src == "dg2p.hip" else []
        jobs.append((obj, [HIPCC] + build.COMMON + extra + defs + ["-c", "-o", obj, os.path.join(build.CSRC, src)]))
    with ThreadPoolExecutor(max_workers=build._jobs()) as ex:
        list(ex.map(lambda j: run(j[1]), jobs))
    lib = os.path.join(outdir, "libdg2p_hostsan.so")
    run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib] + [j[0] for j in jobs] +
        ["-lrocprofiler-sdk-roctx"])
    drv_o = os.path.join(outdir, "abi_host_check.o")
    exe = os.path.join(outdir, "abi_host_check")
    run([CLANG, "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-g", "-O1", "-c",
         "-o", drv_o, os.path.join(HERE, "abi_host_check.c")])
    run([CLANGXX, "-fsanitize=address,undefined", "-o", exe, drv_o, lib, "-Wl,-rpath," + outdir,
         "-Wl,-rpath,/opt/rocm/lib"])
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    res = subprocess.run([exe], capture_output=True, text=True, env=env)
    sys.stdout.write(res.stdout)
    sys.stderr.write(res.stderr)
    return res.returncode


if __name__ == "__main__":
    if len(sys.argv) > 1:
        os.makedirs(sys.argv[1], exist_ok=True)
        sys.exit(build_and_run(sys.argv[1]))
    with tempfile.TemporaryDirectory() as d:
        sys.exit(build_and_run(d))
