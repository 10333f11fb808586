"""Build libpa.so (the HIP kernels and the C ABI) in place for gfx950.

hipcc cross-compiles without a GPU.  Host code is compiled with
-ffp-contract=off so that the double-precision reweighting tables are the
plain IEEE operations written in the source; device code is compiled with
packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
SO = os.path.join(HERE, "libpa.so")
# the vector-ALU issue-rate probe, a measuring instrument of the benchmark
PROBE_SO = os.path.join(HERE, "libpa_probe.so")
PROBE_SOURCE = "pa_probe.hip"
SOURCES = ["pa_kernels.hip", "pa_tables.hip", "pa_api.hip", "pa_batch.hip",
           "pa_mlp.hip", "pa_potts.hip"]
ARCH = os.environ.get("PA_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found: cannot build libpa.so")
    return p


def _flags() -> list:
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-ffp-contract=off", "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC]


def build(verbose: bool = False) -> str:
    """Compile libpa.so (always recompiles) and return its path.  Each
    source is compiled to an object of its own in parallel, then linked."""
    from concurrent.futures import ThreadPoolExecutor
    tag = "%d" % os.getpid()
    objs = [os.path.join(HERE, "_obj_%s_%s.o" % (os.path.splitext(s)[0], tag))
            for s in SOURCES]
    cmds = [[hipcc()] + _flags() + ["-c", "-o", o, os.path.join(CSRC, s)]
            for s, o in zip(SOURCES, objs)]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "0") or 0)
                      or (os.cpu_count() or 1)))
    try:
        with ThreadPoolExecutor(jobs) as ex:
            res = list(ex.map(lambda c: subprocess.run(
                c, capture_output=True, text=True, cwd=ROOT), cmds))
        for r in res:
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError("hipcc failed building libpa.so")
        tmp = SO + ".tmp" + tag
        link = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o",
                tmp] + objs
        r = subprocess.run(link, capture_output=True, text=True, cwd=ROOT)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libpa.so")
        os.replace(tmp, SO)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    build_probe(verbose)
    return SO


def build_probe(verbose: bool = False) -> str:
    """Compile libpa_probe.so (always recompiles) and return its path."""
    tmp = PROBE_SO + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + _flags() + ["-shared", "-o", tmp,
                                  os.path.join(CSRC, PROBE_SOURCE)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=ROOT)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        if os.path.exists(tmp):
            os.remove(tmp)
        raise RuntimeError("hipcc failed building libpa_probe.so")
    os.replace(tmp, PROBE_SO)
    return PROBE_SO


if __name__ == "__main__":
    print(build(verbose=True))
