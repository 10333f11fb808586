"""The oracle and the library's host table code under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; nothing here touches a GPU).

The oracle is rebuilt with gcc -fsanitize=address,undefined and loaded in a
child Python with the sanitizer runtime preloaded, then runs small
populations through every resampling law, both sweep random-number streams,
+-J couplings, the Potts model, the heating start, the replica-parallel
sweep, the overlap and the bisection.  The table code (reweighting and
Poisson tables, observables, overlap, bisection, weighted averages, family
statistics) is built host-only with hipcc and driven over seeded synthetic
histograms by tests/sanitize/tables_driver.cpp."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SRC = os.path.join(ROOT, "oracle", "pa_oracle.c")

SCRIPT = r'''
import numpy as np
import oracle
import pa_workloads as W
def run(**kw):
    L, R = kw.pop("L"), kw.pop("R")
    betas = kw.pop("betas")
    heat = kw.pop("heat", None)
    threads = kw.pop("threads", 1)
    p = oracle.OraclePA(L, R, seed=3, **kw)
    if heat is not None:
        p.start_heating(heat)
    for b in betas:
        if kw.get("q", 0) == 0 and kw.get("J") is None:
            p.overlap(b - p.beta) if b >= p.beta else None
        p.resample(b)
        p.sweep(2, threads=threads)
        p.observables()
    p.bisect_dbeta(0.85, 2.0) if heat is None else None
    p.families()
    p.close()
sched = W.linear_schedule(1.0, 4)
for law in range(5):
    run(L=8, R=300, betas=sched, law=law)
run(L=10, R=200, betas=sched, J=W.pmj_couplings(10, 4))
run(L=8, R=200, betas=sched, rng_mode=oracle.RNG_PLANES)
run(L=12, R=300, betas=sched, rng_mode=oracle.RNG_PLANES, threads=3)
run(L=8, R=150, betas=W.linear_schedule(1.2, 3), q=4)
run(L=8, R=200, betas=[3.5, 3.0, 2.5], heat=4.0)
print("oracle under sanitizers ok")
'''


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name],
                       capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    ubsan = _runtime("libubsan.so")
    if not shutil.which("gcc") or not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    so = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-ffp-contract=off", "-std=c11",
                    "-fPIC", "-shared", "-pthread",
                    "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", so, ORACLE_SRC, "-lm"], check=True)
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan + " " + ubsan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["PA_ORACLE_SO"] = so
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "oracle under sanitizers ok" in r.stdout


def test_host_tables_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not installed")
    exe = str(tmp_path / "tables_san")
    csrc = os.path.join(ROOT, "paper_2006_00561_amd", "csrc")
    cmd = [hipcc, "--offload-host-only", "-x", "hip", "-std=c++17", "-O1",
           "-g", "-ffp-contract=off",
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(csrc, "pa_tables.hip"),
           os.path.join(ROOT, "tests", "sanitize", "tables_driver.cpp"),
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stderr[-4000:]
    assert "tables driver ok" in r.stdout
