#!/usr/bin/env python3
"""Benchmark of the population-annealing hot path on one MI355X.

One benchmark step is one full anneal of a synthetic population, every step
of the method on the device: init at beta_0 = 0, then for each of the K
temperatures the energy histogram, the host reweighting tables, copy counts,
scan, gather-copy, theta Metropolis sweeps and the observables, with the
free energy accumulated on the way.

Default workload: the 2D Ising ferromagnet, L = 64 periodic, R = 65536
replicas, int8 spins, beta 0 -> 1 in 200 linear steps, theta = 10.

Prints one JSON line (rank 0):
  value           spin-flip attempts per ns over the whole timed anneals
  roofline        the sweep kernel (dominant) against the integer VALU peak,
                  from HIP events on the library's stream
  resample        achieved HBM bandwidth of histogram+counts+scatter+gather
  cpu_baseline    the single-threaded oracle timed on a bounded sample of the
                  same workload on this host
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import pa_workloads as W  # noqa: E402

METRIC = ("spin-flip attempts/ns + resample GB/s (% HBM peak); wall time to "
          "β_f plain vs batched+MLP Δβ")
HBM_PEAK_GBPS = 8000.0
# Integer VALU peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one
# 32-bit operation per lane per cycle (gfx950 issues v_mad_u64_u32 and
# v_bitop3_b32 at that rate; packed FP32 does not apply to integer work).
VALU_OPS_PER_S = 256 * 4 * 16 * 2.4e9
# Algorithmic integer work of one spin-flip attempt: a quarter of a
# Philox4x32-10 block (10 rounds of 2 32x32->64 multiplies and 2 three-input
# xors = 40 ops per 4 words) plus one threshold test and one accumulate.
ALGO_OPS_PER_ATTEMPT = 40 / 4 + 2
# Potts: two words per attempt (proposal and acceptance, half a block) plus
# one threshold test and one select.
ALGO_OPS_PER_ATTEMPT_POTTS = 40 / 2 + 2


KERNEL_SOURCES = ("paper_2006_00561_amd/csrc/pa_lattice.h",
                  "paper_2006_00561_amd/csrc/pa_device.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_lattice_C2_traffic.json")


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per k_lattice launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known
    size), or None if it was taken on another workload or an older kernel."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("workload") != workload or t.get("kernel_sha256") != kernel_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def gather_copy(binding, cfg, stream, reps=5):
    """The standalone gather-copy kernel at the workload's size: resamplings
    whose population is read before the sweep, so the copies run as their
    own HBM-bound pass (2 S per new slot plus E, M and the parent index)."""
    layout = binding.PA_BITS if cfg["layout"] == "bits" else binding.PA_INT8
    g = binding.Population(cfg["L"], cfg["R"], seed=cfg["seed"], layout=layout,
                           stream=stream, q=cfg.get("q", 0))
    sched = W.linear_schedule(cfg["beta_f"], cfg["K"])
    g.resample(sched[0])
    g.sweep(sched[0], 1)
    g.set_timing(True, classes=("gather",))
    for b in sched[1:reps + 1]:
        g.resample(b)
        g.energies()            # the read makes the copies now
        g.sweep(b, 1)
    t = g.timing()["gather"]
    g.close()
    gbps = t["bytes"] / (t["ms"] * 1e6) if t["ms"] else 0.0
    return {"launches": t["launches"], "avg_us": 1e3 * t["ms"] / t["launches"],
            "bytes_per_launch": t["bytes"] / t["launches"], "GBps": gbps,
            "frac_hbm": gbps / HBM_PEAK_GBPS}


def run_anneal(binding, cfg, stream, timing=None, rows_per_lane=0,
               families=None):
    """One full anneal; timing: None, or the kernel classes to time;
    families: a dict that receives the final family statistics."""
    layout = binding.PA_BITS if cfg["layout"] == "bits" else binding.PA_INT8
    L, R, theta = cfg["L"], cfg["R"], cfg["theta"]
    g = binding.Population(L, R, seed=cfg["seed"], layout=layout,
                           rows_per_lane=rows_per_lane, stream=stream,
                           capacity=W.deferral_capacity(R), q=cfg.get("q", 0),
                           resampling=cfg.get("law", 0))
    if timing:
        g.set_timing(True, classes=timing)
    attempts = 0
    for b in W.linear_schedule(cfg["beta_f"], cfg["K"]):
        g.resample(b, wait=False)
        g.sweep(b, theta)
        attempts += g.observables()["R"] * L * L * theta
    lnZ, _ = g.free_energy()
    t = g.timing() if timing else None
    if families is not None:
        families.update(g.family_stats())
    g.close()
    return attempts, lnZ, t


def cpu_baseline(cfg, budget_s=15.0):
    """The oracle (single thread) on the first temperature steps of the same
    workload with a reduced population, scaled to attempts/ns."""
    import oracle
    oracle.build(force=False)
    L, theta = cfg["L"], cfg["theta"]
    R = 2048
    sched = W.linear_schedule(cfg["beta_f"], cfg["K"])
    p = oracle.OraclePA(L, R, seed=cfg["seed"])
    t0 = time.perf_counter()
    attempts, steps = 0, 0
    for b in sched:
        p.resample(b)
        attempts += p.R * L * L * theta
        p.sweep(theta)
        p.observables()
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": attempts / (dt * 1e9), "unit": "spin-flip attempts/ns",
            "cores": 1, "kind": "oracle",
            "sample": "%s shape with R=%d replicas, first %d of %d temperature "
                      "steps (resample + %d sweeps + observables), %.1f s, "
                      "single thread" % (cfg.get("name", "?"), R, steps,
                                         cfg["K"], theta, dt)}


def bench_batched(binding, stream, use_graph=True):
    """C4: 64 +-J populations (L in {8..32}, R in [2^10, 2^16]), beta 0 -> 3
    in 300 linear steps, theta = 10; each population alone through the
    single-population path, then all of them in one batch.  Both runs give
    bit-identical ln Z, so accuracy is equal by construction."""
    import torch
    inst = W.batched_glass_instances()
    betas = W.linear_schedule(3.0, 300)
    theta = 10
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lnz_plain, attempts = [], 0
    for c in inst:
        g = binding.Population(c["L"], c["R"], seed=c["seed"],
                               population_id=c["population_id"], J=c["J"],
                               stream=stream)
        for b in betas:
            g.resample(b, wait=False)
            g.sweep(b, theta)
            attempts += g.observables()["R"] * c["L"] ** 2 * theta
        lnz_plain.append(g.free_energy()[0])
        g.close()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    bt = binding.Batch(inst, autotune=True)        # tuning outside the timing
    bt.close()
    t0 = time.perf_counter()
    bt = binding.Batch(inst, autotune=True)
    t_init = time.perf_counter() - t0
    bt.run(betas, theta, use_graph=use_graph)
    lnz_batch = [bt.state(p)[3] for p in range(len(inst))]
    t_batch = time.perf_counter() - t0
    host_ms = bt.host_stats()["host_ms"]
    bt.close()
    return {
        "workload": "C4: 64 +-J EA instances, L in {8,12,16,24,32}, R "
                    "log-uniform in [2^10,2^16], beta 0->3 in 300 linear "
                    "steps, theta=10",
        "plain_s": t_plain, "batched_s": t_batch,
        "batched_init_s": t_init, "batched_host_ms": host_ms,
        "speedup": t_plain / t_batch,
        "batched_attempts_per_ns": attempts / (t_batch * 1e9),
        "graph": bool(use_graph),
        "lnZ_bitwise_equal": lnz_plain == lnz_batch,
    }


def bench_learned(binding, use_graph=True, target=0.85, tol=0.02):
    """Adaptive schedules on the C4 populations to beta_f = 3, theta = 10:
    the exact bisection on the overlap, and the network (trained on the
    exact schedules of 32 other instances) with the bisection as check and
    fallback.  Wall time to beta_f, host time of the decisions, exact
    overlap evaluations, and the ln Z agreement of the two."""
    from paper_2006_00561_amd import learned
    import numpy as np
    inst = W.batched_glass_instances()
    train_inst = W.batched_glass_instances(n=32, seed=4242,
                                           coupling_seed0=10001)
    for k, c in enumerate(train_inst):
        c["population_id"] = 1000 + k
    theta, beta_f = 10, 3.0
    t0 = time.perf_counter()
    X, T = learned.generate(train_inst, [0.8, 0.85, 0.9], beta_f, theta)
    mlp, loss = learned.train(X, T, iters=3000, lr=2e-3, seed=5)
    t_train = time.perf_counter() - t0
    out = {"training_pairs": int(len(X)), "training_s": t_train,
           "final_loss": loss, "target": target, "tol": tol}
    res = {}
    for mode in ("bisection", "learned"):
        b = binding.Batch(inst, autotune=True)
        t0 = time.perf_counter()
        if mode == "bisection":
            steps = b.run_adaptive(target, beta_f, 20000, theta,
                                   use_graph=use_graph)
        else:
            steps, _ = b.run_learned(mlp, target, tol, beta_f, 20000, theta,
                                     use_graph=use_graph)
        dt = time.perf_counter() - t0
        st = b.host_stats()
        lnz = np.array([b.state(p)[3] for p in range(len(inst))])
        res[mode] = (dt, steps, st, lnz)
        b.close()
    for mode, (dt, steps, st, lnz) in res.items():
        out[mode] = {"wall_s": dt, "max_steps": steps,
                     "host_ms": st["host_ms"],
                     "overlap_evals": st["overlap_evals"],
                     "sources": st["sources"]}
    Ns = np.array([c["L"] ** 2 for c in inst], np.float64)
    d = (res["learned"][3] - res["bisection"][3]) / Ns
    out["lnZ_per_spin_rms_diff"] = float(np.sqrt(np.mean(d * d)))
    out["speedup"] = res["bisection"][0] / res["learned"][0]
    mlp.close()
    return out


def bench_accuracy(binding, use_graph=True, M=64, L=32, R=2048, theta=10,
                   beta_f=1.0):
    """Wall time to beta_f against the free-energy error, for M independent
    ferromagnet populations (L, R, theta) run as one batch per schedule:
    linear schedules of several lengths, the exact bisection at two overlap
    targets, and the network at 0.85 (trained on the exact schedules of
    other ferromagnets).  The error is ln Z - ln Z_exact per spin at beta_f,
    ln Z_exact from Kaufman's finite-torus solution."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from exact_ising import kaufman_lnZ
    from paper_2006_00561_amd import learned
    N = L * L
    exact = float(kaufman_lnZ(L, beta_f))
    pops = [dict(L=L, R=R, seed=7000 + k, population_id=k) for k in range(M)]

    def timed(fn):
        b = binding.Batch(pops)
        t0 = time.perf_counter()
        info = fn(b)
        dt = time.perf_counter() - t0
        z = np.array([b.state(p)[3] for p in range(M)])
        steps = max(b.state(p)[2] for p in range(M))
        b.close()
        err = (z - exact) / N
        out = {"steps": int(steps), "wall_s": dt,
               "rms_err_per_spin": float(np.sqrt(np.mean(err ** 2))),
               "mean_err_per_spin": float(err.mean()),
               "sd_err_per_spin": float(err.std(ddof=1))}
        if info:
            out.update(info)
        return out

    runs = {}
    for K in (25, 50, 100, 200, 400):
        betas = np.array(W.linear_schedule(beta_f, K))
        runs["linear K=%d" % K] = timed(
            lambda b: b.run(betas, theta, use_graph=use_graph))
    for target in (0.7, 0.85):
        runs["bisection alpha*=%g" % target] = timed(
            lambda b: (b.run_adaptive(target, beta_f, 5000, theta,
                                      use_graph=use_graph),
                       {"host_ms": b.host_stats()["host_ms"]})[1])
    train = [dict(L=l, R=r, seed=9000 + 10 * i + j, population_id=100 + 10 * i + j)
             for i, l in enumerate((16, 24, 32, 48))
             for j, r in enumerate((1024, 2048, 4096))]
    X, T = learned.generate(train, [0.8, 0.85, 0.9], beta_f, theta)
    mlp, _ = learned.train(X, T, iters=3000, lr=2e-3, seed=17)

    def run_net(b):
        _, src = b.run_learned(mlp, 0.85, 0.02, beta_f, 5000, theta,
                               use_graph=use_graph)
        return {"host_ms": b.host_stats()["host_ms"],
                "sources": [int(v) for v in src]}
    runs["network alpha*=0.85"] = timed(run_net)
    mlp.close()
    return {"workload": "%d independent ferromagnet populations, L=%d, R=%d, "
                        "theta=%d, beta 0->%g; error of ln Z per spin against "
                        "Kaufman's exact finite-torus value" % (M, L, R, theta,
                                                              beta_f),
            "lnZ_exact": exact, "training_pairs": int(len(X)), "runs": runs}


def summarize_profiles(trace_dir, fetch_dir, write_dir, workload, command):
    """Write profiles/ summaries from rocprofv3 CSV output: per-kernel
    durations (--kernel-trace --stats) and HBM traffic (--pmc FETCH_SIZE and
    --pmc WRITE_SIZE runs that also ran a 1 GiB device copy, whose counters
    calibrate the scale)."""
    import csv
    import glob

    def one(pattern):
        f = glob.glob(os.path.join(pattern))
        if not f:
            raise SystemExit("no file matches " + pattern)
        return f[0]

    stats = list(csv.DictReader(open(one(os.path.join(trace_dir,
                                                       "*kernel_stats.csv")))))
    per = {}
    for cnt, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = list(csv.DictReader(open(one(os.path.join(
            d, "*counter_collection.csv")))))
        agg = {}
        for r in rows:
            agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        # the 1 GiB copies are the largest copy dispatches of the run (the
        # library's own small copies share the kernel name)
        copy = sorted(v for k, vs in agg.items() if "copy" in k.lower()
                      for v in vs)[-3:]
        copy_kib = sum(copy) / len(copy) if copy else 0.0
        scale = (1 << 20) / copy_kib if copy_kib > 0 else float("nan")
        per[cnt] = (agg, scale, copy_kib)
    def lattice(agg):
        return [v for k, vs in agg.items() if k.startswith("k_lattice")
                for v in vs]

    lat_f = lattice(per["FETCH_SIZE"][0])
    lat_w = lattice(per["WRITE_SIZE"][0])
    if not lat_f or not lat_w:
        raise SystemExit("no k_lattice dispatch in the counter output")
    fetch_b = (sum(lat_f) / len(lat_f)) * 1024 * per["FETCH_SIZE"][1]
    write_b = (sum(lat_w) / len(lat_w)) * 1024 * per["WRITE_SIZE"][1]
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump({
            "workload": workload, "kernel": "k_lattice",
            "kernel_sha256": kernel_hash(),
            "fetch_scale": per["FETCH_SIZE"][1],
            "write_scale": per["WRITE_SIZE"][1],
            "copy_calibration_KiB": {"FETCH_SIZE": per["FETCH_SIZE"][2],
                                     "WRITE_SIZE": per["WRITE_SIZE"][2],
                                     "expected": 1 << 20},
            "launches": len(lat_f),
            "fetch_bytes_per_launch": fetch_b,
            "write_bytes_per_launch": write_b,
            "hbm_bytes_per_launch": fetch_b + write_b,
            "commands": command}, fh, indent=1)
    lines = ["# rocprofv3 kernel statistics, workload %s" % workload, "",
             "Commands:", ""] + ["    " + c for c in command] + [
             "", "| kernel | calls | average ns | total ns | % |",
             "|---|---|---|---|---|"]
    for r in stats:
        lines.append("| %s | %s | %.0f | %s | %s |" % (
            r["Name"], r["Calls"], float(r["AverageNs"]),
            r["TotalDurationNs"], r["Percentage"]))
    lines += ["", "HBM traffic of k_lattice per launch (counters scaled by "
              "a 1 GiB copy: FETCH_SIZE x%.3f, WRITE_SIZE x%.3f): fetch "
              "%.1f MB, write %.1f MB, total %.1f MB over %d launches." % (
                  per["FETCH_SIZE"][1], per["WRITE_SIZE"][1], fetch_b / 1e6,
                  write_b / 1e6, (fetch_b + write_b) / 1e6, len(lat_f))]
    with open(os.path.join(ROOT, "profiles", "kernels_%s.md" % workload),
              "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_trace(trace_dir, name, command):
    """profiles/kernels_<name>.md from a rocprofv3 --kernel-trace --stats
    run: per-kernel calls and durations, with the command that made it."""
    import csv
    import glob
    f = glob.glob(os.path.join(trace_dir, "*kernel_stats.csv"))
    if not f:
        raise SystemExit("no kernel_stats.csv in " + trace_dir)
    stats = list(csv.DictReader(open(f[0])))
    lines = ["# rocprofv3 kernel statistics, workload %s" % name, "",
             "Commands:", "", "    cd /tmp && export TMPDIR=/tmp",
             "    " + command, "",
             "| kernel | calls | average ns | total ns | % |",
             "|---|---|---|---|---|"]
    for r in stats:
        lines.append("| %s | %s | %.0f | %s | %s |" % (
            r["Name"], r["Calls"], float(r["AverageNs"]),
            r["TotalDurationNs"], r["Percentage"]))
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "kernels_%s.md" % name),
              "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C2", choices=sorted(W.CONFIGS))
    ap.add_argument("--rows-per-lane", type=int, default=0)
    ap.add_argument("--law", default="nearest",
                    choices=["nearest", "poisson", "systematic", "residual",
                             "multinomial"],
                    help="resampling law of the timed anneals")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched comparison (for profiling)")
    ap.add_argument("--accuracy-only", action="store_true",
                    help="only the schedule accuracy comparison")
    ap.add_argument("--eager", action="store_true",
                    help="batched runs without HIP graphs")
    ap.add_argument("--summarize-profiles", nargs=3,
                    metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/ summaries from rocprofv3 output")
    ap.add_argument("--summarize-trace", nargs=3,
                    metavar=("TRACE_DIR", "NAME", "COMMAND"),
                    help="write profiles/kernels_NAME.md from a kernel trace")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy, the reference "
                         "for scaling FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_profiles:
        base = ("python3 <repo>/bench.py --workload %s --no-cpu-baseline "
                "--no-batched --no-learned --no-accuracy" % args.workload)
        cmd = ["cd /tmp && export TMPDIR=/tmp",
               "rocprofv3 --kernel-trace --stats -T -d <TRACE_DIR> -o run "
               "--output-format csv -- %s --steps 2 --warmup 1" % base,
               "rocprofv3 --pmc FETCH_SIZE -T -d <FETCH_DIR> -o run "
               "--output-format csv -- %s --steps 1 --warmup 0 "
               "--calibrate-copy" % base,
               "rocprofv3 --pmc WRITE_SIZE -T -d <WRITE_DIR> -o run "
               "--output-format csv -- %s --steps 1 --warmup 0 "
               "--calibrate-copy" % base,
               "python3 bench.py --workload %s --summarize-profiles "
               "<TRACE_DIR> <FETCH_DIR> <WRITE_DIR>" % args.workload]
        summarize_profiles(*args.summarize_profiles, args.workload, cmd)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU "
              "path (a population would shard by replica slots, with one "
              "histogram all-reduce per temperature step).  Run with "
              "--gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2006_00561_amd import binding

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    if args.batched_only:
        print(json.dumps(bench_batched(binding, stream,
                                       use_graph=not args.eager)), flush=True)
        return
    if args.accuracy_only:
        print(json.dumps(bench_accuracy(binding, use_graph=not args.eager)),
              flush=True)
        return
    cfg = dict(W.CONFIGS[args.workload])
    cfg["name"] = args.workload
    cfg["law"] = ["nearest", "poisson", "systematic", "residual",
                  "multinomial"].index(args.law)
    if args.calibrate_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        run_anneal(binding, cfg, stream, rows_per_lane=args.rows_per_lane)
    torch.cuda.synchronize()

    total_attempts = 0
    tsum = None
    lnZs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        # events on the sweep launches only (two markers per timed launch)
        a, lnZ, t = run_anneal(binding, cfg, stream, timing=("sweep",),
                               rows_per_lane=args.rows_per_lane)
        total_attempts += a
        lnZs.append(lnZ)
        if tsum is None:
            tsum = t
        else:
            for k in binding.KERNEL_CLASSES:
                for f in ("ms", "launches", "bytes"):
                    tsum[k][f] += t[k][f]
            tsum["attempts"] += t["attempts"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    sw = tsum["sweep"]
    sweep_avg_ms = sw["ms"] / max(1, sw["launches"])
    sweep_rate = tsum["attempts"] / (sw["ms"] * 1e6)       # attempts/ns
    ops = ALGO_OPS_PER_ATTEMPT_POTTS if cfg.get("q") else ALGO_OPS_PER_ATTEMPT
    achieved = tsum["attempts"] / sw["launches"] * ops / (
        sweep_avg_ms * 1e-3) / 1e12
    peak = VALU_OPS_PER_S / 1e12
    # every kernel class timed, on one more anneal after the timed region
    fam = {}
    _, _, tall = run_anneal(binding, cfg, stream, timing=binding.KERNEL_CLASSES,
                            rows_per_lane=args.rows_per_lane, families=fam)
    res_k = ("hist", "counts", "scatter", "gather")
    res_ms = sum(tall[k]["ms"] for k in res_k)
    res_bytes = sum(tall[k]["bytes"] for k in res_k)
    res_gbps = res_bytes / (res_ms * 1e6) if res_ms > 0 else 0.0
    sw_all = tall["sweep"]
    # the replica copies of every resampling happen inside the sweep kernel
    # (each new slot loaded from its parent): its read + write of the whole
    # population per launch against HBM
    copy_gbps = sw_all["bytes"] / (sw_all["ms"] * 1e6) if sw_all["ms"] else 0.0

    out = {
        "metric": METRIC,
        "value": total_attempts / (dt * 1e9),
        "unit": "spin-flip attempts/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "%s: 2D %s ferromagnet L=%d periodic, R=%d, %s "
                        "spins, beta 0->%g in %d linear steps, theta=%d, "
                        "seed %d; one step = one full anneal"
                        % (args.workload,
                           ("%d-state Potts" % cfg["q"]) if cfg.get("q")
                           else "Ising", cfg["L"], cfg["R"], cfg["layout"],
                           cfg["beta_f"], cfg["K"], cfg["theta"],
                           cfg["seed"]),
            "L": cfg["L"], "R": cfg["R"], "K": cfg["K"],
            "theta": cfg["theta"], "layout": cfg["layout"],
            "resampling": args.law,
        },
        "roofline": {
            "kernel": (("k_potts_swar" if cfg["L"] in (8, 16, 32, 64, 128)
                        else "k_potts") if cfg.get("q") else "k_lattice") +
                      " (theta fused Metropolis sweeps)",
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "TOP/s (32-bit integer VALU)",
            "frac": achieved / peak,
            "traffic": measured_traffic(args.workload),
            "sweep_attempts_per_ns": sweep_rate,
            "sweep_avg_ms": sweep_avg_ms,
            "ops_per_attempt": ops,
        },
        "resample": {
            "note": "one extra anneal after the timed region with every "
                    "kernel class timed; the replica copies are fused into "
                    "the sweep, so the resampling kernels only move energies, "
                    "counts and parent indices",
            "GBps": res_gbps,
            "frac_hbm": res_gbps / HBM_PEAK_GBPS,
            "ms_per_anneal": res_ms,
            "kernel_ms": {k: tall[k]["ms"] for k in binding.KERNEL_CLASSES},
            "launches": {k: tall[k]["launches"] for k in
                         binding.KERNEL_CLASSES},
            "sweep_with_copy_GBps": copy_gbps,
            "sweep_with_copy_frac_hbm": copy_gbps / HBM_PEAK_GBPS,
            "standalone_gather_copy": gather_copy(binding, cfg, stream),
        },
        "wall_time_to_beta_f_s": dt / args.steps,
        "lnZ_final": lnZs[-1],
        # descendants of the initial replicas at beta_f (the untimed anneal)
        "families_final": fam,
    }
    if not args.no_batched:
        out["batched"] = bench_batched(binding, stream,
                                       use_graph=not args.eager)
    if not args.no_learned:
        out["learned"] = bench_learned(binding, use_graph=not args.eager)
    if not args.no_accuracy:
        out["accuracy"] = bench_accuracy(binding, use_graph=not args.eager)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
