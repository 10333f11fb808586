#!/usr/bin/env python3
"""Benchmark of the population-annealing hot path on one MI355X.

One benchmark step is one full anneal of a synthetic population, every step
of the method on the device: init at beta_0 = 0, then for each of the K
temperatures the energy histogram, the host reweighting tables, copy counts,
scan, gather-copy, theta Metropolis sweeps and the observables, with the
free energy accumulated on the way.

Default workload: the paper's total replica count on one device, the 2D
Ising ferromagnet with L = 64 periodic, R = 2^21 replicas, bit-packed spins,
beta 0 -> 0.5 in 100 linear steps, theta = 10.  The L = 128 population at
the same scale (R = 2^18, bit-packed), the int8 workload (L = 64, R =
65536, beta 0 -> 1 in 200 steps) and the paper's per-GPU shape (R = 20480)
are timed as secondary figures of the same line.

Prints one JSON line (rank 0):
  value           spin-flip attempts per ns over the whole timed anneals
  roofline        the sweep kernel (dominant) against the integer VALU peak,
                  from HIP events on the library's stream
  resample        achieved HBM bandwidth of histogram+counts+scatter+gather
  cpu_baseline    the oracle timed on a bounded sample of the same workload
                  on this host, on every core (replica-parallel sweeps) and
                  on one
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
# Vector ALU of MI355X: 256 CUs x 4 SIMDs at 2.4 GHz.  A wave64 instruction
# that forms a 64-bit product (v_mad_u64_u32, the Philox multiply) holds its
# SIMD for 4 cycles, the rate of the fp64 FMA (78.6 TFLOP/s = 39.3 T lane
# operations/s); plain 32-bit logic and integer instructions take 2 cycles,
# the rate of the fp32 FMA (157.3 TFLOP/s = 78.6 T lane operations/s).  The
# probe in libpa_probe.so measures both rates on the device.  Work is priced
# in multiply-equivalents: a 64-bit-product multiply counts 1, a plain 32-bit
# operation 1/2, so the peak is the multiply rate.
MAD_PER_S = 256 * 4 * 16 * 2.4e9
SIMPLE_PER_S = 2 * MAD_PER_S
VALU_OPS_PER_S = MAD_PER_S
# Algorithmic work of one spin-flip attempt (multiplies, plain operations).
# Word stream: a quarter of a Philox4x32-10 block (10 rounds of 2 multiplies
# and 2 three-input xors, per 4 words) and the decision (threshold test and
# flip).  Plane stream: a sixteenth of a block, a bit-sliced byte comparison
# (16 plane steps per 32 positions), the flip, and for the 1/256 of the
# draws whose byte ties with the threshold the site's own word and a test.
ALGO_WORK = {"word": (5.0, 5.0 + 2.0),
             "planes": (20 / 16 + 5 / 256, 20 / 16 + 0.5 + 1.0 + 6 / 256)}
# Potts: two words per attempt (proposal and acceptance, half a block) plus
# one threshold test and one select.
ALGO_WORK_POTTS = (10.0, 10.0 + 2.0)


def mad_equivalents(work):
    mads, simple = work
    return mads + simple * (MAD_PER_S / SIMPLE_PER_S)


KERNEL_SOURCES = ("paper_2006_00561_amd/csrc/pa_lattice.h",
                  "paper_2006_00561_amd/csrc/pa_device.h")


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", "k_lattice_%s_traffic.json" % workload)


def valu_file(workload, kernel="k_lattice"):
    return os.path.join(ROOT, "profiles", "%s_%s_valu.json" % (kernel,
                                                               workload))


# sources of each profiled kernel beyond the lattice pass
KERNEL_EXTRA = {"k_bsweep": ("paper_2006_00561_amd/csrc/pa_batch.hip",),
                "k_potts_swar": ("paper_2006_00561_amd/csrc/pa_potts.h",
                                 "paper_2006_00561_amd/csrc/pa_potts.hip")}


def kernel_hash(kernel="k_lattice"):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES + KERNEL_EXTRA.get(kernel, ()):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per k_lattice launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known
    size), or None if it was taken on another workload or an older kernel."""
    t = _load_keyed(traffic_file(workload), workload)
    return t.get("hbm_bytes_per_launch") if t else None


def _load_keyed(path, workload, kernel="k_lattice"):
    """A committed counter summary, or None if it was taken on another
    workload or an older kernel."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if (t.get("workload") != workload or
            t.get("kernel_sha256") != kernel_hash(kernel)):
        return None
    return t


def measured_valu(workload):
    """Issued VALU instructions of k_lattice per spin-flip attempt, in lane
    operations (SQ_INSTS_VALU x 64 / attempts), from the committed rocprofv3
    counter summary, or None."""
    t = _load_keyed(valu_file(workload), workload)
    return t.get("valu_lane_ops_per_attempt") if t else None


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
               families=None, step_calls=False, timing_every=1):
    """One full anneal: the whole schedule in one pa_anneal call (the
    device runs it with no host stop between steps), or with step_calls the
    pa_resample / pa_sweep / pa_observables calls of every step (at the
    capacity where no resampling waits for its size).  timing: None, or the
    kernel classes to time; families: a dict that receives the final family
    statistics; timing_every: time the first launch of a class and then
    one in timing_every."""
    layout = binding.PA_BITS if cfg["layout"] == "bits" else binding.PA_INT8
    L, R, theta = cfg["L"], cfg["R"], cfg["theta"]
    g = binding.Population(L, R, seed=cfg["seed"], layout=layout,
                           rows_per_lane=rows_per_lane, stream=stream,
                           capacity=W.deferral_capacity(R) if step_calls
                           else 0, q=cfg.get("q", 0),
                           resampling=cfg.get("law", 0),
                           rng_mode=cfg.get("rng_mode", 0))
    if timing:
        g.set_timing(True, classes=timing, every=timing_every)
    sched = W.linear_schedule(cfg["beta_f"], cfg["K"])
    attempts = 0
    if step_calls:
        for b in sched:
            g.resample(b, wait=False)
            g.sweep(b, theta)
            attempts += g.observables()["R"] * L * L * theta
    else:
        obs, _ = g.anneal(sched, theta, as_dicts=False)
        attempts = int(obs["R"].sum()) * L * L * theta
    lnZ, _ = g.free_energy()
    t = g.timing() if timing else None
    if families is not None:
        families.update(g.family_stats())
    g.close()
    return attempts, lnZ, t


def host_cpu():
    """CPU model and core counts of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    return {"model": model, "nproc": avail, "cpu_count": os.cpu_count()}


def cpu_threads():
    """Threads for the all-core oracle leg: the cores this process may use,
    at most the OMP_NUM_THREADS share when that is set."""
    n = host_cpu()["nproc"]
    try:
        share = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        share = 0
    return max(1, min(n, share) if share > 0 else n)


def _oracle_leg(cfg, R, threads, budget_s):
    """The oracle on the first temperature steps of cfg's schedule with R
    replicas; sweeps split over `threads` POSIX threads (bit-identical to
    one thread).  Returns (attempts/ns, steps, seconds, ln Z)."""
    import oracle
    L, theta = cfg["L"], cfg["theta"]
    sched = W.linear_schedule(cfg["beta_f"], cfg["K"])
    p = oracle.OraclePA(L, R, seed=cfg["seed"],
                        rng_mode=cfg.get("rng_mode", 0))
    t0 = time.perf_counter()
    attempts, steps = 0, 0
    for b in sched:
        p.resample(b)
        attempts += p.R * L * L * theta
        p.sweep(theta, threads=threads)
        p.observables()
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    lnZ = p.free_energy()[0]
    p.close()
    return attempts / (dt * 1e9), steps, dt, lnZ


def cpu_baseline(cfg, budget_s=24.0):
    """The oracle as it stands on the first temperature steps of the same
    workload with a reduced population, scaled to attempts/ns: once with
    the sweeps split over every core this process may use (the headline
    value) and once on one thread."""
    import oracle
    oracle.build(force=False)
    host = host_cpu()
    nt = cpu_threads()
    R1, RN = 2048, 2048 * nt
    v1, s1, d1, _ = _oracle_leg(cfg, R1, 1, budget_s / 2)
    vN, sN, dN, _ = _oracle_leg(cfg, RN, nt, budget_s / 2)
    return {"value": vN, "unit": "spin-flip attempts/ns", "cores": nt,
            "kind": "oracle",
            "sample": "%s shape (L=%d, theta=%d, beta 0->%g in %d steps) with "
                      "R=%d replicas, first %d of %d temperature steps "
                      "(resample + sweeps + observables), %.1f s, sweeps on "
                      "%d threads" % (cfg.get("name", "?"), cfg["L"],
                                      cfg["theta"], cfg["beta_f"], cfg["K"],
                                      RN, sN, cfg["K"], dN, nt),
            "single_thread": {"value": v1, "cores": 1,
                              "sample": "R=%d, first %d steps, %.1f s"
                                        % (R1, s1, d1)},
            "per_core": vN / nt,
            "host": host}


def bench_batched(binding, stream, use_graph=True, rng_mode=0,
                  tune_sweep=True):
    """C4: 64 +-J populations (L in {8..32}, R in [2^10, 2^16]), beta 0 -> 3
    in 300 linear steps, theta = 10; each population alone through the
    single-population path (one pa_anneal call each, the whole schedule on
    the device), then all of them in one batch.  Both runs give
    bit-identical ln Z, so accuracy is equal by construction."""
    import torch
    inst = W.batched_glass_instances()
    for c in inst:
        c["rng_mode"] = rng_mode
    betas = W.linear_schedule(3.0, 300)
    theta = 10
    # tuning outside the timing, and before the population-by-population
    # leg, so that a trace can tell the tuners' scratch batches from the
    # timed batch (both tuners cache their choice)
    bt = binding.Batch(inst, autotune=True, tune_sweep=tune_sweep)
    bt.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lnz_plain, attempts = [], 0
    for c in inst:
        g = binding.Population(c["L"], c["R"], seed=c["seed"],
                               population_id=c["population_id"], J=c["J"],
                               stream=stream, rng_mode=rng_mode)
        obs, _ = g.anneal(betas, theta, as_dicts=False)
        attempts += int(obs["R"].sum()) * c["L"] ** 2 * theta
        lnz_plain.append(g.free_energy()[0])
        g.close()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    bt = binding.Batch(inst, autotune=True, tune_sweep=tune_sweep)
    t_init = time.perf_counter() - t0
    bt.run(betas, theta, use_graph=use_graph)
    lnz_batch = [bt.state(p)[3] for p in range(len(inst))]
    t_batch = time.perf_counter() - t0
    host_ms = bt.host_stats()["host_ms"]
    sweep_shape = bt.sweep_blocks()
    bt.close()
    # the persistent sweep against its roofline, from the committed
    # rocprofv3 summary of this workload while the kernel is unchanged
    prof = _load_keyed(valu_file("C4", "k_bsweep"), "C4", "k_bsweep")
    bsweep = None
    if prof and prof.get("attempts_per_ns"):
        rate = prof["attempts_per_ns"]
        ops = mad_equivalents(ALGO_WORK["planes" if rng_mode else "word"])
        bsweep = {"kernel": "k_bsweep", "attempts_per_ns": rate,
                  "frac": rate * 1e9 * ops / VALU_OPS_PER_S,
                  "valu_lane_ops_per_attempt_counted":
                      prof.get("valu_lane_ops_per_attempt"),
                  "source": "profiles/k_bsweep_C4_valu.json"}
    return {
        "workload": "C4: 64 +-J EA instances, L in {8,12,16,24,32}, R "
                    "log-uniform in [2^10,2^16], beta 0->3 in 300 linear "
                    "steps, theta=10",
        "plain_s": t_plain, "batched_s": t_batch,
        "batched_init_s": t_init, "batched_host_ms": host_ms,
        "speedup": t_plain / t_batch,
        "batched_attempts_per_ns": attempts / (t_batch * 1e9),
        "attempts": attempts,
        "graph": bool(use_graph),
        "rng": ["word", "planes"][rng_mode],
        "sweep_blocks_chunk": list(sweep_shape),
        "k_bsweep_roofline": bsweep,
        "lnZ_bitwise_equal": lnz_plain == lnz_batch,
    }


def bench_learned(binding, use_graph=True, target=0.85, tol=0.02,
                  rng_mode=0):
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
    for c in inst + train_inst:
        c["rng_mode"] = rng_mode
    theta, beta_f = 10, 3.0
    t0 = time.perf_counter()
    X, T = learned.generate(train_inst, [0.8, 0.85, 0.9], beta_f, theta)
    mlp, loss = learned.train(X, T, iters=3000, lr=2e-3, seed=5)
    t_train = time.perf_counter() - t0
    out = {"training_pairs": int(len(X)), "training_s": t_train,
           "final_loss": loss, "target": target, "tol": tol}
    res = {}
    for mode in ("bisection", "bisection_tol", "learned"):
        b = binding.Batch(inst, autotune=True)
        t0 = time.perf_counter()
        if mode == "bisection":
            steps = b.run_adaptive(target, beta_f, 20000, theta,
                                   use_graph=use_graph)
        elif mode == "bisection_tol":
            steps = b.run_adaptive(target, beta_f, 20000, theta,
                                   use_graph=use_graph, tol=tol)
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
    # against the bisection that stops at the network's own acceptance test
    out["speedup_vs_tol_bisection"] = (res["bisection_tol"][0] /
                                       res["learned"][0])
    mlp.close()
    return out


def _rms_and_se(err):
    """RMS of the errors and its standard error (delta method on the mean
    of the squares)."""
    import numpy as np
    e2 = err * err
    rms = float(np.sqrt(e2.mean()))
    se = float(e2.std(ddof=1) / np.sqrt(len(e2)) / (2.0 * rms)) if rms else 0.0
    return rms, se


def matched_linear_time(runs, rms):
    """Wall time of the linear schedule at the RMS error `rms`, by
    interpolating log(wall time) linearly in log(RMS error) between the two
    linear runs that bracket it, or, below the longest schedule's error,
    extrapolating the line through the two longest (flagged); None if the
    error is above every linear run's."""
    import math
    lin = sorted((r["steps"], r["wall_s"], r["rms_err_per_spin"])
                 for k, r in runs.items() if k.startswith("linear"))

    def at(p1, p2, extrapolated):
        (k1, t1, e1), (k2, t2, e2) = p1, p2
        f = (math.log(e1) - math.log(rms)) / (math.log(e1) - math.log(e2))
        return {"K": math.exp(math.log(k1) + f * (math.log(k2) -
                                                  math.log(k1))),
                "wall_s": math.exp(math.log(t1) + f * (math.log(t2) -
                                                        math.log(t1))),
                "extrapolated": extrapolated}
    for p1, p2 in zip(lin, lin[1:]):
        if p1[2] >= rms >= p2[2] and p1[2] > p2[2]:
            return at(p1, p2, False)
    if len(lin) >= 2 and rms < lin[-1][2] and lin[-2][2] > lin[-1][2]:
        return at(lin[-2], lin[-1], True)
    return None


def bench_accuracy(binding, use_graph=True, M=64, L=32, R=2048, theta=10,
                   beta_f=1.0, Ks=(25, 50, 100, 200, 400),
                   train_LR=((16, 24, 32, 48), (1024, 2048, 4096)),
                   target=0.85, tol=0.02, label=None, rng_mode=0):
    """Wall time to beta_f against the free-energy error, for M independent
    ferromagnet populations (L, R, theta) run as one batch per schedule:
    linear schedules of several lengths, the exact bisection on the overlap
    (64 halvings), the bisection stopped at the first step within tol of
    the target (the network's own acceptance test, without a network), and
    the network (trained on the exact schedules of other ferromagnets).
    The error is ln Z - ln Z_exact per spin at beta_f, ln Z_exact from
    Kaufman's finite-torus solution.  `matched` compares the network with
    the linear schedule interpolated to the network's RMS error."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from exact_ising import kaufman_lnZ
    from paper_2006_00561_amd import learned
    N = L * L
    exact = float(kaufman_lnZ(L, beta_f))
    pops = [dict(L=L, R=R, seed=7000 + k, population_id=k, rng_mode=rng_mode)
            for k in range(M)]

    def timed(fn):
        b = binding.Batch(pops)
        t0 = time.perf_counter()
        info = fn(b)
        dt = time.perf_counter() - t0
        z = np.array([b.state(p)[3] for p in range(M)])
        steps = max(b.state(p)[2] for p in range(M))
        st = b.host_stats()
        b.close()
        err = (z - exact) / N
        rms, se = _rms_and_se(err)
        out = {"steps": int(steps), "wall_s": dt,
               "rms_err_per_spin": rms, "rms_se": se,
               "mean_err_per_spin": float(err.mean()),
               "sd_err_per_spin": float(err.std(ddof=1)),
               "host_ms": st["host_ms"], "overlap_evals": st["overlap_evals"]}
        if info:
            out.update(info)
        return out

    runs = {}
    for K in Ks:
        betas = np.array(W.linear_schedule(beta_f, K))
        runs["linear K=%d" % K] = timed(
            lambda b: b.run(betas, theta, use_graph=use_graph))
        progress("accuracy %s: linear K=%d" % (label or L, K))
    runs["bisection alpha*=%g" % target] = timed(
        lambda b: b.run_adaptive(target, beta_f, 5000, theta,
                                 use_graph=use_graph) and None)
    runs["bisection alpha*=%g tol=%g" % (target, tol)] = timed(
        lambda b: b.run_adaptive(target, beta_f, 5000, theta,
                                 use_graph=use_graph, tol=tol) and None)
    train = [dict(L=l, R=r, seed=9000 + 10 * i + j,
                  population_id=100 + 10 * i + j, rng_mode=rng_mode)
             for i, l in enumerate(train_LR[0])
             for j, r in enumerate(train_LR[1])]
    t0 = time.perf_counter()
    X, T = learned.generate(train, [0.8, 0.85, 0.9], beta_f, theta)
    mlp, _ = learned.train(X, T, iters=3000, lr=2e-3, seed=17)
    t_train = time.perf_counter() - t0
    progress("accuracy %s: network trained" % (label or L))

    def run_net(b):
        _, src = b.run_learned(mlp, target, tol, beta_f, 5000, theta,
                               use_graph=use_graph)
        return {"sources": [int(v) for v in src]}
    net_key = "network alpha*=%g tol=%g" % (target, tol)
    runs[net_key] = timed(run_net)
    mlp.close()
    net = runs[net_key]
    m = matched_linear_time(runs, net["rms_err_per_spin"])
    matched = {"network_rms": net["rms_err_per_spin"],
               "network_rms_se": net["rms_se"],
               "network_wall_s": net["wall_s"]}
    if m:
        matched.update({"linear_K_at_network_rms": m["K"],
                        "linear_wall_s_at_network_rms": m["wall_s"],
                        "linear_extrapolated": m["extrapolated"],
                        "speedup_vs_linear": m["wall_s"] / net["wall_s"]})
        # the same at the network's RMS error plus and minus one standard
        # error: how far the comparison moves within the noise
        for sgn, tag in ((1, "hi"), (-1, "lo")):
            mm = matched_linear_time(
                runs, net["rms_err_per_spin"] + sgn * net["rms_se"])
            if mm:
                matched["speedup_vs_linear_rms_%s" % tag] = (
                    mm["wall_s"] / net["wall_s"])
    tb = runs["bisection alpha*=%g tol=%g" % (target, tol)]
    matched["speedup_vs_tol_bisection"] = tb["wall_s"] / net["wall_s"]
    return {"workload": "%d independent ferromagnet populations, L=%d, R=%d, "
                        "theta=%d, beta 0->%g; error of ln Z per spin against "
                        "Kaufman's exact finite-torus value" % (M, L, R, theta,
                                                              beta_f),
            "lnZ_exact": exact, "training_pairs": int(len(X)),
            "training_s": t_train, "rng": ["word", "planes"][rng_mode],
            "runs": runs, "matched": matched}


def _find(path):
    """rocprofv3 output files ending in basename(path) anywhere under
    dirname(path) (the profiler writes them into a per-host folder)."""
    import glob
    d, name = os.path.split(path)
    return sorted(glob.glob(os.path.join(d, "**", "*" + name), recursive=True))


def summarize_profiles(trace_dir, fetch_dir, write_dir, workload, command):
    """Write profiles/ summaries from rocprofv3 CSV output: per-kernel
    durations (--kernel-trace --stats) and HBM traffic (--pmc FETCH_SIZE and
    --pmc WRITE_SIZE runs that also ran a 1 GiB device copy, whose counters
    calibrate the scale)."""
    import csv
    import glob

    def one(pattern):
        f = _find(pattern)
        if not f:
            raise SystemExit("no file matches " + pattern)
        return f[0]

    stats = list(csv.DictReader(open(one(os.path.join(trace_dir,
                                                       "kernel_stats.csv")))))
    per = {}
    for cnt, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = list(csv.DictReader(open(one(os.path.join(
            d, "counter_collection.csv")))))
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
    with open(traffic_file(workload), "w") as fh:
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
    # the sweep launches alone: the trace also holds the initial passes
    # (theta = 0) and the gather timing's single sweeps
    durs = []
    for f in _find(os.path.join(trace_dir, "kernel_trace.csv")):
        for r in csv.DictReader(open(f)):
            if r.get("Kernel_Name", "").startswith("k_lattice"):
                durs.append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    if durs:
        durs.sort()
        lines += ["", "k_lattice launch durations: median %.0f ns over %d "
                  "launches (the initial theta = 0 passes and the single "
                  "sweeps of the gather timing pull the average down)."
                  % (durs[len(durs) // 2], len(durs))]
    lines += ["", "HBM traffic of k_lattice per launch (counters scaled by "
              "a 1 GiB copy: FETCH_SIZE x%.3f, WRITE_SIZE x%.3f): fetch "
              "%.1f MB, write %.1f MB, total %.1f MB over %d launches." % (
                  per["FETCH_SIZE"][1], per["WRITE_SIZE"][1], fetch_b / 1e6,
                  write_b / 1e6, (fetch_b + write_b) / 1e6, len(lat_f))]
    with open(os.path.join(ROOT, "profiles", "kernels_%s.md" % workload),
              "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_valu(pmc_dir, run_json, trace_dir, workload, command,
                   kernel="k_lattice"):
    """profiles/k_lattice_<workload>_valu.json and a line in
    profiles/kernels_<workload>.md from a rocprofv3 --pmc run of
    `bench.py --profile-run` (SQ_INSTS_VALU and the other counters of the
    pass, summed over the k_lattice dispatches) and the run's own count of
    spin-flip attempts; the kernel durations come from a --kernel-trace run
    of the same command."""
    import csv
    import glob
    f = _find(os.path.join(pmc_dir, "counter_collection.csv"))
    if not f:
        raise SystemExit("no counter_collection.csv in " + pmc_dir)
    rows = list(csv.DictReader(open(f[0])))
    # the batched sweep: only the timed batch's dispatches, the ones after
    # the population-by-population leg (its last k_lattice); the tuners'
    # scratch batches run before that leg
    after = -1
    if kernel == "k_bsweep":
        after = max([int(r["Dispatch_Id"]) for r in rows
                     if r["Kernel_Name"].startswith("k_lattice")] or [-1])
    tot, disp = {}, set()
    for r in rows:
        if not r["Kernel_Name"].startswith(kernel):
            continue
        if after >= 0 and int(r["Dispatch_Id"]) <= after:
            continue
        disp.add(r.get("Dispatch_Id", r.get("Correlation_Id", "")))
        tot[r["Counter_Name"]] = tot.get(r["Counter_Name"], 0.0) + float(
            r["Counter_Value"])
    with open(run_json) as fh:
        run = json.loads(fh.read().strip().splitlines()[-1])
    att = run["attempts"]
    dur_ns = None
    if kernel == "k_bsweep":
        tr = _find(os.path.join(trace_dir, "kernel_trace.csv"))
        trows = list(csv.DictReader(open(tr[0]))) if tr else []
        cut = max([int(r["Dispatch_Id"]) for r in trows
                   if r["Kernel_Name"].startswith("k_lattice")] or [-1])
        for r in trows:
            if r["Kernel_Name"].startswith(kernel) and \
                    int(r["Dispatch_Id"]) > cut:
                dur_ns = (dur_ns or 0.0) + float(
                    int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    else:
        tf = _find(os.path.join(trace_dir, "kernel_stats.csv"))
        for r in csv.DictReader(open(tf[0])) if tf else []:
            if r["Name"].startswith(kernel):
                dur_ns = (dur_ns or 0.0) + float(r["TotalDurationNs"])
    out = {"workload": workload, "kernel": kernel,
           "kernel_sha256": kernel_hash(kernel), "dispatches": len(disp),
           "attempts": att, "counters": tot, "commands": command}
    if "SQ_INSTS_VALU" in tot:
        out["valu_lane_ops_per_attempt"] = tot["SQ_INSTS_VALU"] * 64.0 / att
    if "SQ_INSTS_SALU" in tot:
        out["salu_per_attempt_per_wave64"] = tot["SQ_INSTS_SALU"] * 64.0 / att
    if dur_ns and "SQ_INSTS_VALU" in tot:
        # a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles;
        # 1024 SIMDs at 2.4 GHz
        out["kernel_ns_total"] = dur_ns
        out["valu_issue_frac_at_2p4GHz"] = (
            tot["SQ_INSTS_VALU"] * 4.0 / 1024.0) / (dur_ns * 2.4)
        if "GRBM_GUI_ACTIVE" in tot:
            out["grbm_gui_active_per_ns"] = tot["GRBM_GUI_ACTIVE"] / dur_ns
    if dur_ns:
        out["attempts_per_ns"] = att / dur_ns
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(valu_file(workload, kernel), "w") as fh:
        json.dump(out, fh, indent=1)


def summarize_trace(trace_dir, name, command):
    """profiles/kernels_<name>.md from a rocprofv3 --kernel-trace --stats
    run: per-kernel calls and durations, with the command that made it."""
    import csv
    import glob
    f = _find(os.path.join(trace_dir, "kernel_stats.csv"))
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
    ap.add_argument("--workload", default="C3a", choices=sorted(W.CONFIGS))
    ap.add_argument("--rows-per-lane", type=int, default=0)
    ap.add_argument("--law", default="nearest",
                    choices=["nearest", "poisson", "systematic", "residual",
                             "multinomial"],
                    help="resampling law of the timed anneals")
    ap.add_argument("--rng", default="planes", choices=["word", "planes"],
                    help="random numbers of the sweep: one Philox word per "
                         "site, or bit planes (one block per 16 sites)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=24.0,
                    help="seconds of oracle work, split over its two legs")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the vector-ALU issue-rate probe")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the C2 and CP10 figures")
    ap.add_argument("--profile-run", action="store_true",
                    help="only --steps anneals with no timing events, then "
                         "a JSON line with their spin-flip attempts (for "
                         "rocprofv3 counter passes)")
    ap.add_argument("--summarize-valu", nargs=3,
                    metavar=("PMC_DIR", "RUN_JSON", "TRACE_DIR"),
                    help="write profiles/<kernel>_<workload>_valu.json")
    ap.add_argument("--valu-kernel", default="k_lattice",
                    help="kernel name prefix for --summarize-valu")
    ap.add_argument("--valu-command", default=None,
                    help="the profiled command, for --summarize-valu of "
                         "another run than --profile-run")
    ap.add_argument("--valu-tag", default=None,
                    help="workload name of that run (default --workload)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched comparison (for profiling)")
    ap.add_argument("--step-calls", action="store_true",
                    help="time the step-by-step calls (pa_resample, pa_sweep, "
                         "pa_observables per step) instead of pa_anneal")
    ap.add_argument("--no-tune-sweep", action="store_true",
                    help="batched runs at the default persistent-sweep shape "
                         "(no scratch-batch timing, e.g. under a profiler)")
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
    rng_flag = " --rng " + args.rng
    tag = args.workload + ("" if args.rng == "word" else "_planes")
    if args.summarize_valu:
        base = args.valu_command or (
            "python3 <repo>/bench.py --workload %s%s --profile-run "
            "--steps 1 --warmup 0" % (args.workload, rng_flag))
        cmd = ["cd /tmp && export TMPDIR=/tmp",
               "rocprofv3 --kernel-trace --stats -T -d <TRACE_DIR> -o run "
               "--output-format csv -- %s" % base,
               "rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_WAVES "
               "SQ_BUSY_CYCLES GRBM_GUI_ACTIVE -T -d <PMC_DIR> -o run "
               "--output-format csv -- %s > <RUN_JSON>" % base,
               "python3 bench.py --workload %s%s --valu-kernel %s%s "
               "--summarize-valu <PMC_DIR> <RUN_JSON> <TRACE_DIR>"
               % (args.workload, rng_flag, args.valu_kernel,
                  (" --valu-tag %s" % args.valu_tag) if args.valu_tag else "")]
        if args.valu_tag:
            tag = args.valu_tag
        summarize_valu(*args.summarize_valu, tag, cmd,
                       kernel=args.valu_kernel)
        return
    if args.summarize_profiles:
        base = ("python3 <repo>/bench.py --workload %s%s --no-cpu-baseline "
                "--no-batched --no-learned --no-accuracy --no-secondary "
                "--no-probe" % (args.workload, rng_flag))
        cmd = ["cd /tmp && export TMPDIR=/tmp",
               "rocprofv3 --kernel-trace --stats -T -d <TRACE_DIR> -o run "
               "--output-format csv -- %s --steps 2 --warmup 1" % base,
               "rocprofv3 --pmc FETCH_SIZE -T -d <FETCH_DIR> -o run "
               "--output-format csv -- %s --steps 1 --warmup 0 "
               "--calibrate-copy" % base,
               "rocprofv3 --pmc WRITE_SIZE -T -d <WRITE_DIR> -o run "
               "--output-format csv -- %s --steps 1 --warmup 0 "
               "--calibrate-copy" % base,
               "python3 bench.py --workload %s%s --summarize-profiles "
               "<TRACE_DIR> <FETCH_DIR> <WRITE_DIR>" % (args.workload,
                                                        rng_flag)]
        summarize_profiles(*args.summarize_profiles, tag, cmd)
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
    rng_mode = ["word", "planes"].index(args.rng)
    if args.batched_only:
        print(json.dumps(bench_batched(binding, stream,
                                       use_graph=not args.eager,
                                       rng_mode=rng_mode,
                                       tune_sweep=not args.no_tune_sweep)),
              flush=True)
        return
    if args.accuracy_only:
        print(json.dumps({
            "accuracy": bench_accuracy(binding, use_graph=not args.eager,
                                       label="L32", rng_mode=rng_mode),
            "accuracy_C2": bench_accuracy(
                binding, use_graph=not args.eager, M=16, L=64, R=65536,
                Ks=(50, 100, 200, 400),
                train_LR=((32, 48, 64), (4096, 16384, 65536)),
                label="C2", rng_mode=rng_mode)}), flush=True)
        return
    law = ["nearest", "poisson", "systematic", "residual",
           "multinomial"].index(args.law)
    cfg = dict(W.CONFIGS[args.workload])
    cfg["name"] = args.workload
    cfg["law"] = law
    cfg["rng_mode"] = ["word", "planes"].index(args.rng)
    if args.calibrate_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.profile_run:
        att = 0
        for _ in range(args.steps):
            att += run_anneal(binding, cfg, stream,
                              rows_per_lane=args.rows_per_lane,
                              step_calls=args.step_calls)[0]
        torch.cuda.synchronize()
        print(json.dumps({"workload": args.workload, "anneals": args.steps,
                          "attempts": att}), flush=True)
        return

    head = time_workload(binding, cfg, stream, args.steps, args.warmup,
                         args.rows_per_lane, verbose=True,
                         step_calls=args.step_calls)
    dt = head["seconds"]
    # every kernel class timed, on one more anneal after the timed region
    fam = {}
    _, _, tall = run_anneal(binding, cfg, stream, timing=binding.KERNEL_CLASSES,
                            rows_per_lane=args.rows_per_lane, families=fam,
                            step_calls=args.step_calls)
    res_k = ("hist", "counts", "scatter", "gather")
    res_ms = sum(tall[k]["ms"] for k in res_k)
    res_bytes = sum(tall[k]["bytes"] for k in res_k)
    res_gbps = res_bytes / (res_ms * 1e6) if res_ms > 0 else 0.0
    sw_all = tall["sweep"]
    # the replica copies of every resampling happen inside the sweep kernel
    # (each new slot loaded from its parent): its read + write of the whole
    # population per launch against HBM
    copy_gbps = sw_all["bytes"] / (sw_all["ms"] * 1e6) if sw_all["ms"] else 0.0
    progress("resampling kernels timed: %.2f ms per anneal" % res_ms)

    roof = head["roofline"]
    tag = args.workload + ("" if cfg["rng_mode"] == 0 else "_planes")
    roof["traffic"] = measured_traffic(tag)
    roof["valu_lane_ops_per_attempt_counted"] = measured_valu(tag)
    if not args.no_probe:
        roof["valu_probe"] = valu_probe()
        progress("VALU probe done")
    out = {
        "metric": METRIC,
        "value": head["value"],
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
            "workload": describe(args.workload, cfg),
            "L": cfg["L"], "R": cfg["R"], "K": cfg["K"],
            "theta": cfg["theta"], "layout": cfg["layout"],
            "resampling": args.law,
            "rng": args.rng,
        },
        "roofline": roof,
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
        "lnZ_final": head["lnZ"],
        # descendants of the initial replicas at beta_f (the untimed anneal)
        "families_final": fam,
    }
    if not args.no_secondary:
        # the headline workload in the other random-number stream, and the
        # L = 128 paper-scale population (R = 2^18, bit-packed), the int8
        # workload and the paper's per-GPU shape in the headline's
        sec = {}
        other = 1 - cfg["rng_mode"]
        todo = [(args.workload, other, False)] + [
            (n, cfg["rng_mode"], False) for n in ("C3b", "C2", "CP10", "CP1")
            if n != args.workload]
        # the paper's theta = 1 shape also through the step-by-step calls
        todo.append(("CP1", cfg["rng_mode"], True))
        for name, rm, calls in todo:
            c2 = dict(W.CONFIGS[name])
            c2["name"] = name
            c2["law"] = law
            c2["rng_mode"] = rm
            reps = 2 if c2["R"] > (1 << 20) else 3
            r = time_workload(binding, c2, stream, reps, 1, 0,
                              step_calls=calls)
            r["roofline"]["traffic"] = measured_traffic(
                name + ("" if rm == 0 else "_planes"))
            key = "%s_%s%s" % (name, ["word", "planes"][rm],
                               "_step_calls" if calls else "")
            sec[key] = {"workload": describe(name, c2), "value": r["value"],
                        "ms_per_anneal": r["seconds"] * 1e3 / reps,
                        "roofline": r["roofline"], "lnZ_final": r["lnZ"]}
            progress("secondary %s: %.1f attempts/ns" % (key, r["value"]))
        out["secondary"] = sec
    if not args.no_batched:
        out["batched"] = bench_batched(binding, stream,
                                       use_graph=not args.eager,
                                       rng_mode=cfg["rng_mode"])
        progress("batched comparison done")
    if not args.no_learned:
        out["learned"] = bench_learned(binding, use_graph=not args.eager,
                                       rng_mode=cfg["rng_mode"])
        progress("learned comparison done")
    if not args.no_accuracy:
        out["accuracy"] = bench_accuracy(binding, use_graph=not args.eager,
                                         label="L32",
                                         rng_mode=cfg["rng_mode"])
        progress("accuracy comparison done")
        # the same comparison on C2-shaped populations
        out["accuracy_C2"] = bench_accuracy(
            binding, use_graph=not args.eager, M=16, L=64, R=65536,
            Ks=(50, 100, 200, 400),
            train_LR=((32, 48, 64), (4096, 16384, 65536)), label="C2",
            rng_mode=cfg["rng_mode"])
        progress("C2-shape accuracy comparison done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_budget)
        progress("cpu baseline done")
    print(json.dumps(out), flush=True)


def progress(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def describe(name, cfg):
    return ("%s: 2D %s ferromagnet L=%d periodic, R=%d, %s spins, beta "
            "0->%g in %d linear steps, theta=%d, seed %d, %s random numbers; "
            "one step = one full anneal"
            % (name, ("%d-state Potts" % cfg["q"]) if cfg.get("q") else
               "Ising", cfg["L"], cfg["R"], cfg["layout"], cfg["beta_f"],
               cfg["K"], cfg["theta"], cfg["seed"],
               "bit-plane" if cfg.get("rng_mode") else "one Philox word per "
               "site"))


# In the timed anneals the sweep launches are timed with HIP events on a
# systematic sample, the first and then every tenth: each timed launch adds
# two event markers to the stream, which at theta = 1 would lengthen a step
# of about 65 us by several microseconds.
SWEEP_TIMING_EVERY = 10


def time_workload(binding, cfg, stream, steps, warmup, rows_per_lane,
                  verbose=False, step_calls=False):
    """`warmup` untimed anneals, then `steps` timed ones between device
    synchronisations, with HIP events around each sweep launch on the
    library's stream.  Returns the whole-anneal rate, the wall seconds of
    the timed anneals and the sweep kernel against its roofline."""
    import torch
    for i in range(warmup):
        run_anneal(binding, cfg, stream, rows_per_lane=rows_per_lane,
                   step_calls=step_calls)
        if verbose:
            progress("warmup anneal %d/%d" % (i + 1, warmup))
    torch.cuda.synchronize()
    total_attempts = 0
    tsum = None
    lnZ = None
    t0 = time.perf_counter()
    for i in range(steps):
        # events on the sweep launches only (two markers per timed launch)
        a, lnZ, t = run_anneal(binding, cfg, stream, timing=("sweep",),
                               rows_per_lane=rows_per_lane,
                               step_calls=step_calls,
                               timing_every=SWEEP_TIMING_EVERY)
        total_attempts += a
        if tsum is None:
            tsum = t
        else:
            for k in binding.KERNEL_CLASSES:
                for f in ("ms", "launches", "bytes"):
                    tsum[k][f] += t[k][f]
            tsum["attempts"] += t["attempts"]
        if verbose:
            progress("timed anneal %d/%d" % (i + 1, steps))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sw = tsum["sweep"]
    sweep_avg_ms = sw["ms"] / max(1, sw["launches"])
    sweep_rate = tsum["attempts"] / (sw["ms"] * 1e6)       # attempts/ns
    work = ALGO_WORK_POTTS if cfg.get("q") else ALGO_WORK[
        ["word", "planes"][cfg.get("rng_mode", 0)]]
    ops = mad_equivalents(work)
    achieved = tsum["attempts"] / sw["launches"] * ops / (
        sweep_avg_ms * 1e-3) / 1e12
    peak = VALU_OPS_PER_S / 1e12
    L = cfg["L"]
    return {
        "value": total_attempts / (dt * 1e9), "seconds": dt, "lnZ": lnZ,
        "roofline": {
            "kernel": (("k_potts_swar" if L in (8, 16, 32, 64, 128)
                        else "k_potts") if cfg.get("q") else "k_lattice") +
                      " (theta fused Metropolis sweeps)",
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "T multiply-equivalent VALU ops/s (64-bit-product "
                    "multiply 1, plain 32-bit op 1/2)",
            "frac": achieved / peak,
            "traffic": None,
            "sweep_attempts_per_ns": sweep_rate,
            "sweep_avg_ms": sweep_avg_ms,
            "sweep_launches": sw["launches"],
            "sweep_timing_sample_every": SWEEP_TIMING_EVERY,
            "ops_per_attempt": ops,
            "algorithmic_multiplies_and_plain_ops_per_attempt": list(work),
            "rng": ["word", "planes"][cfg.get("rng_mode", 0)],
        }}


# VALU instructions per lane and round of the probe kernels (from the gfx950
# assembly of libpa_probe.so: 128 three-input xors + 8, 128 v_mad_u64_u32 +
# 2, 8 Philox blocks = 331)
PROBE_VALU = {0: 136, 1: 130, 3: 331}


def valu_probe(stream=None):
    """Measured issue rates of the vector ALU: lane operations per second of
    the three-input xor, the 64-bit-product multiply-add and the Philox
    block mix, each as 8192 workgroups of 256 lanes."""
    import ctypes as C
    path = os.path.join(ROOT, "paper_2006_00561_amd", "libpa_probe.so")
    lib = C.CDLL(path)
    lib.pa_probe_valu.argtypes = [C.c_int32, C.c_int32, C.c_int32,
                                  C.c_void_p, C.POINTER(C.c_double)]
    out = {}
    for kind, name in ((0, "xor3"), (1, "mad_u64_u32"), (3, "philox")):
        blocks, iters = 8192, (2000 if kind != 3 else 800)
        ms = C.c_double()
        rc = lib.pa_probe_valu(kind, blocks, iters, stream, C.byref(ms))
        if rc != 0:
            raise RuntimeError("VALU probe failed: %d" % rc)
        instr = blocks * 4.0 * iters * PROBE_VALU[kind]
        out[name] = {"lane_ops_per_s": instr * 64 / (ms.value * 1e-3),
                     "wave64_instr_per_simd_cycle_at_2p4GHz":
                         instr / 1024 / (ms.value * 1e-3 * 2.4e9)}
    return out


if __name__ == "__main__":
    main()
