"""Parity of the schedule run on the device (pa_anneal) with the oracle.

pa_anneal runs every step of a cooling schedule with the nearest-integer
law without a host stop: the histogram's last workgroup builds the step's
tables.  The bar is the one of the step-by-step calls: sizes, spins,
energies, magnetisations, families and copy counts bit-exact; ln Q and ln Z
identical (the device sums S in the host tables' order and the host takes
the logarithm), observables from exact sums.  The failed steps (capacity,
empty population) must leave the context as the failed pa_resample does."""
import os

import numpy as np
import pytest

import oracle
import pa_workloads as W
from test_gpu_parity import _close, _cmp_obs, _cmp_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pa():
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU")
    from paper_2006_00561_amd import binding
    binding.lib()
    return binding


def _run_oracle(o, sched, theta):
    """The oracle step by step: per step its size, ln Q and observables."""
    out = []
    for b in sched:
        Rn = o.resample(b)
        o.sweep(theta)
        out.append((Rn, o.free_energy()[1], o.observables()))
    return out


SCHEDULES = [
    # L, R, layout, rows per lane, glass, rng mode, theta, K, beta_f, q, cap
    (16, 1000, 0, 0, False, 0, 5, 100, 1.0, 0, 0),      # C1, every step
    (12, 513, 1, 0, True, 0, 2, 20, 1.5, 0, 0),
    (32, 300, 1, 4, False, 1, 3, 15, 0.9, 0, 0),
    (64, 129, 0, 0, False, 1, 2, 10, 0.6, 0, 0),
    (64, 70, 1, 2, True, 1, 2, 8, 0.8, 0, 0),
    (128, 40, 1, 0, False, 0, 1, 6, 0.5, 0, 0),          # histogram window
    (8, 70000, 0, 0, False, 0, 1, 4, 0.4, 0, 0),         # 294 tiles
    (16, 2000, 0, 0, False, 1, 2, 12, 1.0, 0, 8192),     # roomy capacity
    (16, 400, 0, 0, False, 0, 2, 10, 1.2, 3, 0),         # Potts q = 3
    (10, 300, 0, 0, False, 0, 3, 8, 1.5, 5, 0),
]


@pytest.mark.parametrize("L,R,layout,rpl,glass,rng,theta,K,beta_f,q,cap",
                         SCHEDULES)
def test_anneal_matches_oracle(pa, L, R, layout, rpl, glass, rng, theta, K,
                               beta_f, q, cap):
    print("anneal L=%d R=%d layout=%d rpl=%d glass=%s rng=%d theta=%d K=%d "
          "q=%d cap=%d" % (L, R, layout, rpl, glass, rng, theta, K, q, cap),
          flush=True)
    J = W.pmj_couplings(L, 200 + L) if glass else None
    seed = 11 + L
    g = pa.Population(L, R, seed=seed, J=J, layout=layout, rows_per_lane=rpl,
                      rng_mode=rng, q=q, capacity=cap)
    o = oracle.OraclePA(L, R, seed=seed, J=J, q=q,
                        rng_mode=oracle.RNG_PLANES if rng else
                        oracle.RNG_WORD)
    sched = W.linear_schedule(beta_f, K)
    obs_g, q_g = g.anneal(sched, theta)
    ref = _run_oracle(o, sched, theta)
    assert len(obs_g) == K and len(q_g) == K
    for i, (Rn, lnQ, oo) in enumerate(ref):
        assert obs_g[i]["R"] == Rn, i
        assert q_g[i] == lnQ, (i, q_g[i], lnQ)
        _cmp_obs(obs_g[i], oo)
    assert g.state() == (ref[-1][0], sched[-1], K)
    _cmp_state(g, o, "end")
    # the copy counts of the last step, against the oracle's
    assert np.array_equal(g.counts(), o.counts(ref[-2][0] if K > 1 else R))
    # the step-by-step calls continue from where the schedule ended
    b = sched[-1] + 0.05
    assert g.resample(b) == o.resample(b)
    g.sweep(b, theta)
    o.sweep(theta)
    _cmp_state(g, o, "after")
    g.close()
    o.close()


def test_anneal_in_pieces_and_timing(pa):
    """A schedule in several calls equals one call, and the sweep timing
    counts every attempt with the size each sweep acted on."""
    L, R, theta = 24, 700, 2
    sched = W.linear_schedule(1.0, 12)
    g = pa.Population(L, R, seed=4)
    h = pa.Population(L, R, seed=4)
    g.set_timing(True, classes=("sweep", "hist", "counts", "scatter"))
    obs_g, q_g = g.anneal(sched, theta)
    obs_h, q_h = [], []
    for part in (sched[:1], sched[1:5], sched[5:]):
        a, b = h.anneal(part, theta)
        obs_h += a
        q_h += b
    assert q_g == q_h
    for a, b in zip(obs_g, obs_h):
        assert a == b
    for x, y in zip(g.population(), h.population()):
        assert np.array_equal(x, y)
    assert g.free_energy() == h.free_energy()
    t = g.timing()
    assert t["sweep"]["launches"] == 12 and t["hist"]["launches"] == 13
    # counts, scan and parent map are one single-pass launch per step
    assert t["counts"]["launches"] == 12 and t["scatter"]["launches"] == 0
    assert t["attempts"] == sum(o["R"] for o in obs_g) * L * L * theta
    # a systematic sample of the launches: the first, then every fifth
    s = pa.Population(L, R, seed=4)
    s.set_timing(True, classes=("sweep",), every=5)
    obs_s, _ = s.anneal(sched, theta)
    ts = s.timing()
    assert ts["sweep"]["launches"] == 3
    assert ts["attempts"] == sum(obs_s[i]["R"] for i in (0, 5, 10)) * \
        L * L * theta
    with pytest.raises(pa.PAError):
        s.set_timing(True, classes=("sweep",), every=0)
    g.close()
    h.close()
    s.close()


def test_anneal_on_reused_memory(pa):
    """A context made after another was freed may get its memory back, with
    the single-pass scan's status words of that context's launches in it;
    the new schedule must not read them (it equals the first one)."""
    L, R, theta = 32, 30000, 1
    sched = W.linear_schedule(1.0, 40)
    runs = []
    for _ in range(3):
        g = pa.Population(L, R, seed=21)
        obs, q = g.anneal(sched, theta)
        runs.append(([o["R"] for o in obs], q, g.free_energy(),
                     g.energies()))
        g.close()
    for r in runs[1:]:
        assert r[0] == runs[0][0] and r[1] == runs[0][1]
        assert r[2] == runs[0][2]
        assert np.array_equal(r[3][0], runs[0][3][0])


def test_anneal_capacity_stop_matches_step_calls(pa):
    """A size above the capacity stops the schedule at that step with the
    context as the failed pa_resample leaves it; calls continue from it."""
    L, R, theta, K = 6, 400, 1, 30
    sched = W.linear_schedule(1.5, K)
    for seed in range(1, 80):
        o = oracle.OraclePA(L, R, seed=seed)
        sizes = [r[0] for r in _run_oracle(o, sched, theta)]
        o.close()
        top = max(sizes)
        k_fail = sizes.index(top)
        if top - 1 < R or k_fail == 0:
            continue
        cap = top - 1
        print("capacity stop seed=%d cap=%d step=%d" % (seed, cap, k_fail),
              flush=True)
        g = pa.Population(L, R, seed=seed, capacity=cap)
        rc, done, obs, q = g.anneal_rc(sched, theta)
        assert rc == pa.PA_ECAPACITY and done == k_fail
        assert [x["R"] for x in obs] == sizes[:k_fail]
        h = pa.Population(L, R, seed=seed, capacity=cap)
        for b in sched[:k_fail]:
            h.resample(b)
            h.sweep(b, theta)
        rc2, Rn = h.resample_rc(sched[k_fail])
        assert rc2 == pa.PA_ECAPACITY and Rn == top
        assert g.state() == h.state()
        for x, y in zip(g.population(), h.population()):
            assert np.array_equal(x, y)
        assert np.array_equal(g.families()[0], h.families()[0])
        assert g.free_energy() == h.free_energy()
        # the same step fails again, at once, and changes nothing
        rc, done, _, _ = g.anneal_rc(sched[k_fail:], theta)
        assert rc == pa.PA_ECAPACITY and done == 0
        assert g.state() == h.state()
        # a smaller step from there goes on like the step-by-step calls
        b = sched[k_fail - 1] + 1e-4
        rg, dg, og, qg = g.anneal_rc([b], theta)
        Rh = h.resample(b)
        h.sweep(b, theta)
        assert rg == pa.PA_OK and dg == 1 and og[0]["R"] == Rh
        assert qg[0] == h.free_energy()[1]
        for x, y in zip(g.population(), h.population()):
            assert np.array_equal(x, y)
        g.close()
        h.close()
        return
    raise AssertionError("no seed overflowed")


def test_anneal_empty_stop(pa):
    """L = 4, R_target = 2, seed 233: the oracle's population dies out at the
    fourth step of beta 0 -> 2 in 8 steps (theta = 1); the schedule stops
    there with PA_EEMPTY and the population of the step before."""
    L, R, seed, theta = 4, 2, 233, 1
    sched = W.linear_schedule(2.0, 8)
    o = oracle.OraclePA(L, R, seed=seed)
    for b in sched[:3]:
        o.resample(b)
        o.sweep(theta)
    assert o.resample_rc(sched[3]) == (oracle.EEMPTY, 0)
    g = pa.Population(L, R, seed=seed)
    rc, done, obs, q = g.anneal_rc(sched, theta)
    assert rc == pa.PA_EEMPTY and done == 3
    _cmp_state(g, o, "emptied")
    g.close()
    o.close()


@pytest.mark.parametrize("law", [1, 2, 4])
def test_anneal_other_laws_run_step_calls(pa, law):
    """Laws other than the nearest-integer one run the step-by-step calls:
    the same results as the oracle's."""
    L, R, theta = 12, 300, 2
    sched = W.linear_schedule(0.9, 6)
    g = pa.Population(L, R, seed=8, resampling=law)
    o = oracle.OraclePA(L, R, seed=8, law=law)
    obs_g, q_g = g.anneal(sched, theta)
    for i, (Rn, lnQ, oo) in enumerate(_run_oracle(o, sched, theta)):
        assert obs_g[i]["R"] == Rn and _close(q_g[i], lnQ)
        _cmp_obs(obs_g[i], oo)
    _cmp_state(g, o, "law %d" % law)


def test_anneal_heating_and_zero_sweeps(pa):
    """Heating steps and theta = 0 take the step-by-step calls too."""
    L, R = 16, 300
    g = pa.Population(L, R, seed=3)
    o = oracle.OraclePA(L, R, seed=3)
    g.start_heating(2.0)
    o.start_heating(2.0)
    sched = [1.9, 1.8, 1.7]
    obs_g, q_g = g.anneal(sched, 2)
    for i, (Rn, lnQ, oo) in enumerate(_run_oracle(o, sched, 2)):
        assert obs_g[i]["R"] == Rn and _close(q_g[i], lnQ)
    _cmp_state(g, o, "heated")
    h = pa.Population(L, R, seed=5)
    p = oracle.OraclePA(L, R, seed=5)
    obs_h, _ = h.anneal([0.1, 0.2], 0)
    for i, b in enumerate((0.1, 0.2)):
        assert obs_h[i]["R"] == p.resample(b)
    _cmp_state(h, p, "theta 0")


def test_anneal_argument_checks(pa):
    g = pa.Population(8, 50, seed=1)
    for betas, theta in (([0.1], -1), ([0.1], 40000), ([float("nan")], 1),
                         ([-0.5], 1)):
        rc, done, _, _ = g.anneal_rc(betas, theta)
        assert rc == pa.PA_EINVAL and done == 0
    rc, done, _, _ = g.anneal_rc([], 1)
    assert rc == pa.PA_OK and done == 0
    assert g.state() == (50, 0.0, 0)


@pytest.mark.parametrize("name,start,rng", [
    ("CP1", 1, 1), ("CP1", 88, 1), ("C2", 88, 1), ("C2", 2, 0),
    # the paper's total population on one device, bit-packed: 8192 tiles,
    # so the counts, scan and parent map are three kernels
    ("C3a", 1, 1), ("C3a", 88, 1)])
def test_anneal_full_size_sampled(pa, name, start, rng):
    """At the benchmark sizes, in the benchmark's configuration: the
    schedule runs on the device up to step start - 1; then one more step of
    it, checked like the step-by-step path (every copy count, R_new and
    ln Q from the oracle's count step on the device energies, families, a
    sample of new replicas through their sweeps)."""
    c = W.CONFIGS[name]
    L, R, theta = c["L"], c["R"], c["theta"]
    layout = 1 if c["layout"] == "bits" else 0
    print("anneal full size %s start=%d rng=%d" % (name, start, rng),
          flush=True)
    g = pa.Population(L, R, seed=c["seed"], layout=layout, rng_mode=rng)
    sched = W.linear_schedule(c["beta_f"], c["K"])
    if start > 1:
        g.anneal(sched[:start - 1], theta)
    fam, _ = g.families()
    zlast = g.free_energy()[0]
    b = sched[start - 1]
    E, M = g.energies()
    n_o, Rn_o, lnQ_o = oracle.counts(L * L, E, R, b - g.beta, c["seed"], 0,
                                     start)
    parent = np.repeat(np.arange(len(E)), n_o)
    gen = np.random.default_rng(start)
    slots = np.sort(gen.choice(Rn_o, size=32, replace=False))
    s_pre, E_pre, M_pre = g.replicas(parent[slots])
    obs, q = g.anneal([b], theta)
    assert obs[0]["R"] == Rn_o and g.state()[0] == Rn_o
    assert np.array_equal(g.counts(), n_o)
    assert np.array_equal(g.families()[0], fam[parent])
    assert _close(q[0], lnQ_o)
    assert _close(g.free_energy()[0], zlast + lnQ_o)
    s_post, E_post, M_post = g.replicas(slots)
    rng_o = oracle.RNG_PLANES if rng else oracle.RNG_WORD
    for k, j in enumerate(slots):
        so, eo, mo = oracle.sweep_replica(s_pre[k], E_pre[k], M_pre[k], b,
                                          c["seed"], 0, start, 0, theta,
                                          int(j), rng_mode=rng_o)
        assert np.array_equal(s_post[k], so), (name, start, j)
        assert E_post[k] == eo and M_post[k] == mo
    g.close()


@pytest.mark.parametrize("name", ["CP1", "C2", "C3a"])
def test_anneal_whole_schedule_equals_step_calls(pa, name):
    """The whole benchmark schedule: pa_anneal and the step-by-step calls
    (whose full-size steps are checked against the oracle elsewhere) end in
    the same population, families and ln Z, bit for bit, through the same
    sizes and ln Q at every step."""
    c = W.CONFIGS[name]
    L, R, theta = c["L"], c["R"], c["theta"]
    layout = 1 if c["layout"] == "bits" else 0
    sched = W.linear_schedule(c["beta_f"], c["K"])
    print("anneal whole schedule %s" % name, flush=True)
    g = pa.Population(L, R, seed=c["seed"], layout=layout, rng_mode=1)
    obs, q = g.anneal(sched, theta)
    h = pa.Population(L, R, seed=c["seed"], layout=layout, rng_mode=1,
                      capacity=W.deferral_capacity(R))
    for i, b in enumerate(sched):
        h.resample(b, wait=False)
        h.sweep(b, theta)
        if i % 50 == 49 or i == len(sched) - 1:
            oh = h.observables()
            assert oh == obs[i], i
            assert h.free_energy()[1] == q[i], i
    assert g.free_energy() == h.free_energy()
    Eg, Mg = g.energies()
    Eh, Mh = h.energies()
    assert np.array_equal(Eg, Eh) and np.array_equal(Mg, Mh)
    assert np.array_equal(g.families()[0], h.families()[0])
    g.close()
    h.close()


def test_anneal_zero_steps_and_repeated_betas(pa):
    """dbeta = 0 (weights all exp(-0) = 1): a step at the current beta keeps
    every replica once when R = R_target, also in the middle of a schedule
    that repeats a beta; the whole run equals the oracle's."""
    L, R, theta = 12, 300, 2
    g = pa.Population(L, R, seed=17)
    o = oracle.OraclePA(L, R, seed=17)
    obs, q = g.anneal([0.0], theta)
    assert obs[0]["R"] == R and q[0] == 0.0
    assert np.all(g.counts() == 1)
    o.resample(0.0)
    o.sweep(theta)
    sched = [0.2, 0.2, 0.5, 0.5, 0.5, 0.9]
    obs_g, q_g = g.anneal(sched, theta)
    for i, (Rn, lnQ, oo) in enumerate(_run_oracle(o, sched, theta)):
        assert obs_g[i]["R"] == Rn and q_g[i] == lnQ, i
        _cmp_obs(obs_g[i], oo)
    _cmp_state(g, o, "repeated betas")
    g.close()
    o.close()


@pytest.mark.parametrize("L,R", [(4, 1), (4, 255), (6, 256), (8, 257),
                                 (4, 3000)])
def test_anneal_tile_edges_and_smallest_lattice(pa, L, R):
    """Populations of one replica, one tile less one, one tile, one tile plus
    one, and the smallest lattice with many tiles, each for a one-step and a
    longer schedule."""
    print("anneal edges L=%d R=%d" % (L, R), flush=True)
    for K in (1, 9):
        sched = W.linear_schedule(1.5, K)
        g = pa.Population(L, R, seed=5 + K)
        o = oracle.OraclePA(L, R, seed=5 + K)
        obs_g, q_g = g.anneal(sched, 3)
        for i, (Rn, lnQ, oo) in enumerate(_run_oracle(o, sched, 3)):
            assert obs_g[i]["R"] == Rn and q_g[i] == lnQ, (K, i)
            _cmp_obs(obs_g[i], oo)
        _cmp_state(g, o, "L=%d R=%d K=%d" % (L, R, K))
        g.close()
        o.close()
