"""Randomised parity: seeded random combinations of lattice size, population,
layout, sweep shape, model (ferromagnet, +-J glass, q-state Potts), resampling
law, sweeps per step, cooling or heating, capacity, waiting or deferred
population sizes and reads of the population between a resampling and its
sweep.  Every step is compared with the oracle bit for bit (spins, E, M,
copy counts, families) and to 1e-12 for ln Z and the observables.  Random
batches of mixed populations are compared with each population's single
run, which the oracle pins."""
import os

import numpy as np
import pytest

import oracle
import pa_workloads as W

pytestmark = pytest.mark.gpu

REL = 1e-12


def _close(a, b):
    return abs(a - b) <= REL * max(1.0, abs(a), abs(b))


def _configs(n=120, seed=20061):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        model = ["ferro", "glass", "potts"][int(rng.integers(0, 3))]
        L = int(rng.choice([4, 6, 8, 10, 12, 16, 24, 32, 48]))
        if model == "potts":
            L = int(rng.choice([6, 8, 12, 16, 32]))
        R = int(rng.integers(20, 700))
        layout = 0 if model == "potts" else int(rng.integers(0, 2))
        rpl = int(rng.choice([0, 1, 2, 3, 4]))
        if rpl and (L % rpl or L // rpl > 64):
            rpl = 0
        out.append(dict(
            k=k, model=model, L=L, R=R, layout=layout, rpl=rpl,
            q=int(rng.integers(2, 17)) if model == "potts" else 0,
            law=int(rng.integers(0, 5)), steps=int(rng.integers(3, 8)),
            beta_f=float(rng.uniform(0.3, 2.0)),
            heating=bool(model != "glass" and rng.random() < 0.25),
            big_cap=bool(rng.random() < 0.5),
            seed=int(rng.integers(1, 1 << 30)), pop=int(rng.integers(0, 50)),
            plan=[(int(rng.integers(0, 4)), bool(rng.random() < 0.5),
                   bool(rng.random() < 0.3)) for _ in range(8)]))
    return out


CONFIGS = _configs()


@pytest.fixture(scope="module")
def pa():
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU")
    from paper_2006_00561_amd import binding
    binding.lib()
    return binding


def _cmp(g, o, tag):
    sg, Eg, Mg = g.population()
    so, Eo, Mo = o.population()
    assert np.array_equal(Eg, Eo) and np.array_equal(Mg, Mo), tag
    assert np.array_equal(sg, so), tag
    fg, n0g = g.families()
    fo, n0o = o.families()
    assert n0g == n0o and np.array_equal(fg, fo), tag
    zg, qg = g.free_energy()
    zo, qo = o.free_energy()
    assert _close(zg, zo) and _close(qg, qo), (tag, zg, zo)


@pytest.mark.parametrize("c", CONFIGS, ids=lambda c: "cfg%02d" % c["k"])
def test_random_configuration_matches_oracle(pa, c):
    print("random config", c, flush=True)
    L, R = c["L"], c["R"]
    J = W.pmj_couplings(L, 500 + c["k"]) if c["model"] == "glass" else None
    cap = W.deferral_capacity(R) if c["big_cap"] else 0
    g = pa.Population(L, R, seed=c["seed"], population_id=c["pop"], J=J,
                      layout=c["layout"], rows_per_lane=c["rpl"],
                      resampling=c["law"], q=c["q"], capacity=cap)
    o = oracle.OraclePA(L, R, seed=c["seed"], pop=c["pop"], J=J, law=c["law"],
                        q=c["q"], capacity=cap)
    if c["heating"]:
        b0 = c["beta_f"] + 1.0
        g.start_heating(b0)
        o.start_heating(b0)
        betas = W.linear_schedule(c["beta_f"] / 3, c["steps"], beta0=b0)
    else:
        betas = W.linear_schedule(c["beta_f"], c["steps"])
    _cmp(g, o, "start")
    for i, b in enumerate(betas, start=1):
        theta, wait, peek = c["plan"][(i - 1) % len(c["plan"])]
        R_old = g.R
        ro_rc, ro = o.resample_rc(b)
        if ro_rc != oracle.OK:
            # both sides refuse the step and keep the population
            rg_rc, rg = g.resample_rc(b)
            assert rg_rc == ro_rc
            break
        if wait:
            assert g.resample(b) == ro, i
        else:
            g.resample(b, wait=False)
        if peek:
            # a read before the sweep makes the copies with the gather
            E, _ = g.energies()
            assert np.array_equal(E, o.population()[1]), i
        assert np.array_equal(g.counts(), o.counts(R_old)), i
        g.sweep(b, theta)
        o.sweep(theta)
        _cmp(g, o, "step %d" % i)
        og, oo = g.observables(), o.observables()
        for k in ("R", "sumE", "sumE2", "sumAbsM", "sumM2", "Emin", "Emax"):
            assert og[k] == oo[k], (i, k)
        for k in ("e", "abs_m", "m2", "C"):
            assert _close(og[k], oo[k]), (i, k)
    g.close()
    o.close()


def _batches(n=8, seed=4242):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        pops = []
        for i in range(int(rng.integers(2, 8))):
            model = ["ferro", "glass", "potts"][int(rng.integers(0, 3))]
            if model == "potts":
                L = int(rng.choice([8, 16, 32, 64]))
                pop = dict(L=L, q=int(rng.integers(2, 17)))
            else:
                L = int(rng.choice([4, 6, 8, 12, 16, 24, 32, 48, 64]))
                rpl = int(rng.choice([0, 1, 2, 3, 4]))
                if rpl and (L % rpl or L // rpl > 64):
                    rpl = 0
                pop = dict(L=L, layout=int(rng.integers(0, 2)),
                           rows_per_lane=rpl)
                if model == "glass":
                    pop["J"] = W.pmj_couplings(L, 900 + 10 * k + i)
            pop.update(R=int(rng.integers(30, 600)),
                       seed=int(rng.integers(1, 1 << 30)),
                       population_id=int(rng.integers(0, 1000)))
            pops.append(pop)
        out.append(dict(k=k, pops=pops, steps=int(rng.integers(3, 9)),
                        theta=int(rng.integers(1, 4)),
                        beta_f=float(rng.uniform(0.4, 1.5)),
                        autotune=bool(rng.random() < 0.5)))
    return out


BATCHES = _batches()


@pytest.mark.parametrize("c", BATCHES, ids=lambda c: "batch%d" % c["k"])
def test_random_batch_matches_single_runs(pa, c):
    print("random batch", c["k"], [(p["L"], p["R"], p.get("q", 0),
                                   "J" in p) for p in c["pops"]],
          flush=True)
    betas = np.array(W.linear_schedule(c["beta_f"], c["steps"]))
    b = pa.Batch(c["pops"], autotune=c["autotune"])
    b.run(betas, c["theta"], use_graph=True)
    for p, pop in enumerate(c["pops"]):
        g = pa.Population(pop["L"], pop["R"], seed=pop["seed"],
                          population_id=pop["population_id"],
                          J=pop.get("J"), q=pop.get("q", 0),
                          layout=pop.get("layout", 0))
        for beta in betas:
            g.resample(beta)
            g.sweep(beta, c["theta"])
        sg, Eg, Mg = g.population()
        sb, Eb, Mb = b.population(p)
        assert np.array_equal(Eg, Eb) and np.array_equal(Mg, Mb), p
        assert np.array_equal(sg, sb), p
        assert g.free_energy()[0] == b.state(p)[3], p
        assert np.array_equal(g.families()[0], b.families(p)[0]), p
        g.close()
    b.close()
