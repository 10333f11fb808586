"""Failure handling forced from the host (the PA_FAULT injector) and the
per-step JSONL log (PA_LOG_JSONL): every kernel still runs to its normal
end; the tests check the error codes, that a failed call leaves the
population and ln Z as they were, and that the log records what the C ABI
reports."""
import json
import os

import numpy as np
import pytest

import pa_workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pa():
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU")
    from paper_2006_00561_amd import binding
    binding.lib()
    return binding


@pytest.fixture
def env():
    keep = {k: os.environ.get(k) for k in ("PA_FAULT", "PA_LOG_JSONL")}
    yield os.environ
    for k, v in keep.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


def test_allocation_failure_is_reported_and_leaves_nothing(pa, env):
    env["PA_FAULT"] = "alloc"
    for _ in range(3):
        with pytest.raises(pa.PAError) as e:
            pa.Population(16, 500, seed=1)
        assert e.value.code == pa.PA_ENOMEM
    del env["PA_FAULT"]
    g = pa.Population(16, 500, seed=1)       # the device is still usable
    g.resample(0.2)
    g.sweep(0.2, 2)
    g.close()


@pytest.mark.parametrize("fault,code", [("energy", "PA_EDEVICE"),
                                        ("capacity", "PA_ECAPACITY")])
def test_failed_resampling_leaves_the_population(pa, env, fault, code):
    g = pa.Population(12, 400, seed=2)
    for b in W.linear_schedule(0.6, 3):
        g.resample(b)
        g.sweep(b, 2)
    before = g.population()
    z0, q0 = g.free_energy()
    st0 = g.state()
    env["PA_FAULT"] = fault
    with pytest.raises(pa.PAError) as e:
        g.resample(0.7)
    assert e.value.code == getattr(pa, code)
    del env["PA_FAULT"]
    assert g.state() == st0
    assert g.free_energy() == (z0, q0)
    for a, b in zip(before, g.population()):
        assert np.array_equal(a, b)
    # and the run goes on as if the failed call had not happened
    ref = pa.Population(12, 400, seed=2)
    for b in W.linear_schedule(0.6, 3) + [0.7]:
        ref.resample(b)
        ref.sweep(b, 2)
    g.resample(0.7)
    g.sweep(0.7, 2)
    for a, b in zip(ref.population(), g.population()):
        assert np.array_equal(a, b)
    assert ref.free_energy() == g.free_energy()
    g.close()
    ref.close()


def test_step_log_records_each_resampling(pa, env, tmp_path):
    path = str(tmp_path / "steps.jsonl")
    env["PA_LOG_JSONL"] = path
    g = pa.Population(16, 600, seed=4)
    sched = W.linear_schedule(0.8, 5)
    want = []
    for b in sched:
        R_prev = g.R
        obs_prev = g.observables()
        R_new = g.resample(b)
        want.append((b, R_prev, R_new, g.free_energy(), obs_prev))
        g.sweep(b, 2)
    g.close()
    del env["PA_LOG_JSONL"]
    lines = [json.loads(l) for l in open(path)]
    assert len(lines) == len(sched)
    for k, (rec, (b, R_prev, R_new, (lnZ, lnQ), o)) in enumerate(
            zip(lines, want)):
        assert rec["step"] == k + 1 and rec["beta"] == b
        assert rec["R_prev"] == R_prev and rec["R"] == R_new
        assert rec["lnQ"] == lnQ and rec["lnZ"] == lnZ
        assert abs(rec["e_prev"] - o["e"]) <= 1e-12 * max(1.0, abs(o["e"]))
        assert 0.0 <= rec["overlap"] <= 1.0 + 1e-12
        assert abs(rec["culling"] - (1.0 - rec["overlap"])) <= 1e-15
        assert rec["source"] == "caller"


def test_batch_step_log_names_the_decision_source(pa, env, tmp_path):
    path = str(tmp_path / "batch.jsonl")
    env["PA_LOG_JSONL"] = path
    pops = [dict(L=12, R=500, seed=5, population_id=0),
            dict(L=16, R=400, seed=6, population_id=1)]
    b = pa.Batch(pops)
    b.run_adaptive(0.85, 1.0, 200, 2)
    del env["PA_LOG_JSONL"]
    lines = [json.loads(l) for l in open(path)]
    for p in range(2):
        mine = [r for r in lines if r["pop"] == p]
        obs, lnZ = b.trajectory(p)
        assert len(mine) == len(obs)
        assert [r["lnZ"] for r in mine] == list(lnZ)
        assert set(r["source"] for r in mine) <= {"bisection", "rest"}
        assert mine[-1]["beta"] == 1.0
    b.close()
