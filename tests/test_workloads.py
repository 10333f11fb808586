"""The synthetic workloads match the paper's printed task (golden fixture),
and the input generators are seeded and deterministic."""
import json
import os

import numpy as np

import pa_workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden",
                      "paper_workload.json")


def test_paper_shape_workloads_match_the_printed_task():
    g = json.load(open(GOLDEN))
    for name, theta in (("CP1", 1), ("CP10", 10)):
        c = W.CONFIGS[name]
        assert c["L"] == g["L"] and c["R"] == g["replicas_per_gpu"]
        assert c["K"] == g["K"] and c["beta_f"] == g["beta_K"]
        assert theta in g["theta"] and c["theta"] == theta
        sched = W.linear_schedule(c["beta_f"], c["K"])
        assert abs(sched[0] - g["dbeta"]) < 1e-15
        assert sched[-1] == g["beta_K"]


def test_linear_schedule_is_computed_from_the_index():
    s = W.linear_schedule(1.0, 200)
    assert s == [(1.0 * i) / 200.0 for i in range(1, 201)]


def test_coupling_generators_are_seeded():
    a = W.pmj_couplings(16, 5)
    b = W.pmj_couplings(16, 5)
    c = W.pmj_couplings(16, 6)
    assert a.dtype == np.int8 and set(np.unique(a)) <= {-1, 1}
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert abs((a == -1).mean() - 0.5) < 0.1
    J, eps = W.gauge_couplings(8, 3)
    assert np.array_equal(J[0], eps * np.roll(eps, -1, axis=1))


def test_batched_instances_cover_the_stated_ranges():
    inst = W.batched_glass_instances()
    assert len(inst) == 64
    assert {i["L"] for i in inst} <= {8, 12, 16, 24, 32}
    assert all(2 ** 10 <= i["R"] <= 2 ** 16 for i in inst)
    assert [i["population_id"] for i in inst] == list(range(64))
    again = W.batched_glass_instances()
    assert all(np.array_equal(a["J"], b["J"]) for a, b in zip(inst, again))


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits at once with a message
    (no device is touched)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 1" in r.stderr
