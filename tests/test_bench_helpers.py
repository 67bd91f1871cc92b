"""Host-side helpers of bench.py (no GPU): the plain first-come-first-served
queue model of the serving comparison, and the readers of the committed
profile summaries that the bench line quotes."""
import importlib.util
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_fcfs_queue(bench):
    # all at once: each waits for the ones before it
    lat, done = bench._fcfs(np.array([0.0, 0.0, 0.0]), np.array([1.0, 2.0, 3.0]))
    assert np.allclose(lat, [1.0, 3.0, 6.0]) and done == 6.0
    # spaced wider than the service times: nobody waits
    lat, done = bench._fcfs(np.array([0.0, 5.0, 10.0]), np.array([1.0, 2.0, 3.0]))
    assert np.allclose(lat, [1.0, 2.0, 3.0]) and done == 13.0
    # a busy period followed by an idle server
    lat, _ = bench._fcfs(np.array([0.0, 0.5, 4.0]), np.array([2.0, 1.0, 1.0]))
    assert np.allclose(lat, [2.0, 2.5, 1.0])


def test_serve_sweep_summary_parses(bench):
    sw = bench.serve_sweep_from_profile()
    assert sw is not None and "not measured by this run" in sw["source"]
    rates = [r["x_plain_capacity"] for r in sw["rates"]]
    assert rates == sorted(rates) and {0.25, 0.5, 0.75, 0.9, 1.0, 1.25, 2.0} <= set(rates)
    for r in sw["rates"]:
        assert r["n"] >= 1000 and r["completed"] == r["n"]
        assert r["p50_s"] <= r["p99_s"] and r["plain_p50_s"] <= r["plain_p99_s"]
        assert 0 < r["solves_per_s"] <= r["offered_per_s"] * 1.2
    cur = sw["current_policy"]["rates"]
    assert cur and all(r["n"] >= 1000 and r["completed"] == r["n"] for r in cur)
    assert {r["x_plain_capacity"] for r in cur} <= set(rates)
    txt = open(bench.PROFILE_SERVE).read()
    assert "Ns 10..16" in txt and "12870^2" in txt


def test_counter_summaries_name_their_plans(bench):
    # every plan the summaries list has a traffic figure the reader finds
    # (or the reader reports the source as changed since the counters)
    for dt in ("f64", "f32"):
        txt = open(bench.PROFILE_PMC[dt]).read()
        plans = [p.split(",") for p in re.findall(r"traffic\[([0-9,]+)\]", txt)]
        assert plans, dt
        keys = ("mode", "col_cols", "col_threads", "row_rows", "row_cols", "col_order")
        for p in plans:
            val, why = bench.traffic_from_profile(dict(zip(keys, map(int, p))), dt)
            assert (why == "ok" and val > 0) or why == "stale", (dt, p, why)
        val, why = bench.traffic_from_profile(dict(zip(keys, (2, 9, 64, 1, 1, 0))), dt)
        assert val is None and why in ("plan not profiled", "stale")
