"""Host-side helpers of bench.py (no GPU): the 1-flip descent that polishes
the reference cut, checked against exhaustive single-flip improvement."""
import itertools
import os
import sys

import numpy as np

import synth

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _cut(g, s):
    iu, ju, wu = g.upper_edges()
    return float(np.sum(wu[s[iu] != s[ju]]))


def test_one_flip_descent_reaches_a_local_optimum():
    g = synth.torus(12, 12, seed=3)
    rng = np.random.default_rng(0)
    for _ in range(3):
        s0 = rng.integers(0, 2, g.n).astype(np.int8)
        got = bench._one_flip_descent(g, s0)
        # the same descent, done slowly: flip the best vertex while it helps
        s = s0.copy()
        while True:
            base = _cut(g, s)
            gains = []
            for i in range(g.n):
                s[i] ^= 1
                gains.append(_cut(g, s) - base)
                s[i] ^= 1
            i = int(np.argmax(gains))
            if gains[i] <= 1e-12:
                break
            s[i] ^= 1
        assert got == _cut(g, s)
        assert got >= _cut(g, s0)


def test_one_flip_descent_on_a_tiny_graph_is_at_most_the_maximum_cut():
    g = synth.random_small(10, 0.5, seed=5, weights="pm1")
    best = max(_cut(g, np.array(b, np.int8)) for b in itertools.product([0, 1], repeat=g.n))
    for seed in range(5):
        s0 = np.random.default_rng(seed).integers(0, 2, g.n).astype(np.int8)
        assert bench._one_flip_descent(g, s0) <= best


def test_oracle_sample_longer_than_the_schedule_reruns_it(monkeypatch):
    # the rate counts only steps the sampler was asked to run, each call no
    # longer than the schedule
    host = bench.host_cpu()
    host["threads_used"] = 2
    monkeypatch.setattr(bench, "host_cpu", lambda: host)
    calls = []

    def run(R, steps, threads):
        calls.append((R, steps, threads))

    out = bench.oracle_baseline(run, 10.0, {"desc": "x", "replicas": 1, "max_steps": 7},
                                target_1t=1e-4, target_nt=1e-4)
    assert calls and max(c[1] for c in calls) <= 7
    # every timed leg ran exactly the steps it reports
    s1 = int(out["sample"].split("and 1 replica x ")[1].split(" steps")[0])
    legs = [c for c in calls if c[2] == 1][1:]  # after the 2-step probe
    assert sum(c[1] for c in legs) == s1
