"""Host-side helpers of bench.py (no GPU): the 1-flip descent that polishes
the reference cut, checked against exhaustive single-flip improvement, and
the lookup of profile figures by launch shape and source hash."""
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


def test_profile_figures_are_keyed_by_launch_shape_and_sources(tmp_path, monkeypatch):
    # a figure is used only for the launch shape it was measured on and only
    # while the kernel sources hash as recorded; missing sources give none
    assert bench._shape_suffix(256, {"block": 768, "slices_per_wave": 4,
                                     "rows_per_lane": 4}) == "R256_768x4x4"
    assert bench._shape_suffix(1, {"block": 1024, "slices_per_wave": 1}) == "R1_1024x1x4"
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    prof = tmp_path / "p.md"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setitem(bench.PROFILES, "t", ("p.md", ["k.hip"]))
    h = bench.source_hash(["k.hip"])
    prof.write_text(f"traffic_bytes_per_launch_R256_768x4x4: 123 source_sha256: {h}\n")
    assert bench._profile_value("t", "traffic_bytes_per_launch_R256_768x4x4") == 123.0
    assert bench._profile_value("t", "traffic_bytes_per_launch_R256_1024x3x4") is None
    src.write_text("kernel v2\n")
    assert bench._profile_value("t", "traffic_bytes_per_launch_R256_768x4x4") is None
    src.unlink()
    assert bench._profile_value("t", "traffic_bytes_per_launch_R256_768x4x4") is None
