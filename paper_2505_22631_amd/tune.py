"""Autotuning of the LDS-resident loop's launch shape, with a persistent cache.

`tuned(problem, theta, K, Ks, sigma, seeds, q=..., dt=...)` looks the
problem's shape bucket up in a JSON cache (path from OIM_TUNE_CACHE, else
~/.cache/oim_tune.json); on a hit it applies the cached launch variant with
oim_set_tuning, otherwise it runs oim_autotune on a prefix of the schedule and
stores the winner.  The bucket is (device architecture, instances, largest
instance in 64-quad slices, mean degree rounded, replicas, SHIL order class),
so problems of the same shape share one measurement.
"""
from __future__ import annotations

import json
import os

import torch

from . import oim_autotune, oim_set_tuning


def cache_path() -> str:
    return os.environ.get("OIM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "oim_tune.json"))


def bucket(problem, R: int, q: int) -> str:
    info = problem.info
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    n_inst = int(info["n_instances"])
    deg = round(info["nnz"] / max(info["n"], 1))
    qc = "2" if q == 2 else "3" if q == 3 else "q"
    slices = -(-(-(-int(info["max_instance_n"]) // 4)) // 64)  # 64-quad slices
    return f"{arch}|inst{n_inst}|slices{slices}|deg{deg}|R{R}|q{qc}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tuned(problem, theta, K, Ks, sigma, seeds, *, q, dt, trial_steps=None, retune=False):
    """Apply (or measure and cache) the launch variant for this problem shape.
    Returns (entry, measured): the cache entry and whether it was measured now."""
    R = int(theta.shape[0])
    key = bucket(problem, R, q)
    path = cache_path()
    cache = _load(path)
    if not retune and key in cache:
        e = cache[key]
        oim_set_tuning(problem.handle, q, e["block"], e["slices_per_wave"],
                       e.get("rows_per_lane", 4))
        return e, False
    steps = int(K.shape[0])
    ts = trial_steps or max(1, min(steps, 500))
    rep = oim_autotune(problem.handle, problem.n, theta, K, Ks, sigma, seeds, q=q, dt=dt,
                       trial_steps=ts)
    e = {"block": rep["block"], "slices_per_wave": rep["slices_per_wave"],
         "rows_per_lane": rep["rows_per_lane"], "trial_ms": rep["ms"],
         "trial_steps": ts, "tried": rep["tried"]}
    cache[key] = e
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass
    return e, True
