"""Benchmark of the SHIL-Kuramoto Euler-Maruyama hot path on one MI355X.

Headline workload (the `value` of the JSON line): sparse max-cut at scale --
a 100x100 toroidal grid (n = 10000, degree 4) with +-1 weights (seed 1),
256 replicas (seeds 0..255), q = 2, dt = 0.01, 10000 Euler-Maruyama steps,
noise sigma = 0.1, linear K ramp and triangular Ks, in-run readout every
100 steps.  One benchmark "step" is one full solve of that workload: oim_run
over the 10000 steps (noise, coupling, SHIL, update, periodic thresholding
and energy readout with best-so-far tracking), then thresholding of the
final phases and the exact cut readout.  The metric is edge-updates per
second: one edge-update is J_ij sin(th_i - th_j) for one stored nonzero, one
replica, one Euler-Maruyama step.

The same JSON line carries, under "workloads", every other configuration of
the benchmark set, each with its own timing, roofline and oracle baseline:
  gnp800_plain / gnp800_batched  G(800, 0.06) max-cut, 1 replica / 256 replicas
  colouring                      1024 planted 3-colourable graphs in one launch
  sk4096_bf16x3 / sk4096_fp32    dense SK n = 4096, 512 replicas, MFMA coupling
  adjoint                        128 x G(2000, 10/1999) schedule gradient
Inputs are synthetic and resident in device memory before any timing.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edge-updates/s & time-to-99%-best-cut, batched vs plain, 1 MI355X"
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0
MFMA_FP32_PEAK_TFLOPS = 157.3
DT = float(np.float32(0.01))

SPARSE_SOURCES = ["paper_2505_22631_amd/csrc/sparse_persistent.hip",
                  "paper_2505_22631_amd/csrc/sparse_persistent_uw.hip",
                  "paper_2505_22631_amd/csrc/persistent_kernel.hpp",
                  "paper_2505_22631_amd/csrc/noise.hpp", "paper_2505_22631_amd/csrc/phase.hpp",
                  "paper_2505_22631_amd/csrc/tree.hpp"]
DENSE_SOURCES = ["paper_2505_22631_amd/csrc/dense.hip", "paper_2505_22631_amd/csrc/noise.hpp",
                 "paper_2505_22631_amd/csrc/phase.hpp"]
ADJOINT_SOURCES = ["paper_2505_22631_amd/csrc/adjoint.hip", "paper_2505_22631_amd/csrc/noise.hpp",
                   "paper_2505_22631_amd/csrc/phase.hpp"]
STEPWISE_SOURCES = ["paper_2505_22631_amd/csrc/stepwise.hip",
                    "paper_2505_22631_amd/csrc/noise.hpp", "paper_2505_22631_amd/csrc/phase.hpp",
                    "paper_2505_22631_amd/csrc/tree.hpp"]
PROFILES = {
    "torus": ("profiles/persistent_sparse_kernel__torus100x100_R256.md", SPARSE_SOURCES),
    "stepwise": ("profiles/stepwise_step_kernel__torus100x100_R256.md", STEPWISE_SOURCES),
    "gnp800": ("profiles/persistent_sparse_kernel__gnp800_R256.md", SPARSE_SOURCES),
    "colouring": ("profiles/persistent_sparse_kernel__colouring1024_q3.md", SPARSE_SOURCES),
    "sk4096": ("profiles/dense_step_kernel__sk4096_R512.md", DENSE_SOURCES),
    "sk20000": ("profiles/dense_step_kernel__sk20000_R512.md", DENSE_SOURCES),
    "adjoint": ("profiles/adjoint_kernels__128xG2000_deg10.md", ADJOINT_SOURCES),
}


def source_hash(sources) -> str:
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _launch_shape(args, prob, q):
    """--launch BxSxL: that launch shape of the LDS-resident kernel (threads,
    slices per wave, rows per lane) instead of the autotuner's choice, so
    counters can be taken on a given shape; None without it."""
    if not getattr(args, "launch", None):
        return None
    import paper_2505_22631_amd as oim
    b, s, l = (int(x) for x in args.launch.lower().split("x"))
    oim.oim_set_tuning(prob.handle, q, b, s, l)
    return {"block": b, "slices_per_wave": s, "rows_per_lane": l}


def _shape_suffix(R, launch):
    """Profile key suffix of a launch of the LDS-resident kernel: replicas and
    launch shape (threads x slices per wave x rows per lane), since counters
    such as register-spill traffic depend on the shape the tuner picked."""
    return (f"R{R}_{launch['block']}x{launch['slices_per_wave']}"
            f"x{launch.get('rows_per_lane', 4)}")


def _profile_value(name, key):
    """A figure from a committed profile summary (`key: value ... source_sha256:
    hash`), if it was taken on the kernel sources as they are now."""
    path, sources = PROFILES[name]
    try:
        want = source_hash(sources)
    except OSError:  # sources not at hand: the figure cannot be matched to them
        return None
    try:
        for line in open(os.path.join(ROOT, path)):
            if line.startswith(key + ":"):
                parts = line.split()
                if parts[-1] == want:
                    return float(parts[1])
    except (OSError, IndexError, ValueError):
        pass
    return None


# ------------------------------------------------------------ host CPU ----
def host_cpu():
    """Model string, physical cores of the host, and the threads this process
    may use (its affinity mask, capped by OMP_NUM_THREADS when that is set:
    the share of the host given to one GPU)."""
    model, cores_per_socket, sockets = None, None, None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            v = v.strip()
            if k == "Model name" and not model:
                model = v
            elif k == "Core(s) per socket":
                cores_per_socket = int(v)
            elif k == "Socket(s)":
                sockets = int(v)
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                m = line.split(":", 1)[1].strip()
                if not model or len(m) > len(model):
                    model = m
                break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    share = avail
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        share = min(share, int(env))
    phys = cores_per_socket * sockets if cores_per_socket and sockets else None
    return {"model": model or platform.processor() or "unknown", "physical_cores": phys,
            "threads_available": avail, "threads_used": max(1, share)}


def oracle_baseline(run_sample, unit_eu, what, target_1t=4.0, target_nt=6.0):
    """Times the oracle as it stands on a bounded sample of a workload: once on
    one thread and once on every thread this process may use.
    run_sample(replicas, steps, threads) runs the sample; unit_eu is the
    edge-updates of one replica-step; a sample longer than the schedule
    (what["max_steps"]) runs the schedule again from its start as many times
    as it takes.  Returns the cpu_baseline object."""
    cpu = host_cpu()
    N = cpu["threads_used"]
    cap = int(what.get("max_steps", 1 << 62))

    def timed(R, steps, threads):
        t0 = time.perf_counter()
        left = steps
        while left > 0:
            run_sample(R, min(left, cap), threads)
            left -= min(left, cap)
        return time.perf_counter() - t0

    # one thread, one replica
    probe = timed(1, 2, 1) / 2
    s1 = int(max(2, target_1t / max(probe, 1e-9)))
    t1 = timed(1, s1, 1)
    eu1 = unit_eu * s1 / t1
    # every thread: one replica per thread (rows shared among threads when the
    # workload has a single replica)
    Rn = N if what.get("replicas", N) >= N else what.get("replicas", 1)
    probe = timed(Rn, 2, N) / 2
    sn = int(max(2, target_nt / max(probe, 1e-9)))
    tn = timed(Rn, sn, N)
    eun = unit_eu * Rn * sn / tn
    return {"value": eun, "unit": "edge-updates/s", "cores": N, "kind": "oracle",
            "sample": f"{what['desc']}: {Rn} replica(s) x {sn} steps on {N} threads "
                      f"({tn:.1f} s), and 1 replica x {s1} steps on 1 thread ({t1:.1f} s); "
                      f"FP64, direct sin per edge",
            "single_thread_value": eu1, "host": cpu["model"],
            "host_physical_cores": cpu["physical_cores"],
            "host_threads_available": cpu["threads_available"]}


# --------------------------------------------------------------- timing ----
def _events(n):
    import torch
    return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(n)]


def _timed_runs(fn, steps, warmup):
    """Runs fn(ev) warmup + steps times; returns (wall ms per run, mean
    HIP-event ms per run).  fn records ev[0] / ev[1] on the launch stream
    around the kernel(s) it times."""
    import torch
    for _ in range(warmup):
        fn(None)
    torch.cuda.synchronize()
    evs = _events(steps)
    t0 = time.perf_counter()
    for k in range(steps):
        fn(evs[k])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    return wall, float(np.mean([a.elapsed_time(b) for a, b in evs]))


def _sync_time(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def sparse_bytes_per_step(n, nnz, R):
    """Algorithmic bytes of one sparse Euler-Maruyama step: phases read and
    written once per oscillator and replica, the coupling's CSR once
    (8 bytes per stored entry) and its row pointers."""
    return 8.0 * n * R + 8.0 * nnz + 4.0 * (n + 1)


def hbm_roofline(bytes_per_step, steps, kernel_ms, kernel, extra=None):
    achieved = bytes_per_step * steps / (kernel_ms * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kernel,
         "kernel_ms": kernel_ms, "bytes_per_em_step": bytes_per_step,
         "note": "algorithmic bytes as the metric defines them; the LDS-resident kernel keeps "
                 "the state on chip, so measured HBM traffic is far lower (see traffic)"}
    if extra:
        r.update(extra)
    return r


def _one_flip_descent(g, colour):
    """Cut after greedy single-vertex flips from a 0/1 state until no flip
    raises the cut (host, for the reference value only)."""
    s = np.asarray(colour, np.int8).copy()
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    w = g.w.astype(np.float64)
    same = s[rows] == s[g.col]
    gain = np.zeros(g.n)
    np.add.at(gain, rows, np.where(same, w, -w))  # cut change if vertex flips
    for _ in range(10 * g.n):
        i = int(np.argmax(gain))
        if gain[i] <= 1e-12:
            break
        s[i] ^= 1
        gain[i] = -gain[i]
        for e in range(g.row_ptr[i], g.row_ptr[i + 1]):
            j = g.col[e]
            gain[j] += 2.0 * w[e] if s[i] == s[j] else -2.0 * w[e]
    iu, ju, wu = g.upper_edges()
    return float(np.sum(wu[s[iu] != s[ju]]))


# -------------------------------------------------------- sparse max-cut ----
SEED_SETS = 5
T99_READOUT = 10  # readout period of the untimed seed-set runs that locate T99


def maxcut_workload(args, name, g, R, steps, M, label, timed_steps, plain_replicas,
                    stepwise=False):
    """One sparse max-cut workload on the LDS-resident loop: the batched solve
    of R replicas in one launch (timed), time to 99 % of the best cut from
    five seed sets read out every 10 steps, the plain loop of one launch per
    replica, and the oracle baseline."""
    import torch
    import paper_2505_22631_amd as oim
    import synth
    from paper_2505_22631_amd import tune
    dev = torch.device("cuda:0")
    q = 2
    t_up = time.perf_counter()
    prob = oim.Problem.from_csr(g.n, g.row_ptr, g.col, (-g.w).astype(np.float32))
    upload_ms = (time.perf_counter() - t_up) * 1e3
    K, Ks, sg, kmax, ksmax = synth.workload_schedule(name, prob.info["max_abs_row_sum"], steps,
                                                     DT)
    dK, dKs, dsg = (torch.from_numpy(x).to(dev) for x in (K, Ks, sg))
    th_init = torch.from_numpy(synth.theta0(R, g.n, seed=100)).to(dev)
    seeds = torch.from_numpy(synth.seeds(R, 0)).to(dev)
    theta = torch.empty_like(th_init)
    nr = oim.n_readouts(steps, M)
    trace = torch.empty((nr, R), dtype=torch.float64, device=dev)
    best_h = torch.empty(R, dtype=torch.float64, device=dev)
    best_step = torch.empty(R, dtype=torch.int32, device=dev)
    colour = torch.empty((R, g.n), dtype=torch.int8, device=dev)
    stream = torch.cuda.current_stream()
    launch = _launch_shape(args, prob, q) or tune.tuned(
        prob, th_init, dK, dKs, dsg, seeds, q=q, dt=DT, trial_steps=min(steps, 500))[0]
    cuts = []

    def solve(ev):
        theta.copy_(th_init)
        if ev:
            ev[0].record(stream)
        oim.oim_run(prob.handle, g.n, theta, dK, dKs, dsg, seeds, q=q, dt=DT, readout_every=M,
                    trace=trace, best_h=best_h, best_step=best_step)
        if ev:
            ev[1].record(stream)
        oim.oim_round(q, theta, colour)
        cuts.append(oim.oim_cut(prob.handle, colour))

    wall_ms, kern_ms = _timed_runs(solve, timed_steps, args.warmup)
    eu_per_solve = float(g.nnz) * R * steps
    W = -prob.info["sum_J_upper"]
    final_cut = int(max(int(c.max()) for c in cuts))

    # ---- time to 99 % of the best cut ----
    # best_ref: the best cut of the timed solves, of the five seed sets, of
    # one 10x longer run (same schedule shape stretched, other seeds), all
    # untimed, polished by a host 1-flip descent from the best state seen.
    sets, best_cut_seen, best_state = [], -np.inf, None
    for k in range(SEED_SETS):
        th_k = torch.from_numpy(synth.theta0(R, g.n, seed=100 + k)).to(dev)
        sd_k = torch.from_numpy(synth.seeds(R, k * 1000003)).to(dev)
        ro_k = oim.run(prob, th_k, dK, dKs, dsg, sd_k, q=q, dt=DT, readout_every=T99_READOUT,
                       want_best=True)
        sets.append((W - ro_k["trace"].cpu().numpy()) / 2.0)
        bh = ro_k["best_h"].cpu().numpy()
        r_best = int(np.argmin(bh))
        if (W - bh[r_best]) / 2.0 > best_cut_seen:
            best_cut_seen = (W - bh[r_best]) / 2.0
            best_state = ro_k["best_colour"][r_best].cpu().numpy()
    best_ref = max(float(final_cut), best_cut_seen, float((W - trace.cpu().numpy().min()) / 2.0))
    if args.ref_mult > 0:
        rs = steps * args.ref_mult
        rK, rKs, rsg, _, _ = synth.workload_schedule(name, prob.info["max_abs_row_sum"], rs, DT)
        th_r = torch.from_numpy(synth.theta0(R, g.n, seed=7)).to(dev)
        sd_r = torch.from_numpy(synth.seeds(R, 1 << 20)).to(dev)
        ro_r = oim.run(prob, th_r, torch.from_numpy(rK).to(dev), torch.from_numpy(rKs).to(dev),
                       torch.from_numpy(rsg).to(dev), sd_r, q=q, dt=DT, readout_every=M,
                       want_best=True)
        bh = ro_r["best_h"].cpu().numpy()
        r_best = int(np.argmin(bh))
        if (W - bh[r_best]) / 2.0 > best_cut_seen:
            best_cut_seen = (W - bh[r_best]) / 2.0
            best_state = ro_r["best_colour"][r_best].cpu().numpy()
        best_ref = max(best_ref, best_cut_seen)
    polished = _one_flip_descent(g, best_state) if best_state is not None else None
    if polished is not None:
        best_ref = max(best_ref, polished)
    target = 0.99 * best_ref
    t99s, successes = [], 0
    for ct in sets:
        best_so_far = np.maximum.accumulate(ct.max(axis=1))
        hit = np.nonzero(best_so_far >= target)[0]
        t99s.append(min((int(hit[0]) + 1) * T99_READOUT, steps) / steps * kern_ms
                    if hit.size else None)
        successes += int(np.sum(ct.max(axis=0) >= target))
    t99_median = (float(np.median(t99s)) if all(t is not None for t in t99s) else None)
    p_success = successes / float(R * len(sets))
    # time to solution at 99 % confidence for one replica's share of a
    # batched run (kern_ms / R per replica-run), from the per-replica success rate
    if p_success >= 1.0:
        tts99 = kern_ms / R
    elif p_success > 0.0:
        tts99 = kern_ms / R * np.log(0.01) / np.log(1.0 - p_success)
    else:
        tts99 = None

    # ---- plain loop: one launch per replica (R = 1), same schedule and seeds,
    # one after the other until a replica reaches the target ----
    plain = None
    if plain_replicas > 0:
        th1 = th_init[:1].clone()
        tr1 = torch.empty((oim.n_readouts(steps, T99_READOUT), 1), dtype=torch.float64,
                          device=dev)
        oim.oim_run(prob.handle, g.n, th1, dK, dKs, dsg, seeds[:1], q=q, dt=DT)  # warm
        evs = _events(plain_replicas)
        elapsed, t99_plain, per = 0.0, None, []
        for r in range(plain_replicas):
            th1.copy_(th_init[r:r + 1])
            evs[r][0].record(stream)
            oim.oim_run(prob.handle, g.n, th1, dK, dKs, dsg, seeds[r:r + 1], q=q, dt=DT,
                        readout_every=T99_READOUT, trace=tr1)
            evs[r][1].record(stream)
            torch.cuda.synchronize()
            dtr = evs[r][0].elapsed_time(evs[r][1]) * 1e-3
            per.append(dtr)
            c1 = (W - tr1[:, 0].cpu().numpy()) / 2.0
            h1 = np.nonzero(np.maximum.accumulate(c1) >= target)[0]
            if h1.size and t99_plain is None:
                t99_plain = (elapsed + min((int(h1[0]) + 1) * T99_READOUT, steps) / steps * dtr) * 1e3
            elapsed += dtr
        pl = float(np.mean(per))
        plain = {"eu_per_s": float(g.nnz) * steps / pl, "ms_per_replica": pl * 1e3,
                 "replicas_timed": plain_replicas, "time_to_99pct_best_cut_ms": t99_plain,
                 "note": "HIP events around each one-replica launch (readout every "
                         f"{T99_READOUT} steps)"}

    # ---- the same solve on the stepwise loop (state in device memory, chunks
    # of steps replayed from a captured hipGraph) ----
    sw = None
    if stepwise:
        th_s = th_init.clone()
        sw_steps = min(steps, args.stepwise_steps or steps)

        def solve_sw(ev):
            th_s.copy_(th_init)
            if ev:
                ev[0].record(stream)
            oim.oim_run(prob.handle, g.n, th_s, dK[:sw_steps], dKs[:sw_steps], dsg[:sw_steps],
                        seeds, q=q, dt=DT, readout_every=M,
                        trace=trace[:oim.n_readouts(sw_steps, M)], flags=oim.OIM_LOOP_STEPWISE)
            if ev:
                ev[1].record(stream)
        sw_wall, sw_ms = _timed_runs(solve_sw, max(1, min(3, timed_steps)), 1)
        sw = {"em_steps": sw_steps, "ms_per_solve": sw_ms, "wall_ms_per_solve": sw_wall,
              "eu_per_s": eu_per_solve * sw_steps / steps / (sw_ms * 1e-3),
              "slowdown_vs_lds_resident": sw_ms / (kern_ms * sw_steps / steps),
              "roofline": hbm_roofline(sparse_bytes_per_step(g.n, g.nnz, R), sw_steps, sw_ms,
                                       "stepwise_step_kernel (hipGraph loop)")}
        if name == "torus":
            per_step = _profile_value("stepwise", f"traffic_bytes_per_step_R{R}")
            sw["roofline"]["traffic"] = per_step * sw_steps if per_step is not None else None

    roof = hbm_roofline(sparse_bytes_per_step(g.n, g.nnz, R), steps, kern_ms,
                        "persistent_sparse_kernel",
                        {"launch": {"block": launch["block"],
                                    "slices_per_wave": launch["slices_per_wave"],
                                    "rows_per_lane": launch.get("rows_per_lane", 4)}})
    prof = name if name in PROFILES else None
    if prof:
        sfx = _shape_suffix(R, launch)
        roof["traffic"] = _profile_value(prof, "traffic_bytes_per_launch_" + sfx)
        valu = _profile_value(prof, "valu_busy_frac_" + sfx)
        if valu is not None:
            roof["valu_busy_frac"] = valu
    out = {
        "value": eu_per_solve / (wall_ms * 1e-3), "unit": "edge-updates/s",
        "ms_per_solve": wall_ms, "kernel_ms": kern_ms, "dtype": "f32",
        "config": {"workload": label, "n": g.n, "nnz": g.nnz, "replicas": R, "em_steps": steps,
                   "q": q, "dt": DT, "sigma": synth.WORKLOAD_SCHEDULES[name]["sigma"],
                   "K_max": kmax, "Ks_max": ksmax, "readout_every": M},
        "roofline": roof,
        "time_to_99pct_best_cut_ms_median_5_seed_sets": t99_median,
        "time_to_99pct_best_cut_ms_per_seed_set": t99s,
        "replica_success_rate_99pct": p_success,
        "tts99_ms_per_replica_run": tts99,
        "best_cut_ref": best_ref, "best_cut_ref_polish": polished,
        "best_cut_timed_solves": float(final_cut),
        "plain": plain, "problem_upload_ms": upload_ms,
    }
    if sw is not None:
        out["stepwise_hipgraph_loop"] = sw
    if not args.no_cpu_baseline:
        import oracle
        J = (-g.w).astype(np.float32)

        def sample(Rs, st, threads):
            oracle.run_csr(g.row_ptr, g.col, J, synth.theta0(Rs, g.n, seed=100), q=q, dt=DT,
                           K=K[:st], Ks=Ks[:st], sigma=sg[:st], seeds=synth.seeds(Rs, 0),
                           nthreads=threads)
        out["cpu_baseline"] = oracle_baseline(sample, float(g.nnz),
                                              {"desc": f"{label}, the schedule from its start",
                                               "replicas": R, "max_steps": steps},
                                              target_1t=args.cpu_seconds * 0.4,
                                              target_nt=args.cpu_seconds * 0.6)
    prob.close()
    return out


# ------------------------------------------------------------ colouring ----
def colouring_workload(args):
    """Batched Potts 3-colouring: 1024 planted 3-colourable graphs, n uniform in
    [100, 600] (seed 2), average degree 4.6, J = -1, q = 3, 5000 steps,
    readout every 50 steps; all graphs (R replicas each) in one launch of the
    LDS-resident kernel against a plain loop of one launch per (graph,
    replica).  The objective is the number of satisfied edges.  Two targets:
    99 % of the best satisfied count known for each graph (the best over
    every run of the campaign, as for max-cut), and 99 % of the planted
    optimum (every edge satisfied)."""
    import torch
    import paper_2505_22631_amd as oim
    import synth
    from paper_2505_22631_amd import tune
    count, steps, q, M = 1024, 5000, 3, 50
    R = args.colour_replicas
    graphs = [g for g, _ in synth.planted_batch(count, 100, 600, 4.6, q, seed=2)]
    big, off = synth.block_diagonal(graphs)
    dev = torch.device("cuda:0")
    prob = oim.Problem.from_csr_blocks(big.n, big.row_ptr, big.col,
                                       -np.ones(big.nnz, np.float32), off)
    K, Ks, sg, kmax, ksmax = synth.workload_schedule("colouring", prob.info["max_abs_row_sum"],
                                                     steps, DT)
    dK, dKs, dsg = (torch.from_numpy(x).to(dev) for x in (K, Ks, sg))
    th_init = torch.from_numpy(synth.theta0(R, big.n, seed=100)).to(dev)
    seeds = torch.from_numpy(synth.seeds(R, 0)).to(dev)
    theta = torch.empty_like(th_init)
    nr = oim.n_readouts(steps, M)
    trace = torch.empty((nr, R * count), dtype=torch.float64, device=dev)
    best_h = torch.empty(R * count, dtype=torch.float64, device=dev)
    best_step = torch.empty(R * count, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    edges = np.array([g.nnz // 2 for g in graphs], np.float64)
    launch = _launch_shape(args, prob, q) or tune.tuned(
        prob, th_init, dK, dKs, dsg, seeds, q=q, dt=DT, trial_steps=500)[0]

    def solve(ev):
        theta.copy_(th_init)
        if ev:
            ev[0].record(stream)
        oim.oim_run(prob.handle, big.n, theta, dK, dKs, dsg, seeds, q=q, dt=DT, readout_every=M,
                    trace=trace, best_h=best_h, best_step=best_step)
        if ev:
            ev[1].record(stream)

    wall_ms, run_ms = _timed_runs(solve, max(1, min(args.steps, 10)), args.warmup)
    eu = float(big.nnz) * R * steps
    # satisfied edges per readout, best over the graph's replicas so far
    # (the Eq. 2 energy of J = -1 is the number of conflicting edges)
    sat = edges[None, :] - trace.cpu().numpy().reshape(nr, R, count).min(axis=1)
    sat_so_far = np.maximum.accumulate(sat, axis=0)

    # best known per graph: the timed solve, two more seed sets (also the
    # restarts of the batch below) and one run four times as long, all untimed
    best_known = sat_so_far[-1].copy()
    launches = [sat_so_far]
    for k in range(2):
        th_k = torch.from_numpy(synth.theta0(R, big.n, seed=200 + k)).to(dev)
        sd_k = torch.from_numpy(synth.seeds(R, (k + 1) * 1000003)).to(dev)
        ro = oim.run(prob, th_k, dK, dKs, dsg, sd_k, q=q, dt=DT, readout_every=M)
        c = ro["trace"].cpu().numpy().reshape(nr, R, count).min(axis=1)
        launches.append(np.maximum.accumulate(edges[None, :] - c, axis=0))
        best_known = np.maximum(best_known, launches[-1][-1])
    lK, lKs, lsg, _, _ = synth.workload_schedule("colouring", prob.info["max_abs_row_sum"],
                                                 4 * steps, DT)
    th_l = torch.from_numpy(synth.theta0(R, big.n, seed=300)).to(dev)
    ro = oim.run(prob, th_l, torch.from_numpy(lK).to(dev), torch.from_numpy(lKs).to(dev),
                 torch.from_numpy(lsg).to(dev), torch.from_numpy(synth.seeds(R, 1 << 21)).to(dev),
                 q=q, dt=DT, readout_every=M)
    c = ro["trace"].cpu().numpy().reshape(-1, R, count).min(axis=(0, 1))
    best_known = np.maximum(best_known, edges - c)
    target_best = 0.99 * best_known
    target_planted = 0.99 * edges
    # further relaunches of the batch (other seeds, untimed, not counted in
    # best_known) while some graph has not reached 99 % of its best known
    max_launches = 8
    k = len(launches)
    while k < max_launches and not np.all(
            np.max([l_[-1] for l_ in launches], axis=0) >= target_best):
        th_k = torch.from_numpy(synth.theta0(R, big.n, seed=400 + k)).to(dev)
        sd_k = torch.from_numpy(synth.seeds(R, (k + 7) * 1000003)).to(dev)
        ro = oim.run(prob, th_k, dK, dKs, dsg, sd_k, q=q, dt=DT, readout_every=M)
        c = ro["trace"].cpu().numpy().reshape(nr, R, count).min(axis=1)
        launches.append(np.maximum.accumulate(edges[None, :] - c, axis=0))
        k += 1

    def t_all(target):
        """Time until every graph has reached its target: a graph that
        misses it in one launch of the batch is caught by the next launch
        (other seeds), as the plain loop moves on to the graph's next
        replica; None if some graph misses it in every launch.  Also the
        graphs reaching it in the first launch."""
        t_g = np.full(count, np.inf)
        for k, sat_k in enumerate(launches):
            ok = sat_k >= target[None, :]
            hit = ok[-1] & ~np.isfinite(t_g)
            first = np.argmax(ok, axis=0)
            t_g[hit] = (k + (first[hit] + 1) * M / steps) * run_ms
        first_launch = int(np.sum(launches[0][-1] >= target))
        return (float(t_g.max()) if np.all(np.isfinite(t_g)) else None), first_launch

    t99_best, reach_best = t_all(target_best)
    t99_planted, reach_planted = t_all(target_planted)

    # plain loop over a sample of the graphs: one problem per graph, one
    # launch per replica (R = 1), replicas in turn until the graph reaches
    # the target
    sample = min(args.plain_graphs, count)
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(count, size=sample, replace=False))
    per, hit_best, hit_planted = [], [], []
    tr1 = torch.empty((nr, 1), dtype=torch.float64, device=dev)
    for b in pick:
        g = graphs[b]
        with oim.Problem.from_csr(g.n, g.row_ptr, g.col, -np.ones(g.nnz, np.float32)) as p1:
            th1 = th_init[:, off[b]:off[b + 1]].contiguous()
            oim.oim_run(p1.handle, g.n, th1[:1].clone(), dK, dKs, dsg, seeds[:1], q=q, dt=DT)
            elapsed, hb, hp, best1 = 0.0, None, None, -np.inf
            # replicas in turn (the batch's R, then further seeds, up to as
            # many runs as the batch may use) until both targets are met
            for r in range(max_launches * R):
                if hb is not None and hp is not None:
                    break
                if r >= R and hb is not None:
                    break
                th1c = (th1[r:r + 1].clone() if r < R else torch.from_numpy(
                    synth.theta0(1, g.n, seed=10_000 + r)).to(dev))
                sd1 = seeds[r:r + 1] if r < R else torch.from_numpy(synth.seeds(1, 77_000 + r)).to(dev)

                def one():
                    oim.oim_run(p1.handle, g.n, th1c, dK, dKs, dsg, sd1, q=q, dt=DT,
                                readout_every=M, trace=tr1)
                el = _sync_time(one)
                per.append(el)
                s1 = np.maximum(np.maximum.accumulate(edges[b] - tr1.cpu().numpy()[:, 0]), best1)
                best1 = s1[-1]
                for tgt, name in ((target_best[b], "b"), (target_planted[b], "p")):
                    h = np.nonzero(s1 >= tgt)[0]
                    if h.size and (hb if name == "b" else hp) is None:
                        t = (elapsed + min((int(h[0]) + 1) * M, steps) / steps * el) * 1e3
                        if name == "b":
                            hb = t
                        else:
                            hp = t
                elapsed += el
        hit_best.append(hb)
        hit_planted.append(hp)
    plain_ms_per_run = float(np.mean(per)) * 1e3
    plain_total_ms = plain_ms_per_run * count * R

    def plain_t(hits):
        return float(np.mean(hits)) * count if all(h is not None for h in hits) else None

    plain_t99_best = plain_t(hit_best)
    plain_t99_planted = plain_t(hit_planted)
    bps = sparse_bytes_per_step(big.n, big.nnz, R)
    roof = hbm_roofline(bps, steps, run_ms, "persistent_sparse_kernel",
                        {"launch": {"block": launch["block"],
                                    "slices_per_wave": launch["slices_per_wave"],
                                    "rows_per_lane": launch.get("rows_per_lane", 4)}})
    sfx = _shape_suffix(R, launch)
    roof["traffic"] = _profile_value("colouring", "traffic_bytes_per_launch_" + sfx)
    valu = _profile_value("colouring", "valu_busy_frac_" + sfx)
    if valu is not None:
        roof["valu_busy_frac"] = valu
    out = {
        "value": eu / (wall_ms * 1e-3), "unit": "edge-updates/s", "ms_per_solve": wall_ms,
        "kernel_ms": run_ms, "dtype": "f32",
        "config": {"workload": "batched Potts 3-colouring: 1024 planted graphs, n in [100,600], "
                               "avg degree 4.6, one launch", "graphs": count,
                   "replicas_per_graph": R, "n_total": big.n, "nnz": big.nnz, "em_steps": steps,
                   "q": q, "K_max": kmax, "Ks_max": ksmax, "readout_every": M},
        "roofline": roof,
        "mean_satisfied_fraction_best_replica": float(np.mean(sat_so_far[-1] / edges)),
        "mean_satisfied_fraction_best_known": float(np.mean(best_known / edges)),
        "graphs_reaching_99pct_best_known_first_launch": reach_best,
        "time_to_99pct_best_known_all_graphs_ms": t99_best,
        "graphs_reaching_99pct_planted_first_launch": reach_planted,
        "time_to_99pct_planted_all_graphs_ms": t99_planted,
        "time_to_target_note": "the batch is relaunched with other seeds while a graph misses "
                               "the target (up to 8 launches), as the plain loop runs a graph's "
                               "replicas in turn (up to 8 x R); null if some graph misses it",
        "batch_launches_used": len(launches),
        "best_known": "per graph: the most satisfied edges over the timed solve, two more "
                      "seed sets and one run 4x as long (all untimed)",
        "plain": {"ms_per_graph_replica_run": plain_ms_per_run,
                  "total_ms_extrapolated": plain_total_ms,
                  "time_to_99pct_best_known_all_graphs_ms_extrapolated": plain_t99_best,
                  "time_to_99pct_planted_all_graphs_ms_extrapolated": plain_t99_planted,
                  "graphs_timed": sample,
                  "graphs_timed_reaching_99pct_best_known": int(sum(h is not None for h in hit_best)),
                  "graphs_timed_reaching_99pct_planted": int(sum(h is not None for h in hit_planted)),
                  "eu_per_s": eu / (plain_total_ms * 1e-3),
                  "note": "one launch per (graph, replica), replicas in turn until the graph "
                          "reaches the target; a sample of graphs, extrapolated to all"},
        "speedup_time_to_99pct_best_known": (plain_t99_best / t99_best
                                             if plain_t99_best and t99_best else None),
        "speedup_batched_vs_plain": plain_total_ms / wall_ms,
    }
    if not args.no_cpu_baseline:
        import oracle
        gs = graphs[:64]
        sb, so = synth.block_diagonal(gs)
        Jb = -np.ones(sb.nnz)

        def sample_fn(Rs, st, threads):
            oracle.run_csr_blocks(sb.row_ptr, sb.col, Jb, so, synth.theta0(Rs, sb.n, seed=100),
                                  q=q, dt=DT, K=K[:st], Ks=Ks[:st], sigma=sg[:st],
                                  seeds=synth.seeds(Rs, 0), nthreads=threads)
        out["cpu_baseline"] = oracle_baseline(
            sample_fn, float(sb.nnz),
            {"desc": "the first 64 graphs of the batch as one block-diagonal problem",
             "max_steps": steps},
            target_1t=args.cpu_seconds * 0.2, target_nt=args.cpu_seconds * 0.3)
    prob.close()
    return out


# ---------------------------------------------------------------- dense ----
def dense_workload(args, n=4096, fp32=False):
    """Dense SK Ising: J_ij ~ N(0, 1/n) (seed 3), 512 replicas, coupling as a
    GEMM on the matrix cores (BF16x3 or FP32 products); n = 4096, 1000 steps
    (or the paper's largest all-to-all size n = 20000, 100 steps)."""
    import torch
    import paper_2505_22631_amd as oim
    import synth
    R, q = 512, 2
    steps = args.dense_steps or (1000 if n == 4096 else 100)
    J = synth.sk_dense(n, seed=3)
    dev = torch.device("cuda:0")
    t_up = time.perf_counter()
    prob = oim.Problem.from_dense(J)
    upload_ms = (time.perf_counter() - t_up) * 1e3
    Kh, Ksh, sgh, kmax, ksmax = synth.workload_schedule("sk", prob.info["max_abs_row_sum"],
                                                        steps, DT)
    K, Ks, sg = (torch.from_numpy(x).to(dev) for x in (Kh, Ksh, sgh))
    th_init = torch.from_numpy(synth.theta0(R, n, seed=100)).to(dev)
    seeds = torch.from_numpy(synth.seeds(R, 0)).to(dev)
    theta = torch.empty_like(th_init)
    stream = torch.cuda.current_stream()
    flags = oim.OIM_PREC_FP32 if fp32 else oim.OIM_PREC_BF16X3

    def solve(ev):
        theta.copy_(th_init)
        if ev:
            ev[0].record(stream)
        oim.oim_run(prob.handle, n, theta, K, Ks, sg, seeds, q=q, dt=DT, flags=flags)
        if ev:
            ev[1].record(stream)

    reps = max(1, min(args.steps, args.dense_reps))
    wall_ms, run_ms = _timed_runs(solve, reps, max(1, min(args.warmup, 2)))
    eu = float(n) * (n - 1) * R * steps
    col = oim.oim_round(q, theta)
    hm, _ = oim.oim_energy(prob.handle, q, colour=col)
    e_per_spin = float(hm.min().item()) / n
    # executed MFMA flops per step: 3 products of an n x n by n x 2R GEMM for
    # the BF16x3 coupling, one FP32 product for the FP32 coupling
    flops_step = (1.0 if fp32 else 3.0) * 2.0 * n * n * 2 * R
    peak = MFMA_FP32_PEAK_TFLOPS if fp32 else MFMA_BF16_PEAK_TFLOPS
    # counters from the profile of this size and precision, when there is one
    prof = {4096: "sk4096", 20000: "sk20000"}.get(n)
    prec = "fp32" if fp32 else "bf16x3"
    achieved = flops_step * steps / (run_ms * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": (_profile_value(prof, "traffic_bytes_per_step_" + prec)
                        if prof else None),
            "kernel": ("dense_step32_kernel" if fp32 else "dense_step_kernel")
                      + " (per step, epilogue fused)",
            "kernel_ms_per_em_step": run_ms / steps, "flops_per_step": flops_step,
            "useful_flops_per_step": 4.0 * n * n * R,
            "useful_frac": 4.0 * n * n * R * steps / (run_ms * 1e-3) / 1e12 / peak}
    busy = _profile_value(prof, "mfma_busy_frac_" + prec) if prof else None
    if busy is not None:
        roof["mfma_busy_frac"] = busy
    out = {"value": eu / (wall_ms * 1e-3), "unit": "edge-updates/s", "ms_per_solve": wall_ms,
           "kernel_ms": run_ms, "dtype": "f32" if fp32 else "bf16x3",
           "config": {"workload": f"dense SK Ising n={n}, 512 replicas, "
                                  f"{'FP32' if fp32 else 'BF16x3'} MFMA coupling",
                      "n": n, "replicas": R, "em_steps": steps, "K_max": kmax, "Ks_max": ksmax},
           "roofline": roof, "best_energy_per_spin": e_per_spin, "problem_upload_ms": upload_ms}
    if not args.no_cpu_baseline and n == 4096:
        import oracle
        Jd = J.astype(np.float64)
        out["cpu_baseline"] = oracle_baseline(
            lambda Rs, st, threads: oracle.run_dense(
                Jd, synth.theta0(Rs, n, seed=100), q=q, dt=DT, K=Kh[:st], Ks=Ksh[:st],
                sigma=sgh[:st], seeds=synth.seeds(Rs, 0), nthreads=threads),
            float(n) * (n - 1), {"desc": "the same J and schedule, first steps",
                                 "max_steps": len(Kh)},
            target_1t=args.cpu_seconds * 0.2, target_nt=args.cpu_seconds * 0.3)
        # the GPU result on a sample against the FP64 oracle
        Rs, st = 4, 50
        want = oracle.run_dense(Jd, synth.theta0(R, n, seed=100)[:Rs], q=q, dt=DT, K=Kh[:st],
                                Ks=Ksh[:st], sigma=sgh[:st], seeds=synth.seeds(Rs, 0),
                                nthreads=host_cpu()["threads_used"])
        got = th_init[:Rs].clone()
        oim.oim_run(prob.handle, n, got, K[:st].contiguous(), Ks[:st].contiguous(),
                    sg[:st].contiguous(), seeds[:Rs].contiguous(), q=q, dt=DT, flags=flags)
        d = np.abs(got.cpu().numpy().astype(np.float64) - want)
        out["max_abs_dtheta_vs_fp64_rad"] = float(np.max(np.minimum(d, 2 * np.pi - d)))
        out["max_abs_dtheta_sample"] = f"{Rs} replicas x {st} steps"
    prob.close()
    return out


# -------------------------------------------------------------- adjoint ----
def adjoint_workload(args):
    """Adjoint schedule tuning: 128 graphs G(2000, 10/1999) with +-1 weights
    (graph g with seed 4 + g) in one block-diagonal batch, one replica each,
    2000 steps with fixed Philox noise, checkpoints every 64 steps; gradient of
    the relaxed cut with respect to the per-step K, Ks and sigma.  Forward and
    backward (with recomputation) are timed separately, and against a plain
    loop of one adjoint per graph."""
    import torch
    import paper_2505_22631_amd as oim
    import synth
    count, n, steps, C, q = 128, 2000, 2000, 64, 2
    graphs = [synth.gnp_avg_degree(n, 10.0, seed=4 + g, signed=True) for g in range(count)]
    big, off = synth.block_diagonal(graphs)
    dev = torch.device("cuda:0")
    prob = oim.Problem.from_csr_blocks(big.n, big.row_ptr, big.col, (-big.w).astype(np.float32),
                                       off)
    K, Ks, sg, kmax, ksmax = synth.workload_schedule("adjoint", prob.info["max_abs_row_sum"],
                                                     steps, DT)
    dK, dKs, dsg = (torch.from_numpy(x).to(dev) for x in (K, Ks, sg))
    th0 = torch.from_numpy(synth.theta0(1, big.n, seed=100)).to(dev)
    seeds = torch.from_numpy(synth.seeds(1, 0)).to(dev)
    words = oim.oim_adjoint_checkpoint_words(prob.handle, q=q, R=1, steps=steps, dt=DT,
                                             checkpoint_every=C)
    ckpt = torch.empty(words, dtype=torch.uint32, device=dev)
    loss = torch.empty(count, dtype=torch.float64, device=dev)
    g3 = [torch.empty(steps, dtype=torch.float64, device=dev) for _ in range(3)]
    stream = torch.cuda.current_stream()

    def fwd(ev):
        if ev:
            ev[0].record(stream)
        oim.oim_adjoint_forward(prob.handle, big.n, th0, dK, dKs, dsg, seeds, ckpt, q=q, dt=DT,
                                checkpoint_every=C, loss=loss)
        if ev:
            ev[1].record(stream)

    def bwd(ev):
        if ev:
            ev[0].record(stream)
        oim.oim_adjoint_backward(prob.handle, 1, dK, dKs, dsg, seeds, ckpt, *g3, q=q, dt=DT,
                                 checkpoint_every=C)
        if ev:
            ev[1].record(stream)

    reps = max(1, min(args.steps, 10))
    _, t_f = _timed_runs(fwd, reps, args.warmup)
    _, t_b = _timed_runs(bwd, reps, args.warmup)
    eu = float(big.nnz) * steps
    # plain: one problem and one adjoint per graph, a sample of them
    sample = min(args.plain_graphs, count)
    per = []
    for b in range(sample):
        g = graphs[b]
        with oim.Problem.from_csr(g.n, g.row_ptr, g.col, (-g.w).astype(np.float32)) as p1:
            w1 = oim.oim_adjoint_checkpoint_words(p1.handle, q=q, R=1, steps=steps, dt=DT,
                                                  checkpoint_every=C)
            ck1 = torch.empty(w1, dtype=torch.uint32, device=dev)
            t1 = th0[:, off[b]:off[b + 1]].contiguous()
            h1 = [torch.empty(steps, dtype=torch.float64, device=dev) for _ in range(3)]

            def one():
                oim.oim_adjoint_forward(p1.handle, g.n, t1, dK, dKs, dsg, seeds, ck1, q=q, dt=DT,
                                        checkpoint_every=C)
                oim.oim_adjoint_backward(p1.handle, 1, dK, dKs, dsg, seeds, ck1, *h1, q=q,
                                         dt=DT, checkpoint_every=C)
            one()
            per.append(_sync_time(one))
    plain_ms = float(np.mean(per)) * 1e3 * count
    bps = sparse_bytes_per_step(big.n, big.nnz, 1)
    out = {
        "value": 3.0 * eu / ((t_f + t_b) * 1e-3), "unit": "edge-updates/s",
        "ms_per_solve": t_f + t_b, "dtype": "f32",
        "config": {"workload": "adjoint schedule gradient: 128 x G(2000, 10/1999) +-1, one launch",
                   "graphs": count, "n_total": big.n, "nnz": big.nnz, "em_steps": steps,
                   "checkpoint_every": C, "K_max": kmax, "Ks_max": ksmax,
                   "edge_updates_counted": "forward 1x, backward (recompute + adjoint) 2x"},
        "forward_ms": t_f, "backward_ms": t_b,
        "roofline": {"bound": "hbm", "achieved": bps * steps / (t_f * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": bps * steps / (t_f * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": _profile_value("adjoint", "traffic_bytes_per_forward_launch"),
                     "kernel": "adjoint_forward_kernel", "kernel_ms": t_f,
                     "bytes_per_em_step": bps,
                     "backward_frac": 3.0 * bps * steps / (t_b * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "loss": float(loss.sum().item()),
        "grad_norms": [float(x.norm().item()) for x in g3],
        "plain": {"ms_total_extrapolated": plain_ms, "graphs_timed": sample,
                  "speedup_batched": plain_ms / (t_f + t_b)},
    }
    if not args.no_cpu_baseline:
        import oracle
        g = graphs[0]
        J1 = -g.w.astype(np.float64)
        out["cpu_baseline"] = oracle_baseline(
            lambda Rs, st, threads: oracle.run_csr(
                g.row_ptr, g.col, J1, synth.theta0(Rs, g.n, seed=100), q=q, dt=DT, K=K[:st],
                Ks=Ks[:st], sigma=sg[:st], seeds=synth.seeds(Rs, 0), nthreads=threads),
            float(g.nnz), {"desc": "forward integration of graph 0 (the oracle's forward "
                                   "trajectory; its adjoint stores every state)",
                           "max_steps": steps},
            target_1t=args.cpu_seconds * 0.2, target_nt=args.cpu_seconds * 0.3)
    prob.close()
    return out


# ---------------------------------------------------------------- sweep ----
def sweep_workload(args):
    """Batched annealing-schedule sweep (the kind of study of Sec. III-D /
    Fig. 3b) on the 100x100 +-1 torus: an 8 x 8 grid of (K_max, Ks_max)
    multipliers, 4 replicas per cell, every replica with its own ramp of K and
    triangular Ks, all 256 replicas in one launch, against one launch per
    cell."""
    import torch
    import paper_2505_22631_amd as oim
    import synth
    from paper_2505_22631_amd import tune
    g = synth.torus(100, 100, seed=1, signed=True)
    steps, q, M, per_cell = 10000, 2, 100, 4
    kg = [0.25, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0]
    ksg = [0.125, 0.25, 0.5, 0.75, 1.0, 1.5, 2.0, 3.0]
    dev = torch.device("cuda:0")
    prob = oim.Problem.from_csr(g.n, g.row_ptr, g.col, (-g.w).astype(np.float32))
    rowsum = prob.info["max_abs_row_sum"]
    cells = [(a, b) for a in kg for b in ksg]
    R = len(cells) * per_cell
    K = np.stack([synth.ramp(0.0, a * 0.5 / (DT * rowsum), steps) for a, b in cells
                  for _ in range(per_cell)]).astype(np.float32)
    Ks = np.stack([synth.triangle(b * 0.5 / (DT * q), 5, steps) for a, b in cells
                   for _ in range(per_cell)]).astype(np.float32)
    sg = np.full((R, steps), 0.1, np.float32)
    dK, dKs, dsg = (torch.from_numpy(x).to(dev) for x in (K, Ks, sg))
    th_init = torch.from_numpy(synth.theta0(R, g.n, seed=100)).to(dev)
    seeds = torch.from_numpy(synth.seeds(R, 0)).to(dev)
    theta = torch.empty_like(th_init)
    best_h = torch.empty(R, dtype=torch.float64, device=dev)
    trace = torch.empty((oim.n_readouts(steps, M), R), dtype=torch.float64, device=dev)
    best_step = torch.empty(R, dtype=torch.int32, device=dev)
    launch, _ = tune.tuned(prob, th_init, dK[0], dKs[0], dsg[0], seeds, q=q, dt=DT,
                           trial_steps=500)

    def sweep():
        theta.copy_(th_init)
        oim.oim_run(prob.handle, g.n, theta, dK, dKs, dsg, seeds, q=q, dt=DT, readout_every=M,
                    trace=trace, best_h=best_h, best_step=best_step)

    for _ in range(args.warmup):
        sweep()
    t_batched = float(np.median([_sync_time(sweep) for _ in range(max(1, args.steps))]))
    W = -prob.info["sum_J_upper"]
    cut = (W - best_h.cpu().numpy()) / 2.0
    grid = cut.reshape(len(kg), len(ksg), per_cell).max(axis=2)
    per = []
    for c in range(min(8, len(cells))):
        sl = slice(c * per_cell, (c + 1) * per_cell)
        thc = th_init[sl].clone()

        def one():
            thc.copy_(th_init[sl])
            oim.oim_run(prob.handle, g.n, thc, dK[sl].contiguous(), dKs[sl].contiguous(),
                        dsg[sl].contiguous(), seeds[sl].contiguous(), q=q, dt=DT)
        one()
        per.append(_sync_time(one))
    plain_total = float(np.mean(per)) * len(cells)
    eu = float(g.nnz) * R * steps
    bi, bj = np.unravel_index(np.argmax(grid), grid.shape)
    out = {
        "value": eu / t_batched, "unit": "edge-updates/s", "ms_per_solve": t_batched * 1e3,
        "dtype": "f32",
        "config": {"workload": "schedule sweep on the 100x100 +-1 torus: 8 x 8 (K_max, Ks_max) "
                               "grid x 4 replicas, per-replica schedules, one launch",
                   "replicas": R, "em_steps": steps, "K_multipliers": kg, "Ks_multipliers": ksg},
        "launch": {"block": launch["block"], "slices_per_wave": launch["slices_per_wave"],
                   "rows_per_lane": launch.get("rows_per_lane", 4)},
        "best_cut_grid": grid.tolist(),
        "best_cell": {"K_mult": kg[bi], "Ks_mult": ksg[bj], "cut": float(grid[bi, bj])},
        "plain": {"ms_per_cell": float(np.mean(per)) * 1e3, "ms_total_extrapolated":
                  plain_total * 1e3, "speedup_batched": plain_total / t_batched},
    }
    prob.close()
    return out


# ----------------------------------------------------------------- main ----
# The paper's own figures (its Table 1, Table 2 and abstract), on its own
# hardware and its own instances: context for the numbers above, not a target
# (it reports no edge-updates/s, no per-step time and no time to a target).
PAPER_CONTEXT = {
    "hardware": "one NVIDIA A100 SXM4 80 GB, FP32 kernels; CPU baseline: the same algorithm "
                "in C on an AMD EPYC 7513 (32 cores, 2.6 GHz)",
    "maxcut_speedup_over_cpu": "795x to 11295x over 32 G-set graphs of 800 to 20000 nodes "
                               "(Table 1); 11295x on the 20000-node graph",
    "maxcut_accuracy": "94.08 % to 99.27 % of the best known cut (Table 1)",
    "maxcut_gpu_time": "0.45 s to 0.53 s per graph at 800 to 1000 nodes, 23.37 s at "
                       "20000 nodes (Table 1)",
    "colouring_speedup_over_cpu": "1.5x to 50x on 50 to 200-node flat graphs, 1091x to "
                                  "8550x on 1000 to 8000-node graphs (Table 2)",
    "colouring_accuracy": "95.2 % to 99.5 % (Table 2)",
    "note": "other hardware and other instances; the paper's CPU code is dense O(n^2) per step",
}


def _line(args, w, headline_name):
    """The contract's JSON line around a workload's result."""
    out = {"metric": METRIC, "value": w["value"], "unit": w["unit"], "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": w["ms_per_solve"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": w.get("dtype", "f32"), "data": "synthetic"}
    for k, v in w.items():
        if k not in ("value", "unit", "ms_per_solve", "dtype"):
            out[k] = v
    cb = w.get("cpu_baseline")
    if cb:
        # the GPU's rate over the oracle's on this host, all threads and one
        out["gpu_over_oracle"] = {"all_threads": w["value"] / cb["value"],
                                  "one_thread": w["value"] / cb["single_thread_value"]}
    out["headline_workload"] = headline_name
    out["paper_context"] = PAPER_CONTEXT
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed solves of the headline workload")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="all",
                    choices=["all", "torus", "gnp800", "gnp800_plain", "sk4096", "sk4096_fp32",
                             "sk20000", "colouring", "adjoint", "sweep"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="oracle seconds per baseline (the headline's; others take a share)")
    ap.add_argument("--plain", type=int, default=8,
                    help="replicas timed in the plain one-launch-per-replica loop")
    ap.add_argument("--dense-steps", type=int, default=0,
                    help="EM steps per dense solve (0: 1000 at n = 4096, 100 at n = 20000)")
    ap.add_argument("--dense-reps", type=int, default=5, help="timed dense solves")
    ap.add_argument("--plain-graphs", type=int, default=32,
                    help="graphs timed in the plain per-graph loop of the batched workloads")
    ap.add_argument("--colour-replicas", type=int, default=8,
                    help="replicas per graph in the colouring batch")
    ap.add_argument("--stepwise", type=int, default=1,
                    help="also time the torus solve on the stepwise hipGraph loop (0: skip)")
    ap.add_argument("--launch", default="",
                    help="BxSxL: run the torus, G(800, 0.06) and colouring workloads with "
                         "that launch shape (threads x slices per wave x rows per lane) "
                         "instead of the autotuner's (for counter runs on a given shape)")
    ap.add_argument("--stepwise-steps", type=int, default=0,
                    help="EM steps of the stepwise solve (0: the whole schedule; fewer for "
                         "counter runs, which serialise every step kernel)")
    ap.add_argument("--ref-mult", type=int, default=10,
                    help="length multiple of the untimed reference run that sets best_ref")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(replicas shard across GPUs with no exchange, see the design notes)",
              file=sys.stderr)
        raise SystemExit(2)

    import synth

    def torus(a):
        return maxcut_workload(a, "torus", synth.torus(100, 100, seed=1, signed=True), 256,
                               10000, 100, "sparse max-cut at scale: 100x100 +-1 torus",
                               a.steps, a.plain, stepwise=bool(a.stepwise))

    def gnp(a, R):
        return maxcut_workload(a, "gnp800", synth.erdos_renyi(800, 0.06, seed=0), R, 1000, 10,
                               f"plain Ising max-cut: G(800, 0.06) unit weights, {R} replica(s)",
                               max(1, min(a.steps, 10)), a.plain if R > 1 else 0)

    single = {"torus": torus, "gnp800": lambda a: gnp(a, 256), "gnp800_plain": lambda a: gnp(a, 1),
              "sk4096": lambda a: dense_workload(a), "sk4096_fp32": lambda a: dense_workload(a, fp32=True),
              "sk20000": lambda a: dense_workload(a, n=20000), "colouring": colouring_workload,
              "adjoint": adjoint_workload, "sweep": sweep_workload}
    if args.workload != "all":
        print(json.dumps(_line(args, single[args.workload](args), args.workload)))
        return
    # every configuration; the headline is the torus
    head = torus(args)
    sub_args = argparse.Namespace(**vars(args))
    sub_args.ref_mult = min(args.ref_mult, 10)
    sub_args.cpu_seconds = args.cpu_seconds / 3.0
    workloads = {}
    for name, fn in (("gnp800_plain", lambda a: gnp(a, 1)), ("gnp800_batched", lambda a: gnp(a, 256)),
                     ("colouring", colouring_workload),
                     ("sk4096_bf16x3", lambda a: dense_workload(a)),
                     ("sk4096_fp32", lambda a: dense_workload(a, fp32=True)),
                     ("adjoint", adjoint_workload)):
        t0 = time.perf_counter()
        workloads[name] = fn(sub_args)
        workloads[name]["bench_wall_s"] = time.perf_counter() - t0
        cb = workloads[name].get("cpu_baseline")
        if cb:
            workloads[name]["gpu_over_oracle"] = {
                "all_threads": workloads[name]["value"] / cb["value"],
                "one_thread": workloads[name]["value"] / cb["single_thread_value"]}
        print(f"[bench] {name} done in {workloads[name]['bench_wall_s']:.1f} s", file=sys.stderr,
              flush=True)
    out = _line(args, head, "torus")
    out["workloads"] = workloads
    print(json.dumps(out))


if __name__ == "__main__":
    main()
