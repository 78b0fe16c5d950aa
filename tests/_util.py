"""Shared helpers of the test suite (workload recipes, comparisons)."""
import numpy as np

import synth

TWO_PI = 2 * np.pi
DT = float(np.float32(0.01))  # the FP32 time step both sides see


def wrapdiff(a, b):
    d = np.mod(np.asarray(a, np.float64) - np.asarray(b, np.float64), TWO_PI)
    return np.minimum(d, TWO_PI - d)


def ramp_schedule(max_row_sum, q, total_steps, use_steps=None, sigma=0.1, dt=DT):
    """Linear K and Ks ramps from 0 to K_max = 0.5 / (dt max_i sum_j |J_ij|) and
    Ks_max = 0.5 / (dt q) over `total_steps`, constant noise; the first
    `use_steps` steps are returned."""
    kmax = 0.5 / (dt * max(max_row_sum, 1e-30))
    ksmax = 0.5 / (dt * q)
    K = synth.ramp(0.0, kmax, total_steps)
    Ks = synth.ramp(0.0, ksmax, total_steps)
    sg = synth.const(sigma, total_steps)
    u = total_steps if use_steps is None else use_steps
    return K[:u].copy(), Ks[:u].copy(), sg[:u].copy()


def c1_graph():
    """Plain Ising max-cut workload: G(n=800, p=0.06), unit weights, seed 0."""
    return synth.erdos_renyi(800, 0.06, seed=0)


def c2_graph():
    """Sparse max-cut at scale: 100x100 torus, +-1 weights, seed 1."""
    return synth.torus(100, 100, seed=1, signed=True)


def c5_batch(count=128, n=2000, avg_degree=10.0):
    """Adjoint schedule-tuning workload: `count` graphs G(n, p = d/(n-1)) with
    +-1 weights (graph g drawn with seed 4 + g), as one block-diagonal batch."""
    gs = [synth.gnp_avg_degree(n, avg_degree, seed=4 + g, signed=True) for g in range(count)]
    return synth.block_diagonal(gs)
