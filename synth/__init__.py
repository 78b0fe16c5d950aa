"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method itself: it only builds graphs
(edge weights w, symmetric CSR), dense coupling matrices, initial phases,
per-step schedule arrays and per-replica seeds.  Mapping a problem onto the
Ising/Potts coupling J (e.g. J = -w for max-cut) is done separately by each
consumer.  All randomness is numpy PCG64 with an explicit seed.

Workload shapes follow the paper's benchmarks, which are not available here:
  * G(n=800, p=0.06) unit-weight graphs stand in for the 800-node G-set rows
    (Table 1).
  * a 100x100 +-1 torus stands in for the 10000-node toroidal G-set rows.
  * planted 3-colourable graphs with average degree 4.6 stand in for the SATLIB
    "flat" colouring instances (Table 2).
  * a Sherrington-Kirkpatrick matrix J_ij ~ N(0, 1/n) is the all-to-all case.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

TWO_PI = 2.0 * np.pi


@dataclass
class Graph:
    """Undirected graph as a symmetric CSR: both (i,j) and (j,i) are stored,
    columns sorted per row, no self loops, no duplicates.  `w` are edge
    weights (not couplings)."""
    n: int
    row_ptr: np.ndarray  # int64 [n+1]
    col: np.ndarray      # int32 [nnz]
    w: np.ndarray        # float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def n_edges(self) -> int:
        return self.nnz // 2

    def upper_edges(self):
        """(i, j, w) for i < j."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        m = rows < self.col
        return rows[m], self.col[m].astype(np.int64), self.w[m]


def csr_from_edges(n: int, ei, ej, w) -> Graph:
    """Symmetric CSR from an undirected edge list (each edge listed once)."""
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    w = np.asarray(w, dtype=np.float32)
    if ei.size and (ei.min() < 0 or ej.min() < 0 or max(ei.max(), ej.max()) >= n):
        raise ValueError("edge endpoint out of range")
    if np.any(ei == ej):
        raise ValueError("self loop")
    rows = np.concatenate([ei, ej])
    cols = np.concatenate([ej, ei])
    vals = np.concatenate([w, w])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size > 1 and np.any((rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])):
        raise ValueError("duplicate edge")
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return Graph(n, np.cumsum(row_ptr), cols.astype(np.int32), vals.astype(np.float32))


# ------------------------------------------------------------ workloads ----
def erdos_renyi(n: int, p: float, seed: int, signed: bool = False) -> Graph:
    """G(n, p): each pair i < j kept with probability p; weights +1 (or +-1)."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.size) < p
    ei, ej = iu[keep], ju[keep]
    if signed:
        w = np.where(rng.random(ei.size) < 0.5, 1.0, -1.0)
    else:
        w = np.ones(ei.size)
    return csr_from_edges(n, ei, ej, w)


def gnp_avg_degree(n: int, avg_degree: float, seed: int, signed: bool = True) -> Graph:
    """G(n, p = d / (n - 1)) with +-1 weights (p = 0.5 each) when signed."""
    return erdos_renyi(n, avg_degree / (n - 1), seed, signed=signed)


def torus(rows: int, cols: int, seed: int, signed: bool = True) -> Graph:
    """2-D periodic grid: vertex id = cols*r + c, edges to the right and down
    neighbours (with wrap-around); weights +-1 with probability 1/2 each."""
    rng = np.random.default_rng(seed)
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    v = (cols * r + c).ravel()
    right = (cols * r + (c + 1) % cols).ravel()
    down = (cols * ((r + 1) % rows) + c).ravel()
    ei = np.concatenate([v, v])
    ej = np.concatenate([right, down])
    if signed:
        w = np.where(rng.random(ei.size) < 0.5, 1.0, -1.0)
    else:
        w = np.ones(ei.size)
    return csr_from_edges(rows * cols, ei, ej, w)


def planted_colouring(n: int, avg_degree: float, q: int, seed: int):
    """A q-colourable graph: a random vertex permutation is split into the
    classes (index mod q); round(avg_degree * n / 2) distinct edges between
    different classes are drawn uniformly.  Returns (Graph, planted colour)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    colour = np.empty(n, np.int8)
    colour[perm] = (np.arange(n) % q).astype(np.int8)
    m = int(round(avg_degree * n / 2.0))
    max_edges = (n * n - sum(int(np.sum(colour == k)) ** 2 for k in range(q))) // 2
    if m > max_edges:
        raise ValueError("too many edges requested")
    chosen = set()
    ei, ej = [], []
    while len(ei) < m:
        need = m - len(ei)
        a = rng.integers(0, n, size=2 * need + 16)
        b = rng.integers(0, n, size=2 * need + 16)
        for x, y in zip(a.tolist(), b.tolist()):
            if x == y or colour[x] == colour[y]:
                continue
            key = (x, y) if x < y else (y, x)
            if key in chosen:
                continue
            chosen.add(key)
            ei.append(key[0])
            ej.append(key[1])
            if len(ei) == m:
                break
    return csr_from_edges(n, ei, ej, np.ones(m)), colour


def planted_batch(count: int, n_lo: int, n_hi: int, avg_degree: float, q: int, seed: int):
    """`count` planted q-colourable graphs with n uniform in [n_lo, n_hi]."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=count)
    return [planted_colouring(int(nv), avg_degree, q, seed * 100003 + g)
            for g, nv in enumerate(sizes)]


def block_diagonal(graphs):
    """One CSR holding several graphs as disjoint diagonal blocks, and the
    instance offsets (graph b owns nodes off[b] .. off[b+1]-1)."""
    off = np.cumsum([0] + [g.n for g in graphs]).astype(np.int32)
    ei, ej, w = [], [], []
    for g, o in zip(graphs, off[:-1]):
        a, b, c = g.upper_edges()
        ei.append(a + o)
        ej.append(b + o)
        w.append(c)
    return csr_from_edges(int(off[-1]), np.concatenate(ei), np.concatenate(ej),
                          np.concatenate(w)), off


def sk_dense(n: int, seed: int) -> np.ndarray:
    """Sherrington-Kirkpatrick coupling: J_ij = z / sqrt(n), z ~ N(0,1) drawn in
    FP64 for i < j, mirrored, zero diagonal, stored as FP32 [n][n]."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, n)) / np.sqrt(n)
    J = np.triu(z, k=1)
    J = J + J.T
    return J.astype(np.float32)


# ------------------------------------------------------ small pin graphs ----
def cycle(n: int) -> Graph:
    i = np.arange(n)
    return csr_from_edges(n, i, (i + 1) % n, np.ones(n))


def complete(n: int) -> Graph:
    iu, ju = np.triu_indices(n, k=1)
    return csr_from_edges(n, iu, ju, np.ones(iu.size))


def complete_bipartite(a: int, b: int) -> Graph:
    ei = np.repeat(np.arange(a), b)
    ej = a + np.tile(np.arange(b), a)
    return csr_from_edges(a + b, ei, ej, np.ones(a * b))


def petersen() -> Graph:
    outer = [(k, (k + 1) % 5) for k in range(5)]
    spokes = [(k, k + 5) for k in range(5)]
    inner = [(5 + k, 5 + (k + 2) % 5) for k in range(5)]
    e = np.array(outer + spokes + inner)
    return csr_from_edges(10, e[:, 0], e[:, 1], np.ones(len(e)))


def random_small(n: int, p: float, seed: int, weights: str = "unit") -> Graph:
    """Tiny random graphs for brute-force checks; weights 'unit', 'pm1' or
    'int' (integers in [-3, 3] without 0) or 'real' (uniform (-1, 1))."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.size) < p
    ei, ej = iu[keep], ju[keep]
    m = ei.size
    if weights == "unit":
        w = np.ones(m)
    elif weights == "pm1":
        w = np.where(rng.random(m) < 0.5, 1.0, -1.0)
    elif weights == "int":
        w = rng.integers(1, 4, size=m) * np.where(rng.random(m) < 0.5, 1, -1)
    elif weights == "real":
        w = rng.uniform(-1.0, 1.0, size=m).astype(np.float32)
    else:
        raise ValueError(weights)
    return csr_from_edges(n, ei, ej, w)


# ----------------------------------------------- phases, schedules, seeds ----
def theta0(R: int, n: int, seed: int) -> np.ndarray:
    """Initial phases uniform in [0, 2 pi), FP32, shape [R][n]."""
    rng = np.random.default_rng(seed)
    th = (rng.random((R, n)) * TWO_PI).astype(np.float32)
    top = np.nextafter(np.float32(TWO_PI), np.float32(0))
    return np.where(th.astype(np.float64) >= TWO_PI, top, th).astype(np.float32)


def ramp(a: float, b: float, steps: int) -> np.ndarray:
    """Linear schedule from a (first step) to b (last step), FP32."""
    if steps <= 1:
        return np.full(max(steps, 0), b, np.float32)
    return (a + (b - a) * np.arange(steps) / (steps - 1)).astype(np.float32)


def const(v: float, steps: int) -> np.ndarray:
    return np.full(steps, v, np.float32)


def triangle(amp: float, periods: int, steps: int) -> np.ndarray:
    """Triangular waveform rising from 0 to amp and back to 0, `periods` times
    over the run (the annealing waveform of Algorithm 1 / Sec. III-D)."""
    t = np.arange(steps, dtype=np.float64)
    frac = (periods * t / max(steps, 1)) % 1.0
    return (amp * (1.0 - np.abs(2.0 * frac - 1.0))).astype(np.float32)


def seeds(R: int, base: int = 0) -> np.ndarray:
    return (np.uint64(base) + np.arange(R, dtype=np.uint64)).astype(np.uint64)


# ---------------------------------------------------- benchmark configs ----
def gershgorin(g: Graph) -> float:
    """max_i sum_j |w_ij| of a graph (stability bound used to size K)."""
    s = np.zeros(g.n)
    np.add.at(s, np.repeat(np.arange(g.n), np.diff(g.row_ptr)), np.abs(g.w))
    return float(s.max()) if g.n else 0.0


# ------------------------------------------------ benchmark schedules ----
# The paper prints no K, Ks or noise values.  The benchmark workloads use
# linear K ramps from 0 to k_mul * 0.5 / (dt * max_i sum_j |J_ij|), Ks either
# a linear ramp to ks_mul * 0.5 / (dt * q) or the triangular annealing
# waveform with that amplitude, and a constant noise amplitude; the
# multipliers were frozen from sweeps on each workload before any timing.
WORKLOAD_SCHEDULES = {
    # plain Ising max-cut, G(800, 0.06) unit weights, 1000 steps
    "gnp800": dict(q=2, k_mul=8.0, ks_mul=0.25, ks_shape="ramp", periods=0, sigma=0.1),
    # sparse max-cut at scale, 100 x 100 +-1 torus, 10000 steps
    "torus": dict(q=2, k_mul=2.0, ks_mul=1.0, ks_shape="triangle", periods=5, sigma=0.1),
    # batched Potts 3-colouring, 1024 planted graphs, 5000 steps
    "colouring": dict(q=3, k_mul=4.0, ks_mul=0.5, ks_shape="triangle", periods=10, sigma=0.2),
    # dense SK, n = 4096 (the Gershgorin bound is loose for all-to-all
    # couplings, hence the large K multiplier), 1000 steps
    "sk": dict(q=2, k_mul=32.0, ks_mul=0.03, ks_shape="ramp", periods=0, sigma=0.1),
    # adjoint schedule tuning, 128 x G(2000, 10/1999) +-1, 2000 steps
    "adjoint": dict(q=2, k_mul=2.0, ks_mul=1.0, ks_shape="triangle", periods=5, sigma=0.1),
}


def workload_schedule(name: str, max_row_sum: float, steps: int, dt: float):
    """(K, Ks, sigma, K_max, Ks_max) of a benchmark workload's frozen recipe."""
    wl = WORKLOAD_SCHEDULES[name]
    q = wl["q"]
    kmax = wl["k_mul"] * 0.5 / (dt * max_row_sum)
    ksmax = wl["ks_mul"] * 0.5 / (dt * q)
    K = ramp(0.0, kmax, steps)
    if wl["ks_shape"] == "triangle":
        Ks = triangle(ksmax, wl["periods"], steps)
    else:
        Ks = ramp(0.0, ksmax, steps)
    return K, Ks, const(wl["sigma"], steps), kmax, ksmax
