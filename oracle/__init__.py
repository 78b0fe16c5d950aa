"""Plain FP64 CPU oracle for the simulated oscillator Ising/Potts machine.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It shares no
code with the GPU library; the only thing both sides use is the seeded input
generator module ``synth``.

The arithmetic lives in ``oracle.c`` (FP64, Algorithm 1 / Eq. 5 of the paper,
Philox4x32-10 + Box-Muller noise); this module marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_i32, _i64, _u32, _u64, _f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                ctypes.c_uint64, ctypes.c_double)
_P = ctypes.c_void_p


def lib():
    """Load liboracle.so, compiling it with gcc first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_philox4x32_10.argtypes = [_P, _P, _P]
        L.orc_philox4x32_10.restype = None
        L.orc_normal.argtypes = [_u64, _u32, _u32]
        L.orc_normal.restype = _f64
        L.orc_normals.argtypes = [_u64, _u32, _i64, _u32, _P]
        L.orc_normals.restype = None
        L.orc_normal_b.argtypes = [_u64, _u32, _u32, _u32]
        L.orc_normal_b.restype = _f64
        L.orc_run_csr_blocks.argtypes = [_i32, _P, _P, _P, _i32, _P, _i32, _i32, _i32, _i64, _f64,
                                         _P, _P, _P, _P, _P, _i32]
        L.orc_run_csr_blocks.restype = ctypes.c_int
        L.orc_run_csr.argtypes = [_i32, _P, _P, _P, _i32, _i32, _i32, _i64, _f64, _P, _P, _P, _P,
                                  _P, _i32]
        L.orc_run_csr.restype = ctypes.c_int
        L.orc_adjoint_csr.argtypes = [_i32, _P, _P, _P, _i32, _i32, _i32, _i64, _f64, _P, _P, _P,
                                      _P, _P, _P, _P, _P, _P]
        L.orc_adjoint_csr.restype = ctypes.c_int
        L.orc_adjoint_csr_blocks.argtypes = [_i32, _P, _P, _P, _i32, _P, _i32, _i32, _i32, _i64,
                                             _f64, _P, _P, _P, _P, _P, _P, _P, _P, _P]
        L.orc_adjoint_csr_blocks.restype = ctypes.c_int
        L.orc_run_dense.argtypes = [_i32, _P, _i32, _i32, _i32, _i64, _f64, _P, _P, _P, _P, _P,
                                    _i32]
        L.orc_run_dense.restype = ctypes.c_int
        L.orc_run_dense_bf16x3.argtypes = [_i32, _P, _i32, _i32, _i32, _i64, _f64, _P, _P, _P, _P,
                                           _P, _i32]
        L.orc_run_dense_bf16x3.restype = ctypes.c_int
        L.orc_coupling_dense_bf16x3.argtypes = [_i32, _P, _P, _P]
        L.orc_coupling_dense_bf16x3.restype = None
        L.orc_bf16_round.argtypes = [ctypes.c_float]
        L.orc_bf16_round.restype = ctypes.c_float
        L.orc_round_f32.argtypes = [_i64, _P, _i32, _P]
        L.orc_round_f32.restype = None
        L.orc_cut_int.argtypes = [_i32, _P, _P, _P, _P]
        L.orc_cut_int.restype = _i64
        L.orc_cut_f64.argtypes = [_i32, _P, _P, _P, _P]
        L.orc_cut_f64.restype = _f64
        L.orc_conflicts.argtypes = [_i32, _P, _P, _P, _P]
        L.orc_conflicts.restype = _i64
        L.orc_h_model.argtypes = [_i32, _P, _P, _P, _i32, _P]
        L.orc_h_model.restype = _f64
        L.orc_h_eq6.argtypes = [_i32, _P, _P, _P, _P]
        L.orc_h_eq6.restype = _f64
        L.orc_run_csr_instance.argtypes = [_i32, _P, _P, _P, _u32, _i32, _i32, _i32, _i64, _f64,
                                           _P, _P, _P, _P, _P, _i32]
        L.orc_run_csr_instance.restype = ctypes.c_int
        L.orc_pairwise_tree.argtypes = [_P, _i64]
        L.orc_pairwise_tree.restype = _f64
        L.orc_upper_row_sums.argtypes = [_i32, _P, _P, _P, _i32, _i32, _P, _P, _P]
        L.orc_upper_row_sums.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------- noise ----
def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block function (Salmon et al., SC'11)."""
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    assert c.shape == (4,) and k.shape == (2,)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normal(seed: int, i: int, t: int, instance: int = 0) -> float:
    """The standard normal that drives oscillator i (of `instance`) at global step t."""
    return lib().orc_normal_b(int(seed), int(i), int(t), int(instance))


def normals(seed: int, i0: int, count: int, t: int) -> np.ndarray:
    out = np.zeros(int(count), np.float64)
    lib().orc_normals(int(seed), int(i0), int(count), int(t), _ptr(out))
    return out


# ----------------------------------------------------------- integrator ----
def _sched(a, steps):
    a = _c(a, np.float64)
    if a.shape != (steps,):
        raise ValueError(f"schedule must have shape ({steps},), got {a.shape}")
    return a


def _per_replica(fn, theta0, K, Ks, sigma, seeds, **kw):
    """Schedules given per replica ([R][steps]): replicas are independent, so
    each one is integrated on its own with its own row of the schedules."""
    th = np.atleast_2d(np.asarray(theta0, np.float64))
    sd = np.asarray(seeds, np.uint64)
    out = np.empty_like(th)
    for r in range(th.shape[0]):
        out[r] = fn(th[r:r + 1], K=np.asarray(K)[r], Ks=np.asarray(Ks)[r],
                    sigma=np.asarray(sigma)[r], seeds=sd[r:r + 1], **kw)[0]
    return out


def run_csr(row_ptr, col, J, theta0, *, q, dt, K, Ks, sigma, seeds, step0=0, nthreads=0,
            instance=0):
    """Integrate Eq. 5 (Algorithm 1) on a CSR coupling; returns theta [R][n] in FP64.
    K, Ks, sigma are [steps] (shared) or [R][steps] (one schedule per replica).
    `instance` = b integrates the graph as instance b of a block-diagonal batch
    (the noise counter carries b)."""
    if np.ndim(K) == 2:
        return _per_replica(lambda th, **k: run_csr(row_ptr, col, J, th, **k), theta0, K, Ks,
                            sigma, seeds, q=q, dt=dt, step0=step0, nthreads=nthreads,
                            instance=instance)
    rp = _c(row_ptr, np.int64)
    cl = _c(col, np.int32)
    Jv = _c(J, np.float64)
    th = np.array(theta0, dtype=np.float64, order="C", copy=True)
    if th.ndim == 1:
        th = th[None, :]
    R, n = th.shape
    steps = len(K)
    sd = _c(seeds, np.uint64)
    assert sd.shape == (R,) and rp.shape == (n + 1,)
    rc = lib().orc_run_csr_instance(n, _ptr(rp), _ptr(cl), _ptr(Jv), int(instance), int(q), R,
                                    steps, int(step0), float(dt), _ptr(_sched(K, steps)),
                                    _ptr(_sched(Ks, steps)), _ptr(_sched(sigma, steps)),
                                    _ptr(sd), _ptr(th), int(nthreads))
    if rc != 0:
        raise ValueError("orc_run_csr_instance rejected its arguments")
    return th


def run_csr_blocks(row_ptr, col, J, inst_off, theta0, *, q, dt, K, Ks, sigma, seeds, step0=0,
                   nthreads=0):
    """Integrate a block-diagonal batch of instances (inst_off[b]..inst_off[b+1]-1)."""
    if np.ndim(K) == 2:
        return _per_replica(lambda th, **k: run_csr_blocks(row_ptr, col, J, inst_off, th, **k),
                            theta0, K, Ks, sigma, seeds, q=q, dt=dt, step0=step0,
                            nthreads=nthreads)
    rp = _c(row_ptr, np.int64)
    cl = _c(col, np.int32)
    Jv = _c(J, np.float64)
    io = _c(inst_off, np.int32)
    th = np.array(theta0, dtype=np.float64, order="C", copy=True)
    if th.ndim == 1:
        th = th[None, :]
    R, n = th.shape
    steps = len(K)
    sd = _c(seeds, np.uint64)
    assert sd.shape == (R,) and rp.shape == (n + 1,) and io[-1] == n
    rc = lib().orc_run_csr_blocks(n, _ptr(rp), _ptr(cl), _ptr(Jv), len(io) - 1, _ptr(io), int(q), R,
                                  steps, int(step0), float(dt), _ptr(_sched(K, steps)),
                                  _ptr(_sched(Ks, steps)), _ptr(_sched(sigma, steps)), _ptr(sd),
                                  _ptr(th), int(nthreads))
    if rc != 0:
        raise ValueError("orc_run_csr_blocks rejected its arguments")
    return th


def adjoint_csr(row_ptr, col, J, theta0, *, q, dt, K, Ks, sigma, seeds, step0=0,
                inst_off=None):
    """Relaxed-cut loss of the final phases (sum over replicas and instances) and its
    gradient with respect to the per-step K, Ks and sigma of the fixed-noise
    trajectory.  inst_off splits the graph into block-diagonal instances."""
    rp = _c(row_ptr, np.int64)
    cl = _c(col, np.int32)
    Jv = _c(J, np.float64)
    th = np.ascontiguousarray(np.atleast_2d(np.asarray(theta0, np.float64)))
    R, n = th.shape
    steps = len(K)
    sd = _c(seeds, np.uint64)
    io = _c([0, n] if inst_off is None else inst_off, np.int32)
    assert sd.shape == (R,) and rp.shape == (n + 1,) and io[-1] == n
    loss = np.zeros(1)
    gK, gKs, gS = np.zeros(steps), np.zeros(steps), np.zeros(steps)
    rc = lib().orc_adjoint_csr_blocks(n, _ptr(rp), _ptr(cl), _ptr(Jv), len(io) - 1, _ptr(io),
                                      int(q), R, steps, int(step0), float(dt),
                                      _ptr(_sched(K, steps)), _ptr(_sched(Ks, steps)),
                                      _ptr(_sched(sigma, steps)), _ptr(sd), _ptr(th), _ptr(loss),
                                      _ptr(gK), _ptr(gKs), _ptr(gS))
    if rc != 0:
        raise ValueError("orc_adjoint_csr_blocks rejected its arguments")
    return float(loss[0]), gK, gKs, gS


def relaxed_cut(row_ptr, col, J, theta):
    """sum over replicas of sum_{i<j} w_ij (1 - cos(th_i - th_j)) / 2, w = -J (numpy)."""
    th = np.atleast_2d(np.asarray(theta, np.float64))
    rp = np.asarray(row_ptr)
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    cl = np.asarray(col)
    up = rows < cl
    w = -np.asarray(J, np.float64)[up]
    d = th[:, rows[up]] - th[:, cl[up]]
    return float(np.sum(0.5 * w * (1.0 - np.cos(d))))


def run_dense(J, theta0, *, q, dt, K, Ks, sigma, seeds, step0=0, nthreads=0, precision="fp64"):
    """Integrate Eq. 5 with the all-pairs (dense) coupling sum, diagonal ignored.

    precision "fp64": the direct sum of J_ij sin(th_i - th_j) in FP64.
    precision "bf16x3": the coupling through sin(a - b) = sin a cos b - cos a sin b
    with every GEMM operand split into two BF16 halves and the three products
    J_hi X_hi + J_hi X_lo + J_lo X_hi (FP64 products and sums); the rest of the
    step in FP64."""
    if np.ndim(K) == 2:
        return _per_replica(lambda th, **k: run_dense(J, th, precision=precision, **k), theta0,
                            K, Ks, sigma, seeds, q=q, dt=dt, step0=step0, nthreads=nthreads)
    if precision not in ("fp64", "bf16x3"):
        raise ValueError(f"unknown precision {precision!r}")
    Jd = _c(J, np.float64)
    th = np.array(theta0, dtype=np.float64, order="C", copy=True)
    if th.ndim == 1:
        th = th[None, :]
    R, n = th.shape
    assert Jd.shape == (n, n)
    steps = len(K)
    sd = _c(seeds, np.uint64)
    fn = lib().orc_run_dense if precision == "fp64" else lib().orc_run_dense_bf16x3
    rc = fn(n, _ptr(Jd), int(q), R, steps, int(step0), float(dt), _ptr(_sched(K, steps)),
            _ptr(_sched(Ks, steps)), _ptr(_sched(sigma, steps)), _ptr(sd), _ptr(th),
            int(nthreads))
    if rc != 0:
        raise ValueError("dense oracle run rejected its arguments")
    return th


def coupling_dense_bf16x3(J, theta) -> np.ndarray:
    """One coupling evaluation c_i of the BF16x3 split-product form (see
    run_dense) for one phase vector; FP64 out."""
    Jd = _c(J, np.float64)
    th = _c(theta, np.float64)
    n = th.shape[0]
    assert Jd.shape == (n, n) and th.ndim == 1
    out = np.zeros(n, np.float64)
    lib().orc_coupling_dense_bf16x3(n, _ptr(Jd), _ptr(th), _ptr(out))
    return out


def bf16_round(x: float) -> float:
    """BF16 rounding (to nearest, ties to even) of an FP32 value, as the
    oracle's split uses it."""
    return float(lib().orc_bf16_round(float(np.float32(x))))


# -------------------------------------------------------------- readout ----
def round_f32(theta, q) -> np.ndarray:
    """Nearest stable phase index k = floor(q theta / 2 pi + 1/2) mod q (FP32 decision)."""
    th = _c(theta, np.float32)
    out = np.zeros(th.shape, np.int8)
    lib().orc_round_f32(th.size, _ptr(th), int(q), _ptr(out))
    return out


def dense_to_csr(J):
    """Off-diagonal nonzeros of a dense coupling as (row_ptr, col, values)."""
    J = np.asarray(J, dtype=np.float64)
    n = J.shape[0]
    mask = J != 0.0
    np.fill_diagonal(mask, False)
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr), cols.astype(np.int32), J[rows, cols]


def cut_int(row_ptr, col, J, colour) -> int:
    rp, cl = _c(row_ptr, np.int64), _c(col, np.int32)
    Ji = _c(J, np.int64)
    co = _c(colour, np.int8)
    return int(lib().orc_cut_int(len(rp) - 1, _ptr(rp), _ptr(cl), _ptr(Ji), _ptr(co)))


def cut_f64(row_ptr, col, J, colour) -> float:
    rp, cl = _c(row_ptr, np.int64), _c(col, np.int32)
    Jv = _c(J, np.float64)
    co = _c(colour, np.int8)
    return float(lib().orc_cut_f64(len(rp) - 1, _ptr(rp), _ptr(cl), _ptr(Jv), _ptr(co)))


def conflicts(row_ptr, col, J, colour) -> int:
    rp, cl = _c(row_ptr, np.int64), _c(col, np.int32)
    Jv = _c(J, np.float64)
    co = _c(colour, np.int8)
    return int(lib().orc_conflicts(len(rp) - 1, _ptr(rp), _ptr(cl), _ptr(Jv), _ptr(co)))


def h_model(row_ptr, col, J, q, colour) -> float:
    """Eq. 1 (q = 2) or Eq. 2 (q >= 3) at the given colours."""
    rp, cl = _c(row_ptr, np.int64), _c(col, np.int32)
    Jv = _c(J, np.float64)
    co = _c(colour, np.int8)
    return float(lib().orc_h_model(len(rp) - 1, _ptr(rp), _ptr(cl), _ptr(Jv), int(q), _ptr(co)))


def h_eq6(row_ptr, col, J, theta) -> float:
    """Eq. 6 with w = -J at continuous phases theta (radians)."""
    rp, cl = _c(row_ptr, np.int64), _c(col, np.int32)
    Jv = _c(J, np.float64)
    th = _c(theta, np.float64)
    return float(lib().orc_h_eq6(len(rp) - 1, _ptr(rp), _ptr(cl), _ptr(Jv), _ptr(th)))


# ------------------------------------------------- fixed-order readouts ----
# The order every GPU readout of a real-weighted sum follows: per row i, the
# terms of j > i in ascending column order, summed in FP64 from +0; then the
# pairwise tree over the rows (zero-padded to a power of two, adjacent pairs
# first).  Integer weights give the same value in any order.
def pairwise_tree(values) -> float:
    v = _c(values, np.float64)
    return float(lib().orc_pairwise_tree(_ptr(v), v.size))


def upper_row_sums(row_ptr, col, J, kind, *, q=2, colour=None, theta=None) -> np.ndarray:
    """Per-row FP64 sums over j > i: kind 'cut' (-J when colours differ),
    'model' (Eq. 1 for q = 2, Eq. 2 for q >= 3) or 'eq6' (-J cos(th_i - th_j))."""
    rp, cl = _c(row_ptr, np.int64), _c(col, np.int32)
    Jv = _c(J, np.float64)
    n = len(rp) - 1
    k = {"cut": 0, "model": 1, "eq6": 2}[kind]
    co = _c(colour if colour is not None else np.zeros(n), np.int8)
    th = _c(theta if theta is not None else np.zeros(n), np.float64)
    assert co.shape == (n,) and th.shape == (n,)
    out = np.zeros(n, np.float64)
    lib().orc_upper_row_sums(n, _ptr(rp), _ptr(cl), _ptr(Jv), k, int(q), _ptr(co), _ptr(th),
                             _ptr(out))
    return out


def _fixed(row_ptr, col, J, kind, inst_off, **kw):
    rows = upper_row_sums(row_ptr, col, J, kind, **kw)
    if inst_off is None:
        return pairwise_tree(rows)
    return np.array([pairwise_tree(rows[inst_off[b]:inst_off[b + 1]])
                     for b in range(len(inst_off) - 1)])


def cut_fixed(row_ptr, col, J, colour, inst_off=None):
    """Max-cut value sum_{i<j} (-J_ij) [k_i != k_j] in the fixed FP64 order
    (per instance when inst_off is given)."""
    return _fixed(row_ptr, col, J, "cut", inst_off, colour=colour)


def h_model_fixed(row_ptr, col, J, q, colour, inst_off=None):
    """Eq. 1 (q = 2) or Eq. 2 (q >= 3) in the fixed FP64 order."""
    return _fixed(row_ptr, col, J, "model", inst_off, q=q, colour=colour)


def h_eq6_fixed(row_ptr, col, J, theta, inst_off=None):
    """Eq. 6 with w = -J at continuous phases, in the fixed FP64 order."""
    return _fixed(row_ptr, col, J, "eq6", inst_off, theta=theta)
