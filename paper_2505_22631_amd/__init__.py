"""MI355X simulated oscillator Ising/Potts machine (arXiv 2505.22631).

Thin Python binding of liboim.so (include/oim.h).  Every function here only
checks and marshals arguments; all of the work runs in the HIP kernels.  torch
supplies device memory and the current HIP stream.

Functions carry the C names: oim_problem_from_csr, oim_problem_from_dense,
oim_problem_destroy, oim_problem_info_get, oim_run, oim_round, oim_cut,
oim_conflicts, oim_energy, oim_adjoint_forward, oim_adjoint_backward.
`Problem` and `run` are small conveniences on top; `autograd.RelaxedCut` puts
the adjoint kernels behind a torch.autograd.Function.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from ._lib import (OIM_LOOP_AUTO, OIM_LOOP_PERSISTENT, OIM_LOOP_STEPWISE, OIM_PREC_BF16X3,
                   OIM_PREC_FP32, OIM_SCHED_PER_REPLICA, AdjointCfg, OimError, Readout, RunCfg, check, lib)

__all__ = [
    "OIM_LOOP_AUTO", "OIM_LOOP_PERSISTENT", "OIM_LOOP_STEPWISE", "OIM_PREC_FP32",
    "OIM_PREC_BF16X3", "OIM_SCHED_PER_REPLICA", "OimError", "Problem", "oim_abi_version", "oim_problem_from_csr",
    "oim_problem_from_csr_blocks", "oim_problem_from_dense", "oim_problem_destroy", "oim_problem_info_get", "oim_run",
    "oim_run_noalloc", "oim_noalloc_scratch_bytes",
    "oim_round", "oim_cut", "oim_conflicts", "oim_energy", "oim_phase_from_theta",
    "oim_theta_from_phase", "oim_autotune", "oim_set_tuning",
    "oim_adjoint_checkpoint_words", "oim_adjoint_forward",
    "oim_adjoint_backward", "run", "n_readouts",
]


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dev(t, dtype, shape=None, name="tensor", allow_none=False):
    """Device pointer of a contiguous CUDA(HIP) tensor of the given dtype/shape."""
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def oim_abi_version() -> int:
    return int(lib().oim_abi_version())


def oim_problem_from_csr(n, row_ptr, col_idx, J, flags=0):
    """Upload a symmetric CSR coupling (host arrays, copied).  Returns a handle."""
    rp = _host(row_ptr, np.int64)
    ci = _host(col_idx, np.int32)
    Jv = _host(J, np.float32)
    if rp.shape != (int(n) + 1,):
        raise ValueError("row_ptr must have n+1 entries")
    if ci.shape != Jv.shape:
        raise ValueError("col_idx and J must have the same length")
    h = ctypes.c_void_p()
    check(lib().oim_problem_from_csr(int(n), int(ci.size), _np_ptr(rp), _np_ptr(ci), _np_ptr(Jv),
                                     int(flags), ctypes.byref(h)))
    return h


def oim_problem_from_csr_blocks(n, row_ptr, col_idx, J, inst_off, flags=0):
    """Upload a block-diagonal batch: instance b = oscillators inst_off[b]..inst_off[b+1]-1."""
    rp = _host(row_ptr, np.int64)
    ci = _host(col_idx, np.int32)
    Jv = _host(J, np.float32)
    io = _host(inst_off, np.int32)
    if rp.shape != (int(n) + 1,):
        raise ValueError("row_ptr must have n+1 entries")
    if ci.shape != Jv.shape:
        raise ValueError("col_idx and J must have the same length")
    h = ctypes.c_void_p()
    check(lib().oim_problem_from_csr_blocks(int(n), int(ci.size), _np_ptr(rp), _np_ptr(ci),
                                            _np_ptr(Jv), int(io.size - 1), _np_ptr(io),
                                            int(flags), ctypes.byref(h)))
    return h


def oim_problem_from_dense(J, flags=0):
    """Upload a dense symmetric coupling J[n][n] (host array, copied)."""
    Jd = _host(J, np.float32)
    if Jd.ndim != 2 or Jd.shape[0] != Jd.shape[1]:
        raise ValueError("J must be square")
    h = ctypes.c_void_p()
    check(lib().oim_problem_from_dense(int(Jd.shape[0]), _np_ptr(Jd), int(flags), ctypes.byref(h)))
    return h


def oim_problem_destroy(h) -> None:
    if h:
        lib().oim_problem_destroy(h)


def oim_problem_info_get(h) -> dict:
    info = _lib.ProblemInfo()
    check(lib().oim_problem_info_get(h, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in _lib.ProblemInfo._fields_}


def n_readouts(steps: int, readout_every: int) -> int:
    return 0 if readout_every <= 0 else -(-int(steps) // int(readout_every))


def _run_args(h, n, theta, K, Ks, sigma, seeds, q, dt, readout_every, flags, step0, phase,
              trace, best_h, best_step, best_colour, stream):
    if theta.dim() != 2 or theta.shape[1] != n:
        raise ValueError("theta must be [R][n]")
    R = int(theta.shape[0])
    per_replica = K.dim() == 2
    steps = int(K.shape[-1])
    if per_replica:
        flags = int(flags) | OIM_SCHED_PER_REPLICA
    sshape = (R, steps) if per_replica else (steps,)
    cfg = RunCfg(int(q), R, steps, float(dt), int(readout_every), int(flags))
    nr = n_readouts(steps, readout_every)
    RI = R * int(oim_problem_info_get(h)["n_instances"])
    ro = Readout(_dev(trace, torch.float64, (nr, RI), "trace", True),
                 _dev(best_h, torch.float64, (RI,), "best_h", True),
                 _dev(best_step, torch.int32, (RI,), "best_step", True),
                 _dev(best_colour, torch.int8, (R, n), "best_colour", True))
    return (h, ctypes.byref(cfg), _dev(K, torch.float32, sshape, "K"),
            _dev(Ks, torch.float32, sshape, "Ks"), _dev(sigma, torch.float32, sshape, "sigma"),
            _dev(seeds, torch.uint64, (R,), "seeds"), int(step0),
            _dev(theta, torch.float32, None, "theta"),
            _dev(phase, torch.uint32, (R, n), "phase", True), ctypes.byref(ro),
            _stream(stream)), (cfg, ro)


def oim_run(h, n, theta, K, Ks, sigma, seeds, *, q, dt, readout_every=0, flags=0, step0=0,
            phase=None, trace=None, best_h=None, best_step=None, best_colour=None,
            stream=None):
    """Run len(K) Euler-Maruyama steps on theta[R][n] (FP32, radians, in place).
    With `phase` (uint32 [R][n] phase words) the run starts from and updates
    the exact device state."""
    args, keep = _run_args(h, n, theta, K, Ks, sigma, seeds, q, dt, readout_every, flags, step0,
                           phase, trace, best_h, best_step, best_colour, stream)
    check(lib().oim_run(*args))


def oim_run_noalloc(h, n, theta, K, Ks, sigma, seeds, *, q, dt, readout_every=0, flags=0,
                    step0=0, phase=None, trace=None, best_h=None, best_step=None,
                    best_colour=None, stream=None):
    """oim_run without any device allocation (workspace from the library's
    fixed per-device array; see oim_noalloc_scratch_bytes)."""
    args, keep = _run_args(h, n, theta, K, Ks, sigma, seeds, q, dt, readout_every, flags, step0,
                           phase, trace, best_h, best_step, best_colour, stream)
    check(lib().oim_run_noalloc(*args))


def oim_noalloc_scratch_bytes() -> int:
    return int(lib().oim_noalloc_scratch_bytes())


def oim_autotune(h, n, theta, K, Ks, sigma, seeds, *, q, dt, trial_steps, stream=None) -> dict:
    """Time every launch variant of the LDS-resident loop on trial_steps steps
    (theta[R][n] is read, not modified) and keep the fastest for this problem
    and SHIL order; returns the report as a dict."""
    if theta.dim() != 2 or theta.shape[1] != n:
        raise ValueError("theta must be [R][n]")
    R = int(theta.shape[0])
    steps = int(K.shape[0])
    cfg = RunCfg(int(q), R, steps, float(dt), 0, 0)
    rep = _lib.TuneReport()
    check(lib().oim_autotune(h, ctypes.byref(cfg), _dev(K, torch.float32, (steps,), "K"),
                             _dev(Ks, torch.float32, (steps,), "Ks"),
                             _dev(sigma, torch.float32, (steps,), "sigma"),
                             _dev(seeds, torch.uint64, (R,), "seeds"),
                             _dev(theta, torch.float32, None, "theta"), int(trial_steps),
                             ctypes.byref(rep), _stream(stream)))
    k = rep.n_tried
    return {"block": rep.chosen_block, "slices_per_wave": rep.chosen_slices_per_wave,
            "rows_per_lane": rep.chosen_rows_per_lane, "ms": rep.chosen_ms,
            "tried": [(rep.block[i], rep.slices_per_wave[i], rep.rows_per_lane[i], rep.ms[i])
                      for i in range(k)]}


def oim_set_tuning(h, q, block, slices_per_wave, rows_per_lane=4) -> None:
    check(lib().oim_set_tuning(h, int(q), int(block), int(slices_per_wave),
                               int(rows_per_lane)))


def _adj_cfg(q, R, steps, dt, checkpoint_every):
    return AdjointCfg(int(q), int(R), int(steps), float(dt), int(checkpoint_every), 0)


def oim_adjoint_checkpoint_words(h, *, q, R, steps, dt, checkpoint_every) -> int:
    cfg = _adj_cfg(q, R, steps, dt, checkpoint_every)
    w = ctypes.c_int64(0)
    check(lib().oim_adjoint_checkpoint_words(h, ctypes.byref(cfg), ctypes.byref(w)))
    return int(w.value)


def oim_adjoint_forward(h, n, theta0, K, Ks, sigma, seeds, ckpt, *, q, dt, checkpoint_every,
                        step0=0, theta_T=None, loss=None, stream=None):
    """Forward pass of the schedule adjoint from theta0[R][n]: checkpoints
    into ckpt (uint32 [words]), optional final phases and per-(replica,
    instance) relaxed cut (FP64 [R * I])."""
    if theta0.dim() != 2 or theta0.shape[1] != n:
        raise ValueError("theta0 must be [R][n]")
    R, steps = int(theta0.shape[0]), int(K.shape[0])
    cfg = _adj_cfg(q, R, steps, dt, checkpoint_every)
    RI = R * int(oim_problem_info_get(h)["n_instances"])
    check(lib().oim_adjoint_forward(h, ctypes.byref(cfg), _dev(K, torch.float32, (steps,), "K"),
                                    _dev(Ks, torch.float32, (steps,), "Ks"),
                                    _dev(sigma, torch.float32, (steps,), "sigma"),
                                    _dev(seeds, torch.uint64, (R,), "seeds"), int(step0),
                                    _dev(theta0, torch.float32, None, "theta0"),
                                    _dev(ckpt, torch.uint32, None, "ckpt", steps == 0),
                                    _dev(theta_T, torch.float32, (R, n), "theta_T", True),
                                    _dev(loss, torch.float64, (RI,), "loss", True),
                                    _stream(stream)))


def oim_adjoint_backward(h, R, K, Ks, sigma, seeds, ckpt, gK, gKs, gsigma, *, q, dt,
                         checkpoint_every, step0=0, stream=None):
    """Backward pass: dL/dK, dL/dKs, dL/dsigma (FP64 [steps]) from the checkpoints."""
    steps = int(K.shape[0])
    cfg = _adj_cfg(q, R, steps, dt, checkpoint_every)
    check(lib().oim_adjoint_backward(h, ctypes.byref(cfg), _dev(K, torch.float32, (steps,), "K"),
                                     _dev(Ks, torch.float32, (steps,), "Ks"),
                                     _dev(sigma, torch.float32, (steps,), "sigma"),
                                     _dev(seeds, torch.uint64, (R,), "seeds"), int(step0),
                                     _dev(ckpt, torch.uint32, None, "ckpt", steps == 0),
                                     _dev(gK, torch.float64, (steps,), "gK"),
                                     _dev(gKs, torch.float64, (steps,), "gKs"),
                                     _dev(gsigma, torch.float64, (steps,), "gsigma"),
                                     _stream(stream)))


def oim_phase_from_theta(theta, phase=None, stream=None):
    """Phase words rint(frac(theta / 2pi) 2^32) of every element of theta."""
    if phase is None:
        phase = torch.empty(theta.shape, dtype=torch.uint32, device=theta.device)
    check(lib().oim_phase_from_theta(int(theta.numel()),
                                     _dev(theta, torch.float32, None, "theta"),
                                     _dev(phase, torch.uint32, tuple(theta.shape), "phase"),
                                     _stream(stream)))
    return phase


def oim_theta_from_phase(phase, theta=None, stream=None):
    """FP32 radians in [0, 2pi) of every phase word."""
    if theta is None:
        theta = torch.empty(phase.shape, dtype=torch.float32, device=phase.device)
    check(lib().oim_theta_from_phase(int(phase.numel()),
                                     _dev(phase, torch.uint32, None, "phase"),
                                     _dev(theta, torch.float32, tuple(phase.shape), "theta"),
                                     _stream(stream)))
    return theta


def oim_round(q, theta, colour=None, stream=None):
    """Nearest stable phase index of every element of theta (int8, -1 if invalid)."""
    if colour is None:
        colour = torch.empty(theta.shape, dtype=torch.int8, device=theta.device)
    check(lib().oim_round(int(q), int(theta.numel()), _dev(theta, torch.float32, None, "theta"),
                          _dev(colour, torch.int8, tuple(theta.shape), "colour"), _stream(stream)))
    return colour


def oim_cut(h, colour, exact=True, stream=None):
    """Cut value per replica for colours [R][n]: int64 if exact else float64."""
    R = int(colour.shape[0])
    out = torch.empty(R, dtype=torch.int64 if exact else torch.float64, device=colour.device)
    check(lib().oim_cut(h, R, _dev(colour, torch.int8, None, "colour"),
                        _dev(out, torch.int64, None, "cut") if exact else None,
                        None if exact else _dev(out, torch.float64, None, "cut"), _stream(stream)))
    return out


def oim_conflicts(h, colour, stream=None):
    R = int(colour.shape[0])
    out = torch.empty(R, dtype=torch.int64, device=colour.device)
    check(lib().oim_conflicts(h, R, _dev(colour, torch.int8, None, "colour"),
                              _dev(out, torch.int64, None, "conflicts"), _stream(stream)))
    return out


def oim_energy(h, q, theta=None, colour=None, stream=None):
    """(H_model at colour or None, H_eq6 at theta or None), FP64 per replica."""
    ref = theta if theta is not None else colour
    R = int(ref.shape[0])
    hm = torch.empty(R, dtype=torch.float64, device=ref.device) if colour is not None else None
    h6 = torch.empty(R, dtype=torch.float64, device=ref.device) if theta is not None else None
    check(lib().oim_energy(h, int(q), R, _dev(theta, torch.float32, None, "theta", True),
                           _dev(colour, torch.int8, None, "colour", True),
                           _dev(hm, torch.float64, None, "h_model", True),
                           _dev(h6, torch.float64, None, "h_eq6", True), _stream(stream)))
    return hm, h6


class Problem:
    """Owning wrapper of an oim_problem handle."""

    def __init__(self, handle, n):
        self.handle = handle
        self.n = int(n)
        self.info = oim_problem_info_get(handle)

    @classmethod
    def from_csr(cls, n, row_ptr, col_idx, J):
        return cls(oim_problem_from_csr(n, row_ptr, col_idx, J), n)

    @classmethod
    def from_csr_blocks(cls, n, row_ptr, col_idx, J, inst_off):
        return cls(oim_problem_from_csr_blocks(n, row_ptr, col_idx, J, inst_off), n)

    @classmethod
    def from_dense(cls, J):
        return cls(oim_problem_from_dense(J), np.asarray(J).shape[0])

    def close(self):
        if self.handle:
            oim_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def run(problem: Problem, theta, K, Ks, sigma, seeds, *, q, dt, readout_every=0, flags=0,
        step0=0, want_best=False, phase=None, stream=None):
    """oim_run on a Problem; returns the readout tensors when readout_every > 0."""
    R, n = theta.shape
    steps = int(K.shape[-1])
    out = {}
    if readout_every > 0:
        dev = theta.device
        RI = R * int(problem.info["n_instances"])
        out["trace"] = torch.empty((n_readouts(steps, readout_every), RI), dtype=torch.float64,
                                   device=dev)
        out["best_h"] = torch.empty(RI, dtype=torch.float64, device=dev)
        out["best_step"] = torch.empty(RI, dtype=torch.int32, device=dev)
        if want_best:
            out["best_colour"] = torch.empty((R, n), dtype=torch.int8, device=dev)
    oim_run(problem.handle, problem.n, theta, K, Ks, sigma, seeds, q=q, dt=dt,
            readout_every=readout_every, flags=flags, step0=step0, phase=phase, stream=stream,
            **out)
    return out


def two_pi() -> float:
    return 2.0 * math.pi
