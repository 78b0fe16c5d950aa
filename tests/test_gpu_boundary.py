"""Boundary behaviour through the C ABI on the GPU: every invalid run
configuration is rejected before any device work (theta untouched), handles
are dead after destroy, non-finite input phases are defined, and the
stepwise loop's calls are asynchronous and reuse their captured graph."""
import ctypes

import numpy as np
import pytest

import synth
from _util import DT, ramp_schedule, wrapdiff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oim():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_22631_amd as m
    m.lib()
    return m


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_invalid_run_configs_leave_theta_untouched(oim):
    from paper_2505_22631_amd import _lib
    g = synth.erdos_renyi(200, 0.05, seed=1)
    steps, R, n = 20, 3, g.n
    th0 = synth.theta0(R, n, seed=2)
    K = _t(synth.const(0.5, steps))
    sd = _t(synth.seeds(R))
    L = oim.lib()
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, -g.w) as prob, \
            oim.Problem.from_dense(synth.sk_dense(64, seed=1)) as dprob:
        cases = [
            (prob, dict(q=1), _lib.OIM_E_ARG),
            (prob, dict(q=17), _lib.OIM_E_ARG),
            (prob, dict(R=0), _lib.OIM_E_ARG),
            (prob, dict(steps=-1), _lib.OIM_E_ARG),
            (prob, dict(dt=0.0), _lib.OIM_E_ARG),
            (prob, dict(dt=-0.01), _lib.OIM_E_ARG),
            (prob, dict(dt=float("nan")), _lib.OIM_E_ARG),
            (prob, dict(dt=float("inf")), _lib.OIM_E_ARG),
            (prob, dict(readout_every=-1), _lib.OIM_E_ARG),
            (prob, dict(flags=oim.OIM_LOOP_PERSISTENT | oim.OIM_LOOP_STEPWISE), _lib.OIM_E_ARG),
            (prob, dict(flags=0x30), _lib.OIM_E_ARG),
            (prob, dict(flags=0x1000), _lib.OIM_E_ARG),
            (prob, dict(flags=oim.OIM_PREC_BF16X3), _lib.OIM_E_UNSUPPORTED),
            (dprob, dict(flags=oim.OIM_LOOP_PERSISTENT), _lib.OIM_E_UNSUPPORTED),
        ]
        for pr, over, code in cases:
            nn = pr.n
            th = _t(synth.theta0(R, nn, seed=2))
            before = th.cpu().numpy().copy()
            c = dict(q=2, R=R, steps=steps, dt=DT, readout_every=0, flags=0)
            c.update(over)
            cfg = _lib.RunCfg(c["q"], c["R"], c["steps"], c["dt"], c["readout_every"], c["flags"])
            ro = _lib.Readout(None, None, None, None)
            p = lambda x: ctypes.c_void_p(x.data_ptr())
            st = L.oim_run(pr.handle, ctypes.byref(cfg), p(K), p(K), p(K), p(sd), 0, p(th), None,
                           ctypes.byref(ro), None)
            assert st == code, (over, st, L.oim_last_error())
            assert L.oim_last_error()
            np.testing.assert_array_equal(th.cpu().numpy(), before)
        # readout buffers without a readout period, and a step index past 2^32
        cfg = _lib.RunCfg(2, R, steps, DT, 0, 0)
        tr = _t(np.zeros((4, R)))
        ro = _lib.Readout(ctypes.c_void_p(tr.data_ptr()), None, None, None)
        th = _t(th0)
        p = lambda x: ctypes.c_void_p(x.data_ptr())
        assert L.oim_run(prob.handle, ctypes.byref(cfg), p(K), p(K), p(K), p(sd), 0, p(th), None,
                         ctypes.byref(ro), None) == _lib.OIM_E_ARG
        assert L.oim_run(prob.handle, ctypes.byref(cfg), p(K), p(K), p(K), p(sd), 2**32 - 5, p(th),
                         None, None, None) == _lib.OIM_E_ARG
        assert L.oim_run(prob.handle, ctypes.byref(cfg), None, p(K), p(K), p(sd), 0, p(th),
                         None, None, None) == _lib.OIM_E_ARG
        np.testing.assert_array_equal(th.cpu().numpy(), th0)


def test_handle_dead_after_destroy(oim):
    from paper_2505_22631_amd import _lib
    g = synth.erdos_renyi(50, 0.1, seed=1)
    prob = oim.Problem.from_csr(g.n, g.row_ptr, g.col, -g.w)
    h = prob.handle
    info = _lib.ProblemInfo()
    L = oim.lib()
    assert L.oim_problem_info_get(h, ctypes.byref(info)) == 0
    prob.close()
    assert L.oim_problem_info_get(h, ctypes.byref(info)) == _lib.OIM_E_STATE
    col = _t(np.zeros((1, g.n), np.int8))
    out = _t(np.zeros(1, np.int64))
    assert L.oim_cut(h, 1, ctypes.c_void_p(col.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                     None, None) == _lib.OIM_E_STATE
    L.oim_problem_destroy(h)  # a second destroy is a no-op
    # a new problem gets a new handle, and the old one stays dead
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, -g.w) as p2:
        assert p2.handle.value != h.value
        assert L.oim_problem_info_get(h, ctypes.byref(info)) == _lib.OIM_E_STATE


@pytest.mark.parametrize("loop", [0, 2])
def test_nonfinite_input_phases_are_zero(oim, loop):
    g = synth.erdos_renyi(300, 0.05, seed=3)
    R, steps = 2, 30
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, -g.w) as prob:
        K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], 2, 300, steps)
        th = synth.theta0(R, g.n, seed=4)
        bad = th.copy()
        bad[0, [0, 7, 299]] = [np.nan, np.inf, -np.inf]
        bad[1, 5] = np.nan
        ref = th.copy()
        ref[0, [0, 7, 299]] = 0.0
        ref[1, 5] = 0.0
        outs = []
        for x in (bad, ref):
            d = _t(x)
            oim.run(prob, d, _t(K), _t(Ks), _t(sg), _t(synth.seeds(R)), q=2, dt=DT, flags=loop)
            outs.append(d.cpu().numpy())
        np.testing.assert_array_equal(outs[0], outs[1])
        assert np.all(np.isfinite(outs[0]))
    w = oim.oim_phase_from_theta(_t(np.array([np.nan, np.inf, -np.inf, 1.0], np.float32)))
    assert w.cpu().numpy()[:3].tolist() == [0, 0, 0]


def test_stepwise_calls_are_asynchronous_and_reuse_the_graph(oim, orc):
    import time
    import torch
    g = synth.torus(60, 70, seed=5, signed=True)
    R, steps, q = 64, 300, 2
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, -g.w) as prob:
        K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], q, 3000, steps)
        dK, dKs, dsg = _t(K), _t(Ks), _t(sg)
        thA, thB = synth.theta0(R, g.n, seed=6), synth.theta0(R, g.n, seed=7)
        sdA, sdB = _t(synth.seeds(R, 0)), _t(synth.seeds(R, 500))
        F = oim.OIM_LOOP_STEPWISE
        # reference: one call at a time, synchronised
        refs = []
        for th, sd in ((thA, sdA), (thB, sdB)):
            d = _t(th)
            oim.run(prob, d, dK, dKs, dsg, sd, q=q, dt=DT, flags=F, readout_every=50)
            torch.cuda.synchronize()
            refs.append(d.cpu().numpy())
        # two calls back to back with no synchronisation in between, into
        # different buffers and with different seeds, on the cached graph
        a, b = _t(thA), _t(thB)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outA = oim.run(prob, a, dK, dKs, dsg, sdA, q=q, dt=DT, flags=F, readout_every=50)
        outB = oim.run(prob, b, dK, dKs, dsg, sdB, q=q, dt=DT, flags=F, readout_every=50)
        t_enqueue = time.perf_counter() - t0
        torch.cuda.synchronize()
        t_total = time.perf_counter() - t0
        print(f"two stepwise calls: enqueue {t_enqueue * 1e3:.2f} ms, complete {t_total * 1e3:.2f} ms",
              flush=True)
        np.testing.assert_array_equal(a.cpu().numpy(), refs[0])
        np.testing.assert_array_equal(b.cpu().numpy(), refs[1])
        assert t_enqueue < t_total
        # and both agree with the oracle on a sampled replica
        want = orc.run_csr(g.row_ptr, g.col, -g.w, thB[:1], q=q, dt=DT, K=K, Ks=Ks, sigma=sg,
                           seeds=synth.seeds(1, 500))
        assert wrapdiff(refs[1][:1], want).max() < 1e-5
        assert outA["best_h"].shape == (R,) and outB["trace"].shape == (6, R)
