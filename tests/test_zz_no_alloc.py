"""The allocation-free run entry point (oim_run_noalloc) against oim_run,
through the C ABI: bit-identical phases and readouts on the stepwise and dense
loops (the ones with a workspace) and on the LDS-resident loop, on two calls
in a row, the second with a smaller input, plus the size limit."""
import numpy as np
import pytest

import synth
from _util import DT

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


def _both(oim, prob, n, R, steps, q, flags, M, seed):
    """The same run through oim_run and oim_run_noalloc; returns both
    (theta, trace, best_h, best_step, best_colour)."""
    import torch
    K = synth.ramp(0.0, 2.0, steps)
    Ks = synth.ramp(0.0, 3.0, steps)
    sg = synth.const(0.2, steps)
    th0 = synth.theta0(R, n, seed=seed)
    sd = synth.seeds(R, seed)
    outs = []
    for fn in (oim.oim_run, oim.oim_run_noalloc):
        th = _t(th0)
        ro = {}
        if M > 0:
            nr = oim.n_readouts(steps, M)
            ro = dict(trace=torch.full((nr, R), np.nan, dtype=torch.float64, device="cuda"),
                      best_h=torch.zeros(R, dtype=torch.float64, device="cuda"),
                      best_step=torch.zeros(R, dtype=torch.int32, device="cuda"),
                      best_colour=torch.zeros((R, n), dtype=torch.int8, device="cuda"))
        print(f"  {fn.__name__}: n={n} R={R} steps={steps} q={q} flags={flags:#x} M={M}",
              flush=True)
        fn(prob.handle, n, th, _t(K), _t(Ks), _t(sg), _t(sd), q=q, dt=DT, readout_every=M,
           flags=flags, step0=5, **ro)
        torch.cuda.synchronize()
        outs.append((th.cpu().numpy(),) + tuple(v.cpu().numpy() for v in ro.values()))
    return outs


def _same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_stepwise_two_calls_second_smaller(oim):
    g = synth.torus(20, 30, seed=1, signed=True)
    J = (-g.w).astype(np.float32)
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, J) as prob:
        a, b = _both(oim, prob, g.n, 96, 130, 2, oim.OIM_LOOP_STEPWISE, 50, 1)
        _same(a, b)
        a, b = _both(oim, prob, g.n, 7, 61, 2, oim.OIM_LOOP_STEPWISE, 20, 2)
        _same(a, b)


def test_dense_two_calls_second_smaller(oim):
    n = 200
    J = synth.sk_dense(n, seed=3)
    with oim.Problem.from_dense(J) as prob:
        for prec in (oim.OIM_PREC_BF16X3, oim.OIM_PREC_FP32):
            a, b = _both(oim, prob, n, 70, 40, 2, prec, 10, 3)
            _same(a, b)
            a, b = _both(oim, prob, n, 5, 23, 3, prec, 7, 4)
            _same(a, b)


def test_lds_resident_loop_needs_no_workspace(oim):
    g = synth.erdos_renyi(300, 0.05, seed=2)
    J = (-g.w).astype(np.float32)
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, J) as prob:
        a, b = _both(oim, prob, g.n, 16, 90, 2, oim.OIM_LOOP_PERSISTENT, 30, 5)
        _same(a, b)
        a, b = _both(oim, prob, g.n, 3, 41, 2, oim.OIM_LOOP_PERSISTENT, 0, 6)
        _same(a, b)


def test_workspace_beyond_the_array_is_rejected(oim):
    import torch
    limit = oim.oim_noalloc_scratch_bytes()
    assert limit == 64 << 20
    g = synth.torus(100, 100, seed=1, signed=True)
    R = 1024  # 8 bytes x 10000 x 1024 > 64 MiB
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, (-g.w).astype(np.float32)) as prob:
        th = _t(synth.theta0(R, g.n, seed=1))
        before = th.clone()
        z = _t(np.zeros(4, np.float32))
        with pytest.raises(oim.OimError, match="workspace"):
            oim.oim_run_noalloc(prob.handle, g.n, th, z, z, z, _t(synth.seeds(R, 0)), q=2, dt=DT,
                                flags=oim.OIM_LOOP_STEPWISE)
        torch.cuda.synchronize()
        assert torch.equal(th, before)
