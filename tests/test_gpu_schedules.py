"""GPU tests of per-replica annealing schedules (one K, Ks, sigma row per
replica in one launch) on every loop form, against the FP64 oracle and
against single-replica runs."""
import numpy as np
import pytest

import synth
from _util import DT, wrapdiff

pytestmark = pytest.mark.gpu
TOL_RAD = 1e-5


@pytest.fixture(scope="module")
def oim():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_22631_amd as m
    m.lib()
    return m


def _grid(R, steps, rowsum, q):
    """A K_max x Ks_max grid of linear ramps, one per replica, constant noise
    varying with the replica too."""
    kmax = 0.5 / (DT * rowsum)
    ksmax = 0.5 / (DT * q)
    K = np.stack([synth.ramp(0.0, kmax * (0.5 + r % 3), steps) for r in range(R)])
    Ks = np.stack([synth.ramp(0.0, ksmax * (0.25 + 0.5 * (r // 3)), steps) for r in range(R)])
    sg = np.stack([synth.const(0.05 + 0.05 * (r % 2), steps) for r in range(R)])
    return K.astype(np.float32), Ks.astype(np.float32), sg.astype(np.float32)


def _gpu(oim, prob, th0, K, Ks, sg, sd, q, flags=0, readout_every=0):
    import torch
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    th = t(th0)
    out = oim.run(prob, th, t(K), t(Ks), t(sg), t(np.asarray(sd, np.uint64)), q=q, dt=DT,
                  flags=flags, readout_every=readout_every)
    torch.cuda.synchronize()
    return th.cpu().numpy(), {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("loop", ["persistent", "stepwise"])
def test_per_replica_schedules_match_oracle(oim, orc, loop):
    g = synth.erdos_renyi(300, 0.05, seed=3, signed=True)
    J = (-g.w).astype(np.float32)
    R, steps, q = 6, 100, 2
    K, Ks, sg = _grid(R, steps, synth.gershgorin(g), q)
    th0 = synth.theta0(R, g.n, seed=4)
    sd = synth.seeds(R, 9)
    flags = oim.OIM_LOOP_PERSISTENT if loop == "persistent" else oim.OIM_LOOP_STEPWISE
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, J) as prob:
        got, _ = _gpu(oim, prob, th0, K, Ks, sg, sd, q, flags=flags)
    want = orc.run_csr(g.row_ptr, g.col, J, th0, q=q, dt=DT, K=K, Ks=Ks, sigma=sg, seeds=sd)
    err = wrapdiff(got, want).max()
    print(f"{loop}: per-replica schedules, max |dtheta| = {err:.3e} rad", flush=True)
    assert err < TOL_RAD


def test_per_replica_equals_single_replica_runs(oim):
    # each replica of the per-replica launch is bit-identical to a run of that
    # replica alone with its schedule shared
    gs = [synth.planted_colouring(nv, 4.6, 3, seed=nv)[0] for nv in (120, 75)]
    big, off = synth.block_diagonal(gs)
    J = -np.ones(big.nnz, np.float32)
    R, steps, q = 4, 150, 3
    K, Ks, sg = _grid(R, steps, synth.gershgorin(big), q)
    th0 = synth.theta0(R, big.n, seed=2)
    sd = synth.seeds(R, 5)
    with oim.Problem.from_csr_blocks(big.n, big.row_ptr, big.col, J, off) as prob:
        got, ro = _gpu(oim, prob, th0, K, Ks, sg, sd, q, readout_every=50)
        for r in range(R):
            one, ro1 = _gpu(oim, prob, th0[r:r + 1], K[r], Ks[r], sg[r], sd[r:r + 1], q,
                            readout_every=50)
            np.testing.assert_array_equal(got[r:r + 1], one)
            np.testing.assert_array_equal(ro["trace"][:, r * 2:(r + 1) * 2], ro1["trace"])


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_per_replica_schedules_dense(oim, orc, prec):
    n, R, steps, q = 160, 4, 60, 2
    Jd = synth.sk_dense(n, seed=8)
    flags = oim.OIM_PREC_BF16X3 if prec == "bf16x3" else oim.OIM_PREC_FP32
    with oim.Problem.from_dense(Jd) as prob:
        K, Ks, sg = _grid(R, steps, prob.info["max_abs_row_sum"], q)
        th0 = synth.theta0(R, n, seed=3)
        sd = synth.seeds(R, 2)
        got, _ = _gpu(oim, prob, th0, K, Ks, sg, sd, q, flags=flags)
    # each path against the oracle in its own precision: the BF16x3 split
    # products, or the FP64 all-pairs loop for the FP32 products
    want = orc.run_dense(Jd.astype(np.float64), th0, q=q, dt=DT, K=K, Ks=Ks, sigma=sg, seeds=sd,
                         precision="bf16x3" if prec == "bf16x3" else "fp64")
    err = wrapdiff(got, want).max()
    print(f"dense {prec} per-replica schedules: max |dtheta| = {err:.3e} rad", flush=True)
    assert err < 1e-5
