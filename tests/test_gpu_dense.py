"""GPU parity of the dense (all-to-all) path: coupling as a BF16 three-term
split GEMM on the matrix cores, against the oracle's BF16x3 form of the same
coupling (split products in FP64, within the FP32 paths' 1e-5 rad after 100
steps), with the split's own distance from the FP64 all-pairs loop stated; and
the FP32 matrix-core path against the FP64 oracle directly."""
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


def _run(oim, prob, th0, K, Ks, sg, sd, q, step0=0, readout_every=0, want_best=False,
         flags=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(th0)).cuda()
    out = oim.run(prob, t, torch.from_numpy(K).cuda(), torch.from_numpy(Ks).cuda(),
                  torch.from_numpy(sg).cuda(),
                  torch.from_numpy(np.ascontiguousarray(sd, np.uint64)).cuda(), q=q, dt=DT,
                  readout_every=readout_every,
                  flags=oim.OIM_PREC_BF16X3 if flags is None else flags, step0=step0,
                  want_best=want_best)
    torch.cuda.synchronize()
    return t.cpu().numpy(), {k: v.cpu().numpy() for k, v in out.items()}


TOL_RAD = 1e-5


def _check_bf16x3(orc, got, J, th0, K, Ks, sg, sd, q, step0=0, label="", nthreads=0):
    """The GPU's BF16x3 phases against the oracle's BF16x3 form (the bar:
    1e-5 rad) and, for the record, both against the FP64 oracle: the GPU's
    distance from FP64 is the split's own error plus FP32 rounding."""
    Jd = J.astype(np.float64)
    kw = dict(q=q, dt=DT, K=K, Ks=Ks, sigma=sg, seeds=sd, step0=step0, nthreads=nthreads)
    want3 = orc.run_dense(Jd, th0, precision="bf16x3", **kw)
    want64 = orc.run_dense(Jd, th0, **kw)
    err = wrapdiff(got, want3).max()
    err64 = wrapdiff(got, want64).max()
    split64 = wrapdiff(want3, want64).max()
    print(f"dense BF16x3 {label}: max |dtheta| vs oracle BF16x3 = {err:.3e} rad; "
          f"vs FP64 = {err64:.3e} rad (the split alone: {split64:.3e})", flush=True)
    assert np.all(np.isfinite(got))
    assert err < TOL_RAD
    assert err64 <= split64 + TOL_RAD
    return err, err64


@pytest.mark.parametrize("n,R,q", [(200, 5, 2), (256, 64, 2), (130, 3, 3)])
def test_dense_parity_sk(oim, orc, n, R, q):
    J = synth.sk_dense(n, seed=3)
    with oim.Problem.from_dense(J) as prob:
        rowsum = prob.info["max_abs_row_sum"]
        K, Ks, sg = ramp_schedule(rowsum, q, 1000, 100)
        th0 = synth.theta0(R, n, seed=21)
        sd = synth.seeds(R, 7)
        got, _ = _run(oim, prob, th0, K, Ks, sg, sd, q, step0=50)
    _check_bf16x3(orc, got, J, th0, K, Ks, sg, sd, q, step0=50, label=f"n={n} R={R} q={q}")


def test_dense_matches_sparse_on_same_coupling(oim, orc):
    # the same J through the dense BF16x3 path and the FP32 sparse path
    g = synth.erdos_renyi(300, 0.1, seed=4)
    Jd = np.zeros((300, 300), np.float32)
    ei, ej, w = g.upper_edges()
    Jd[ei, ej] = -w
    Jd[ej, ei] = -w
    K, Ks, sg = ramp_schedule(synth.gershgorin(g), 2, 1000, 100)
    th0 = synth.theta0(4, 300, seed=5)
    sd = synth.seeds(4, 1)
    with oim.Problem.from_dense(Jd) as pd, oim.Problem.from_csr(300, g.row_ptr, g.col, -g.w) as ps:
        a, _ = _run(oim, pd, th0, K, Ks, sg, sd, 2)
        import torch
        t = torch.from_numpy(th0.copy()).cuda()
        oim.run(ps, t, torch.from_numpy(K).cuda(), torch.from_numpy(Ks).cuda(),
                torch.from_numpy(sg).cuda(), torch.from_numpy(sd).cuda(), q=2, dt=DT)
        b = t.cpu().numpy()
    # unit weights are exact in BF16, so the split only rounds sin/cos
    assert wrapdiff(a, b).max() < 1e-5


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_dense_in_run_readout(oim, orc, prec):
    n, R = 160, 4
    J = synth.sk_dense(n, seed=8)
    flags = oim.OIM_PREC_BF16X3 if prec == "bf16x3" else oim.OIM_PREC_FP32
    with oim.Problem.from_dense(J) as prob:
        K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], 2, 120)
        th0 = synth.theta0(R, n, seed=2)
        th, ro = _run(oim, prob, th0, K, Ks, sg, synth.seeds(R, 3), 2, readout_every=40,
                      want_best=True, flags=flags)
    rp, cl, Jv = orc.dense_to_csr(J)
    tr = ro["trace"]
    assert tr.shape == (3, R)
    np.testing.assert_array_equal(ro["best_h"], tr.min(axis=0))
    for r in range(R):
        # Eq. 1 at the best colours, in the oracle's fixed FP64 order: equal
        assert ro["best_h"][r] == orc.h_model_fixed(rp, cl, Jv, 2, ro["best_colour"][r])


def test_dense_rejects_unknown_precision(oim):
    import torch
    J = synth.sk_dense(64, seed=1)
    with oim.Problem.from_dense(J) as prob:
        t = torch.zeros((1, 64), device="cuda")
        z = torch.zeros(3, device="cuda")
        with pytest.raises(oim.OimError):
            oim.run(prob, t, z, z, z, torch.zeros(1, dtype=torch.uint64, device="cuda"), q=2,
                    dt=DT, flags=0x20)


@pytest.mark.parametrize("n,R,q", [(200, 5, 2), (130, 3, 3), (97, 2, 5)])
def test_dense_fp32_parity(oim, orc, n, R, q):
    # FP32 products on the matrix cores (OIM_PREC_FP32): the paper's precision,
    # within the sparse path's tolerance of the FP64 oracle after 100 steps,
    # and at least as close as the BF16x3 split on the same case
    J = synth.sk_dense(n, seed=3)
    with oim.Problem.from_dense(J) as prob:
        rowsum = prob.info["max_abs_row_sum"]
        K, Ks, sg = ramp_schedule(rowsum, q, 1000, 100)
        th0 = synth.theta0(R, n, seed=21)
        sd = synth.seeds(R, 7)
        got, _ = _run(oim, prob, th0, K, Ks, sg, sd, q, step0=50, flags=oim.OIM_PREC_FP32)
        got3, _ = _run(oim, prob, th0, K, Ks, sg, sd, q, step0=50)
    want = orc.run_dense(J.astype(np.float64), th0, q=q, dt=DT, K=K, Ks=Ks, sigma=sg, seeds=sd,
                         step0=50)
    err = wrapdiff(got, want).max()
    err3 = wrapdiff(got3, want).max()
    print(f"dense FP32 n={n} R={R} q={q}: max |dtheta| = {err:.3e} rad (BF16x3 {err3:.3e})",
          flush=True)
    assert np.all(np.isfinite(got))
    assert err < 1e-5
    assert err <= max(err3, 2e-6)


def test_dense_fp32_full_size_sampled_replica(oim, orc):
    # the n = 4096 SK coupling with 128 replicas on the FP32 path; the last
    # replica checked against the oracle over 5 steps, readout included
    n, R, steps = 4096, 128, 5
    J = synth.sk_dense(n, seed=3)
    with oim.Problem.from_dense(J) as prob:
        kmax = 32.0 * 0.5 / (DT * prob.info["max_abs_row_sum"])
        K = synth.ramp(0.0, kmax, 1000)[:steps].copy()
        Ks = synth.ramp(0.0, 0.03 * 0.5 / (DT * 2), 1000)[:steps].copy()
        sg = synth.const(0.1, steps)
        th0 = synth.theta0(R, n, seed=100)
        sd = synth.seeds(R, 0)
        got, ro = _run(oim, prob, th0, K, Ks, sg, sd, 2, readout_every=5,
                       flags=oim.OIM_PREC_FP32)
    pick = [R - 1]
    want = orc.run_dense(J.astype(np.float64), th0[pick], q=2, dt=DT, K=K, Ks=Ks, sigma=sg,
                         seeds=sd[pick])
    err = wrapdiff(got[pick], want).max()
    print(f"dense FP32 n=4096 R={R} replica {pick}: max |dtheta| = {err:.3e} rad", flush=True)
    assert np.all(np.isfinite(got)) and got.min() >= 0 and got.max() < 2 * np.pi
    assert err < 1e-5
    assert ro["trace"].shape == (1, R) and np.all(np.isfinite(ro["trace"]))


def test_dense_full_size_sampled_replicas(oim, orc):
    # the n = 4096, 512-replica SK workload in the benchmark's launch
    # configuration (32 x 8 workgroups); replicas are independent, so two of
    # them (first and last) are checked against the oracle over the first 100
    # steps of the benchmark's schedule, the others must stay finite and in
    # [0, 2pi)
    n, R, steps = 4096, 512, 100
    J = synth.sk_dense(n, seed=3)
    with oim.Problem.from_dense(J) as prob:
        kmax = 32.0 * 0.5 / (DT * prob.info["max_abs_row_sum"])
        K = synth.ramp(0.0, kmax, 1000)[:steps].copy()
        Ks = synth.ramp(0.0, 0.03 * 0.5 / (DT * 2), 1000)[:steps].copy()
        sg = synth.const(0.1, steps)
        th0 = synth.theta0(R, n, seed=100)
        sd = synth.seeds(R, 0)
        got, _ = _run(oim, prob, th0, K, Ks, sg, sd, 2)
    pick = [0, R - 1]
    assert np.all(np.isfinite(got)) and got.min() >= 0 and got.max() < 2 * np.pi
    _check_bf16x3(orc, got[pick], J, th0[pick], K, Ks, sg, sd[pick], 2,
                  label=f"n=4096 R=512 replicas {pick}, {steps} steps")


def test_dense_paper_scale_sampled_replica(oim, orc):
    # the paper's largest all-to-all size, n = 20000 (J is 1.6 GB in FP32;
    # 20000 is not a multiple of the 128-row tile, so the last row tile is
    # ragged), 64 replicas; the last replica is checked against the oracle
    # over 2 steps, the others must stay finite and in [0, 2pi)
    n, R, steps = 20000, 64, 2
    rng = np.random.default_rng(11)
    J = (rng.standard_normal((n, n), dtype=np.float32) / np.float32(np.sqrt(n)))
    J = np.triu(J, k=1)
    J += J.T
    with oim.Problem.from_dense(J) as prob:
        kmax = 32.0 * 0.5 / (DT * prob.info["max_abs_row_sum"])
        K = synth.ramp(0.0, kmax, 100)[50:50 + steps].copy()
        Ks = synth.const(0.5, steps)
        sg = synth.const(0.1, steps)
        th0 = synth.theta0(R, n, seed=101)
        sd = synth.seeds(R, 3)
        got, _ = _run(oim, prob, th0, K, Ks, sg, sd, 2, step0=7)
    pick = [R - 1]
    assert np.all(np.isfinite(got)) and got.min() >= 0 and got.max() < 2 * np.pi
    _check_bf16x3(orc, got[pick], J, th0[pick], K, Ks, sg, sd[pick], 2, step0=7,
                  label=f"n={n} R={R} replica {pick}, {steps} steps")
