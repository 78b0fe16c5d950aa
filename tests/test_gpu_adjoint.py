"""GPU parity of the schedule adjoint (forward with checkpoints, backward with
recomputation) against the FP64 oracle's adjoint, through the C ABI."""
import numpy as np
import pytest

import synth
from _util import DT, c5_batch, wrapdiff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def oim():
    import paper_2505_22631_amd as m
    m.lib()
    return m


def _t(x, dtype=None):
    import torch
    a = np.ascontiguousarray(x if dtype is None else np.asarray(x, dtype))
    return torch.from_numpy(a).cuda()


def _gpu_adjoint(oim, prob, th0, K, Ks, sg, sd, q, C, step0=0):
    """(loss per replica-instance, theta_T, gK, gKs, gS) from the GPU."""
    import torch
    R, n = th0.shape
    steps = len(K)
    dK, dKs, dS = _t(K, np.float32), _t(Ks, np.float32), _t(sg, np.float32)
    dsd = _t(sd, np.uint64)
    words = oim.oim_adjoint_checkpoint_words(prob.handle, q=q, R=R, steps=steps, dt=DT,
                                             checkpoint_every=C)
    ckpt = torch.zeros(max(words, 1), dtype=torch.uint32, device="cuda")
    thT = torch.empty((R, n), dtype=torch.float32, device="cuda")
    RI = R * prob.info["n_instances"]
    loss = torch.empty(RI, dtype=torch.float64, device="cuda")
    oim.oim_adjoint_forward(prob.handle, n, _t(th0, np.float32), dK, dKs, dS, dsd, ckpt, q=q,
                            dt=DT, checkpoint_every=C, step0=step0, theta_T=thT, loss=loss)
    g = [torch.full((steps,), np.nan, dtype=torch.float64, device="cuda") for _ in range(3)]
    oim.oim_adjoint_backward(prob.handle, R, dK, dKs, dS, dsd, ckpt, *g, q=q, dt=DT,
                             checkpoint_every=C, step0=step0)
    torch.cuda.synchronize()
    return (loss.cpu().numpy(), thT.cpu().numpy(), *(x.cpu().numpy() for x in g))


def _close_vec(got, ref, rel):
    """Entry-wise agreement scaled by the vector's magnitude."""
    scale = float(np.max(np.abs(ref)))
    err = float(np.max(np.abs(got - ref)))
    return err <= rel * scale, err / max(scale, 1e-300)


def _schedules(steps):
    K = synth.ramp(0.2, 1.5, steps).astype(np.float32)
    Ks = synth.ramp(0.0, 2.0, steps).astype(np.float32)
    sg = synth.const(0.15, steps).astype(np.float32)
    return K, Ks, sg


def test_adjoint_single_graph_matches_oracle(oim, orc, dev):
    g = synth.random_small(40, 0.2, seed=12, weights="pm1")
    J = -g.w
    steps, R, C, step0 = 60, 3, 16, 7
    K, Ks, sg = _schedules(steps)
    th0 = synth.theta0(R, g.n, seed=3)
    sd = synth.seeds(R, 11)
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, J.astype(np.float32)) as prob:
        loss, thT, gK, gKs, gS = _gpu_adjoint(oim, prob, th0, K, Ks, sg, sd, 2, C, step0)
    Jd = J.astype(np.float64)
    L, oK, oKs, oS = orc.adjoint_csr(g.row_ptr, g.col, Jd, th0.astype(np.float64), q=2, dt=DT,
                                     K=K, Ks=Ks, sigma=sg, seeds=sd, step0=step0)
    th_ref = orc.run_csr(g.row_ptr, g.col, Jd, th0, q=2, dt=DT, K=K, Ks=Ks, sigma=sg, seeds=sd,
                         step0=step0)
    assert np.max(wrapdiff(thT, th_ref)) < 1e-5
    assert loss.sum() == pytest.approx(L, rel=1e-5)
    for got, ref, name in ((gK, oK, "K"), (gKs, oKs, "Ks"), (gS, oS, "sigma")):
        ok, rel = _close_vec(got, ref, 1e-4)
        print(f"d/d{name}: max rel err {rel:.2e}")
        assert ok, (name, rel)


def test_adjoint_ragged_batch_q3_matches_oracle(oim, orc, dev):
    gs = [synth.planted_colouring(nv, 4.6, 3, seed=40 + nv)[0] for nv in (37, 100, 61)]
    big, off = synth.block_diagonal(gs)
    J = -big.w
    steps, R, C = 45, 2, 7  # segments of 7 with a ragged last one
    K, Ks, sg = _schedules(steps)
    th0 = synth.theta0(R, big.n, seed=8)
    sd = synth.seeds(R, 2)
    with oim.Problem.from_csr_blocks(big.n, big.row_ptr, big.col, J.astype(np.float32),
                                     off) as prob:
        loss, thT, gK, gKs, gS = _gpu_adjoint(oim, prob, th0, K, Ks, sg, sd, 3, C)
    Jd = J.astype(np.float64)
    L, oK, oKs, oS = orc.adjoint_csr(big.row_ptr, big.col, Jd, th0.astype(np.float64), q=3,
                                     dt=DT, K=K, Ks=Ks, sigma=sg, seeds=sd, inst_off=off)
    th_ref = orc.run_csr_blocks(big.row_ptr, big.col, Jd, off, th0, q=3, dt=DT, K=K, Ks=Ks,
                                sigma=sg, seeds=sd)
    assert np.max(wrapdiff(thT, th_ref)) < 1e-5
    assert loss.sum() == pytest.approx(L, rel=1e-5)
    # per (replica, instance) losses: entry r * I + b
    for r in range(R):
        for b in range(3):
            sl = slice(off[b], off[b + 1])
            ref = orc.relaxed_cut(gs[b].row_ptr, gs[b].col, -gs[b].w, th_ref[r:r + 1, sl])
            assert loss[r * 3 + b] == pytest.approx(ref, rel=1e-5, abs=1e-6)
    for got, ref, name in ((gK, oK, "K"), (gKs, oKs, "Ks"), (gS, oS, "sigma")):
        ok, rel = _close_vec(got, ref, 1e-4)
        print(f"d/d{name}: max rel err {rel:.2e}")
        assert ok, (name, rel)


def test_adjoint_generic_q_matches_oracle(oim, orc, dev):
    g = synth.random_small(18, 0.35, seed=5, weights="int")
    J = -g.w
    steps, R, C = 30, 2, 9
    K, Ks, sg = _schedules(steps)
    th0 = synth.theta0(R, g.n, seed=6)
    sd = synth.seeds(R, 4)
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, J.astype(np.float32)) as prob:
        loss, thT, gK, gKs, gS = _gpu_adjoint(oim, prob, th0, K, Ks, sg, sd, 5, C)
    L, oK, oKs, oS = orc.adjoint_csr(g.row_ptr, g.col, J.astype(np.float64),
                                     th0.astype(np.float64), q=5, dt=DT, K=K, Ks=Ks, sigma=sg,
                                     seeds=sd)
    assert loss.sum() == pytest.approx(L, rel=1e-5)
    for got, ref, name in ((gK, oK, "K"), (gKs, oKs, "Ks"), (gS, oS, "sigma")):
        ok, rel = _close_vec(got, ref, 1e-4)
        assert ok, (name, rel)


def test_adjoint_checkpoint_interval_is_exact(oim, dev):
    # recomputation from checkpoints is exact: every interval gives the same bits
    g = synth.gnp_avg_degree(300, 8, seed=2)
    steps = 50
    K, Ks, sg = _schedules(steps)
    th0 = synth.theta0(2, g.n, seed=1)
    sd = synth.seeds(2, 0)
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, (-g.w).astype(np.float32)) as prob:
        ref = _gpu_adjoint(oim, prob, th0, K, Ks, sg, sd, 2, 1)
        for C in (7, 50, 64):
            out = _gpu_adjoint(oim, prob, th0, K, Ks, sg, sd, 2, C)
            for a, b in zip(out, ref):
                np.testing.assert_array_equal(a, b)


def test_adjoint_zero_steps_and_validation(oim, dev):
    import torch
    g = synth.cycle(8)
    th0 = synth.theta0(1, 8, seed=0)
    with oim.Problem.from_csr(8, g.row_ptr, g.col, (-g.w).astype(np.float32)) as prob:
        e = np.zeros(0, np.float32)
        loss, thT, gK, gKs, gS = _gpu_adjoint(oim, prob, th0, e, e, e, synth.seeds(1), 2, 4)
        assert gK.size == 0
        np.testing.assert_allclose(thT, th0, atol=1e-6)
        ref = 0.5 * np.sum(1.0 - np.cos(th0[0] - np.roll(th0[0], -1)))
        assert loss[0] == pytest.approx(ref, rel=1e-6)
        K = torch.ones(5, device="cuda")
        sd = torch.zeros(1, dtype=torch.uint64, device="cuda")
        ck = torch.zeros(64, dtype=torch.uint32, device="cuda")
        with pytest.raises(oim.OimError, match="checkpoint_every"):
            oim.oim_adjoint_forward(prob.handle, 8, _t(th0, np.float32), K, K, K, sd, ck, q=2,
                                    dt=DT, checkpoint_every=0)
    big = synth.gnp_avg_degree(4100, 3, seed=1)
    with oim.Problem.from_csr(big.n, big.row_ptr, big.col, (-big.w).astype(np.float32)) as prob:
        with pytest.raises(oim.OimError, match="4096"):
            oim.oim_adjoint_checkpoint_words(prob.handle, q=2, R=1, steps=5, dt=DT,
                                             checkpoint_every=2)
    dense = synth.sk_dense(16, seed=0)
    with oim.Problem.from_dense(dense) as prob:
        with pytest.raises(oim.OimError, match="sparse"):
            oim.oim_adjoint_checkpoint_words(prob.handle, q=2, R=1, steps=5, dt=DT,
                                             checkpoint_every=2)


def test_autograd_function_matches_kernels(oim, dev):
    import torch
    from paper_2505_22631_amd.autograd import relaxed_cut
    g = synth.random_small(30, 0.25, seed=3, weights="pm1")
    steps = 40
    K, Ks, sg = _schedules(steps)
    th0 = synth.theta0(2, g.n, seed=2)
    sd = synth.seeds(2, 9)
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, (-g.w).astype(np.float32)) as prob:
        ref = _gpu_adjoint(oim, prob, th0, K, Ks, sg, sd, 2, 8)
        tK = _t(K, np.float32).requires_grad_()
        tKs = _t(Ks, np.float32).requires_grad_()
        tS = _t(sg, np.float32).requires_grad_()
        L = relaxed_cut(prob, _t(th0, np.float32), tK, tKs, tS, _t(sd, np.uint64), q=2, dt=DT,
                        checkpoint_every=8)
        (2.0 * L).backward()
        torch.cuda.synchronize()
    assert float(L) == pytest.approx(float(ref[0].sum()), rel=1e-12)
    for t, r in ((tK, ref[2]), (tKs, ref[3]), (tS, ref[4])):
        np.testing.assert_allclose(t.grad.cpu().numpy(), (2.0 * r).astype(np.float32), rtol=1e-6)


def test_adjoint_gradient_against_gpu_finite_differences(oim, dev):
    # central differences (eps = 1e-3) of the GPU forward loss; coarse check
    # of the kernels' own consistency at the entries with the largest gradients
    import torch
    g = synth.gnp_avg_degree(200, 6, seed=9)
    steps = 40
    K, Ks, sg = _schedules(steps)
    th0 = synth.theta0(4, g.n, seed=4)
    sd = synth.seeds(4, 1)
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, (-g.w).astype(np.float32)) as prob:
        _, _, gK, gKs, gS = _gpu_adjoint(oim, prob, th0, K, Ks, sg, sd, 2, 10)

        def L(K_, Ks_, sg_):
            return float(_gpu_adjoint(oim, prob, th0, K_, Ks_, sg_, sd, 2, 64)[0].sum())

        eps = 1e-3
        for vec, grad in ((K, gK), (Ks, gKs), (sg, gS)):
            for s in np.argsort(-np.abs(grad))[:2]:
                up, dn = vec.astype(np.float64).copy(), vec.astype(np.float64).copy()
                up[s] += eps
                dn[s] -= eps
                a = [up if v is vec else v for v in (K, Ks, sg)]
                b = [dn if v is vec else v for v in (K, Ks, sg)]
                fd = (L(*a) - L(*b)) / (2 * eps)
                assert grad[s] == pytest.approx(fd, rel=0.05), (s, grad[s], fd)
    torch.cuda.synchronize()


def test_adjoint_full_batch_prefix_matches_oracle(oim, orc, dev):
    # the 128-graph batch of G(2000, 10/1999) in the benchmark's launch
    # configuration (one workgroup per graph, checkpoints every 64 steps),
    # on a 50-step prefix of its schedule that the oracle integrates in seconds
    big, off = c5_batch()
    steps_total, steps = 2000, 50
    kmax = 0.5 / (DT * synth.gershgorin(big))
    K = synth.ramp(0.0, kmax, steps_total)[:steps].astype(np.float32)
    Ks = synth.ramp(0.0, 0.5 / (DT * 2), steps_total)[:steps].astype(np.float32)
    sg = synth.const(0.1, steps).astype(np.float32)
    th0 = synth.theta0(1, big.n, seed=5)
    sd = synth.seeds(1, 0)
    J = -big.w
    with oim.Problem.from_csr_blocks(big.n, big.row_ptr, big.col, J.astype(np.float32),
                                     off) as prob:
        loss, thT, gK, gKs, gS = _gpu_adjoint(oim, prob, th0, K, Ks, sg, sd, 2, 64)
    L, oK, oKs, oS = orc.adjoint_csr(big.row_ptr, big.col, J.astype(np.float64),
                                     th0.astype(np.float64), q=2, dt=DT, K=K, Ks=Ks, sigma=sg,
                                     seeds=sd, inst_off=off)
    assert loss.sum() == pytest.approx(L, rel=1e-6)
    for got, ref, name in ((gK, oK, "K"), (gKs, oKs, "Ks"), (gS, oS, "sigma")):
        ok, rel = _close_vec(got, ref, 1e-4)
        print(f"full batch d/d{name}: max rel err {rel:.2e}")
        assert ok, (name, rel)


def test_adjoint_rows_from_global_memory_match_oracle(oim, orc, dev):
    # an instance whose rows do not fit in LDS next to the tables (about
    # 90 000 stored entries) is gathered from global memory instead
    g = synth.gnp_avg_degree(1500, 60.0, seed=6)
    J = -g.w
    steps, R, C = 25, 1, 10
    K, Ks, sg = _schedules(steps)
    K = (K / 20.0).astype(np.float32)  # keep dt * K * degree small
    th0 = synth.theta0(R, g.n, seed=2)
    sd = synth.seeds(R, 1)
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, J.astype(np.float32)) as prob:
        loss, thT, gK, gKs, gS = _gpu_adjoint(oim, prob, th0, K, Ks, sg, sd, 2, C)
    L, oK, oKs, oS = orc.adjoint_csr(g.row_ptr, g.col, J.astype(np.float64),
                                     th0.astype(np.float64), q=2, dt=DT, K=K, Ks=Ks, sigma=sg,
                                     seeds=sd)
    assert loss.sum() == pytest.approx(L, rel=1e-5)
    for got, ref, name in ((gK, oK, "K"), (gKs, oKs, "Ks"), (gS, oS, "sigma")):
        ok, rel = _close_vec(got, ref, 1e-4)
        print(f"global rows d/d{name}: max rel err {rel:.2e}")
        assert ok, (name, rel)


def test_adjoint_row_placements_give_identical_bits(oim, dev, monkeypatch):
    # a ragged unit-weight batch runs with the padded row image in LDS by
    # default; the CSR copy in LDS and the global CSR (forced through
    # OIM_ADJ_ROWS) must give the same loss, final phases and gradients bit
    # for bit: every placement sums each row in the same order
    graphs = [synth.gnp_avg_degree(n, 6.0, seed=40 + i) for i, n in enumerate([300, 517, 129])]
    big, off = synth.block_diagonal(graphs)
    steps, R, C = 40, 2, 16
    K, Ks, sg = _schedules(steps)
    th0 = synth.theta0(R, big.n, seed=9)
    sd = synth.seeds(R, 21)
    outs = {}
    with oim.Problem.from_csr_blocks(big.n, big.row_ptr, big.col, (-big.w).astype(np.float32),
                                     off) as prob:
        for mode in ("", "csr", "global"):
            if mode:
                monkeypatch.setenv("OIM_ADJ_ROWS", mode)
            else:
                monkeypatch.delenv("OIM_ADJ_ROWS", raising=False)
            outs[mode] = _gpu_adjoint(oim, prob, th0, K, Ks, sg, sd, 3, C)
    monkeypatch.delenv("OIM_ADJ_ROWS", raising=False)
    assert np.all(np.isfinite(outs[""][0]))
    for mode in ("csr", "global"):
        for a, b in zip(outs[""], outs[mode]):
            np.testing.assert_array_equal(a, b)
