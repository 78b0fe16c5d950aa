"""GPU readouts of real-weighted sums against the oracle's fixed FP64 order,
through the C ABI: cut values (Sec. II-C), Eq. 1 / Eq. 2 energies at
identical colours must be equal bit for bit -- standalone, in-run on the
LDS-resident, stepwise and dense loops, and per instance of a batch.  Eq. 6
at continuous phases depends on the FP64 cosine of each side's maths
library; it is checked against one rounding per term, and how many replicas
agree exactly is printed.  |GPU - correctly rounded sum| is reported."""
import math

import numpy as np
import pytest

import synth
from _util import DT, ramp_schedule

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oim():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_22631_amd as m
    m.lib()
    return m


def _t(x, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x if dtype is None else x.astype(dtype))).cuda()


def _words(theta):
    x = np.asarray(theta, np.float64) / (2 * np.pi)
    return (np.rint((x - np.floor(x)) * 2.0**32).astype(np.uint64) % (1 << 32)).astype(np.uint32)


def _colours_from_words(u, q):
    return (((q * u.astype(np.uint64) + (1 << 31)) >> 32) % q).astype(np.int8)


def _fsum_terms(g_rows, g_col, J, col, kind, q=2):
    i = g_rows
    j = g_col
    up = i < j
    i, j, Jv = i[up], j[up], np.asarray(J, np.float64)[up]
    if kind == "cut":
        t = np.where(col[i] != col[j], -Jv, 0.0)
    elif q == 2:
        t = np.where(col[i] == col[j], -Jv, Jv)
    else:
        t = np.where(col[i] == col[j], -Jv, 0.0)
    return math.fsum(t.tolist())


def _real_graph(n=3001, deg=9.0, seed=21):
    g = synth.gnp_avg_degree(n, deg, seed=seed, signed=True)
    rng = np.random.default_rng(seed)
    # real weights of both signs over a few orders of magnitude, symmetric
    ei, ej, _ = g.upper_edges()
    w = (rng.standard_normal(ei.size) * np.exp(rng.uniform(-6, 3, ei.size))).astype(np.float32)
    return synth.csr_from_edges(n, ei, ej, w)


def test_standalone_readouts_real_weights(oim, orc):
    g = _real_graph()
    J = (-g.w).astype(np.float32)
    R = 5
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, J) as prob:
        assert prob.info["integer_weights"] == 0
        th = synth.theta0(R, g.n, seed=3)
        dth = _t(th)
        for q in (2, 3):
            col = oim.oim_round(q, dth)
            hm, h6 = oim.oim_energy(prob.handle, q, dth, col)
            col, hm, h6 = col.cpu().numpy(), hm.cpu().numpy(), h6.cpu().numpy()
            same6 = 0
            for r in range(R):
                want = orc.h_model_fixed(g.row_ptr, g.col, J, q, col[r])
                assert hm[r] == want, (q, r, hm[r], want)
                w6 = orc.h_eq6_fixed(g.row_ptr, g.col, J, th[r].astype(np.float64))
                assert abs(h6[r] - w6) <= 2.0**-51 * np.abs(J).astype(np.float64).sum() / 2
                same6 += int(h6[r] == w6)
                fs = _fsum_terms(rows, g.col, J, col[r], "model", q)
                print(f"q={q} r={r}: Eq.{1 if q == 2 else 2} {hm[r]!r}, |GPU - fsum| = "
                      f"{abs(hm[r] - fs):.3e}", flush=True)
            print(f"q={q}: Eq. 6 equal bit for bit on {same6}/{R} replicas", flush=True)
        col = oim.oim_round(2, dth)
        cutf = oim.oim_cut(prob.handle, col, exact=False).cpu().numpy()
        col = col.cpu().numpy()
        for r in range(R):
            want = orc.cut_fixed(g.row_ptr, g.col, J, col[r])
            assert cutf[r] == want
            print(f"cut r={r}: {cutf[r]!r}, |GPU - fsum| = "
                  f"{abs(cutf[r] - _fsum_terms(rows, g.col, J, col[r], 'cut')):.3e}", flush=True)


@pytest.mark.parametrize("loop", ["persistent", "stepwise"])
def test_in_run_readout_real_weights_exact(oim, orc, loop):
    g = _real_graph(n=2100, deg=7.0, seed=5)
    J = (-g.w).astype(np.float32)
    R, q, steps, M = 3, 2, 230, 50
    flags = oim.OIM_LOOP_STEPWISE if loop == "stepwise" else oim.OIM_LOOP_PERSISTENT
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, J) as prob:
        K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], q, steps)
        th0 = synth.theta0(R, g.n, seed=6)
        ph = _t(_words(th0))
        dth = _t(th0)
        out = oim.run(prob, dth, _t(K), _t(Ks), _t(sg), _t(synth.seeds(R, 2)), q=q, dt=DT,
                      readout_every=M, flags=flags, want_best=True, phase=ph)
        ro = {k: v.cpu().numpy() for k, v in out.items()}
        w = ph.cpu().numpy()
    for r in range(R):
        bh = orc.h_model_fixed(g.row_ptr, g.col, J, q, ro["best_colour"][r])
        assert ro["best_h"][r] == bh
        last = orc.h_model_fixed(g.row_ptr, g.col, J, q, _colours_from_words(w[r], q))
        assert ro["trace"][-1, r] == last
    print(f"{loop}: best H {ro['best_h'].tolist()}", flush=True)


def test_stepwise_readout_exact_many_blocks(oim, orc):
    # 70000 oscillators: 4375 row blocks of partial sums, padded to 8192,
    # folded in two rounds of 4096 with 16 per thread -- still the fixed
    # order, so equal to the oracle's
    n = 70000
    rng = np.random.default_rng(9)
    a, b = rng.integers(0, n, size=(2, 3 * n))
    keep = a != b
    pairs = np.unique(np.stack([np.minimum(a, b)[keep], np.maximum(a, b)[keep]], axis=1), axis=0)
    w = (rng.standard_normal(len(pairs)) * np.exp(rng.uniform(-6, 3, len(pairs))))
    g = synth.csr_from_edges(n, pairs[:, 0], pairs[:, 1], w.astype(np.float32))
    J = (-g.w).astype(np.float32)
    R, q, steps, M = 2, 2, 20, 10
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, J) as prob:
        K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], q, steps)
        th0 = synth.theta0(R, g.n, seed=3)
        ph = _t(_words(th0))
        out = oim.run(prob, _t(th0), _t(K), _t(Ks), _t(sg), _t(synth.seeds(R, 4)), q=q, dt=DT,
                      readout_every=M, flags=oim.OIM_LOOP_STEPWISE, want_best=True, phase=ph)
        ro = {k: v.cpu().numpy() for k, v in out.items()}
        w = ph.cpu().numpy()
    for r in range(R):
        assert ro["best_h"][r] == orc.h_model_fixed(g.row_ptr, g.col, J, q, ro["best_colour"][r])
        last = orc.h_model_fixed(g.row_ptr, g.col, J, q, _colours_from_words(w[r], q))
        assert ro["trace"][-1, r] == last


@pytest.mark.parametrize("rows,cols", [(100, 100), (120, 150)])
def test_lds_resident_readout_tree_over_slices(oim, orc, rows, cols):
    # the 100 x 100 torus (40 slices) keeps every slice's sum in LDS; the
    # 120 x 150 torus (71 slices) leaves no room for them and folds them one
    # round at a time: both give the fixed-order value
    g0 = synth.torus(rows, cols, seed=4)
    rng = np.random.default_rng(rows)
    ei, ej, _ = g0.upper_edges()
    w = (rng.standard_normal(ei.size) * np.exp(rng.uniform(-4, 2, ei.size))).astype(np.float32)
    g = synth.csr_from_edges(g0.n, ei, ej, w)
    J = (-g.w).astype(np.float32)
    R, q, steps, M = 2, 2, 30, 10
    with oim.Problem.from_csr(g.n, g.row_ptr, g.col, J) as prob:
        K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], q, steps)
        th0 = synth.theta0(R, g.n, seed=rows + cols)
        ph = _t(_words(th0))
        out = oim.run(prob, _t(th0), _t(K), _t(Ks), _t(sg), _t(synth.seeds(R, 1)), q=q, dt=DT,
                      readout_every=M, flags=oim.OIM_LOOP_PERSISTENT, want_best=True, phase=ph)
        ro = {k: v.cpu().numpy() for k, v in out.items()}
        w = ph.cpu().numpy()
    for r in range(R):
        assert ro["best_h"][r] == orc.h_model_fixed(g.row_ptr, g.col, J, q, ro["best_colour"][r])
        last = orc.h_model_fixed(g.row_ptr, g.col, J, q, _colours_from_words(w[r], q))
        assert ro["trace"][-1, r] == last


def test_batch_in_run_readout_real_weights_exact(oim, orc):
    gs = [_real_graph(n=n, deg=5.0, seed=30 + k) for k, n in enumerate([700, 260, 1031, 64])]
    big, off = synth.block_diagonal(gs)
    J = (-big.w).astype(np.float32)
    R, q, steps, M = 2, 3, 120, 40
    with oim.Problem.from_csr_blocks(big.n, big.row_ptr, big.col, J, off) as prob:
        K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], q, steps)
        th0 = synth.theta0(R, big.n, seed=7)
        ph = _t(_words(th0))
        out = oim.run(prob, _t(th0), _t(K), _t(Ks), _t(sg), _t(synth.seeds(R, 8)), q=q, dt=DT,
                      readout_every=M, want_best=True, phase=ph)
        ro = {k: v.cpu().numpy() for k, v in out.items()}
        w = ph.cpu().numpy()
    I = len(gs)
    for r in range(R):
        fin = orc.h_model_fixed(big.row_ptr, big.col, J, q, _colours_from_words(w[r], q),
                                inst_off=off)
        best = orc.h_model_fixed(big.row_ptr, big.col, J, q, ro["best_colour"][r], inst_off=off)
        for b in range(I):
            assert ro["trace"][-1, r * I + b] == fin[b]
            assert ro["best_h"][r * I + b] == best[b]


@pytest.mark.parametrize("n,R", [(600, 70), (4096, 512)])
def test_dense_readouts_exact(oim, orc, n, R):
    # SK couplings (real FP32 values spanning many binades): in-run Eq. 1 on
    # the dense loop (BF16x3 and FP32 products), and the standalone readouts
    J = synth.sk_dense(n, seed=3)
    rp, cl, Jv = orc.dense_to_csr(J)
    q, steps, M = 2, 40, 20
    with oim.Problem.from_dense(J) as prob:
        kmax = 32 * 0.5 / (DT * prob.info["max_abs_row_sum"])
        K = synth.ramp(0.0, kmax, 1000)[500:500 + steps].copy()
        Ks = synth.const(0.3, steps)
        sg = synth.const(0.1, steps)
        th0 = synth.theta0(R, n, seed=9)
        sample = sorted({0, R // 2, R - 1})
        for prec in (oim.OIM_PREC_BF16X3, oim.OIM_PREC_FP32):
            ph = _t(_words(th0))
            dth = _t(th0)
            out = oim.run(prob, dth, _t(K), _t(Ks), _t(sg), _t(synth.seeds(R, 4)), q=q, dt=DT,
                          readout_every=M, flags=prec, want_best=True, phase=ph)
            ro = {k: v.cpu().numpy() for k, v in out.items()}
            w = ph.cpu().numpy()
            for r in sample:
                assert ro["best_h"][r] == orc.h_model_fixed(rp, cl, Jv, q, ro["best_colour"][r])
                assert ro["trace"][-1, r] == orc.h_model_fixed(rp, cl, Jv, q,
                                                               _colours_from_words(w[r], q))
        col = oim.oim_round(q, dth)
        hm, _ = oim.oim_energy(prob.handle, q, colour=col)
        cutf = oim.oim_cut(prob.handle, col, exact=False).cpu().numpy()
        hm, col = hm.cpu().numpy(), col.cpu().numpy()
        rows = np.repeat(np.arange(n), np.diff(rp))
        for r in sample:
            assert hm[r] == orc.h_model_fixed(rp, cl, Jv, q, col[r])
            assert cutf[r] == orc.cut_fixed(rp, cl, Jv, col[r])
            print(f"dense n={n} r={r}: H {hm[r]!r}, |GPU - fsum| = "
                  f"{abs(hm[r] - _fsum_terms(rows, cl, Jv, col[r], 'model')):.3e}", flush=True)
