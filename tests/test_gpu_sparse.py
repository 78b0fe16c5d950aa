"""GPU parity of the LDS-resident sparse Euler-Maruyama kernel and the
readout kernels against the FP64 oracle, through the C ABI."""
import os

import numpy as np
import pytest

import synth
from _util import DT, c1_graph, c2_graph, ramp_schedule, wrapdiff

pytestmark = pytest.mark.gpu
TOL_RAD = 1e-5


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


def _gpu_run(oim, prob, th0, K, Ks, sg, sd, q, step0=0, readout_every=0, flags=0,
             want_best=False, phase=None):
    """Returns (theta, readouts) or (theta, readouts, phase words) with `phase`."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(th0)).cuda()
    dph = torch.from_numpy(np.ascontiguousarray(phase)).cuda() if phase is not None else None
    dK = torch.from_numpy(K).cuda()
    dKs = torch.from_numpy(Ks).cuda()
    ds = torch.from_numpy(sg).cuda()
    dsd = torch.from_numpy(np.ascontiguousarray(sd, np.uint64)).cuda()
    out = oim.run(prob, t, dK, dKs, ds, dsd, q=q, dt=DT, readout_every=readout_every,
                  flags=flags, step0=step0, want_best=want_best, phase=dph)
    torch.cuda.synchronize()
    ro = {k: v.cpu().numpy() for k, v in out.items()}
    if phase is not None:
        return t.cpu().numpy(), ro, dph.cpu().numpy()
    return t.cpu().numpy(), ro


def _phase_words(theta):
    """Reference phase words rint(frac(theta / 2pi) 2^32) mod 2^32 in float64."""
    x = np.asarray(theta, np.float64) / (2 * np.pi)
    return (np.rint((x - np.floor(x)) * 2.0**32).astype(np.uint64) % (1 << 32)).astype(np.uint32)


def _colours_from_words(u, q):
    """floor(q u / 2^32 + 1/2) mod q, exactly, in integers."""
    return (((q * u.astype(np.uint64) + (1 << 31)) >> 32) % q).astype(np.int8)


def _problem(oim, g, J):
    return oim.Problem.from_csr(g.n, g.row_ptr, g.col, J)


def _check_parity(orc, oim, g, J, q, R, steps_total, use, seed_th=7, seed_base=0, step0=0,
                  flags=0):
    prob = _problem(oim, g, J)
    K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], q, steps_total, use)
    th0 = synth.theta0(R, g.n, seed=seed_th)
    sd = synth.seeds(R, seed_base)
    got, _ = _gpu_run(oim, prob, th0, K, Ks, sg, sd, q, step0=step0, flags=flags)
    want = orc.run_csr(g.row_ptr, g.col, J, th0, q=q, dt=DT, K=K, Ks=Ks, sigma=sg, seeds=sd,
                       step0=step0)
    err = wrapdiff(got, want).max()
    print(f"n={g.n} q={q} R={R} steps={use}: max |dtheta| = {err:.3e} rad", flush=True)
    assert np.all(np.isfinite(got)) and got.min() >= 0 and got.max() < 2 * np.pi
    assert err < TOL_RAD
    prob.close()
    return got


def test_plain_maxcut_parity_100_steps(dev, oim, orc):
    g = c1_graph()
    _check_parity(orc, oim, g, -g.w, q=2, R=4, steps_total=1000, use=100)


def test_torus_parity_100_steps(dev, oim, orc):
    g = c2_graph()
    _check_parity(orc, oim, g, -g.w, q=2, R=4, steps_total=10000, use=100, step0=1234)


def test_potts_colouring_parity_ragged(dev, oim, orc):
    g, _ = synth.planted_colouring(503, 4.6, 3, seed=2)
    _check_parity(orc, oim, g, -np.ones(g.nnz, np.float32), q=3, R=3, steps_total=5000,
                  use=100)


@pytest.mark.parametrize("q", [4, 5, 16])
def test_generic_q_parity(dev, oim, orc, q):
    g = synth.random_small(97, 0.08, seed=q, weights="real")
    _check_parity(orc, oim, g, -g.w, q=q, R=2, steps_total=1000, use=100)


@pytest.mark.parametrize("loop", ["persistent", "stepwise"])
def test_isolated_oscillators_and_tiny_n(dev, oim, orc, loop):
    # n = 1 (no edges): SHIL and noise only; n = 6 with empty rows and a
    # partial last quad; both loop forms
    flags = oim.OIM_LOOP_STEPWISE if loop == "stepwise" else oim.OIM_LOOP_PERSISTENT
    g = synth.csr_from_edges(1, [], [], [])
    _check_parity(orc, oim, g, np.zeros(0, np.float32), q=2, R=5, steps_total=300, use=100,
                  flags=flags)
    g = synth.csr_from_edges(6, [0, 1, 2], [1, 2, 3], [1.0, -2.0, 0.5])
    _check_parity(orc, oim, g, -g.w, q=2, R=2, steps_total=300, use=100, flags=flags)


def test_full_width_sampled_replicas(dev, oim, orc):
    # the benchmark's launch: 100x100 torus, 256 replicas in one launch; the
    # oracle integrates four sampled replicas (replicas are independent)
    g = c2_graph()
    prob = _problem(oim, g, -g.w)
    K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], 2, 10000, 100)
    th0 = synth.theta0(256, g.n, seed=11)
    sd = synth.seeds(256, 0)
    got, _ = _gpu_run(oim, prob, th0, K, Ks, sg, sd, 2)
    for r in (0, 1, 128, 255):
        want = orc.run_csr(g.row_ptr, g.col, -g.w, th0[r:r + 1], q=2, dt=DT, K=K, Ks=Ks,
                           sigma=sg, seeds=sd[r:r + 1])
        assert wrapdiff(got[r:r + 1], want).max() < TOL_RAD


def test_largest_lds_resident_graph(dev, oim, orc):
    # a 120 x 150 torus (n = 18000, 71 slices of 256 oscillators) is close to
    # the largest replica that fits one workgroup's LDS; it must run on the
    # LDS-resident loop (requested explicitly) and match the oracle on two
    # sampled replicas of 16, readout included
    g = synth.torus(120, 150, seed=9)
    prob = _problem(oim, g, -g.w)
    K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], 2, 1000, 100)
    R = 16
    th0 = synth.theta0(R, g.n, seed=33)
    sd = synth.seeds(R, 12)
    got, ro = _gpu_run(oim, prob, th0, K, Ks, sg, sd, 2, readout_every=25,
                       flags=oim.OIM_LOOP_PERSISTENT)
    pick = [0, R - 1]
    want = orc.run_csr(g.row_ptr, g.col, -g.w, th0[pick], q=2, dt=DT, K=K, Ks=Ks, sigma=sg,
                       seeds=sd[pick])
    err = wrapdiff(got[pick], want).max()
    print(f"persistent n={g.n} R={R} replicas {pick}: max |dtheta| = {err:.3e} rad", flush=True)
    assert np.all(np.isfinite(got)) and got.min() >= 0 and got.max() < 2 * np.pi
    assert err < TOL_RAD
    assert ro["trace"].shape[0] == 4 and np.all(np.isfinite(ro["trace"]))
    prob.close()


def test_resume_and_determinism_bit_exact(dev, oim, orc):
    g = c2_graph()
    prob = _problem(oim, g, -g.w)
    K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], 2, 300)
    th0 = synth.theta0(8, g.n, seed=3)
    sd = synth.seeds(8, 50)
    full, _ = _gpu_run(oim, prob, th0, K, Ks, sg, sd, 2)
    again, _ = _gpu_run(oim, prob, th0, K, Ks, sg, sd, 2)
    np.testing.assert_array_equal(full, again)
    # with the phase words the split run equals the uninterrupted one bit for bit
    w0 = _phase_words(th0)
    full_t, _, full_w = _gpu_run(oim, prob, th0, K, Ks, sg, sd, 2, phase=w0)
    np.testing.assert_array_equal(full_t, full)
    _, _, wa = _gpu_run(oim, prob, th0, K[:120], Ks[:120], sg[:120], sd, 2, phase=w0)
    tb, _, wb = _gpu_run(oim, prob, th0 * 0, K[120:], Ks[120:], sg[120:], sd, 2, step0=120,
                         phase=wa)
    np.testing.assert_array_equal(full_w, wb)
    np.testing.assert_array_equal(full, tb)
    # through FP32 radians only, the state is quantised once at the split; the
    # chaotic dynamics may amplify that, but the bulk of the phases stay close
    ta, _ = _gpu_run(oim, prob, th0, K[:120], Ks[:120], sg[:120], sd, 2)
    tc, _ = _gpu_run(oim, prob, ta, K[120:], Ks[120:], sg[120:], sd, 2, step0=120)
    assert np.median(wrapdiff(tc, full)) < 1e-6


def test_phase_word_conversions(dev, oim):
    import torch
    rng = np.random.default_rng(0)
    th = np.concatenate([rng.uniform(-50, 50, 100000), [0.0, 2 * np.pi, -2 * np.pi, 1e-30,
                                                         np.pi]]).astype(np.float32)
    w = oim.oim_phase_from_theta(torch.from_numpy(th).cuda()).cpu().numpy()
    np.testing.assert_array_equal(w, _phase_words(th))
    back = oim.oim_theta_from_phase(torch.from_numpy(w).cuda()).cpu().numpy()
    assert back.min() >= 0 and back.max() < 2 * np.pi
    assert wrapdiff(back, th).max() < 5e-7


def test_block_size_variants_agree(dev, oim, orc):
    g = c2_graph()
    prob = _problem(oim, g, -g.w)
    K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], 2, 1000, 50)
    th0 = synth.theta0(2, g.n, seed=4)
    sd = synth.seeds(2, 9)
    outs = []
    try:
        for tb in ("256", "512", "1024"):
            os.environ["OIM_PERSIST_TB"] = tb
            outs.append(_gpu_run(oim, prob, th0, K, Ks, sg, sd, 2)[0])
    finally:
        os.environ.pop("OIM_PERSIST_TB", None)
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])


@pytest.mark.parametrize("case", ["maxcut_unit", "ferro", "colouring_batch"])
def test_unit_weight_image_is_bit_identical(dev, oim, case, monkeypatch):
    # couplings that all share one weight, -1 or +1, run on the half-size
    # image of neighbour offsets; phases, phase words and every in-run
    # readout equal the general image's bit for bit
    import torch
    if case == "maxcut_unit":
        g, w, q, R, off = c1_graph(), -1.0, 2, 3, None
    elif case == "ferro":
        g, w, q, R, off = synth.torus(20, 30, seed=2), 1.0, 2, 4, None
    else:
        g, off, _ = _batch(24, 11)
        w, q, R = -1.0, 3, 2
    J = np.full(g.nnz, w, np.float32)
    outs = []
    for general in (False, True):
        if general:
            monkeypatch.setenv("OIM_UNIFORM_WEIGHT_IMAGE", "0")
        else:
            monkeypatch.delenv("OIM_UNIFORM_WEIGHT_IMAGE", raising=False)
        prob = (oim.Problem.from_csr(g.n, g.row_ptr, g.col, J) if off is None else
                oim.Problem.from_csr_blocks(g.n, g.row_ptr, g.col, J, off))
        assert prob.info["uniform_weight"] == (0.0 if general else w)
        K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], q, 600, 300)
        th0 = synth.theta0(R, g.n, seed=3)
        th, ro, words = _gpu_run(oim, prob, th0, K, Ks, sg, synth.seeds(R, 5), q,
                                 readout_every=25, want_best=True,
                                 phase=_phase_words(th0))
        outs.append((th, ro, words))
        prob.close()
    (th_u, ro_u, w_u), (th_g, ro_g, w_g) = outs
    np.testing.assert_array_equal(w_u, w_g)
    np.testing.assert_array_equal(th_u, th_g)
    for name in ("trace", "best_h", "best_step", "best_colour"):
        np.testing.assert_array_equal(ro_u[name], ro_g[name], err_msg=name)
    print(f"{case}: unit-weight image bit-identical ({R} replicas)", flush=True)


def test_steps_zero_leaves_theta(dev, oim):
    g = synth.cycle(10)
    prob = _problem(oim, g, -g.w)
    th0 = synth.theta0(2, 10, seed=0) * 3.0  # out-of-range values stay as given
    e = np.zeros(0, np.float32)
    got, _ = _gpu_run(oim, prob, th0, e, e, e, synth.seeds(2), 2)
    np.testing.assert_array_equal(got, th0)


def test_readouts_bit_exact_from_identical_phases(dev, oim, orc):
    import torch
    g = c1_graph()
    J = -g.w
    prob = _problem(oim, g, J)
    K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], 2, 400)
    th0 = synth.theta0(6, g.n, seed=5)
    th, _ = _gpu_run(oim, prob, th0, K, Ks, sg, synth.seeds(6, 1), 2)
    # plus hand-made phases on and around the thresholds
    edge = np.float32(np.pi / 2) + np.array([-1e-6, 0, 1e-6], np.float32)
    th[0, :3] = edge
    for q in (2, 3):
        dth = torch.from_numpy(th).cuda()
        col = oim.oim_round(q, dth).cpu().numpy()
        np.testing.assert_array_equal(col, orc.round_f32(th, q))
        dcol = torch.from_numpy(col).cuda()
        hm, h6 = oim.oim_energy(prob.handle, q, dth, dcol)
        hm, h6 = hm.cpu().numpy(), h6.cpu().numpy()
        for r in range(th.shape[0]):
            assert hm[r] == orc.h_model(g.row_ptr, g.col, J, q, col[r])
            want6 = orc.h_eq6_fixed(g.row_ptr, g.col, J, th[r].astype(np.float64))
            # one FP64 cosine rounding per term at most (each side's maths library)
            assert abs(h6[r] - want6) <= 2.0**-52 * np.abs(J).astype(np.float64).sum()
        conf = oim.oim_conflicts(prob.handle, dcol).cpu().numpy()
        for r in range(th.shape[0]):
            assert conf[r] == orc.conflicts(g.row_ptr, g.col, J, col[r])
    col = oim.oim_round(2, torch.from_numpy(th).cuda())
    cut = oim.oim_cut(prob.handle, col).cpu().numpy()
    cutf = oim.oim_cut(prob.handle, col, exact=False).cpu().numpy()
    col = col.cpu().numpy()
    for r in range(th.shape[0]):
        want = orc.cut_int(g.row_ptr, g.col, J.astype(np.int64), col[r])
        assert cut[r] == want and cutf[r] == want


def test_round_special_values(dev, oim, orc):
    import torch
    th = np.array([np.nan, np.inf, -np.inf, 2e6, -2e6, -0.1, 0.0, 6.2831853, 1e5], np.float32)
    for q in (2, 3, 16):
        got = oim.oim_round(q, torch.from_numpy(th).cuda()).cpu().numpy()
        np.testing.assert_array_equal(got, orc.round_f32(th, q))


def test_real_weight_cut_needs_f64(dev, oim, orc):
    # the exact int64 cut is refused for real weights; the FP64 cut follows
    # the oracle's fixed order bit for bit (more cases in the readout tests)
    import torch
    g = synth.random_small(300, 0.05, seed=9, weights="real")
    J = -g.w
    prob = _problem(oim, g, J)
    assert prob.info["integer_weights"] == 0
    col = np.random.default_rng(0).integers(0, 2, size=(3, 300)).astype(np.int8)
    dcol = torch.from_numpy(col).cuda()
    with pytest.raises(oim.OimError):
        oim.oim_cut(prob.handle, dcol)
    cutf = oim.oim_cut(prob.handle, dcol, exact=False).cpu().numpy()
    for r in range(3):
        assert cutf[r] == orc.cut_fixed(g.row_ptr, g.col, J, col[r])


def test_in_run_readout_trace(dev, oim, orc):
    g = c1_graph()
    J = -g.w
    prob = _problem(oim, g, J)
    K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], 2, 230)
    th0 = synth.theta0(3, g.n, seed=6)
    th, ro = _gpu_run(oim, prob, th0, K, Ks, sg, synth.seeds(3, 2), 2, readout_every=50,
                      want_best=True)
    tr = ro["trace"]
    assert tr.shape == (5, 3)
    np.testing.assert_array_equal(ro["best_h"], tr.min(axis=0))
    for r in range(3):
        k = int(np.argmin(tr[:, r]))
        assert ro["best_step"][r] == min(50 * (k + 1), 230)
        assert orc.h_model(g.row_ptr, g.col, J, 2, ro["best_colour"][r]) == ro["best_h"][r]
    # the last readout thresholds the final phase words exactly
    th2, _, w = _gpu_run(oim, prob, th0, K, Ks, sg, synth.seeds(3, 2), 2,
                         phase=_phase_words(th0))
    for r in range(3):
        assert tr[-1, r] == orc.h_model(g.row_ptr, g.col, J, 2, _colours_from_words(w[r], 2))
    # same trajectory with and without the readout
    np.testing.assert_array_equal(th, th2)


# ---------------------------------------------------------------- stepwise ----
def test_stepwise_parity(dev, oim, orc):
    # the device-memory, graph-captured loop on the same cases
    for g, J, q, R, total in [
        (c1_graph(), None, 2, 3, 1000),
        (c2_graph(), None, 2, 70, 10000),
        (synth.planted_colouring(503, 4.6, 3, seed=2)[0], "colour", 3, 2, 5000),
        (synth.random_small(97, 0.08, seed=5, weights="real"), None, 5, 2, 1000),
    ]:
        Jv = -np.ones(g.nnz, np.float32) if J == "colour" else -g.w
        prob = _problem(oim, g, Jv)
        K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], q, total, 101)
        th0 = synth.theta0(R, g.n, seed=31)
        sd = synth.seeds(R, 4)
        got, _ = _gpu_run(oim, prob, th0, K, Ks, sg, sd, q, step0=9, flags=oim.OIM_LOOP_STEPWISE)
        want = orc.run_csr(g.row_ptr, g.col, Jv, th0, q=q, dt=DT, K=K, Ks=Ks, sigma=sg,
                           seeds=sd, step0=9)
        err = wrapdiff(got, want).max()
        print(f"stepwise n={g.n} q={q} R={R}: max |dtheta| = {err:.3e} rad", flush=True)
        assert err < TOL_RAD
        prob.close()


def test_graph_beyond_lds_runs_stepwise(dev, oim, orc):
    # a 200 x 300 torus (n = 60000) does not fit one workgroup's LDS: the
    # persistent loop is refused with an error, the automatic choice runs the
    # stepwise loop, and two sampled replicas of eight match the oracle
    g = synth.torus(200, 300, seed=8)
    prob = _problem(oim, g, -g.w)
    K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], 2, 2000, 100)
    R = 8
    th0 = synth.theta0(R, g.n, seed=32)
    sd = synth.seeds(R, 6)
    with pytest.raises(oim.OimError):
        _gpu_run(oim, prob, th0, K, Ks, sg, sd, 2, flags=oim.OIM_LOOP_PERSISTENT)
    got, _ = _gpu_run(oim, prob, th0, K, Ks, sg, sd, 2, step0=3)
    pick = [0, R - 1]
    want = orc.run_csr(g.row_ptr, g.col, -g.w, th0[pick], q=2, dt=DT, K=K, Ks=Ks, sigma=sg,
                       seeds=sd[pick], step0=3)
    err = wrapdiff(got[pick], want).max()
    print(f"stepwise n={g.n} R={R} replicas {pick}: max |dtheta| = {err:.3e} rad", flush=True)
    assert np.all(np.isfinite(got)) and got.min() >= 0 and got.max() < 2 * np.pi
    assert err < TOL_RAD
    prob.close()


@pytest.mark.parametrize("case", ["torus_auto", "irregular_forced", "ragged_cycle"])
def test_stepwise_forms_are_bit_identical(dev, oim, case, monkeypatch):
    # the stepwise loop's four forms: entries from the CSR or from the padded
    # row image (every row the same length, padding of weight 0), state
    # words addressed as buffer offsets or at 64-bit global addresses;
    # phases, phase words and every in-run readout equal bit for bit
    if case == "torus_auto":
        g, q, R, mode = synth.torus(20, 30, seed=2), 2, 70, None
    elif case == "irregular_forced":
        g, q, R, mode = synth.random_small(203, 0.05, seed=7, weights="real"), 3, 5, "1"
    else:
        # generic q (sin(q theta) from the phase word), ragged last quad
        g, q, R, mode = synth.cycle(11), 5, 3, None
    J = -g.w
    outs = []
    for csr, global_addr in ((True, False), (False, False), (False, True), (True, True)):
        if csr:
            monkeypatch.setenv("OIM_STEPWISE_ELL", "0")
        elif mode is None:
            monkeypatch.delenv("OIM_STEPWISE_ELL", raising=False)
        else:
            monkeypatch.setenv("OIM_STEPWISE_ELL", mode)
        if global_addr:
            monkeypatch.setenv("OIM_STEPWISE_GLOBAL_ADDR", "1")
        else:
            monkeypatch.delenv("OIM_STEPWISE_GLOBAL_ADDR", raising=False)
        prob = _problem(oim, g, J)
        D = prob.info["stepwise_row_length"]
        dmax = int(np.diff(g.row_ptr).max())
        if csr:
            assert D == 0
        else:
            assert D % 4 == 0 and dmax <= D < max(dmax, 1) + 4, D
        K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], q, 400, 230)
        th0 = synth.theta0(R, g.n, seed=13)
        th, ro, words = _gpu_run(oim, prob, th0, K, Ks, sg, synth.seeds(R, 8), q, step0=5,
                                 readout_every=23, want_best=True, flags=oim.OIM_LOOP_STEPWISE,
                                 phase=_phase_words(th0))
        outs.append((th, ro, words))
        prob.close()
    th_c, ro_c, w_c = outs[0]
    for th_e, ro_e, w_e in outs[1:]:
        np.testing.assert_array_equal(w_c, w_e)
        np.testing.assert_array_equal(th_c, th_e)
        for name in ("trace", "best_h", "best_step", "best_colour"):
            np.testing.assert_array_equal(ro_c[name], ro_e[name], err_msg=name)
    print(f"{case}: four stepwise forms bit-identical (n={g.n}, {R} replicas)", flush=True)


def test_stepwise_readout_and_resume(dev, oim, orc):
    g = c1_graph()
    J = -g.w
    prob = _problem(oim, g, J)
    K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], 2, 230)
    th0 = synth.theta0(3, g.n, seed=6)
    w0 = _phase_words(th0)
    F = oim.OIM_LOOP_STEPWISE
    th, ro, w = _gpu_run(oim, prob, th0, K, Ks, sg, synth.seeds(3, 2), 2, readout_every=50,
                         want_best=True, flags=F, phase=w0)
    tr = ro["trace"]
    assert tr.shape == (5, 3)
    np.testing.assert_array_equal(ro["best_h"], tr.min(axis=0))
    for r in range(3):
        k = int(np.argmin(tr[:, r]))
        assert ro["best_step"][r] == min(50 * (k + 1), 230)
        assert orc.h_model(g.row_ptr, g.col, J, 2, ro["best_colour"][r]) == ro["best_h"][r]
        assert tr[-1, r] == orc.h_model(g.row_ptr, g.col, J, 2, _colours_from_words(w[r], 2))
    # split run with phase words == uninterrupted run, bit for bit
    _, _, wa = _gpu_run(oim, prob, th0, K[:77], Ks[:77], sg[:77], synth.seeds(3, 2), 2, flags=F,
                        phase=w0)
    _, _, wb = _gpu_run(oim, prob, th0, K[77:], Ks[77:], sg[77:], synth.seeds(3, 2), 2,
                        step0=77, flags=F, phase=wa)
    np.testing.assert_array_equal(w, wb)
    # and the persistent kernel reaches the same phases within the parity bound
    th_p, _ = _gpu_run(oim, prob, th0, K, Ks, sg, synth.seeds(3, 2), 2)
    assert wrapdiff(th_p, th).max() < TOL_RAD


# ------------------------------------------------------ block-diagonal batch ----
def _batch(count, seed):
    pairs = synth.planted_batch(count, 100, 600, 4.6, 3, seed)
    graphs = [g for g, _ in pairs]
    off = np.cumsum([0] + [g.n for g in graphs]).astype(np.int32)
    ei, ej = [], []
    for g, o in zip(graphs, off[:-1]):
        a, b, _ = g.upper_edges()
        ei.append(a + o)
        ej.append(b + o)
    big = synth.csr_from_edges(int(off[-1]), np.concatenate(ei), np.concatenate(ej),
                               np.ones(sum(len(x) for x in ei)))
    return big, off, graphs


def test_ragged_batch_parity_and_readout(dev, oim, orc):
    big, off, graphs = _batch(24, seed=2)
    J = -np.ones(big.nnz, np.float32)
    prob = oim.Problem.from_csr_blocks(big.n, big.row_ptr, big.col, J, off)
    assert prob.info["n_instances"] == 24
    K, Ks, sg = ramp_schedule(prob.info["max_abs_row_sum"], 3, 5000, 100)
    R = 2
    th0 = synth.theta0(R, big.n, seed=12)
    sd = synth.seeds(R, 40)
    w0 = _phase_words(th0)
    got, ro, w = _gpu_run(oim, prob, th0, K, Ks, sg, sd, 3, step0=3, readout_every=25,
                          want_best=True, phase=w0)
    want = orc.run_csr_blocks(big.row_ptr, big.col, J, off, th0, q=3, dt=DT, K=K, Ks=Ks,
                              sigma=sg, seeds=sd, step0=3)
    err = wrapdiff(got, want).max()
    print(f"batch of 24, n_total={big.n}: max |dtheta| = {err:.3e} rad", flush=True)
    assert err < TOL_RAD
    tr = ro["trace"]
    assert tr.shape == (4, R * 24)
    for r in range(R):
        for b, g in enumerate(graphs):
            cols = _colours_from_words(w[r, off[b]:off[b + 1]], 3)
            Jb = -np.ones(g.nnz)
            # the last readout is this instance's Eq. 2 energy = conflicts for J = -1
            assert tr[-1, r * 24 + b] == orc.h_model(g.row_ptr, g.col, Jb, 3, cols)
            bc = ro["best_colour"][r, off[b]:off[b + 1]]
            assert ro["best_h"][r * 24 + b] == orc.conflicts(g.row_ptr, g.col, Jb, bc)


def test_batch_instance_zero_matches_standalone(dev, oim, orc):
    big, off, graphs = _batch(5, seed=7)
    g0 = graphs[0]
    K, Ks, sg = ramp_schedule(10.0, 3, 1000, 60)
    th0 = synth.theta0(3, big.n, seed=2)
    sd = synth.seeds(3, 1)
    with oim.Problem.from_csr_blocks(big.n, big.row_ptr, big.col, -np.ones(big.nnz), off) as pb, \
            oim.Problem.from_csr(g0.n, g0.row_ptr, g0.col, -np.ones(g0.nnz)) as p0:
        a, _ = _gpu_run(oim, pb, th0, K, Ks, sg, sd, 3)
        b, _ = _gpu_run(oim, p0, np.ascontiguousarray(th0[:, :g0.n]), K, Ks, sg, sd, 3)
    np.testing.assert_array_equal(a[:, :g0.n], b)
