"""Pins of the oracle's integrator (Eq. 5 / Algorithm 1 with the readings
stated in oracle.c) against closed forms and invariants of the dynamics."""
import numpy as np
import pytest

import synth

TWO_PI = 2 * np.pi


def _pair():
    # one max-cut edge of weight 1  ->  Ising coupling J = -1
    return np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32), np.array([-1.0, -1.0])


def _wrapdiff(a, b):
    d = np.mod(a - b, TWO_PI)
    return np.minimum(d, TWO_PI - d)


def test_noise_only_is_sum_of_kicks(orc):
    # K = Ks = 0: theta_T = wrap(theta_0 + sum_t sigma_t sqrt(dt) xi_t)
    g = synth.random_small(9, 0.5, seed=1, weights="int")
    steps, dt = 25, 0.01
    th0 = synth.theta0(3, 9, seed=2)
    sig = synth.ramp(0.05, 0.3, steps)
    sd = np.array([3, 1 << 33, 12345], np.uint64)
    out = orc.run_csr(g.row_ptr, g.col, -g.w, th0, q=2, dt=dt, K=np.zeros(steps),
                      Ks=np.zeros(steps), sigma=sig, seeds=sd, step0=7)
    for r in range(3):
        acc = th0[r].astype(np.float64).copy()
        for s in range(steps):
            acc += float(sig[s]) * np.sqrt(dt) * orc.normals(int(sd[r]), 0, 9, 7 + s)
        assert np.max(_wrapdiff(out[r], np.mod(acc, TWO_PI))) < 1e-12
        assert np.all((out[r] >= 0) & (out[r] < TWO_PI))


@pytest.mark.parametrize("K", [0.7, 2.0])
def test_pair_closed_form_and_first_order(orc, K):
    # For J = -1 the phase difference d obeys d' = 2K sin d, solved by
    # tan(d/2) = tan(d0/2) exp(2 K t): the edge is driven to anti-phase (cut).
    rp, cl, J = _pair()
    th0 = np.array([[1.0, 0.6]])
    T = 1.0
    exact = 2 * np.arctan(np.tan(0.4 / 2) * np.exp(2 * K * T))
    errs = []
    for dt in (1e-3, 5e-4, 2.5e-4):
        steps = int(round(T / dt))
        out = orc.run_csr(rp, cl, J, th0, q=2, dt=dt, K=np.full(steps, K), Ks=np.zeros(steps),
                          sigma=np.zeros(steps), seeds=np.zeros(1, np.uint64))
        d = np.mod(out[0, 0] - out[0, 1], TWO_PI)
        errs.append(abs(d - exact))
        # the mean phase does not move
        m = np.angle(np.exp(1j * out[0]).sum())
        assert abs(np.mod(m - 0.8 + np.pi, TWO_PI) - np.pi) < 1e-12
    assert errs[0] < 2e-2
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2


@pytest.mark.parametrize("q", [2, 3, 4])
def test_shil_closed_form(orc, q):
    # K = sigma = 0: u = q theta obeys u' = -q Ks sin u, tan(u/2) = tan(u0/2) exp(-q Ks t)
    Ks, T, dt = 1.3, 0.8, 1e-4
    steps = int(round(T / dt))
    th0 = np.array([[0.3 / q, 1.0 / q, 2.9 / q]])
    rp = np.zeros(4, np.int64)
    out = orc.run_csr(rp, np.zeros(0, np.int32), np.zeros(0), th0, q=q, dt=dt, K=np.zeros(steps),
                      Ks=np.full(steps, Ks), sigma=np.zeros(steps), seeds=np.zeros(1, np.uint64))
    u0 = q * th0[0]
    exact = 2 * np.arctan(np.tan(u0 / 2) * np.exp(-q * Ks * T)) / q
    assert np.max(np.abs(out[0] - exact)) < 1e-4


@pytest.mark.parametrize("q", [2, 3, 5])
def test_shil_fixed_points(orc, q):
    # stable at 2 pi k / q, unstable at (2k+1) pi / q
    steps, dt = 4000, 0.01
    k = np.arange(q)
    stable = 2 * np.pi * k / q
    th0 = np.concatenate([stable + 0.2 * np.pi / q, stable - 0.2 * np.pi / q,
                          stable + np.pi / q + 1e-3])[None, :]
    n = th0.shape[1]
    out = orc.run_csr(np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0), th0, q=q,
                      dt=dt, K=np.zeros(steps), Ks=np.full(steps, 1.0), sigma=np.zeros(steps),
                      seeds=np.zeros(1, np.uint64))[0]
    np.testing.assert_allclose(_wrapdiff(out[:2 * q], np.tile(stable, 2)), 0, atol=1e-9)
    # the points started just past an unstable point fell to the next stable one
    assert np.max(_wrapdiff(out[2 * q:], np.mod(stable + 2 * np.pi / q, TWO_PI))) < 1e-9
    # exactly at a stable point nothing moves
    still = orc.run_csr(np.zeros(q + 1, np.int64), np.zeros(0, np.int32), np.zeros(0),
                        stable[None, :], q=q, dt=dt, K=np.zeros(10), Ks=np.full(10, 1.0),
                        sigma=np.zeros(10), seeds=np.zeros(1, np.uint64))[0]
    assert np.max(_wrapdiff(still, stable)) < 1e-12


def test_coupling_conserves_phase_sum(orc):
    # Ks = 0: the coupling of a symmetric J cancels pairwise, so the sum of
    # phases moves by the noise alone (mod 2 pi).
    g = synth.random_small(14, 0.4, seed=8, weights="real")
    steps, dt = 40, 0.02
    th0 = synth.theta0(2, 14, seed=3)
    sig = synth.const(0.2, steps)
    sd = synth.seeds(2, 9)
    out = orc.run_csr(g.row_ptr, g.col, -g.w, th0, q=2, dt=dt, K=synth.const(1.5, steps),
                      Ks=np.zeros(steps), sigma=sig, seeds=sd)
    for r in range(2):
        kicks = sum(float(sig[s]) * np.sqrt(dt) * orc.normals(int(sd[r]), 0, 14, s).sum()
                    for s in range(steps))
        lhs = out[r].sum() - th0[r].astype(np.float64).sum() - kicks
        assert abs(np.mod(lhs + np.pi, TWO_PI) - np.pi) < 1e-10


def _lyapunov(theta, g, J, K, Ks, q):
    ei, ej, _ = g.upper_edges()
    Jup = J[np.repeat(np.arange(g.n), np.diff(g.row_ptr)) < g.col]
    return (-K * np.sum(Jup * np.cos(theta[ei] - theta[ej]))
            - Ks / q * np.sum(np.cos(q * theta)))


@pytest.mark.parametrize("q", [2, 3])
def test_noiseless_flow_descends_energy(orc, q):
    # sigma = 0, constant K and Ks: Euler steps on dtheta/dt = -grad E with a
    # small dt never raise E = -K sum J cos(d) - Ks/q sum cos(q theta).
    g = synth.random_small(16, 0.35, seed=10, weights="pm1")
    J = -g.w.astype(np.float64)
    K, Ks, dt = 1.0, 0.7, 0.005
    th = synth.theta0(1, 16, seed=4).astype(np.float64)
    E = [_lyapunov(th[0], g, J, K, Ks, q)]
    for _ in range(200):
        th = orc.run_csr(g.row_ptr, g.col, J, th, q=q, dt=dt, K=[K], Ks=[Ks], sigma=[0.0],
                         seeds=np.zeros(1, np.uint64))
        E.append(_lyapunov(th[0], g, J, K, Ks, q))
    assert np.all(np.diff(E) <= 1e-12)
    assert E[-1] < E[0] - 0.5


@pytest.mark.parametrize("q", [2, 3])
def test_euler_first_order_in_dt(orc, q):
    # sigma = 0: Algorithm 1 is the explicit Euler method on the flow of
    # Eq. 5, so the error at a fixed time T falls linearly with the step:
    # halving dt halves the distance to a 128x finer reference.
    g = synth.random_small(14, 0.4, seed=21, weights="pm1")
    J = -g.w.astype(np.float64)
    K, Ks, T = 1.3, 0.9, 0.64
    th0 = synth.theta0(1, 14, seed=8).astype(np.float64)

    def run(dt):
        steps = int(round(T / dt))
        return orc.run_csr(g.row_ptr, g.col, J, th0, q=q, dt=dt, K=np.full(steps, K),
                           Ks=np.full(steps, Ks), sigma=np.zeros(steps),
                           seeds=np.zeros(1, np.uint64))
    ref = run(0.04 / 128)
    err = [float(np.max(_wrapdiff(run(dt), ref))) for dt in (0.04, 0.02, 0.01)]
    assert err[0] > 1e-4  # the step error is visible at the coarsest dt
    for a, b in zip(err, err[1:]):
        assert 1.7 < a / b < 2.4, err


def test_csr_and_dense_agree(orc):
    g = synth.random_small(12, 0.5, seed=11, weights="real")
    Jd = np.zeros((12, 12))
    ei, ej, w = g.upper_edges()
    Jd[ei, ej] = -w
    Jd[ej, ei] = -w
    np.fill_diagonal(Jd, 5.0)  # the diagonal of a dense coupling is ignored
    steps = 30
    kw = dict(q=3, dt=0.01, K=synth.ramp(0.1, 2.0, steps), Ks=synth.ramp(0, 3.0, steps),
              sigma=synth.const(0.1, steps), seeds=synth.seeds(2, 4), step0=3)
    th0 = synth.theta0(2, 12, seed=5)
    a = orc.run_csr(g.row_ptr, g.col, -g.w, th0, **kw)
    b = orc.run_dense(Jd, th0, **kw)
    assert np.max(_wrapdiff(a, b)) < 1e-12


def test_resume_and_replica_independence(orc):
    g = synth.erdos_renyi(40, 0.2, seed=12)
    steps = 20
    K, Ks, sig = synth.ramp(0.1, 1, steps), synth.ramp(0, 2, steps), synth.const(0.1, steps)
    th0 = synth.theta0(3, 40, seed=6)
    sd = synth.seeds(3, 100)
    full = orc.run_csr(g.row_ptr, g.col, -g.w, th0, q=2, dt=0.01, K=K, Ks=Ks, sigma=sig, seeds=sd)
    half = orc.run_csr(g.row_ptr, g.col, -g.w, th0, q=2, dt=0.01, K=K[:8], Ks=Ks[:8],
                       sigma=sig[:8], seeds=sd)
    rest = orc.run_csr(g.row_ptr, g.col, -g.w, half, q=2, dt=0.01, K=K[8:], Ks=Ks[8:],
                       sigma=sig[8:], seeds=sd, step0=8)
    np.testing.assert_array_equal(full, rest)
    one = orc.run_csr(g.row_ptr, g.col, -g.w, th0[1:2], q=2, dt=0.01, K=K, Ks=Ks, sigma=sig,
                      seeds=sd[1:2])
    np.testing.assert_array_equal(full[1:2], one)


def _concat(graphs):
    return synth.block_diagonal(graphs)


def test_block_batch_instances(orc):
    # instance 0 of a block-diagonal batch is the standalone run of its graph;
    # every instance draws its noise with local indices and its instance number
    gs = [synth.random_small(n, 0.3, seed=n, weights="pm1") for n in (9, 14, 6)]
    big, off = _concat(gs)
    steps = 25
    kw = dict(q=2, dt=0.01, K=synth.ramp(0.1, 1.0, steps), Ks=synth.ramp(0, 2.0, steps),
              sigma=synth.const(0.1, steps), seeds=synth.seeds(2, 5), step0=4)
    th0 = synth.theta0(2, big.n, seed=1)
    out = orc.run_csr_blocks(big.row_ptr, big.col, -big.w, off, th0, **kw)
    alone = orc.run_csr(gs[0].row_ptr, gs[0].col, -gs[0].w, th0[:, :9], **kw)
    np.testing.assert_array_equal(out[:, :9], alone)
    # noise-only check of instance 2 (K = Ks = 0)
    kw0 = dict(kw, K=np.zeros(steps), Ks=np.zeros(steps))
    out0 = orc.run_csr_blocks(big.row_ptr, big.col, -big.w, off, th0, **kw0)
    acc = th0[1, off[2]:off[3]].astype(np.float64).copy()
    for s in range(steps):
        acc += float(kw["sigma"][s]) * np.sqrt(0.01) * np.array([orc.normal(int(kw["seeds"][1]), i, 4 + s, 2)
                                               for i in range(6)])
    assert np.max(_wrapdiff(out0[1, off[2]:off[3]], np.mod(acc, TWO_PI))) < 1e-12
    # and a different instance number gives a different stream
    assert orc.normal(5, 3, 7, 1) != orc.normal(5, 3, 7, 0)


def test_single_instance_is_its_block(orc):
    # a graph integrated alone as instance b follows instance b of the batch
    gs = [synth.random_small(n, 0.3, seed=n, weights="pm1") for n in (9, 14, 6)]
    big, off = _concat(gs)
    steps = 20
    kw = dict(q=3, dt=0.01, K=synth.ramp(0.1, 1.0, steps), Ks=synth.ramp(0, 2.0, steps),
              sigma=synth.const(0.2, steps), seeds=synth.seeds(2, 9), step0=11)
    th0 = synth.theta0(2, big.n, seed=4)
    out = orc.run_csr_blocks(big.row_ptr, big.col, -big.w, off, th0, **kw)
    for b, g in enumerate(gs):
        alone = orc.run_csr(g.row_ptr, g.col, -g.w, th0[:, off[b]:off[b + 1]], instance=b, **kw)
        np.testing.assert_array_equal(out[:, off[b]:off[b + 1]], alone)


def test_threads_over_rows_give_the_same_bits(orc):
    # one replica with its rows shared among threads, and the dense loop,
    # equal the single-thread run bit for bit
    g = synth.gnp_avg_degree(300, 8.0, seed=3, signed=True)
    steps = 30
    kw = dict(q=2, dt=0.01, K=synth.ramp(0.5, 3.0, steps), Ks=synth.ramp(0, 5.0, steps),
              sigma=synth.const(0.1, steps), seeds=synth.seeds(1, 2))
    th0 = synth.theta0(1, g.n, seed=5)
    one = orc.run_csr(g.row_ptr, g.col, -g.w, th0, nthreads=1, **kw)
    for t in (2, 3, 8):
        np.testing.assert_array_equal(orc.run_csr(g.row_ptr, g.col, -g.w, th0, nthreads=t, **kw),
                                      one)
    Jd = synth.sk_dense(64, seed=1).astype(np.float64)
    th1 = synth.theta0(2, 64, seed=6)
    kw2 = dict(kw, seeds=synth.seeds(2, 2))
    d1 = orc.run_dense(Jd, th1, nthreads=1, **kw2)
    np.testing.assert_array_equal(orc.run_dense(Jd, th1, nthreads=5, **kw2), d1)


@pytest.mark.parametrize("q", [2, 3])
def test_adjoint_matches_finite_differences(orc, q):
    # The FP64 adjoint's gradient of the relaxed cut against central
    # differences of the same loss, per schedule entry.
    g = synth.random_small(12, 0.4, seed=21, weights="pm1")
    J = -g.w.astype(np.float64)
    steps, dt = 30, 0.02
    K = synth.ramp(0.2, 1.5, steps).astype(np.float64)
    Ks = synth.ramp(0.0, 2.0, steps).astype(np.float64)
    sg = synth.const(0.15, steps).astype(np.float64)
    th0 = synth.theta0(2, 12, seed=9).astype(np.float64)
    sd = synth.seeds(2, 3)

    def loss(K_, Ks_, sg_):
        th = orc.run_csr(g.row_ptr, g.col, J, th0, q=q, dt=dt, K=K_, Ks=Ks_, sigma=sg_,
                         seeds=sd, step0=5)
        return orc.relaxed_cut(g.row_ptr, g.col, J, th)

    L, gK, gKs, gS = orc.adjoint_csr(g.row_ptr, g.col, J, th0, q=q, dt=dt, K=K, Ks=Ks, sigma=sg,
                                     seeds=sd, step0=5)
    assert L == pytest.approx(loss(K, Ks, sg), rel=1e-12)
    eps = 1e-5
    for s in (0, 7, 18, 29):
        for vec, grad in ((K, gK), (Ks, gKs), (sg, gS)):
            up, dn = vec.copy(), vec.copy()
            up[s] += eps
            dn[s] -= eps
            args_up = [up if v is vec else v for v in (K, Ks, sg)]
            args_dn = [dn if v is vec else v for v in (K, Ks, sg)]
            fd = (loss(*args_up) - loss(*args_dn)) / (2 * eps)
            assert grad[s] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_adjoint_block_batch_matches_finite_differences(orc):
    # the batched adjoint (noise per instance) against central differences of
    # the block-diagonal forward integrator, and its loss against the relaxed
    # cut of that integrator's final phases
    gs = [synth.random_small(n, 0.45, seed=30 + n, weights="pm1") for n in (7, 11)]
    big, off = _concat(gs)
    J = -big.w.astype(np.float64)
    steps, dt = 20, 0.02
    K = synth.ramp(0.3, 1.2, steps).astype(np.float64)
    Ks = synth.ramp(0.0, 1.5, steps).astype(np.float64)
    sg = synth.const(0.2, steps).astype(np.float64)
    th0 = synth.theta0(2, big.n, seed=4).astype(np.float64)
    sd = synth.seeds(2, 8)

    def loss(K_, Ks_, sg_):
        th = orc.run_csr_blocks(big.row_ptr, big.col, J, off, th0, q=2, dt=dt, K=K_, Ks=Ks_,
                                sigma=sg_, seeds=sd, step0=3)
        return orc.relaxed_cut(big.row_ptr, big.col, J, th)

    L, gK, gKs, gS = orc.adjoint_csr(big.row_ptr, big.col, J, th0, q=2, dt=dt, K=K, Ks=Ks,
                                     sigma=sg, seeds=sd, step0=3, inst_off=off)
    assert L == pytest.approx(loss(K, Ks, sg), rel=1e-12)
    eps = 1e-5
    for s in (0, 11, 19):
        for vec, grad in ((K, gK), (Ks, gKs), (sg, gS)):
            up, dn = vec.copy(), vec.copy()
            up[s] += eps
            dn[s] -= eps
            fd = (loss(*[up if v is vec else v for v in (K, Ks, sg)]) -
                  loss(*[dn if v is vec else v for v in (K, Ks, sg)])) / (2 * eps)
            assert grad[s] == pytest.approx(fd, rel=1e-5, abs=1e-9)
