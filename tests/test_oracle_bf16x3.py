"""Pins of the oracle's BF16x3 split-product form of the dense coupling (the
precision of the dense all-to-all workload): the BF16 rounding against
PyTorch's own float32 -> bfloat16 conversion, a coherent case whose split
products are written out by hand from that conversion, the error bound of the
split against the exact coupling, and the integrator around it."""
import numpy as np
import pytest
import torch

import synth

TWO_PI = 2 * np.pi


def _bf16_torch(x):
    """float32 -> bfloat16 -> float64 by PyTorch (round to nearest, ties to even)."""
    t = torch.from_numpy(np.asarray(x, np.float32).copy()).to(torch.bfloat16)
    return t.to(torch.float64).numpy()


def test_bf16_round_matches_torch(orc):
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(4000).astype(np.float32),
        (rng.standard_normal(2000) * 1e-3).astype(np.float32),
        rng.uniform(-1, 1, 2000).astype(np.float32),
    ])
    # constructed ties: low 16 bits exactly 0x8000, kept LSB even and odd
    bits = rng.integers(0x3e000000, 0x40000000, 2000, dtype=np.uint32)
    ties = ((bits & 0xffff0000) | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, -ties, np.float32([0.0, 1.0, -2.5, 1 / 3])])
    want = _bf16_torch(x)
    got = np.array([orc.bf16_round(float(v)) for v in x])
    assert np.array_equal(got, want)
    # ties do go to even: both parities of the kept bit occur among the cases
    kept = (ties.view(np.uint32) >> 16) & 1
    assert kept.min() == 0 and kept.max() == 1


def _split(x):
    h = _bf16_torch(x)
    lo = _bf16_torch(np.float32(x) - np.float32(h))
    return h, lo


@pytest.mark.parametrize("theta", [0.7, 2.1, 5.3])
def test_coherent_case_by_hand(orc, theta):
    # J_ij = a for every i != j and every phase equal: the split products of
    # every row are the same three terms, summed n - 1 times.  The exact
    # coupling is 0; the BF16x3 value is the residue of the splits.
    n = 37
    a = np.float32(1.0 / 3.0)
    J = np.full((n, n), a, np.float64)
    np.fill_diagonal(J, 0.0)
    th = np.full(n, theta)
    s32, c32 = np.float32(np.sin(theta)), np.float32(np.cos(theta))
    ah, al = _split(a)
    sh, sl = _split(s32)
    ch, cl = _split(c32)
    ys = (n - 1) * (ah * sh + ah * sl + al * sh)
    yc = (n - 1) * (ah * ch + ah * cl + al * ch)
    want = np.sin(theta) * yc - np.cos(theta) * ys
    got = orc.coupling_dense_bf16x3(J, th)
    scale = (n - 1) * float(a)
    assert np.max(np.abs(got - want)) <= 1e-13 * scale
    # the dropped and split terms leave a residue of the order 2^-16 of the
    # row sum, not of 2^-8 (which a dropped cross term would leave)
    assert np.max(np.abs(got)) <= 3.01 * 2.0 ** -16 * scale


def test_split_error_bound_against_exact(orc):
    # |c(bf16x3) - c| <= 3 * 2^-16 * sum_j |J_ij| (up to higher-order terms),
    # and the error is not zero: the splits are really applied
    n = 300
    J = synth.sk_dense(n, seed=5).astype(np.float64)
    rng = np.random.default_rng(3)
    for _ in range(3):
        th = rng.uniform(0, TWO_PI, n)
        exact = (J * np.sin(th[:, None] - th[None, :])).sum(axis=1)
        got = orc.coupling_dense_bf16x3(J, th)
        bound = 3.01 * 2.0 ** -16 * np.abs(J).sum(axis=1)
        err = np.abs(got - exact)
        assert np.all(err <= bound + 1e-13)
        assert err.max() > 1e-4 * bound.max()


def test_integrator_without_coupling_equals_fp64(orc):
    # with K = 0 the coupling form cannot matter: both precisions give the
    # same trajectory bit for bit
    n, R, steps = 40, 3, 30
    J = synth.sk_dense(n, seed=2).astype(np.float64)
    th0 = synth.theta0(R, n, seed=4)
    sd = synth.seeds(R, 9)
    z = np.zeros(steps)
    Ks = synth.ramp(0.0, 20.0, steps)
    sg = synth.const(0.3, steps)
    a = orc.run_dense(J, th0, q=2, dt=0.01, K=z, Ks=Ks, sigma=sg, seeds=sd, step0=11)
    b = orc.run_dense(J, th0, q=2, dt=0.01, K=z, Ks=Ks, sigma=sg, seeds=sd, step0=11,
                      precision="bf16x3")
    assert np.array_equal(a, b)


def test_bf16x3_trajectory_close_to_fp64(orc):
    # with coupling, one step moves each phase by dt K (c_bf16x3 - c) more
    # than the FP64 step: within dt K 3 * 2^-16 * max row sum
    n, R = 64, 2
    J = synth.sk_dense(n, seed=6).astype(np.float64)
    th0 = synth.theta0(R, n, seed=8)
    sd = synth.seeds(R, 1)
    K = np.array([3.0])
    kw = dict(q=2, dt=0.01, K=K, Ks=np.array([1.0]), sigma=np.array([0.1]), seeds=sd)
    a = orc.run_dense(J, th0, **kw)
    b = orc.run_dense(J, th0, precision="bf16x3", **kw)
    d = np.mod(a - b, TWO_PI)
    d = np.minimum(d, TWO_PI - d)
    bound = 0.01 * 3.0 * 3.01 * 2.0 ** -16 * np.abs(J).sum(axis=1).max()
    assert 0 < d.max() <= bound + 1e-15


def test_threaded_rows_match_serial(orc):
    # one replica over several threads (rows split, barriers between the
    # split of the phases, the coupling and the update) equals one thread
    n, steps = 50, 12
    J = synth.sk_dense(n, seed=7).astype(np.float64)
    th0 = synth.theta0(1, n, seed=1)
    kw = dict(q=3, dt=0.01, K=synth.ramp(0, 5, steps), Ks=synth.ramp(0, 8, steps),
              sigma=synth.const(0.2, steps), seeds=synth.seeds(1, 3), precision="bf16x3")
    a = orc.run_dense(J, th0, nthreads=1, **kw)
    b = orc.run_dense(J, th0, nthreads=4, **kw)
    assert np.array_equal(a, b)
