"""Pins of the oracle's noise generator: Philox4x32-10 known answers and the
statistics of the Box-Muller normals it feeds (SC'11 Philox; Box & Muller)."""
import os

import numpy as np
import pytest
from scipy import stats

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_philox_known_answers(orc, ctr, key, expect):
    out = orc.philox4x32_10(ctr, key)
    assert [int(x) for x in out] == expect


def test_philox_word_statistics(orc):
    # 4 words per call over 2^15 counters: byte histogram is flat (chi^2) and
    # every bit is balanced.
    words = np.concatenate([orc.philox4x32_10([c, 7, 0, 0], [123, 456]) for c in range(1 << 15)])
    b = words.view(np.uint8)
    hist = np.bincount(b, minlength=256)
    chi2 = stats.chisquare(hist)
    assert chi2.pvalue > 1e-4
    bits = np.unpackbits(b).reshape(-1, 8).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.01)


def test_normals_moments_and_ks(orc):
    z = np.concatenate([orc.normals(seed, 0, 4096, t) for seed in (0, 1, 2**40 + 5) for t in range(40)])
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    assert abs(stats.kurtosis(z, fisher=False) - 3.0) < 0.05
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # 24-bit uniforms: u1 >= 2^-24 bounds |z| by sqrt(2 * 24 ln 2)
    assert np.abs(z).max() <= np.sqrt(-2.0 * np.log(2.0 ** -24)) + 1e-12


def test_box_muller_pair_structure(orc):
    # Within a Box-Muller pair (i = 4m, 4m+1), z0^2 + z1^2 = -2 ln u1 is
    # Exponential(mean 2) and the angle atan2(z1, z0) is uniform; the two
    # pairs of one Philox call (i = 4m.. and 4m+2..) are uncorrelated.
    z = orc.normals(99, 0, 1 << 18, 3).reshape(-1, 4)
    r2 = z[:, 0] ** 2 + z[:, 1] ** 2
    assert stats.kstest(r2, "expon", args=(0, 2.0)).pvalue > 1e-4
    ang = np.arctan2(z[:, 1], z[:, 0])
    assert stats.kstest(ang, "uniform", args=(-np.pi, 2 * np.pi)).pvalue > 1e-4
    assert abs(np.corrcoef(z[:, 0], z[:, 2])[0, 1]) < 0.01
    assert abs(np.corrcoef(z[:, 1], z[:, 3])[0, 1]) < 0.01


def test_normals_match_documented_word_layout(orc):
    # The normal of oscillator i at step t comes from the Philox call with
    # counter (i/4, t, 0, 0) and key (seed lo, seed hi); word pair (x0, x1)
    # for i%4 in {0,1}, (x2, x3) for {2,3}: u1 = ((xa>>8)+1)/2^24, u2 = (xb>>8)/2^24.
    seed, t = (5 << 32) | 17, 11
    for i in range(8):
        x = orc.philox4x32_10([i // 4, t, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
        p = (i // 2) % 2
        u1 = ((int(x[2 * p]) >> 8) + 1) / 2.0**24
        u2 = (int(x[2 * p + 1]) >> 8) / 2.0**24
        rho = np.sqrt(-2 * np.log(u1))
        want = rho * (np.sin if i % 2 else np.cos)(2 * np.pi * u2)
        assert orc.normal(seed, i, t) == pytest.approx(want, abs=1e-14)


def test_noise_streams_distinct(orc):
    a = orc.normals(0, 0, 64, 0)
    assert not np.allclose(a, orc.normals(1, 0, 64, 0))
    assert not np.allclose(a, orc.normals(0, 0, 64, 1))
    assert not np.allclose(a, orc.normals(1 << 32, 0, 64, 0))
    np.testing.assert_array_equal(a, orc.normals(0, 0, 64, 0))
