"""Pins of the oracle's thresholding and readouts (Eq. 1, Eq. 2, Eq. 6, the
max-cut and colouring mappings of Sec. II-C) against brute force and closed
forms on small graphs."""
import itertools

import numpy as np
import pytest

import synth


def _all_colourings(n, q):
    """Every colouring with vertex 0 fixed to 0 (global symmetry), as int8."""
    grid = np.array(list(itertools.product(range(q), repeat=n - 1)), dtype=np.int8)
    return np.concatenate([np.zeros((grid.shape[0], 1), np.int8), grid], axis=1)


def _maxcut_bruteforce(orc, g):
    J = (-g.w).astype(np.int64)
    best = None
    for col in _all_colourings(g.n, 2):
        c = orc.cut_int(g.row_ptr, g.col, J, col)
        best = c if best is None else max(best, c)
    return best


@pytest.mark.parametrize("n", [4, 6, 8, 10, 13])
def test_cycle_maxcut_closed_form(orc, n):
    # even cycle: every edge cut (n); odd cycle: n - 1
    assert _maxcut_bruteforce(orc, synth.cycle(n)) == (n if n % 2 == 0 else n - 1)


@pytest.mark.parametrize("n", [3, 4, 5, 8, 11])
def test_complete_graph_maxcut_closed_form(orc, n):
    assert _maxcut_bruteforce(orc, synth.complete(n)) == n * n // 4


@pytest.mark.parametrize("a,b", [(1, 4), (3, 3), (4, 5)])
def test_bipartite_maxcut_is_all_edges(orc, a, b):
    g = synth.complete_bipartite(a, b)
    assert _maxcut_bruteforce(orc, g) == a * b
    col = np.array([0] * a + [1] * b, np.int8)
    assert orc.cut_int(g.row_ptr, g.col, (-g.w).astype(np.int64), col) == g.n_edges


def test_torus_even_maxcut_is_all_edges(orc):
    g = synth.torus(4, 4, 0, signed=False)
    assert _maxcut_bruteforce(orc, g) == 2 * 16 == g.n_edges


def test_petersen_maxcut(orc):
    # the Petersen graph (15 edges, girth 5) has maximum cut 12
    assert _maxcut_bruteforce(orc, synth.petersen()) == 12


def test_cut_matches_quadratic_form_n20(orc):
    # A 20-node random signed graph: the oracle's edge-loop cut equals
    # (W - s^T A s / 2) / 2 from the dense weight matrix, for every one of
    # 2^19 spin vectors at once; and the best of them is the brute-force max.
    g = synth.random_small(20, 0.3, seed=3, weights="int")
    A = np.zeros((20, 20))
    ei, ej, w = g.upper_edges()
    A[ei, ej] = w
    A[ej, ei] = w
    W = w.sum()
    cols = _all_colourings(20, 2)
    s = 1.0 - 2.0 * cols
    cut_qf = (W - np.einsum("ki,ij,kj->k", s, A, s, optimize=True) / 2.0) / 2.0
    best_k = int(np.argmax(cut_qf))
    J = (-g.w).astype(np.int64)
    for k in [best_k, 0, 1, 12345, len(cols) - 1]:
        assert orc.cut_int(g.row_ptr, g.col, J, cols[k]) == int(round(cut_qf[k]))
    # H_Ising (Eq. 1 with J = -w) = W - 2 cut at the same spins
    for k in [best_k, 77]:
        h = orc.h_model(g.row_ptr, g.col, -g.w.astype(np.float64), 2, cols[k])
        assert h == pytest.approx(W - 2 * cut_qf[k], abs=1e-9)


def test_real_weight_cut(orc):
    g = synth.random_small(12, 0.5, seed=4, weights="real")
    col = (np.arange(12) % 2).astype(np.int8)
    ei, ej, w = g.upper_edges()
    want = float(np.sum(w.astype(np.float64) * (col[ei] != col[ej])))
    assert orc.cut_f64(g.row_ptr, g.col, -g.w.astype(np.float64), col) == pytest.approx(want, abs=1e-12)


def _min_conflicts(orc, g, q):
    J = -np.ones(g.nnz)
    return min(orc.conflicts(g.row_ptr, g.col, J, c) for c in _all_colourings(g.n, q))


def test_colouring_closed_forms(orc):
    assert _min_conflicts(orc, synth.complete(4), 3) == 1          # K4 is not 3-colourable
    assert _min_conflicts(orc, synth.petersen(), 3) == 0           # chromatic number 3
    assert _min_conflicts(orc, synth.petersen(), 2) == 3           # 15 - maxcut 12
    assert _min_conflicts(orc, synth.cycle(7), 2) == 1             # odd cycle
    assert _min_conflicts(orc, synth.cycle(7), 3) == 0
    # K_n with q colours: balanced classes, sum C(size, 2)
    n, q = 7, 3
    sizes = [n // q + (1 if k < n % q else 0) for k in range(q)]
    assert _min_conflicts(orc, synth.complete(n), q) == sum(s * (s - 1) // 2 for s in sizes)


def test_planted_colouring_has_zero_conflicts(orc):
    g, col = synth.planted_colouring(300, 4.6, 3, seed=5)
    J = -np.ones(g.nnz)
    assert orc.conflicts(g.row_ptr, g.col, J, col) == 0
    # Eq. 2 with J = -1 counts the same conflicts
    bad = col.copy()
    bad[g.col[g.row_ptr[0]]] = bad[0]
    assert orc.conflicts(g.row_ptr, g.col, J, bad) >= 1
    assert orc.h_model(g.row_ptr, g.col, J, 3, bad) == orc.conflicts(g.row_ptr, g.col, J, bad)


def test_eq6_at_thresholded_phases(orc):
    # Eq. 6 (w = -J) at the stable phases 2 pi k / q: equals Eq. 1 for q = 2
    # and 1.5 * H_Potts + 0.5 * sum_{i<j} J for q = 3 (cos 0 = 1, cos 2pi/3 = -1/2).
    g = synth.random_small(11, 0.5, seed=6, weights="int")
    J = -g.w.astype(np.float64)
    rng = np.random.default_rng(0)
    for q in (2, 3):
        col = rng.integers(0, q, size=11).astype(np.int8)
        th = 2 * np.pi * col / q
        h6 = orc.h_eq6(g.row_ptr, g.col, J, th)
        hm = orc.h_model(g.row_ptr, g.col, J, q, col)
        if q == 2:
            assert h6 == pytest.approx(hm, abs=1e-9)
        else:
            sumJ = J[np.repeat(np.arange(11), np.diff(g.row_ptr)) < g.col].sum()
            assert h6 == pytest.approx(1.5 * hm + 0.5 * sumJ, abs=1e-9)


@pytest.mark.parametrize("q", [2, 3, 4, 5])
def test_round_nearest_stable_phase(orc, q):
    # constructed phases at the stable points 2 pi k / q, perturbed inside the
    # basin, and a wrap-around just below 2 pi
    k = np.arange(q)
    eps = np.array([-0.3, -1e-4, 0.0, 1e-4, 0.3]) * (np.pi / q)
    th = (2 * np.pi * k[:, None] / q + eps[None, :]).astype(np.float32)
    got = orc.round_f32(th, q)
    np.testing.assert_array_equal(got, np.repeat(k, len(eps)).reshape(q, -1))
    assert orc.round_f32(np.array([np.float32(2 * np.pi) - np.float32(1e-6)]), q)[0] == 0
    assert orc.round_f32(np.array([-0.1], np.float32), q)[0] == 0
    assert orc.round_f32(np.array([np.nan, np.inf, 2e6], np.float32), q).tolist() == [-1, -1, -1]


def test_round_matches_float64_away_from_ties(orc):
    rng = np.random.default_rng(1)
    th = rng.uniform(-20, 20, size=200000).astype(np.float32)
    for q in (2, 3, 7):
        x = q * th.astype(np.float64) / (2 * np.pi) + 0.5
        far = np.abs(x - np.round(x)) > 1e-4
        want = np.mod(np.floor(x), q).astype(np.int8)
        got = orc.round_f32(th, q)
        np.testing.assert_array_equal(got[far], want[far])
