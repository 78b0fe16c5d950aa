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


# ------------------------------------------------------- round, FP32 ties ----
def _fraction_to_f32(x):
    """Correctly rounded (ties to even) FP32 value of an exact rational, for
    normal-range magnitudes."""
    from fractions import Fraction
    if x == 0:
        return 0.0
    sign = -1 if x < 0 else 1
    a = abs(Fraction(x))
    e = a.numerator.bit_length() - a.denominator.bit_length() - 24
    while a / Fraction(2) ** e >= 2**24:
        e += 1
    while a / Fraction(2) ** e < 2**23:
        e -= 1
    m = a / Fraction(2) ** e                       # in [2^23, 2^24)
    mi = m.numerator // m.denominator
    rem = m - mi
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and mi % 2 == 1):
        mi += 1
    return sign * float(Fraction(mi) * Fraction(2) ** e)


@pytest.mark.parametrize("q", [2, 3, 5, 7, 16])
def test_round_fp32_decision_at_constructed_ties(orc, q):
    # Around each half-way phase 2 pi (k - 1/2) / q the FP32 phases are walked
    # one ulp at a time.  The decision is floor of the single-rounded
    # fma(theta, fl32(q / 2 pi), 1/2), evaluated here in exact rational
    # arithmetic; among the walked phases are the constructed ties whose
    # exact value lies below the integer k but rounds to k, which must go up
    # to k (an FP64 evaluation would give k - 1).
    from fractions import Fraction
    scale = np.float32(q / (2 * np.pi))
    ties_seen = 0
    for k in range(-3, 2 * q + 3):
        centre = np.float32(2 * np.pi * (k - 0.5) / q)
        th = [centre]
        for _ in range(40):
            th.append(np.nextafter(th[-1], np.float32(np.inf), dtype=np.float32))
        lo = [centre]
        for _ in range(40):
            lo.append(np.nextafter(lo[-1], np.float32(-np.inf), dtype=np.float32))
        th = np.array(sorted(set(th + lo)), np.float32)
        th = th[np.abs(th) < 2**20]
        got = orc.round_f32(th, q)
        for t, c in zip(th, got):
            exact = Fraction(float(t)) * Fraction(float(scale)) + Fraction(1, 2)
            r = _fraction_to_f32(exact)
            want = int(np.floor(r)) % q
            assert c == want, (q, k, float(t))
            if r == np.floor(r) and exact < r:
                ties_seen += 1
                assert c == int(r) % q       # rounded up to the integer: goes up
    assert ties_seen > 0


# ---------------------------------------------- fixed-order FP64 readouts ----
def test_pairwise_tree_order(orc):
    # [2^53, 1, 1, -2^53]: the tree adds (2^53 + 1) -> 2^53 and (1 - 2^53)
    # exactly, giving 1; left-to-right gives 0; the exact sum is 2
    big = float(2**53)
    v = [big, 1.0, 1.0, -big]
    assert orc.pairwise_tree(v) == 1.0
    assert ((v[0] + v[1]) + v[2]) + v[3] == 0.0
    # zero padding to a power of two: 3 values are ((a + b) + (c + 0))
    assert orc.pairwise_tree([big, 1.0, 3.0]) == big + 4.0
    assert orc.pairwise_tree([]) == 0.0
    assert orc.pairwise_tree([2.5]) == 2.5
    # integers below 2^53 sum exactly in any order
    rng = np.random.default_rng(3)
    x = rng.integers(-10**6, 10**6, size=1001).astype(np.float64)
    assert orc.pairwise_tree(x) == float(x.astype(np.int64).sum())


@pytest.mark.parametrize("weights", ["int", "pm1", "unit"])
def test_fixed_order_readouts_equal_exact_for_integer_weights(orc, weights):
    g = synth.random_small(37, 0.3, seed=11, weights=weights)
    J = -g.w.astype(np.float64)
    rng = np.random.default_rng(5)
    for q in (2, 3):
        col = rng.integers(0, q, size=g.n).astype(np.int8)
        if q == 2:
            assert orc.cut_fixed(g.row_ptr, g.col, J, col) == \
                orc.cut_int(g.row_ptr, g.col, J.astype(np.int64), col)
        assert orc.h_model_fixed(g.row_ptr, g.col, J, q, col) == \
            orc.h_model(g.row_ptr, g.col, J, q, col)
        assert orc.conflicts(g.row_ptr, g.col, J, col) >= 0


def test_fixed_order_readouts_real_weights_within_bound(orc):
    # real weights: the fixed order differs from the correctly rounded sum
    # (math.fsum of the same terms) by at most (rows' depth + tree depth) ulps
    # of the magnitude sum
    import math
    g = synth.random_small(200, 0.2, seed=12, weights="real")
    J = -g.w.astype(np.float64)
    ei, ej, w = g.upper_edges()
    rng = np.random.default_rng(6)
    col = rng.integers(0, 2, size=g.n).astype(np.int8)
    th = rng.uniform(0, 2 * np.pi, size=g.n)
    deg = int(np.diff(g.row_ptr).max())
    gamma = (deg + 9) * 2.0**-53
    terms = {
        "cut": np.where(col[ei] != col[ej], w.astype(np.float64), 0.0),
        "model": np.where(col[ei] == col[ej], w.astype(np.float64), -w.astype(np.float64)),
        "eq6": w.astype(np.float64) * np.cos(th[ei] - th[ej]),
    }
    got = {"cut": orc.cut_fixed(g.row_ptr, g.col, J, col),
           "model": orc.h_model_fixed(g.row_ptr, g.col, J, 2, col),
           "eq6": orc.h_eq6_fixed(g.row_ptr, g.col, J, th)}
    for k, t in terms.items():
        exact = math.fsum(t.tolist())
        assert abs(got[k] - exact) <= gamma * np.abs(t).sum(), k
    # the plain (row-order) oracle functions agree to the same bound
    assert abs(orc.cut_f64(g.row_ptr, g.col, J, col) - got["cut"]) <= 2 * gamma * np.abs(w).sum()
    assert abs(orc.h_eq6(g.row_ptr, g.col, J, th) - got["eq6"]) <= 2 * gamma * np.abs(w).sum()


def test_fixed_order_per_instance(orc):
    gs = [synth.random_small(n, 0.4, seed=20 + n, weights="real") for n in (5, 9, 17)]
    big, off = synth.block_diagonal(gs)
    J = -big.w.astype(np.float64)
    col = (np.arange(big.n) % 2).astype(np.int8)
    per = orc.cut_fixed(big.row_ptr, big.col, J, col, inst_off=off)
    for b, g in enumerate(gs):
        assert per[b] == orc.cut_fixed(g.row_ptr, g.col, -g.w.astype(np.float64),
                                       col[off[b]:off[b + 1]])


# ------------------------------------------------------------ relaxed cut ----
@pytest.mark.parametrize("weights", ["unit", "pm1", "int"])
def test_relaxed_cut_is_the_cut_at_binary_phases(orc, weights):
    # sum_{i<j} w (1 - cos(th_i - th_j)) / 2 at th in {0, pi} counts the cut
    # edges: 1 - cos(pi) = 2 and 1 - cos(0) = 0 exactly in FP64
    rng = np.random.default_rng(8)
    for n, p, seed in [(12, 0.5, 1), (30, 0.2, 2), (64, 0.1, 3)]:
        g = synth.random_small(n, p, seed=seed, weights=weights)
        J = -g.w.astype(np.float64)
        for _ in range(4):
            col = rng.integers(0, 2, size=n).astype(np.int8)
            th = np.pi * col.astype(np.float64)
            assert orc.relaxed_cut(g.row_ptr, g.col, J, th) == \
                orc.cut_int(g.row_ptr, g.col, J.astype(np.int64), col)


def test_relaxed_cut_binary_phases_real_weights_and_replicas(orc):
    g = synth.random_small(40, 0.3, seed=9, weights="real")
    J = -g.w.astype(np.float64)
    rng = np.random.default_rng(9)
    cols = rng.integers(0, 2, size=(3, g.n)).astype(np.int8)
    th = np.pi * cols.astype(np.float64)
    want = sum(orc.cut_f64(g.row_ptr, g.col, J, c) for c in cols)
    assert orc.relaxed_cut(g.row_ptr, g.col, J, th) == pytest.approx(want, rel=1e-13)
    # all phases equal: no edge is cut
    assert orc.relaxed_cut(g.row_ptr, g.col, J, np.full(g.n, 1.3)) == 0.0
