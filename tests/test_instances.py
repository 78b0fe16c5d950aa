"""Readers and writers of the instance-file formats (weighted edge lists for
max-cut, DIMACS graphs for colouring): hand-written fixtures, round trips of
synthetic graphs, malformed input, and a read graph solved end to end by the
oracle's brute force."""
import io
import itertools

import numpy as np
import pytest

import synth
from paper_2505_22631_amd import problems as P


def _same_csr(a, b):
    return (np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
            and (len(a) < 3 or np.array_equal(a[2], b[2])))


def test_gset_hand_written():
    # a 4-cycle 1-2-3-4 with a chord 1-3, weights +1 except the chord -1
    text = "4 5\n1 2 1\n2 3 1\n3 4 1\n4 1 1\n1 3 -1\n"
    n, row_ptr, col, w = P.read_gset(io.StringIO(text))
    assert n == 4
    assert row_ptr.tolist() == [0, 3, 5, 8, 10]
    assert col.tolist() == [1, 2, 3, 0, 2, 0, 1, 3, 0, 2]
    assert w.tolist() == [1, -1, 1, 1, 1, -1, 1, 1, 1, 1]


def test_dimacs_hand_written_merges_both_directions():
    text = ("c a triangle plus a pendant vertex\nc second comment\n"
            "p edge 4 5\ne 1 2\ne 2 3\ne 3 1\ne 2 1\ne 4 3\n")
    n, row_ptr, col = P.read_dimacs_col(io.StringIO(text))
    assert n == 4
    assert row_ptr.tolist() == [0, 2, 4, 7, 8]
    assert col.tolist() == [1, 2, 0, 2, 0, 1, 3, 2]


@pytest.mark.parametrize("which", ["torus", "gnp", "real"])
def test_gset_round_trip(tmp_path, which):
    if which == "torus":
        g = synth.torus(6, 7, seed=1)
    elif which == "gnp":
        g = synth.erdos_renyi(40, 0.2, seed=2, signed=True)
    else:
        g = synth.random_small(12, 0.5, seed=3, weights="real")
    ei, ej, w = g.upper_edges()
    path = tmp_path / "g.txt"
    P.write_gset(path, g.n, ei, ej, w)
    n, row_ptr, col, wr = P.read_gset(path)
    assert n == g.n
    assert _same_csr((row_ptr, col, wr), (g.row_ptr, g.col, g.w))


def test_dimacs_round_trip(tmp_path):
    g, _ = synth.planted_colouring(60, 4.6, 3, seed=5)
    ei, ej, _ = g.upper_edges()
    path = tmp_path / "g.col"
    P.write_dimacs_col(path, g.n, ej, ei, comment="planted 3-colourable\nsynthetic")
    n, row_ptr, col = P.read_dimacs_col(path)
    assert n == g.n
    assert _same_csr((row_ptr, col), (g.row_ptr, g.col))


def test_csr_from_edge_list_matches_synth_builder():
    rng = np.random.default_rng(9)
    n = 30
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < 0.3
    ei, ej = iu[keep], ju[keep]
    w = rng.integers(-3, 4, ei.size).astype(np.float64)
    w[w == 0] = 1
    flip = rng.random(ei.size) < 0.5
    a = np.where(flip, ej, ei)
    b = np.where(flip, ei, ej)
    got = P.csr_from_edge_list(n, a, b, w)
    g = synth.csr_from_edges(n, ei, ej, w)
    assert _same_csr(got, (g.row_ptr, g.col, g.w))


@pytest.mark.parametrize("text,msg", [
    ("", "empty"),
    ("3\n1 2 1\n", "header"),
    ("3 2\n1 2 1\n", "announces 2"),
    ("3 1\n1 4 1\n", "out of range"),
    ("3 1\n0 2 1\n", "out of range"),
    ("3 1\n2 2 1\n", "self loop"),
    ("3 2\n1 2 1\n2 1 1\n", "twice"),
    ("3 1\n1 2\n", "expected 'i j w'"),
    ("3 1\n1 2 nan\n", "non-finite"),
])
def test_gset_rejects_malformed(text, msg):
    with pytest.raises(ValueError, match=msg):
        P.read_gset(io.StringIO(text))


@pytest.mark.parametrize("text,msg", [
    ("c only comments\n", "no 'p edge"),
    ("e 1 2\np edge 2 1\n", "before the 'p'"),
    ("p edge 3 1\np edge 3 1\ne 1 2\n", "one 'p edge"),
    ("p edge 3 2\ne 1 2\n", "announces 2"),
    ("p edge 3 1\ne 1 5\n", "out of range"),
    ("p edge 3 1\ne 3 3\n", "self loop"),
    ("p edge 3 1\nx 1 2\n", "unknown line"),
    ("p edge 3 1\ne 1\n", "expected 'e i j'"),
])
def test_dimacs_rejects_malformed(text, msg):
    with pytest.raises(ValueError, match=msg):
        P.read_dimacs_col(io.StringIO(text))


def test_read_gset_solved_by_brute_force(orc):
    # the best cut of a read instance, from the oracle's exact cut readout over
    # every spin assignment, equals a direct count over the file's edge list
    text = "6 8\n1 2 1\n2 3 1\n3 1 1\n3 4 -1\n4 5 1\n5 6 1\n6 4 1\n1 6 1\n"
    n, row_ptr, col, w = P.read_gset(io.StringIO(text))
    rp, c, J = P.maxcut_coupling(row_ptr, col, w)
    edges = [tuple(map(int, l.split())) for l in text.splitlines()[1:]]
    best_direct = best_oracle = None
    for bits in itertools.product([0, 1], repeat=n):
        s = np.array(bits, np.int8)
        direct = sum(wt for a, b, wt in edges if s[a - 1] != s[b - 1])
        via = orc.cut_int(rp, c, J.astype(np.int64), s)
        assert via == direct
        best_direct = direct if best_direct is None else max(best_direct, direct)
        best_oracle = via if best_oracle is None else max(best_oracle, via)
    # two triangles cut 2 each, the +1 edge 1-6 cut, the -1 edge 3-4 uncut
    assert best_oracle == best_direct == 5
