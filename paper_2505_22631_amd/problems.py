"""Mapping combinatorial problems onto the Ising/Potts coupling J (Sec. II-C).

  max-cut with edge weights w   ->  J = -w, q = 2        (spins: phases 0 / pi)
  graph colouring with q colours ->  J = -1 on each edge  (colours: 2 pi k / q)

The cut, conflict and energy readouts themselves run on the device
(oim_cut, oim_conflicts, oim_energy).
"""
from __future__ import annotations

import numpy as np


def maxcut_coupling(row_ptr, col, w):
    """CSR of J = -w for a max-cut instance given as a symmetric weighted CSR."""
    return (np.asarray(row_ptr, np.int64), np.asarray(col, np.int32),
            (-np.asarray(w, np.float64)).astype(np.float32))


def colouring_coupling(row_ptr, col):
    """CSR of J = -1 on every edge of a symmetric adjacency CSR."""
    col = np.asarray(col, np.int32)
    return np.asarray(row_ptr, np.int64), col, np.full(col.shape, -1.0, np.float32)


# ------------------------------------------------------ instance files ----
# Readers for the two text formats of the paper's benchmark sets (Sec. IV):
# the max-cut graphs of Table 1 come as weighted edge lists ("n m" header,
# then "i j w" lines, vertices numbered from 1), the colouring graphs of
# Table 2 in the DIMACS graph format ("c" comments, one "p edge n m" line,
# then "e i j" lines, vertices numbered from 1).  Both return the symmetric
# CSR (each edge stored in both rows, columns sorted) that the problem
# constructors take.  The instance files themselves are not shipped.

def csr_from_edge_list(n, ei, ej, w, *, merge_duplicates=False):
    """Symmetric CSR (row_ptr int64, col int32, w float32) of an undirected
    edge list given with 0-based endpoints.  Self loops are rejected; a pair
    listed more than once is an error unless merge_duplicates, which keeps one
    copy when all copies carry the same weight."""
    n = int(n)
    ei = np.asarray(ei, np.int64).ravel()
    ej = np.asarray(ej, np.int64).ravel()
    w = np.asarray(w, np.float64).ravel()
    if not (ei.shape == ej.shape == w.shape):
        raise ValueError("edge arrays differ in length")
    if n < 1:
        raise ValueError("a graph needs at least one vertex")
    if ei.size and (min(ei.min(), ej.min()) < 0 or max(ei.max(), ej.max()) >= n):
        raise ValueError("edge endpoint out of range")
    if np.any(ei == ej):
        k = int(np.flatnonzero(ei == ej)[0])
        raise ValueError(f"self loop at vertex {int(ei[k]) + 1}")
    if not np.all(np.isfinite(w)):
        raise ValueError("non-finite edge weight")
    lo, hi = np.minimum(ei, ej), np.maximum(ei, ej)
    order = np.lexsort((hi, lo))
    lo, hi, w = lo[order], hi[order], w[order]
    dup = (lo[1:] == lo[:-1]) & (hi[1:] == hi[:-1]) if lo.size > 1 else np.zeros(0, bool)
    if np.any(dup):
        k = int(np.flatnonzero(dup)[0])
        if not merge_duplicates:
            raise ValueError(f"edge ({int(lo[k]) + 1}, {int(hi[k]) + 1}) listed twice")
        if np.any(w[1:][dup] != w[:-1][dup]):
            raise ValueError(f"edge ({int(lo[k]) + 1}, {int(hi[k]) + 1}) listed with "
                             "different weights")
        keep = np.concatenate([[True], ~dup])
        lo, hi, w = lo[keep], hi[keep], w[keep]
    rows = np.concatenate([lo, hi])
    cols = np.concatenate([hi, lo])
    vals = np.concatenate([w, w])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr), cols.astype(np.int32), vals.astype(np.float32)


def _lines(source):
    if hasattr(source, "read"):
        yield from enumerate(source, 1)
        return
    with open(source, "r", encoding="ascii") as fh:
        yield from enumerate(fh, 1)


def read_gset(source):
    """Weighted edge-list file (the Table 1 max-cut format).  Returns
    (n, row_ptr, col, w) with the edge weights w (not couplings; see
    maxcut_coupling)."""
    n = m = None
    ei, ej, w = [], [], []
    for ln, line in _lines(source):
        f = line.split()
        if not f:
            continue
        if n is None:
            if len(f) != 2:
                raise ValueError(f"line {ln}: expected the header 'n m'")
            n, m = int(f[0]), int(f[1])
            if n < 1 or m < 0:
                raise ValueError(f"line {ln}: bad header {n} {m}")
            continue
        if len(f) != 3:
            raise ValueError(f"line {ln}: expected 'i j w'")
        i, j = int(f[0]), int(f[1])
        if not (1 <= i <= n and 1 <= j <= n):
            raise ValueError(f"line {ln}: vertex out of range 1..{n}")
        ei.append(i - 1)
        ej.append(j - 1)
        w.append(float(f[2]))
    if n is None:
        raise ValueError("empty file")
    if len(ei) != m:
        raise ValueError(f"header announces {m} edges, file has {len(ei)}")
    row_ptr, col, wv = csr_from_edge_list(n, ei, ej, w)
    return n, row_ptr, col, wv


def read_dimacs_col(source):
    """DIMACS graph file (the Table 2 colouring format).  Edges listed in both
    directions or repeated are merged.  Returns (n, row_ptr, col)."""
    n = m = None
    ei, ej = [], []
    for ln, line in _lines(source):
        f = line.split()
        if not f or f[0] == "c":
            continue
        if f[0] == "p":
            if n is not None or len(f) != 4 or f[1] not in ("edge", "edges", "col"):
                raise ValueError(f"line {ln}: expected one 'p edge n m' line")
            n, m = int(f[2]), int(f[3])
            if n < 1 or m < 0:
                raise ValueError(f"line {ln}: bad problem line")
            continue
        if f[0] == "e":
            if n is None:
                raise ValueError(f"line {ln}: edge before the 'p' line")
            if len(f) != 3:
                raise ValueError(f"line {ln}: expected 'e i j'")
            i, j = int(f[1]), int(f[2])
            if not (1 <= i <= n and 1 <= j <= n):
                raise ValueError(f"line {ln}: vertex out of range 1..{n}")
            ei.append(i - 1)
            ej.append(j - 1)
            continue
        raise ValueError(f"line {ln}: unknown line type {f[0]!r}")
    if n is None:
        raise ValueError("no 'p edge n m' line")
    if len(ei) != m:
        raise ValueError(f"problem line announces {m} edges, file has {len(ei)}")
    row_ptr, col, _ = csr_from_edge_list(n, ei, ej, np.ones(len(ei)), merge_duplicates=True)
    return n, row_ptr, col


def write_gset(path, n, ei, ej, w):
    """Write an edge list (0-based endpoints) in the Table 1 format."""
    ei, ej, w = np.asarray(ei), np.asarray(ej), np.asarray(w)
    with open(path, "w", encoding="ascii") as fh:
        fh.write(f"{int(n)} {len(ei)}\n")
        for a, b, c in zip(ei.tolist(), ej.tolist(), w.tolist()):
            fh.write(f"{a + 1} {b + 1} {int(c) if float(c).is_integer() else repr(c)}\n")


def write_dimacs_col(path, n, ei, ej, comment=None):
    """Write an edge list (0-based endpoints) in the DIMACS graph format."""
    ei, ej = np.asarray(ei), np.asarray(ej)
    with open(path, "w", encoding="ascii") as fh:
        if comment:
            for c in str(comment).splitlines():
                fh.write(f"c {c}\n")
        fh.write(f"p edge {int(n)} {len(ei)}\n")
        for a, b in zip(ei.tolist(), ej.tolist()):
            fh.write(f"e {a + 1} {b + 1}\n")
