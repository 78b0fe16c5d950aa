"""Mapping combinatorial problems onto the Ising/Potts coupling J (Sec. II-C).

  max-cut with edge weights w   ->  J = -w, q = 2        (spins: phases 0 / pi)
  graph colouring with q colours ->  J = -1 on each edge  (colours: 2 pi k / q)

and the readout conversions between the Hamiltonian and the objective:
  cut = (W - H_Ising) / 2 with W = sum_{i<j} w_ij = -sum_{i<j} J_ij
  conflicts = H_Potts for the colouring coupling J = -1.
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


def cut_from_h(h_ising, sum_J_upper):
    """Max-cut value from the Ising energy of the coupling J = -w."""
    return (-sum_J_upper - np.asarray(h_ising)) / 2.0


def accuracy(cut, best):
    """Accuracy in percent as the paper's Table 1 reports it: cut / best-known * 100."""
    return 100.0 * np.asarray(cut, np.float64) / float(best)
