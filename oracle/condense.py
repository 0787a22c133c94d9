"""Static condensation of the full Newton system -- CPU FP64 oracle.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.

Sec. "Static-Condensation Strategy", Eq. global (the partitioned system
J [d1; d2] = -[r1; r2]) and Eq. reduced (A d1 = b with the Schur complement
A = J11 - J12 J22^{-1} J21 and b = -r1 + J12 J22^{-1} r2).  J22 is block
diagonal over the cells and J21 is cell-local, so with the per-cell
factors Q_j = J22_jj^{-1} J21_jj and q_j = J22_jj^{-1} r2_j the reduced
system keeps the pattern of J11:
    A_ij = J11_ij - J12_ij Q_j,      b_i = -r1_i + sum_j J12_ij q_j,
and the secondary update follows from the second block row of Eq. global:
    d2_j = J22_jj^{-1} (-r2_j - J21_jj d1_j) = -q_j - Q_j d1_j.
"""
from __future__ import annotations

import numpy as np


def cell_factors(fs):
    """Q_j = J22_jj^{-1} J21_jj and q_j = J22_jj^{-1} r2_j for every cell
    (numpy's LU solve as the per-cell step)."""
    n, n1, n2 = fs.n, fs.n1, fs.n2
    if n2 == 0:
        return np.zeros((n, 0, n1)), np.zeros((n, 0))
    rhs = np.concatenate([fs.J21, fs.r2.reshape(n, n2, 1)], axis=2)       # [n, n2, n1 + 1]
    sol = np.linalg.solve(fs.J22, rhs)
    return sol[:, :, :n1], sol[:, :, n1]


def condense(fs):
    """(A blocks [nnzb, n1, n1], b [n * n1], Q [n, n2, n1], q [n, n2]) of Eq. reduced."""
    Q, q = cell_factors(fs)
    cols = fs.col_idx
    A = fs.J11 - np.einsum("erk,ekc->erc", fs.J12, Q[cols])
    contrib = np.einsum("erk,ek->er", fs.J12, q[cols])                     # J12_ij q_j per block
    rows = np.repeat(np.arange(fs.n), np.diff(fs.row_ptr))
    bsum = np.zeros((fs.n, fs.n1))
    np.add.at(bsum, rows, contrib)
    b = -fs.r1.reshape(fs.n, fs.n1) + bsum
    return A, b.reshape(-1), Q, q


def recover(Q, q, d1):
    """d2_j = -q_j - Q_j d1_j (the second block row of Eq. global)."""
    n, n2, n1 = Q.shape
    return (-q - np.einsum("jkc,jc->jk", Q, d1.reshape(n, n1))).reshape(-1)


def full_dense(fs):
    """The whole of Eq. global as one dense matrix and right-hand side, unknowns
    ordered [d1 (all cells, cell-interleaved); d2 (all cells)] (for tests on
    tiny systems)."""
    n, n1, n2 = fs.n, fs.n1, fs.n2
    N1 = n * n1
    J = np.zeros((N1 + n * n2, N1 + n * n2))
    for i in range(n):
        for e in range(fs.row_ptr[i], fs.row_ptr[i + 1]):
            j = fs.col_idx[e]
            J[i * n1:(i + 1) * n1, j * n1:(j + 1) * n1] = fs.J11[e]
            J[i * n1:(i + 1) * n1, N1 + j * n2:N1 + (j + 1) * n2] = fs.J12[e]
        J[N1 + i * n2:N1 + (i + 1) * n2, i * n1:(i + 1) * n1] = fs.J21[i]
        J[N1 + i * n2:N1 + (i + 1) * n2, N1 + i * n2:N1 + (i + 1) * n2] = fs.J22[i]
    r = np.concatenate([fs.r1, fs.r2])
    return J, r
