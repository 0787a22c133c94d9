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


# ---------------------------------------------------------------------------
# well elimination (remark closing Sec. "Static-Condensation Strategy": the
# well unknowns are eliminated exactly by a Schur complement; with one
# perforation per well the reservoir pattern is kept)
# ---------------------------------------------------------------------------
#
# Reading: a well w with nw unknowns perforates one cell c_w, and couples to
# that cell's primary unknowns only: the primary rows of c_w carry a block
# J1w_w (n1 x nw) against the well unknowns, the well's equations a block
# Jw1_w (nw x n1) against c_w's primary unknowns and Jww_w (nw x nw) against
# its own.  With the full system J [d1; d2; dw] = -[r1; r2; rw] and
#   Qw_w = Jww_w^{-1} Jw1_w,   qw_w = Jww_w^{-1} rw_w,
# eliminating dw changes only the diagonal block of c_w and its right-hand
# side:  A_cc -= J1w_w Qw_w,  b_c += J1w_w qw_w  (wells taken in order), and
# the well update follows from the well rows:  dw_w = -qw_w - Qw_w d1_c.


def well_factors(W):
    """Qw [nwells, nw, n1], qw [nwells, nw] (numpy's LU solve per well)."""
    rhs = np.concatenate([W.Jw1, W.rw.reshape(W.count, W.nw, 1)], axis=2)
    sol = np.linalg.solve(W.Jww, rhs)
    n1 = W.Jw1.shape[2]
    return sol[:, :, :n1], sol[:, :, n1]


def eliminate_wells(A, b, row_ptr, col_idx, W):
    """(A', b', Qw, qw): the reduced blocks A [nnzb, n1, n1] and right-hand
    side b [n * n1] with the wells eliminated (copies)."""
    A = np.array(A, dtype=np.float64, copy=True)
    n1 = A.shape[1]
    b = np.array(b, dtype=np.float64, copy=True).reshape(-1, n1)
    Qw, qw = well_factors(W)
    for w in range(W.count):
        c = int(W.cell[w])
        lo, hi = row_ptr[c], row_ptr[c + 1]
        e = lo + int(np.nonzero(col_idx[lo:hi] == c)[0][0])
        A[e] = A[e] - W.J1w[w] @ Qw[w]
        b[c] = b[c] + W.J1w[w] @ qw[w]
    return A, b.reshape(-1), Qw, qw


def recover_wells(W, Qw, qw, d1):
    """dw_w = -qw_w - Qw_w d1_{c_w} (the well rows of the full system)."""
    n1 = Qw.shape[2]
    d1 = d1.reshape(-1, n1)
    return np.concatenate([-qw[w] - Qw[w] @ d1[int(W.cell[w])] for w in range(W.count)]) if W.count else np.zeros(0)


def full_dense_with_wells(fs, W):
    """The whole system with wells as one dense matrix and right-hand side,
    unknowns ordered [d1; d2; dw] (for tests on tiny systems)."""
    J, r = full_dense(fs)
    N = J.shape[0]
    nwt = W.count * W.nw
    Jf = np.zeros((N + nwt, N + nwt))
    Jf[:N, :N] = J
    n1 = fs.n1
    for w in range(W.count):
        c = int(W.cell[w])
        o = N + w * W.nw
        Jf[c * n1:(c + 1) * n1, o:o + W.nw] = W.J1w[w]
        Jf[o:o + W.nw, c * n1:(c + 1) * n1] = W.Jw1[w]
        Jf[o:o + W.nw, o:o + W.nw] = W.Jww[w]
    return Jf, np.concatenate([r, W.rw])
