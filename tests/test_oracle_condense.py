"""Pins of the static-condensation oracle (Sec. "Static-Condensation
Strategy", Eqs. global and reduced) against what the mathematics fixes:
  * the condensed system and the recovered secondary update reproduce the
    solution of the whole Newton system, solved densely;
  * without J12 the reduced system is (J11, -r1) exactly;
  * without secondary unknowns it is (J11, -r1) exactly;
  * one primary and one secondary unknown per cell: the scalar closed form;
  * wells (remark closing the same section): secondary and well unknowns
    eliminated, the reduced solve and both recoveries reproduce the dense
    solution of the whole system with its well rows; wells without coupling
    leave the reduced system unchanged; the scalar closed form of one well;
    two wells in one cell add their Schur terms."""
import numpy as np
import pytest

from oracle import condense as C
from synthetic import FullSystem, Wells, full_system, tiny, wells


def _dense_bsr(row_ptr, col_idx, blocks, n, b):
    M = np.zeros((n * b, n * b))
    for i in range(n):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            j = col_idx[e]
            M[i * b:(i + 1) * b, j * b:(j + 1) * b] = blocks[e]
    return M


@pytest.mark.parametrize("n1,n2", [(3, 2), (2, 4), (6, 3), (8, 1)])
def test_condensed_solution_equals_full_solution(n1, n2):
    base = tiny(5, 4, n1, peclet=1.0, seed=7)
    fs = full_system(base, n2, seed=3, j12_scale=0.2)
    J, r = C.full_dense(fs)
    full = np.linalg.solve(J, -r)
    A, b, Q, q = C.condense(fs)
    d1 = np.linalg.solve(_dense_bsr(fs.row_ptr, fs.col_idx, A, fs.n, n1), b)
    d2 = C.recover(Q, q, d1)
    N1 = fs.n * n1
    assert np.allclose(d1, full[:N1], rtol=0, atol=1e-10 * np.abs(full).max())
    assert np.allclose(d2, full[N1:], rtol=0, atol=1e-10 * np.abs(full).max())


def test_no_coupling_to_secondary_unknowns():
    fs = full_system(tiny(6, 5, 4, seed=2), 3, seed=1)
    fs.J12[:] = 0.0
    A, b, Q, q = C.condense(fs)
    assert np.array_equal(A, fs.J11)
    assert np.array_equal(b, -fs.r1)


def test_no_secondary_unknowns():
    fs = full_system(tiny(6, 5, 4, seed=2), 0, seed=1)
    A, b, Q, q = C.condense(fs)
    assert np.array_equal(A, fs.J11) and np.array_equal(b, -fs.r1)
    assert Q.shape == (fs.n, 0, 4) and C.recover(Q, q, np.ones(fs.n * 4)).shape == (0,)


def test_scalar_closed_form():
    # three cells on a line, one primary and one secondary unknown each
    rng = np.random.default_rng(5)
    row_ptr = np.array([0, 2, 5, 7], np.int32)
    col_idx = np.array([0, 1, 0, 1, 2, 1, 2], np.int32)
    fs = FullSystem(3, 1, 1, 1, row_ptr, col_idx, rng.uniform(1, 2, (7, 1, 1)), rng.uniform(-1, 1, (7, 1, 1)),
                    rng.uniform(-1, 1, (3, 1, 1)), rng.uniform(1, 2, (3, 1, 1)), rng.uniform(-1, 1, 3),
                    rng.uniform(-1, 1, 3))
    A, b, Q, q = C.condense(fs)
    for i in range(fs.n):
        acc = -fs.r1[i]
        for e in range(fs.row_ptr[i], fs.row_ptr[i + 1]):
            j = fs.col_idx[e]
            a12, a21, a22 = fs.J12[e, 0, 0], fs.J21[j, 0, 0], fs.J22[j, 0, 0]
            assert abs(A[e, 0, 0] - (fs.J11[e, 0, 0] - a12 * a21 / a22)) <= 1e-14 * abs(fs.J11[e, 0, 0])
            acc += a12 * fs.r2[j] / a22
        assert abs(b[i] - acc) <= 1e-13 * max(1.0, abs(acc))


@pytest.mark.parametrize("n1,n2,nw,cells", [(3, 2, 2, None), (6, 3, 1, None), (4, 0, 3, [7, 0, 19]),
                                            (8, 1, 2, [5, 5])])
def test_wells_eliminated_solution_equals_full_solution(n1, n2, nw, cells):
    base = tiny(5, 4, n1, peclet=1.0, seed=7)
    fs = full_system(base, n2, seed=3, j12_scale=0.2)
    W = wells(5, 4, n1, nw, cells=cells, seed=2)
    J, r = C.full_dense_with_wells(fs, W)
    full = np.linalg.solve(J, -r)
    A, b, Q, q = C.condense(fs)
    A2, b2, Qw, qw = C.eliminate_wells(A, b, fs.row_ptr, fs.col_idx, W)
    d1 = np.linalg.solve(_dense_bsr(fs.row_ptr, fs.col_idx, A2, fs.n, n1), b2)
    d2 = C.recover(Q, q, d1)
    dw = C.recover_wells(W, Qw, qw, d1)
    N1, N2 = fs.n * n1, fs.n * n2
    tol = 1e-10 * np.abs(full).max()
    assert np.allclose(d1, full[:N1], rtol=0, atol=tol)
    assert np.allclose(d2, full[N1:N1 + N2], rtol=0, atol=tol)
    assert np.allclose(dw, full[N1 + N2:], rtol=0, atol=tol)
    # only the perforated cells' diagonal blocks and right-hand sides change
    rows = np.repeat(np.arange(fs.n), np.diff(fs.row_ptr))
    touched = np.isin(rows, W.cell) & (rows == fs.col_idx)
    assert np.array_equal(A2[~touched], A[~touched]) and not np.array_equal(A2[touched], A[touched])
    cell_of = np.repeat(np.arange(fs.n), n1)
    assert np.array_equal(b2[~np.isin(cell_of, W.cell)], b[~np.isin(cell_of, W.cell)])


def test_wells_without_coupling_change_nothing():
    fs = full_system(tiny(6, 5, 4, seed=2), 2, seed=1)
    A, b, Q, q = C.condense(fs)
    W = wells(6, 5, 4, 2, seed=4)
    W.J1w[:] = 0.0
    A2, b2, Qw, qw = C.eliminate_wells(A, b, fs.row_ptr, fs.col_idx, W)
    assert np.array_equal(A2, A) and np.array_equal(b2, b)
    assert np.allclose(C.recover_wells(W, Qw, qw, np.zeros(fs.n * 4)), -qw.reshape(-1))


def test_one_well_scalar_closed_form():
    """n1 = nw = 1: a_cc' = a_cc - j1w jw1 / jww and b_c' = b_c + j1w rw / jww."""
    row_ptr = np.array([0, 2, 5, 7], np.int32)
    col_idx = np.array([0, 1, 0, 1, 2, 1, 2], np.int32)
    A = np.arange(1.0, 8.0).reshape(7, 1, 1)
    b = np.array([1.0, 2.0, 3.0])
    W = Wells(np.array([1], np.int32), 1, np.array([[[0.5]]]), np.array([[[-2.0]]]), np.array([[[4.0]]]),
              np.array([3.0]))
    A2, b2, Qw, qw = C.eliminate_wells(A, b, row_ptr, col_idx, W)
    assert A2[3, 0, 0] == 4.0 - 0.5 * (-2.0) / 4.0 and b2[1] == 2.0 + 0.5 * 3.0 / 4.0
    assert np.array_equal(np.delete(A2.reshape(-1), 3), np.delete(A.reshape(-1), 3))
    assert C.recover_wells(W, Qw, qw, np.array([0.0, 2.0, 0.0]))[0] == -(3.0 / 4.0) - (-2.0 / 4.0) * 2.0
