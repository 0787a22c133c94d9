"""Pins of the static-condensation oracle (Sec. "Static-Condensation
Strategy", Eqs. global and reduced) against what the mathematics fixes:
  * the condensed system and the recovered secondary update reproduce the
    solution of the whole Newton system, solved densely;
  * without J12 the reduced system is (J11, -r1) exactly;
  * without secondary unknowns it is (J11, -r1) exactly;
  * one primary and one secondary unknown per cell: the scalar closed form."""
import numpy as np
import pytest

from oracle import condense as C
from synthetic import FullSystem, full_system, tiny


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
