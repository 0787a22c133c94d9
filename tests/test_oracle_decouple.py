"""Pins for the oracle's left decoupling (Eqs. CPTR31, CPTR32, CPR, CPTR1).

Each check is independent of the per-cell C routine: global dense block
matrices assembled with numpy following the paper's matrix formulas, zero
blocks the construction guarantees, a closed form at b = 3, and invariance of
the solution under left scaling."""
import numpy as np
import pytest

import oracle as O
from synthetic import tiny


def _groups(n, b, ip=0, it=1):
    cells = np.arange(n)
    s = [k for k in range(b) if k not in (ip, it)]
    P = cells * b + ip
    T = cells * b + it
    S = (cells[:, None] * b + np.array(s, dtype=int)[None, :]).reshape(-1) if s else np.zeros(0, int)
    return P, T, S


def _celldiag(M, rows, cols, n, b):
    """Keep only the cell-local entries (row cell == column cell) of a global block."""
    rc = rows // b
    cc = cols // b
    return np.where(rc[:, None] == cc[None, :], M, 0.0)


@pytest.mark.parametrize("b", [3, 6, 8])
def test_cptr3_matches_dense_schur_formulas(b):
    sys_ = tiny(3, 3, b, peclet=2.0, seed=b)
    A = O.bsr_of(sys_)
    dec = O.decouple(A, sys_.rhs, variant=O.CPTR3)
    Ad = A.to_dense()
    n = sys_.n
    P, T, S = _groups(n, b)
    A_PP, A_PT, A_TP, A_TT = Ad[np.ix_(P, P)], Ad[np.ix_(P, T)], Ad[np.ix_(T, P)], Ad[np.ix_(T, T)]
    A_sP, A_sT = Ad[np.ix_(S, P)], Ad[np.ix_(S, T)]
    D_ss = _celldiag(Ad[np.ix_(S, S)], S, S, n, b)
    D_Ps = _celldiag(Ad[np.ix_(P, S)], P, S, n, b)
    D_Ts = _celldiag(Ad[np.ix_(T, S)], T, S, n, b)
    Dssi = np.linalg.inv(D_ss)
    B_PP = A_PP - D_Ps @ Dssi @ A_sP
    B_PT = A_PT - D_Ps @ Dssi @ A_sT
    B_Tp = A_TP - D_Ts @ Dssi @ A_sP
    B_TT = A_TT - D_Ts @ Dssi @ A_sT
    D_Tp = np.diag(np.diag(B_Tp))
    D_PP = np.diag(np.diag(B_PP))
    C_TT = B_TT - D_Tp @ np.linalg.inv(D_PP) @ B_PT
    Z_Tp = B_Tp - D_Tp @ np.linalg.inv(D_PP) @ B_PP
    Abd = dec.Abar.to_dense()
    scale = np.abs(Ad).max()
    assert np.allclose(Abd[np.ix_(P, P)], B_PP, atol=1e-13 * scale, rtol=0)
    assert np.allclose(Abd[np.ix_(P, T)], B_PT, atol=1e-13 * scale, rtol=0)
    assert np.allclose(Abd[np.ix_(T, T)], C_TT, atol=1e-13 * scale, rtol=0)
    assert np.allclose(Abd[np.ix_(T, P)], Z_Tp, atol=1e-13 * scale, rtol=0)
    # s rows untouched
    assert np.array_equal(Abd[S], Ad[S])
    # the scaled rhs is the same left factor applied to b
    assert np.allclose(dec.rhsbar, dec.apply_left(sys_.rhs), atol=1e-14 * np.abs(sys_.rhs).max())


@pytest.mark.parametrize("b", [3, 6, 8])
def test_cptr3_cell_local_zero_blocks(b):
    """By construction of D (remark on diagonal extraction) the cell-local parts of
    Z_Ps, Z_Ts and Z_Tp vanish (to rounding)."""
    sys_ = tiny(5, 4, b, peclet=10.0, seed=7)
    A = O.bsr_of(sys_)
    dec = O.decouple(A, sys_.rhs, variant=O.CPTR3)
    rows = np.repeat(np.arange(sys_.n), np.diff(A.rp))
    diag = dec.Abar.vals[rows == A.ci]
    orig = A.vals[rows == A.ci]
    s = list(range(2, b))
    scale = np.abs(orig).max(axis=(1, 2))
    assert np.all(np.abs(diag[:, 0, s]).max(axis=1) <= 1e-13 * scale)
    assert np.all(np.abs(diag[:, 1, s]).max(axis=1) <= 1e-13 * scale)
    assert np.all(np.abs(diag[:, 1, 0]) <= 1e-13 * scale)


def test_cptr3_closed_form_b3():
    """b = 3: D_ss is 1x1, so w_P = A_ii[P,s] / A_ii[s,s] and w_T = A_ii[T,s] / A_ii[s,s]."""
    sys_ = tiny(4, 3, 3, seed=3)
    A = O.bsr_of(sys_)
    dec = O.decouple(A, sys_.rhs, variant=O.CPTR3)
    rows = np.repeat(np.arange(sys_.n), np.diff(A.rp))
    D = A.vals[rows == A.ci]
    assert np.allclose(dec.wp[:, 2], D[:, 0, 2] / D[:, 2, 2], rtol=1e-15, atol=0)
    assert np.allclose(dec.wt[:, 2], D[:, 1, 2] / D[:, 2, 2], rtol=1e-15, atol=0)
    hp = D[:, 0, 0] - dec.wp[:, 2] * D[:, 2, 0]
    ht = D[:, 1, 0] - dec.wt[:, 2] * D[:, 2, 0]
    assert np.allclose(dec.beta, ht / hp, rtol=1e-14, atol=0)


@pytest.mark.parametrize("variant", [O.CPTR3, O.CPR, O.CPTR])
def test_left_scaling_keeps_the_solution(variant):
    sys_ = tiny(4, 4, 6, peclet=0.5, seed=11)
    A = O.bsr_of(sys_)
    dec = O.decouple(A, sys_.rhs, variant=variant)
    x1 = np.linalg.solve(A.to_dense(), sys_.rhs)
    x2 = np.linalg.solve(dec.Abar.to_dense(), dec.rhsbar)
    assert np.allclose(x1, x2, rtol=1e-10, atol=1e-12 * np.abs(x1).max())
    # N (unscale) inverts N^{-1}
    v = np.random.default_rng(0).standard_normal(sys_.n * 6)
    assert np.allclose(dec.unscale(dec.apply_left(v)), v, atol=1e-12)


def test_cpr_zeroes_pressure_row_against_h():
    """CPR (Eq. CPR): h = s u {T}; the cell-local Z_Ph vanishes."""
    sys_ = tiny(4, 4, 6, seed=5)
    A = O.bsr_of(sys_)
    dec = O.decouple(A, sys_.rhs, variant=O.CPR)
    rows = np.repeat(np.arange(sys_.n), np.diff(A.rp))
    diag = dec.Abar.vals[rows == A.ci]
    scale = np.abs(A.vals).max()
    assert np.abs(diag[:, 0, 1:]).max() <= 1e-13 * scale
    # T and s rows unchanged
    assert np.array_equal(dec.Abar.vals[:, 1:, :], A.vals[:, 1:, :])


def test_cptr_zeroes_elliptic_rows_against_s():
    sys_ = tiny(4, 4, 6, seed=6)
    A = O.bsr_of(sys_)
    dec = O.decouple(A, sys_.rhs, variant=O.CPTR)
    rows = np.repeat(np.arange(sys_.n), np.diff(A.rp))
    diag = dec.Abar.vals[rows == A.ci]
    scale = np.abs(A.vals).max()
    assert np.abs(diag[:, :2, 2:]).max() <= 1e-13 * scale
    assert not np.allclose(diag[:, 1, 0], 0)   # no second scaling in CPTR


def test_singular_ss_block_is_reported():
    sys_ = tiny(3, 3, 4, seed=1)
    A = O.bsr_of(sys_)
    rows = np.repeat(np.arange(sys_.n), np.diff(A.rp))
    e = np.nonzero((rows == 4) & (A.ci == 4))[0][0]
    A.vals[e, 2:, 2:] = 0.0
    with pytest.raises(O.OracleError, match="cell 4"):
        O.decouple(A, sys_.rhs)


def test_peclet_table_value():
    """Eq. pe with the paper's Table table::Pe gives Pe = O(1) (about 1.09)."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "peclet_table.json")))
    pe = g["q_m3_per_day"] * g["rho_kg_per_m3"] * g["c_p_kJ_per_kg_K"] / (g["kappa_kJ_per_m_day_K"] * g["L_m"])
    assert abs(pe - g["pe_expected"]) < g["pe_tolerance"]
    # the generator's rho c_p / K_T follow the same definition: Pe = rho c_p u L / K_T
    s = tiny(10, 4, 3, peclet=3.0)
    m = s.meta
    assert abs(m["rho_cp"] * 1.0 * 10 / m["k_thermal"] - 3.0) < 1e-9
