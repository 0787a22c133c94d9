"""Pins for the oracle's AMG sub-solver (the amg(.) of Eqs. CPRM1, CPTR3M1,
CPTRM2): strength on hand-worked rows, PMIS properties by brute force,
extended+i against exact linear interpolation on the 1-D Laplacian, Galerkin
products against dense numpy products, dense coarse solve against LAPACK, and
V-cycle properties (direct solve on one level, symmetry, convergence)."""
import json
import os

import numpy as np
import pytest

import oracle as O
import oracle.core as OC
from synthetic import tiny

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def csr_from_dense(M):
    n, m = M.shape
    rp = [0]
    ci, v = [], []
    for i in range(n):
        for j in range(m):
            if M[i, j] != 0 or i == j:
                ci.append(j); v.append(M[i, j])
        rp.append(len(ci))
    return O.CSR(n, m, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v, float))


def poisson1d(n):
    return 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)


def poisson2d(nx, ny, shift=0.0):
    return np.kron(np.eye(ny), poisson1d(nx)) + np.kron(poisson1d(ny), np.eye(nx)) + shift * np.eye(nx * ny)


def test_strength_hand_worked_rows():
    g = json.load(open(os.path.join(GOLD, "strength_example.json")))
    for row in g["rows"]:
        k = len(row["offdiag"])
        M = np.zeros((k + 1, k + 1))
        M[0, 0] = row["diag"]
        M[0, 1:] = row["offdiag"]
        M[1:, 1:] = np.eye(k)
        A = csr_from_dense(M)
        s = O.strength(A, g["theta"])
        got = [int(s[e]) for e in range(A.rp[0], A.rp[1]) if A.ci[e] != 0]
        assert got == row["strong"]


def _sym_strong(A, s):
    n = A.nrows
    S = np.zeros((n, n), bool)
    rows = np.repeat(np.arange(n), np.diff(A.rp))
    S[rows[s == 1], A.ci[s == 1]] = True
    return S


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pmis_independent_and_maximal(seed):
    """No two C points are strongly connected (either direction); every point
    that something depends on is C or strongly depends on a C point
    (De Sterck, Yang & Heys 2006)."""
    rng = np.random.default_rng(seed)
    M = poisson2d(9, 7) + np.diag(rng.uniform(0, 0.5, 63))
    M[np.abs(M) > 0] *= rng.uniform(0.5, 1.5, M[np.abs(M) > 0].shape)
    A = csr_from_dense(M)
    s = O.strength(A, 0.25)
    cf, rounds = O.pmis(A, s, seed)
    S = _sym_strong(A, s)
    C = cf == 1
    assert not np.any((S | S.T)[np.ix_(C, C)])
    has_dep = S.T.any(axis=1)          # |S^T_i| > 0
    for i in np.nonzero(has_dep & ~C)[0]:
        assert np.any(S[i] & C), f"F point {i} has no strong C dependence"
    assert rounds >= 1


def test_pmis_isolated_points_are_f():
    A = csr_from_dense(np.diag([1.0, 2.0, 3.0]))
    cf, _ = O.pmis(A, O.strength(A, 0.25), 0)
    assert cf.tolist() == [0, 0, 0]


def test_exti_linear_interpolation_1d_poisson():
    g = json.load(open(os.path.join(GOLD, "exti_1d_poisson.json")))
    for case in g["cases"]:
        A = csr_from_dense(poisson1d(case["n"]))
        s = O.strength(A, 0.25)
        cf = np.array(case["cf"], np.int32)
        P = O.interp_exti(A, s, cf, pmax=0).to_dense()
        cidx = np.cumsum(cf) - cf
        for i in range(case["n"]):
            if cf[i]:
                row = np.zeros(P.shape[1]); row[cidx[i]] = 1.0
                assert np.array_equal(P[i], row)
        for i, want in case["rows"].items():
            expect = np.zeros(P.shape[1])
            for c, w in want.items():
                expect[int(c)] = w
            assert np.allclose(P[int(i)], expect, atol=1e-15), (case["cf"], i, P[int(i)])


def test_exti_hand_worked_branches():
    """Every branch of the extended+i formula on one hand-worked matrix: a
    weak neighbour lumped into the diagonal, a positive coupling removed by
    the sign filter abar, a strong F neighbour with d_k = 0 lumped, a
    distance-two C point reached through a strong F neighbour, a weak
    neighbour inside Chat entering the numerator, empty interpolatory sets,
    and the truncation's row-sum rescaling."""
    from fractions import Fraction
    g = json.load(open(os.path.join(GOLD, "exti_branches.json")))
    M = np.array(g["matrix"])
    A = csr_from_dense(M)
    s = O.strength(A, g["theta"])
    for i in range(A.nrows):
        got = [int(A.ci[e]) for e in range(A.rp[i], A.rp[i + 1]) if s[e] and A.ci[e] != i]
        assert got == g["strong"][str(i)], (i, got)
    cf = np.array(g["cf"], np.int32)
    for pmax in (0, 1):
        P = O.interp_exti(A, s, cf, pmax=pmax).to_dense()
        rows = g["P"][f"pmax_{pmax}"]
        fr = g["fractions"][f"pmax_{pmax}"]
        for i, want in rows.items():
            expect = np.zeros(P.shape[1])
            for c, w in want.items():
                expect[int(c)] = w
            if i in fr:          # the decimal values equal the hand-worked fractions
                vals = [float(Fraction(q)) for q in fr[i]]
                assert np.allclose(sorted(vals), sorted(want.values()), rtol=0, atol=0)
            assert np.allclose(P[int(i)], expect, rtol=2e-16, atol=1e-16), (pmax, i, P[int(i)], expect)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exti_preserves_constants_on_zero_row_sums(seed):
    """On rows whose entries sum to exactly zero, extended+i interpolates
    constants exactly: sum_j w_ij = 1 follows from d_k's definition (the
    sum over Chat_i of abar_kj is d_k - abar_ki) and atilde_ii's lumping,
    whatever the signs, the strength pattern and the lumped terms.  Random
    positive and negative couplings on a 2-D pattern, diagonals set to make
    every row sum zero; the truncation with rescaling keeps it."""
    rng = np.random.default_rng(seed)
    nx, ny = 9, 8
    n = nx * ny
    M = np.zeros((n, n))
    for y in range(ny):
        for x in range(nx):
            i = x + nx * y
            for dx, dy in ((1, 0), (0, 1)):
                if x + dx < nx and y + dy < ny:
                    j = (x + dx) + nx * (y + dy)
                    M[i, j] = -rng.uniform(0.1, 2.0)
                    M[j, i] = -rng.uniform(0.1, 2.0)
    for i in range(n):                  # one positive off-diagonal in some rows
        nb = np.flatnonzero(M[i])
        if len(nb) >= 3 and rng.random() < 0.4:
            M[i, rng.choice(nb)] *= -0.05
    np.fill_diagonal(M, 0.0)
    np.fill_diagonal(M, -M.sum(axis=1))
    assert np.all(np.diag(M) > 0)
    A = csr_from_dense(M)
    assert np.max(np.abs([A.v[A.rp[i]:A.rp[i + 1]].sum() for i in range(n)])) < 1e-14
    s = O.strength(A, 0.25)
    cf, _ = O.pmis(A, s, seed)
    for pmax in (0, 4, 2):
        P = O.interp_exti(A, s, cf, pmax=pmax).to_dense()
        nonempty = np.count_nonzero(P, axis=1) > 0
        assert nonempty.sum() > n // 2
        assert np.max(np.abs(P.sum(axis=1)[nonempty] - 1.0)) < 1e-14, pmax


def test_exti_truncation_keeps_pmax_and_row_sum():
    A = csr_from_dense(poisson2d(10, 10, shift=0.1))
    s = O.strength(A, 0.25)
    cf, _ = O.pmis(A, s, 1)
    P0 = O.interp_exti(A, s, cf, pmax=0)
    P2 = O.interp_exti(A, s, cf, pmax=2)
    assert np.diff(P2.rp).max() <= 2
    assert np.allclose(P0.to_dense().sum(axis=1), P2.to_dense().sum(axis=1), atol=1e-14)
    # kept entries are the largest in magnitude of the untruncated row
    D0, D2 = P0.to_dense(), P2.to_dense()
    for i in range(100):
        kept = np.nonzero(D2[i])[0]
        if len(kept) and np.count_nonzero(D0[i]) > 2:
            assert np.abs(D0[i, kept]).min() >= np.sort(np.abs(D0[i]))[-2] - 1e-15


def test_transpose_and_galerkin_against_dense():
    rng = np.random.default_rng(4)
    M = poisson2d(7, 6, shift=0.2) + 0.1 * np.triu(np.tril(rng.standard_normal((42, 42)), 1), -1)
    A = csr_from_dense(M)
    s = O.strength(A, 0.25)
    cf, _ = O.pmis(A, s, 2)
    P = O.interp_exti(A, s, cf, pmax=4)
    R = P.transpose()
    assert np.array_equal(R.to_dense(), P.to_dense().T)
    Ac = O.galerkin(A, P, R)
    dense = P.to_dense().T @ M @ P.to_dense()
    assert np.allclose(Ac.to_dense(), dense, atol=1e-13 * np.abs(dense).max())
    # rows sorted, pattern symmetric
    for i in range(Ac.nrows):
        c = Ac.ci[Ac.rp[i]:Ac.rp[i + 1]]
        assert np.all(np.diff(c) > 0)
    Dp = Ac.to_dense() != 0
    pat = np.zeros_like(Dp)
    rows = np.repeat(np.arange(Ac.nrows), np.diff(Ac.rp))
    pat[rows, Ac.ci] = True
    assert np.array_equal(pat, pat.T)


def test_dense_lu_against_lapack():
    rng = np.random.default_rng(9)
    M = rng.standard_normal((40, 40)) + 5 * np.eye(40)
    f = rng.standard_normal(40)
    h = O.amg_setup(csr_from_dense(M), O.AMGOptions(max_coarse=100))
    assert len(h.levels) == 1
    assert np.allclose(O.coarse_solve(h, f), np.linalg.solve(M, f), rtol=1e-12, atol=1e-13)
    assert np.allclose(O.vcycle(h, f), np.linalg.solve(M, f), rtol=1e-12, atol=1e-13)


def _vcycle_matrix(h, n):
    return np.column_stack([O.vcycle(h, e) for e in np.eye(n)])


def test_vcycle_symmetric_for_spd():
    """Symmetric smoothing (one Jacobi sweep before and after) with R = P^T gives
    a symmetric V-cycle operator on an SPD matrix."""
    M = poisson2d(10, 9, shift=0.05)
    h = O.amg_setup(csr_from_dense(M), O.AMGOptions(max_coarse=10))
    assert len(h.levels) >= 3
    V = _vcycle_matrix(h, 90)
    assert np.allclose(V, V.T, atol=1e-12 * np.abs(V).max())


def test_first_jacobi_sweep_closed_form():
    M = poisson2d(6, 6, shift=0.3)
    A = csr_from_dense(M)
    L = O.Level(A, A.diagonal(), smooth_diag=A.diagonal())
    b = np.arange(36, dtype=float)
    x = O.smooth(L, O.AMGOptions(), b, None, 1)
    assert np.allclose(x, (2 / 3) * b / np.diag(M), rtol=1e-15)


def test_vcycle_converges_on_poisson_and_rho_bounds():
    M = poisson2d(24, 24, shift=0.01)
    h = O.amg_setup(csr_from_dense(M), O.AMGOptions(max_coarse=20))
    rho = O.conv_factor(h, cycles=10)
    assert 0 < rho < 0.5
    V = _vcycle_matrix(h, 576)
    E = np.eye(576) - V @ M
    assert rho <= np.linalg.norm(E, 2) + 1e-12
    # a single level is exact: rho = 0
    h1 = O.amg_setup(csr_from_dense(poisson2d(5, 5, 0.1)), O.AMGOptions(max_coarse=100))
    assert O.conv_factor(h1, cycles=3) < 1e-12


@pytest.mark.parametrize("smoother", [O.SMOOTH_L1JACOBI, O.SMOOTH_CHEBYSHEV])
def test_other_smoothers_converge(smoother):
    M = poisson2d(16, 16, shift=0.01)
    h = O.amg_setup(csr_from_dense(M), O.AMGOptions(max_coarse=20, smoother=smoother))
    assert O.conv_factor(h, cycles=10) < 0.6


def _cheb_level(M):
    A = csr_from_dense(M)
    L = O.Level(A, A.diagonal())
    OC._smoother_setup(L, O.AMGOptions(smoother=O.SMOOTH_CHEBYSHEV))
    return L


def test_chebyshev_gershgorin_bound():
    """lam_max is the Gershgorin bound max_i sum_j |a_ij| / |a_ii| (hand value
    on a 3 x 3 matrix) and bounds the spectrum of D^{-1} A from above."""
    M = np.array([[4.0, -1.0, 0.0], [-2.0, 5.0, -2.0], [0.0, -3.0, 2.0]])
    assert _cheb_level(M).lam_max == 2.5                 # row 2: (3 + 2) / 2
    M = poisson2d(7, 6, shift=0.2)
    L = _cheb_level(M)
    ev = np.linalg.eigvals(M / np.diag(M)[:, None])
    assert np.max(np.abs(ev)) <= L.lam_max * (1 + 1e-14)


@pytest.mark.parametrize("degree", [1, 2, 3, 5])
@pytest.mark.parametrize("zero_start", [True, False])
def test_chebyshev_error_polynomial(degree, zero_start):
    """The error after a degree-k Chebyshev iteration is p_k(D^{-1} A) e_0 with
    p_k(t) = T_k((theta - t) / delta) / T_k(theta / delta) over the interval
    [lam/30, 1.1 lam]; T_k here from the matrix form of the Chebyshev
    polynomials' own recurrence T_{k+1} = 2 Z T_k - T_{k-1}."""
    rng = np.random.default_rng(degree)
    M = poisson2d(6, 5, shift=0.1) + np.diag(rng.uniform(0, 2, 30))
    L = _cheb_level(M)
    b = rng.standard_normal(30)
    x0 = None if zero_start else rng.standard_normal(30)
    xs = np.linalg.solve(M, b)
    x = O.smooth(L, O.AMGOptions(smoother=O.SMOOTH_CHEBYSHEV, cheb_degree=degree), b, x0, 1)
    lo, hi = L.lam_max / 30.0, 1.1 * L.lam_max
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    Z = (theta * np.eye(30) - M / np.diag(M)[:, None]) / delta
    Tm, T = np.eye(30), Z.copy()
    tm, t = 1.0, theta / delta
    for _ in range(degree - 1):
        Tm, T = T, 2 * Z @ T - Tm
        tm, t = t, 2 * (theta / delta) * t - tm
    e0 = xs - (np.zeros(30) if x0 is None else x0)
    assert np.allclose(xs - x, (T / t) @ e0, rtol=0, atol=1e-12 * np.abs(e0).max())


def test_hierarchy_on_generated_temperature_block():
    """The Schur-extracted temperature block of a generated system coarsens and
    its V-cycle converges."""
    s = tiny(24, 16, 6, peclet=1.0, seed=2)
    dec = O.decouple(O.bsr_of(s), s.rhs)
    h = O.amg_setup(dec.Abar.scalar_block(1, 1), O.AMGOptions(max_coarse=30))
    assert len(h.levels) >= 3
    assert h.operator_complexity() < 3.0
    assert O.conv_factor(h) < 0.7
