"""Pins for the last stage (ilu(Abar), block Jacobi), the multi-stage
composition (Eq. multistageprec vs Algorithms 1/2) and the Krylov driver, plus
the one-iteration invariants of stages made exact (the paper's exact
sub-solver study, Eqs. for M_PP, M_TT, M_ee with direct solves)."""
import numpy as np
import pytest

import oracle as O
from synthetic import tiny, config1


def _rows(A):
    return np.repeat(np.arange(A.n), np.diff(A.rp))


def _lu_product(ilu):
    """Dense L and U of the block factorisation in the elimination order."""
    A, F, rank = ilu.A, ilu.F, ilu.rank
    n, b = A.n, A.b
    L = np.eye(n * b)
    U = np.zeros((n * b, n * b))
    rows = _rows(A)
    for e in range(len(A.ci)):
        i, j = rows[e], A.ci[e]
        blk = F[e]
        if rank[j] < rank[i]:
            L[i * b:(i + 1) * b, j * b:(j + 1) * b] = blk
        else:
            U[i * b:(i + 1) * b, j * b:(j + 1) * b] = blk
    return L, U


@pytest.mark.parametrize("order", ["natural", "redblack", "tiles"])
def test_bilu0_defining_property(order):
    """ILU(0): (L U)_IJ = Abar_IJ on every stored block (any elimination order)."""
    s = tiny(7, 5, 4, seed=3)
    dec = O.decouple(O.bsr_of(s), s.rhs)
    color = {"natural": np.arange(s.n), "redblack": s.checkerboard(),
             "tiles": O.tile_colors(7, 5, 3, 2)}[order]
    ilu = O.BlockILU0(dec.Abar, O.rank_from_colors(color))
    L, U = _lu_product(ilu)
    LU = L @ U
    Ad = dec.Abar.to_dense()
    rows = _rows(dec.Abar)
    b = 4
    for e in range(len(dec.Abar.ci)):
        i, j = rows[e], dec.Abar.ci[e]
        assert np.allclose(LU[i * b:(i + 1) * b, j * b:(j + 1) * b], Ad[i * b:(i + 1) * b, j * b:(j + 1) * b],
                           atol=1e-12 * np.abs(Ad).max())
    # the apply solves with L U
    u = np.random.default_rng(1).standard_normal(s.n * b)
    assert np.allclose(ilu(u), np.linalg.solve(LU, u), rtol=1e-10, atol=1e-12)


def test_bilu0_five_point_changes_only_diagonal_blocks():
    """On the 5-point pattern (a triangle-free graph) zero fill means only the
    diagonal blocks are modified: U's off-diagonal blocks are Abar's, L's are
    Abar_ik U_kk^{-1}."""
    s = tiny(6, 6, 3, seed=2)
    dec = O.decouple(O.bsr_of(s), s.rhs)
    rank = O.rank_from_colors(O.tile_colors(6, 6, 4, 4))
    ilu = O.BlockILU0(dec.Abar, rank)
    rows = _rows(dec.Abar)
    for e in range(len(dec.Abar.ci)):
        i, k = rows[e], dec.Abar.ci[e]
        if rank[k] > rank[i]:
            assert np.array_equal(ilu.F[e], dec.Abar.vals[e])
        elif rank[k] < rank[i]:
            assert np.allclose(ilu.F[e], dec.Abar.vals[e] @ ilu.dinv[k], atol=1e-14)


def test_natural_bilu0_exact_on_a_line():
    """ny = 1: Abar is block tridiagonal and natural-order BILU(0) is its exact
    block LU factorisation."""
    s = tiny(12, 1, 5, seed=4)
    dec = O.decouple(O.bsr_of(s), s.rhs)
    ilu = O.BlockILU0(dec.Abar, O.rank_from_colors(np.arange(12)))
    x = ilu(dec.rhsbar)
    assert np.allclose(x, np.linalg.solve(dec.Abar.to_dense(), dec.rhsbar), rtol=1e-11, atol=1e-13)


def test_block_jacobi_inverse():
    s = tiny(4, 4, 6, seed=1)
    A = O.bsr_of(s)
    bj = O.BlockJacobi(A)
    rows = _rows(A)
    D = A.vals[rows == A.ci]
    assert np.allclose(bj.dinv, np.linalg.inv(D), rtol=1e-12, atol=1e-14)


def test_multistage_formula_equals_algorithms():
    """Eq. multistageprec == Algorithm 2 (three stages) and Algorithm 1 (two);
    error propagation I - Abar M^{-1} = prod (I - Abar M_j^{-1})."""
    s = tiny(3, 3, 3, seed=8)
    dec = O.decouple(O.bsr_of(s), s.rhs)
    Ab = dec.Abar.to_dense()
    N = Ab.shape[0]
    rng = np.random.default_rng(0)
    Ms = [rng.standard_normal((N, N)) * 0.1 for _ in range(3)]
    I = np.eye(N)
    Minv = Ms[0] + Ms[1] @ (I - Ab @ Ms[0]) + Ms[2] @ (I - Ab @ Ms[1]) @ (I - Ab @ Ms[0])
    r = rng.standard_normal(N)
    ops = [lambda v, M=M: M @ v for M in Ms]
    y_alg2 = O.multistage_apply_alg2(dec.Abar, *ops, r)
    y_gen = O.multistage_apply(dec.Abar, ops, r)
    assert np.allclose(y_alg2, Minv @ r, rtol=1e-12, atol=1e-13)
    assert np.allclose(y_gen, Minv @ r, rtol=1e-12, atol=1e-13)
    E = I - Ab @ Minv
    assert np.allclose(E, (I - Ab @ Ms[2]) @ (I - Ab @ Ms[1]) @ (I - Ab @ Ms[0]), atol=1e-12)
    Minv2 = Ms[0] + Ms[1] @ (I - Ab @ Ms[0])
    assert np.allclose(O.multistage_apply(dec.Abar, ops[:2], r), Minv2 @ r, atol=1e-13)


def test_gmres_iterate_is_krylov_least_squares():
    """Without restart the k-th iterate minimises |b - A x| over
    x in M^{-1} K_k(A M^{-1}, b) (right preconditioning)."""
    s = tiny(4, 3, 3, seed=5)
    dec = O.decouple(O.bsr_of(s), s.rhs)
    A = dec.Abar.to_dense()
    N = A.shape[0]
    rng = np.random.default_rng(2)
    Minv = np.linalg.inv(A + 0.3 * np.diag(np.abs(np.diag(A))) * rng.uniform(0.5, 1.5, N))
    b = dec.rhsbar
    for k in range(1, 7):
        res = O.gmres(lambda v: A @ v, b, lambda v: Minv @ v, restart=30, rtol=1e-30, max_iters=k)
        K = np.zeros((N, k))
        v = b.copy()
        for j in range(k):
            K[:, j] = v
            v = A @ (Minv @ v)
        c, *_ = np.linalg.lstsq(A @ Minv @ K, b, rcond=None)
        x_ls = Minv @ K @ c
        assert res.iterations == k
        assert np.allclose(res.x, x_ls, rtol=1e-8, atol=1e-10 * np.abs(x_ls).max())


def test_gmres_monotone_and_finite_termination():
    s = tiny(3, 3, 3, seed=6)
    dec = O.decouple(O.bsr_of(s), s.rhs)
    A = dec.Abar.to_dense()
    res = O.gmres(lambda v: A @ v, dec.rhsbar, lambda v: v, restart=100, rtol=1e-10, max_iters=100)
    h = np.array(res.history)
    assert np.all(np.diff(h) <= 1e-14)
    assert res.converged and res.iterations <= A.shape[0]
    # restarted (GMRES(m) may stagnate, but never increases the residual)
    bj = O.BlockJacobi(dec.Abar)
    res = O.gmres(lambda v: A @ v, dec.rhsbar, bj, restart=3, rtol=1e-10, max_iters=60)
    h = np.array(res.history)
    assert res.restarts >= 1 and np.all(np.diff(h) <= 1e-12)


def test_fgmres_equals_gmres_for_a_fixed_preconditioner():
    s = config1()
    o1 = O.Options(color=O.tile_colors(20, 20), amg=O.AMGOptions(max_coarse=40))
    o2 = O.Options(color=O.tile_colors(20, 20), amg=O.AMGOptions(max_coarse=40), krylov=O.FGMRES)
    r1, r2 = O.solve(s, o1), O.solve(s, o2)
    assert r1.iterations == r2.iterations
    assert np.allclose(r1.x, r2.x, rtol=1e-9, atol=1e-12)


def test_solution_close_to_direct_solve():
    s = tiny(8, 6, 6, peclet=1.0, seed=9)
    r = O.solve(s, O.Options(color=O.tile_colors(8, 6, 4, 4), amg=O.AMGOptions(max_coarse=10)))
    x = np.linalg.solve(O.bsr_of(s).to_dense(), s.rhs)
    assert r.converged and r.rel_res_scaled <= 1e-8
    kappa = np.linalg.cond(r.dec.Abar.to_dense())
    assert np.linalg.norm(r.x - x) / np.linalg.norm(x) <= kappa * 1e-8


# --- stages made exact converge in one iteration ---------------------------

def test_one_iteration_exact_last_stage():
    s = tiny(5, 4, 6, seed=1)
    r = O.solve(s, O.Options(exact_last_stage=True, amg=O.AMGOptions(max_coarse=4)))
    assert r.iterations == 1 and r.rel_res_scaled <= 1e-12


def test_one_iteration_natural_bilu_on_a_line():
    s = tiny(16, 1, 6, seed=2)
    r = O.solve(s, O.Options(color=np.arange(16), amg=O.AMGOptions(max_coarse=4)))
    assert r.iterations == 1 and r.rel_res_scaled <= 1e-12


def test_one_iteration_block_diagonal_system():
    s = tiny(6, 5, 4, seed=3, transmissibility=False, flow=False)
    r = O.solve(s, O.Options(color=O.tile_colors(6, 5), amg=O.AMGOptions(max_coarse=4)))
    assert r.iterations == 1 and r.rel_res_scaled <= 1e-12


def test_one_iteration_direct_subsolves_uncoupled_upwind():
    """Exact T and P solves (the paper's exact operators) + zero cross coupling +
    flow only toward +x/+y: the composition rows are lower triangular in the
    natural order, ILU(0) is exact on them, so M^{-1} = Abar^{-1}."""
    s = tiny(6, 5, 5, seed=4, zero_coupling=True)
    r = O.solve(s, O.Options(color=np.arange(30), exact_subsolves=True))
    assert r.iterations == 1 and r.rel_res_scaled <= 1e-12


def test_stage_order_matters_but_both_converge():
    s = tiny(10, 8, 6, peclet=0.3, seed=5)
    base = dict(color=O.tile_colors(10, 8, 4, 4), amg=O.AMGOptions(max_coarse=8))
    a = O.solve(s, O.Options(stage_order=O.T_THEN_P, **base))
    b = O.solve(s, O.Options(stage_order=O.P_THEN_T, **base))
    assert a.converged and b.converged
    assert not np.allclose(a.history[:3], b.history[:3])


def _unscaled_case():
    """A system whose pressure equations lean on a composition unknown inside
    each cell (A_ii[P, c1] = 5 A_ii[c1, c1]): the decoupling's weights are
    large and the unscaled residual runs about 2.4x the scaled one."""
    s = tiny(20, 12, 4, peclet=3.0, seed=7)
    rows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
    diag = np.nonzero(rows == s.col_idx)[0]
    s.vals[diag, 0, 2] = 5.0 * s.vals[diag, 2, 2]
    return s


def test_stop_on_the_unscaled_residual():
    """With stop_unscaled the solve ends only when |b - A x| <= rtol |b| as
    well: at a tolerance the scaled residual meets after k steps while the
    unscaled one does not, the plain test stops at k with the unscaled
    residual above rtol, the unscaled test restarts with a tighter target
    and ends with both residuals below rtol (both checked from x here)."""
    s = _unscaled_case()
    color = O.tile_colors(s.nx, s.ny)
    amg = O.AMGOptions(max_coarse=30)
    base = O.solve(s, O.Options(color=color, restart=30, amg=amg))
    A = O.bsr_of(s)
    for k in (4, 6, 8):
        rtol = base.history[k - 1] * 1.05
        plain = O.solve(s, O.Options(color=color, restart=30, rtol=rtol, amg=amg))
        both = O.solve(s, O.Options(color=color, restart=30, rtol=rtol, amg=amg, stop_unscaled=True))
        ru = lambda x: np.linalg.norm(s.rhs - A.matvec(x)) / np.linalg.norm(s.rhs)  # noqa: E731
        assert plain.iterations == k and ru(plain.x) > rtol
        assert both.converged and both.iterations > k and both.restarts >= 1
        assert ru(both.x) <= rtol and both.rel_res_scaled <= rtol
        assert abs(both.rel_res_unscaled - ru(both.x)) <= 1e-12


def test_large_direct_subsolve_is_exact():
    """Above the dense size the oracle's exact sub-solve is a sparse LU
    (library step): on a 72 x 70 grid operator (5040 rows, non-symmetric
    5-point stencil) its solution satisfies A x = b to rounding and equals
    LAPACK's dense solve."""
    from oracle.core import DIRECT_DENSE_MAX, _Direct
    nx, ny = 72, 70
    n = nx * ny
    assert n > DIRECT_DENSE_MAX
    rng = np.random.default_rng(3)
    M = np.zeros((n, n))
    for y in range(ny):
        for x in range(nx):
            i = x + nx * y
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                if 0 <= x + dx < nx and 0 <= y + dy < ny:
                    M[i, i + dx + nx * dy] = -rng.uniform(0.2, 1.0)
            M[i, i] = -M[i].sum() + rng.uniform(0.01, 0.1)
    rp, ci, v = [0], [], []
    for i in range(n):
        nz = np.nonzero(M[i])[0]
        ci.extend(nz.tolist())
        v.extend(M[i, nz].tolist())
        rp.append(len(ci))
    A = O.CSR(n, n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v))
    b = rng.uniform(-1, 1, n)
    x = _Direct(A)(b)
    assert np.linalg.norm(M @ x - b) <= 1e-12 * np.linalg.norm(b) * np.linalg.norm(M, 1)
    assert np.allclose(x, np.linalg.solve(M, b), rtol=0, atol=1e-10 * np.abs(x).max())
