"""Pins of the two-stage CPTR scheme with unknown-based system AMG on the
elliptic block B_ee (Sec. "Two-stage Constrained Pressure-Temperature
Residual", Algorithm 1; the system-AMG direction of the conclusions):
  * B_ee assembled as one CSR equals the dense (P, T) block of the scaled
    matrix;
  * with the P-T couplings removed, the system hierarchy is the two scalar
    hierarchies side by side (block-diagonal levels, the scalar C/F splits);
  * the system V-cycle on an SPD system is symmetric (Jacobi smoothing, R = P^T);
  * with an exact last stage the two-stage apply is exact whatever the
    first stage (Algorithm 1's residual update), so GMRES converges at once;
  * CPTR with AMG converges on the config-2 recipe."""
import numpy as np
import pytest

import oracle as O
from synthetic import config2, tiny


def _dense_ee(dec, ip=0, it=1):
    D = dec.Abar.to_dense()
    n, b = dec.Abar.n, dec.Abar.b
    idx = np.concatenate([np.arange(n) * b + ip, np.arange(n) * b + it])
    return D[np.ix_(idx, idx)]


def test_elliptic_system_assembly():
    s = tiny(9, 7, 5, peclet=2.0, seed=3)
    dec = O.decouple(O.bsr_of(s), s.rhs, variant=O.CPTR)
    B = O.elliptic_system(dec.Abar)
    assert np.array_equal(B.to_dense(), _dense_ee(dec))
    for i in range(B.nrows):
        row = B.ci[B.rp[i]:B.rp[i + 1]]
        assert np.all(np.diff(row) > 0)


def test_uncoupled_system_equals_scalar_hierarchies():
    s = tiny(40, 30, 6, peclet=1.0, seed=5)
    dec = O.decouple(O.bsr_of(s), s.rhs, variant=O.CPTR)
    n = dec.Abar.n
    B = O.elliptic_system(dec.Abar)
    rows = np.repeat(np.arange(B.nrows), np.diff(B.rp))
    cross = (rows < n) != (B.ci < n)
    Bu = O.CSR(B.nrows, B.ncols, B.rp, B.ci, np.where(cross, 0.0, B.v))
    opts = O.AMGOptions(max_coarse=60)
    hs = O.amg_setup_system(Bu, [n, n], opts)
    hP = O.amg_setup(O.submatrix(Bu, 0, n), opts)
    hT = O.amg_setup(O.submatrix(Bu, n, n), opts)
    depth = min(len(hP.levels), len(hT.levels), len(hs.levels))
    for lvl in range(depth - 1):
        Ls = hs.levels[lvl]
        assert np.array_equal(Ls.cf, np.concatenate([hP.levels[lvl].cf, hT.levels[lvl].cf]))
        mP = hP.levels[lvl].A.nrows
        dense = Ls.P.to_dense()
        ncP = hP.levels[lvl].P.ncols
        assert np.allclose(dense[:mP, :ncP], hP.levels[lvl].P.to_dense(), rtol=0, atol=0)
        assert np.allclose(dense[mP:, ncP:], hT.levels[lvl].P.to_dense(), rtol=0, atol=0)
        assert not dense[:mP, ncP:].any() and not dense[mP:, :ncP].any()


def test_system_vcycle_symmetric_on_spd():
    rng = np.random.default_rng(0)
    n = 30
    # two 1-D Laplacians coupled by a small symmetric diagonal coupling
    import scipy.sparse as sp
    L = sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    C = sp.diags(0.1 * np.ones(n))
    M = sp.bmat([[L, C], [C, 2.0 * L]]).tocsr()
    M.sort_indices()
    A = O.CSR(2 * n, 2 * n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(float))
    h = O.amg_setup_system(A, [n, n], O.AMGOptions(max_coarse=8))
    assert len(h.levels) > 1
    x, y = rng.standard_normal(2 * n), rng.standard_normal(2 * n)
    assert abs(x @ O.vcycle(h, y) - y @ O.vcycle(h, x)) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(y)


def test_two_stage_exact_with_exact_last_stage():
    s = tiny(8, 6, 4, peclet=1.0, seed=2)
    opts = O.Options(variant=O.CPTR, amg=O.AMGOptions(max_coarse=20), exact_last_stage=True, restart=10)
    res = O.solve(s, opts)
    assert res.converged and res.iterations <= 2
    assert len(res.hierarchies["ee"].levels) > 1


def test_cptr_amg_converges_config2():
    s = config2(1)
    res = O.solve(s, O.Options(variant=O.CPTR, color=O.tile_colors(s.nx, s.ny), restart=30))
    assert res.converged and res.iterations < 60
    print("config2-1 CPTR-AMG iterations", res.iterations, "levels", res.hierarchies["ee"].sizes)


def test_two_stage_exact_subsolve_uncoupled_upwind():
    """Exact B_ee solve (the paper's M_ee = B_ee) + zero cross coupling + flow
    only toward +x/+y: the stage-1 residual vanishes on (P, T), the
    composition rows are lower triangular in the natural order so ILU(0) is
    exact on them, and M^{-1} = Abar^{-1}: GMRES converges in one step."""
    s = tiny(6, 5, 5, seed=4, zero_coupling=True)
    r = O.solve(s, O.Options(color=np.arange(30), variant=O.CPTR, exact_subsolves=True))
    assert r.iterations == 1 and r.rel_res_scaled <= 1e-12


def test_two_stage_single_level_amg_is_the_exact_subsolve():
    """A system hierarchy with a single level applies B_ee^{-1} (dense LU of
    the coarsest level), so it reproduces the exact sub-solve variant."""
    s = tiny(12, 9, 4, peclet=3.0, seed=8)
    base = dict(color=O.tile_colors(12, 9, 4, 3), variant=O.CPTR, restart=40)
    a = O.solve(s, O.Options(exact_subsolves=True, **base))
    b = O.solve(s, O.Options(amg=O.AMGOptions(max_coarse=10000), **base))
    assert len(b.hierarchies["ee"].levels) == 1
    assert a.iterations == b.iterations
    assert np.linalg.norm(a.x - b.x) <= 1e-12 * np.linalg.norm(a.x)
