"""Oracle pins for hierarchy reuse over a sequence of systems and for the
V-cycle convergence factor that judges it."""
import numpy as np
import pytest

import oracle as O
from oracle import core as OC
from synthetic import generator as G


def _poisson_1d(n, shift=0.0):
    rows, cols, vals = [], [], []
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 2.0 + shift), (i + 1, -1.0)):
            if 0 <= j < n:
                rows.append(i); cols.append(j); vals.append(v)
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, np.array(rows) + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return O.CSR(n, n, rp, np.array(cols, np.int32), np.array(vals))


def _temperature_block(seed=0, nx=24, ny=16, b=4):
    s = G.tiny(nx, ny, b, peclet=10.0, seed=seed)
    dec = O.decouple(O.bsr_of(s), s.rhs)
    return dec.Abar.scalar_block(1, 1)


def test_refresh_with_the_same_values_is_the_same_hierarchy():
    A = _temperature_block()
    h = O.amg_setup(A, O.AMGOptions(max_coarse=20))
    assert len(h.levels) >= 3
    hr = O.amg_refresh(h, A)
    assert len(hr.levels) == len(h.levels)
    for L, Lr in zip(h.levels, hr.levels):
        assert np.array_equal(L.A.rp, Lr.A.rp) and np.array_equal(L.A.ci, Lr.A.ci)
        assert np.array_equal(L.A.v, Lr.A.v)
    assert np.array_equal(h.lu, hr.lu)


def test_refresh_coarse_operators_are_galerkin_products_of_the_new_values():
    A = _temperature_block(seed=1)
    h = O.amg_setup(A, O.AMGOptions(max_coarse=20))
    A2 = _temperature_block(seed=2)          # same pattern, other values
    hr = O.amg_refresh(h, A2)
    cur = A2.to_dense()
    for lvl, L in enumerate(hr.levels[:-1]):
        assert L.P is h.levels[lvl].P            # the interpolation is kept
        P = L.P.to_dense()
        cur = P.T @ cur @ P
        nxt = hr.levels[lvl + 1].A.to_dense()
        assert np.allclose(nxt, cur, rtol=1e-12, atol=1e-12 * np.abs(cur).max())


def test_conv_factor_tends_to_the_spectral_radius_of_the_error_propagator():
    """rho is the K-th root of the error reduction of e <- (I - V A) e; for
    many cycles it approaches the spectral radius of I - V A, computed here
    from the dense propagator (V is linear: one V-cycle per unit vector)."""
    A = _poisson_1d(120)
    h = O.amg_setup(A, O.AMGOptions(max_coarse=8, theta=0.25))
    assert len(h.levels) >= 3
    n = A.nrows
    Ad = A.to_dense()
    V = np.column_stack([O.vcycle(h, np.eye(n)[:, j]) for j in range(n)])
    E = np.eye(n) - V @ Ad
    spec = max(abs(np.linalg.eigvals(E)))
    rho_long = O.conv_factor(h, cycles=200)
    assert abs(rho_long - spec) <= 0.02 * spec
    rho10 = O.conv_factor(h, cycles=10)
    assert rho10 <= np.linalg.norm(E, 2) * (1 + 1e-12)
    # the definition on the same start vector, with the dense propagator
    u = OC._splitmix_vec(0, n)
    e0 = (u >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 * 2.0 - 1.0
    eK = np.linalg.matrix_power(E, 10) @ e0
    assert rho10 == pytest.approx((np.linalg.norm(eK) / np.linalg.norm(e0)) ** 0.1, rel=1e-9)


def test_conv_factor_start_vector_is_uniform_in_minus_one_one():
    u = OC._splitmix_vec(0, 100000)
    e = (u >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 * 2.0 - 1.0
    assert e.min() >= -1.0 and e.max() < 1.0
    assert abs(e.mean()) < 0.01 and abs(e.var() - 1.0 / 3.0) < 0.01
    # SplitMix64 published test value: first output for state 0 is 0xE220A8397B1DCDAF
    assert int(O.lib().orc_splitmix64(0, 0)) == 0xE220A8397B1DCDAF


def test_direct_coarse_solve_gives_tiny_rho():
    A = _poisson_1d(30)
    h = O.amg_setup(A, O.AMGOptions(max_coarse=1000))
    assert len(h.levels) == 1
    assert O.conv_factor(h) < 0.05   # only rounding is left after one cycle


def _c5_small(step, perm):
    return G.config5(step, perm, nx=96, ny=48)


def test_sequence_reuse_keeps_or_rebuilds_by_threshold():
    perm = G.config5_field(96, 48)
    s0, s1 = _c5_small(0, perm), _c5_small(1, perm)
    col = O.tile_colors(96, 48)
    base = O.Options(color=col, amg=O.AMGOptions(max_coarse=100))
    r0 = O.solve(s0, base)
    assert r0.converged and r0.reused == {}
    # a generous threshold keeps both refreshed hierarchies
    keep = O.Options(color=col, amg=O.AMGOptions(max_coarse=100), reuse_rho_max=0.99)
    r1 = O.solve(s1, keep, previous=r0)
    assert r1.reused == {"T": True, "P": True}
    assert all(0.0 < v < 0.99 for v in r1.rho.values())
    assert r1.converged
    # a threshold below every factor rebuilds: identical to a fresh solve
    never = O.Options(color=col, amg=O.AMGOptions(max_coarse=100), reuse_rho_max=1e-9)
    r2 = O.solve(s1, never, previous=r0)
    fresh = O.solve(s1, base)
    assert r2.reused == {"T": False, "P": False}
    assert r2.iterations == fresh.iterations
    assert np.array_equal(r2.x, fresh.x)


def test_band_moves_five_cells_per_system():
    perm = G.config5_field(96, 48)
    d = [np.array([_c5_small(s, perm).meta["band"][0]]) for s in range(3)]
    assert [int(v[0]) for v in d] == [24, 29, 34]


def test_rejected_trials_back_off():
    """With every trial rejected, trials happen at systems 1, 3, 6 (skips of
    1, 2, 4 systems after each rejection)."""
    perm = G.config5_field(24, 12)
    opts = O.Options(color=O.tile_colors(24, 12), amg=O.AMGOptions(max_coarse=10), reuse_rho_max=1e-9)
    prev, trials = None, []
    for k in range(8):
        r = O.solve(G.config5(k, perm, nx=24, ny=12), opts, previous=prev)
        if r.rho:
            assert set(r.rho) == {"T", "P"} and not any(r.reused.values())
            trials.append(k)
        prev = r
    assert trials == [1, 3, 6]
    assert prev.reuse_state["T"] == (3, 8)
