"""Pins of the learned-interpolation oracle (features, network, loss gradient,
Adam step, judge).  Its definitions are this build's, so the pins are
closed forms, special cases and finite differences."""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import learned as L
from synthetic import mlp_init, tiny

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _poisson_1d(n):
    rp = [0]
    ci, v = [], []
    for i in range(n):
        for j, a in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                ci.append(j)
                v.append(a)
        rp.append(len(ci))
    return O.CSR(n, n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v))


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -1e-40]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(L.bf16(x), ref)


def test_features_on_a_1d_poisson_row():
    A = _poisson_1d(9)
    s = O.strength(A, 0.25)
    cf = np.array([1, 0, 1, 0, 1, 0, 1, 0, 1], np.int32)
    P = O.interp_exti(A, s, cf, 4)
    e = L.edge_features(A, s, cf, P)
    assert list(e.frows) == [1, 3, 5, 7]
    # row 3 (interior F point between C points 2 and 4): weights 1/2, 1/2
    q = list(e.frows).index(3)
    a, b = e.start[q], e.start[q + 1]
    assert list(e.fine[a:b]) == [2, 4]
    for x in e.X[a:b]:
        expect = [-0.5, -0.5, 1.0, 0.0, 0.5, 0.0, 0.0, 0.5, 0.0, 1.0, 1.0, 0.5, 0.0, 1.0, 1.0, 0.0]
        assert np.allclose(x, expect, rtol=0, atol=1e-15)
    # row 1: its C neighbour 0 is a boundary point (row sum 1, so f12 = 1/2)
    q = list(e.frows).index(1)
    x0 = e.X[e.start[q]]
    assert e.fine[e.start[q]] == 0 and x0[12] == 0.5


def test_distance_two_edge_path_term():
    """A 2-D 5-point Laplacian with C points on a diagonal pattern: the
    path term of an edge sums a_ik a_kj / (a_ii a_kk) over common neighbours."""
    s = tiny(6, 6, 2, peclet=1.0, seed=1)
    Abar = O.decouple(O.bsr_of(s), s.rhs).Abar.scalar_block(1, 1)
    st = O.strength(Abar, 0.25)
    cf, _ = O.pmis(Abar, st, 0)
    P = O.interp_exti(Abar, st, cf, 0)
    e = L.edge_features(Abar, st, cf, P)
    D = Abar.to_dense()
    for k in range(len(e.row)):
        i, j = e.row[k], e.fine[k]
        path = sum(D[i, m] * D[m, j] / (D[i, i] * D[m, m]) for m in range(Abar.nrows)
                   if m not in (i, j) and D[i, m] != 0 and D[m, j] != 0)
        assert e.X[k, 5] == pytest.approx(path, rel=1e-12, abs=1e-15)
        assert e.X[k, 3] == (0.0 if D[i, j] != 0 else 1.0)


def _setup(seed=3, nx=20, ny=14, b=4):
    s = tiny(nx, ny, b, peclet=5.0, seed=seed)
    A = O.decouple(O.bsr_of(s), s.rhs).Abar.scalar_block(1, 1)
    st = O.strength(A, 0.25)
    cf, _ = O.pmis(A, st, 0)
    P = O.interp_exti(A, st, cf, 4)
    return A, st, cf, P, L.edge_features(A, st, cf, P)


def test_network_wiring_hand_worked():
    """The network's wiring (blob layout, biases, ReLU after each hidden
    layer, BF16 rounding of the input) against a hand-built network whose
    outputs are worked by hand; the blob is filled from raw offsets, not
    through pack/unpack."""
    g = json.load(open(os.path.join(GOLD, "mlp_wiring.json")))
    params = np.zeros(L.NPARAMS)
    for off, v in g["params"].items():
        params[int(off)] = v
    X = np.zeros((len(g["inputs"]), L.NF))
    for e, case in enumerate(g["inputs"]):
        for f, v in case["x"].items():
            X[e, int(f)] = v
    o, _ = L.forward(params, X)
    assert o.tolist() == [c["o"] for c in g["inputs"]]
    o_exact, _ = L.forward(params, X, exact=True)
    assert o_exact[2] == g["inputs"][2]["o_unrounded"]
    assert o_exact[:2].tolist() == [c["o"] for c in g["inputs"][:2]]


def test_zero_last_layer_reproduces_the_classical_weights():
    A, st, cf, P, e = _setup()
    p = L.unpack(mlp_init(0).astype(np.float64))
    p["W3"][:] = 0.0
    p["b3"][:] = 0.0
    o, _ = L.forward(L.pack(p), e.X)
    assert np.all(o == 0.0)
    Pl = L.learned_weights(P, e, L.delta_of(o))
    assert np.array_equal(Pl.v, P.v)


def test_learned_row_sums_equal_the_classical_ones():
    A, st, cf, P, e = _setup()
    p = L.unpack(mlp_init(1).astype(np.float64))
    p["W3"] *= 100.0            # a sizeable correction
    o, _ = L.forward(L.pack(p), e.X)
    d = L.delta_of(o)
    assert np.max(np.abs(d)) > 0.05
    Pl = L.learned_weights(P, e, d)
    for q, i in enumerate(e.frows):
        a, b = P.rp[i], P.rp[i + 1]
        assert Pl.v[a:b].sum() == pytest.approx(P.v[a:b].sum(), rel=1e-12)


def test_learned_hierarchy_keeps_the_classical_coarse_structure():
    """The learned hierarchy differs from the classical one only in the fine
    level's interpolation weights: same levels, the classical C/F split and
    pattern of P_0 with other values and R_0 = P_0^T, the classical C/F splits
    and transfer operators below, and every coarse operator the Galerkin
    product of its own finer level (checked with dense products)."""
    s = tiny(40, 28, 4, peclet=5.0, seed=3)
    A = O.decouple(O.bsr_of(s), s.rhs).Abar.scalar_block(1, 1)
    h = O.amg_setup(A, O.AMGOptions(max_coarse=30))
    assert len(h.levels) >= 3
    p = L.unpack(mlp_init(1).astype(np.float64))
    p["W3"] *= 100.0
    hl = L.learned_hierarchy(L.pack(p), h)
    assert len(hl.levels) == len(h.levels)
    a, b = hl.levels[0], h.levels[0]
    assert a.A is b.A and np.array_equal(a.cf, b.cf)
    assert np.array_equal(a.P.rp, b.P.rp) and np.array_equal(a.P.ci, b.P.ci)
    assert np.max(np.abs(a.P.v - b.P.v)) > 1e-3          # the weights did change
    assert np.array_equal(a.R.to_dense(), a.P.to_dense().T)
    for a, b in zip(hl.levels[1:-1], h.levels[1:-1]):
        assert a.P is b.P and a.R is b.R and np.array_equal(a.cf, b.cf)
    for l in range(len(hl.levels) - 1):
        Lf, Lc = hl.levels[l], hl.levels[l + 1]
        ref = Lf.R.to_dense() @ Lf.A.to_dense() @ Lf.P.to_dense()
        got = Lc.A.to_dense()
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # a zero correction gives the classical hierarchy, value for value
    p["W3"][:] = 0.0
    p["b3"][:] = 0.0
    h0 = L.learned_hierarchy(L.pack(p), h)
    for a, b in zip(h0.levels, h.levels):
        assert np.array_equal(a.A.v, b.A.v) and np.array_equal(a.A.ci, b.A.ci)


def test_gradient_against_finite_differences():
    A, st, cf, P, e = _setup(seed=4, nx=12, ny=10)
    E = L.smooth_vectors(A, K=4, seed=2)
    p = mlp_init(5).astype(np.float64)
    q = L.unpack(p)
    q["W3"] *= 50.0
    q["b1"][:] = 0.05
    p = L.pack(q)
    loss, g = L.loss_and_grad(p, P, e, E, exact=True)
    rng = np.random.default_rng(9)
    idx = np.concatenate([rng.choice(L.NPARAMS, 40, replace=False), [L.NPARAMS - 1]])
    for k in idx:
        h = 1e-6 * max(1.0, abs(p[k]))
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (L.loss_and_grad(pp, P, e, E, exact=True)[0] - L.loss_and_grad(pm, P, e, E, exact=True)[0]) / (2 * h)
        # central differences of an O(1) loss at h = 1e-6 carry ~1e-10 of rounding
        assert abs(fd - g[k]) <= 1e-4 * abs(fd) + 2e-9, (k, fd, g[k])


def test_loss_is_zero_for_exactly_interpolated_vectors():
    """If every smooth vector is interpolated exactly by the weights, the
    loss vanishes: vectors built as e_F = P e_C."""
    A, st, cf, P, e = _setup()
    p = L.unpack(mlp_init(0).astype(np.float64))
    p["W3"][:] = 0.0
    p["b3"][:] = 0.0
    rng = np.random.default_rng(1)
    ec = rng.standard_normal((3, P.ncols))
    E = np.array([P.matvec(v) for v in ec])
    loss, _ = L.loss_and_grad(L.pack(p), P, e, E)
    assert loss < 1e-28


def test_adam_first_step_is_signed_learning_rate():
    opt = L.Adam(lr=1e-3)
    p = np.zeros(5)
    g = np.array([2.0, -3.0, 1e-3, -1e-5, 0.0])
    p1 = opt.step(p, g)
    expect = -1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p1, expect, rtol=1e-12, atol=0)


def test_judge_keeps_classical_when_the_correction_is_zero():
    s = tiny(32, 24, 4, peclet=5.0, seed=2)
    p = L.unpack(mlp_init(0).astype(np.float64))
    p["W3"][:] = 0.0
    p["b3"][:] = 0.0
    opts = O.Options(color=O.tile_colors(32, 24), amg=O.AMGOptions(max_coarse=30), mlp_params=L.pack(p))
    r = O.solve(s, opts)
    assert r.learned["rho_learned"] == r.learned["rho_classical"]
    assert r.learned["used"] is False


def test_judge_on_every_full_build():
    """Every full build of the temperature hierarchy judges the learned
    interpolation, also inside a sequence with reuse on, and the chosen
    hierarchy never has a larger V-cycle convergence factor than the
    classical one: rho_learned < rho_classical when the learned weights are
    used.  The chosen hierarchy equals an explicit learned or classical
    setup.  A refreshed hierarchy kept by the reuse test is not rebuilt and
    not judged again.  The learned hierarchy is the classical one with the
    learned fine-level weights (its coarser levels keep the classical splits
    and transfer operators)."""
    from synthetic import generator as G
    perm = G.config5_field(48, 24)
    systems = [G.config5(k, perm, nx=48, ny=24) for k in range(4)]
    chosen = []
    for scale, seed in ((3.0, 5), (10.0, 1), (0.0, 0)):
        p = L.unpack(mlp_init(seed).astype(np.float64))
        p["W3"] *= scale
        p["b1"][:] = 0.02
        params = L.pack(p)

        def opts(thr):
            return O.Options(color=O.tile_colors(48, 24), amg=O.AMGOptions(max_coarse=30), mlp_params=params,
                             reuse_rho_max=thr)

        # a threshold no refreshed hierarchy meets: every system is rebuilt and judged
        prev = None
        for s in systems:
            r = O.solve(s, opts(1e-9), previous=prev)
            rc, rl = r.learned["rho_classical"], r.learned["rho_learned"]
            assert rc > 0 and rl > 0
            assert r.learned["used"] == (rl < rc)
            if r.learned["used"]:
                assert rl < rc
            chosen.append(r.learned["used"])
            A = r.dec.Abar.scalar_block(1, 1)
            h = O.amg_setup(A, opts(1e-9).amg)
            if r.learned["used"]:
                h = L.learned_hierarchy(params, h)
            got = r.hierarchies["T"]
            assert len(got.levels) == len(h.levels)
            for a, b in zip(got.levels[:-1], h.levels[:-1]):
                assert np.array_equal(a.P.ci, b.P.ci) and np.array_equal(a.P.v, b.P.v)
            assert O.conv_factor(got, opts(1e-9).judge_cycles, 0) == (rl if r.learned["used"] else rc)
            prev = r
        # a threshold every refreshed hierarchy meets: kept, not judged
        r0 = O.solve(systems[0], opts(0.99))
        r1 = O.solve(systems[1], opts(0.99), previous=r0)
        assert r1.reused.get("T") is True and r1.learned == {}
    assert True in chosen and False in chosen      # both outcomes are exercised
