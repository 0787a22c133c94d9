"""GPU parity of the learned temperature interpolation against the oracle:
edge features (bit for bit), the BF16 matrix-core network, one training step
(loss, gradient, Adam), the learned weights and the V-cycle judge.

Tolerances.  The oracle sums the BF16 products exactly; the matrix cores
accumulate in FP32 (relative error about 2^-24 per addition over 16 or 64
terms) and a first-layer value that lands within that distance of a BF16
rounding boundary rounds the other way (one BF16 step, 2^-8 relative).  Such
flips are rare, so outputs agree to about 1e-6 relative for nearly all edges
and to a few 1e-3 of the output scale for the rare flipped ones; gradients
collect BF16 roundings of the backward products (2^-9 relative each) and
agree to about 1e-2 of their largest entry."""
import numpy as np
import pytest

import oracle as O
from oracle import learned as L
from synthetic import mlp_init, tiny

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1912_04385_amd import cptr  # noqa: E402


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _case(nx=48, ny=40, b=6, seed=3, peclet=0.5, max_coarse=30):
    s = tiny(nx, ny, b, peclet=peclet, seed=seed)
    ref = O.solve(s, O.Options(color=O.tile_colors(nx, ny), amg=O.AMGOptions(max_coarse=max_coarse), max_iters=1))
    h = ref.hierarchies["T"]
    L0 = h.levels[0]
    edges = L.edge_features(L0.A, L0.strong, L0.cf, L0.P)
    return s, ref, L0, edges


def _params(seed=1, scale=100.0):
    p = L.unpack(mlp_init(seed).astype(np.float64))
    p["W3"] *= scale
    p["b1"][:] = 0.02
    return L.pack(p).astype(np.float32)


def test_edge_features_bitwise():
    print("case learned features tiny48x40b6", flush=True)
    s, ref, L0, edges = _case()
    solver = cptr.solver_for(s, amg_max_coarse=30)
    net = cptr.MLP(_params())
    X, _ = net.edges(solver, with_outputs=False)
    net.close()
    solver.close()
    assert X.shape == edges.X.shape
    assert np.array_equal(X, edges.X.astype(np.float32))


def test_network_outputs():
    print("case learned forward", flush=True)
    s, ref, L0, edges = _case()
    p = _params()
    solver = cptr.solver_for(s, amg_max_coarse=30)
    net = cptr.MLP(p)
    X, o = net.edges(solver)
    net.close()
    solver.close()
    ro, _ = L.forward(p.astype(np.float64), X.astype(np.float64))
    d = np.abs(o - ro)
    scale = np.max(np.abs(ro))
    print(f"  edges={len(o)} |o|max={scale:.3e} max diff={d.max():.3e} median={np.median(d):.3e} "
          f"frac>1e-5={np.mean(d > 1e-5 * scale):.4f}", flush=True)
    assert scale > 0.1
    assert d.max() <= 2e-2 * scale
    assert np.median(d) <= 1e-5 * scale
    assert np.mean(d > 1e-4 * scale) < 0.02


def test_training_step():
    print("case learned train step", flush=True)
    s, ref, L0, edges = _case()
    p = _params(seed=2, scale=30.0)
    solver = cptr.solver_for(s, amg_max_coarse=30)
    net = cptr.MLP(p)
    loss = net.train_step(solver, n_vectors=8, seed=5, lr=1e-3)
    g = net.grad()
    p1 = net.params()
    net.close()
    solver.close()
    E = L.smooth_vectors(L0.A, K=8, seed=5)
    rloss, rg = L.loss_and_grad(p.astype(np.float64), L0.P, edges, E)
    gmax = np.max(np.abs(rg))
    print(f"  loss gpu={loss:.10e} oracle={rloss:.10e} |g|max={gmax:.3e} "
          f"max grad diff={np.max(np.abs(g - rg)):.3e}", flush=True)
    assert abs(loss - rloss) <= 1e-4 * rloss
    assert np.max(np.abs(g - rg)) <= 2e-2 * gmax
    # Adam's first step moves every parameter by lr * g / (|g| + eps)
    opt = L.Adam(lr=1e-3)
    rp1 = opt.step(p.astype(np.float64), g.astype(np.float64))
    assert np.allclose(p1, rp1, rtol=0, atol=1e-6)
    big = np.abs(rg) > 0.05 * gmax
    assert np.all(np.sign(p1 - p)[big] == -np.sign(rg)[big])


def test_learned_weights_forced():
    print("case learned weights forced", flush=True)
    s, ref, L0, edges = _case()
    p = _params()
    solver = cptr.Solver(amg_max_coarse=30, t_interp=cptr.INTERP_LEARNED_FORCED)
    solver.load_mlp(p)
    solver.setup(torch.from_numpy(s.row_ptr), torch.from_numpy(s.col_idx), torch.from_numpy(s.vals.reshape(-1)),
                 0, 1, s.nx, s.ny)
    x, res = solver.solve(_t(s.rhs))
    g = solver.amg_level(0, 0)
    solver.close()
    assert res["used_learned"] == 1
    ro, _ = L.forward(p.astype(np.float64), edges.X)
    Pl = L.learned_weights(L0.P, edges, L.delta_of(ro))
    assert np.array_equal(g["prp"], Pl.rp) and np.array_equal(g["pci"], Pl.ci)
    d = np.abs(g["pv"] - Pl.v)
    print(f"  max weight diff={d.max():.3e} max changed={np.max(np.abs(Pl.v - L0.P.v)):.3e}", flush=True)
    assert np.max(np.abs(Pl.v - L0.P.v)) > 1e-2         # the correction is not trivial
    assert d.max() <= 1e-2 * np.max(np.abs(Pl.v))
    assert res["converged"] == 1 and res["rel_res_scaled"] <= 1e-8


def test_judge_against_oracle():
    print("case learned judge", flush=True)
    s = tiny(48, 40, 6, peclet=0.5, seed=3)
    p = _params(seed=3, scale=20.0)
    opts = O.Options(color=O.tile_colors(48, 40), amg=O.AMGOptions(max_coarse=30), mlp_params=p.astype(np.float64))
    ref = O.solve(s, opts)
    solver = cptr.Solver(amg_max_coarse=30, t_interp=cptr.INTERP_LEARNED)
    solver.load_mlp(p)
    solver.setup(torch.from_numpy(s.row_ptr), torch.from_numpy(s.col_idx), torch.from_numpy(s.vals.reshape(-1)),
                 0, 1, s.nx, s.ny)
    x, res = solver.solve(_t(s.rhs))
    solver.close()
    rc, rl = ref.learned["rho_classical"], ref.learned["rho_learned"]
    print(f"  oracle rho classical={rc:.6f} learned={rl:.6f} used={ref.learned['used']}; gpu "
          f"{res['rho_T_classical']:.6f} {res['rho_T_learned']:.6f} used={res['used_learned']}", flush=True)
    assert abs(res["rho_T_classical"] - rc) <= 1e-10 * rc        # classical hierarchy is bit-identical
    assert abs(res["rho_T_learned"] - rl) <= 2e-2 * rl
    if abs(rl - rc) > 0.05 * rc:
        assert res["used_learned"] == int(ref.learned["used"])
    assert res["converged"] == 1 and res["rel_res_scaled"] <= 1e-8


def test_sequence_judged_at_every_build():
    """Within a sequence (update_values with reuse on) the GPU judges the
    learned interpolation at every full build of the temperature hierarchy,
    as the oracle does: both convergence factors are measured on every
    rebuilt system, the classical one bit-identical to the oracle's, and the
    chosen hierarchy never has the larger factor.  A hierarchy kept by the
    reuse test is not judged again."""
    print("case learned judge at every build", flush=True)
    from synthetic import generator as G
    perm = G.config5_field(48, 24)
    systems = [G.config5(k, perm, nx=48, ny=24) for k in range(3)]
    p = _params(seed=1, scale=100.0)
    opts = O.Options(color=O.tile_colors(48, 24), amg=O.AMGOptions(max_coarse=30), mlp_params=p.astype(np.float64),
                     reuse_rho_max=1e-9)
    refs, prev = [], None
    for s in systems:
        prev = O.solve(s, opts, previous=prev)
        refs.append(prev)
    solver = cptr.Solver(amg_max_coarse=30, t_interp=cptr.INTERP_LEARNED, reuse_rho_max=1e-9)
    try:
        solver.load_mlp(p)
        s0 = systems[0]
        solver.setup(torch.from_numpy(s0.row_ptr), torch.from_numpy(s0.col_idx),
                     torch.from_numpy(s0.vals.reshape(-1)), 0, 1, s0.nx, s0.ny)
        for k, (s, ref) in enumerate(zip(systems, refs)):
            if k > 0:
                solver.update_values(torch.from_numpy(s.vals.reshape(-1)))
            x, res = solver.solve(_t(s.rhs))
            print(f"  system {k}: gpu used={res['used_learned']} rho {res['rho_T_classical']:.4f} "
                  f"{res['rho_T_learned']:.4f} its={res['iterations']}; oracle used={ref.learned['used']} "
                  f"its={ref.iterations}", flush=True)
            assert res["converged"] == 1 and res["rel_res_scaled"] <= 1e-8
            rc, rl = ref.learned["rho_classical"], ref.learned["rho_learned"]
            assert rc > 0 and rl > 0
            assert abs(res["rho_T_classical"] - rc) <= 1e-10 * rc
            assert abs(res["rho_T_learned"] - rl) <= 2e-2 * rl
            if res["used_learned"]:
                assert res["rho_T_learned"] < res["rho_T_classical"]
            if abs(rl - rc) > 0.05 * rc:
                assert res["used_learned"] == int(ref.learned["used"])
            if res["used_learned"] == int(ref.learned["used"]):
                assert abs(res["iterations"] - ref.iterations) <= 1
        # a threshold every refreshed hierarchy meets: kept and not judged
        solver.close()
        solver = cptr.Solver(amg_max_coarse=30, t_interp=cptr.INTERP_LEARNED, reuse_rho_max=0.99)
        solver.load_mlp(p)
        solver.setup(torch.from_numpy(s0.row_ptr), torch.from_numpy(s0.col_idx),
                     torch.from_numpy(s0.vals.reshape(-1)), 0, 1, s0.nx, s0.ny)
        _, r0 = solver.solve(_t(s0.rhs))
        solver.update_values(torch.from_numpy(systems[1].vals.reshape(-1)))
        _, r1 = solver.solve(_t(systems[1].rhs))
        assert r1["reused"] & 1
        assert r1["rho_T_classical"] == -1.0 and r1["rho_T_learned"] == -1.0
        assert r1["used_learned"] == r0["used_learned"]
    finally:
        solver.close()


def test_fp32_judge_and_reuse_measure_the_fp32_vcycle():
    """With the FP32 preconditioner the judge and the reuse test measure the
    FP32 V-cycle the solver applies.  The hierarchies are the oracle's (built
    in FP64), only the V-cycle's rounding differs, so the convergence factors
    agree with the oracle's FP64 ones to 1e-4 relative (classical hierarchy,
    reuse trial) and 2e-2 (learned, whose weights come from the BF16
    network), and the decisions follow them."""
    print("case learned judge and reuse trial with the FP32 V-cycle", flush=True)
    from synthetic import generator as G
    perm = G.config5_field(48, 24)
    systems = [G.config5(k, perm, nx=48, ny=24) for k in range(3)]
    p = _params(seed=1, scale=100.0)
    opts = O.Options(color=O.tile_colors(48, 24), amg=O.AMGOptions(max_coarse=30), mlp_params=p.astype(np.float64),
                     reuse_rho_max=1e-9)
    refs, prev = [], None
    for s in systems:
        prev = O.solve(s, opts, previous=prev)
        refs.append(prev)
    solver = cptr.Solver(amg_max_coarse=30, t_interp=cptr.INTERP_LEARNED, reuse_rho_max=1e-9, krylov=cptr.FGMRES,
                         precond_precision=cptr.FP32)
    try:
        solver.load_mlp(p)
        s0 = systems[0]
        solver.setup(torch.from_numpy(s0.row_ptr), torch.from_numpy(s0.col_idx),
                     torch.from_numpy(s0.vals.reshape(-1)), 0, 1, s0.nx, s0.ny)
        trials = 0
        for k, (s, ref) in enumerate(zip(systems, refs)):
            if k > 0:
                solver.update_values(torch.from_numpy(s.vals.reshape(-1)))
            x, res = solver.solve(_t(s.rhs))
            rc, rl = ref.learned["rho_classical"], ref.learned["rho_learned"]
            print(f"  system {k}: gpu rho_T {res['rho_T']:.8f} judge {res['rho_T_classical']:.8f} "
                  f"{res['rho_T_learned']:.8f} used={res['used_learned']}; oracle rho {ref.rho} judge {rc:.8f} "
                  f"{rl:.8f} used={ref.learned['used']}", flush=True)
            assert res["converged"] == 1 and res["rel_res_scaled"] <= 1e-8
            assert abs(res["rho_T_classical"] - rc) <= 1e-4 * rc
            assert abs(res["rho_T_learned"] - rl) <= 2e-2 * rl
            if res["used_learned"]:
                assert res["rho_T_learned"] < res["rho_T_classical"]
            if abs(rl - rc) > 0.05 * rc:
                assert res["used_learned"] == int(ref.learned["used"])
            if "T" in ref.rho:
                trials += 1
                assert abs(res["rho_T"] - ref.rho["T"]) <= 1e-4 * ref.rho["T"]
                assert not (res["reused"] & 1)
            else:
                assert res["rho_T"] == -1.0
        assert trials >= 1
    finally:
        solver.close()
