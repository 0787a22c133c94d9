"""GPU parity of the Chebyshev smoother option of the AMG V-cycle (the
polynomial smoother on D^{-1} A over [lam/30, 1.1 lam], lam the Gershgorin
bound, degree cheb_degree x sweeps), through the C ABI, against the CPU FP64
oracle: the V-cycle itself and its convergence factor at 1e-12 / 1e-10
relative, solves at 1e-10 relative with iterations within one (scalar AMG
stages, the two-stage system AMG, hierarchy reuse over a sequence), and the
FP32 preconditioner reaching the FP64 true-residual tolerance."""
import numpy as np
import pytest

import oracle as O
from synthetic import config1, tiny
from synthetic import generator as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1912_04385_amd import cptr  # noqa: E402

GPU_VARIANT = {O.CPTR3: cptr.VARIANT_CPTR3, O.CPR: cptr.VARIANT_CPR, O.CPTR: cptr.VARIANT_CPTR}


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _amg(max_coarse, degree=2, pre=1, post=1):
    return O.AMGOptions(max_coarse=max_coarse, smoother=O.SMOOTH_CHEBYSHEV, cheb_degree=degree, pre=pre, post=post)


def _gpu(max_coarse, degree=2, pre=1, post=1, **kw):
    return dict(amg_max_coarse=max_coarse, smoother=cptr.SMOOTH_CHEBYSHEV, cheb_degree=degree, pre_sweeps=pre,
                post_sweeps=post, **kw)


@pytest.mark.parametrize("degree,pre,post", [(1, 1, 1), (2, 1, 1), (3, 2, 1), (2, 0, 1), (4, 1, 0)])
def test_chebyshev_vcycle_parity(degree, pre, post):
    print(f"case chebyshev vcycle degree={degree} pre={pre} post={post}", flush=True)
    s = tiny(48, 40, 6, peclet=0.5, seed=3)
    ref = O.solve(s, O.Options(color=O.tile_colors(48, 40), amg=_amg(30, degree, pre, post), max_iters=1))
    solver = cptr.solver_for(s, **_gpu(30, degree, pre, post))
    try:
        rng = np.random.default_rng(7)
        for which, key in ((0, "T"), (1, "P")):
            assert solver.amg_levels(which) == len(ref.hierarchies[key].levels) >= 3
            bvec = rng.standard_normal(s.n)
            x = solver.vcycle(which, _t(bvec)).cpu().numpy()
            xr = O.vcycle(ref.hierarchies[key], bvec)
            err = np.abs(x - xr).max() / np.abs(xr).max()
            print(f"  {key}: levels={solver.amg_levels(which)} max rel diff {err:.2e}", flush=True)
            assert np.allclose(x, xr, rtol=1e-12, atol=1e-12 * np.abs(xr).max())
            rho = solver.conv_factor(which, 10, 0)
            rr = O.conv_factor(ref.hierarchies[key], 10, 0)
            print(f"  {key}: rho gpu {rho:.15f} oracle {rr:.15f}", flush=True)
            assert abs(rho - rr) <= 1e-10 * rr
    finally:
        solver.close()


def _case(name):
    if name == "c1":
        return config1(), 100
    if name == "t48x40b6":
        return tiny(48, 40, 6, peclet=0.5, seed=3), 30
    if name == "t64x20b8":
        return tiny(64, 20, 8, peclet=20.0, seed=4), 40
    raise KeyError(name)


@pytest.mark.parametrize("name,variant,degree", [("c1", O.CPTR3, 2), ("t48x40b6", O.CPTR3, 2),
                                                 ("t48x40b6", O.CPR, 3), ("t64x20b8", O.CPTR3, 1),
                                                 ("t48x40b6", O.CPTR, 2), ("t64x20b8", O.CPTR, 2)])
def test_chebyshev_solve_parity(name, variant, degree):
    """Solves with every AMG stage smoothed by Chebyshev: CPTR3 and CPR
    (scalar hierarchies) and the two-stage CPTR (the unknown-based system
    hierarchy on B_ee)."""
    print(f"case chebyshev solve {name} variant={variant} degree={degree}", flush=True)
    s, mc = _case(name)
    ref = O.solve(s, O.Options(color=O.tile_colors(s.nx, s.ny, 32, 8), amg=_amg(mc, degree), variant=variant))
    solver = cptr.solver_for(s, **_gpu(mc, degree, variant=GPU_VARIANT[variant], ilu_tile_x=32, ilu_tile_y=8))
    try:
        x, res = solver.solve(_t(s.rhs))
    finally:
        solver.close()
    x = x.cpu().numpy()
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    print(f"  gpu its={res['iterations']} oracle its={ref.iterations} err={err:.2e}", flush=True)
    assert res["converged"] == 1 and res["rel_res_scaled"] <= 1e-8
    assert abs(res["iterations"] - ref.iterations) <= 1
    assert err <= 1e-10


@pytest.mark.parametrize("variant", [O.CPTR3, O.CPTR])
def test_chebyshev_fp32_preconditioner(variant):
    """The Chebyshev V-cycles in FP32 inside FP64 FGMRES reach the FP64 true
    residual 1e-8, recomputed by the oracle."""
    print(f"case chebyshev fp32 variant={variant}", flush=True)
    s, mc = _case("t64x20b8")
    solver = cptr.solver_for(s, **_gpu(mc, 2, variant=GPU_VARIANT[variant], krylov=cptr.FGMRES,
                                       precond_precision=cptr.FP32, ilu_tile_x=32, ilu_tile_y=8))
    try:
        x, res = solver.solve(_t(s.rhs))
    finally:
        solver.close()
    dec = O.decouple(O.bsr_of(s), s.rhs, variant=variant)
    r = dec.rhsbar - dec.Abar.matvec(x.cpu().numpy())
    rel = np.linalg.norm(r) / np.linalg.norm(dec.rhsbar)
    print(f"  its={res['iterations']} rel={rel:.2e}", flush=True)
    assert res["converged"] == 1 and rel <= 1e-8 * (1 + 1e-6)


def test_chebyshev_sequence_reuse():
    """Hierarchy reuse over a sequence with the Chebyshev smoother: the kept
    hierarchies' Galerkin products, diagonals and Gershgorin bounds are
    recomputed from the new values, and every system solves to the oracle's
    solution with the same reuse decisions."""
    print("case chebyshev sequence reuse", flush=True)
    perm = G.config5_field(96, 48)
    systems = [G.config5(k, perm, nx=96, ny=48) for k in range(4)]
    thr = 0.99
    prev, refs = None, []
    for s in systems:
        r = O.solve(s, O.Options(color=O.tile_colors(s.nx, s.ny), amg=_amg(100), reuse_rho_max=thr), previous=prev)
        refs.append(r)
        prev = r
    solver = cptr.solver_for(systems[0], **_gpu(100, reuse_rho_max=thr))
    try:
        for k, (s, r) in enumerate(zip(systems, refs)):
            if k > 0:
                solver.update_values(torch.from_numpy(s.vals.reshape(-1)))
            x, res = solver.solve(_t(s.rhs))
            x = x.cpu().numpy()
            err = np.linalg.norm(x - r.x) / np.linalg.norm(r.x)
            mask = sum(1 << i for i, key in enumerate(("T", "P")) if r.reused.get(key))
            print(f"  system {k}: oracle reused={r.reused} its={r.iterations}; gpu reused={res['reused']} "
                  f"its={res['iterations']} err={err:.2e}", flush=True)
            assert res["reused"] == mask
            assert res["converged"] == 1 and abs(res["iterations"] - r.iterations) <= 1 and err <= 1e-10
    finally:
        solver.close()


def test_chebyshev_with_unbounded_level_limit():
    """amg_max_levels at its largest value: the per-level bounds take room for
    the levels actually built (coarsening stops at the max coarse size), and
    the solve matches the oracle's."""
    print("case chebyshev with amg_max_levels = 2^31 - 1", flush=True)
    s, mc = _case("t48x40b6")
    ref = O.solve(s, O.Options(color=O.tile_colors(s.nx, s.ny, 32, 8), amg=_amg(mc)))
    solver = cptr.solver_for(s, **_gpu(mc, amg_max_levels=2**31 - 1, ilu_tile_x=32, ilu_tile_y=8))
    try:
        x, res = solver.solve(_t(s.rhs))
        assert solver.amg_levels(0) == len(ref.hierarchies["T"].levels)
    finally:
        solver.close()
    err = np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x)
    print(f"  gpu its={res['iterations']} oracle its={ref.iterations} err={err:.2e}", flush=True)
    assert res["converged"] == 1 and abs(res["iterations"] - ref.iterations) <= 1 and err <= 1e-10
