"""GPU parity of the exact-sub-solver variants: the paper's study of the
Schur-complement approximations themselves (Sec. "Numerical Results"), where
every AMG stage applies its operator exactly -- M_PP = B_PP (CPR, CPTR3),
M_TT = C_TT (CPTR3), M_ee = B_ee (two-stage CPTR).  On the GPU the exact
solve is the dense Gauss-Jordan inverse of the operator up to 8192 rows and
the block-tridiagonal LU over grid rows above (exact_subsolves = 2 takes the
latter at any size); the oracle uses a dense LU with partial pivoting, and a
sparse LU above 4096 rows.  Bars: solution to 1e-10 relative and iterations
within one; exactness shown by one-step convergence on the uncoupled upwind
case."""
import numpy as np
import pytest

import oracle as O
from synthetic import config1, tiny

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1912_04385_amd import cptr  # noqa: E402

GPU_VARIANT = {O.CPTR3: cptr.VARIANT_CPTR3, O.CPR: cptr.VARIANT_CPR, O.CPTR: cptr.VARIANT_CPTR}


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _case(name):
    if name == "c1":
        return config1()
    if name == "t32x24b6":
        return tiny(32, 24, 6, peclet=5.0, seed=21)
    if name == "t48x40b6":
        return tiny(48, 40, 6, peclet=0.5, seed=3)
    if name == "t30x20b2":
        return tiny(30, 20, 2, peclet=50.0, seed=22)
    raise KeyError(name)


@pytest.mark.parametrize("name,variant", [("c1", O.CPTR3), ("c1", O.CPR), ("c1", O.CPTR),
                                          ("t32x24b6", O.CPTR3), ("t32x24b6", O.CPR), ("t32x24b6", O.CPTR),
                                          ("t48x40b6", O.CPTR3), ("t48x40b6", O.CPR), ("t30x20b2", O.CPTR)])
def test_exact_subsolve_solve_parity(name, variant):
    print(f"case exact sub-solves {name} variant={variant}", flush=True)
    s = _case(name)
    ref = O.solve(s, O.Options(color=O.tile_colors(s.nx, s.ny, 32, 8), variant=variant, exact_subsolves=True))
    solver = cptr.solver_for(s, variant=GPU_VARIANT[variant], exact_subsolves=1, ilu_tile_x=32, ilu_tile_y=8)
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
    assert res["levels_T"] == (1 if variant != O.CPR else 0)
    assert res["levels_P"] == (1 if variant != O.CPTR else 0)


@pytest.mark.parametrize("variant", [O.CPTR3, O.CPTR])
def test_exact_subsolves_with_exact_ilu_converge_in_one_step(variant):
    """Zero cross coupling, flow toward +x/+y only, one ILU tile (natural
    order): the composition rows are lower triangular, ILU(0) is exact on
    them, and the exact sub-solves make M^{-1} = Abar^{-1}."""
    print(f"case exact sub-solves uncoupled upwind variant={variant}", flush=True)
    s = tiny(6, 5, 5, seed=4, zero_coupling=True)
    solver = cptr.solver_for(s, variant=GPU_VARIANT[variant], exact_subsolves=1, ilu_tile_x=6, ilu_tile_y=5)
    try:
        _, res = solver.solve(_t(s.rhs))
    finally:
        solver.close()
    assert res["iterations"] == 1 and res["rel_res_scaled"] <= 1e-12


def test_exact_subsolve_beyond_the_dense_limit_needs_the_grid():
    """Above the dense limit the exact solve is block tridiagonal over grid
    rows: without the grid shape (an unstructured pattern, block Jacobi last
    stage) it is rejected before any kernel runs."""
    print("case exact sub-solve beyond the dense limit without the grid", flush=True)
    s = tiny(100, 90, 3, seed=1)                       # 9000 rows > 8192
    solver = cptr.Solver(exact_subsolves=1, last_stage=cptr.LAST_BJACOBI)
    try:
        with pytest.raises(cptr.CptrError, match="grid shape"):
            solver.setup(torch.from_numpy(s.row_ptr), torch.from_numpy(s.col_idx),
                         torch.from_numpy(s.vals.reshape(-1)), 0, 1, 0, 0)
    finally:
        solver.close()


@pytest.mark.parametrize("name,variant", [("c1", O.CPTR), ("t32x24b6", O.CPTR3), ("t32x24b6", O.CPR),
                                          ("t32x24b6", O.CPTR), ("t30x20b2", O.CPTR)])
def test_block_tridiagonal_exact_subsolves_parity(name, variant):
    """exact_subsolves = 2: the block-tridiagonal LU over grid rows at every
    size, against the oracle's dense LU."""
    print(f"case block-tridiagonal exact sub-solves {name} variant={variant}", flush=True)
    s = _case(name)
    ref = O.solve(s, O.Options(color=O.tile_colors(s.nx, s.ny, 32, 8), variant=variant, exact_subsolves=True))
    solver = cptr.solver_for(s, variant=GPU_VARIANT[variant], exact_subsolves=2, ilu_tile_x=32, ilu_tile_y=8)
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
def test_exact_subsolves_beyond_the_dense_limit(variant):
    """100 x 90 cells, b = 3: B_PP and C_TT have 9000 rows and B_ee 18000,
    beyond the dense inverse: the block-tridiagonal solves against the
    oracle's sparse LU."""
    print(f"case exact sub-solves beyond the dense limit variant={variant}", flush=True)
    s = tiny(100, 90, 3, peclet=2.0, seed=1)
    ref = O.solve(s, O.Options(color=O.tile_colors(s.nx, s.ny, 32, 8), variant=variant, exact_subsolves=True))
    solver = cptr.solver_for(s, variant=GPU_VARIANT[variant], exact_subsolves=1, ilu_tile_x=32, ilu_tile_y=8)
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
def test_block_tridiagonal_exact_with_exact_ilu_converge_in_one_step(variant):
    print(f"case block-tridiagonal exact sub-solves uncoupled upwind variant={variant}", flush=True)
    s = tiny(6, 5, 5, seed=4, zero_coupling=True)
    solver = cptr.solver_for(s, variant=GPU_VARIANT[variant], exact_subsolves=2, ilu_tile_x=6, ilu_tile_y=5)
    try:
        _, res = solver.solve(_t(s.rhs))
    finally:
        solver.close()
    assert res["iterations"] == 1 and res["rel_res_scaled"] <= 1e-12


@pytest.mark.parametrize("variant,exact", [(O.CPTR3, 1), (O.CPTR, 1), (O.CPTR3, 2), (O.CPTR, 2)])
def test_exact_subsolves_fp32_preconditioner(variant, exact):
    """Exact sub-solves inside the FP32 preconditioner (the dense inverses'
    FP32 copies) reach the FP64 true residual 1e-8 recomputed by the oracle."""
    print(f"case exact sub-solves fp32 variant={variant} exact={exact}", flush=True)
    s = _case("t32x24b6")
    solver = cptr.solver_for(s, variant=GPU_VARIANT[variant], exact_subsolves=exact, krylov=cptr.FGMRES,
                             precond_precision=cptr.FP32, ilu_tile_x=32, ilu_tile_y=8)
    try:
        x, res = solver.solve(_t(s.rhs))
    finally:
        solver.close()
    dec = O.decouple(O.bsr_of(s), s.rhs, variant=variant)
    r = dec.rhsbar - dec.Abar.matvec(x.cpu().numpy())
    rel = np.linalg.norm(r) / np.linalg.norm(dec.rhsbar)
    print(f"  its={res['iterations']} rel={rel:.2e}", flush=True)
    assert res["converged"] == 1 and rel <= 1e-8 * (1 + 1e-6)


def test_exact_subsolves_over_a_sequence():
    """update_values with reuse on keeps the single-level hierarchies and
    recomputes their dense inverses from the new values: each system solves
    to the oracle's exact-sub-solve solution."""
    print("case exact sub-solves over a sequence", flush=True)
    systems = [tiny(32, 24, 6, peclet=5.0, seed=21 + k) for k in range(3)]
    solver = cptr.solver_for(systems[0], variant=cptr.VARIANT_CPTR3, exact_subsolves=1, reuse_rho_max=0.3,
                             ilu_tile_x=32, ilu_tile_y=8)
    try:
        for k, s in enumerate(systems):
            if k > 0:
                solver.update_values(torch.from_numpy(s.vals.reshape(-1)))
            x, res = solver.solve(_t(s.rhs))
            ref = O.solve(s, O.Options(color=O.tile_colors(s.nx, s.ny, 32, 8), variant=O.CPTR3,
                                       exact_subsolves=True))
            x = x.cpu().numpy()
            err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
            print(f"  system {k}: gpu its={res['iterations']} oracle its={ref.iterations} err={err:.2e}", flush=True)
            assert res["converged"] == 1 and abs(res["iterations"] - ref.iterations) <= 1 and err <= 1e-10
    finally:
        solver.close()
