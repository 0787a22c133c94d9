"""Degenerate inputs through the C ABI: an empty system is rejected before any
GPU work; a single cell, two cells and one-cell-wide grids (every tile
ragged, a one-colour tile schedule, single-level hierarchies) solve to the
oracle's solution for every variant (1e-10 relative, iterations within one);
one context set up in turn on systems of different shapes."""
import numpy as np
import pytest

import oracle as O
from synthetic import tiny

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1912_04385_amd import cptr  # noqa: E402

VARIANTS = {O.CPTR3: cptr.VARIANT_CPTR3, O.CPR: cptr.VARIANT_CPR, O.CPTR: cptr.VARIANT_CPTR,
            O.BJ_ONLY: cptr.VARIANT_LAST_ONLY}


def test_empty_system_is_rejected():
    print("case empty system", flush=True)
    sv = cptr.Solver()
    try:
        with pytest.raises(cptr.CptrError) as ei:
            sv.setup(torch.zeros(1, dtype=torch.int32), torch.zeros(0, dtype=torch.int32),
                     torch.zeros(0, dtype=torch.float64), 0, 1, 0, 0)
        assert ei.value.status == -1
    finally:
        sv.close()


@pytest.mark.parametrize("variant", [O.CPTR3, O.CPR, O.CPTR, O.BJ_ONLY])
@pytest.mark.parametrize("nx,ny,b", [(1, 1, 3), (2, 1, 2), (40, 1, 4), (1, 37, 6)])
def test_degenerate_grid_solve(nx, ny, b, variant):
    print(f"case degenerate grid {nx}x{ny} b={b} variant={variant}", flush=True)
    s = tiny(nx, ny, b, seed=5)
    ref = O.solve(s, O.Options(color=O.tile_colors(nx, ny, 32, 8), variant=variant))
    solver = cptr.solver_for(s, variant=VARIANTS[variant], ilu_tile_x=32, ilu_tile_y=8)
    try:
        x, res = solver.solve(torch.from_numpy(s.rhs).cuda())
    finally:
        solver.close()
    x = x.cpu().numpy()
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    print(f"  gpu its={res['iterations']} oracle its={ref.iterations} err={err:.2e}", flush=True)
    assert res["converged"] == 1 and res["rel_res_scaled"] <= 1e-8
    assert abs(res["iterations"] - ref.iterations) <= 1
    assert err <= 1e-10


@pytest.mark.parametrize("variant", [O.CPTR3, O.CPTR])
def test_one_context_many_shapes(variant):
    """One context set up in turn on systems of different sizes and block
    sizes (larger, smaller, larger again): every setup replaces the previous
    state, and each solve matches the oracle's."""
    from synthetic import config1, config2
    systems = [config2(0), tiny(45, 29, 8, peclet=3.0, seed=31), config1(), tiny(64, 20, 2, peclet=0.3, seed=32),
               config2(3)]
    solver = cptr.Solver(variant=VARIANTS[variant], ilu_tile_x=32, ilu_tile_y=8)
    try:
        for k, s in enumerate(systems):
            print(f"case one context, system {k}: {s.nx}x{s.ny} b={s.b} variant={variant}", flush=True)
            ref = O.solve(s, O.Options(color=O.tile_colors(s.nx, s.ny, 32, 8), variant=variant))
            solver.setup(torch.from_numpy(s.row_ptr), torch.from_numpy(s.col_idx),
                         torch.from_numpy(s.vals.reshape(-1)), 0, 1, s.nx, s.ny)
            x, res = solver.solve(torch.from_numpy(s.rhs).cuda())
            x = x.cpu().numpy()
            err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
            print(f"  gpu its={res['iterations']} oracle its={ref.iterations} err={err:.2e}", flush=True)
            assert res["converged"] == 1 and res["rel_res_scaled"] <= 1e-8
            assert abs(res["iterations"] - ref.iterations) <= 1
            assert err <= 1e-10
    finally:
        solver.close()


def test_singular_coarse_operator_is_reported():
    """Two cells, b = 2, no pressure-temperature coupling, C_TT = [[1, 1], [1,
    1]]: its dense inverse (a single-level hierarchy) meets an exactly zero
    pivot, and setup reports the singular coarsest operator."""
    print("case singular coarse operator", flush=True)
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    diag = [[2.0, 0.0], [0.0, 1.0]]
    off = [[-1.0, 0.0], [0.0, 1.0]]
    vals = np.array([diag, off, off, diag], np.float64).reshape(-1)
    sv = cptr.Solver(ilu_tile_x=32, ilu_tile_y=8)
    try:
        with pytest.raises(cptr.CptrError, match="singular coarsest AMG operator") as ei:
            sv.setup(torch.from_numpy(rp), torch.from_numpy(ci), torch.from_numpy(vals), 0, 1, 2, 1)
        assert ei.value.status == -3
    finally:
        sv.close()


def test_setup_without_grid_shape():
    """Without the grid shape (nx = ny = 0) the block-Jacobi last stage works
    on any BSR pattern and matches the oracle; BILU(0), whose order needs the
    grid, is rejected."""
    from synthetic import config1
    print("case setup without grid shape", flush=True)
    s = config1()
    ref = O.solve(s, O.Options(color=O.tile_colors(s.nx, s.ny, 32, 8), last_stage=O.LAST_BJACOBI))
    sv = cptr.Solver(last_stage=cptr.LAST_BJACOBI)
    try:
        sv.setup(torch.from_numpy(s.row_ptr), torch.from_numpy(s.col_idx), torch.from_numpy(s.vals.reshape(-1)),
                 0, 1, 0, 0)
        x, res = sv.solve(torch.from_numpy(s.rhs).cuda())
    finally:
        sv.close()
    err = np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x)
    print(f"  gpu its={res['iterations']} oracle its={ref.iterations} err={err:.2e}", flush=True)
    assert res["converged"] == 1 and abs(res["iterations"] - ref.iterations) <= 1 and err <= 1e-10
    sv = cptr.Solver()
    try:
        with pytest.raises(cptr.CptrError, match="grid shape") as ei:
            sv.setup(torch.from_numpy(s.row_ptr), torch.from_numpy(s.col_idx),
                     torch.from_numpy(s.vals.reshape(-1)), 0, 1, 0, 0)
        assert ei.value.status == -1
    finally:
        sv.close()
