"""GPU parity at the benchmark's full size: the 1000 x 500-cell, b = 8 system
(4M unknowns) that bench.py times, in the same launch configuration
(CPTR3, BILU(0) in 64 x 8 tiles, two Jacobi sweeps before and after,
restart 50).

The oracle handles this size in seconds for the setup arithmetic (C
routines) and in about ten seconds for a whole FP64 solve, so the checks are
element by element: the scaled matrix and both AMG hierarchies bit for bit,
the plain FP64 solve to 1e-10 with iterations within one, and the FP32
preconditioner to the FP64 true residual 1e-8 recomputed by the oracle."""
import numpy as np
import pytest

import oracle as O
from synthetic import config3

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1912_04385_amd import cptr  # noqa: E402

NX, NY = 1000, 500
TILE = (64, 8)
SWEEPS = 2


@pytest.fixture(scope="module")
def c3():
    print("case full-size config 3 (system 0): generating", flush=True)
    s = config3(0)
    A = O.bsr_of(s)
    dec = O.decouple(A, s.rhs)
    return s, A, dec


def _solver(s, **kw):
    sv = cptr.Solver(restart=50, ilu_tile_x=TILE[0], ilu_tile_y=TILE[1], pre_sweeps=SWEEPS, post_sweeps=SWEEPS, **kw)
    sv.setup(torch.from_numpy(s.row_ptr), torch.from_numpy(s.col_idx), torch.from_numpy(s.vals.reshape(-1)), 0, 1,
             NX, NY)
    return sv


def test_scaled_matrix_and_hierarchies_bitwise(c3):
    s, A, dec = c3
    print("case full-size decoupling and hierarchies", flush=True)
    sv = _solver(s)
    try:
        abar, rb = sv.scaled(torch.from_numpy(s.rhs).cuda())
        assert np.array_equal(abar.cpu().numpy(), dec.Abar.vals.reshape(-1))
        assert np.array_equal(rb.cpu().numpy(), dec.rhsbar)
        for which, comp in ((0, 1), (1, 0)):
            h = O.amg_setup(dec.Abar.scalar_block(comp, comp), O.AMGOptions())
            assert sv.amg_levels(which) == len(h.levels), h.sizes
            for lvl, L in enumerate(h.levels):
                g = sv.amg_level(which, lvl)
                assert np.array_equal(g["rp"], L.A.rp) and np.array_equal(g["ci"], L.A.ci)
                assert np.array_equal(g["v"], L.A.v), f"hierarchy {which} level {lvl} operator"
                if lvl + 1 < len(h.levels):
                    assert np.array_equal(g["cf"], L.cf)
                    assert np.array_equal(g["pci"], L.P.ci) and np.array_equal(g["pv"], L.P.v)
            print(f"  hierarchy {which}: sizes {h.sizes} identical", flush=True)
    finally:
        sv.close()


def test_plain_fp64_solve_matches_the_oracle(c3):
    s, A, dec = c3
    print("case full-size plain FP64 solve (oracle solve ~10 s)", flush=True)
    ref = O.solve(s, O.Options(color=O.tile_colors(NX, NY, *TILE), restart=50,
                               amg=O.AMGOptions(pre=SWEEPS, post=SWEEPS)))
    sv = _solver(s)
    try:
        x, res = sv.solve(torch.from_numpy(s.rhs).cuda())
    finally:
        sv.close()
    x = x.cpu().numpy()
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    print(f"  gpu its={res['iterations']} oracle its={ref.iterations} err={err:.2e}", flush=True)
    assert res["converged"] == 1 and res["rel_res_scaled"] <= 1e-8
    assert abs(res["iterations"] - ref.iterations) <= 1
    assert err <= 1e-10


def test_fp32_preconditioner_reaches_the_fp64_tolerance(c3):
    s, A, dec = c3
    print("case full-size FP32-preconditioned FGMRES(50)", flush=True)
    sv = _solver(s, krylov=cptr.FGMRES, precond_precision=cptr.FP32)
    try:
        x, res = sv.solve(torch.from_numpy(s.rhs).cuda())
    finally:
        sv.close()
    x = x.cpu().numpy()
    r = dec.rhsbar - dec.Abar.matvec(x)
    rel = np.linalg.norm(r) / np.linalg.norm(dec.rhsbar)
    print(f"  its={res['iterations']} gpu rel_res={res['rel_res_scaled']:.3e} oracle-recomputed {rel:.3e}", flush=True)
    assert res["converged"] == 1
    assert rel <= 1e-8 * (1 + 1e-6)


def test_two_stage_cptr_system_amg(c3):
    """The two-stage CPTR scheme at full size: the unknown-based system
    hierarchy of the 1M-row elliptic block bit for bit, and the plain FP64
    solve to 1e-10 with iterations within one."""
    s, A, dec = c3
    print("case full-size two-stage CPTR (oracle solve ~20 s)", flush=True)
    ref = O.solve(s, O.Options(color=O.tile_colors(NX, NY, *TILE), restart=50, variant=O.CPTR,
                               amg=O.AMGOptions(pre=SWEEPS, post=SWEEPS)))
    h = ref.hierarchies["ee"]
    sv = _solver(s, variant=cptr.VARIANT_CPTR)
    try:
        assert sv.amg_levels(0) == len(h.levels), h.sizes
        for lvl, L in enumerate(h.levels):
            g = sv.amg_level(0, lvl)
            assert np.array_equal(g["rp"], L.A.rp) and np.array_equal(g["ci"], L.A.ci)
            assert np.array_equal(g["v"], L.A.v), f"system level {lvl} operator"
            if lvl + 1 < len(h.levels):
                assert np.array_equal(g["cf"], L.cf)
                assert np.array_equal(g["pci"], L.P.ci) and np.array_equal(g["pv"], L.P.v)
        print(f"  system hierarchy: sizes {h.sizes} identical", flush=True)
        x, res = sv.solve(torch.from_numpy(s.rhs).cuda())
    finally:
        sv.close()
    x = x.cpu().numpy()
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    print(f"  gpu its={res['iterations']} oracle its={ref.iterations} err={err:.2e}", flush=True)
    assert res["converged"] == 1 and res["rel_res_scaled"] <= 1e-8
    assert abs(res["iterations"] - ref.iterations) <= 1
    assert err <= 1e-10
