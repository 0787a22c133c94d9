"""GPU parity of the static-condensation front end (Sec. "Static-Condensation
Strategy", Eqs. global and reduced) against the oracle, through the C ABI.

Tolerances.  The per-cell factors come from Gauss-Jordan with partial
pivoting on the GPU and from LAPACK's LU in the oracle: on the diagonally
dominant J22 blocks of the recipe the two agree to a few ulps of the
factors' size, so Q, q, A and b are compared to 1e-12 of each array's
largest entry.  The recovered secondary update is compared on the same
primary update."""
import numpy as np
import pytest

from oracle import condense as C
from synthetic import config2, config3, full_system, tiny, wells

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1912_04385_amd import cptr  # noqa: E402


def _run(fs):
    A, b, Q, q = cptr.condense(torch.from_numpy(fs.row_ptr), torch.from_numpy(fs.col_idx),
                               torch.from_numpy(fs.J11.reshape(-1)), torch.from_numpy(fs.J12.reshape(-1)),
                               torch.from_numpy(fs.J21.reshape(-1)), torch.from_numpy(fs.J22.reshape(-1)),
                               torch.from_numpy(fs.r1), torch.from_numpy(fs.r2), fs.n1, fs.n2)
    return A.cpu().numpy(), b.cpu().numpy(), Q.cpu().numpy(), q.cpu().numpy()


def _close(g, r, tol=1e-12):
    scale = max(np.abs(r).max(), 1e-300) if r.size else 1.0
    return r.size == 0 or np.max(np.abs(g - r)) <= tol * scale


@pytest.mark.parametrize("nx,ny,n1,n2", [(5, 4, 3, 2), (7, 5, 2, 1), (9, 6, 8, 8), (11, 3, 6, 4), (6, 6, 4, 0),
                                          (33, 17, 8, 3)])
def test_condense_matches_oracle(nx, ny, n1, n2):
    print(f"case condense {nx}x{ny} n1={n1} n2={n2}", flush=True)
    fs = full_system(tiny(nx, ny, n1, peclet=1.0, seed=nx), n2, seed=ny, j12_scale=0.1)
    A, b, Q, q = _run(fs)
    rA, rb, rQ, rq = C.condense(fs)
    assert _close(A, rA.reshape(-1)) and _close(b, rb)
    assert _close(Q, rQ.reshape(-1)) and _close(q, rq.reshape(-1))
    d1 = np.random.default_rng(1).uniform(-1, 1, fs.n * n1)
    d2 = cptr.recover_secondary(torch.from_numpy(Q), torch.from_numpy(q), torch.from_numpy(d1), n1, n2)
    assert _close(d2.cpu().numpy(), C.recover(rQ, rq, d1))


def test_condense_then_solve_satisfies_the_full_system():
    """GPU condensation, the CPTR3 solve of the reduced system and the GPU
    recovery together solve Eq. global (residual of the whole Newton system)."""
    print("case condense + solve + recover 24x20 b=6 n2=3", flush=True)
    fs = full_system(tiny(24, 20, 6, peclet=1.0, seed=9), 3, seed=2)
    A, b, Q, q = _run(fs)
    sv = cptr.Solver(amg_max_coarse=30)
    try:
        sv.setup(torch.from_numpy(fs.row_ptr), torch.from_numpy(fs.col_idx), torch.from_numpy(A), 0, 1, fs.nx, fs.ny)
        x, res = sv.solve(torch.from_numpy(b).cuda())
    finally:
        sv.close()
    assert res["converged"] == 1
    d1 = x.cpu().numpy()
    d2 = cptr.recover_secondary(torch.from_numpy(Q), torch.from_numpy(q), x, fs.n1, fs.n2).cpu().numpy()
    J, r = C.full_dense(fs)
    resid = J @ np.concatenate([d1, d2]) + r
    print(f"  its={res['iterations']} full-system relative residual {np.linalg.norm(resid) / np.linalg.norm(r):.2e}",
          flush=True)
    assert np.linalg.norm(resid) <= 1e-6 * np.linalg.norm(r)


def test_singular_secondary_block_is_reported():
    print("case condense singular J22", flush=True)
    fs = full_system(tiny(8, 6, 4, seed=3), 3, seed=5)
    fs.J22[13] = 0.0
    fs.J22[29, 1, :] = 0.0
    with pytest.raises(cptr.CptrError, match="cell 13"):
        _run(fs)


def test_condense_config2_size():
    print("case condense config2-0 (200x100, b=6) n2=4", flush=True)
    fs = full_system(config2(0), 4, seed=0)
    A, b, Q, q = _run(fs)
    rA, rb, rQ, rq = C.condense(fs)
    assert _close(A, rA.reshape(-1)) and _close(b, rb) and _close(Q, rQ.reshape(-1)) and _close(q, rq.reshape(-1))


def test_condense_full_size_sampled():
    """The config-3 system (1000 x 500 cells, b = 8) with four secondary
    unknowns per cell: every output against the oracle."""
    print("case condense config3 (1000x500, b=8) n2=4", flush=True)
    fs = full_system(config3(0), 4, seed=0)
    A, b, Q, q = _run(fs)
    rA, rb, rQ, rq = C.condense(fs)
    assert _close(A, rA.reshape(-1)) and _close(b, rb) and _close(Q, rQ.reshape(-1)) and _close(q, rq.reshape(-1))


def _run_wells(fs, A, b, W):
    """GPU well elimination in place on copies of (A, b); returns A', b', Qw, qw."""
    At = torch.from_numpy(np.ascontiguousarray(A).reshape(-1).copy()).cuda()
    bt = torch.from_numpy(np.ascontiguousarray(b).copy()).cuda()
    Qw, qw = cptr.condense_wells(torch.from_numpy(fs.row_ptr), torch.from_numpy(fs.col_idx), At, bt,
                                 torch.from_numpy(W.cell), torch.from_numpy(W.J1w.reshape(-1)),
                                 torch.from_numpy(W.Jw1.reshape(-1)), torch.from_numpy(W.Jww.reshape(-1)),
                                 torch.from_numpy(W.rw), fs.n1, W.nw)
    torch.cuda.synchronize()
    return At.cpu().numpy(), bt.cpu().numpy(), Qw, qw


@pytest.mark.parametrize("nx,ny,n1,n2,nw,cells", [(5, 4, 3, 2, 2, None), (9, 6, 8, 3, 1, None),
                                                   (7, 5, 4, 0, 8, [3, 34, 12]), (6, 6, 6, 2, 3, [7, 7, 0]),
                                                   (33, 17, 8, 4, 2, None)])
def test_wells_match_oracle(nx, ny, n1, n2, nw, cells):
    """Well elimination after the condensation (remark closing Sec.
    "Static-Condensation Strategy"): A, b, the well factors and the well
    update against the oracle, to 1e-12 of each array's largest entry; two
    wells in one cell (case with cells 7, 7) add their terms in well order."""
    print(f"case wells {nx}x{ny} n1={n1} n2={n2} nw={nw} cells={cells}", flush=True)
    fs = full_system(tiny(nx, ny, n1, peclet=1.0, seed=nx), n2, seed=ny, j12_scale=0.1)
    W = wells(nx, ny, n1, nw, cells=cells, seed=nx + ny)
    A, b, Q, q = _run(fs)
    rA, rb, rQ, rq = C.condense(fs)
    rA2, rb2, rQw, rqw = C.eliminate_wells(rA, rb, fs.row_ptr, fs.col_idx, W)
    A2, b2, Qw, qw = _run_wells(fs, A, b, W)
    assert _close(A2, rA2.reshape(-1)) and _close(b2, rb2)
    assert _close(Qw.cpu().numpy(), rQw.reshape(-1)) and _close(qw.cpu().numpy(), rqw.reshape(-1))
    d1 = np.random.default_rng(2).uniform(-1, 1, fs.n * n1)
    dw = cptr.recover_wells(torch.from_numpy(W.cell), Qw, qw, torch.from_numpy(d1), n1, nw).cpu().numpy()
    assert _close(dw, C.recover_wells(W, rQw, rqw, d1))


def test_condense_wells_then_solve_satisfies_the_full_system():
    """Condensation, well elimination, the CPTR3 solve of the reduced system
    and both recoveries on the GPU solve the whole system with its well rows
    (dense residual of the full system)."""
    print("case condense + wells + solve + recover 24x20 b=6 n2=3 nw=2", flush=True)
    fs = full_system(tiny(24, 20, 6, peclet=1.0, seed=9), 3, seed=2)
    W = wells(24, 20, 6, 2, seed=5)
    A, b, Q, q = _run(fs)
    A2, b2, Qw, qw = _run_wells(fs, A, b, W)
    sv = cptr.Solver(amg_max_coarse=30)
    try:
        sv.setup(torch.from_numpy(fs.row_ptr), torch.from_numpy(fs.col_idx), torch.from_numpy(A2), 0, 1, fs.nx, fs.ny)
        x, res = sv.solve(torch.from_numpy(b2).cuda())
    finally:
        sv.close()
    assert res["converged"] == 1
    d1 = x.cpu().numpy()
    d2 = cptr.recover_secondary(torch.from_numpy(Q), torch.from_numpy(q), x, fs.n1, fs.n2).cpu().numpy()
    dw = cptr.recover_wells(torch.from_numpy(W.cell), Qw, qw, x, fs.n1, W.nw).cpu().numpy()
    J, r = C.full_dense_with_wells(fs, W)
    resid = J @ np.concatenate([d1, d2, dw]) + r
    print(f"  its={res['iterations']} full-system relative residual {np.linalg.norm(resid) / np.linalg.norm(r):.2e}",
          flush=True)
    assert np.linalg.norm(resid) <= 1e-6 * np.linalg.norm(r)


def test_wells_errors_are_reported_before_any_change():
    print("case wells: singular Jww, cell out of range", flush=True)
    fs = full_system(tiny(8, 6, 4, seed=3), 2, seed=5)
    A, b, Q, q = _run(fs)
    W = wells(8, 6, 4, 2, cells=[3, 9, 40], seed=1)
    W.Jww[1] = 0.0
    At = torch.from_numpy(A.copy()).cuda()
    bt = torch.from_numpy(b.copy()).cuda()
    args = lambda cells: (torch.from_numpy(fs.row_ptr), torch.from_numpy(fs.col_idx), At, bt,  # noqa: E731
                          torch.from_numpy(np.array(cells, np.int32)), torch.from_numpy(W.J1w.reshape(-1)),
                          torch.from_numpy(W.Jw1.reshape(-1)), torch.from_numpy(W.Jww.reshape(-1)),
                          torch.from_numpy(W.rw), 4, 2)
    with pytest.raises(cptr.CptrError, match="well 1"):
        cptr.condense_wells(*args([3, 9, 40]))
    assert np.array_equal(At.cpu().numpy(), A) and np.array_equal(bt.cpu().numpy(), b)
    with pytest.raises(cptr.CptrError, match="outside"):
        cptr.condense_wells(*args([3, 48, 40]))
