"""GPU parity of the V-cycle convergence factor and of hierarchy reuse over a
sequence of systems on one pattern (the Newton sequence with a moving
combustion band), through the C ABI, against the CPU FP64 oracle."""
import numpy as np
import pytest

import oracle as O
from synthetic import generator as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1912_04385_amd import cptr  # noqa: E402

NX, NY = 96, 48


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _opts(s, **kw):
    return O.Options(color=O.tile_colors(s.nx, s.ny), amg=O.AMGOptions(max_coarse=100), **kw)


def test_conv_factor_parity():
    print("case conv_factor tiny48x40b6", flush=True)
    s = G.tiny(48, 40, 6, peclet=0.5, seed=3)
    ref = O.solve(s, O.Options(color=O.tile_colors(48, 40), amg=O.AMGOptions(max_coarse=30), max_iters=1))
    solver = cptr.solver_for(s, amg_max_coarse=30)
    for which, key in ((0, "T"), (1, "P")):
        for cycles, seed in ((10, 0), (3, 12345)):
            rho = solver.conv_factor(which, cycles, seed)
            rr = O.conv_factor(ref.hierarchies[key], cycles, seed)
            print(f"  {key} cycles={cycles} seed={seed}: gpu {rho:.15f} oracle {rr:.15f}", flush=True)
            assert abs(rho - rr) <= 1e-10 * rr
    solver.close()


def _gpu_sequence(systems, thr):
    solver = cptr.solver_for(systems[0], amg_max_coarse=100, reuse_rho_max=thr)
    out = []
    try:
        for k, s in enumerate(systems):
            if k > 0:
                solver.update_values(torch.from_numpy(s.vals.reshape(-1)))
            x, res = solver.solve(_t(s.rhs))
            levels = {key: [solver.amg_level(w, l) for l in range(solver.amg_levels(w))]
                      for w, key in ((0, "T"), (1, "P"))}
            out.append((x.cpu().numpy(), res, levels))
    finally:
        solver.close()
    return out


def _oracle_sequence(systems, thr):
    out, prev = [], None
    for s in systems:
        r = O.solve(s, _opts(s, reuse_rho_max=thr), previous=prev)
        out.append(r)
        prev = r
    return out


def _check_levels(glev, h):
    assert len(glev) == len(h.levels)
    for g, L in zip(glev, h.levels):
        assert np.array_equal(g["rp"], L.A.rp) and np.array_equal(g["ci"], L.A.ci)
        assert np.array_equal(g["v"], L.A.v)


@pytest.mark.parametrize("mode", ["default", "keep_all"])
def test_sequence_reuse_parity(mode):
    print(f"case sequence reuse {mode}", flush=True)
    perm = G.config5_field(NX, NY)
    systems = [G.config5(k, perm, nx=NX, ny=NY) for k in range(6)]
    # 0.3 keeps the temperature hierarchy and rebuilds the pressure one on
    # this recipe (rho_T ~ 0.17, rho_P ~ 0.33, so the pressure trials back
    # off: trials at systems 1, 3 and 6); 0.99 keeps both
    thr = 0.3 if mode == "default" else 0.99
    ref = _oracle_sequence(systems, thr)
    got = _gpu_sequence(systems, thr)
    for k, (r, (x, res, levels)) in enumerate(zip(ref, got)):
        err = np.linalg.norm(x - r.x) / np.linalg.norm(r.x)
        mask = sum(1 << i for i, key in enumerate(("T", "P")) if r.reused.get(key))
        print(f"  system {k}: oracle rho={r.rho} reused={r.reused} its={r.iterations}; gpu rho=({res['rho_T']:.6f}, "
              f"{res['rho_P']:.6f}) reused={res['reused']} its={res['iterations']} err={err:.2e}", flush=True)
        if k == 0:
            assert res["reused"] == 0 and res["rho_T"] == -1.0 and res["rho_P"] == -1.0
        else:
            for key, g in (("T", res["rho_T"]), ("P", res["rho_P"])):
                if key not in r.rho:        # no trial: rebuilt during the back-off
                    assert g == -1.0
                    continue
                assert abs(g - r.rho[key]) <= 1e-9 * r.rho[key]
                assert abs(r.rho[key] - thr) > 1e-6, "decision too close to the threshold to compare"
            assert res["reused"] == mask
        for key in ("T", "P"):
            _check_levels(levels[key], r.hierarchies[key])
        assert res["converged"] == 1 and res["rel_res_scaled"] <= 1e-8
        assert abs(res["iterations"] - r.iterations) <= 1
        assert err <= 1e-10
    if mode == "keep_all":
        assert got[1][1]["reused"] == 3


def test_rebuild_equals_fresh_setup():
    print("case rebuild equals fresh setup", flush=True)
    perm = G.config5_field(NX, NY)
    s0, s1 = G.config5(0, perm, nx=NX, ny=NY), G.config5(1, perm, nx=NX, ny=NY)
    seq = _gpu_sequence([s0, s1], 1e-9)
    fresh = cptr.solver_for(s1, amg_max_coarse=100)
    x, res = fresh.solve(_t(s1.rhs))
    fresh.close()
    assert seq[1][1]["reused"] == 0
    assert seq[1][1]["iterations"] == res["iterations"]
    assert np.array_equal(seq[1][0], x.cpu().numpy())


def test_fp32_sequence_reaches_fp64_tolerance():
    print("case fp32 sequence", flush=True)
    perm = G.config5_field(NX, NY)
    systems = [G.config5(k, perm, nx=NX, ny=NY) for k in range(3)]
    solver = cptr.solver_for(systems[0], amg_max_coarse=100, krylov=cptr.FGMRES, restart=50,
                             precond_precision=cptr.FP32)
    try:
        for k, s in enumerate(systems):
            if k:
                solver.update_values(torch.from_numpy(s.vals.reshape(-1)))
            x, res = solver.solve(_t(s.rhs))
            r = s.rhs - O.bsr_of(s).matvec(x.cpu().numpy())
            print(f"  system {k}: its={res['iterations']} reused={res['reused']} rel_res={res['rel_res_scaled']:.2e}",
                  flush=True)
            assert res["converged"] == 1 and res["rel_res_scaled"] <= 1e-8
            assert np.linalg.norm(r) / np.linalg.norm(s.rhs) <= 2e-8
    finally:
        solver.close()
