"""ctypes binding of libcptr.so (include/cptr.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream (``torch.cuda.current_stream().cuda_stream``); every step of the solve
runs in the library's HIP kernels.  Importing this module does not need a GPU;
using a Solver does, and fails loudly when the library is missing.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcptr.so")

VARIANT_CPTR3, VARIANT_CPR, VARIANT_CPTR, VARIANT_LAST_ONLY = 0, 1, 2, 3
T_THEN_P, P_THEN_T = 0, 1
LAST_BILU0, LAST_BJACOBI = 0, 1
GMRES, FGMRES = 0, 1
FP64, FP32 = 0, 1
SMOOTH_JACOBI, SMOOTH_L1JACOBI, SMOOTH_CHEBYSHEV = 0, 1, 2
INTERP_CLASSICAL, INTERP_LEARNED, INTERP_LEARNED_FORCED = 0, 1, 2
MLP_NPARAMS = 5313

STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "E_ARG", -2: "E_HIP", -3: "E_SINGULAR_BLOCK",
          -4: "E_NONFINITE", -5: "E_OOM", -6: "E_STATE"}


class CptrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32), ("stage_order", ctypes.c_int32), ("last_stage", ctypes.c_int32),
        ("krylov", ctypes.c_int32), ("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32),
        ("rtol", ctypes.c_double), ("precond_precision", ctypes.c_int32), ("reorth", ctypes.c_int32),
        ("amg_theta", ctypes.c_double), ("amg_max_coarse", ctypes.c_int32), ("amg_max_levels", ctypes.c_int32),
        ("amg_pmax", ctypes.c_int32), ("smoother", ctypes.c_int32), ("pre_sweeps", ctypes.c_int32),
        ("post_sweeps", ctypes.c_int32), ("jacobi_omega", ctypes.c_double), ("pmis_seed", ctypes.c_uint64),
        ("ilu_tile_x", ctypes.c_int32), ("ilu_tile_y", ctypes.c_int32), ("t_interp", ctypes.c_int32),
        ("reuse_rho_max", ctypes.c_double), ("timing", ctypes.c_int32), ("setup_kernels", ctypes.c_int32),
        ("exact_subsolves", ctypes.c_int32), ("cheb_degree", ctypes.c_int32), ("stop_unscaled", ctypes.c_int32),
        ("judge_cycles", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32), ("converged", ctypes.c_int32),
        ("used_learned", ctypes.c_int32), ("rel_res_scaled", ctypes.c_double),
        ("rel_res_unscaled", ctypes.c_double), ("rho_T", ctypes.c_double), ("rho_P", ctypes.c_double),
        ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double), ("levels_T", ctypes.c_int32),
        ("levels_P", ctypes.c_int32), ("reused", ctypes.c_int32), ("timed_steps", ctypes.c_int32),
        ("t_stage1_ms", ctypes.c_double), ("t_stage2_ms", ctypes.c_double), ("t_last_ms", ctypes.c_double),
        ("t_spmv_ms", ctypes.c_double), ("t_arnoldi_ms", ctypes.c_double),
        ("rho_T_classical", ctypes.c_double), ("rho_T_learned", ctypes.c_double),
        ("t_setup_scale_ms", ctypes.c_double), ("t_setup_amgT_ms", ctypes.c_double),
        ("t_setup_amgP_ms", ctypes.c_double), ("t_setup_values_ms", ctypes.c_double),
    ]

    def to_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Load libcptr.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        sig = {
            "cptr_default_options": [ctypes.POINTER(Options)],
            "cptr_create": [ctypes.POINTER(P), I32, P, ctypes.POINTER(Options)],
            "cptr_setup": [P, I32, I32, I32, P, P, P, I32, I32, I32, I32],
            "cptr_update_values": [P, P],
            "cptr_solve": [P, P, P, ctypes.POINTER(Result)],
            "cptr_residual_history": [P, P, I32, ctypes.POINTER(I32)],
            "cptr_destroy": [P],
            "cptr_decouple": [I32, I32, I32, P, P, P, P, I32, I32, P, P, P],
            "cptr_decouple_noalloc": [I32, I32, I32, P, P, P, P, I32, I32, P, P, P],
            "cptr_bsr_spmv": [I32, I32, P, P, P, P, P, P],
            "cptr_stream_read": [P, ctypes.c_uint64, P, ctypes.POINTER(I32), P],
            "cptr_amg_levels": [P, I32, ctypes.POINTER(I32)],
            "cptr_amg_level_info": [P, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)],
            "cptr_amg_level_copy": [P, I32, I32, P, P, P, P, P, P, P],
            "cptr_amg_vcycle": [P, I32, P, P],
            "cptr_amg_conv_factor": [P, I32, I32, ctypes.c_uint64, ctypes.POINTER(D)],
            "cptr_precond_apply": [P, P, P],
            "cptr_get_scaled": [P, P, P, P],
            "cptr_load_mlp": [P, P],
            "cptr_mlp_create": [ctypes.POINTER(P), I32, P],
            "cptr_mlp_get": [P, P, P],
            "cptr_mlp_train_step": [P, P, I32, ctypes.c_uint64, D, ctypes.POINTER(D)],
            "cptr_mlp_edges": [P, P, P, P, I32, ctypes.POINTER(I32)],
            "cptr_mlp_destroy": [P],
            "cptr_condense": [I32, I32, I32, I32, P, P, P, P, P, P, P, P, P, P, P, P, P],
            "cptr_recover_secondary": [I32, I32, I32, P, P, P, P, P],
            "cptr_condense_wells": [I32, I32, I32, P, P, I32, I32, P, P, P, P, P, P, P, P, P, P],
            "cptr_recover_wells": [I32, I32, I32, P, P, P, P, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.cptr_last_error.restype = ctypes.c_char_p
        L.cptr_last_error.argtypes = []
        _lib = L
    return _lib


def _check(rc: int, soft_ok: bool = False) -> int:
    if rc < 0 or (rc > 0 and not soft_ok):
        raise CptrError(rc, lib().cptr_last_error().decode())
    return rc


def default_options(**kw) -> Options:
    o = Options()
    _check(lib().cptr_default_options(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype):
    import torch
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    return t.to(device="cuda", dtype=dtype).contiguous()


_live_solvers = weakref.WeakSet()


@atexit.register
def _close_all():
    """Destroy every live context while the HIP runtime is certainly up."""
    for s in list(_live_solvers):
        try:
            s.close()
        except Exception:
            pass


class Solver:
    """One context of the C library: setup() once per matrix, solve() per rhs."""

    def __init__(self, device: int = 0, **opts):
        import torch
        self.ctx = ctypes.c_void_p()
        self.opts = default_options(**opts)
        torch.cuda.set_device(device)
        _check(lib().cptr_create(ctypes.byref(self.ctx), device, _stream(), ctypes.byref(self.opts)))
        _live_solvers.add(self)
        self.n = self.b = 0

    def setup(self, row_ptr, col_idx, vals, p_index: int = 0, T_index: int = 1, nx: int = 0, ny: int = 0):
        import torch
        self._rp = _dev(row_ptr, torch.int32)
        self._ci = _dev(col_idx, torch.int32)
        v = _dev(vals, torch.float64)
        self.n = self._rp.numel() - 1
        nnzb = self._ci.numel()
        self.b = int(round((v.numel() / max(nnzb, 1)) ** 0.5))
        _check(lib().cptr_setup(self.ctx, self.n, self.b, nnzb, _ptr(self._rp), _ptr(self._ci), _ptr(v),
                                p_index, T_index, nx, ny))
        return self

    def load_mlp(self, params):
        """Parameters of the learned temperature interpolation (float32 blob
        of MLP_NPARAMS values; None removes them)."""
        import numpy as np
        if params is None:
            _check(lib().cptr_load_mlp(self.ctx, None))
            return
        blob = np.ascontiguousarray(params, dtype=np.float32)
        if blob.size != MLP_NPARAMS:
            raise ValueError(f"need {MLP_NPARAMS} parameters, got {blob.size}")
        _check(lib().cptr_load_mlp(self.ctx, blob.ctypes.data_as(ctypes.c_void_p)))

    def update_values(self, vals):
        import torch
        v = _dev(vals, torch.float64)
        _check(lib().cptr_update_values(self.ctx, _ptr(v)))

    def solve(self, rhs, x=None):
        import torch
        r = _dev(rhs, torch.float64)
        if x is None:
            x = torch.empty_like(r)
        res = Result()
        rc = _check(lib().cptr_solve(self.ctx, _ptr(r), _ptr(x), ctypes.byref(res)), soft_ok=True)
        d = res.to_dict()
        d["status"] = STATUS.get(rc, rc)
        return x, d

    def residual_history(self):
        n = ctypes.c_int32()
        _check(lib().cptr_residual_history(self.ctx, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_double * max(n.value, 1))()
        _check(lib().cptr_residual_history(self.ctx, buf, n.value, ctypes.byref(n)))
        return list(buf)[: n.value]

    def amg_levels(self, which: int) -> int:
        n = ctypes.c_int32()
        _check(lib().cptr_amg_levels(self.ctx, which, ctypes.byref(n)))
        return n.value

    def amg_level_sizes(self, which: int, level: int) -> tuple:
        """(rows, operator nnz, P nnz) of one level (P nnz 0 on the coarsest)."""
        nr, nnz, pn = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().cptr_amg_level_info(self.ctx, which, level, ctypes.byref(nr), ctypes.byref(nnz),
                                         ctypes.byref(pn)))
        return nr.value, nnz.value, pn.value

    def amg_level(self, which: int, level: int) -> dict:
        import numpy as np
        nr, nnz, pn = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().cptr_amg_level_info(self.ctx, which, level, ctypes.byref(nr), ctypes.byref(nnz),
                                         ctypes.byref(pn)))
        rp = np.zeros(nr.value + 1, np.int32)
        ci = np.zeros(max(nnz.value, 1), np.int32)
        v = np.zeros(max(nnz.value, 1))
        has_p = pn.value > 0
        cf = np.zeros(nr.value, np.int32) if has_p else None
        prp = np.zeros(nr.value + 1, np.int32) if has_p else None
        pci = np.zeros(max(pn.value, 1), np.int32) if has_p else None
        pv = np.zeros(max(pn.value, 1)) if has_p else None
        a = lambda x: x.ctypes.data_as(ctypes.c_void_p) if x is not None else None  # noqa: E731
        _check(lib().cptr_amg_level_copy(self.ctx, which, level, a(rp), a(ci), a(v), a(cf), a(prp), a(pci), a(pv)))
        out = dict(n=nr.value, rp=rp, ci=ci[: nnz.value], v=v[: nnz.value])
        if has_p:
            out.update(cf=cf, prp=prp, pci=pci[: pn.value], pv=pv[: pn.value])
        return out

    def vcycle(self, which: int, b):
        import torch
        bb = _dev(b, torch.float64)
        x = torch.empty_like(bb)
        _check(lib().cptr_amg_vcycle(self.ctx, which, _ptr(bb), _ptr(x)))
        return x

    def conv_factor(self, which: int, cycles: int = 10, seed: int = 0) -> float:
        rho = ctypes.c_double(0.0)
        _check(lib().cptr_amg_conv_factor(self.ctx, which, cycles, ctypes.c_uint64(seed), ctypes.byref(rho)))
        return rho.value

    def precond_apply(self, r):
        import torch
        rr = _dev(r, torch.float64)
        y = torch.empty_like(rr)
        _check(lib().cptr_precond_apply(self.ctx, _ptr(rr), _ptr(y)))
        return y

    def scaled(self, rhs=None):
        import torch
        nnzb = self._ci.numel()
        abar = torch.empty(nnzb * self.b * self.b, dtype=torch.float64, device="cuda")
        if rhs is not None:
            r = _dev(rhs, torch.float64)
            rb = torch.empty_like(r)
            _check(lib().cptr_get_scaled(self.ctx, _ptr(abar), _ptr(rb), _ptr(r)))
            return abar, rb
        _check(lib().cptr_get_scaled(self.ctx, _ptr(abar), None, None))
        return abar, None

    def close(self):
        if self.ctx:
            lib().cptr_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decouple(variant, row_ptr, col_idx, vals, rhs, p_index=0, T_index=1):
    """Left scaling alone (Eqs. CPTR31/CPTR32 or CPR) on device tensors."""
    import torch
    rp, ci = _dev(row_ptr, torch.int32), _dev(col_idx, torch.int32)
    v, r = _dev(vals, torch.float64), _dev(rhs, torch.float64)
    n = rp.numel() - 1
    b = r.numel() // n
    abar = torch.empty_like(v)
    rb = torch.empty_like(r)
    _check(lib().cptr_decouple(variant, n, b, _ptr(rp), _ptr(ci), _ptr(v), _ptr(r), p_index, T_index,
                               _ptr(abar), _ptr(rb), _stream()))
    torch.cuda.synchronize()
    return abar, rb


def decouple_noalloc(variant, row_ptr, col_idx, vals, rhs, abar, rhsbar, p_index=0, T_index=1):
    """cptr_decouple_noalloc into caller-provided device tensors abar, rhsbar
    (the library allocates nothing)."""
    import torch
    n = row_ptr.numel() - 1
    b = rhs.numel() // n
    _check(lib().cptr_decouple_noalloc(variant, n, b, _ptr(row_ptr), _ptr(col_idx), _ptr(vals), _ptr(rhs),
                                       p_index, T_index, _ptr(abar), _ptr(rhsbar), _stream()))
    torch.cuda.synchronize()
    return abar, rhsbar


def stream_read(x, part=None):
    """One streaming read of the float64 device tensor x (cptr_stream_read);
    returns the per-workgroup partial sums (their total equals x.sum() up to
    rounding)."""
    import torch
    blocks = ctypes.c_int32()
    _check(lib().cptr_stream_read(None, x.numel(), None, ctypes.byref(blocks), None))
    if part is None:
        part = torch.empty(blocks.value, dtype=torch.float64, device=x.device)
    _check(lib().cptr_stream_read(_ptr(x), x.numel(), _ptr(part), ctypes.byref(blocks), _stream()))
    return part


def bsr_spmv(row_ptr, col_idx, vals, x, b: int):
    import torch
    rp, ci = _dev(row_ptr, torch.int32), _dev(col_idx, torch.int32)
    v, xx = _dev(vals, torch.float64), _dev(x, torch.float64)
    y = torch.empty_like(xx)
    _check(lib().cptr_bsr_spmv(rp.numel() - 1, b, _ptr(rp), _ptr(ci), _ptr(v), _ptr(xx), _ptr(y), _stream()))
    return y


def condense(row_ptr, col_idx, J11, J12, J21, J22, r1, r2, n1: int, n2: int):
    """Static condensation of the full Newton system (cptr_condense): returns
    the reduced blocks A (nnzb*n1*n1), b (n*n1) and the cell factors Q, q."""
    import torch
    rp, ci = _dev(row_ptr, torch.int32), _dev(col_idx, torch.int32)
    n, nnzb = rp.numel() - 1, ci.numel()
    t = [_dev(x, torch.float64) for x in (J11, J12, J21, J22, r1, r2)]
    dev = t[0].device
    A = torch.empty(nnzb * n1 * n1, dtype=torch.float64, device=dev)
    b = torch.empty(n * n1, dtype=torch.float64, device=dev)
    Q = torch.empty(max(n * n2 * n1, 1), dtype=torch.float64, device=dev)
    q = torch.empty(max(n * n2, 1), dtype=torch.float64, device=dev)
    _check(lib().cptr_condense(n, n1, n2, nnzb, _ptr(rp), _ptr(ci), *[_ptr(x) for x in t], _ptr(A), _ptr(b),
                               _ptr(Q), _ptr(q), _stream()))
    return A, b, Q[: n * n2 * n1], q[: n * n2]


def condense_wells(row_ptr, col_idx, A, b, well_cell, J1w, Jw1, Jww, rw, n1: int, nw: int):
    """Eliminate single-perforation wells in place on the reduced system (A,
    b) (cptr_condense_wells); returns the well factors Qw, qw."""
    import torch
    rp, ci = _dev(row_ptr, torch.int32), _dev(col_idx, torch.int32)
    wc = _dev(well_cell, torch.int32)
    t = [_dev(x, torch.float64) for x in (J1w, Jw1, Jww, rw)]
    W = wc.numel()
    Qw = torch.empty(max(W * nw * n1, 1), dtype=torch.float64, device=A.device)
    qw = torch.empty(max(W * nw, 1), dtype=torch.float64, device=A.device)
    _check(lib().cptr_condense_wells(rp.numel() - 1, n1, ci.numel(), _ptr(rp), _ptr(ci), W, nw, _ptr(wc),
                                     *[_ptr(x) for x in t], _ptr(A), _ptr(b), _ptr(Qw), _ptr(qw), _stream()))
    return Qw[: W * nw * n1], qw[: W * nw]


def recover_wells(well_cell, Qw, qw, delta1, n1: int, nw: int):
    """dw_w = -qw_w - Qw_w d1_{c_w} (cptr_recover_wells)."""
    import torch
    wc = _dev(well_cell, torch.int32)
    d1 = _dev(delta1, torch.float64)
    W = wc.numel()
    dw = torch.empty(max(W * nw, 1), dtype=torch.float64, device=d1.device)
    _check(lib().cptr_recover_wells(W, n1, nw, _ptr(wc), _ptr(Qw), _ptr(qw), _ptr(d1), _ptr(dw), _stream()))
    return dw[: W * nw]


def recover_secondary(Q, q, delta1, n1: int, n2: int):
    """d2_j = -q_j - Q_j d1_j (cptr_recover_secondary)."""
    import torch
    d1 = _dev(delta1, torch.float64)
    n = d1.numel() // n1
    d2 = torch.empty(max(n * n2, 1), dtype=torch.float64, device=d1.device)
    Qd, qd = _dev(Q, torch.float64), _dev(q, torch.float64)
    _check(lib().cptr_recover_secondary(n, n1, n2, _ptr(Qd), _ptr(qd), _ptr(d1), _ptr(d2), _stream()))
    return d2[: n * n2]


def solver_for(system, **opts) -> Solver:
    """Solver set up on a generated system (cell c = x + nx*y on an nx x ny grid)."""
    import torch
    s = Solver(**opts)
    try:
        s.setup(torch.from_numpy(system.row_ptr), torch.from_numpy(system.col_idx),
                torch.from_numpy(system.vals.reshape(-1)), 0, 1, system.nx, system.ny)
    except Exception:
        s.close()
        raise
    return s


class MLP:
    """Trainable edge-MLP of the learned temperature interpolation (device
    FP32 master weights and Adam moments)."""

    def __init__(self, params, device: int = 0):
        import numpy as np
        import torch
        torch.cuda.set_device(device)
        blob = np.ascontiguousarray(params, dtype=np.float32)
        if blob.size != MLP_NPARAMS:
            raise ValueError(f"need {MLP_NPARAMS} parameters, got {blob.size}")
        self.h = ctypes.c_void_p()
        _check(lib().cptr_mlp_create(ctypes.byref(self.h), device, blob.ctypes.data_as(ctypes.c_void_p)))
        _live_solvers.add(self)

    def params(self):
        import numpy as np
        out = np.empty(MLP_NPARAMS, np.float32)
        _check(lib().cptr_mlp_get(self.h, out.ctypes.data_as(ctypes.c_void_p), None))
        return out

    def grad(self):
        import numpy as np
        out = np.empty(MLP_NPARAMS, np.float32)
        _check(lib().cptr_mlp_get(self.h, None, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def train_step(self, solver: "Solver", n_vectors: int = 8, seed: int = 0, lr: float = 1e-3) -> float:
        loss = ctypes.c_double(0.0)
        _check(lib().cptr_mlp_train_step(self.h, solver.ctx, n_vectors, ctypes.c_uint64(seed), lr,
                                         ctypes.byref(loss)))
        return loss.value

    def edges(self, solver: "Solver", with_outputs: bool = True):
        """(features [E, 16], outputs [E] or None) on the solver's temperature edges."""
        import numpy as np
        n = ctypes.c_int32()
        _check(lib().cptr_mlp_edges(self.h, solver.ctx, None, None, 0, ctypes.byref(n)))
        X = np.empty((max(n.value, 1), 16), np.float32)
        o = np.empty(max(n.value, 1), np.float32)
        _check(lib().cptr_mlp_edges(self.h, solver.ctx, X.ctypes.data_as(ctypes.c_void_p),
                                    o.ctypes.data_as(ctypes.c_void_p) if with_outputs else None, n.value,
                                    ctypes.byref(n)))
        return X[: n.value], (o[: n.value] if with_outputs else None)

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _check(lib().cptr_mlp_destroy(self.h))
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
