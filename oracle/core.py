"""Orchestration of the CPU oracle: the stages of the method in the paper's
order, calling the plain C routines of ``orc.c`` for the arithmetic that has a
fixed evaluation order and numpy for vector algebra.

Notation follows the paper (Sec. "Multi-Stage Preconditioning"): ``A`` is the
reduced (primary) system, ``Abar = N^{-1} A`` the left-scaled matrix, ``B_PP``
the pressure block after the first decoupling (Eq. CPTR31), ``C_TT`` the
temperature block after the second (Eq. CPTR32), ``M_i`` the stages of the
right preconditioner (Eq. multistageprec, Algorithms 1 and 2).

TEST INFRASTRUCTURE, like the rest of ``oracle``: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

# option values shared by name with the GPU library's options (plain integers)
CPTR3, CPR, CPTR, BJ_ONLY = 0, 1, 2, 3
T_THEN_P, P_THEN_T = 0, 1
LAST_BILU0, LAST_BJACOBI = 0, 1
GMRES, FGMRES = 0, 1
SMOOTH_JACOBI, SMOOTH_L1JACOBI, SMOOTH_CHEBYSHEV = 0, 1, 2
MAX_REUSE_BACKOFF = 8


def build(force: bool = True) -> str:
    """Compile ``orc.c`` into ``liborc.so`` (plain gcc, contraction off)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        I, D, P, U64 = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_uint64
        sig = {
            "orc_dense_lu_factor": (I, [I, P, P]),
            "orc_dense_lu_solve": (None, [I, P, P, P]),
            "orc_decouple": (I, [I, I, I, P, P, P, P, I, I, P, P, P, P, P]),
            "orc_bsr_spmv": (None, [I, I, P, P, P, P, P]),
            "orc_csr_spmv": (None, [I, P, P, P, P, P]),
            "orc_csr_transpose": (None, [I, I, P, P, P, P, P, P]),
            "orc_spgemm_count": (I, [I, I, P, P, P, P, P]),
            "orc_spgemm_fill": (None, [I, I, P, P, P, P, P, P, P, P, P]),
            "orc_strength": (None, [I, P, P, P, D, P]),
            "orc_splitmix64": (U64, [U64, U64]),
            "orc_pmis": (I, [I, P, P, P, U64, P, P]),
            "orc_exti_count": (I, [I, P, P, P, P, P, I, P]),
            "orc_exti_fill": (None, [I, P, P, P, P, P, I, P, P, P]),
            "orc_bilu0_factor": (I, [I, I, P, P, P, P, P, P]),
            "orc_bilu0_solve": (None, [I, I, P, P, P, P, P, P, P]),
            "orc_bjacobi_factor": (I, [I, I, P, P, P, P]),
            "orc_block_diag_apply": (None, [I, I, P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


# ---------------------------------------------------------------------------
# sparse containers
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class CSR:
    nrows: int
    ncols: int
    rp: np.ndarray
    ci: np.ndarray
    v: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rp[-1])

    def matvec(self, x: np.ndarray) -> np.ndarray:
        x = _f64(x)
        y = np.empty(self.nrows)
        lib().orc_csr_spmv(self.nrows, _p(self.rp), _p(self.ci), _p(self.v), _p(x), _p(y))
        return y

    def diagonal(self) -> np.ndarray:
        d = np.zeros(self.nrows)
        rows = np.repeat(np.arange(self.nrows), np.diff(self.rp))
        m = rows == self.ci
        d[rows[m]] = self.v[m]
        return d

    def transpose(self) -> "CSR":
        rpT = np.empty(self.ncols + 1, np.int32)
        ciT = np.empty(self.nnz, np.int32)
        vT = np.empty(self.nnz)
        lib().orc_csr_transpose(self.nrows, self.ncols, _p(self.rp), _p(self.ci), _p(self.v),
                                _p(rpT), _p(ciT), _p(vT))
        return CSR(self.ncols, self.nrows, rpT, ciT, vT)

    def to_dense(self) -> np.ndarray:
        M = np.zeros((self.nrows, self.ncols))
        rows = np.repeat(np.arange(self.nrows), np.diff(self.rp))
        np.add.at(M, (rows, self.ci), self.v)
        return M


def spgemm(A: CSR, B: CSR) -> CSR:
    """Gustavson product C = A B (orc_spgemm_count / orc_spgemm_fill)."""
    assert A.ncols == B.nrows
    crp = np.empty(A.nrows + 1, np.int32)
    nnz = lib().orc_spgemm_count(A.nrows, B.ncols, _p(A.rp), _p(A.ci), _p(B.rp), _p(B.ci), _p(crp))
    cci = np.empty(max(nnz, 1), np.int32)
    cv = np.empty(max(nnz, 1))
    lib().orc_spgemm_fill(A.nrows, B.ncols, _p(A.rp), _p(A.ci), _p(A.v), _p(B.rp), _p(B.ci), _p(B.v),
                          _p(crp), _p(cci), _p(cv))
    return CSR(A.nrows, B.ncols, crp, cci[:nnz], cv[:nnz])


@dataclasses.dataclass
class BSR:
    n: int
    b: int
    rp: np.ndarray
    ci: np.ndarray
    vals: np.ndarray   # (nnzb, b, b)

    def matvec(self, x: np.ndarray) -> np.ndarray:
        x = _f64(x)
        y = np.empty(self.n * self.b)
        lib().orc_bsr_spmv(self.n, self.b, _p(self.rp), _p(self.ci), _p(self.vals), _p(x), _p(y))
        return y

    def to_dense(self) -> np.ndarray:
        n, b = self.n, self.b
        M = np.zeros((n * b, n * b))
        rows = np.repeat(np.arange(n), np.diff(self.rp))
        for e in range(len(self.ci)):
            i, j = rows[e], self.ci[e]
            M[i * b:(i + 1) * b, j * b:(j + 1) * b] = self.vals[e]
        return M

    def scalar_block(self, r: int, c: int) -> CSR:
        """The scalar matrix of entry (r, c) of every block, on the BSR pattern."""
        return CSR(self.n, self.n, self.rp, self.ci, np.ascontiguousarray(self.vals[:, r, c]))


def bsr_of(system) -> BSR:
    return BSR(system.n, system.b, _i32(system.row_ptr), _i32(system.col_idx), _f64(system.vals))


# ---------------------------------------------------------------------------
# left decoupling (Eq. splitPrec1 with Eqs. CPTR31/CPTR32, CPR, CPTR1)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Decoupled:
    Abar: BSR
    rhsbar: np.ndarray
    wp: np.ndarray      # (n, b)
    wt: np.ndarray      # (n, b)
    beta: np.ndarray    # (n,)
    ip: int
    it: int
    variant: int

    def apply_left(self, v: np.ndarray) -> np.ndarray:
        """N^{-1} v for a cell-interleaved vector (the same factor as on the rows)."""
        n, b, ip, it = self.Abar.n, self.Abar.b, self.ip, self.it
        V = v.reshape(n, b).copy()
        hp = V[:, ip] - np.einsum("ik,ik->i", self.wp, V) if self.variant != BJ_ONLY else V[:, ip]
        out = V.copy()
        out[:, ip] = hp
        if self.variant in (CPTR3, CPTR):
            ht = V[:, it] - np.einsum("ik,ik->i", self.wt, V)
            out[:, it] = ht - self.beta * hp if self.variant == CPTR3 else ht
        return out.reshape(-1)

    def unscale(self, v: np.ndarray) -> np.ndarray:
        """N v: undo the left scaling of a cell-interleaved vector."""
        n, b, ip, it = self.Abar.n, self.Abar.b, self.ip, self.it
        V = v.reshape(n, b).copy()
        if self.variant == BJ_ONLY:
            return v.copy()
        if self.variant == CPTR3:
            V[:, it] = V[:, it] + self.beta * V[:, ip]
        out = V.copy()
        out[:, ip] = V[:, ip] + np.einsum("ik,ik->i", self.wp, V)
        if self.variant in (CPTR3, CPTR):
            out[:, it] = V[:, it] + np.einsum("ik,ik->i", self.wt, V)
        return out.reshape(-1)


def decouple(A: BSR, rhs: np.ndarray, ip: int = 0, it: int = 1, variant: int = CPTR3) -> Decoupled:
    """Per-cell left scaling N^{-1} (see orc_decouple).  ``variant`` BJ_ONLY
    applies no scaling."""
    n, b = A.n, A.b
    if variant == BJ_ONLY:
        return Decoupled(BSR(n, b, A.rp, A.ci, A.vals.copy()), _f64(rhs).copy(),
                         np.zeros((n, b)), np.zeros((n, b)), np.zeros(n), ip, it, variant)
    Abar = np.empty_like(A.vals)
    rb = np.empty(n * b)
    wp = np.empty((n, b)); wt = np.empty((n, b)); beta = np.empty(n)
    rc = lib().orc_decouple(variant, n, b, _p(A.rp), _p(A.ci), _p(A.vals), _p(_f64(rhs)), ip, it,
                            _p(Abar), _p(rb), _p(wp), _p(wt), _p(beta))
    if rc != 0:
        raise OracleError(f"singular decoupling block in cell {-rc - 1}")
    return Decoupled(BSR(n, b, A.rp, A.ci, Abar), rb, wp, wt, beta, ip, it, variant)


# ---------------------------------------------------------------------------
# classical AMG: strength, PMIS, extended+i, Galerkin RAP, V-cycle
# (the AMG sub-solver amg(.) of Eqs. CPRM1, CPTR3M1, CPTRM2)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class AMGOptions:
    theta: float = 0.25
    max_coarse: int = 1000
    max_levels: int = 25
    pmax: int = 4
    smoother: int = SMOOTH_JACOBI
    omega: float = 2.0 / 3.0
    pre: int = 1
    post: int = 1
    cheb_degree: int = 2
    seed: int = 0


@dataclasses.dataclass
class Level:
    A: CSR
    diag: np.ndarray
    P: CSR | None = None
    R: CSR | None = None
    strong: np.ndarray | None = None
    cf: np.ndarray | None = None
    smooth_diag: np.ndarray | None = None
    lam_max: float = 0.0


@dataclasses.dataclass
class Hierarchy:
    levels: list
    lu: np.ndarray
    piv: np.ndarray
    opts: AMGOptions

    @property
    def sizes(self):
        return [L.A.nrows for L in self.levels]

    @property
    def nnzs(self):
        return [L.A.nnz for L in self.levels]

    def operator_complexity(self) -> float:
        return sum(self.nnzs) / self.nnzs[0]


def strength(A: CSR, theta: float) -> np.ndarray:
    s = np.empty(max(A.nnz, 1), np.uint8)
    lib().orc_strength(A.nrows, _p(A.rp), _p(A.ci), _p(A.v), float(theta), _p(s))
    return s[:A.nnz]


def pmis(A: CSR, s: np.ndarray, seed: int) -> tuple[np.ndarray, int]:
    cf = np.empty(A.nrows, np.int32)
    rounds = np.zeros(1, np.int32)
    lib().orc_pmis(A.nrows, _p(A.rp), _p(A.ci), _p(np.ascontiguousarray(s, np.uint8)),
                   ctypes.c_uint64(seed), _p(cf), _p(rounds))
    return cf, int(rounds[0])


def interp_exti(A: CSR, s: np.ndarray, cf: np.ndarray, pmax: int) -> CSR:
    s = np.ascontiguousarray(s, np.uint8)
    cf = _i32(cf)
    prp = np.empty(A.nrows + 1, np.int32)
    nnz = lib().orc_exti_count(A.nrows, _p(A.rp), _p(A.ci), _p(A.v), _p(s), _p(cf), int(pmax), _p(prp))
    pci = np.empty(max(nnz, 1), np.int32)
    pv = np.empty(max(nnz, 1))
    lib().orc_exti_fill(A.nrows, _p(A.rp), _p(A.ci), _p(A.v), _p(s), _p(cf), int(pmax), _p(prp),
                        _p(pci), _p(pv))
    nc = int(cf.sum())
    return CSR(A.nrows, nc, prp, pci[:nnz], pv[:nnz])


def galerkin(A: CSR, P: CSR, R: CSR) -> CSR:
    """A_c = R (A P), both products by Gustavson."""
    return spgemm(R, spgemm(A, P))


def amg_setup(A: CSR, opts: AMGOptions | None = None) -> Hierarchy:
    """Classical AMG hierarchy: strength -> PMIS -> extended+i (+ truncation)
    -> R = P^T -> A_c = R A P, until the level has at most ``max_coarse`` rows,
    ``max_levels`` is reached or coarsening stalls; the coarsest level is
    factored densely (LU with partial pivoting)."""
    opts = opts or AMGOptions()
    levels = []
    cur = A
    while True:
        L = Level(cur, cur.diagonal())
        levels.append(L)
        if cur.nrows <= opts.max_coarse or len(levels) >= opts.max_levels:
            break
        s = strength(cur, opts.theta)
        cf, _ = pmis(cur, s, opts.seed)
        nc = int(cf.sum())
        if nc == 0 or nc == cur.nrows:
            break
        P = interp_exti(cur, s, cf, opts.pmax)
        R = P.transpose()
        L.P, L.R, L.strong, L.cf = P, R, s, cf
        cur = galerkin(cur, P, R)
    return _finish_hierarchy(levels, opts)


# ---------------------------------------------------------------------------
# unknown-based system AMG for the 2x2 elliptic block B_ee of the two-stage
# CPTR scheme (Sec. "Two-stage Constrained Pressure-Temperature Residual";
# the system-AMG direction of the conclusions)
# ---------------------------------------------------------------------------

def elliptic_system(Abar: BSR, ip: int = 0, it: int = 1) -> CSR:
    """B_ee = [[B_PP, B_PT], [B_TP, B_TT]] of the scaled matrix as one scalar
    CSR of 2n rows, unknowns ordered [P of every cell; T of every cell]; a
    row holds its P-block columns, then its T-block columns (shifted by n)."""
    n = Abar.n
    rp, ci = Abar.rp.astype(np.int64), Abar.ci.astype(np.int64)
    cnt = np.diff(rp)
    srp = np.concatenate([[0], np.cumsum(np.concatenate([2 * cnt, 2 * cnt]))])
    nnzb = ci.size
    rows = np.repeat(np.arange(n), cnt)
    t = np.arange(nnzb) - rp[rows]
    sci = np.empty(4 * nnzb, np.int64)
    sv = np.empty(4 * nnzb)
    for u, ru in enumerate((ip, it)):
        base = srp[u * n + rows]
        sci[base + t] = ci
        sv[base + t] = Abar.vals[:, ru, ip]
        sci[base + cnt[rows] + t] = ci + n
        sv[base + cnt[rows] + t] = Abar.vals[:, ru, it]
    return CSR(2 * n, 2 * n, _i32(srp), _i32(sci), sv)


def submatrix(A: CSR, o: int, m: int) -> CSR:
    """Rows and columns [o, o + m) of A, columns shifted by -o (order kept)."""
    a, b_ = int(A.rp[o]), int(A.rp[o + m])
    rows = np.repeat(np.arange(m), np.diff(A.rp[o:o + m + 1]))
    c = A.ci[a:b_]
    keep = (c >= o) & (c < o + m)
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=m))])
    return CSR(m, m, _i32(rp), _i32(c[keep] - o), _f64(A.v[a:b_][keep]))


def block_diagonal(Ps: list) -> CSR:
    """blockdiag(P_0, P_1, ...): rows and columns of each block after the previous ones."""
    rp = [np.zeros(1, np.int64)]
    ci, v = [], []
    r0 = c0 = nz = 0
    for P in Ps:
        rp.append(P.rp[1:].astype(np.int64) + nz)
        ci.append(P.ci.astype(np.int64) + c0)
        v.append(P.v)
        nz += P.nnz
        r0 += P.nrows
        c0 += P.ncols
    return CSR(r0, c0, _i32(np.concatenate(rp)), _i32(np.concatenate(ci)), _f64(np.concatenate(v)))


def amg_setup_system(A: CSR, parts: list, opts: AMGOptions | None = None) -> Hierarchy:
    """Unknown-based AMG: A holds len(parts) unknowns in consecutive row
    ranges.  On every level each unknown's diagonal block is coarsened on its
    own (strength, PMIS and extended+i with truncation as in amg_setup, the
    PMIS measure indexed within the block), P = blockdiag(P_u), R = P^T and
    A_c = R A P keeps every coupling between the unknowns.  Coarsening stops
    when the level has at most ``max_coarse`` rows, at ``max_levels``, or when
    some unknown's block stalls (no C point, or no F point); the coarsest
    level is factored densely."""
    opts = opts or AMGOptions()
    levels = []
    cur = A
    parts = list(parts)
    while True:
        L = Level(cur, cur.diagonal())
        levels.append(L)
        if cur.nrows <= opts.max_coarse or len(levels) >= opts.max_levels:
            break
        Ps, cfs, ss, ncs = [], [], [], []
        o = 0
        stalled = False
        for m in parts:
            Au = submatrix(cur, o, m)
            s = strength(Au, opts.theta)
            cf, _ = pmis(Au, s, opts.seed)
            nc = int(cf.sum())
            if nc == 0 or nc == m:
                stalled = True
                break
            Ps.append(interp_exti(Au, s, cf, opts.pmax))
            cfs.append(cf)
            ss.append(s)
            ncs.append(nc)
            o += m
        if stalled:
            break
        P = block_diagonal(Ps)
        R = P.transpose()
        L.P, L.R, L.cf = P, R, np.concatenate(cfs)
        L.strong = ss
        cur = galerkin(cur, P, R)
        parts = ncs
    return _finish_hierarchy(levels, opts)


class SystemStage:
    """M_ee^{-1} of the two-stage CPTR scheme (Eq. CPTRM1 with the elliptic
    block): gather the P and T components of every cell into [r_P; r_T],
    apply ``solve`` to B_ee, scatter back with zeros elsewhere."""

    def __init__(self, n: int, b: int, ip: int, it: int, solve):
        self.n, self.b, self.ip, self.it, self.solve = n, b, ip, it, solve

    def __call__(self, r: np.ndarray) -> np.ndarray:
        n, b = self.n, self.b
        x = self.solve(np.concatenate([r[self.ip::b], r[self.it::b]]))
        y = np.zeros(n * b)
        y[self.ip::b] = x[:n]
        y[self.it::b] = x[n:]
        return y


def _finish_hierarchy(levels: list, opts: AMGOptions) -> Hierarchy:
    """Smoother data of every level but the last; dense LU of the last."""
    for L in levels[:-1]:
        _smoother_setup(L, opts)
    Ac = levels[-1].A.to_dense()
    piv = np.zeros(Ac.shape[0], np.int32)
    lu = np.ascontiguousarray(Ac)
    if lib().orc_dense_lu_factor(Ac.shape[0], _p(lu), _p(piv)) != 0:
        raise OracleError("singular coarsest AMG level")
    return Hierarchy(levels, lu, piv, opts)


def amg_refresh(h: Hierarchy, A: CSR, P0: CSR | None = None) -> Hierarchy:
    """Reuse of hierarchy ``h`` for new level-0 values ``A`` on the same
    pattern (the next system of a Newton sequence): the C/F splits and the
    transfer operators P, R = P^T of every level are kept; the Galerkin
    products A_{l+1} = R A_l P, the smoother data and the coarsest LU are
    recomputed from the new values.  ``P0`` (optional) replaces the fine
    level's interpolation by other weights on the same C/F split (the learned
    interpolation), with R_0 = P0^T; the coarser levels keep h's splits and
    transfer operators."""
    levels = []
    cur = A
    for l, old in enumerate(h.levels):
        P, R = old.P, old.R
        if l == 0 and P0 is not None and P is not None:
            P, R = P0, P0.transpose()
        L = Level(cur, cur.diagonal(), P, R, old.strong, old.cf)
        levels.append(L)
        if P is None:
            break
        cur = galerkin(cur, P, R)
    return _finish_hierarchy(levels, h.opts)


def _smoother_setup(L: Level, opts: AMGOptions) -> None:
    A = L.A
    if opts.smoother == SMOOTH_L1JACOBI:
        # l1-Jacobi: d_i = a_ii + sign(a_ii) sum_{j != i} |a_ij|
        rows = np.repeat(np.arange(A.nrows), np.diff(A.rp))
        off = np.where(rows != A.ci, np.abs(A.v), 0.0)
        l1 = np.bincount(rows, weights=off, minlength=A.nrows)
        sg = np.where(L.diag < 0, -1.0, 1.0)
        L.smooth_diag = L.diag + sg * l1
    else:
        L.smooth_diag = L.diag.copy()
    if opts.smoother == SMOOTH_CHEBYSHEV:
        # Gershgorin bound on the spectrum of D^{-1} A
        rows = np.repeat(np.arange(A.nrows), np.diff(A.rp))
        rs = np.bincount(rows, weights=np.abs(A.v), minlength=A.nrows)
        L.lam_max = float(np.max(rs / np.abs(L.diag)))


def coarse_solve(h: Hierarchy, b: np.ndarray) -> np.ndarray:
    f = _f64(b).copy()
    lib().orc_dense_lu_solve(h.lu.shape[0], _p(h.lu), _p(h.piv), _p(f))
    return f


def smooth(L: Level, opts: AMGOptions, b: np.ndarray, x: np.ndarray | None, sweeps: int) -> np.ndarray:
    """``sweeps`` smoothing steps on A x = b from x (None = zero guess)."""
    if opts.smoother == SMOOTH_CHEBYSHEV:
        return _chebyshev(L, b, x, opts.cheb_degree * sweeps)
    d = L.smooth_diag
    w = opts.omega if opts.smoother == SMOOTH_JACOBI else 1.0
    for _ in range(sweeps):
        if x is None:
            x = w * b / d
        else:
            x = x + w * (b - L.A.matvec(x)) / d
    return x


def _chebyshev(L: Level, b: np.ndarray, x: np.ndarray | None, degree: int) -> np.ndarray:
    """Chebyshev iteration on D^{-1} A over [lmax/30, 1.1 lmax] (three-term
    recurrence of Saad, Iterative Methods, Alg. 12.1)."""
    lmax = 1.1 * L.lam_max
    lmin = L.lam_max / 30.0
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = L.diag
    x = np.zeros_like(b) if x is None else x.copy()
    r = (b - L.A.matvec(x)) / d
    dk = r / theta
    for _ in range(degree):
        x = x + dk
        r = r - L.A.matvec(dk) / d
        rho_new = 1.0 / (2.0 * sigma - rho)
        dk = rho_new * rho * dk + (2.0 * rho_new / delta) * r
        rho = rho_new
    return x


def vcycle(h: Hierarchy, b: np.ndarray, lvl: int = 0, x0: np.ndarray | None = None) -> np.ndarray:
    """One V-cycle for A x = b (zero initial guess unless x0 is given):
    pre-smooth, residual, restrict by R, recurse, prolong by P, post-smooth;
    the coarsest level is solved directly."""
    opts = h.opts
    if lvl == len(h.levels) - 1:
        if x0 is None:
            return coarse_solve(h, b)
        return x0 + coarse_solve(h, b - h.levels[lvl].A.matvec(x0))
    L = h.levels[lvl]
    x = smooth(L, opts, b, x0, opts.pre)
    r = b - L.A.matvec(x)
    xc = vcycle(h, L.R.matvec(r), lvl + 1)
    x = x + L.P.matvec(xc)
    x = smooth(L, opts, b, x, opts.post)
    return x


def conv_factor(h: Hierarchy, cycles: int = 10, seed: int = 0) -> float:
    """Asymptotic V-cycle convergence factor on A e = 0: e <- e - V(A e)
    from a SplitMix64-uniform start in (-1, 1); rho = (|e_K|/|e_0|)^(1/K)."""
    n = h.levels[0].A.nrows
    u = _splitmix_vec(seed, n)
    e = (u >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0
    e0 = np.linalg.norm(e)
    A = h.levels[0].A
    for _ in range(cycles):
        e = e - vcycle(h, A.matvec(e))
    return float((np.linalg.norm(e) / e0) ** (1.0 / cycles))


def _splitmix_vec(seed: int, n: int) -> np.ndarray:
    """Vectorised SplitMix64 (same definition as orc_splitmix64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.arange(n, dtype=np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


# ---------------------------------------------------------------------------
# last stage: block ILU(0) / block Jacobi on Abar  (ilu(Abar) of Eq. CPTR3M3)
# ---------------------------------------------------------------------------

def rank_from_colors(color: np.ndarray) -> np.ndarray:
    """Elimination order: colour ascending, cell index ascending inside a
    colour.  Colour = x + y gives the natural (lexicographic) order's level
    sets; colour = (x + y) mod 2 gives red-black."""
    order = np.lexsort((np.arange(len(color)), color))
    rank = np.empty(len(color), np.int32)
    rank[order] = np.arange(len(color), dtype=np.int32)
    return rank


def tile_colors(nx: int, ny: int, tile_x: int = 32, tile_y: int = 8) -> np.ndarray:
    """Red-black colouring of tile_x x tile_y tiles of the grid (cell c = x + nx y):
    colour ((x // tile_x) + (y // tile_y)) mod 2.  With rank_from_colors this
    orders all red tiles before all black tiles and keeps the natural order
    inside every tile; a single tile covering the grid is the natural order."""
    x = np.arange(nx)[None, :] // tile_x
    y = np.arange(ny)[:, None] // tile_y
    return ((x + y) % 2).astype(np.int32).reshape(-1)


class BlockILU0:
    def __init__(self, A: BSR, rank: np.ndarray):
        self.A, self.rank = A, _i32(rank)
        self.F = np.empty_like(A.vals)
        self.dinv = np.empty((A.n, A.b, A.b))
        rc = lib().orc_bilu0_factor(A.n, A.b, _p(A.rp), _p(A.ci), _p(A.vals), _p(self.rank),
                                    _p(self.F), _p(self.dinv))
        if rc != 0:
            raise OracleError(f"singular BILU(0) pivot block in cell {-rc - 1}")

    def __call__(self, u: np.ndarray) -> np.ndarray:
        w = np.empty(self.A.n * self.A.b)
        A = self.A
        lib().orc_bilu0_solve(A.n, A.b, _p(A.rp), _p(A.ci), _p(self.F), _p(self.dinv), _p(self.rank),
                              _p(_f64(u)), _p(w))
        return w


class BlockJacobi:
    def __init__(self, A: BSR):
        self.A = A
        self.dinv = np.empty((A.n, A.b, A.b))
        rc = lib().orc_bjacobi_factor(A.n, A.b, _p(A.rp), _p(A.ci), _p(A.vals), _p(self.dinv))
        if rc != 0:
            raise OracleError(f"singular diagonal block in cell {-rc - 1}")

    def __call__(self, u: np.ndarray) -> np.ndarray:
        w = np.empty(self.A.n * self.A.b)
        lib().orc_block_diag_apply(self.A.n, self.A.b, _p(self.dinv), _p(_f64(u)), _p(w))
        return w


# ---------------------------------------------------------------------------
# multi-stage right preconditioner (Eq. multistageprec, Algorithms 1 and 2)
# ---------------------------------------------------------------------------

class ScalarStage:
    """M_i^{-1} that acts on one unknown of every cell (Eqs. CPRM1, CPTR3M1,
    CPTRM2): gather that component, apply ``solve`` to the scalar subsystem,
    scatter back with zeros elsewhere."""

    def __init__(self, n: int, b: int, comp: int, solve):
        self.n, self.b, self.comp, self.solve = n, b, comp, solve

    def __call__(self, r: np.ndarray) -> np.ndarray:
        y = np.zeros(self.n * self.b)
        y[self.comp::self.b] = self.solve(np.ascontiguousarray(r[self.comp::self.b]))
        return y


def multistage_apply(Abar: BSR, stages: list, r: np.ndarray) -> np.ndarray:
    """y = M^{-1} r for the multi-stage preconditioner: Algorithm 1 for two
    stages, Algorithm 2 for three (written for any number of stages: apply a
    stage to the current residual, add its output to y, update the residual
    with Abar)."""
    y = stages[0](r)
    if len(stages) == 1:
        return y
    z = r - Abar.matvec(y)
    for k, M in enumerate(stages[1:]):
        v = M(z)
        y = y + v
        if k + 2 < len(stages):
            z = z - Abar.matvec(v)
    return y


def multistage_apply_alg2(Abar: BSR, M1, M2, M3, r: np.ndarray) -> np.ndarray:
    """Algorithm 2 exactly as printed: x = M1 r; z = r - Abar x; v = M2 z;
    u = z - Abar v; y = x + v + M3 u."""
    x = M1(r)
    z = r - Abar.matvec(x)
    v = M2(z)
    u = z - Abar.matvec(v)
    return x + v + M3(u)


# ---------------------------------------------------------------------------
# right-preconditioned restarted GMRES / FGMRES
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class GmresResult:
    x: np.ndarray
    iterations: int
    restarts: int
    converged: bool
    history: list
    true_rel_res: float
    breakdown: bool = False


def gmres(matvec, b: np.ndarray, M, restart: int = 30, rtol: float = 1e-8, max_iters: int = 1000,
          flexible: bool = False, unscaled=None) -> GmresResult:
    """Right-preconditioned GMRES(m) (Saad & Schultz; right preconditioning as in
    the paper's split form Eq. splitPrec2) with x0 = 0, modified Gram-Schmidt
    Arnoldi and Givens rotations.  Stops inside a cycle when the Givens
    residual estimate |g_{j+1}| <= rtol |b|, then forms x and checks the true
    residual |b - A x| <= rtol |b|; restarts otherwise.  ``flexible`` stores the
    preconditioned vectors Z and updates x += Z y (FGMRES, Saad 1993); the
    plain variant updates x += M^{-1}(V y).  Happy breakdown when
    h_{j+1,j} <= 1e-14 |A z_j|.  Iterations count Arnoldi steps.

    ``unscaled`` (optional): a function of x returning the relative residual
    of the unscaled system, |b0 - A0 x| / |b0|; the solve then also requires
    it to be <= rtol.  When a cycle ends with that residual above rtol, the
    cycles that follow stop their Givens estimate at
    min(target, |r| (rtol / unscaled(x)) / 2) instead of rtol |b| (the scaled
    residual needed for the unscaled one, if the two stay proportional, with
    a factor 2 of margin)."""
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = float(np.linalg.norm(b))
    history = []
    its = 0
    restarts = 0
    if bnorm == 0.0:
        return GmresResult(x, 0, 0, True, [], 0.0)
    r = b.copy()
    beta = bnorm
    breakdown = False
    target = rtol * bnorm
    while True:
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n)) if flexible else None
        H = np.zeros((m + 1, m))
        cs = np.zeros(m); sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            z = M(V[j])
            if flexible:
                Z[j] = z
            w = matvec(z)
            wnorm0 = float(np.linalg.norm(w))
            for i in range(j + 1):
                H[i, j] = float(np.dot(V[i], w))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            hj1 = H[j + 1, j]
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if hj1 <= 1e-14 * wnorm0:
                breakdown = True
                break
            if abs(g[j + 1]) <= target or its >= max_iters:
                break
            V[j + 1] = w / hj1
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        if flexible:
            x = x + Z[:k].T @ y
        else:
            x = x + M(V[:k].T @ y)
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        true_rel = beta / bnorm
        ok = true_rel <= rtol
        if unscaled is not None:
            ru = unscaled(x)
            if ru > rtol:
                ok = False
                target = min(target, beta * (rtol / ru) * 0.5)
        if ok:
            return GmresResult(x, its, restarts, True, history, true_rel, breakdown)
        if its >= max_iters or (breakdown and beta == 0.0):
            return GmresResult(x, its, restarts, False, history, true_rel, breakdown)
        restarts += 1
        breakdown = False


# ---------------------------------------------------------------------------
# the whole path
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Options:
    variant: int = CPTR3
    stage_order: int = T_THEN_P
    last_stage: int = LAST_BILU0
    color: np.ndarray | None = None      # elimination colouring for BILU(0); None = natural order
    krylov: int = GMRES
    restart: int = 30
    max_iters: int = 1000
    rtol: float = 1e-8
    amg: AMGOptions = dataclasses.field(default_factory=AMGOptions)
    exact_subsolves: bool = False        # replace amg(.) by direct solves (the paper's exact study)
    exact_last_stage: bool = False       # replace ilu(Abar) by an exact solve (tests only)
    reuse_rho_max: float = 0.3           # keep a reused AMG hierarchy while rho < this
    rho_cycles: int = 10                 # V-cycles of the reuse test's factor
    judge_cycles: int = 4                # V-cycles of the learned interpolation's judge
    mlp_params: np.ndarray | None = None # learned T-interpolation weights (None = classical only)
    stop_unscaled: bool = False          # also require |b - A x| <= rtol |b| (unscaled system)


@dataclasses.dataclass
class SolveResult:
    x: np.ndarray
    iterations: int
    restarts: int
    converged: bool
    rel_res_scaled: float
    rel_res_unscaled: float
    history: list
    hierarchies: dict
    dec: Decoupled
    rho: dict = dataclasses.field(default_factory=dict)      # measured for reused hierarchies
    reused: dict = dataclasses.field(default_factory=dict)   # name -> kept?
    # name -> (skip, backoff)
    reuse_state: dict = dataclasses.field(default_factory=dict)
    learned: dict = dataclasses.field(default_factory=dict)  # judge of the learned interpolation


DIRECT_DENSE_MAX = 4096


class _Direct:
    """Direct solve of a scalar CSR system (the paper's exact sub-solves):
    dense LU with partial pivoting up to DIRECT_DENSE_MAX rows, above it the
    sparse LU of SuperLU (scipy.sparse.linalg.splu, partial pivoting) as a
    library step; both are exact solves up to rounding."""

    def __init__(self, A: CSR):
        self.sparse = None
        if A.nrows > DIRECT_DENSE_MAX:
            import scipy.sparse as sp
            from scipy.sparse.linalg import splu
            M = sp.csr_matrix((A.v, A.ci, A.rp), shape=(A.nrows, A.ncols)).tocsc()
            self.sparse = splu(M)
            return
        self.lu = np.ascontiguousarray(A.to_dense())
        self.piv = np.zeros(A.nrows, np.int32)
        if lib().orc_dense_lu_factor(A.nrows, _p(self.lu), _p(self.piv)) != 0:
            raise OracleError("singular subsystem")

    def __call__(self, b):
        if self.sparse is not None:
            return self.sparse.solve(_f64(b).copy())
        f = _f64(b).copy()
        lib().orc_dense_lu_solve(self.lu.shape[0], _p(self.lu), _p(self.piv), _p(f))
        return f


def build_preconditioner(dec: Decoupled, opts: Options, previous: dict | None = None,
                         info: dict | None = None):
    """The stages of the chosen variant on Abar, in the paper's order:
    CPTR3: M1 = amg(C_TT), M2 = amg(B_PP), M3 = ilu(Abar) (Eqs. CPTR3M1,
    CPTRM2, CPTR3M3); CPR: M1 = amg(B_PP), M2 = ilu(Abar) (Eqs. CPRM1 ff.);
    CPTR: M1 = unknown-based system amg(B_ee), M2 = ilu(Abar) (two-stage
    CPTR, Algorithm 1); BJ_ONLY: the last stage alone.  Returns (apply, stages, hierarchies).

    ``previous`` (name -> Hierarchy of the previous system of a sequence)
    switches on reuse: each scalar stage first refreshes the previous
    hierarchy with the new values and measures its V-cycle convergence
    factor; it is kept if rho < opts.reuse_rho_max, else rebuilt.  The
    factors and decisions are written into ``info["rho"]``, ``info["reused"]``.
    After a rejected trial the next ``skip`` systems rebuild without a trial,
    ``skip`` doubling (up to MAX_REUSE_BACKOFF) with each rejection in a row
    and resetting to 1 on acceptance; ``info["state"]`` carries (skip,
    backoff) per stage in and out.  Every full build of the temperature
    hierarchy with learned parameters judges the learned interpolation
    against the classical one (``info["learned"]``)."""
    Abar = dec.Abar
    n, b, ip, it = Abar.n, Abar.b, dec.ip, dec.it
    hier = {}

    def scalar_solver(name, comp):
        A = Abar.scalar_block(comp, comp)
        if opts.exact_subsolves:
            return _Direct(A)
        h = None
        skip, backoff = (info or {}).get("state", {}).get(name, (0, 1))
        if previous and name in previous and opts.reuse_rho_max > 0:
            if skip > 0:
                skip -= 1                   # rebuild without a trial
            else:
                hr = amg_refresh(previous[name], A)
                rho = conv_factor(hr, opts.rho_cycles, 0)
                keep = rho < opts.reuse_rho_max
                if info is not None:
                    info.setdefault("rho", {})[name] = rho
                    info.setdefault("reused", {})[name] = keep
                if keep:
                    h = hr
                    backoff = 1
                else:
                    skip, backoff = backoff, min(2 * backoff, MAX_REUSE_BACKOFF)
        else:
            skip, backoff = 0, 1
        if info is not None:
            info.setdefault("state", {})[name] = (skip, backoff)
        if h is None:
            h = amg_setup(A, opts.amg)
            if name == "T" and opts.mlp_params is not None and len(h.levels) > 1:
                # the learned fine-level interpolation, judged at every full
                # build by the V-cycle convergence factor against the
                # classical one: kept only when its factor is lower.  The
                # learned hierarchy differs from the classical one only in
                # the fine level's weights (coarser levels: the classical
                # C/F splits and transfer operators, Galerkin products
                # formed from the learned fine level down)
                from .learned import learned_hierarchy
                hl = learned_hierarchy(opts.mlp_params, h)
                rc = conv_factor(h, opts.judge_cycles, 0)
                rl = conv_factor(hl, opts.judge_cycles, 0)
                use = rl < rc
                if info is not None:
                    info["learned"] = dict(used=use, rho_classical=rc, rho_learned=rl)
                if use:
                    h = hl
        hier[name] = h
        return lambda rr, h=h: vcycle(h, rr)

    if opts.exact_last_stage:
        dense = Abar.to_dense()
        lu = np.ascontiguousarray(dense)
        piv = np.zeros(dense.shape[0], np.int32)
        lib().orc_dense_lu_factor(dense.shape[0], _p(lu), _p(piv))

        def last(u, lu=lu, piv=piv):
            f = _f64(u).copy()
            lib().orc_dense_lu_solve(lu.shape[0], _p(lu), _p(piv), _p(f))
            return f
    elif opts.last_stage == LAST_BJACOBI:
        last = BlockJacobi(Abar)
    else:
        color = opts.color
        if color is None:
            color = np.arange(n, dtype=np.int32)       # natural order
        last = BlockILU0(Abar, rank_from_colors(np.asarray(color)))

    stages = []
    if opts.variant == CPTR3:
        sT = ScalarStage(n, b, it, scalar_solver("T", it))
        sP = ScalarStage(n, b, ip, scalar_solver("P", ip))
        stages = [sT, sP] if opts.stage_order == T_THEN_P else [sP, sT]
    elif opts.variant == CPR:
        stages = [ScalarStage(n, b, ip, scalar_solver("P", ip))]
    elif opts.variant == CPTR:
        # two stages: system AMG on B_ee, then the last stage
        B = elliptic_system(Abar, ip, it)
        if opts.exact_subsolves:
            ee = _Direct(B)
        else:
            h = amg_setup_system(B, [n, n], opts.amg)
            hier["ee"] = h
            ee = lambda rr, h=h: vcycle(h, rr)  # noqa: E731
        stages = [SystemStage(n, b, ip, it, ee)]
    stages.append(last)
    return (lambda r: multistage_apply(Abar, stages, r)), stages, hier


def solve(system, opts: Options | None = None, ip: int = 0, it: int = 1,
          previous: "SolveResult | None" = None) -> SolveResult:
    """Left-scale (Eq. splitPrec1), build the right preconditioner, run
    right-preconditioned GMRES/FGMRES on Abar x = bbar (Eq. splitPrec2).
    ``previous``: the result for the previous system of a sequence on the same
    pattern, whose AMG hierarchies are offered for reuse."""
    opts = opts or Options()
    A = bsr_of(system)
    dec = decouple(A, system.rhs, ip, it, opts.variant)
    info = {"state": dict(previous.reuse_state) if previous else {}}
    apply, _, hier = build_preconditioner(dec, opts, previous.hierarchies if previous else None, info)
    bn0 = float(np.linalg.norm(system.rhs))
    unscaled = None
    if opts.stop_unscaled and bn0 > 0:
        unscaled = lambda x: float(np.linalg.norm(system.rhs - A.matvec(x))) / bn0  # noqa: E731
    res = gmres(dec.Abar.matvec, dec.rhsbar, apply, opts.restart, opts.rtol, opts.max_iters,
                flexible=(opts.krylov == FGMRES), unscaled=unscaled)
    r = system.rhs - A.matvec(res.x)
    unscaled = float(np.linalg.norm(r) / np.linalg.norm(system.rhs))
    return SolveResult(res.x, res.iterations, res.restarts, res.converged, res.true_rel_res, unscaled,
                       res.history, hier, dec, info.get("rho", {}), info.get("reused", {}), info.get("state", {}),
                       info.get("learned", {}))
