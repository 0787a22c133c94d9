"""Seeded synthetic linear systems shaped like the reduced thermal-compositional
Jacobians the multi-stage preconditioner is built for.

This module only *produces inputs*.  It holds none of the solver's arithmetic
(no decoupling, no AMG, no ILU, no Krylov); both the CPU oracle and the GPU
library consume what it returns.

What the paper fixes and what is a reading of ours
--------------------------------------------------
* Cell-interleaved ordering with small dense blocks per cell (Sec. "Constrained
  Pressure Residual", remark on interleaving): the matrix is BSR, one b x b
  block per pair of coupled cells, unknowns per cell ordered
  ``[p, T, c_1 .. c_{b-2}]``.
* Pressure rows are elliptic (mass conservation under Darcy flow, Eq. Darcy),
  temperature rows combine conduction and advection (Eq. energy), composition
  rows are advective transport; the thermal Peclet number Pe = u L rho c_p / kappa
  (Eq. pe) sets the balance, and like the paper we vary only the conductivity
  to move Pe.
* Everything else (stencil, permeability fields, coupling magnitudes, the
  combustion band) is a stand-in for the simulator output the paper uses and
  that is not available here; the recipe is written out in each function.

Layout of a generated system (all numpy, host memory):
  row_ptr  int32 [n+1]     block-row pointers
  col_idx  int32 [nnzb]    block columns, ascending within a row
  vals     float64 [nnzb, b, b]  row-major dense blocks
  rhs      float64 [n*b]   right-hand side, cell-interleaved
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Index of the pressure and temperature unknowns inside a cell block.
P_INDEX = 0
T_INDEX = 1


@dataclasses.dataclass
class BSRSystem:
    nx: int
    ny: int
    b: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    vals: np.ndarray
    rhs: np.ndarray
    meta: dict

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])

    def checkerboard(self) -> np.ndarray:
        """Two-colouring of the 5-point grid graph: colour (x + y) mod 2."""
        x = np.arange(self.nx)[None, :]
        y = np.arange(self.ny)[:, None]
        return ((x + y) % 2).astype(np.int32).reshape(-1)

    def antidiagonals(self) -> np.ndarray:
        """Level sets x + y of the natural (x fastest) ordering of the grid."""
        x = np.arange(self.nx)[None, :]
        y = np.arange(self.ny)[:, None]
        return (x + y).astype(np.int32).reshape(-1)


# ---------------------------------------------------------------------------
# permeability fields
# ---------------------------------------------------------------------------

def gaussian_field(rng: np.random.Generator, nx: int, ny: int, corr_len: float) -> np.ndarray:
    """Unit-variance Gaussian random field: white noise filtered (periodic FFT
    convolution) with the kernel exp(-r^2 / l^2), then shifted and scaled to
    mean 0 and standard deviation 1.  Shape (ny, nx)."""
    noise = rng.standard_normal((ny, nx))
    dx = np.minimum(np.arange(nx), nx - np.arange(nx)).astype(np.float64)
    dy = np.minimum(np.arange(ny), ny - np.arange(ny)).astype(np.float64)
    r2 = dy[:, None] ** 2 + dx[None, :] ** 2
    kern = np.exp(-r2 / (corr_len * corr_len))
    g = np.fft.irfft2(np.fft.rfft2(noise) * np.fft.rfft2(kern), s=(ny, nx))
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g /= sd
    return g


def channel_indicator(nx: int, ny: int) -> np.ndarray:
    """Sinusoidal high-permeability bands: chi = [sin(2 pi (y + 8 sin(2 pi x/250))/50) > 0.6]."""
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    arg = 2.0 * math.pi * (y + 8.0 * np.sin(2.0 * math.pi * x / 250.0)) / 50.0
    return (np.sin(arg) > 0.6).astype(np.float64)


def permeability(kind: str, nx: int, ny: int, rng: np.random.Generator,
                 ln_sigma: float = 1.0, corr_len: float = 10.0) -> np.ndarray:
    if kind == "homogeneous":
        return np.ones((ny, nx))
    lnk = ln_sigma * gaussian_field(rng, nx, ny, corr_len)
    if kind == "lognormal":
        return np.exp(lnk)
    if kind == "channelised":
        return np.exp(lnk + math.log(100.0) * channel_indicator(nx, ny))
    raise ValueError(f"unknown permeability kind {kind!r}")


# ---------------------------------------------------------------------------
# assembly
# ---------------------------------------------------------------------------

def _harmonic(a: np.ndarray, c: np.ndarray) -> np.ndarray:
    return 2.0 * a * c / (a + c)


def assemble(nx: int, ny: int, b: int, perm: np.ndarray, *, peclet: float,
             k_thermal: float | None = None, dt: float = 1e-2,
             coupling: float = 0.1, seed: int = 0,
             field_seed: int | None = None, band: tuple[int, int, float] | None = None,
             zero_coupling: bool = False, flow: bool = True,
             transmissibility: bool = True, coupling_ref: str = "flux",
             heat_capacity: float = 1.0) -> BSRSystem:
    """Assemble the BSR system on an nx x ny grid of unit cells (index c = x + nx*y).

    Stencil: two-point flux 5-point, no-flow outer boundary.  Per interior face f
    between cells a and c:
      * transmissibility T_f = 2 k_a k_c / (k_a + k_c);
      * a constant driving gradient along (1,1)/sqrt(2) gives a flux F_f
        proportional to T_f, directed to +x / +y, normalised so the face mean
        |F_f| is 1; the upwind cell of a face is its west / south cell.
    Peclet number Pe = rho c_p * u * L / K_T with u = 1 and L = nx.  If
    ``k_thermal`` is given it is kept and rho c_p is chosen to hit Pe; otherwise
    rho c_p = 1 and K_T = L / Pe (only the conductivity varies, like the paper).
    Accumulation: acc = 1e-3 / dt on the pressure and composition diagonals;
    the energy rows carry the heat capacity of the rock-fluid system,
    acc_T = heat_capacity / dt (the accumulation term of the energy balance,
    Eq. energy; volumetric heat capacity 1 in the units where rho c_p = 1).

    Principal (same-unknown) entries, J a neighbour of I across f:
      pressure row    diag acc + sum_f T_f,                  off-diag -T_f
      temperature row diag acc_T + sum_f K_T + rcp sum_out F, off-diag -K_T - rcp F_f [J upwind of I]
      composition row diag acc + sum_out F,                  off-diag -F_f [J upwind of I]
    Cross-unknown entries (``coupling_ref="flux"``, the default): conservative
      face couplings, see ``_flux_couplings``.  Alternative readings kept for
      comparison: "row" sets A_IJ[r, c] = xi * A_IJ[r, r] and "col" sets
      A_IJ[r, c] = xi * A_IJ[c, c] on every stored block independently; both
      break conservation, and with the near-incompressible pressure
      accumulation the decoupled pressure block then turns indefinite.
    ``band = (x0, x1, factor)`` multiplies A_II[T, T] by ``factor`` for x0 <= x < x1
    (the moving combustion front of the Newton sequence).

    Random streams (numpy PCG64): field [field_seed, 1], coupling [seed, 2], rhs [seed, 3].
    ``perm`` is the (ny, nx) permeability (drawn by the caller from stream 1).
    """
    if b < 2:
        raise ValueError("block size must be >= 2 (pressure and temperature)")
    n = nx * ny
    acc = 1e-3 / dt

    # face transmissibilities and fluxes ------------------------------------
    tx = _harmonic(perm[:, :-1], perm[:, 1:]) if nx > 1 else np.zeros((ny, 0))
    ty = _harmonic(perm[:-1, :], perm[1:, :]) if ny > 1 else np.zeros((0, nx))
    if not transmissibility:
        tx = np.zeros_like(tx)
        ty = np.zeros_like(ty)
    nfaces = tx.size + ty.size
    tmean = (tx.sum() + ty.sum()) / nfaces if nfaces else 1.0
    if tmean == 0:
        tmean = 1.0
    fx = tx / tmean if flow else np.zeros_like(tx)
    fy = ty / tmean if flow else np.zeros_like(ty)
    fx_abs = np.abs(fx)
    fmean = (fx_abs.sum() + np.abs(fy).sum()) / nfaces if nfaces else 1.0
    u_char = fmean if fmean > 0 else 1.0
    length = float(nx)
    if k_thermal is not None:
        kt = float(k_thermal)
        rcp = peclet * kt / (u_char * length)
    else:
        rcp = 1.0
        kt = u_char * length / peclet
    if not transmissibility:
        kt = 0.0

    # neighbour existence masks (ny, nx) and per-face values seen by each cell
    zero = np.zeros((ny, nx))
    has_w = np.zeros((ny, nx), bool); has_w[:, 1:] = True
    has_e = np.zeros((ny, nx), bool); has_e[:, :-1] = True
    has_s = np.zeros((ny, nx), bool); has_s[1:, :] = True
    has_n = np.zeros((ny, nx), bool); has_n[:-1, :] = True
    t_w = zero.copy(); t_w[:, 1:] = tx
    t_e = zero.copy(); t_e[:, :-1] = tx
    t_s = zero.copy(); t_s[1:, :] = ty
    t_n = zero.copy(); t_n[:-1, :] = ty
    f_w = zero.copy(); f_w[:, 1:] = fx      # inflow from the west neighbour
    f_e = zero.copy(); f_e[:, :-1] = fx     # outflow to the east neighbour
    f_s = zero.copy(); f_s[1:, :] = fy
    f_n = zero.copy(); f_n[:-1, :] = fy
    nfc = has_w.astype(float) + has_e + has_s + has_n   # number of faces of the cell
    out_flux = f_e + f_n

    # block-row structure: order S, W, I, E, N (ascending column index).  The
    # values are assembled on a dense (ny, nx, 5, b, b) array, one slot per
    # possible neighbour, so every update is a strided slice; the slots of
    # absent neighbours are dropped at the end.
    masks = [has_s, has_w, np.ones((ny, nx), bool), has_e, has_n]
    counts = sum(m.astype(np.int64) for m in masks).reshape(-1)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnzb = int(row_ptr[-1])
    col_idx = np.empty(nnzb, np.int32)
    dense = np.empty((ny, nx, 5, b, b), np.float64)

    cell = np.arange(n, dtype=np.int64).reshape(ny, nx)
    offsets = [cell - nx, cell - 1, cell, cell + 1, cell + nx]
    before = np.zeros((ny, nx), np.int64)
    slot = []
    for m in masks:
        slot.append(row_ptr[:-1].reshape(ny, nx) + before)
        before = before + m
    # principal diagonals per neighbour type: (p, T, comp)
    diag_p = acc + (t_w + t_e + t_s + t_n)
    acc_t = heat_capacity / dt
    diag_t = acc_t + kt * nfc + rcp * out_flux
    diag_c = acc + out_flux
    offd = {
        0: (-t_s, -kt * has_s - rcp * f_s, -f_s),   # south neighbour is upwind
        1: (-t_w, -kt * has_w - rcp * f_w, -f_w),   # west neighbour is upwind
        3: (-t_e, -kt * has_e + 0.0 * f_e, 0.0 * f_e),  # east is downwind
        4: (-t_n, -kt * has_n + 0.0 * f_n, 0.0 * f_n),  # north is downwind
    }
    for k, m in enumerate(masks):
        col_idx[slot[k][m]] = offsets[k][m].astype(np.int32)
    principal = []
    for k, m in enumerate(masks):
        ep, et, ec = (diag_p, diag_t, diag_c) if k == 2 else offd[k]
        principal.append([np.where(m, v, 0.0) for v in (ep, et, ec)])

    def fill_rows(y0, y1):
        dense[y0:y1] = 0.0
        for k, (ep, et, ec) in enumerate(principal):
            dense[y0:y1, :, k, P_INDEX, P_INDEX] = ep[y0:y1]
            dense[y0:y1, :, k, T_INDEX, T_INDEX] = et[y0:y1]
            for r in range(2, b):
                dense[y0:y1, :, k, r, r] = ec[y0:y1]

    with _pool() as pool:
        for f in [pool.submit(fill_rows, y0, min(ny, y0 + 16)) for y0 in range(0, ny, 16)]:
            f.result()

    # cross-unknown couplings ------------------------------------------------
    rng_c = np.random.default_rng([seed, 2])
    if coupling_ref == "flux" and not zero_coupling:
        acc_col = np.full(b, acc)
        acc_col[T_INDEX] = acc_t
        _flux_couplings(dense, b, tx, ty, fx, fy, acc_col, coupling, rng_c)
    present = np.stack(masks, axis=-1)
    vals = np.empty((nnzb, b, b), np.float64)

    def compress_rows(y0, y1):
        lo, hi = row_ptr[y0 * nx], row_ptr[y1 * nx]
        vals[lo:hi] = dense[y0:y1].reshape(-1, b, b)[present[y0:y1].reshape(-1)]

    with _pool() as pool:
        for f in [pool.submit(compress_rows, y0, min(ny, y0 + 16)) for y0 in range(0, ny, 16)]:
            f.result()
    del dense
    if coupling_ref != "flux":
        xi = rng_c.uniform(-coupling, coupling, size=(nnzb, b, b))
        if zero_coupling:
            xi[:] = 0.0
        d = np.diagonal(vals, axis1=1, axis2=2).copy()   # (nnzb, b)
        off = ~np.eye(b, dtype=bool)
        ref = d[:, None, :] if coupling_ref == "col" else d[:, :, None]
        vals += np.where(off[None], xi * ref, 0.0)
        del xi

    if band is not None:
        x0, x1, factor = band
        xs = np.arange(nx)
        sel = np.zeros((ny, nx), bool)
        sel[:, (xs >= x0) & (xs < x1)] = True
        vals[slot[2][sel], T_INDEX, T_INDEX] *= factor

    rng_r = np.random.default_rng([seed, 3])
    rhs = rng_r.uniform(-1.0, 1.0, size=n * b)

    meta = dict(nx=nx, ny=ny, b=b, peclet=peclet, k_thermal=kt, rho_cp=rcp,
                dt=dt, acc=acc, seed=seed, field_seed=field_seed, band=band)
    return BSRSystem(nx, ny, b, row_ptr.astype(np.int32), col_idx, vals, rhs, meta)


def _flux_couplings(dense, b, tx, ty, fx, fy, acc_col, coupling, rng):
    """Conservative cross-unknown couplings (reading of "coupling entries
    uniform(-0.1, 0.1) times the diagonal").  For every interior face f from
    an upwind cell I to a downwind cell J and every pair r != c, the flux of
    quantity r across f depends on unknown c with a coefficient xi times the
    face's own (diagonal) flux coefficient of c: the transmissibility T_f for
    pressure (flux_r += xi T_f (p_I - p_J)), the Darcy flux F_f for every other
    unknown, taken upwind (flux_r += xi F_f c_I).  The flux leaves row I and
    enters row J, so every face term has zero column sum like the principal
    terms (conservation).  Each cell's accumulation of r also depends on its
    own unknown c with xi times c's accumulation coefficient.
    xi ~ U(-coupling, coupling), independent per face (or cell), r and c;
    drawn in the order: x-faces, y-faces, cells.  ``dense`` is the
    (ny, nx, 5, b, b) slot array (slots S, W, I, E, N)."""
    off = ~np.eye(b, dtype=bool)
    S, W, I, E, N = range(5)
    pcol = np.zeros(b, bool)
    pcol[P_INDEX] = True
    ny, nx = dense.shape[:2]

    def face_terms(xi, tf, ff):
        xi = xi * off
        scale = np.empty(tf.shape + (1, b))
        scale[..., :] = ff[..., None, None]
        scale[..., P_INDEX] = tf[..., None]
        coef = xi * scale                         # (.., r, c)
        cp = np.where(pcol, coef, 0.0)            # pressure derivatives: central
        cu = np.where(pcol, 0.0, coef)            # other unknowns: upwind (cell I)
        return cp, cu

    # Rows are taken in chunks: the random draws are made in order on this
    # thread, the arithmetic of the chunks runs on a thread pool.  Every entry
    # receives its terms in the order x-faces (as upwind cell, then as
    # downwind cell), y-faces (likewise), cell; chunks touch disjoint rows
    # except for the downwind term of a chunk's last y-face row, which is
    # added after the next chunk's upwind terms.
    chunk = 16

    def x_chunk(y0, y1, xi):
        cp, cu = face_terms(xi, tx[y0:y1], fx[y0:y1])
        dense[y0:y1, :-1, I] += cp + cu
        dense[y0:y1, :-1, E] += -cp
        dense[y0:y1, 1:, W] += -cp - cu
        dense[y0:y1, 1:, I] += cp

    def y_chunk(y0, y1, xi):
        cp, cu = face_terms(xi, ty[y0:y1], fy[y0:y1])
        dense[y0:y1, :, I] += cp + cu
        dense[y0:y1, :, N] += -cp
        dense[y0 + 1:y1 + 1, :, S] += -cp - cu
        dense[y0 + 1:y1, :, I] += cp[:-1]
        return cp[-1]

    def cell_chunk(y0, y1, xi):
        dense[y0:y1, :, I] += (xi * off) * acc_col[None, None, None, :]

    with _pool() as pool:
        if tx.size:
            futs = [pool.submit(x_chunk, y0, min(ny, y0 + chunk),
                                rng.uniform(-coupling, coupling, size=(min(ny, y0 + chunk) - y0, nx - 1, b, b)))
                    for y0 in range(0, ny, chunk)]
            for f in futs:
                f.result()
        if ty.size:
            starts = list(range(0, ny - 1, chunk))
            futs = [pool.submit(y_chunk, y0, min(ny - 1, y0 + chunk),
                                rng.uniform(-coupling, coupling, size=(min(ny - 1, y0 + chunk) - y0, nx, b, b)))
                    for y0 in starts]
            last = [f.result() for f in futs]
            for y0, cp_last in zip(starts, last):
                dense[min(ny - 1, y0 + chunk), :, I] += cp_last
        futs = [pool.submit(cell_chunk, y0, min(ny, y0 + chunk),
                            rng.uniform(-coupling, coupling, size=(min(ny, y0 + chunk) - y0, nx, b, b)))
                for y0 in range(0, ny, chunk)]
        for f in futs:
            f.result()


def _pool():
    import concurrent.futures
    import os
    return concurrent.futures.ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1)))


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

def tiny(nx: int, ny: int, b: int, *, peclet: float = 1.0, seed: int = 0,
         kind: str = "lognormal", ln_sigma: float = 1.0, **kw) -> BSRSystem:
    """Small systems for oracle pins and parity cases."""
    rng_f = np.random.default_rng([seed, 1])
    perm = permeability(kind, nx, ny, rng_f, ln_sigma=ln_sigma, corr_len=3.0)
    return assemble(nx, ny, b, perm, peclet=peclet, seed=seed, field_seed=seed, **kw)


def config1() -> BSRSystem:
    """20x20, b = 3 (p, T, S_w), homogeneous k = 1, K_T = 1, Pe = 1, seed 0."""
    perm = np.ones((20, 20))
    return assemble(20, 20, 3, perm, peclet=1.0, k_thermal=1.0, seed=0, field_seed=0)


CONFIG2_PECLET = (0.1, 1.0, 10.0, 100.0)


def config2(index: int) -> BSRSystem:
    """200x100, b = 6, log-normal k (ln-sigma 1, correlation length 10 cells),
    Pe in {0.1, 1, 10, 100} (system ``index`` uses seed ``index``)."""
    pe = CONFIG2_PECLET[index]
    rng_f = np.random.default_rng([index, 1])
    perm = permeability("lognormal", 200, 100, rng_f, ln_sigma=1.0, corr_len=10.0)
    return assemble(200, 100, 6, perm, peclet=pe, seed=index, field_seed=index)


CONFIG3_PECLET = (0.1, 100.0)


def config3(index: int, nx: int = 1000, ny: int = 500) -> BSRSystem:
    """1000x500, b = 8, channelised field (ln-sigma 2 plus sinusoidal bands of
    100x contrast), Pe 0.1 (seed 0) or Pe 100 (seed 1)."""
    pe = CONFIG3_PECLET[index]
    rng_f = np.random.default_rng([index, 1])
    perm = permeability("channelised", nx, ny, rng_f, ln_sigma=2.0, corr_len=10.0)
    return assemble(nx, ny, 8, perm, peclet=pe, seed=index, field_seed=index)


def config4_train(index: int, nx: int = 256, ny: int = 128) -> BSRSystem:
    """Training systems for the learned temperature interpolation: 256x128,
    b = 6, seeds 1000 + index, Pe log-uniform in [0.01, 1000], ln-sigma U[0.5, 2]."""
    seed = 1000 + index
    rng_p = np.random.default_rng([seed, 4])
    pe = float(10.0 ** rng_p.uniform(-2.0, 3.0))
    sig = float(rng_p.uniform(0.5, 2.0))
    rng_f = np.random.default_rng([seed, 1])
    perm = permeability("lognormal", nx, ny, rng_f, ln_sigma=sig, corr_len=10.0)
    return assemble(nx, ny, 6, perm, peclet=pe, seed=seed, field_seed=seed)


def config5_field(nx: int = 2000, ny: int = 1000) -> np.ndarray:
    rng_f = np.random.default_rng([0, 1])
    return permeability("lognormal", nx, ny, rng_f, ln_sigma=1.5, corr_len=10.0)


def config5(step: int, perm: np.ndarray | None = None, nx: int = 2000, ny: int = 1000) -> BSRSystem:
    """System ``step`` (0..19) of the Newton sequence: 2000x1000, b = 8,
    ln-sigma 1.5, Pe 10; a 20-cell band x in [nx/4 + 5 s, nx/4 + 5 s + 20) has
    its T-diagonal multiplied by 50."""
    if perm is None:
        perm = config5_field(nx, ny)
    x0 = nx // 4 + 5 * step
    return assemble(nx, ny, 8, perm, peclet=10.0, seed=step, field_seed=0,
                    band=(x0, x0 + 20, 50.0))


def named(name: str) -> BSRSystem:
    """'c1', 'c2-<i>', 'c3-<i>', 'c4t-<i>', 'c5-<s>' and small-grid variants
    like 'c3s-<i>-<nx>x<ny>' (the config-3 recipe on a smaller grid)."""
    parts = name.split("-")
    if parts[0] == "c1":
        return config1()
    if parts[0] == "c2":
        return config2(int(parts[1]))
    if parts[0] == "c3":
        return config3(int(parts[1]))
    if parts[0] == "c3s":
        nx, ny = (int(v) for v in parts[2].split("x"))
        return config3(int(parts[1]), nx, ny)
    if parts[0] == "c4t":
        return config4_train(int(parts[1]))
    if parts[0] == "c5":
        return config5(int(parts[1]))
    raise ValueError(name)
