"""Seeded full Newton systems (primary plus cell-local secondary unknowns) for
the static-condensation front end.

Input recipe only: none of the condensation arithmetic lives here.  The paper
partitions each cell's unknowns into primary ones (globally coupled) and
secondary ones whose equations couple only within the cell (Sec.
"Static-Condensation Strategy"): J22 is block diagonal, J21 (secondary
equations against primary unknowns) is cell-local, and J11 / J12 (primary
equations) carry the flux couplings to the neighbours.  The recipe, a
stand-in for simulator output:
  * J11 and the pattern: a reduced system from ``generator`` (n1 = its b);
  * J22_jj: diagonal 1 + U(0, 1), off-diagonal U(-0.1, 0.1) (row diagonally
    dominant up to n2 = 8, so every block is invertible);
  * J21_jj: U(-0.5, 0.5);
  * J12_ij (every stored block): xi * J11_ij[r][r] for row r, xi ~ U(-0.02, 0.02);
  * r1 = -(the reduced system's right-hand side), r2 ~ U(-1, 1).
Streams: numpy PCG64 ``default_rng([seed, 11 .. 14])``.

Layout (host numpy): J12 float64 [nnzb, n1, n2]; J21 [n, n2, n1];
J22 [n, n2, n2]; r1 [n * n1]; r2 [n * n2] (cell-interleaved)."""
from __future__ import annotations

import dataclasses

import numpy as np

from .generator import BSRSystem


@dataclasses.dataclass
class FullSystem:
    nx: int
    ny: int
    n1: int
    n2: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    J11: np.ndarray
    J12: np.ndarray
    J21: np.ndarray
    J22: np.ndarray
    r1: np.ndarray
    r2: np.ndarray

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])


def full_system(base: BSRSystem, n2: int, seed: int = 0, j12_scale: float = 0.02) -> FullSystem:
    n, n1, nnzb = base.n, base.b, base.nnzb
    g22 = np.random.default_rng([seed, 11])
    g21 = np.random.default_rng([seed, 12])
    g12 = np.random.default_rng([seed, 13])
    gr = np.random.default_rng([seed, 14])
    J22 = g22.uniform(-0.1, 0.1, size=(n, n2, n2))
    idx = np.arange(n2)
    J22[:, idx, idx] = 1.0 + g22.uniform(0.0, 1.0, size=(n, n2))
    J21 = g21.uniform(-0.5, 0.5, size=(n, n2, n1))
    diag = base.vals[:, np.arange(n1), np.arange(n1)]          # [nnzb, n1]: J11_ij[r][r]
    J12 = g12.uniform(-j12_scale, j12_scale, size=(nnzb, n1, n2)) * diag[:, :, None]
    r1 = -base.rhs.copy()
    r2 = gr.uniform(-1.0, 1.0, size=n * n2)
    return FullSystem(base.nx, base.ny, n1, n2, base.row_ptr.copy(), base.col_idx.copy(), base.vals.copy(),
                      J12, J21, J22, r1, r2)


@dataclasses.dataclass
class Wells:
    """Wells with one perforation each: well w has nw unknowns and couples to
    the primary unknowns of cell ``cell[w]`` (J1w [count, n1, nw]: that
    cell's primary rows against the well unknowns; Jw1 [count, nw, n1]: the
    well rows against the cell's primary unknowns; Jww [count, nw, nw];
    rw [count * nw])."""
    cell: np.ndarray
    nw: int
    J1w: np.ndarray
    Jw1: np.ndarray
    Jww: np.ndarray
    rw: np.ndarray

    @property
    def count(self) -> int:
        return int(self.cell.shape[0])


def wells(nx: int, ny: int, n1: int, nw: int = 2, cells=None, seed: int = 0, scale: float = 0.5) -> Wells:
    """Seeded wells (input recipe).  By default an injector and a producer at
    opposite corners, cells 0 and nx*ny - 1 (the corner-to-corner pattern of
    the paper's two-well cases); Jww_w: diagonal 1 + U(0, 1), off-diagonal
    U(-0.1, 0.1); J1w, Jw1: U(-scale, scale); rw: U(-1, 1).  Streams
    default_rng([seed, 21 .. 24])."""
    cell = np.array([0, nx * ny - 1] if cells is None else cells, dtype=np.int32)
    W = cell.shape[0]
    gww = np.random.default_rng([seed, 21])
    g1w = np.random.default_rng([seed, 22])
    gw1 = np.random.default_rng([seed, 23])
    gr = np.random.default_rng([seed, 24])
    Jww = gww.uniform(-0.1, 0.1, size=(W, nw, nw))
    idx = np.arange(nw)
    Jww[:, idx, idx] = 1.0 + gww.uniform(0.0, 1.0, size=(W, nw))
    J1w = g1w.uniform(-scale, scale, size=(W, n1, nw))
    Jw1 = gw1.uniform(-scale, scale, size=(W, nw, n1))
    rw = gr.uniform(-1.0, 1.0, size=W * nw)
    return Wells(cell, nw, J1w, Jw1, Jww, rw)
