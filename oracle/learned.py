"""Oracle of the learned temperature-stage interpolation (an extension of the
multi-stage preconditioner: the AMG sub-solver amg(C_TT) of Eq. CPTR3M1 with
its fine-level prolongation weights corrected by a small edge-MLP).

TEST INFRASTRUCTURE, like the rest of ``oracle``.

Parity unpinned (nothing in the paper fixes these numbers): the features,
the network and the loss are this build's definitions.  They are pinned by
properties only: closed-form features on a 1-D Poisson row, a zero last layer
reproducing the classical weights exactly, the gradient against finite
differences, and the Adam step against its published update rule.

Definitions (all in FP64 here):

* Edges: the entries (i, J) of the classical (extended+i, truncated) fine
  interpolation P for F rows i, in P's storage order; j is the fine index of
  coarse point J.
* Features x_e (16 per edge), with A the fine operator, a_ii its diagonal,
  s_i = sign(a_ii), w0 the classical weights of row i:
    0  a_ij / a_ii                      1  a_ji / a_jj
    2  (-s_i a_ij) / max_{k!=i}(-s_i a_ik)   (0 if that max <= 0)
    3  1 if j is not in the pattern of row i (a distance-2 point)
    4  w0_ij                            5  sum_{k in row i, k != i, j} a_ik a_kj / (a_ii a_kk)
    6  (sum_k a_ik) / a_ii              7  1 / (number of P entries of row i)
    8  (a_ij - a_ji) / (|a_ij| + |a_ji|)   (0 if both are 0)
    9  sum_J w0_iJ                      10 w0_ij / max_J |w0_iJ|
    11 |a_jj| / (|a_ii| + |a_jj|)       12 (sum_k a_jk) / a_jj
    13 (number of strong couplings of i) / (row length of i - 1)
    14 1                                15 0
* Network: 16 -> 64 -> 64 -> 1 with ReLU, weights in BF16; the input and the
  first hidden layer are rounded to BF16 (the operands of the matrix-core
  products), sums are exact here (FP32 accumulation on the GPU);
  delta_e = tanh(o_e) / 2.
* Learned weights of row i: u_e = w0_e (1 + delta_e), rescaled to the
  classical row sum, w_e = u_e S_i / D_i with S_i = sum w0, D_i = sum u, when
  |D_i| > 0 and S_i / D_i lies in [1/4, 4]; otherwise w_e = u_e.
* Loss over K smooth error vectors e^k (20 damped-Jacobi sweeps, omega 2/3,
  on A e = 0 from SplitMix64-uniform starts): the mean over F rows of
  sum_k (e^k_i - sum_J w_iJ e^k_j)^2 / sum_k (e^k_i)^2.
* Parameter blob (float32, NPARAMS): W1 [64][16], b1 [64], W2 [64][64],
  b2 [64], W3 [64], b3 [1].
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .core import CSR, _splitmix_vec

NF, NH = 16, 64
NPARAMS = NH * NF + NH + NH * NH + NH + NH + 1
SMOOTH_SWEEPS = 20
SMOOTH_OMEGA = 2.0 / 3.0


def unpack(p: np.ndarray) -> dict:
    p = np.asarray(p, np.float64)
    o = 0
    out = {}
    for name, shape in (("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)),
                        ("b3", (1,))):
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[k], np.float64).reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    Values are first rounded to float32 (the GPU holds them in FP32)."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


@dataclasses.dataclass
class Edges:
    row: np.ndarray      # fine row i of each edge
    fine: np.ndarray     # fine index j of the coarse point
    pos: np.ndarray      # position in P's value array
    X: np.ndarray        # features [E, 16]
    frows: np.ndarray    # F rows with at least one edge, ascending
    start: np.ndarray    # edges of frows[q] are start[q]:start[q+1]


def _seqsum(a) -> float:
    """Left-to-right sum (the order the features are defined in)."""
    s = 0.0
    for x in a:
        s += float(x)
    return s


def _entry(A: CSR, i: int, j: int):
    lo, hi = A.rp[i], A.rp[i + 1]
    k = lo + np.searchsorted(A.ci[lo:hi], j)
    if k < hi and A.ci[k] == j:
        return float(A.v[k]), True
    return 0.0, False


def edge_features(A: CSR, strong: np.ndarray, cf: np.ndarray, P: CSR) -> Edges:
    """The 16 features of every F-row edge of the classical interpolation."""
    cf = np.asarray(cf)
    fine_of = np.flatnonzero(cf == 1).astype(np.int64)    # coarse index -> fine index
    diag = A.diagonal()
    rows, fines, poss, feats, frows, start = [], [], [], [], [], [0]
    for i in range(A.nrows):
        if cf[i] == 1 or P.rp[i + 1] == P.rp[i]:
            continue
        lo, hi = A.rp[i], A.rp[i + 1]
        aii = diag[i]
        si = -1.0 if aii < 0 else 1.0
        offd = [(A.ci[e], A.v[e]) for e in range(lo, hi) if A.ci[e] != i]
        smax = max([-si * v for _, v in offd], default=0.0)
        rowsum_i = _seqsum(A.v[lo:hi])
        nstrong = int(np.sum(strong[lo:hi]))
        plo, phi = P.rp[i], P.rp[i + 1]
        w0 = P.v[plo:phi]
        S = _seqsum(w0)
        wmax = float(np.max(np.abs(w0)))
        for e in range(plo, phi):
            j = int(fine_of[P.ci[e]])
            aij, present = _entry(A, i, j)
            aji, _ = _entry(A, j, i)
            ajj = diag[j]
            path = 0.0
            for k, aik in offd:
                if k == j:
                    continue
                akj, ok = _entry(A, k, j)
                if ok:
                    path += aik * akj / (aii * diag[k])
            den = abs(aij) + abs(aji)
            jlo, jhi = A.rp[j], A.rp[j + 1]
            x = np.zeros(NF)
            x[0] = aij / aii
            x[1] = aji / ajj
            x[2] = (-si * aij) / smax if smax > 0 else 0.0
            x[3] = 0.0 if present else 1.0
            x[4] = P.v[e]
            x[5] = path
            x[6] = rowsum_i / aii
            x[7] = 1.0 / (phi - plo)
            x[8] = (aij - aji) / den if den > 0 else 0.0
            x[9] = S
            x[10] = P.v[e] / wmax if wmax > 0 else 0.0
            x[11] = abs(ajj) / (abs(aii) + abs(ajj))
            x[12] = _seqsum(A.v[jlo:jhi]) / ajj
            x[13] = nstrong / (hi - lo - 1) if hi - lo > 1 else 0.0
            x[14] = 1.0
            rows.append(i)
            fines.append(j)
            poss.append(e)
            feats.append(x)
        frows.append(i)
        start.append(len(rows))
    X = np.array(feats).reshape(-1, NF)
    return Edges(np.array(rows, np.int64), np.array(fines, np.int64), np.array(poss, np.int64), X,
                 np.array(frows, np.int64), np.array(start, np.int64))


def forward(params: np.ndarray, X: np.ndarray, exact: bool = False):
    """o_e for every edge (and the intermediates for the backward pass).
    ``exact=True`` drops every BF16 rounding (for finite-difference checks)."""
    rnd = (lambda v: np.asarray(v, np.float64)) if exact else bf16
    q = unpack(params)
    W1, W2, W3 = rnd(q["W1"]), rnd(q["W2"]), rnd(q["W3"])
    xb = rnd(X)
    z1 = xb @ W1.T + q["b1"]
    h1 = np.maximum(z1, 0.0)
    h1b = rnd(h1)
    z2 = h1b @ W2.T + q["b2"]
    h2 = np.maximum(z2, 0.0)
    o = h2 @ W3 + q["b3"][0]
    return o, dict(xb=xb, z1=z1, h1b=h1b, z2=z2, h2=h2, W2=W2, W3=W3)


def delta_of(o: np.ndarray) -> np.ndarray:
    return 0.5 * np.tanh(o)


def _row_weights(w0: np.ndarray, delta: np.ndarray):
    u = w0 * (1.0 + delta)
    S, D = float(np.sum(w0)), float(np.sum(u))
    if D != 0.0 and 0.25 <= S / D <= 4.0:
        return u * (S / D), True, S, D
    return u, False, S, D


def learned_weights(P: CSR, edges: Edges, delta: np.ndarray) -> CSR:
    """The interpolation with corrected F-row weights (same pattern)."""
    v = P.v.copy()
    for q, i in enumerate(edges.frows):
        a, b = edges.start[q], edges.start[q + 1]
        w, _, _, _ = _row_weights(P.v[edges.pos[a:b]], delta[a:b])
        v[edges.pos[a:b]] = w
    return CSR(P.nrows, P.ncols, P.rp.copy(), P.ci.copy(), v)


def smooth_vectors(A: CSR, K: int = 8, seed: int = 0, sweeps: int = SMOOTH_SWEEPS) -> np.ndarray:
    """K algebraically smooth vectors: damped Jacobi (omega 2/3) on A e = 0,
    vector k starting from u(seed, k n + i) in [-1, 1)."""
    n = A.nrows
    d = A.diagonal()
    u = _splitmix_vec(seed, K * n)
    E = ((u >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 * 2.0 - 1.0).reshape(K, n)
    for k in range(K):
        e = E[k]
        for _ in range(sweeps):
            e = e - SMOOTH_OMEGA * A.matvec(e) / d
        E[k] = e
    return E


def loss_and_grad(params: np.ndarray, P: CSR, edges: Edges, E: np.ndarray, exact: bool = False):
    """Loss (see the module header) and its gradient with respect to the
    parameter blob (the BF16 roundings are passed straight through)."""
    o, c = forward(params, edges.X, exact)
    t = np.tanh(o)
    delta = 0.5 * t
    nrows = len(edges.frows)
    loss = 0.0
    ddelta = np.zeros_like(o)
    for q, i in enumerate(edges.frows):
        a, b = edges.start[q], edges.start[q + 1]
        w0 = P.v[edges.pos[a:b]]
        w, scaled, S, D = _row_weights(w0, delta[a:b])
        ej = E[:, edges.fine[a:b]]               # [K, m]
        ei = E[:, i]
        r = ei - ej @ w
        den = float(np.sum(ei * ei)) + 1e-300
        loss += float(np.sum(r * r)) / den
        g = -2.0 * (ej.T @ r) / den / nrows      # dL/dw
        if scaled:
            ddelta[a:b] = (w0 / D) * (S * g - float(np.sum(g * w)))
        else:
            ddelta[a:b] = g * w0
    loss /= max(nrows, 1)
    do = ddelta * 0.5 * (1.0 - t * t)
    # backward through the network
    dW3 = c["h2"].T @ do
    db3 = np.array([np.sum(do)])
    dz2 = np.outer(do, c["W3"]) * (c["z2"] > 0)
    dW2 = dz2.T @ c["h1b"]
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ c["W2"]) * (c["z1"] > 0)
    dW1 = dz1.T @ c["xb"]
    db1 = dz1.sum(axis=0)
    grad = pack(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3))
    return loss, grad


@dataclasses.dataclass
class Adam:
    """Adam (Kingma & Ba 2015, Algorithm 1) on the parameter blob."""
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: np.ndarray | None = None
    v: np.ndarray | None = None

    def step(self, params: np.ndarray, grad: np.ndarray) -> np.ndarray:
        if self.m is None:
            self.m = np.zeros_like(grad)
            self.v = np.zeros_like(grad)
        self.t += 1
        self.m = self.beta1 * self.m + (1.0 - self.beta1) * grad
        self.v = self.beta2 * self.v + (1.0 - self.beta2) * grad * grad
        mhat = self.m / (1.0 - self.beta1 ** self.t)
        vhat = self.v / (1.0 - self.beta2 ** self.t)
        return params - self.lr * mhat / (np.sqrt(vhat) + self.eps)


def learned_fine_interp(params: np.ndarray, A, s: np.ndarray, cf: np.ndarray, P):
    """The learned weights of the classical fine-level interpolation P of
    operator A (strength flags s, C/F split cf): P itself when it has no F-row
    edge."""
    e = edge_features(A, s, cf, P)
    if len(e.row) == 0:
        return P
    o, _ = forward(params, e.X)
    return learned_weights(P, e, delta_of(o))


def learned_hierarchy(params: np.ndarray, h):
    """The learned counterpart of the classical hierarchy h: its fine level's
    interpolation with the learned weights, and below it h's C/F splits and
    transfer operators, the Galerkin products formed from the learned fine
    level down (h's refresh with a new fine-level interpolation)."""
    from .core import amg_refresh
    L0 = h.levels[0]
    return amg_refresh(h, L0.A, learned_fine_interp(params, L0.A, L0.strong, L0.cf, L0.P))
