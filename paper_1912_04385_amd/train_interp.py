"""Train the edge-MLP of the learned temperature interpolation on the GPU.

The training set is the temperature subsystems C_TT that the method itself
extracts (left scaling and Schur extraction of the energy block, as in the
setup of the three-stage preconditioner) from 256 seeded 256 x 128, b = 6
systems with Peclet numbers drawn log-uniformly in [0.01, 1000] and ln-sigma
in [0.5, 2].  Each system is set up once with classical interpolation; every
training step (``cptr_mlp_train_step``) draws fresh smooth error vectors on
one system and takes an Adam step.  Everything numerical runs in the
library's kernels; this script only sequences the calls.

    python -m paper_1912_04385_amd.train_interp --out interp_mlp.npy
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "interp_mlp.npy")


def load_weights(path: str = DEFAULT_WEIGHTS) -> np.ndarray:
    """The trained parameter blob (float32, safe numpy load)."""
    w = np.load(path, allow_pickle=False)
    return np.ascontiguousarray(w, dtype=np.float32)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--systems", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--vectors", type=int, default=8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)

    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1912_04385_amd import cptr
    from synthetic import config4_train, mlp_init

    t0 = time.perf_counter()
    solvers = []
    for i in range(args.systems):
        s = config4_train(i)
        sv = cptr.Solver(restart=1)
        sv.setup(torch.from_numpy(s.row_ptr), torch.from_numpy(s.col_idx), torch.from_numpy(s.vals.reshape(-1)),
                 0, 1, s.nx, s.ny)
        solvers.append(sv)
        if (i + 1) % 64 == 0:
            print(f"# set up {i + 1} training systems ({time.perf_counter() - t0:.1f} s)", flush=True)

    # loss of the classical weights (zero last layer) as the reference level
    zero = mlp_init(args.seed).copy()
    zero[-65:] = 0.0
    ref = cptr.MLP(zero)
    base = float(np.mean([ref.train_step(sv, args.vectors, 12345 + k, 1e-30) for k, sv in enumerate(solvers)]))
    ref.close()
    print(f"# classical interpolation loss {base:.6e}", flush=True)

    net = cptr.MLP(mlp_init(args.seed))
    rng = np.random.default_rng([args.seed, 11])
    history = []
    for ep in range(args.epochs):
        losses = []
        for k in rng.permutation(len(solvers)):
            losses.append(net.train_step(solvers[k], args.vectors, 1000003 * (ep + 1) + int(k), args.lr))
        history.append(float(np.mean(losses)))
        print(f"# epoch {ep}: mean loss {history[-1]:.6e} (classical {base:.6e}) "
              f"{time.perf_counter() - t0:.1f} s", flush=True)
    params = net.params()
    net.close()
    for sv in solvers:
        sv.close()
    np.save(args.out, params)
    print(f"# wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
