"""Seeded initial parameters of the interpolation edge-MLP (16 -> 64 -> 64 -> 1).

Only random numbers: He-uniform first and second layers, a small last layer
(so that the initial correction is close to zero), zero biases.  Blob layout
(float32): W1 [64][16], b1 [64], W2 [64][64], b2 [64], W3 [64], b3 [1].
"""
from __future__ import annotations

import numpy as np

NF, NH = 16, 64
NPARAMS = NH * NF + NH + NH * NH + NH + NH + 1


def mlp_init(seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng([seed, 7])
    w1 = rng.uniform(-1.0, 1.0, (NH, NF)) * np.sqrt(6.0 / NF)
    w2 = rng.uniform(-1.0, 1.0, (NH, NH)) * np.sqrt(6.0 / NH)
    w3 = rng.uniform(-1.0, 1.0, NH) * 0.01
    blob = np.concatenate([w1.reshape(-1), np.zeros(NH), w2.reshape(-1), np.zeros(NH), w3, np.zeros(1)])
    assert blob.size == NPARAMS
    return blob.astype(np.float32)
