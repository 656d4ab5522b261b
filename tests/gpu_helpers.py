"""Test-side helpers for the GPU parity tests: layout conversion between the
library's Morton-ordered weights and the oracle's natural-index arrays."""
import numpy as np


def morton(b1, b2):
    b1 = np.asarray(b1, dtype=np.int64)
    b2 = np.asarray(b2, dtype=np.int64)
    m = np.zeros(np.broadcast(b1, b2).shape, dtype=np.int64)
    for i in range(16):
        m |= ((b2 >> i) & 1) << (2 * i)
        m |= ((b1 >> i) & 1) << (2 * i + 1)
    return m


def weights_to_oracle(w: np.ndarray, N: int, q: int, level: int) -> np.ndarray:
    """Library layout w[(mA * 4^(L-l) + mB) * q^2 + t] -> delta[a1, a2, b1, b2, t1, t2]."""
    L = int(round(np.log2(N)))
    nA, nB = 1 << level, 1 << (L - level)
    a1, a2, b1, b2 = np.meshgrid(np.arange(nA), np.arange(nA), np.arange(nB), np.arange(nB), indexing="ij")
    pair = morton(a1, a2) * (nB * nB) + morton(b1, b2)
    w = np.asarray(w).reshape(N * N, q, q)
    return w[pair]


def rel_l2(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_max(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.abs(a - b).max() / np.abs(b).max())
