"""Seeded synthetic inputs for the butterfly FIO workloads.

Shared by the tests, the benchmark and the oracle checks; holds none of the
method's arithmetic.  The numerical section draws the sources f(k) iid from
the standard normal distribution (white noise) and measures the error on a
set S of 256 points of X; the inputs here follow that recipe:

* f: complex white noise (g1 + i g2)/sqrt(2), g1, g2 ~ N(0,1) iid, so
  E|f(k)|^2 = 1 (the relative error does not depend on the scale);
* S: points of X drawn uniformly without replacement (flat index i1*N+i2);
* phase parameters for the learnable / perturbed variants: a_j ~ U[0.8, 1.2],
  eta_j ~ U[0, 0.3].

Every generator takes an explicit integer seed (numpy PCG64).
"""
from __future__ import annotations

import numpy as np


def white_noise(N: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex white noise of shape (N, N) (or (nrhs, N, N)), complex128."""
    rng = np.random.default_rng(seed)
    shape = (N, N) if nrhs is None else (nrhs, N, N)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def sample_points(N: int, n: int, seed: int) -> np.ndarray:
    """n distinct flat indices of X (all of X, sorted, when n >= N^2)."""
    if n >= N * N:
        return np.arange(N * N, dtype=np.int64)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(N * N, size=n, replace=False)).astype(np.int64)


def velocity_scalings(seed: int) -> tuple[float, float]:
    """(a1, a2) ~ U[0.8, 1.2]^2: learnable scalings of the ellipse axes."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.8, 1.2, size=2)
    return float(a[0]), float(a[1])


def modulation_amplitudes(seed: int, n: int = 1) -> np.ndarray:
    """(n, 2) array of (eta1, eta2) ~ U[0, 0.3]: per-problem perturbations."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 0.3, size=(n, 2))


def amplitude_factors(N: int, rank: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Smooth complex factors of a separated amplitude a(x,k) = sum_t g_t(x)
    h_t(k): g (rank, N, N) on the x grid x = i/N, h (rank, N, N) on the
    frequency grid k = i - N/2; six N(0,1) coefficients per term."""
    rng = np.random.default_rng(seed)
    i = np.arange(N)
    x1, x2 = np.meshgrid(i / N, i / N, indexing="ij")
    k1, k2 = np.meshgrid(i - N // 2, i - N // 2, indexing="ij")
    g = np.empty((rank, N, N), complex)
    h = np.empty((rank, N, N), complex)
    for t in range(rank):
        c = rng.standard_normal(6)
        g[t] = (1 + 0.5 * c[0] * x1 + c[1] * x2 ** 2) * np.exp(1j * (c[2] * x1 - x2))
        h[t] = 1 / (1 + 0.1 * (c[3] * k1 / N) ** 2 + (k2 / N + c[4]) ** 2) * np.exp(1j * c[5] * k1 / N)
    return g, h


def mixed_batch(seed: int, n: int = 32) -> list[dict]:
    """Uneven batch of problems: N ~ U{128,256,512,1024}, tolerance ~
    U{1e-2, 1e-4, 1e-6}, (eta1, eta2) ~ U[0, 0.3]^2, per-problem f seeds."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice([128, 256, 512, 1024], size=n)
    tols = rng.choice([1e-2, 1e-4, 1e-6], size=n)
    etas = rng.uniform(0.0, 0.3, size=(n, 2))
    fseeds = rng.integers(0, 2**31 - 1, size=n)
    return [dict(N=int(Ns[i]), tol=float(tols[i]), eta1=float(etas[i, 0]), eta2=float(etas[i, 1]),
                 f_seed=int(fseeds[i])) for i in range(n)]


_MASK64 = (1 << 64) - 1


def splitmix64(seed: int, k) -> np.ndarray:
    """Output of the SplitMix64 generator (Steele, Lea and Flood, 2014) at
    counters k: state seed + (k+1) 0x9E3779B97F4A7C15, then its two
    xor-shift-multiply rounds and a final xor-shift (uint64 arithmetic)."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK64) + (k + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def probe_phases(N: int, seed: int) -> np.ndarray:
    """The q selector's probe: f(k) = exp(2 pi i v_k), v_k = (SplitMix64(seed,
    k) >> 11) 2^-53, k the flat index of (k1 + N/2, k2 + N/2); complex128 (N, N)."""
    v = (splitmix64(seed, np.arange(N * N)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.exp(2j * np.pi * v).reshape(N, N)


def probe_rows(N: int, nrows: int, seed: int) -> np.ndarray:
    """The q selector's sampled targets: SplitMix64(seed ^ 0x5851F42D4C957F2D, i) mod N^2."""
    return (splitmix64(seed ^ 0x5851F42D4C957F2D, np.arange(nrows)) % np.uint64(N * N)).astype(np.int64)
