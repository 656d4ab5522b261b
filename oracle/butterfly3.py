"""Three-dimensional FIO and its butterfly (TEST INFRASTRUCTURE ONLY: only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import this module; the product path never does).

Sec. 5 (last example) extends the method to three dimensions by using a
three-dimensional Chebyshev grid; its example phase eq:ex3 is

    Phi(x, k) = x . k + c(x) |k|,   c(x) = (3 + sin 2 pi x1 sin 2 pi x2 sin 2 pi x3) / 4,

on X = {i/N : 0 <= i_j < N} and Omega = {-N/2 <= k_j < N/2}.  Here:

  * ``direct3``: u(x) = sum_k e^{2 pi i Phi(x,k)} f(k) by the definition;
  * ``ButterflyModel3``: the steps of Sec. 4 with q x q x q tensor Chebyshev
    grids, octrees (eight children per box) and the same level pairing
    l(A) + l(B) = L as in two dimensions, in plain numpy, FP64.

Readings (the paper gives no details beyond the grid): the frequencies are
mapped to spherical coordinates, the three-dimensional analogue of the polar
map eq:polar,
    p1 = |k| / (sqrt(3) N / 2),  p2 = theta / pi,  p3 = phi / (2 pi) mod 1,
with theta = arccos(k3 / |k|), phi = atan2(k2, k1) and k = 0 -> p = 0, so
that Phi(x, k(p)) = rho(p1) Phi(x, e(p2, p3)) by homogeneity; s and lm as
in two dimensions (s = min(3, floor(L/2)), lm = floor(L/2)); boxes of p are
half-open and clamped like the 2-D ones.

Weights at level l are arrays delta[a1, a2, a3, b1, b2, b3, t1, t2, t3].
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .butterfly import box_of, centre, cheb_nodes, lagrange, nodes

FOURIER = 0
SPHERES = 1
SQRT3_2 = math.sqrt(3.0) / 2.0


def cis(phi):
    """exp(2 pi i phi) after an exact FP64 reduction of phi mod 1."""
    r = phi - np.rint(phi)
    return np.exp(2j * np.pi * r)


def phi3(kind: int, x1, x2, x3, k1, k2, k3):
    """Phi(x, k) of eq:ex3 (kind SPHERES) or x . k (kind FOURIER), broadcasting."""
    d = x1 * k1 + x2 * k2 + x3 * k3
    if kind == FOURIER:
        return d
    c = (3.0 + np.sin(2 * np.pi * x1) * np.sin(2 * np.pi * x2) * np.sin(2 * np.pi * x3)) / 4.0
    return d + c * np.sqrt(k1 * k1 + k2 * k2 + k3 * k3)


def grid3(N: int):
    """Flat (row-major) coordinates of X and of Omega."""
    i = np.arange(N)
    x = np.stack(np.meshgrid(i / N, i / N, i / N, indexing="ij")).reshape(3, -1)
    k = np.stack(np.meshgrid(i - N // 2, i - N // 2, i - N // 2, indexing="ij")).reshape(3, -1).astype(np.float64)
    return x, k


def direct3(N: int, kind: int, f: np.ndarray, rows=None) -> np.ndarray:
    """u at ``rows`` (flat (i1 N + i2) N + i3; default all of X), chunked."""
    x, k = grid3(N)
    f = np.asarray(f, dtype=np.complex128).reshape(-1)
    rows = np.arange(N ** 3) if rows is None else np.asarray(rows)
    out = np.empty(rows.size, dtype=np.complex128)
    step = max(1, (1 << 22) // (N ** 3))
    for a in range(0, rows.size, step):
        r = rows[a:a + step]
        ph = phi3(kind, x[0, r, None], x[1, r, None], x[2, r, None], k[0][None], k[1][None], k[2][None])
        out[a:a + step] = cis(ph) @ f
    return out


def spherical_points(N: int):
    """(k, p): the frequencies of Omega (3, N^3) and their images p (3, N^3)."""
    _, k = grid3(N)
    r = np.sqrt((k * k).sum(axis=0))
    p1 = r / (SQRT3_2 * N)
    safe = np.where(r > 0, r, 1.0)
    p2 = np.where(r > 0, np.arccos(np.clip(k[2] / safe, -1.0, 1.0)) / np.pi, 0.0)
    p3 = np.arctan2(k[1], k[0]) / (2 * np.pi)
    p3 = np.where(p3 < 0, p3 + 1.0, p3)
    p3 = np.where(r > 0, p3, 0.0)
    return k, np.stack([p1, p2, p3])


def k_of_p3(N: int, p1, p2, p3):
    """Inverse map k(p) = (sqrt(3)/2) N p1 (sin pi p2 cos 2 pi p3, sin pi p2 sin 2 pi p3, cos pi p2)."""
    rho = SQRT3_2 * N * np.asarray(p1, dtype=np.float64)
    th, ph = np.pi * np.asarray(p2, dtype=np.float64), 2 * np.pi * np.asarray(p3, dtype=np.float64)
    return rho * np.sin(th) * np.cos(ph), rho * np.sin(th) * np.sin(ph), rho * np.cos(th)


def default_schedule3(N: int):
    L = int(round(math.log2(N)))
    return min(3, L // 2), L // 2


class ButterflyModel3:
    """FP64 three-dimensional butterfly of Sec. 4 (see the module notes)."""

    def __init__(self, N: int, q: int, kind: int, s: int | None = None, lm: int | None = None):
        L = int(round(math.log2(N)))
        if (1 << L) != N or N < 2:
            raise ValueError("N must be a power of two")
        ds, dlm = default_schedule3(N)
        self.N, self.q, self.L, self.kind = N, q, L, kind
        self.s = ds if s is None else int(s)
        self.lm = dlm if lm is None else int(lm)
        if not (0 <= self.s <= self.lm <= L - self.s):
            raise ValueError(f"need 0 <= s <= lm <= L-s (s={self.s}, lm={self.lm}, L={L})")
        self.z = cheb_nodes(q)
        self.k, self.p = spherical_points(N)

    # -- kernel values -----------------------------------------------------
    def E(self, x1, x2, x3, k1, k2, k3):
        return cis(phi3(self.kind, x1, x2, x3, k1, k2, k3))

    def E_p(self, x1, x2, x3, p1, p2, p3):
        return self.E(x1, x2, x3, *k_of_p3(self.N, p1, p2, p3))

    @staticmethod
    def _grid(a, b, c):
        """Broadcast three 1-D arrays to the grid [i, j, k]."""
        a, b, c = (np.asarray(v, dtype=np.float64) for v in (a, b, c))
        return a[:, None, None], b[None, :, None], c[None, None, :]

    # -- step 2: initialisation (eq:alg2a) ---------------------------------
    def init(self, f: np.ndarray) -> np.ndarray:
        N, q, L, s, z = self.N, self.q, self.L, self.s, self.z
        lB = L - s
        nA, nB = 1 << s, 1 << lB
        f = np.asarray(f, dtype=np.complex128).reshape(-1)
        b = [box_of(self.p[d], lB) for d in range(3)]
        u = [(self.p[d] - centre(lB, b[d])) * nB for d in range(3)]          # local coordinates
        lag = (lagrange(u[0], z)[:, :, None, None] * lagrange(u[1], z)[:, None, :, None]
               * lagrange(u[2], z)[:, None, None, :]).reshape(N ** 3, q ** 3)  # L^B_t(p)
        onehot = sp.csr_matrix((np.ones(N ** 3), ((b[0] * nB + b[1]) * nB + b[2], np.arange(N ** 3))),
                               shape=(nB ** 3, N ** 3))
        pn = nodes(lB, np.arange(nB), z)                                      # (nB, q)
        P1 = pn[:, None, None, :, None, None]
        P2 = pn[None, :, None, None, :, None]
        P3 = pn[None, None, :, None, None, :]
        out = np.zeros((nA, nA, nA, nB, nB, nB, q, q, q), dtype=np.complex128)
        for a1 in range(nA):
            for a2 in range(nA):
                for a3 in range(nA):
                    x0 = centre(s, a1), centre(s, a2), centre(s, a3)
                    g = self.E(*x0, *self.k) * f                              # E(x0(A), p) f(p)
                    acc = (onehot @ (g[:, None] * lag)).reshape(nB, nB, nB, q, q, q)
                    out[a1, a2, a3] = np.conj(self.E_p(*x0, P1, P2, P3)) * acc
        return out

    # -- 1-D interpolation matrices (Sec. 4; the same in every dimension) ----
    def child_interp(self):
        """Mc[c, t, t'] = L_t((z_t' + c - 1/2) / 2): parent basis t at child node t'."""
        z = self.z
        return np.stack([lagrange((z + c - 0.5) / 2.0, z).T for c in (0, 1)])

    # -- step 3: p-recursion (eq:alg2b) ------------------------------------
    def p_level(self, prev: np.ndarray, l: int) -> np.ndarray:
        q, L, z = self.q, self.L, self.z
        lB = L - l
        nA, nB = 1 << l, 1 << lB
        Mc = self.child_interp()                                              # (c, t, t')
        pc = nodes(lB + 1, np.arange(2 * nB), z).reshape(2 * nB, q)          # child nodes per dim
        pn = nodes(lB, np.arange(nB), z)
        out = np.zeros((nA, nA, nA, nB, nB, nB, q, q, q), dtype=np.complex128)
        for a1 in range(nA):
            for a2 in range(nA):
                for a3 in range(nA):
                    x0 = centre(l, a1), centre(l, a2), centre(l, a3)
                    # prefactor E(x0(A), p^{B_c}_t') on the grid of all children
                    G = self.E_p(*x0, *self._grid(pc.ravel(), pc.ravel(), pc.ravel()))
                    G = G.reshape(2 * nB, q, 2 * nB, q, 2 * nB, q).transpose(0, 2, 4, 1, 3, 5)
                    V = G * prev[a1 // 2, a2 // 2, a3 // 2]                   # (bc1,bc2,bc3,t'1,t'2,t'3)
                    V = V.reshape(nB, 2, nB, 2, nB, 2, q, q, q)
                    # sum over children c and nodes t' of prod_d Mc[c_d, t_d, t'_d]
                    acc = np.einsum("xaybzcklm,aik,bjl,cpm->xyzijp", V, Mc, Mc, Mc, optimize=True)
                    post = np.conj(self.E_p(*x0, pn[:, None, None, :, None, None],
                                            pn[None, :, None, None, :, None], pn[None, None, :, None, None, :]))
                    out[a1, a2, a3] = post * acc
        return out

    # -- step 4: switch (eq:alg2m) -----------------------------------------
    def switch(self, d: np.ndarray) -> np.ndarray:
        q, L, l, z = self.q, self.L, self.lm, self.z
        nA, nB = 1 << l, 1 << (L - l)
        pn = nodes(L - l, np.arange(nB), z)                                   # (nB, q)
        out = np.zeros_like(d)
        for a1 in range(nA):
            for a2 in range(nA):
                for a3 in range(nA):
                    xa = nodes(l, a1, z), nodes(l, a2, z), nodes(l, a3, z)
                    X = [v.reshape((1,) * 3 + tuple(q if j == i else 1 for j in range(3)) + (1,) * 3)
                         for i, v in enumerate(xa)]
                    P = [pn.reshape(tuple(nB if j == i else 1 for j in range(3)) + (1,) * 3
                                    + tuple(q if j == i else 1 for j in range(3))) for i in range(3)]
                    K = self.E_p(*X, *P)                                      # (b, t, s)
                    out[a1, a2, a3] = np.einsum("xyzijkabc,xyzabc->xyzijk", K, d[a1, a2, a3], optimize=True)
        return out

    # -- step 5: x-recursion (eq:alg2c) ------------------------------------
    def x_level(self, prev: np.ndarray, l: int) -> np.ndarray:
        q, L, z = self.q, self.L, self.z
        lB = L - l
        nA, nB = 1 << l, 1 << lB
        Mc = self.child_interp()                         # Mc[a, t', t] = L_t'(x^A_t), A the child a of A_p
        pc0 = centre(lB + 1, np.arange(2 * nB))          # p0(B_c) per dimension
        PC = [pc0.reshape(tuple(2 * nB if j == i else 1 for j in range(3)) + (1, 1, 1)) for i in range(3)]
        out = np.zeros((nA, nA, nA, nB, nB, nB, q, q, q), dtype=np.complex128)
        for a1 in range(nA):
            for a2 in range(nA):
                for a3 in range(nA):
                    ap = a1 // 2, a2 // 2, a3 // 2
                    xp = [nodes(l - 1, ap[i], z).reshape((1, 1, 1) + tuple(q if j == i else 1 for j in range(3)))
                          for i in range(3)]
                    W = np.conj(self.E_p(*xp, *PC)) * prev[ap]               # (bc1,bc2,bc3,t'1,t'2,t'3)
                    W = np.einsum("uvwklm,ki,lj,mp->uvwijp", W, Mc[a1 & 1], Mc[a2 & 1], Mc[a3 & 1], optimize=True)
                    xa = [nodes(l, (a1, a2, a3)[i], z).reshape((1, 1, 1) + tuple(q if j == i else 1 for j in range(3)))
                          for i in range(3)]
                    R = self.E_p(*xa, *PC)
                    T = (R * W).reshape(nB, 2, nB, 2, nB, 2, q, q, q)
                    out[a1, a2, a3] = T.sum(axis=(1, 3, 5))
        return out

    # -- step 6: termination (eq:alg2d) ------------------------------------
    def terminate(self, d: np.ndarray) -> np.ndarray:
        N, q, L, s, z = self.N, self.q, self.L, self.s, self.z
        lA = L - s
        nA, nB, m = 1 << lA, 1 << s, 1 << s
        Tm = lagrange(np.arange(m) / m - 0.5, z)                               # (j, t)
        p0 = centre(s, np.arange(nB))
        PB = [p0.reshape(tuple(nB if j == i else 1 for j in range(3)) + (1, 1, 1)) for i in range(3)]
        u = np.zeros((N, N, N), dtype=np.complex128)
        for a1 in range(nA):
            for a2 in range(nA):
                for a3 in range(nA):
                    a = (a1, a2, a3)
                    xa = [nodes(lA, a[i], z).reshape((1, 1, 1) + tuple(q if j == i else 1 for j in range(3)))
                          for i in range(3)]
                    pre = np.conj(self.E_p(*xa, *PB)) * d[a]
                    V = np.einsum("ik,jl,pm,xyzklm->xyzijp", Tm, Tm, Tm, pre, optimize=True)
                    xg = [((a[i] * m + np.arange(m)) / N).reshape((1, 1, 1) + tuple(m if j == i else 1
                                                                                    for j in range(3)))
                          for i in range(3)]
                    post = self.E_p(*xg, *PB)
                    u[a1 * m:(a1 + 1) * m, a2 * m:(a2 + 1) * m, a3 * m:(a3 + 1) * m] = (post * V).sum(axis=(0, 1, 2))
        return u

    # -- full pass -----------------------------------------------------------
    def apply(self, f: np.ndarray, return_levels: bool = False):
        lev = {}
        d = self.init(f)
        lev["init"] = d
        for l in range(self.s + 1, self.lm + 1):
            d = self.p_level(d, l)
            lev[("p", l)] = d
        d = self.switch(d)
        lev["switch"] = d
        for l in range(self.lm + 1, self.L - self.s + 1):
            d = self.x_level(d, l)
            lev[("x", l)] = d
        u = self.terminate(d)
        return (u, lev) if return_levels else u
