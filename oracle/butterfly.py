"""Step-by-step FP64 model of the butterfly FIO algorithm (TEST INFRASTRUCTURE
ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may import this module; the product path never does).

The butterfly is an approximation of eq:dfio, so this oracle takes the
algorithm's own steps in the paper's order and notation (Sec. 4), in plain
vectorised numpy, FP64 throughout:

  0. trees (Sec. 4 step 1) and the polar map p(k) (eq:polar, Sec. 1);
  1. initialisation (eq:alg2a) at pairs (A at level s, B at level L-s);
  2. p-recursion (eq:alg2b) for levels s+1 .. lm;
  3. switch (eq:alg2m) at level lm;
  4. x-recursion (eq:alg2c) for levels lm+1 .. L-s;
  5. termination (eq:alg2d) at pairs (A at level L-s, B at level s),
     summed over the 4^s boxes B.

s is the number of levels skipped at each end of the trees (the numerical
section starts the recursion at level log2(N)-3 of T_P and stops at level 3);
s = 0 is the algorithm of Sec. 4 verbatim.  The adjoint applies the
conjugate transpose of every step in reverse order.

Nothing here is blocked, fused or reordered beyond the formulas: every
Lagrange value L^B_t(p) is evaluated from the product formula at the actual
point (Sec. 3, Chebyshev grid paragraph) and every kernel value from the
phase's definition at the actual (x, k(p)).

Readings of points the paper leaves open (each is also listed with its
reason in the design notes):
  * q is the number of Chebyshev points per dimension, z_i = cos(i pi/(q-1))/2;
  * box of p at level l: min(floor(p 2^l), 2^l - 1) per dimension (half-open,
    clamped); p1 = sqrt(2 (k1^2+k2^2))/N, p2 = atan2(k2,k1)/(2 pi) mod 1, and
    k = 0 maps to p = (0,0) (Phi(x,0) = 0 by homogeneity);
  * s = min(3, floor(L/2)) and lm = floor(L/2) by default, both options;
  * the sources' own kernel values use their integer k; Chebyshev nodes in P
    use k(p) = (sqrt(2)/2) N p1 (cos 2 pi p2, sin 2 pi p2).

Weights at level l are arrays delta[a1, a2, b1, b2, t1, t2]: (a1,a2) is the
box A at level l of T_X, (b1,b2) the box B at level L-l of T_P, (t1,t2) the
tensor Chebyshev index.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .direct import Phase, cis_np, phi_np

SQRT2_2 = math.sqrt(2.0) / 2.0


# ----------------------------------------------------------------------------
# Chebyshev grid and Lagrange basis (Sec. 3)
# ----------------------------------------------------------------------------

def cheb_nodes(q: int) -> np.ndarray:
    """z_i = cos(i pi / (q-1)) / 2, i = 0..q-1, on [-1/2, 1/2]."""
    return 0.5 * np.cos(np.arange(q) * np.pi / (q - 1))


def lagrange(xi, z: np.ndarray) -> np.ndarray:
    """L_i(xi) = prod_{j != i} (xi - z_j) / (z_i - z_j); returns (..., q)."""
    xi = np.asarray(xi, dtype=np.float64)[..., None]
    q = z.shape[0]
    out = np.ones(xi.shape[:-1] + (q,), dtype=np.float64)
    for i in range(q):
        for j in range(q):
            if j != i:
                out[..., i] *= (xi[..., 0] - z[j]) / (z[i] - z[j])
    return out


# ----------------------------------------------------------------------------
# Trees and the polar map (eq:polar, Sec. 4 step 1)
# ----------------------------------------------------------------------------

def centre(level: int, b):
    return (np.asarray(b, dtype=np.float64) + 0.5) / (1 << level)


def nodes(level: int, b, z):
    """1-D Chebyshev nodes of the boxes b at ``level``: (..., q)."""
    return centre(level, b)[..., None] + z / (1 << level)


def polar_points(N: int):
    """(k1, k2, p1, p2) for every k in Omega in row order (k1 major)."""
    k = np.arange(N, dtype=np.float64) - N // 2
    k1, k2 = np.meshgrid(k, k, indexing="ij")
    k1, k2 = k1.ravel(), k2.ravel()
    p1 = np.sqrt(2.0 * (k1 * k1 + k2 * k2)) / N
    p2 = np.arctan2(k2, k1) / (2.0 * np.pi)
    p2 = np.where(p2 < 0.0, p2 + 1.0, p2)
    return k1, k2, p1, p2


def box_of(p, level: int):
    n = 1 << level
    return np.minimum(np.floor(np.asarray(p) * n).astype(np.int64), n - 1)


def k_of_p(N: int, p1, p2):
    """Inverse polar map k(p) = (sqrt(2)/2) N p1 (cos 2 pi p2, sin 2 pi p2)."""
    rho = SQRT2_2 * N * np.asarray(p1, dtype=np.float64)
    th = 2.0 * np.pi * np.asarray(p2, dtype=np.float64)
    return rho * np.cos(th), rho * np.sin(th)


def default_schedule(N: int):
    L = int(round(math.log2(N)))
    return min(3, L // 2), L // 2


# ----------------------------------------------------------------------------
# The model
# ----------------------------------------------------------------------------

class ButterflyModel:
    """FP64 butterfly of Sec. 4 with start offset ``s`` and switch level ``lm``."""

    def __init__(self, N: int, q: int, phase: Phase, s: int | None = None, lm: int | None = None):
        L = int(round(math.log2(N)))
        if (1 << L) != N or N < 4:
            raise ValueError("N must be a power of two >= 4")
        if q < 2:
            raise ValueError("q must be >= 2")
        ds, dlm = default_schedule(N)
        self.N, self.q, self.L, self.ph = N, q, L, phase
        self.s = ds if s is None else int(s)
        self.lm = dlm if lm is None else int(lm)
        if not (0 <= self.s <= self.lm <= L - self.s):
            raise ValueError(f"need 0 <= s <= lm <= L-s (s={self.s}, lm={self.lm}, L={L})")
        self.z = cheb_nodes(q)
        self.k1, self.k2, self.p1, self.p2 = polar_points(N)
        self.active = None     # {level: sorted list of (a1, a2)} when restricted

    # -- which boxes A a step computes -----------------------------------
    def boxes(self, l: int):
        """Boxes A of T_X at level l that the steps compute (all by default)."""
        if self.active is None:
            n = 1 << l
            return [(a1, a2) for a1 in range(n) for a2 in range(n)]
        return self.active[l]

    def new_level(self, l: int, nB: int):
        """Weights of level l: a dense array, or a dict keyed by (a1, a2) when
        only the ancestors of some target boxes are computed."""
        if self.active is None:
            return np.zeros((1 << l, 1 << l, nB, nB, self.q, self.q), dtype=np.complex128)
        return {}

    # -- kernel values ---------------------------------------------------
    def E(self, x1, x2, k1, k2):
        """exp(2 pi i Phi(x,k)) evaluated from the definition (broadcasting)."""
        return cis_np(phi_np(self.ph, x1, x2, k1, k2))

    def E_p(self, x1, x2, p1, p2):
        """exp(2 pi i N Psi(x,p)) = exp(2 pi i Phi(x, k(p)))."""
        k1, k2 = k_of_p(self.N, p1, p2)
        return self.E(x1, x2, k1, k2)

    # -- step 2: initialisation (eq:alg2a) -------------------------------
    def init(self, f: np.ndarray) -> np.ndarray:
        N, q, L, s, z = self.N, self.q, self.L, self.s, self.z
        lB = L - s
        nA, nB = 1 << s, 1 << lB
        f = np.asarray(f, dtype=np.complex128).reshape(-1)
        b1, b2 = box_of(self.p1, lB), box_of(self.p2, lB)
        u1 = (self.p1 - centre(lB, b1)) * nB          # local coordinate in [-1/2, 1/2]
        u2 = (self.p2 - centre(lB, b2)) * nB
        lag = lagrange(u1, z)[:, :, None] * lagrange(u2, z)[:, None, :]   # L^B_t(p)
        lag = lag.reshape(N * N, q * q)
        onehot = sp.csr_matrix((np.ones(N * N), (b1 * nB + b2, np.arange(N * N))),
                               shape=(nB * nB, N * N))
        # Chebyshev nodes of every B (for the remodulation)
        pn1 = nodes(lB, np.arange(nB), z)                 # (nB, q)  p1 nodes
        pn2 = nodes(lB, np.arange(nB), z)                 # (nB, q)  p2 nodes
        P1 = pn1[:, None, :, None]                        # (b1, b2, t1, t2)
        P2 = pn2[None, :, None, :]
        out = self.new_level(s, nB)
        for a1, a2 in self.boxes(s):
                x01, x02 = centre(s, a1), centre(s, a2)
                g = self.E(x01, x02, self.k1, self.k2) * f                 # E(x0(A),p) f(p)
                acc = onehot @ (g[:, None] * lag)                          # sum_{p in B}
                acc = acc.reshape(nB, nB, q, q)
                out[a1, a2] = np.conj(self.E_p(x01, x02, P1, P2)) * acc
        return out

    # -- step 3: p-recursion (eq:alg2b) ----------------------------------
    def p_interp(self, lB: int) -> np.ndarray:
        """Lm[b, c, t, t'] = L^B_t(p^{B_c}_t') for boxes b at level lB of T_P (1-D)."""
        z, nB = self.z, 1 << lB
        b = np.arange(nB)
        child = 2 * b[:, None] + np.arange(2)[None, :]                      # (b, c)
        cn = nodes(lB + 1, child, z)                                        # (b, c, t')
        loc = (cn - centre(lB, b)[:, None, None]) * nB                      # parent-local
        return np.transpose(lagrange(loc, z), (0, 1, 3, 2))

    def p_level(self, prev: np.ndarray, l: int) -> np.ndarray:
        q, L, z = self.q, self.L, self.z
        lB = L - l                       # level of B; children at lB+1
        nA, nB = 1 << l, 1 << lB
        b = np.arange(nB)
        Lm = self.p_interp(lB)                                              # (b, c, t, t')
        # prefactor grid over all children B_c at level lB+1
        pc = nodes(lB + 1, np.arange(2 * nB), z).reshape(-1)                # (2nB*q,)
        PC1, PC2 = pc[:, None], pc[None, :]
        pn = nodes(lB, b, z)                                                # (nB, q)
        PN1 = pn[:, None, :, None]
        PN2 = pn[None, :, None, :]
        out = self.new_level(l, nB)
        for a1, a2 in self.boxes(l):
                x01, x02 = centre(l, a1), centre(l, a2)
                pre = self.E_p(x01, x02, PC1, PC2)                          # (2nB q, 2nB q)
                pre = pre.reshape(2 * nB, q, 2 * nB, q).transpose(0, 2, 1, 3)
                V = pre * prev[a1 // 2, a2 // 2]                            # (bc1, bc2, t'1, t'2)
                V = V.reshape(nB, 2, nB, 2, q, q)                           # (b1,c1,b2,c2,t'1,t'2)
                acc = np.einsum("xcydkl,xcik,ydjl->xyij", V, Lm, Lm, optimize=True)
                out[a1, a2] = np.conj(self.E_p(x01, x02, PN1, PN2)) * acc
        return out

    # -- step 4: switch (eq:alg2m) ---------------------------------------
    def switch_kernel(self, a1: int, a2: int) -> np.ndarray:
        """K[b1, b2, t1, t2, s1, s2] = exp(2 pi i N Psi(x^A_t, p^B_s)) for A=(a1,a2)."""
        q, L, l, z = self.q, self.L, self.lm, self.z
        nB = 1 << (L - l)
        xa1, xa2 = nodes(l, a1, z), nodes(l, a2, z)                        # (q,), (q,)
        pn = nodes(L - l, np.arange(nB), z)                                 # (nB, q)
        X1 = xa1[None, None, :, None, None, None]
        X2 = xa2[None, None, None, :, None, None]
        P1 = pn[:, None, None, None, :, None]
        P2 = pn[None, :, None, None, None, :]
        return self.E_p(X1, X2, P1, P2)

    def switch(self, d: np.ndarray) -> np.ndarray:
        out = self.new_level(self.lm, 1 << (self.L - self.lm))
        for a1, a2 in self.boxes(self.lm):
                K = self.switch_kernel(a1, a2)
                out[a1, a2] = np.einsum("xyijkl,xykl->xyij", K, d[a1, a2], optimize=True)
        return out

    # -- step 5: x-recursion (eq:alg2c) ----------------------------------
    def x_interp(self, l: int) -> np.ndarray:
        """Xm[a, t, t'] = L^{A_p}_{t'}(x^A_t) for boxes a at level l (1-D)."""
        z = self.z
        a = np.arange(1 << l)
        xn = nodes(l, a, z)                                                  # (a, t)
        loc = (xn - centre(l - 1, a // 2)[:, None]) * (1 << (l - 1))        # parent-local
        return lagrange(loc, z)                                              # (a, t, t')

    def x_level(self, prev: np.ndarray, l: int) -> np.ndarray:
        q, L, z = self.q, self.L, self.z
        lB = L - l
        nA, nB = 1 << l, 1 << lB
        Xm = self.x_interp(l)
        pc0 = centre(lB + 1, np.arange(2 * nB))                              # p0(B_c)
        PC1 = pc0[:, None, None, None]
        PC2 = pc0[None, :, None, None]
        out = self.new_level(l, nB)
        for a1, a2 in self.boxes(l):
                ap1, ap2 = a1 // 2, a2 // 2
                xp1, xp2 = nodes(l - 1, ap1, z), nodes(l - 1, ap2, z)
                pre = np.conj(self.E_p(xp1[None, None, :, None], xp2[None, None, None, :], PC1, PC2))
                W = pre * prev[ap1, ap2]                                     # (bc1, bc2, t'1, t'2)
                W = np.einsum("ik,jl,xykl->xyij", Xm[a1], Xm[a2], W, optimize=True)
                xa1, xa2 = nodes(l, a1, z), nodes(l, a2, z)
                R = self.E_p(xa1[None, None, :, None], xa2[None, None, None, :], PC1, PC2)
                T = (R * W).reshape(nB, 2, nB, 2, q, q)
                out[a1, a2] = T.sum(axis=(1, 3))
        return out

    # -- step 6: termination (eq:alg2d) ----------------------------------
    def term_interp(self):
        """Tm[j, t] = L^A_t(x) for the 2^s grid points x of a box A at level L-s."""
        s = self.s
        xi = (np.arange(1 << s) + 0.0) / (1 << s) - 0.5                     # (x - x0(A)) / w(A)
        return lagrange(xi, self.z)

    def terminate(self, d: np.ndarray) -> np.ndarray:
        N, q, L, s, z = self.N, self.q, self.L, self.s, self.z
        lA = L - s
        nA, nB, m = 1 << lA, 1 << s, 1 << s
        Tm = self.term_interp()                                             # (j, t)
        p0 = centre(s, np.arange(nB))
        PB1 = p0[:, None, None, None]
        PB2 = p0[None, :, None, None]
        u = np.zeros((N, N), dtype=np.complex128)
        for a1, a2 in self.boxes(lA):
                xa1, xa2 = nodes(lA, a1, z), nodes(lA, a2, z)
                pre = np.conj(self.E_p(xa1[None, None, :, None], xa2[None, None, None, :], PB1, PB2))
                V = np.einsum("ik,jl,xykl->xyij", Tm, Tm, pre * d[a1, a2], optimize=True)
                xg1 = (a1 * m + np.arange(m)) / N
                xg2 = (a2 * m + np.arange(m)) / N
                post = self.E_p(xg1[None, None, :, None], xg2[None, None, None, :], PB1, PB2)
                u[a1 * m:(a1 + 1) * m, a2 * m:(a2 + 1) * m] = (post * V).sum(axis=(0, 1))
        return u

    # -- full pass ---------------------------------------------------------
    def apply(self, f: np.ndarray, return_levels: bool = False, targets=None):
        """u = B f.  With ``return_levels`` also returns a dict of the weights:
        'init', ('p', l), 'switch', ('x', l).

        ``targets``: optional list of boxes (a1, a2) at level L-s of T_X; then
        only the pairs whose A is one of their ancestors are computed (the same
        formulas, restricted loops), u is exact only on those boxes and zero
        elsewhere, and the levels are dicts keyed by (a1, a2)."""
        if targets is None:
            self.active = None
        else:
            top = self.L - self.s
            self.active = {l: sorted({(a1 >> (top - l), a2 >> (top - l)) for a1, a2 in targets})
                           for l in range(self.s, top + 1)}
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

    # ========================================================================
    # Adjoint: conjugate transpose of each step, in reverse order
    # ========================================================================
    def terminate_adj(self, u: np.ndarray) -> np.ndarray:
        N, q, L, s, z = self.N, self.q, self.L, self.s, self.z
        lA = L - s
        nA, nB, m = 1 << lA, 1 << s, 1 << s
        Tm = self.term_interp()
        p0 = centre(s, np.arange(nB))
        PB1 = p0[:, None, None, None]
        PB2 = p0[None, :, None, None]
        u = np.asarray(u, dtype=np.complex128).reshape(N, N)
        d = np.zeros((nA, nA, nB, nB, q, q), dtype=np.complex128)
        for a1 in range(nA):
            for a2 in range(nA):
                xa1, xa2 = nodes(lA, a1, z), nodes(lA, a2, z)
                xg1 = (a1 * m + np.arange(m)) / N
                xg2 = (a2 * m + np.arange(m)) / N
                post = self.E_p(xg1[None, None, :, None], xg2[None, None, None, :], PB1, PB2)
                V = np.conj(post) * u[a1 * m:(a1 + 1) * m, a2 * m:(a2 + 1) * m][None, None]
                W = np.einsum("ik,jl,xyij->xykl", Tm, Tm, V, optimize=True)
                pre = self.E_p(xa1[None, None, :, None], xa2[None, None, None, :], PB1, PB2)
                d[a1, a2] = pre * W
        return d

    def x_level_adj(self, dout: np.ndarray, l: int) -> np.ndarray:
        q, L, z = self.q, self.L, self.z
        lB = L - l
        nA, nB = 1 << l, 1 << lB
        Xm = self.x_interp(l)
        pc0 = centre(lB + 1, np.arange(2 * nB))
        PC1 = pc0[:, None, None, None]
        PC2 = pc0[None, :, None, None]
        din = np.zeros((nA // 2, nA // 2, 2 * nB, 2 * nB, q, q), dtype=np.complex128)
        for a1 in range(nA):
            for a2 in range(nA):
                ap1, ap2 = a1 // 2, a2 // 2
                xa1, xa2 = nodes(l, a1, z), nodes(l, a2, z)
                R = self.E_p(xa1[None, None, :, None], xa2[None, None, None, :], PC1, PC2)
                # broadcast the output of B to its four children B_c
                T = np.repeat(np.repeat(dout[a1, a2], 2, axis=0), 2, axis=1)
                W = np.conj(R) * T
                W = np.einsum("ik,jl,xyij->xykl", Xm[a1], Xm[a2], W, optimize=True)
                xp1, xp2 = nodes(l - 1, ap1, z), nodes(l - 1, ap2, z)
                pre = self.E_p(xp1[None, None, :, None], xp2[None, None, None, :], PC1, PC2)
                din[ap1, ap2] += pre * W
        return din

    def switch_adj(self, d: np.ndarray) -> np.ndarray:
        nA = 1 << self.lm
        out = np.empty_like(d)
        for a1 in range(nA):
            for a2 in range(nA):
                K = self.switch_kernel(a1, a2)
                out[a1, a2] = np.einsum("xyijkl,xyij->xykl", np.conj(K), d[a1, a2], optimize=True)
        return out

    def p_level_adj(self, dout: np.ndarray, l: int) -> np.ndarray:
        q, L, z = self.q, self.L, self.z
        lB = L - l
        nA, nB = 1 << l, 1 << lB
        b = np.arange(nB)
        Lm = self.p_interp(lB)                                              # (b, c, t, t')
        pc = nodes(lB + 1, np.arange(2 * nB), z).reshape(-1)
        PC1, PC2 = pc[:, None], pc[None, :]
        pn = nodes(lB, b, z)
        PN1 = pn[:, None, :, None]
        PN2 = pn[None, :, None, :]
        din = np.zeros((nA // 2, nA // 2, 2 * nB, 2 * nB, q, q), dtype=np.complex128)
        for a1 in range(nA):
            for a2 in range(nA):
                x01, x02 = centre(l, a1), centre(l, a2)
                G = self.E_p(x01, x02, PN1, PN2) * dout[a1, a2]             # (b1, b2, t1, t2)
                V = np.einsum("xyij,xcik,ydjl->xcydkl", G, Lm, Lm, optimize=True)
                V = V.reshape(2 * nB, 2 * nB, q, q)
                pre = self.E_p(x01, x02, PC1, PC2)
                pre = pre.reshape(2 * nB, q, 2 * nB, q).transpose(0, 2, 1, 3)
                din[a1 // 2, a2 // 2] += np.conj(pre) * V
        return din

    def init_adj(self, d: np.ndarray) -> np.ndarray:
        N, q, L, s, z = self.N, self.q, self.L, self.s, self.z
        lB = L - s
        nA, nB = 1 << s, 1 << lB
        b1, b2 = box_of(self.p1, lB), box_of(self.p2, lB)
        u1 = (self.p1 - centre(lB, b1)) * nB
        u2 = (self.p2 - centre(lB, b2)) * nB
        lag = lagrange(u1, z)[:, :, None] * lagrange(u2, z)[:, None, :]
        lag = lag.reshape(N * N, q * q)
        pn1 = nodes(lB, np.arange(nB), z)
        P1 = pn1[:, None, :, None]
        P2 = pn1[None, :, None, :]
        f = np.zeros(N * N, dtype=np.complex128)
        for a1 in range(nA):
            for a2 in range(nA):
                x01, x02 = centre(s, a1), centre(s, a2)
                W = (self.E_p(x01, x02, P1, P2) * d[a1, a2]).reshape(nB * nB, q * q)
                val = np.sum(lag * W[b1 * nB + b2], axis=1)                 # sum_t L^B_t(p) ...
                f += np.conj(self.E(x01, x02, self.k1, self.k2)) * val
        return f.reshape(N, N)

    # ------------------------------------------------------------------------
    # Adjoint restricted to some source boxes: the same conjugate-transposed
    # formulas, with the loops taken over every box A of T_X and only over the
    # boxes B of T_P that are ancestors of the chosen source boxes (in the
    # adjoint the weights of pair (A, B) feed only the sources inside B).
    # Weights of level l are dicts keyed by B at level L-l, each an array
    # [a1, a2, t1, t2] over all A at level l.
    # ------------------------------------------------------------------------
    def terminate_adj_restricted(self, u: np.ndarray, act) -> dict:
        N, q, L, s, z = self.N, self.q, self.L, self.s, self.z
        lA = L - s
        nA, m = 1 << lA, 1 << s
        Tm = self.term_interp()                                             # (j, t)
        xa = nodes(lA, np.arange(nA), z)                                    # (a, t)
        xg = (np.arange(nA)[:, None] * m + np.arange(m)[None, :]) / N      # (a, j) grid points
        U = np.asarray(u, dtype=np.complex128).reshape(nA, m, nA, m).transpose(0, 2, 1, 3)
        d = {}
        for b1, b2 in act:
            p01, p02 = centre(s, b1), centre(s, b2)
            post = self.E_p(xg[:, None, :, None], xg[None, :, None, :], p01, p02)      # (a1, a2, i, j)
            W = np.einsum("ik,jl,xyij->xykl", Tm, Tm, np.conj(post) * U, optimize=True)
            pre = self.E_p(xa[:, None, :, None], xa[None, :, None, :], p01, p02)        # (a1, a2, k, l)
            d[(b1, b2)] = pre * W
        return d

    def x_level_adj_restricted(self, dout: dict, l: int, act_children) -> dict:
        q, L, z = self.q, self.L, self.z
        lB = L - l
        nA = 1 << l
        Xm = self.x_interp(l)                                               # (a, t, t')
        xa = nodes(l, np.arange(nA), z)
        xp = nodes(l - 1, np.arange(nA // 2), z)
        din = {}
        for c1, c2 in act_children:                                         # B_c at level lB+1
            pc1, pc2 = centre(lB + 1, c1), centre(lB + 1, c2)
            R = self.E_p(xa[:, None, :, None], xa[None, :, None, :], pc1, pc2)          # (a1, a2, t1, t2)
            W = np.conj(R) * dout[(c1 >> 1, c2 >> 1)]
            W = np.einsum("xik,yjl,xyij->xykl", Xm, Xm, W, optimize=True)             # parent nodes t'
            W = W.reshape(nA // 2, 2, nA // 2, 2, q, q).sum(axis=(1, 3))              # sum over children A
            pre = self.E_p(xp[:, None, :, None], xp[None, :, None, :], pc1, pc2)
            din[(c1, c2)] = pre * W
        return din

    def switch_adj_restricted(self, d: dict) -> dict:
        q, L, l, z = self.q, self.L, self.lm, self.z
        lB = L - l
        nA = 1 << l
        xa = nodes(l, np.arange(nA), z)
        X1 = xa[:, None, :, None, None, None]
        X2 = xa[None, :, None, :, None, None]
        out = {}
        for (b1, b2), w in d.items():
            pn1, pn2 = nodes(lB, b1, z), nodes(lB, b2, z)
            K = self.E_p(X1, X2, pn1[None, None, None, None, :, None], pn2[None, None, None, None, None, :])
            out[(b1, b2)] = np.einsum("xyijkl,xyij->xykl", np.conj(K), w, optimize=True)
        return out

    def p_level_adj_restricted(self, dout: dict, l: int, act_children) -> dict:
        q, L, z = self.q, self.L, self.z
        lB = L - l
        nA = 1 << l
        Lm = self.p_interp(lB)                                              # (b, c, t, t')
        x0 = centre(l, np.arange(nA))
        X1, X2 = x0[:, None, None, None], x0[None, :, None, None]
        din = {}
        for c1, c2 in act_children:                                         # B_c at level lB+1
            b1, b2 = c1 >> 1, c2 >> 1
            pn1, pn2 = nodes(lB, b1, z), nodes(lB, b2, z)
            G = self.E_p(X1, X2, pn1[None, None, :, None], pn2[None, None, None, :]) * dout[(b1, b2)]
            V = np.einsum("xyij,ik,jl->xykl", G, Lm[b1, c1 & 1], Lm[b2, c2 & 1], optimize=True)
            pc1, pc2 = nodes(lB + 1, c1, z), nodes(lB + 1, c2, z)
            pre = self.E_p(X1, X2, pc1[None, None, :, None], pc2[None, None, None, :])
            V = np.conj(pre) * V
            din[(c1, c2)] = V.reshape(nA // 2, 2, nA // 2, 2, q, q).sum(axis=(1, 3))
        return din

    def init_adj_restricted(self, d: dict) -> np.ndarray:
        N, q, L, s, z = self.N, self.q, self.L, self.s, self.z
        lB = L - s
        nA, nB = 1 << s, 1 << lB
        b1s, b2s = box_of(self.p1, lB), box_of(self.p2, lB)
        x0 = centre(s, np.arange(nA))
        X1, X2 = x0[:, None, None, None], x0[None, :, None, None]
        f = np.zeros(N * N, dtype=np.complex128)
        for (b1, b2), w in d.items():
            j = np.nonzero((b1s == b1) & (b2s == b2))[0]                    # sources in B
            if j.size == 0:
                continue
            u1 = (self.p1[j] - centre(lB, b1)) * nB
            u2 = (self.p2[j] - centre(lB, b2)) * nB
            lag = (lagrange(u1, z)[:, :, None] * lagrange(u2, z)[:, None, :]).reshape(j.size, q * q)
            pn1, pn2 = nodes(lB, b1, z), nodes(lB, b2, z)
            W = (self.E_p(X1, X2, pn1[None, None, :, None], pn2[None, None, None, :]) * w).reshape(nA * nA, q * q)
            val = W @ lag.T                                                 # (A, source)
            e = self.E(x0[:, None, None], x0[None, :, None], self.k1[j][None, None, :], self.k2[j][None, None, :])
            f[j] = np.sum(np.conj(e).reshape(nA * nA, j.size) * val, axis=0)
        return f.reshape(N, N)

    def adjoint(self, u: np.ndarray, sources=None) -> np.ndarray:
        """f = B^H u (the exact conjugate transpose of ``apply``).

        ``sources``: optional list of boxes (b1, b2) at level L-s of T_P; then
        only the pairs whose B is one of their ancestors are computed (the same
        formulas, restricted loops), f is exact on the sources inside those
        boxes and zero elsewhere."""
        if sources is not None:
            top = self.L - self.s
            act = {m: sorted({(b1 >> (top - m), b2 >> (top - m)) for b1, b2 in sources})
                   for m in range(self.s, top + 1)}
            d = self.terminate_adj_restricted(u, act[self.s])
            for l in range(self.L - self.s, self.lm, -1):
                d = self.x_level_adj_restricted(d, l, act[self.L - l + 1])
            d = self.switch_adj_restricted(d)
            for l in range(self.lm, self.s, -1):
                d = self.p_level_adj_restricted(d, l, act[self.L - l + 1])
            return self.init_adj_restricted(d)
        d = self.terminate_adj(u)
        for l in range(self.L - self.s, self.lm, -1):
            d = self.x_level_adj(d, l)
        d = self.switch_adj(d)
        for l in range(self.lm, self.s, -1):
            d = self.p_level_adj(d, l)
        return self.init_adj(d)
