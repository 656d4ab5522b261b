// Three-dimensional butterfly (Sec. 5, last example; eq:ex3): the steps of
// Sec. 4 with q x q x q tensor Chebyshev grids, octrees (eight children per
// box) and l(A) + l(B) = L.  The frequencies are mapped to spherical
// coordinates p = (|k| / (sqrt(3) N / 2), theta / pi, phi / (2 pi)), so by
// homogeneity Phi(x, k(p)) = rho(p1) G(x, p2, p3) with
//     G(x, p2, p3) = x . e(theta, phi) + c(x),   e = (sin th cos ph, sin th sin ph, cos th),
// c(x) = (3 + sin 2 pi x1 sin 2 pi x2 sin 2 pi x3) / 4 for eq:ex3 and 0 for x . k.
//
// Layout: boxes by row-major index (b1 n + b2) n + b3 at their level;
// weights w[(idxA nB^3 + idxB) q^3 + (t1 q + t2) q + t3].  One workgroup per
// box pair (per box A for the termination); the Kronecker contractions over
// the eight children run as three one-dimensional passes through LDS, so a
// p- or x-level costs 14 q^4 (p) or 24 q^4 (x) real-by-complex products per
// pair instead of 8 q^6.
#include <hip/hip_runtime.h>

#include "fio_kernels_common.h"

namespace fio {

namespace {

struct XP3 {
    double x1, x2, x3, c;
};

__device__ __forceinline__ XP3 make_xp3(const Geom3 &g, double x1, double x2, double x3) {
    XP3 r{x1, x2, x3, 0.0};
    if (g.kind == FIO3_PHASE_SPHERES) r.c = (3.0 + sinpi(2.0 * x1) * sinpi(2.0 * x2) * sinpi(2.0 * x3)) * 0.25;
    return r;
}

// G for the direction of node (p2, p3): th = pi p2, ph = 2 pi p3
struct Dir3 {
    double e1, e2, e3;
};
__device__ __forceinline__ Dir3 dir3(double p2, double p3) {
    double st, ct, sp, cp;
    sincospi(p2, &st, &ct);
    sincospi(2.0 * p3, &sp, &cp);
    return {st * cp, st * sp, ct};
}
__device__ __forceinline__ double g3(const XP3 &x, const Dir3 &d) {
    return fma(x.x1, d.e1, fma(x.x2, d.e2, x.x3 * d.e3)) + x.c;
}
__device__ __forceinline__ double phase3_cart(const XP3 &x, double k1, double k2, double k3) {
    return fma(x.x1, k1, fma(x.x2, k2, x.x3 * k3)) + x.c * sqrt(fma(k1, k1, fma(k2, k2, k3 * k3)));
}

__device__ __forceinline__ void decode3(int idx, int n, int &b1, int &b2, int &b3) {
    b3 = idx % n;
    b2 = (idx / n) % n;
    b1 = idx / (n * n);
}

template <typename T>
__device__ __forceinline__ const T *pick_M3(const Tab3 &tb);
template <>
__device__ __forceinline__ const float *pick_M3<float>(const Tab3 &tb) { return tb.Mf; }
template <>
__device__ __forceinline__ const double *pick_M3<double>(const Tab3 &tb) { return tb.Md; }
template <typename T>
__device__ __forceinline__ const T *pick_T3(const Tab3 &tb);
template <>
__device__ __forceinline__ const float *pick_T3<float>(const Tab3 &tb) { return tb.Tf; }
template <>
__device__ __forceinline__ const double *pick_T3<double>(const Tab3 &tb) { return tb.Td; }

constexpr int C3 = 256;  // sources per chunk of the initialisation

}  // namespace

// Initialisation (eq:alg2a): pair (A at level s, B at level L-s)
//   delta_t = conj E(x0(A), p^B_t) sum_{p in B} L^B_t(p) E(x0(A), p) f(p).
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k3_init(Geom3 g, Tab3 tb, Src3 src, const cpx<T> *__restrict__ f,
                                              cpx<T> *__restrict__ w) {
    constexpr int QQQ = Q * Q * Q, TPT = (QQQ + NT - 1) / NT;
    __shared__ cpx<T> gs[C3];
    __shared__ T lg[3][C3][Q];
    const int tid = threadIdx.x;
    const int lB = g.L - g.s, nA = 1 << g.s, nB = 1 << lB, nB3 = nB * nB * nB;
    if (linear_block() >= ((size_t)nA * nA * nA) * nB3) return;  // past the pairs (uniform)
    const int pair = (int)linear_block(), iA = pair / nB3, iB = pair - iA * nB3;
    int a1, a2, a3, b1, b2, b3;
    decode3(iA, nA, a1, a2, a3);
    decode3(iB, nB, b1, b2, b3);
    const XP3 x0 = make_xp3(g, box_centre(a1, g.s), box_centre(a2, g.s), box_centre(a3, g.s));
    const int beg = src.off[iB], np = src.off[iB + 1] - beg;
    const int N = g.N, h = N / 2;
    cpx<T> acc[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) acc[k] = {(T)0, (T)0};
    for (int j0 = 0; j0 < np; j0 += C3) {
        const int nc = min(C3, np - j0);
        lds_barrier();
        if (tid < nc) {
            const int j = beg + j0 + tid, kk = src.idx[j];
            const int k1 = kk / (N * N), k2 = (kk / N) % N, k3 = kk % N;
            const cpx<T> e = cis<T>(phase3_cart(x0, (double)(k1 - h), (double)(k2 - h), (double)(k3 - h)));
            gs[tid] = cmul(e, f[kk]);
            const int bb[3] = {b1, b2, b3};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double u = (src.p[3 * j + d] - box_centre(bb[d], lB)) * nB;  // in [-1/2, 1/2]
#pragma unroll
                for (int t = 0; t < Q; ++t) {
                    double v = tb.lam[t];
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        if (i != t) v *= u - tb.z[i];
                    lg[d][tid][t] = (T)v;
                }
            }
        }
        lds_barrier();
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            const int t = tid + k * NT;
            if (t < QQQ) {
                const int t1 = t / (Q * Q), t2 = (t / Q) % Q, t3 = t % Q;
                cpx<T> a = acc[k];
                for (int jj = 0; jj < nc; ++jj) crfma(a, lg[0][jj][t1] * lg[1][jj][t2] * lg[2][jj][t3], gs[jj]);
                acc[k] = a;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int t = tid + k * NT;
        if (t < QQQ) {
            const int t1 = t / (Q * Q), t2 = (t / Q) % Q, t3 = t % Q;
            const Dir3 d = dir3(box_node(b2, lB, tb.z[t2]), box_node(b3, lB, tb.z[t3]));
            const double rho = g.rho_scale * box_node(b1, lB, tb.z[t1]);
            w[(size_t)pair * QQQ + t] = cmulc(acc[k], cis<T>(rho * g3(x0, d)));
        }
    }
}

// p-level (eq:alg2b) at level l: pair (A at l, B at L-l), inputs (A_p, B_c)
//   delta_t = conj E(x0(A), p^B_t) sum_c sum_t' prod_d M_{c_d}[t_d][t'_d] E(x0(A), p^{B_c}_t') delta^{A_p B_c}_t'.
// The child index and the node of each dimension form one index u = c q + t'
// of length 2q, contracted one dimension at a time.
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k3_plevel(Geom3 g, Tab3 tb, int level, const cpx<T> *__restrict__ win,
                                                cpx<T> *__restrict__ wout) {
    constexpr int QQQ = Q * Q * Q, Q2 = 2 * Q;
    __shared__ cpx<T> V[Q2 * Q2 * Q2];  // inputs, then the second pass's output
    __shared__ cpx<T> W1[Q2 * Q2 * Q];
    __shared__ T Ms[2][Q][Q];
    const int tid = threadIdx.x;
    const int lB = g.L - level, nA = 1 << level, nB = 1 << lB, nB3 = nB * nB * nB, nBc = 2 * nB;
    if (linear_block() >= ((size_t)nA * nA * nA) * nB3) return;  // past the pairs (uniform)
    const int pair = (int)linear_block(), iA = pair / nB3, iB = pair - iA * nB3;
    int a1, a2, a3, b1, b2, b3;
    decode3(iA, nA, a1, a2, a3);
    decode3(iB, nB, b1, b2, b3);
    const T *Mg = pick_M3<T>(tb);
    for (int i = tid; i < 2 * Q * Q; i += NT) (&Ms[0][0][0])[i] = Mg[i];
    const XP3 x0 = make_xp3(g, box_centre(a1, level), box_centre(a2, level), box_centre(a3, level));
    const int iAp = ((a1 >> 1) * (nA / 2) + (a2 >> 1)) * (nA / 2) + (a3 >> 1);
    const size_t base_in = (size_t)iAp * nBc * nBc * nBc;
    for (int i = tid; i < Q2 * Q2 * Q2; i += NT) {
        const int u1 = i / (Q2 * Q2), u2 = (i / Q2) % Q2, u3 = i % Q2;
        const int c1 = u1 / Q, c2 = u2 / Q, c3 = u3 / Q, s1 = u1 - c1 * Q, s2 = u2 - c2 * Q, s3 = u3 - c3 * Q;
        const int bc1 = 2 * b1 + c1, bc2 = 2 * b2 + c2, bc3 = 2 * b3 + c3;
        const int iBc = (bc1 * nBc + bc2) * nBc + bc3;
        const Dir3 d = dir3(box_node(bc2, lB + 1, tb.z[s2]), box_node(bc3, lB + 1, tb.z[s3]));
        const double rho = g.rho_scale * box_node(bc1, lB + 1, tb.z[s1]);
        V[i] = cmul(cis<T>(rho * g3(x0, d)), win[(base_in + iBc) * QQQ + (s1 * Q + s2) * Q + s3]);
    }
    lds_barrier();
    // dimension 3: W1[u1][u2][t3]
    for (int i = tid; i < Q2 * Q2 * Q; i += NT) {
        const int t3 = i % Q, u12 = i / Q;
        cpx<T> a = {(T)0, (T)0};
#pragma unroll
        for (int u3 = 0; u3 < Q2; ++u3) crfma(a, Ms[u3 / Q][t3][u3 % Q], V[u12 * Q2 + u3]);
        W1[i] = a;
    }
    lds_barrier();
    // dimension 2: V[u1][t2][t3] (reusing V)
    for (int i = tid; i < Q2 * Q * Q; i += NT) {
        const int t3 = i % Q, t2 = (i / Q) % Q, u1 = i / (Q * Q);
        cpx<T> a = {(T)0, (T)0};
#pragma unroll
        for (int u2 = 0; u2 < Q2; ++u2) crfma(a, Ms[u2 / Q][t2][u2 % Q], W1[(u1 * Q2 + u2) * Q + t3]);
        V[i] = a;
    }
    lds_barrier();
    // dimension 1, then the remodulation
    for (int t = tid; t < QQQ; t += NT) {
        const int t1 = t / (Q * Q), t2 = (t / Q) % Q, t3 = t % Q;
        cpx<T> a = {(T)0, (T)0};
#pragma unroll
        for (int u1 = 0; u1 < Q2; ++u1) crfma(a, Ms[u1 / Q][t1][u1 % Q], V[(u1 * Q + t2) * Q + t3]);
        const Dir3 d = dir3(box_node(b2, lB, tb.z[t2]), box_node(b3, lB, tb.z[t3]));
        const double rho = g.rho_scale * box_node(b1, lB, tb.z[t1]);
        wout[(size_t)pair * QQQ + t] = cmulc(a, cis<T>(rho * g3(x0, d)));
    }
}

// Switch (eq:alg2m) at level lm, in place: delta_t <- sum_s E(x^A_t, p^B_s) delta_s.
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k3_switch(Geom3 g, Tab3 tb, cpx<T> *__restrict__ w) {
    constexpr int QQQ = Q * Q * Q, TPT = (QQQ + NT - 1) / NT;
    __shared__ cpx<T> ds[QQQ];
    __shared__ Dir3 dirs[Q * Q];
    __shared__ double rhos[Q];
    const int tid = threadIdx.x;
    const int lA = g.lm, lB = g.L - g.lm, nA = 1 << lA, nB = 1 << lB, nB3 = nB * nB * nB;
    if (linear_block() >= ((size_t)nA * nA * nA) * nB3) return;  // past the pairs (uniform)
    const int pair = (int)linear_block(), iA = pair / nB3, iB = pair - iA * nB3;
    int a1, a2, a3, b1, b2, b3;
    decode3(iA, nA, a1, a2, a3);
    decode3(iB, nB, b1, b2, b3);
    cpx<T> *wp = w + (size_t)pair * QQQ;
    for (int i = tid; i < QQQ; i += NT) ds[i] = wp[i];
    if (tid < Q * Q) dirs[tid] = dir3(box_node(b2, lB, tb.z[tid / Q]), box_node(b3, lB, tb.z[tid % Q]));
    if (tid < Q) rhos[tid] = g.rho_scale * box_node(b1, lB, tb.z[tid]);
    lds_barrier();
    cpx<T> out[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int t = tid + k * NT;
        out[k] = {(T)0, (T)0};
        if (t < QQQ) {
            const int t1 = t / (Q * Q), t2 = (t / Q) % Q, t3 = t % Q;
            const XP3 x = make_xp3(g, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]),
                                   box_node(a3, lA, tb.z[t3]));
            cpx<T> a = {(T)0, (T)0};
            for (int s23 = 0; s23 < Q * Q; ++s23) {
                const double G = g3(x, dirs[s23]);
#pragma unroll
                for (int s1 = 0; s1 < Q; ++s1) cfma(a, cis<T>(rhos[s1] * G), ds[s1 * Q * Q + s23]);
            }
            out[k] = a;
        }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int t = tid + k * NT;
        if (t < QQQ) wp[t] = out[k];  // every read of this pair happened before the barrier above
    }
}

// x-level (eq:alg2c) at level l: pair (A at l, B at L-l), inputs (A_p, B_c)
//   delta_t = sum_c E(x^A_t, p0(B_c)) sum_t' prod_d L_{t'_d}(x^A_{t_d}) conj E(x^{A_p}_t', p0(B_c)) delta^{A_p B_c}_t'.
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k3_xlevel(Geom3 g, Tab3 tb, int level, const cpx<T> *__restrict__ win,
                                                cpx<T> *__restrict__ wout) {
    constexpr int QQQ = Q * Q * Q, TPT = (QQQ + NT - 1) / NT;
    __shared__ cpx<T> V[8][QQQ];
    __shared__ cpx<T> T1[QQQ], T2[QQQ];
    __shared__ T Ms[2][Q][Q];
    const int tid = threadIdx.x;
    const int lB = g.L - level, nA = 1 << level, nB = 1 << lB, nB3 = nB * nB * nB, nBc = 2 * nB;
    if (linear_block() >= ((size_t)nA * nA * nA) * nB3) return;  // past the pairs (uniform)
    const int pair = (int)linear_block(), iA = pair / nB3, iB = pair - iA * nB3;
    int a1, a2, a3, b1, b2, b3;
    decode3(iA, nA, a1, a2, a3);
    decode3(iB, nB, b1, b2, b3);
    const T *Mg = pick_M3<T>(tb);
    for (int i = tid; i < 2 * Q * Q; i += NT) (&Ms[0][0][0])[i] = Mg[i];
    const int ap1 = a1 >> 1, ap2 = a2 >> 1, ap3 = a3 >> 1;
    const int iAp = (ap1 * (nA / 2) + ap2) * (nA / 2) + ap3;
    const size_t base_in = (size_t)iAp * nBc * nBc * nBc;
    for (int i = tid; i < 8 * QQQ; i += NT) {
        const int c = i / QQQ, s = i - c * QQQ;
        const int c1 = c >> 2, c2 = (c >> 1) & 1, c3 = c & 1;
        const int s1 = s / (Q * Q), s2 = (s / Q) % Q, s3 = s % Q;
        const int bc1 = 2 * b1 + c1, bc2 = 2 * b2 + c2, bc3 = 2 * b3 + c3;
        const int iBc = (bc1 * nBc + bc2) * nBc + bc3;
        const XP3 xp = make_xp3(g, box_node(ap1, level - 1, tb.z[s1]), box_node(ap2, level - 1, tb.z[s2]),
                                box_node(ap3, level - 1, tb.z[s3]));
        const Dir3 d = dir3(box_centre(bc2, lB + 1), box_centre(bc3, lB + 1));
        const double rho = g.rho_scale * box_centre(bc1, lB + 1);
        V[c][s] = cmulc(win[(base_in + iBc) * QQQ + s], cis<T>(rho * g3(xp, d)));
    }
    // the target nodes of this thread
    XP3 xt[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int t = min(tid + k * NT, QQQ - 1);
        const int t1 = t / (Q * Q), t2 = (t / Q) % Q, t3 = t % Q;
        xt[k] = make_xp3(g, box_node(a1, level, tb.z[t1]), box_node(a2, level, tb.z[t2]),
                         box_node(a3, level, tb.z[t3]));
    }
    cpx<T> acc[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) acc[k] = {(T)0, (T)0};
    const int x1b = a1 & 1, x2b = a2 & 1, x3b = a3 & 1;  // child bit of A in its parent, per dimension
    for (int c = 0; c < 8; ++c) {
        lds_barrier();  // V written (first child) / T1, T2 free (later children)
        // dimension 3: T1[s1][s2][t3] = sum_s3 L_s3(x_t3) V[c][s1][s2][s3];  L_s(x_t) = M[x3b][s][t]
        for (int i = tid; i < QQQ; i += NT) {
            const int t3 = i % Q, s12 = i / Q;
            cpx<T> a = {(T)0, (T)0};
#pragma unroll
            for (int s3 = 0; s3 < Q; ++s3) crfma(a, Ms[x3b][s3][t3], V[c][s12 * Q + s3]);
            T1[i] = a;
        }
        lds_barrier();
        for (int i = tid; i < QQQ; i += NT) {
            const int t3 = i % Q, t2 = (i / Q) % Q, s1 = i / (Q * Q);
            cpx<T> a = {(T)0, (T)0};
#pragma unroll
            for (int s2 = 0; s2 < Q; ++s2) crfma(a, Ms[x2b][s2][t2], T1[(s1 * Q + s2) * Q + t3]);
            T2[i] = a;
        }
        lds_barrier();
        const int c1 = c >> 2, c2 = (c >> 1) & 1, c3 = c & 1;
        const int bc1 = 2 * b1 + c1, bc2 = 2 * b2 + c2, bc3 = 2 * b3 + c3;
        const Dir3 d = dir3(box_centre(bc2, lB + 1), box_centre(bc3, lB + 1));
        const double rho = g.rho_scale * box_centre(bc1, lB + 1);
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            const int t = tid + k * NT;
            if (t < QQQ) {
                const int t1 = t / (Q * Q), t23 = t % (Q * Q);
                cpx<T> a = {(T)0, (T)0};
#pragma unroll
                for (int s1 = 0; s1 < Q; ++s1) crfma(a, Ms[x1b][s1][t1], T2[s1 * Q * Q + t23]);
                cfma(acc[k], cis<T>(rho * g3(xt[k], d)), a);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int t = tid + k * NT;
        if (t < QQQ) wout[(size_t)pair * QQQ + t] = acc[k];
    }
}

// Termination (eq:alg2d): box A at level L-s, the m^3 points x of A (m = 2^s)
//   u(x) = sum_B E(x, p0(B)) sum_t prod_d L_{t_d}(x_d) conj E(x^A_t, p0(B)) delta^{AB}_t.
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k3_term(Geom3 g, Tab3 tb, const cpx<T> *__restrict__ win,
                                              cpx<T> *__restrict__ u) {
    constexpr int QQQ = Q * Q * Q;
    constexpr int MP = (512 + NT - 1) / NT;  // grid points per thread (m^3 <= 512)
    __shared__ cpx<T> v[QQQ];
    __shared__ cpx<T> P1[Q * Q * 8], P2[Q * 8 * 8];
    __shared__ T Tm[8][Q];
    const int tid = threadIdx.x;
    const int lA = g.L - g.s, nA = 1 << lA, m = 1 << g.s, nB = 1 << g.s, nB3 = nB * nB * nB, m3 = m * m * m;
    if (linear_block() >= (size_t)nA * nA * nA) return;  // past the boxes (uniform)
    const int iA = (int)linear_block();
    int a1, a2, a3;
    decode3(iA, nA, a1, a2, a3);
    const T *Tt = pick_T3<T>(tb);
    for (int i = tid; i < m * Q; i += NT) (&Tm[0][0])[i] = Tt[i];
    XP3 xg[MP];
    cpx<T> acc[MP];
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        const int j = min(tid + k * NT, m3 - 1);
        const int j1 = j / (m * m), j2 = (j / m) % m, j3 = j % m;
        xg[k] = make_xp3(g, (double)(a1 * m + j1) / g.N, (double)(a2 * m + j2) / g.N, (double)(a3 * m + j3) / g.N);
        acc[k] = {(T)0, (T)0};
    }
    for (int iB = 0; iB < nB3; ++iB) {
        int b1, b2, b3;
        decode3(iB, nB, b1, b2, b3);
        const Dir3 d = dir3(box_centre(b2, g.s), box_centre(b3, g.s));
        const double rho = g.rho_scale * box_centre(b1, g.s);
        lds_barrier();  // the previous box's readers are done
        const cpx<T> *src = win + ((size_t)iA * nB3 + iB) * QQQ;
        for (int t = tid; t < QQQ; t += NT) {
            const int t1 = t / (Q * Q), t2 = (t / Q) % Q, t3 = t % Q;
            const XP3 xt = make_xp3(g, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]),
                                    box_node(a3, lA, tb.z[t3]));
            v[t] = cmulc(src[t], cis<T>(rho * g3(xt, d)));
        }
        lds_barrier();
        for (int i = tid; i < Q * Q * m; i += NT) {  // P1[t1][t2][j3]
            const int j3 = i % m, t12 = i / m;
            cpx<T> a = {(T)0, (T)0};
#pragma unroll
            for (int t3 = 0; t3 < Q; ++t3) crfma(a, Tm[j3][t3], v[t12 * Q + t3]);
            P1[i] = a;
        }
        lds_barrier();
        for (int i = tid; i < Q * m * m; i += NT) {  // P2[t1][j2][j3]
            const int j3 = i % m, j2 = (i / m) % m, t1 = i / (m * m);
            cpx<T> a = {(T)0, (T)0};
#pragma unroll
            for (int t2 = 0; t2 < Q; ++t2) crfma(a, Tm[j2][t2], P1[(t1 * Q + t2) * m + j3]);
            P2[i] = a;
        }
        lds_barrier();
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            const int j = tid + k * NT;
            if (j < m3) {
                const int j1 = j / (m * m), j23 = j % (m * m);
                cpx<T> a = {(T)0, (T)0};
#pragma unroll
                for (int t1 = 0; t1 < Q; ++t1) crfma(a, Tm[j1][t1], P2[t1 * m * m + j23]);
                cfma(acc[k], cis<T>(rho * g3(xg[k], d)), a);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        const int j = tid + k * NT;
        if (j < m3) {
            const int j1 = j / (m * m), j2 = (j / m) % m, j3 = j % m;
            u[((size_t)(a1 * m + j1) * g.N + (a2 * m + j2)) * g.N + (a3 * m + j3)] = acc[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint: the conjugate transpose of every step, in reverse order.
// ---------------------------------------------------------------------------

// termination^H: box A at level L-s, for every B (level s)
//   delta_t = E(x^A_t, p0(B)) sum_x prod_d L_{t_d}(x_d) conj E(x, p0(B)) u(x).
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k3_term_adj(Geom3 g, Tab3 tb, const cpx<T> *__restrict__ u,
                                                  cpx<T> *__restrict__ wout) {
    constexpr int QQQ = Q * Q * Q;
    constexpr int MP = (512 + NT - 1) / NT;
    __shared__ cpx<T> U[512];
    __shared__ cpx<T> P2[Q * 8 * 8], P1[Q * Q * 8];
    __shared__ T Tm[8][Q];
    const int tid = threadIdx.x;
    const int lA = g.L - g.s, nA = 1 << lA, m = 1 << g.s, nB = 1 << g.s, nB3 = nB * nB * nB, m3 = m * m * m;
    if (linear_block() >= (size_t)nA * nA * nA) return;  // past the boxes (uniform)
    const int iA = (int)linear_block();
    int a1, a2, a3;
    decode3(iA, nA, a1, a2, a3);
    const T *Tt = pick_T3<T>(tb);
    for (int i = tid; i < m * Q; i += NT) (&Tm[0][0])[i] = Tt[i];
    XP3 xg[MP];
    cpx<T> uv[MP];
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        const int j = min(tid + k * NT, m3 - 1);
        const int j1 = j / (m * m), j2 = (j / m) % m, j3 = j % m;
        xg[k] = make_xp3(g, (double)(a1 * m + j1) / g.N, (double)(a2 * m + j2) / g.N, (double)(a3 * m + j3) / g.N);
        uv[k] = u[((size_t)(a1 * m + j1) * g.N + (a2 * m + j2)) * g.N + (a3 * m + j3)];
    }
    for (int iB = 0; iB < nB3; ++iB) {
        int b1, b2, b3;
        decode3(iB, nB, b1, b2, b3);
        const Dir3 d = dir3(box_centre(b2, g.s), box_centre(b3, g.s));
        const double rho = g.rho_scale * box_centre(b1, g.s);
        lds_barrier();
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            const int j = tid + k * NT;
            if (j < m3) U[j] = cmulc(uv[k], cis<T>(rho * g3(xg[k], d)));
        }
        lds_barrier();
        for (int i = tid; i < Q * m * m; i += NT) {  // P2[t1][j2][j3] = sum_j1 T[j1][t1] U[j1][j2][j3]
            const int j23 = i % (m * m), t1 = i / (m * m);
            cpx<T> a = {(T)0, (T)0};
            for (int j1 = 0; j1 < m; ++j1) crfma(a, Tm[j1][t1], U[j1 * m * m + j23]);
            P2[i] = a;
        }
        lds_barrier();
        for (int i = tid; i < Q * Q * m; i += NT) {  // P1[t1][t2][j3] = sum_j2 T[j2][t2] P2[t1][j2][j3]
            const int j3 = i % m, t2 = (i / m) % Q, t1 = i / (Q * m);
            cpx<T> a = {(T)0, (T)0};
            for (int j2 = 0; j2 < m; ++j2) crfma(a, Tm[j2][t2], P2[(t1 * m + j2) * m + j3]);
            P1[i] = a;
        }
        lds_barrier();
        cpx<T> *dst = wout + ((size_t)iA * nB3 + iB) * QQQ;
        for (int t = tid; t < QQQ; t += NT) {
            const int t1 = t / (Q * Q), t2 = (t / Q) % Q, t3 = t % Q;
            cpx<T> a = {(T)0, (T)0};
            for (int j3 = 0; j3 < m; ++j3) crfma(a, Tm[j3][t3], P1[(t1 * Q + t2) * m + j3]);
            const XP3 xt = make_xp3(g, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]),
                                    box_node(a3, lA, tb.z[t3]));
            dst[t] = cmul(a, cis<T>(rho * g3(xt, d)));
        }
    }
}

// x-level^H at level l: one workgroup per input pair (A_p at l-1, B_c at L-l+1),
// gathering its eight children A (with B the parent of B_c):
//   delta'_t' = E(x^{A_p}_t', p0(B_c)) sum_A sum_t prod_d L_{t'_d}(x^A_{t_d}) conj E(x^A_t, p0(B_c)) delta_t.
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k3_xlevel_adj(Geom3 g, Tab3 tb, int level, const cpx<T> *__restrict__ win,
                                                    cpx<T> *__restrict__ wout) {
    constexpr int QQQ = Q * Q * Q, TPT = (QQQ + NT - 1) / NT;
    __shared__ cpx<T> V[QQQ], T1[QQQ], T2[QQQ];
    __shared__ T Ms[2][Q][Q];
    const int tid = threadIdx.x;
    const int lB = g.L - level, nA = 1 << level, nB = 1 << lB, nB3 = nB * nB * nB;
    const int nAp = nA / 2, nBc = 2 * nB, nBc3 = nBc * nBc * nBc;
    if (linear_block() >= ((size_t)nAp * nAp * nAp) * nBc3) return;  // past the pairs (uniform)
    const int pin = (int)linear_block(), iAp = pin / nBc3, iBc = pin - iAp * nBc3;
    int ap1, ap2, ap3, bc1, bc2, bc3;
    decode3(iAp, nAp, ap1, ap2, ap3);
    decode3(iBc, nBc, bc1, bc2, bc3);
    const int iB = ((bc1 >> 1) * nB + (bc2 >> 1)) * nB + (bc3 >> 1);
    const T *Mg = pick_M3<T>(tb);
    for (int i = tid; i < 2 * Q * Q; i += NT) (&Ms[0][0][0])[i] = Mg[i];
    const Dir3 d = dir3(box_centre(bc2, lB + 1), box_centre(bc3, lB + 1));
    const double rho = g.rho_scale * box_centre(bc1, lB + 1);
    cpx<T> acc[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) acc[k] = {(T)0, (T)0};
    for (int a = 0; a < 8; ++a) {
        const int x1b = a >> 2, x2b = (a >> 1) & 1, x3b = a & 1;
        const int a1 = 2 * ap1 + x1b, a2 = 2 * ap2 + x2b, a3 = 2 * ap3 + x3b;
        const int iA = (a1 * nA + a2) * nA + a3;
        const cpx<T> *src = win + ((size_t)iA * nB3 + iB) * QQQ;
        lds_barrier();  // the previous child's readers are done
        for (int t = tid; t < QQQ; t += NT) {
            const int t1 = t / (Q * Q), t2 = (t / Q) % Q, t3 = t % Q;
            const XP3 xt = make_xp3(g, box_node(a1, level, tb.z[t1]), box_node(a2, level, tb.z[t2]),
                                    box_node(a3, level, tb.z[t3]));
            V[t] = cmulc(src[t], cis<T>(rho * g3(xt, d)));
        }
        lds_barrier();
        for (int i = tid; i < QQQ; i += NT) {  // T1[t1][t2][s3] = sum_t3 L_s3(x_t3) V[t1][t2][t3]
            const int s3 = i % Q, t12 = i / Q;
            cpx<T> v = {(T)0, (T)0};
#pragma unroll
            for (int t3 = 0; t3 < Q; ++t3) crfma(v, Ms[x3b][s3][t3], V[t12 * Q + t3]);
            T1[i] = v;
        }
        lds_barrier();
        for (int i = tid; i < QQQ; i += NT) {  // T2[t1][s2][s3] = sum_t2 L_s2(x_t2) T1[t1][t2][s3]
            const int s3 = i % Q, s2 = (i / Q) % Q, t1 = i / (Q * Q);
            cpx<T> v = {(T)0, (T)0};
#pragma unroll
            for (int t2 = 0; t2 < Q; ++t2) crfma(v, Ms[x2b][s2][t2], T1[(t1 * Q + t2) * Q + s3]);
            T2[i] = v;
        }
        lds_barrier();
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            const int s = tid + k * NT;
            if (s < QQQ) {
                const int s1 = s / (Q * Q), s23 = s % (Q * Q);
                cpx<T> v = acc[k];
#pragma unroll
                for (int t1 = 0; t1 < Q; ++t1) crfma(v, Ms[x1b][s1][t1], T2[t1 * Q * Q + s23]);
                acc[k] = v;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int s = tid + k * NT;
        if (s < QQQ) {
            const int s1 = s / (Q * Q), s2 = (s / Q) % Q, s3 = s % Q;
            const XP3 xp = make_xp3(g, box_node(ap1, level - 1, tb.z[s1]), box_node(ap2, level - 1, tb.z[s2]),
                                    box_node(ap3, level - 1, tb.z[s3]));
            wout[(size_t)pin * QQQ + s] = cmul(acc[k], cis<T>(rho * g3(xp, d)));
        }
    }
}

// switch^H, in place: delta_s <- sum_t conj E(x^A_t, p^B_s) delta_t.
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k3_switch_adj(Geom3 g, Tab3 tb, cpx<T> *__restrict__ w) {
    constexpr int QQQ = Q * Q * Q, TPT = (QQQ + NT - 1) / NT;
    __shared__ cpx<T> ds[QQQ];
    __shared__ XP3 xs[QQQ];
    const int tid = threadIdx.x;
    const int lA = g.lm, lB = g.L - g.lm, nA = 1 << lA, nB = 1 << lB, nB3 = nB * nB * nB;
    if (linear_block() >= ((size_t)nA * nA * nA) * nB3) return;  // past the pairs (uniform)
    const int pair = (int)linear_block(), iA = pair / nB3, iB = pair - iA * nB3;
    int a1, a2, a3, b1, b2, b3;
    decode3(iA, nA, a1, a2, a3);
    decode3(iB, nB, b1, b2, b3);
    cpx<T> *wp = w + (size_t)pair * QQQ;
    for (int t = tid; t < QQQ; t += NT) {
        ds[t] = wp[t];
        const int t1 = t / (Q * Q), t2 = (t / Q) % Q, t3 = t % Q;
        xs[t] = make_xp3(g, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]), box_node(a3, lA, tb.z[t3]));
    }
    lds_barrier();
    cpx<T> out[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int s = tid + k * NT;
        out[k] = {(T)0, (T)0};
        if (s < QQQ) {
            const int s1 = s / (Q * Q), s2 = (s / Q) % Q, s3 = s % Q;
            const Dir3 d = dir3(box_node(b2, lB, tb.z[s2]), box_node(b3, lB, tb.z[s3]));
            const double rho = g.rho_scale * box_node(b1, lB, tb.z[s1]);
            cpx<T> a = {(T)0, (T)0};
            for (int t = 0; t < QQQ; ++t) {
                const cpx<T> e = cis<T>(rho * g3(xs[t], d));
                cfma(a, cpx<T>{e.re, -e.im}, ds[t]);
            }
            out[k] = a;
        }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int s = tid + k * NT;
        if (s < QQQ) wp[s] = out[k];  // every read of this pair happened before the barrier above
    }
}

// p-level^H at level l: one workgroup per input pair (A_p at l-1, B_c at L-l+1),
// B the parent of B_c (child index c), gathering the eight children A of A_p:
//   delta'_t' = sum_A conj E(x0(A), p^{B_c}_t') sum_t prod_d M_{c_d}[t_d][t'_d] E(x0(A), p^B_t) delta_t.
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k3_plevel_adj(Geom3 g, Tab3 tb, int level, const cpx<T> *__restrict__ win,
                                                    cpx<T> *__restrict__ wout) {
    constexpr int QQQ = Q * Q * Q, TPT = (QQQ + NT - 1) / NT;
    __shared__ cpx<T> V[QQQ], T1[QQQ], T2[QQQ];
    __shared__ T Ms[2][Q][Q];
    const int tid = threadIdx.x;
    const int lB = g.L - level, nA = 1 << level, nB = 1 << lB, nB3 = nB * nB * nB;
    const int nAp = nA / 2, nBc = 2 * nB, nBc3 = nBc * nBc * nBc;
    if (linear_block() >= ((size_t)nAp * nAp * nAp) * nBc3) return;  // past the pairs (uniform)
    const int pin = (int)linear_block(), iAp = pin / nBc3, iBc = pin - iAp * nBc3;
    int ap1, ap2, ap3, bc1, bc2, bc3;
    decode3(iAp, nAp, ap1, ap2, ap3);
    decode3(iBc, nBc, bc1, bc2, bc3);
    const int b1 = bc1 >> 1, b2 = bc2 >> 1, b3 = bc3 >> 1, c1 = bc1 & 1, c2 = bc2 & 1, c3 = bc3 & 1;
    const int iB = (b1 * nB + b2) * nB + b3;
    const T *Mg = pick_M3<T>(tb);
    for (int i = tid; i < 2 * Q * Q; i += NT) (&Ms[0][0][0])[i] = Mg[i];
    cpx<T> acc[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) acc[k] = {(T)0, (T)0};
    for (int a = 0; a < 8; ++a) {
        const int a1 = 2 * ap1 + (a >> 2), a2 = 2 * ap2 + ((a >> 1) & 1), a3 = 2 * ap3 + (a & 1);
        const int iA = (a1 * nA + a2) * nA + a3;
        const XP3 x0 = make_xp3(g, box_centre(a1, level), box_centre(a2, level), box_centre(a3, level));
        const cpx<T> *src = win + ((size_t)iA * nB3 + iB) * QQQ;
        lds_barrier();
        for (int t = tid; t < QQQ; t += NT) {
            const int t1 = t / (Q * Q), t2 = (t / Q) % Q, t3 = t % Q;
            const Dir3 d = dir3(box_node(b2, lB, tb.z[t2]), box_node(b3, lB, tb.z[t3]));
            V[t] = cmul(src[t], cis<T>(g.rho_scale * box_node(b1, lB, tb.z[t1]) * g3(x0, d)));
        }
        lds_barrier();
        for (int i = tid; i < QQQ; i += NT) {  // T1[t1][t2][s3] = sum_t3 M_c3[t3][s3] V[t1][t2][t3]
            const int s3 = i % Q, t12 = i / Q;
            cpx<T> v = {(T)0, (T)0};
#pragma unroll
            for (int t3 = 0; t3 < Q; ++t3) crfma(v, Ms[c3][t3][s3], V[t12 * Q + t3]);
            T1[i] = v;
        }
        lds_barrier();
        for (int i = tid; i < QQQ; i += NT) {  // T2[t1][s2][s3] = sum_t2 M_c2[t2][s2] T1[t1][t2][s3]
            const int s3 = i % Q, s2 = (i / Q) % Q, t1 = i / (Q * Q);
            cpx<T> v = {(T)0, (T)0};
#pragma unroll
            for (int t2 = 0; t2 < Q; ++t2) crfma(v, Ms[c2][t2][s2], T1[(t1 * Q + t2) * Q + s3]);
            T2[i] = v;
        }
        lds_barrier();
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            const int s = tid + k * NT;
            if (s < QQQ) {
                const int s1 = s / (Q * Q), s2 = (s / Q) % Q, s3 = s % Q, s23 = s % (Q * Q);
                cpx<T> v = {(T)0, (T)0};
#pragma unroll
                for (int t1 = 0; t1 < Q; ++t1) crfma(v, Ms[c1][t1][s1], T2[t1 * Q * Q + s23]);
                const Dir3 d = dir3(box_node(bc2, lB + 1, tb.z[s2]), box_node(bc3, lB + 1, tb.z[s3]));
                const double rho = g.rho_scale * box_node(bc1, lB + 1, tb.z[s1]);
                cfma(acc[k], cmulc(v, cis<T>(rho * g3(x0, d))), cpx<T>{(T)1, (T)0});
            }
        }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int s = tid + k * NT;
        if (s < QQQ) wout[(size_t)pin * QQQ + s] = acc[k];
    }
}

// initialisation^H: one workgroup per box B (level L-s), its sources in chunks
//   f(k) = sum_A conj E(x0(A), k) sum_t L^B_t(p_k) E(x0(A), p^B_t) delta^{AB}_t.
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k3_init_adj(Geom3 g, Tab3 tb, Src3 src, const cpx<T> *__restrict__ w,
                                                  cpx<T> *__restrict__ f) {
    constexpr int QQQ = Q * Q * Q;
    __shared__ cpx<T> y[QQQ];
    __shared__ T lg[3][C3][Q];
    const int tid = threadIdx.x;
    const int lB = g.L - g.s, nA = 1 << g.s, nA3 = nA * nA * nA, nB = 1 << lB, nB3 = nB * nB * nB;
    if (linear_block() >= (size_t)nB3) return;  // past the boxes (uniform)
    const int iB = (int)linear_block();
    int b1, b2, b3;
    decode3(iB, nB, b1, b2, b3);
    const int beg = src.off[iB], np = src.off[iB + 1] - beg;
    const int N = g.N, h = N / 2;
    for (int j0 = 0; j0 < np; j0 += C3) {
        const int nc = min(C3, np - j0);
        int kk = 0;
        double k1 = 0, k2 = 0, k3 = 0;
        lds_barrier();
        if (tid < nc) {
            const int j = beg + j0 + tid;
            kk = src.idx[j];
            k1 = (double)(kk / (N * N) - h);
            k2 = (double)((kk / N) % N - h);
            k3 = (double)(kk % N - h);
            const int bb[3] = {b1, b2, b3};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double u = (src.p[3 * j + d] - box_centre(bb[d], lB)) * nB;
#pragma unroll
                for (int t = 0; t < Q; ++t) {
                    double v = tb.lam[t];
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        if (i != t) v *= u - tb.z[i];
                    lg[d][tid][t] = (T)v;
                }
            }
        }
        cpx<T> acc = {(T)0, (T)0};
        for (int iA = 0; iA < nA3; ++iA) {
            int a1, a2, a3;
            decode3(iA, nA, a1, a2, a3);
            const XP3 x0 = make_xp3(g, box_centre(a1, g.s), box_centre(a2, g.s), box_centre(a3, g.s));
            lds_barrier();  // lg written (first A) / the previous A's readers of y are done
            const cpx<T> *sw = w + ((size_t)iA * nB3 + iB) * QQQ;
            for (int t = tid; t < QQQ; t += NT) {
                const int t1 = t / (Q * Q), t2 = (t / Q) % Q, t3 = t % Q;
                const Dir3 d = dir3(box_node(b2, lB, tb.z[t2]), box_node(b3, lB, tb.z[t3]));
                y[t] = cmul(sw[t], cis<T>(g.rho_scale * box_node(b1, lB, tb.z[t1]) * g3(x0, d)));
            }
            lds_barrier();
            if (tid < nc) {
                cpx<T> v = {(T)0, (T)0};
                for (int t1 = 0; t1 < Q; ++t1)
                    for (int t2 = 0; t2 < Q; ++t2) {
                        const T l12 = lg[0][tid][t1] * lg[1][tid][t2];
#pragma unroll
                        for (int t3 = 0; t3 < Q; ++t3) crfma(v, l12 * lg[2][tid][t3], y[(t1 * Q + t2) * Q + t3]);
                    }
                cfma(acc, cmulc(v, cis<T>(phase3_cart(x0, k1, k2, k3))), cpx<T>{(T)1, (T)0});
            }
        }
        if (tid < nc) f[kk] = acc;
    }
}

template <typename T>
static hipError_t step3_adj_t(int step, const Geom3 &g, const Tab3 &tb, const Src3 &src, int level, const void *in,
                              void *out, hipStream_t st) {
    const size_t pairs = (size_t)1 << (3 * g.L);
#define L3A(Q)                                                                                                    \
    switch (step) {                                                                                               \
        case 0:                                                                                                   \
            hipLaunchKernelGGL((k3_init_adj<T, Q>), grid_of((size_t)1 << (3 * (g.L - g.s))), dim3(NT), 0, st, g, \
                               tb, src, (const cpx<T> *)in, (cpx<T> *)out);                                      \
            break;                                                                                                \
        case 1:                                                                                                   \
            hipLaunchKernelGGL((k3_plevel_adj<T, Q>), grid_of(pairs), dim3(NT), 0, st, g, tb, level,             \
                               (const cpx<T> *)in, (cpx<T> *)out);                                                \
            break;                                                                                                \
        case 2:                                                                                                   \
            hipLaunchKernelGGL((k3_switch_adj<T, Q>), grid_of(pairs), dim3(NT), 0, st, g, tb, (cpx<T> *)out);    \
            break;                                                                                                \
        case 3:                                                                                                   \
            hipLaunchKernelGGL((k3_xlevel_adj<T, Q>), grid_of(pairs), dim3(NT), 0, st, g, tb, level,             \
                               (const cpx<T> *)in, (cpx<T> *)out);                                                \
            break;                                                                                                \
        default:                                                                                                  \
            hipLaunchKernelGGL((k3_term_adj<T, Q>), grid_of((size_t)1 << (3 * (g.L - g.s))), dim3(NT), 0, st,    \
                               g, tb, (const cpx<T> *)in, (cpx<T> *)out);                                         \
    }
    switch (g.q) {
        case 3: L3A(3) break;
        case 4: L3A(4) break;
        case 5: L3A(5) break;
        case 6: L3A(6) break;
        case 7: L3A(7) break;
        case 8: L3A(8) break;
        default: return hipErrorInvalidValue;
    }
#undef L3A
    return hipGetLastError();
}

hipError_t launch_step3_adj(int dtype, int step, const Geom3 &g, const Tab3 &tb, const Src3 &src, int level,
                            const void *in, void *out, hipStream_t st) {
    return dtype == FIO_C128 ? step3_adj_t<double>(step, g, tb, src, level, in, out, st)
                             : step3_adj_t<float>(step, g, tb, src, level, in, out, st);
}

template <typename T>
static hipError_t step3_t(int step, const Geom3 &g, const Tab3 &tb, const Src3 &src, int level, const void *in,
                          void *out, hipStream_t st) {
    const size_t pairs = (size_t)1 << (3 * g.L);
#define L3(Q)                                                                                                     \
    switch (step) {                                                                                               \
        case 0:                                                                                                   \
            hipLaunchKernelGGL((k3_init<T, Q>), grid_of(pairs), dim3(NT), 0, st, g, tb, src, (const cpx<T> *)in,    \
                               (cpx<T> *)out);                                                                    \
            break;                                                                                                \
        case 1:                                                                                                   \
            hipLaunchKernelGGL((k3_plevel<T, Q>), grid_of(pairs), dim3(NT), 0, st, g, tb, level,                    \
                               (const cpx<T> *)in, (cpx<T> *)out);                                                \
            break;                                                                                                \
        case 2:                                                                                                   \
            hipLaunchKernelGGL((k3_switch<T, Q>), grid_of(pairs), dim3(NT), 0, st, g, tb, (cpx<T> *)out);           \
            break;                                                                                                \
        case 3:                                                                                                   \
            hipLaunchKernelGGL((k3_xlevel<T, Q>), grid_of(pairs), dim3(NT), 0, st, g, tb, level,                    \
                               (const cpx<T> *)in, (cpx<T> *)out);                                                \
            break;                                                                                                \
        default:                                                                                                  \
            hipLaunchKernelGGL((k3_term<T, Q>), grid_of((size_t)1 << (3 * (g.L - g.s))), dim3(NT), 0, st, g, tb,           \
                               (const cpx<T> *)in, (cpx<T> *)out);                                                \
    }
    switch (g.q) {
        case 3: L3(3) break;
        case 4: L3(4) break;
        case 5: L3(5) break;
        case 6: L3(6) break;
        case 7: L3(7) break;
        case 8: L3(8) break;
        default: return hipErrorInvalidValue;
    }
#undef L3
    return hipGetLastError();
}

hipError_t launch_step3(int dtype, int step, const Geom3 &g, const Tab3 &tb, const Src3 &src, int level,
                        const void *in, void *out, hipStream_t st) {
    return dtype == FIO_C128 ? step3_t<double>(step, g, tb, src, level, in, out, st)
                             : step3_t<float>(step, g, tb, src, level, in, out, st);
}

}  // namespace fio
