// HIP kernels (gfx950) of the butterfly FIO pass: the forward steps of
// Sec. 4 (eq:alg2a, eq:alg2b, eq:alg2m, eq:alg2c, eq:alg2d) and their exact
// conjugate transposes.
//
// Weight layout at level l (one right-hand side):
//   w[(mA * 4^(L-l) + mB) * q^2 + t1*q + t2]
// mA: Morton index of A at level l of T_X; mB: Morton index of B at level
// L-l of T_P.  The four children of B are 4 mB + (2 c1 + c2), so the inputs
// of a butterfly block (A_p, B) -- the pairs (A_p, B_c) -- are contiguous.
//
// Every kernel launch covers all N^2 pairs of one level; each output pair
// is written by exactly one workgroup (no atomics).  Phases are recomputed
// on the fly in FP64 and never stored.
#include <hip/hip_runtime.h>

#include "fio_device.h"

namespace fio {

constexpr int NT = 256;  // threads per workgroup for every kernel here

// ---------------------------------------------------------------------------
// Shared helpers
// ---------------------------------------------------------------------------

// Lagrange basis values L_t(u), t < Q, on the Chebyshev grid z (barycentric
// form of the second kind, with lam the barycentric weights).
template <typename T, int Q>
__device__ __forceinline__ void lagrange_row(double u, const double *z, const double *lam, T *out) {
    int exact = -1;
    double ssum = 0.0;
    double tmp[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t) {
        const double d = u - z[t];
        if (d == 0.0) exact = t;
        tmp[t] = lam[t] / d;
        ssum += tmp[t];
    }
    if (exact >= 0) {
#pragma unroll
        for (int t = 0; t < Q; ++t) out[t] = (T)(t == exact ? 1.0 : 0.0);
    } else {
        const double inv = 1.0 / ssum;
#pragma unroll
        for (int t = 0; t < Q; ++t) out[t] = (T)(tmp[t] * inv);
    }
}

template <typename T>
__device__ __forceinline__ const T *pick_M(const Tables &tb);
template <>
__device__ __forceinline__ const float *pick_M<float>(const Tables &tb) { return tb.Mf; }
template <>
__device__ __forceinline__ const double *pick_M<double>(const Tables &tb) { return tb.M; }

template <typename T>
__device__ __forceinline__ const T *pick_T(const Tables &tb);
template <>
__device__ __forceinline__ const float *pick_T<float>(const Tables &tb) { return tb.Ttf; }
template <>
__device__ __forceinline__ const double *pick_T<double>(const Tables &tb) { return tb.Tt; }

// ===========================================================================
// Step 2, initialisation (eq:alg2a): pairs (A at level s, B at level L-s)
//   delta^{AB}_t = conj E(x0(A), p^B_t) * sum_{p in B} L^B_t(p) E(x0(A), p) f(p)
// One workgroup per (B, chunk of A boxes); thread <-> (A, t1) accumulates
// the q values t2 of its row.  Sources of B are staged through LDS in
// chunks of SCH; their kernel values E(x0(A),p) f(p) are formed once per
// (A, p) in LDS and shared by the q threads of A.
// ===========================================================================
constexpr int SCH = 64;

template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_init(Geom g, PhaseDev ph, Tables tb, Sources src,
                                             const cpx<T> *__restrict__ f, cpx<T> *__restrict__ w) {
    constexpr int ACH = (NT / Q) < 64 ? (NT / Q) : 64;  // A boxes per workgroup (4^s <= 64)
    __shared__ T lag1[SCH][Q];
    __shared__ T lag2[SCH][Q];
    __shared__ cpx<T> gA[ACH][SCH];
    __shared__ double2 kk[SCH];
    __shared__ cpx<T> fs[SCH];
    __shared__ double zs[Q], ls[Q];
    __shared__ XP xA[ACH];

    const int tid = threadIdx.x;
    const int lB = g.L - g.s;
    const uint32_t mB = blockIdx.x;
    const int nA = 1 << (2 * g.s);
    const int a0 = blockIdx.y * ACH;
    const int nAc = min(ACH, nA - a0);
    const int aL = tid / Q, t1 = tid - aL * Q;
    const bool active = aL < nAc;

    if (tid < Q) {
        zs[tid] = tb.z[tid];
        ls[tid] = tb.lam[tid];
    }
    if (tid < nAc) {
        int a1, a2;
        morton_decode((uint32_t)(a0 + tid), a1, a2);
        xA[tid] = make_xp(ph, box_centre(a1, g.s), box_centre(a2, g.s));
    }
    int bp1, bp2;
    morton_decode(mB, bp1, bp2);
    const double scale = ldexp(1.0, lB);

    cpx<T> acc[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t) acc[t] = {(T)0, (T)0};

    const int beg = src.off[mB], end = src.off[mB + 1];
    __syncthreads();
    for (int c0 = beg; c0 < end; c0 += SCH) {
        const int n = min(SCH, end - c0);
        if (tid < n) {
            const int j = c0 + tid;
            const int idx = src.idx[j];
            const double2 p = src.p[j];
            const double u1 = p.x * scale - ((double)bp1 + 0.5);
            const double u2 = p.y * scale - ((double)bp2 + 0.5);
            lagrange_row<T, Q>(u1, zs, ls, lag1[tid]);
            lagrange_row<T, Q>(u2, zs, ls, lag2[tid]);
            kk[tid] = make_double2((double)(idx / g.N - g.N / 2), (double)(idx % g.N - g.N / 2));
            fs[tid] = f[idx];
        }
        __syncthreads();
        // kernel values E(x0(A), k) f(k) for this chunk, all A of the workgroup
        for (int it = tid; it < nAc * n; it += NT) {
            const int al = it / n, jj = it - al * n;
            const cpx<T> e = cis<T>(phase_cart(xA[al], kk[jj].x, kk[jj].y));
            gA[al][jj] = cmul(e, fs[jj]);
        }
        __syncthreads();
        if (active) {
            for (int jj = 0; jj < n; ++jj) {
                const cpx<T> gv = gA[aL][jj];
                const T l1 = lag1[jj][t1];
                const cpx<T> h = {l1 * gv.re, l1 * gv.im};
#pragma unroll
                for (int t2 = 0; t2 < Q; ++t2) crfma(acc[t2], lag2[jj][t2], h);
            }
        }
        __syncthreads();
    }
    if (!active) return;
    // remodulation conj E(x0(A), p^B_t) and store
    const uint32_t mA = a0 + aL;
    const XP xp = xA[aL];
    const double rho = g.rho_scale * box_node(bp1, lB, zs[t1]);
    cpx<T> *out = w + ((size_t)mA * ((size_t)1 << (2 * lB)) + mB) * (Q * Q) + t1 * Q;
#pragma unroll
    for (int t2 = 0; t2 < Q; ++t2) {
        double st, ct;
        sincospi(2.0 * box_node(bp2, lB, zs[t2]), &st, &ct);
        const cpx<T> e = cis<T>(rho * phase_dir(xp, ct, st));
        out[t2] = cmulc(acc[t2], e);
    }
}

// ===========================================================================
// Step 3, p-recursion (eq:alg2b) at level l: block (A_p at l-1, B at L-l)
//   delta^{AB}_t = conj E(x0(A), p^B_t) sum_c sum_t' M_c1[t1][t'1] M_c2[t2][t'2]
//                     E(x0(A), p^{B_c}_t') delta^{A_p B_c}_t'
// for the four children A of A_p.  The q x q Kronecker sum over the four
// children B_c is done one dimension at a time (Sec. 4: 6 q^3 per pair).
// One workgroup per block; the four outputs are produced one after another
// by all threads.
// ===========================================================================
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_plevel(Geom g, PhaseDev ph, Tables tb, int level,
                                               const cpx<T> *__restrict__ win,
                                               cpx<T> *__restrict__ wout) {
    constexpr int QQ = Q * Q;
    __shared__ cpx<T> din[4 * QQ];
    __shared__ cpx<T> v[4 * QQ];
    __shared__ cpx<T> W[2 * QQ];
    __shared__ T Ms[2 * QQ];
    __shared__ double rc[2 * Q], ctc[2 * Q], stc[2 * Q];  // child nodes: rho(c1,t'1), theta(c2,t'2)
    __shared__ double rb[Q], ctb[Q], stb[Q];              // B's own nodes
    __shared__ double Gc[2 * Q], Gb[Q];

    const int tid = threadIdx.x;
    const int lB = g.L - level;
    const size_t blk = blockIdx.x;
    const uint32_t mB = (uint32_t)(blk & (((size_t)1 << (2 * lB)) - 1));
    const uint32_t mAp = (uint32_t)(blk >> (2 * lB));
    int b1, b2, ap1, ap2;
    morton_decode(mB, b1, b2);
    morton_decode(mAp, ap1, ap2);

    const cpx<T> *src = win + blk * (4 * QQ);
    for (int i = tid; i < 4 * QQ; i += NT) din[i] = src[i];
    const T *Mg = pick_M<T>(tb);
    for (int i = tid; i < 2 * QQ; i += NT) Ms[i] = Mg[i];
    if (tid < 2 * Q) {
        const int c = tid / Q, t = tid - c * Q;
        const double z = tb.z[t];
        rc[tid] = g.rho_scale * box_node(2 * b1 + c, lB + 1, z);
        double s_, c_;
        sincospi(2.0 * box_node(2 * b2 + c, lB + 1, z), &s_, &c_);
        ctc[tid] = c_;
        stc[tid] = s_;
    } else if (tid >= 64 && tid < 64 + Q) {
        const int t = tid - 64;
        const double z = tb.z[t];
        rb[t] = g.rho_scale * box_node(b1, lB, z);
        double s_, c_;
        sincospi(2.0 * box_node(b2, lB, z), &s_, &c_);
        ctb[t] = c_;
        stb[t] = s_;
    }
    __syncthreads();

    const size_t nBl = (size_t)1 << (2 * lB);
    for (int j = 0; j < 4; ++j) {
        const uint32_t mA = 4 * mAp + j;
        const int a1 = 2 * ap1 + (j >> 1), a2 = 2 * ap2 + (j & 1);
        const XP xp = make_xp(ph, box_centre(a1, level), box_centre(a2, level));
        if (tid < 2 * Q) Gc[tid] = phase_dir(xp, ctc[tid], stc[tid]);
        else if (tid >= 64 && tid < 64 + Q) Gb[tid - 64] = phase_dir(xp, ctb[tid - 64], stb[tid - 64]);
        __syncthreads();
        // prefactor E(x0(A), p^{B_c}_t') delta^{A_p B_c}_t'
        for (int i = tid; i < 4 * QQ; i += NT) {
            const int c = i / QQ, t = i - c * QQ;
            const int c1 = c >> 1, c2 = c & 1;
            const int tp1 = t / Q, tp2 = t - tp1 * Q;
            const cpx<T> e = cis<T>(rc[c1 * Q + tp1] * Gc[c2 * Q + tp2]);
            v[i] = cmul(e, din[i]);
        }
        __syncthreads();
        // pass 1 (second dimension): W[c1][t'1][t2] = sum_c2 sum_t'2 M_c2[t2][t'2] v[c1 c2][t'1][t'2]
        for (int i = tid; i < 2 * QQ; i += NT) {
            const int c1 = i / QQ, r = i - c1 * QQ;
            const int tp1 = r / Q, t2 = r - tp1 * Q;
            cpx<T> acc = {(T)0, (T)0};
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2) {
                const cpx<T> *vv = v + (2 * c1 + c2) * QQ + tp1 * Q;
                const T *m = Ms + c2 * QQ + t2 * Q;
#pragma unroll
                for (int tp2 = 0; tp2 < Q; ++tp2) crfma(acc, m[tp2], vv[tp2]);
            }
            W[i] = acc;
        }
        __syncthreads();
        // pass 2 (first dimension) + remodulation conj E(x0(A), p^B_t)
        cpx<T> *dst = wout + ((size_t)mA * nBl + mB) * QQ;
        for (int i = tid; i < QQ; i += NT) {
            const int t1 = i / Q, t2 = i - t1 * Q;
            cpx<T> acc = {(T)0, (T)0};
#pragma unroll
            for (int c1 = 0; c1 < 2; ++c1) {
                const T *m = Ms + c1 * QQ + t1 * Q;
#pragma unroll
                for (int tp1 = 0; tp1 < Q; ++tp1) crfma(acc, m[tp1], W[c1 * QQ + tp1 * Q + t2]);
            }
            const cpx<T> e = cis<T>(rb[t1] * Gb[t2]);
            dst[i] = cmulc(acc, e);
        }
        __syncthreads();
    }
}

// ===========================================================================
// Step 4, switch (eq:alg2m) at level lm, in place:
//   delta^{AB}_t <- sum_s E(x^A_t, p^B_s) delta^{AB}_s
// Thread <-> (pair, t).  With rho(s1) = rho0 + h_s1 and the Chebyshev nodes
// symmetric (z_{q-1-j} = -z_j), the q values of s1 share one exponential
// exp(2 pi i rho0 G) and the pairs (j, q-1-j) share exp(2 pi i h_j G) and its
// conjugate, so per (t, s2) only 1 + floor(q/2) exponentials are needed;
// the pair sums/differences of delta are formed once per pair.
// ===========================================================================
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_switch(Geom g, PhaseDev ph, Tables tb, cpx<T> *__restrict__ w) {
    constexpr int QQ = Q * Q;
    constexpr int H = Q / 2;
    constexpr int PPB = NT / QQ;  // pairs per workgroup
    __shared__ cpx<T> Sx[PPB][Q][H > 0 ? H : 1];
    __shared__ cpx<T> Dx[PPB][Q][H > 0 ? H : 1];
    __shared__ cpx<T> Mid[PPB][Q];
    __shared__ double cth[PPB][Q], sth[PPB][Q];
    __shared__ double rho0[PPB], hz[PPB][H > 0 ? H : 1];

    const int tid = threadIdx.x;
    const int pl = tid / QQ, t = tid - pl * QQ;
    const size_t npairs = (size_t)1 << (2 * g.L);
    const size_t pair = (size_t)blockIdx.x * PPB + pl;
    const bool active = (pl < PPB) && (pair < npairs);
    const int lA = g.lm, lB = g.L - g.lm;
    const size_t nBl = (size_t)1 << (2 * lB);
    const uint32_t mB = active ? (uint32_t)(pair & (nBl - 1)) : 0;
    const uint32_t mA = active ? (uint32_t)(pair >> (2 * lB)) : 0;
    int b1, b2, a1, a2;
    morton_decode(mB, b1, b2);
    morton_decode(mA, a1, a2);
    cpx<T> *wp = w + pair * QQ;

    if (active) {
        const int t1 = t / Q, t2 = t - t1 * Q;
        // t1 plays the role of the symmetric index j, t2 of s2 in the tables
        if (t1 < H) {
            const cpx<T> a = wp[t1 * Q + t2], b = wp[(Q - 1 - t1) * Q + t2];
            Sx[pl][t2][t1] = {a.re + b.re, a.im + b.im};
            Dx[pl][t2][t1] = {a.re - b.re, a.im - b.im};
        } else if ((Q & 1) && t1 == H) {
            Mid[pl][t2] = wp[H * Q + t2];
        }
        if (t < Q) {
            double s_, c_;
            sincospi(2.0 * box_node(b2, lB, tb.z[t]), &s_, &c_);
            cth[pl][t] = c_;
            sth[pl][t] = s_;
        } else if (t == Q) {
            rho0[pl] = g.rho_scale * box_centre(b1, lB);
        } else if (t > Q && t <= Q + H) {
            hz[pl][t - Q - 1] = g.rho_scale * ldexp(tb.z[t - Q - 1], -lB);
        }
    }
    __syncthreads();
    if (!active) return;

    const int t1 = t / Q, t2 = t - t1 * Q;
    const XP xp = make_xp(ph, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]));
    const double r0 = rho0[pl];
    cpx<T> acc = {(T)0, (T)0};
    for (int s2 = 0; s2 < Q; ++s2) {
        const double G = phase_dir(xp, cth[pl][s2], sth[pl][s2]);
        cpx<T> inner = (Q & 1) ? Mid[pl][s2] : cpx<T>{(T)0, (T)0};
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const cpx<T> d = cis<T>(hz[pl][j] * G);
            const cpx<T> S = Sx[pl][s2][j], D = Dx[pl][s2][j];
            inner.re = fma(d.re, S.re, fma(-d.im, D.im, inner.re));
            inner.im = fma(d.re, S.im, fma(d.im, D.re, inner.im));
        }
        cfma(acc, cis<T>(r0 * G), inner);
    }
    wp[t] = acc;
}

// ===========================================================================
// Step 5, x-recursion (eq:alg2c) at level l: block (A_p at l-1, B at L-l)
//   delta^{AB}_t = sum_c E(x^A_t, p0(B_c)) sum_t' M_a1[t'1][t1] M_a2[t'2][t2]
//                    conj E(x^{A_p}_t', p0(B_c)) delta^{A_p B_c}_t'
// for the four children A = (a1, a2) of A_p.  The prefactor depends only on
// (A_p, B_c) and is applied once per block.
// ===========================================================================
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_xlevel(Geom g, PhaseDev ph, Tables tb, int level,
                                               const cpx<T> *__restrict__ win,
                                               cpx<T> *__restrict__ wout) {
    constexpr int QQ = Q * Q;
    __shared__ cpx<T> v[4 * QQ];
    __shared__ cpx<T> Y[4 * QQ];
    __shared__ T Ms[2 * QQ];
    __shared__ double sx1[Q], cx1[Q], sx2[Q], cx2[Q];   // sin/cos(2 pi x) at the nodes of the current box
    __shared__ double r0c[2], ct0[2], st0[2];           // p0(B_c): rho(c1), theta(c2)

    const int tid = threadIdx.x;
    const int lB = g.L - level;
    const size_t blk = blockIdx.x;
    const uint32_t mB = (uint32_t)(blk & (((size_t)1 << (2 * lB)) - 1));
    const uint32_t mAp = (uint32_t)(blk >> (2 * lB));
    int b1, b2, ap1, ap2;
    morton_decode(mB, b1, b2);
    morton_decode(mAp, ap1, ap2);
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;

    const T *Mg = pick_M<T>(tb);
    for (int i = tid; i < 2 * QQ; i += NT) Ms[i] = Mg[i];
    if (tid < 2) {
        r0c[tid] = g.rho_scale * box_centre(2 * b1 + tid, lB + 1);
        double s_, c_;
        sincospi(2.0 * box_centre(2 * b2 + tid, lB + 1), &s_, &c_);
        ct0[tid] = c_;
        st0[tid] = s_;
    } else if (tid >= 64 && tid < 64 + Q) {
        const int t = tid - 64;
        double s_ = 0, c_ = 1;
        if (ell) sincospi(2.0 * box_node(ap1, level - 1, tb.z[t]), &s_, &c_);
        sx1[t] = s_;
        cx1[t] = c_;
    } else if (tid >= 128 && tid < 128 + Q) {
        const int t = tid - 128;
        double s_ = 0, c_ = 1;
        if (ell) sincospi(2.0 * box_node(ap2, level - 1, tb.z[t]), &s_, &c_);
        sx2[t] = s_;
        cx2[t] = c_;
    }
    __syncthreads();
    // prefactor conj E(x^{A_p}_t', p0(B_c)) delta^{A_p B_c}_t'; thread <-> (c2, t')
    const cpx<T> *src = win + blk * (4 * QQ);
    for (int i = tid; i < 2 * QQ; i += NT) {
        const int c2 = i / QQ, tp = i - c2 * QQ;
        const int tp1 = tp / Q, tp2 = tp - tp1 * Q;
        const XP xp = make_xp_sc(ph, box_node(ap1, level - 1, tb.z[tp1]), box_node(ap2, level - 1, tb.z[tp2]),
                                 sx1[tp1], cx1[tp1], sx2[tp2], cx2[tp2]);
        const double G = phase_dir(xp, ct0[c2], st0[c2]);
#pragma unroll
        for (int c1 = 0; c1 < 2; ++c1) {
            const int c = 2 * c1 + c2;
            v[c * QQ + tp] = cmulc(src[c * QQ + tp], cis<T>(r0c[c1] * G));
        }
    }
    __syncthreads();

    const size_t nBl = (size_t)1 << (2 * lB);
    for (int j = 0; j < 4; ++j) {
        const int j1 = j >> 1, j2 = j & 1;
        const uint32_t mA = 4 * mAp + j;
        const int a1 = 2 * ap1 + j1, a2 = 2 * ap2 + j2;
        // sin/cos tables for the nodes of A (reuse the A_p slots after a barrier)
        if (tid < Q) {
            double s_ = 0, c_ = 1;
            if (ell) sincospi(2.0 * box_node(a1, level, tb.z[tid]), &s_, &c_);
            sx1[tid] = s_;
            cx1[tid] = c_;
        } else if (tid >= 64 && tid < 64 + Q) {
            const int t = tid - 64;
            double s_ = 0, c_ = 1;
            if (ell) sincospi(2.0 * box_node(a2, level, tb.z[t]), &s_, &c_);
            sx2[t] = s_;
            cx2[t] = c_;
        }
        // pass 1 (second dimension): Y[c][t'1][t2] = sum_t'2 M_j2[t'2][t2] v[c][t'1][t'2]
        for (int i = tid; i < 4 * QQ; i += NT) {
            const int c = i / QQ, r = i - c * QQ;
            const int tp1 = r / Q, t2 = r - tp1 * Q;
            const cpx<T> *vv = v + c * QQ + tp1 * Q;
            const T *m = Ms + j2 * QQ + t2;
            cpx<T> acc = {(T)0, (T)0};
#pragma unroll
            for (int tp2 = 0; tp2 < Q; ++tp2) crfma(acc, m[tp2 * Q], vv[tp2]);
            Y[i] = acc;
        }
        __syncthreads();
        // pass 2 (first dimension), remodulation E(x^A_t, p0(B_c)), sum over c
        cpx<T> *dst = wout + ((size_t)mA * nBl + mB) * QQ;
        for (int i = tid; i < QQ; i += NT) {
            const int t1 = i / Q, t2 = i - t1 * Q;
            const XP xp = make_xp_sc(ph, box_node(a1, level, tb.z[t1]), box_node(a2, level, tb.z[t2]),
                                     sx1[t1], cx1[t1], sx2[t2], cx2[t2]);
            const double G0 = phase_dir(xp, ct0[0], st0[0]);
            const double G1 = phase_dir(xp, ct0[1], st0[1]);
            cpx<T> out = {(T)0, (T)0};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int c1 = c >> 1, c2 = c & 1;
                const T *m = Ms + j1 * QQ + t1;
                cpx<T> acc = {(T)0, (T)0};
#pragma unroll
                for (int tp1 = 0; tp1 < Q; ++tp1) crfma(acc, m[tp1 * Q], Y[c * QQ + tp1 * Q + t2]);
                cfma(out, cis<T>(r0c[c1] * (c2 ? G1 : G0)), acc);
            }
            dst[i] = out;
        }
        __syncthreads();
    }
}

// ===========================================================================
// Step 6, termination (eq:alg2d): pairs (A at level L-s, B at level s)
//   u(x) = sum_B E(x, p0(B)) sum_t L^A_t(x) conj E(x^A_t, p0(B)) delta^{AB}_t
// for the 2^s x 2^s grid points x of A.  One workgroup per A; the 4^s
// boxes B are processed in chunks of BCH.  Thread tid always owns grid
// point tid % 4^s, so per-point partial sums stay in registers and are
// combined once at the end.
// ===========================================================================
// B boxes per chunk: keeps the chunk's weights and partial sums within 32 KB of LDS.
template <typename T, int Q>
constexpr int bch() {
    return (32768 / (Q * Q * 2 * (int)sizeof(T))) < 16 ? (32768 / (Q * Q * 2 * (int)sizeof(T))) : 16;
}

template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_term(Geom g, PhaseDev ph, Tables tb,
                                             const cpx<T> *__restrict__ win, cpx<T> *__restrict__ u) {
    constexpr int QQ = Q * Q;
    constexpr int BCH = bch<T, Q>();
    __shared__ cpx<T> v[BCH * QQ];
    __shared__ cpx<T> Y[BCH * Q * 8];
    __shared__ cpx<T> red[NT];
    __shared__ double sx1[Q], cx1[Q], sx2[Q], cx2[Q];
    __shared__ double r0b[BCH], ctb[BCH], stb[BCH];

    const int tid = threadIdx.x;
    const int s = g.s;
    const int m = 1 << s;       // grid points per side of A
    const int np = m * m;       // grid points of A (<= 64)
    const int nBt = 1 << (2 * s);
    const int lA = g.L - s;
    const uint32_t mA = blockIdx.x;
    int a1, a2;
    morton_decode(mA, a1, a2);
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;
    const T *Tt = pick_T<T>(tb);

    if (tid < Q) {
        double s_ = 0, c_ = 1;
        if (ell) sincospi(2.0 * box_node(a1, lA, tb.z[tid]), &s_, &c_);
        sx1[tid] = s_;
        cx1[tid] = c_;
    } else if (tid >= 64 && tid < 64 + Q) {
        const int t = tid - 64;
        double s_ = 0, c_ = 1;
        if (ell) sincospi(2.0 * box_node(a2, lA, tb.z[t]), &s_, &c_);
        sx2[t] = s_;
        cx2[t] = c_;
    }
    // the grid point owned by this thread
    const int jp = tid % np;
    const int j1 = jp / m, j2 = jp - j1 * m;
    const XP xg = make_xp(ph, (double)(a1 * m + j1) / g.N, (double)(a2 * m + j2) / g.N);
    cpx<T> uacc = {(T)0, (T)0};

    const cpx<T> *src = win + (size_t)mA * nBt * QQ;
    for (int b0 = 0; b0 < nBt; b0 += BCH) {
        const int nb = min(BCH, nBt - b0);
        if (tid < nb) {
            int bb1, bb2;
            morton_decode((uint32_t)(b0 + tid), bb1, bb2);
            r0b[tid] = g.rho_scale * box_centre(bb1, s);
            double s_, c_;
            sincospi(2.0 * box_centre(bb2, s), &s_, &c_);
            ctb[tid] = c_;
            stb[tid] = s_;
        }
        __syncthreads();
        // prefactor conj E(x^A_t, p0(B)) delta^{AB}_t
        for (int i = tid; i < nb * QQ; i += NT) {
            const int b = i / QQ, t = i - b * QQ;
            const int t1 = t / Q, t2 = t - t1 * Q;
            const XP xp = make_xp_sc(ph, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]),
                                     sx1[t1], cx1[t1], sx2[t2], cx2[t2]);
            const cpx<T> e = cis<T>(r0b[b] * phase_dir(xp, ctb[b], stb[b]));
            v[i] = cmulc(src[(size_t)(b0 + b) * QQ + t], e);
        }
        __syncthreads();
        // pass 1 (second dimension): Y[b][t1][j2] = sum_t2 Tt[j2][t2] v[b][t1][t2]
        for (int i = tid; i < nb * Q * m; i += NT) {
            const int b = i / (Q * m), r = i - b * (Q * m);
            const int t1 = r / m, jj2 = r - t1 * m;
            const cpx<T> *vv = v + b * QQ + t1 * Q;
            cpx<T> acc = {(T)0, (T)0};
#pragma unroll
            for (int t2 = 0; t2 < Q; ++t2) crfma(acc, Tt[jj2 * Q + t2], vv[t2]);
            Y[i] = acc;
        }
        __syncthreads();
        // pass 2 (first dimension) and the factor E(x, p0(B)), summed per grid point
        for (int i = tid; i < nb * np; i += NT) {
            const int b = i / np;  // i % np == jp since NT % np == 0
            cpx<T> acc = {(T)0, (T)0};
            const cpx<T> *yy = Y + b * Q * m + j2;
#pragma unroll
            for (int t1 = 0; t1 < Q; ++t1) crfma(acc, Tt[j1 * Q + t1], yy[t1 * m]);
            cfma(uacc, cis<T>(r0b[b] * phase_dir(xg, ctb[b], stb[b])), acc);
        }
        __syncthreads();
    }
    red[tid] = uacc;
    __syncthreads();
    if (tid < np) {
        cpx<T> sum = red[tid];
        for (int k = tid + np; k < NT; k += np) {
            sum.re += red[k].re;
            sum.im += red[k].im;
        }
        u[(size_t)(a1 * m + j1) * g.N + (a2 * m + j2)] = sum;
    }
}

// ===========================================================================
// Adjoint kernels: conjugate transposes of the forward steps.
// ===========================================================================

// termination^H: delta^{AB}_t = E(x^A_t, p0(B)) sum_{x in A} L^A_t(x) conj E(x, p0(B)) u(x)
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_term_adj(Geom g, PhaseDev ph, Tables tb,
                                                 const cpx<T> *__restrict__ u, cpx<T> *__restrict__ wout) {
    constexpr int QQ = Q * Q;
    constexpr int BCH = bch<T, Q>();
    __shared__ cpx<T> U[BCH * 64];
    __shared__ cpx<T> Y[BCH * Q * 8];
    __shared__ double sx1[Q], cx1[Q], sx2[Q], cx2[Q];
    __shared__ double r0b[BCH], ctb[BCH], stb[BCH];

    const int tid = threadIdx.x;
    const int s = g.s;
    const int m = 1 << s, np = m * m;
    const int nBt = 1 << (2 * s);
    const int lA = g.L - s;
    const uint32_t mA = blockIdx.x;
    int a1, a2;
    morton_decode(mA, a1, a2);
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;
    const T *Tt = pick_T<T>(tb);

    if (tid < Q) {
        double s_ = 0, c_ = 1;
        if (ell) sincospi(2.0 * box_node(a1, lA, tb.z[tid]), &s_, &c_);
        sx1[tid] = s_;
        cx1[tid] = c_;
    } else if (tid >= 64 && tid < 64 + Q) {
        const int t = tid - 64;
        double s_ = 0, c_ = 1;
        if (ell) sincospi(2.0 * box_node(a2, lA, tb.z[t]), &s_, &c_);
        sx2[t] = s_;
        cx2[t] = c_;
    }
    const int jp = tid % np;
    const int j1 = jp / m, j2 = jp - j1 * m;
    const XP xg = make_xp(ph, (double)(a1 * m + j1) / g.N, (double)(a2 * m + j2) / g.N);
    const cpx<T> uv = u[(size_t)(a1 * m + j1) * g.N + (a2 * m + j2)];

    cpx<T> *dst = wout + (size_t)mA * nBt * QQ;
    for (int b0 = 0; b0 < nBt; b0 += BCH) {
        const int nb = min(BCH, nBt - b0);
        if (tid < nb) {
            int bb1, bb2;
            morton_decode((uint32_t)(b0 + tid), bb1, bb2);
            r0b[tid] = g.rho_scale * box_centre(bb1, s);
            double s_, c_;
            sincospi(2.0 * box_centre(bb2, s), &s_, &c_);
            ctb[tid] = c_;
            stb[tid] = s_;
        }
        __syncthreads();
        for (int i = tid; i < nb * np; i += NT) {
            const int b = i / np;
            U[b * np + jp] = cmulc(uv, cis<T>(r0b[b] * phase_dir(xg, ctb[b], stb[b])));
        }
        __syncthreads();
        // Y[b][t1][j2] = sum_j1 Tt[j1][t1] U[b][j1][j2]
        for (int i = tid; i < nb * Q * m; i += NT) {
            const int b = i / (Q * m), r = i - b * (Q * m);
            const int t1 = r / m, jj2 = r - t1 * m;
            cpx<T> acc = {(T)0, (T)0};
            for (int jj1 = 0; jj1 < m; ++jj1) crfma(acc, Tt[jj1 * Q + t1], U[b * np + jj1 * m + jj2]);
            Y[i] = acc;
        }
        __syncthreads();
        // delta[b][t1][t2] = E(x^A_t, p0(B)) sum_j2 Tt[j2][t2] Y[b][t1][j2]
        for (int i = tid; i < nb * QQ; i += NT) {
            const int b = i / QQ, t = i - b * QQ;
            const int t1 = t / Q, t2 = t - t1 * Q;
            cpx<T> acc = {(T)0, (T)0};
            for (int jj2 = 0; jj2 < m; ++jj2) crfma(acc, Tt[jj2 * Q + t2], Y[b * Q * m + t1 * m + jj2]);
            const XP xp = make_xp_sc(ph, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]),
                                     sx1[t1], cx1[t1], sx2[t2], cx2[t2]);
            dst[(size_t)(b0 + b) * QQ + t] = cmul(acc, cis<T>(r0b[b] * phase_dir(xp, ctb[b], stb[b])));
        }
        __syncthreads();
    }
}

// x-level^H at level l: from the outputs (A_j, B) back to the inputs (A_p, B_c)
//   delta^{A_p B_c}_t' = E(x^{A_p}_t', p0(B_c)) sum_j sum_t M_j1[t'1][t1] M_j2[t'2][t2]
//                          conj E(x^{A_j}_t, p0(B_c)) delta^{A_j B}_t
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_xlevel_adj(Geom g, PhaseDev ph, Tables tb, int level,
                                                   const cpx<T> *__restrict__ win,
                                                   cpx<T> *__restrict__ wout) {
    constexpr int QQ = Q * Q;
    __shared__ cpx<T> v[4 * QQ];    // one output pair A_j, split per c by the remodulation
    __shared__ cpx<T> Y[4 * QQ];
    __shared__ cpx<T> acc4[4 * QQ]; // accumulated over j, per c
    __shared__ T Ms[2 * QQ];
    __shared__ double sx1[Q], cx1[Q], sx2[Q], cx2[Q];
    __shared__ double r0c[2], ct0[2], st0[2];

    const int tid = threadIdx.x;
    const int lB = g.L - level;
    const size_t blk = blockIdx.x;
    const uint32_t mB = (uint32_t)(blk & (((size_t)1 << (2 * lB)) - 1));
    const uint32_t mAp = (uint32_t)(blk >> (2 * lB));
    int b1, b2, ap1, ap2;
    morton_decode(mB, b1, b2);
    morton_decode(mAp, ap1, ap2);
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;
    const size_t nBl = (size_t)1 << (2 * lB);

    const T *Mg = pick_M<T>(tb);
    for (int i = tid; i < 2 * QQ; i += NT) Ms[i] = Mg[i];
    for (int i = tid; i < 4 * QQ; i += NT) acc4[i] = {(T)0, (T)0};
    if (tid < 2) {
        r0c[tid] = g.rho_scale * box_centre(2 * b1 + tid, lB + 1);
        double s_, c_;
        sincospi(2.0 * box_centre(2 * b2 + tid, lB + 1), &s_, &c_);
        ct0[tid] = c_;
        st0[tid] = s_;
    }
    for (int j = 0; j < 4; ++j) {
        const int j1 = j >> 1, j2 = j & 1;
        const uint32_t mA = 4 * mAp + j;
        const int a1 = 2 * ap1 + j1, a2 = 2 * ap2 + j2;
        if (tid >= 64 && tid < 64 + Q) {
            const int t = tid - 64;
            double s_ = 0, c_ = 1;
            if (ell) sincospi(2.0 * box_node(a1, level, tb.z[t]), &s_, &c_);
            sx1[t] = s_;
            cx1[t] = c_;
        } else if (tid >= 128 && tid < 128 + Q) {
            const int t = tid - 128;
            double s_ = 0, c_ = 1;
            if (ell) sincospi(2.0 * box_node(a2, level, tb.z[t]), &s_, &c_);
            sx2[t] = s_;
            cx2[t] = c_;
        }
        __syncthreads();
        // v[c][t] = conj E(x^{A_j}_t, p0(B_c)) delta^{A_j B}_t
        const cpx<T> *src = win + ((size_t)mA * nBl + mB) * QQ;
        for (int i = tid; i < QQ; i += NT) {
            const int t1 = i / Q, t2 = i - t1 * Q;
            const XP xp = make_xp_sc(ph, box_node(a1, level, tb.z[t1]), box_node(a2, level, tb.z[t2]),
                                     sx1[t1], cx1[t1], sx2[t2], cx2[t2]);
            const double G0 = phase_dir(xp, ct0[0], st0[0]);
            const double G1 = phase_dir(xp, ct0[1], st0[1]);
            const cpx<T> d = src[i];
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c * QQ + i] = cmulc(d, cis<T>(r0c[c >> 1] * ((c & 1) ? G1 : G0)));
        }
        __syncthreads();
        // Y[c][t1][t'2] = sum_t2 M_j2[t'2][t2] v[c][t1][t2]
        for (int i = tid; i < 4 * QQ; i += NT) {
            const int c = i / QQ, r = i - c * QQ;
            const int t1 = r / Q, tp2 = r - t1 * Q;
            const cpx<T> *vv = v + c * QQ + t1 * Q;
            const T *mm = Ms + j2 * QQ + tp2 * Q;
            cpx<T> a = {(T)0, (T)0};
#pragma unroll
            for (int t2 = 0; t2 < Q; ++t2) crfma(a, mm[t2], vv[t2]);
            Y[i] = a;
        }
        __syncthreads();
        // acc4[c][t'1][t'2] += sum_t1 M_j1[t'1][t1] Y[c][t1][t'2]
        for (int i = tid; i < 4 * QQ; i += NT) {
            const int c = i / QQ, r = i - c * QQ;
            const int tp1 = r / Q, tp2 = r - tp1 * Q;
            const T *mm = Ms + j1 * QQ + tp1 * Q;
            cpx<T> a = acc4[i];
#pragma unroll
            for (int t1 = 0; t1 < Q; ++t1) crfma(a, mm[t1], Y[c * QQ + t1 * Q + tp2]);
            acc4[i] = a;
        }
        __syncthreads();
    }
    // sin/cos tables of A_p's nodes, then the factor E(x^{A_p}_t', p0(B_c))
    if (tid < Q) {
        double s_ = 0, c_ = 1;
        if (ell) sincospi(2.0 * box_node(ap1, level - 1, tb.z[tid]), &s_, &c_);
        sx1[tid] = s_;
        cx1[tid] = c_;
    } else if (tid >= 64 && tid < 64 + Q) {
        const int t = tid - 64;
        double s_ = 0, c_ = 1;
        if (ell) sincospi(2.0 * box_node(ap2, level - 1, tb.z[t]), &s_, &c_);
        sx2[t] = s_;
        cx2[t] = c_;
    }
    __syncthreads();
    cpx<T> *dst = wout + blk * (4 * QQ);
    for (int i = tid; i < 2 * QQ; i += NT) {
        const int c2 = i / QQ, tp = i - c2 * QQ;
        const int tp1 = tp / Q, tp2 = tp - tp1 * Q;
        const XP xp = make_xp_sc(ph, box_node(ap1, level - 1, tb.z[tp1]), box_node(ap2, level - 1, tb.z[tp2]),
                                 sx1[tp1], cx1[tp1], sx2[tp2], cx2[tp2]);
        const double G = phase_dir(xp, ct0[c2], st0[c2]);
#pragma unroll
        for (int c1 = 0; c1 < 2; ++c1) {
            const int c = 2 * c1 + c2;
            dst[c * QQ + tp] = cmul(acc4[c * QQ + tp], cis<T>(r0c[c1] * G));
        }
    }
}

template <typename T, int Q>
constexpr int swadj_ppb() {
    return (32768 / (Q * Q * (int)sizeof(cpx<T>))) < (NT / Q) ? (32768 / (Q * Q * (int)sizeof(cpx<T>))) : (NT / Q);
}

// switch^H at level lm, in place: delta_s <- sum_t conj E(x^A_t, p^B_s) delta_t.
// Thread <-> (pair, s2) accumulates all q values of s1, using the same
// rho0 + h_j symmetry as the forward switch.
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_switch_adj(Geom g, PhaseDev ph, Tables tb, cpx<T> *__restrict__ w) {
    constexpr int QQ = Q * Q;
    constexpr int H = Q / 2;
    constexpr int PPB = swadj_ppb<T, Q>();
    __shared__ cpx<T> dl[PPB][QQ];
    __shared__ double sx[PPB][2][Q], cx[PPB][2][Q];

    const int tid = threadIdx.x;
    const int pl = tid / Q, s2 = tid - pl * Q;
    const size_t npairs = (size_t)1 << (2 * g.L);
    const size_t pair = (size_t)blockIdx.x * PPB + pl;
    const bool active = (pl < PPB) && (pair < npairs);
    const int lA = g.lm, lB = g.L - g.lm;
    const size_t nBl = (size_t)1 << (2 * lB);
    const uint32_t mB = active ? (uint32_t)(pair & (nBl - 1)) : 0;
    const uint32_t mA = active ? (uint32_t)(pair >> (2 * lB)) : 0;
    int b1, b2, a1, a2;
    morton_decode(mB, b1, b2);
    morton_decode(mA, a1, a2);
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;
    cpx<T> *wp = w + pair * QQ;
    if (active) {
        for (int i = s2; i < QQ; i += Q) dl[pl][i] = wp[i];
        double s_ = 0, c_ = 1;
        if (ell) sincospi(2.0 * box_node(a1, lA, tb.z[s2]), &s_, &c_);
        sx[pl][0][s2] = s_;
        cx[pl][0][s2] = c_;
        s_ = 0;
        c_ = 1;
        if (ell) sincospi(2.0 * box_node(a2, lA, tb.z[s2]), &s_, &c_);
        sx[pl][1][s2] = s_;
        cx[pl][1][s2] = c_;
    }
    __syncthreads();
    if (!active) return;
    double st, ct;
    sincospi(2.0 * box_node(b2, lB, tb.z[s2]), &st, &ct);
    const double r0 = g.rho_scale * box_centre(b1, lB);
    double hz[H > 0 ? H : 1];
#pragma unroll
    for (int j = 0; j < H; ++j) hz[j] = g.rho_scale * ldexp(tb.z[j], -lB);
    cpx<T> acc[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) acc[k] = {(T)0, (T)0};
    for (int t1 = 0; t1 < Q; ++t1) {
        for (int t2 = 0; t2 < Q; ++t2) {
            const XP xp = make_xp_sc(ph, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]),
                                     sx[pl][0][t1], cx[pl][0][t1], sx[pl][1][t2], cx[pl][1][t2]);
            const double G = phase_dir(xp, ct, st);
            // b = conj(exp(2 pi i r0 G)) delta_t
            const cpx<T> bb = cmulc(dl[pl][t1 * Q + t2], cis<T>(r0 * G));
            if (Q & 1) {
                acc[H].re += bb.re;
                acc[H].im += bb.im;
            }
#pragma unroll
            for (int j = 0; j < H; ++j) {
                const cpx<T> d = cis<T>(hz[j] * G);
                // conj(d) b -> s1 = j ; d b -> s1 = q-1-j
                const T pr = d.re * bb.re, pi = d.re * bb.im;
                const T qr = d.im * bb.im, qi = d.im * bb.re;
                acc[j].re += pr + qr;
                acc[j].im += pi - qi;
                acc[Q - 1 - j].re += pr - qr;
                acc[Q - 1 - j].im += pi + qi;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) wp[k * Q + s2] = acc[k];
}

// p-level^H at level l: from the outputs (A_j, B) back to the inputs (A_p, B_c)
//   delta^{A_p B_c}_t' = sum_j conj E(x0(A_j), p^{B_c}_t') sum_t M_c1[t1][t'1] M_c2[t2][t'2]
//                          E(x0(A_j), p^B_t) delta^{A_j B}_t
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_plevel_adj(Geom g, PhaseDev ph, Tables tb, int level,
                                                   const cpx<T> *__restrict__ win,
                                                   cpx<T> *__restrict__ wout) {
    constexpr int QQ = Q * Q;
    __shared__ cpx<T> gj[QQ];
    __shared__ cpx<T> Y[2 * QQ];
    __shared__ cpx<T> acc4[4 * QQ];
    __shared__ T Ms[2 * QQ];
    __shared__ double rc[2 * Q], ctc[2 * Q], stc[2 * Q];
    __shared__ double rb[Q], ctb[Q], stb[Q];
    __shared__ double Gc[2 * Q], Gb[Q];

    const int tid = threadIdx.x;
    const int lB = g.L - level;
    const size_t blk = blockIdx.x;
    const uint32_t mB = (uint32_t)(blk & (((size_t)1 << (2 * lB)) - 1));
    const uint32_t mAp = (uint32_t)(blk >> (2 * lB));
    int b1, b2, ap1, ap2;
    morton_decode(mB, b1, b2);
    morton_decode(mAp, ap1, ap2);
    const size_t nBl = (size_t)1 << (2 * lB);

    const T *Mg = pick_M<T>(tb);
    for (int i = tid; i < 2 * QQ; i += NT) Ms[i] = Mg[i];
    for (int i = tid; i < 4 * QQ; i += NT) acc4[i] = {(T)0, (T)0};
    if (tid < 2 * Q) {
        const int c = tid / Q, t = tid - c * Q;
        const double z = tb.z[t];
        rc[tid] = g.rho_scale * box_node(2 * b1 + c, lB + 1, z);
        double s_, c_;
        sincospi(2.0 * box_node(2 * b2 + c, lB + 1, z), &s_, &c_);
        ctc[tid] = c_;
        stc[tid] = s_;
    } else if (tid >= 64 && tid < 64 + Q) {
        const int t = tid - 64;
        const double z = tb.z[t];
        rb[t] = g.rho_scale * box_node(b1, lB, z);
        double s_, c_;
        sincospi(2.0 * box_node(b2, lB, z), &s_, &c_);
        ctb[t] = c_;
        stb[t] = s_;
    }
    __syncthreads();
    for (int j = 0; j < 4; ++j) {
        const uint32_t mA = 4 * mAp + j;
        const int a1 = 2 * ap1 + (j >> 1), a2 = 2 * ap2 + (j & 1);
        const XP xp = make_xp(ph, box_centre(a1, level), box_centre(a2, level));
        if (tid < 2 * Q) Gc[tid] = phase_dir(xp, ctc[tid], stc[tid]);
        else if (tid >= 64 && tid < 64 + Q) Gb[tid - 64] = phase_dir(xp, ctb[tid - 64], stb[tid - 64]);
        __syncthreads();
        const cpx<T> *src = win + ((size_t)mA * nBl + mB) * QQ;
        for (int i = tid; i < QQ; i += NT) {
            const int t1 = i / Q, t2 = i - t1 * Q;
            gj[i] = cmul(src[i], cis<T>(rb[t1] * Gb[t2]));
        }
        __syncthreads();
        // Y[c1][t1][t'2]... first the second dimension: Y[c2][t1][t'2] = sum_t2 M_c2[t2][t'2] g[t1][t2]
        for (int i = tid; i < 2 * QQ; i += NT) {
            const int c2 = i / QQ, r = i - c2 * QQ;
            const int t1 = r / Q, tp2 = r - t1 * Q;
            const T *mm = Ms + c2 * QQ + tp2;
            const cpx<T> *gg = gj + t1 * Q;
            cpx<T> a = {(T)0, (T)0};
#pragma unroll
            for (int t2 = 0; t2 < Q; ++t2) crfma(a, mm[t2 * Q], gg[t2]);
            Y[i] = a;
        }
        __syncthreads();
        // then the first dimension and the conj prefactor, accumulated over j
        for (int i = tid; i < 4 * QQ; i += NT) {
            const int c = i / QQ, r = i - c * QQ;
            const int c1 = c >> 1, c2 = c & 1;
            const int tp1 = r / Q, tp2 = r - tp1 * Q;
            const T *mm = Ms + c1 * QQ + tp1;
            cpx<T> a = {(T)0, (T)0};
#pragma unroll
            for (int t1 = 0; t1 < Q; ++t1) crfma(a, mm[t1 * Q], Y[c2 * QQ + t1 * Q + tp2]);
            const cpx<T> e = cis<T>(rc[c1 * Q + tp1] * Gc[c2 * Q + tp2]);
            const cpx<T> add = cmulc(a, e);
            acc4[i].re += add.re;
            acc4[i].im += add.im;
        }
        __syncthreads();
    }
    cpx<T> *dst = wout + blk * (4 * QQ);
    for (int i = tid; i < 4 * QQ; i += NT) dst[i] = acc4[i];
}

// initialisation^H: f(p) = sum_A conj E(x0(A), p) sum_t L^B_t(p) E(x0(A), p^B_t) delta^{AB}_t
// One workgroup per B box at level L-s; the weighted sums over t are formed
// per (A, t) in LDS in chunks of A, then every source of B accumulates over A.
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_init_adj(Geom g, PhaseDev ph, Tables tb, Sources src,
                                                 const cpx<T> *__restrict__ win, cpx<T> *__restrict__ f) {
    constexpr int QQ = Q * Q;
    constexpr int ACH2 = 8;
    __shared__ cpx<T> gA[ACH2][QQ];
    __shared__ double zs[Q], ls[Q];
    __shared__ double ctb[Q], stb[Q];
    __shared__ XP xA[ACH2];

    const int tid = threadIdx.x;
    const int lB = g.L - g.s;
    const uint32_t mB = blockIdx.x;
    const int nA = 1 << (2 * g.s);
    const size_t nBl = (size_t)1 << (2 * lB);
    int bp1, bp2;
    morton_decode(mB, bp1, bp2);
    const double scale = ldexp(1.0, lB);
    if (tid < Q) {
        zs[tid] = tb.z[tid];
        ls[tid] = tb.lam[tid];
        double s_, c_;
        sincospi(2.0 * box_node(bp2, lB, tb.z[tid]), &s_, &c_);
        ctb[tid] = c_;
        stb[tid] = s_;
    }
    __syncthreads();
    const int beg = src.off[mB], end = src.off[mB + 1];
    for (int c0 = beg; c0 < end; c0 += NT) {
        const int jsrc = c0 + tid;
        const bool has = jsrc < end;
        T l1[Q], l2[Q];
        double k1 = 0, k2 = 0;
        int idx = 0;
        if (has) {
            idx = src.idx[jsrc];
            const double2 p = src.p[jsrc];
            lagrange_row<T, Q>(p.x * scale - ((double)bp1 + 0.5), zs, ls, l1);
            lagrange_row<T, Q>(p.y * scale - ((double)bp2 + 0.5), zs, ls, l2);
            k1 = (double)(idx / g.N - g.N / 2);
            k2 = (double)(idx % g.N - g.N / 2);
        }
        cpx<T> out = {(T)0, (T)0};
        for (int a0 = 0; a0 < nA; a0 += ACH2) {
            const int na = min(ACH2, nA - a0);
            __syncthreads();
            if (tid < na) {
                int a1, a2;
                morton_decode((uint32_t)(a0 + tid), a1, a2);
                xA[tid] = make_xp(ph, box_centre(a1, g.s), box_centre(a2, g.s));
            }
            __syncthreads();
            for (int i = tid; i < na * QQ; i += NT) {
                const int al = i / QQ, t = i - al * QQ;
                const int t1 = t / Q, t2 = t - t1 * Q;
                const double rho = g.rho_scale * box_node(bp1, lB, zs[t1]);
                const cpx<T> e = cis<T>(rho * phase_dir(xA[al], ctb[t2], stb[t2]));
                gA[al][t] = cmul(win[((size_t)(a0 + al) * nBl + mB) * QQ + t], e);
            }
            __syncthreads();
            if (has) {
                for (int al = 0; al < na; ++al) {
                    cpx<T> sacc = {(T)0, (T)0};
#pragma unroll
                    for (int t1 = 0; t1 < Q; ++t1) {
                        cpx<T> r = {(T)0, (T)0};
#pragma unroll
                        for (int t2 = 0; t2 < Q; ++t2) crfma(r, l2[t2], gA[al][t1 * Q + t2]);
                        crfma(sacc, l1[t1], r);
                    }
                    cfma(out, sacc, cis<T>(-phase_cart(xA[al], k1, k2)));
                }
            }
        }
        if (has) f[idx] = out;
    }
}

// ===========================================================================
// Launchers: dispatch on (dtype, q)
// ===========================================================================
#define FIO_DISPATCH_Q(q, MACRO) \
    switch (q) {                 \
        case 3: MACRO(3); break; \
        case 4: MACRO(4); break; \
        case 5: MACRO(5); break; \
        case 6: MACRO(6); break; \
        case 7: MACRO(7); break; \
        case 8: MACRO(8); break; \
        case 9: MACRO(9); break; \
        case 10: MACRO(10); break; \
        case 11: MACRO(11); break; \
        case 12: MACRO(12); break; \
        case 13: MACRO(13); break; \
        case 14: MACRO(14); break; \
        case 15: MACRO(15); break; \
        case 16: MACRO(16); break; \
        default: return hipErrorInvalidValue; \
    }

template <typename T>
static hipError_t init_t(const Geom &g, const PhaseDev &ph, const Tables &tb, const Sources &src,
                         const void *f, void *w, hipStream_t st) {
    const unsigned nB = 1u << (2 * (g.L - g.s));
    const int nA = 1 << (2 * g.s);
#define L_INIT(Q)                                                                                    \
    {                                                                                                \
        constexpr int ACH = (NT / Q) < 64 ? (NT / Q) : 64;                                           \
        dim3 grid(nB, (nA + ACH - 1) / ACH);                                                         \
        hipLaunchKernelGGL((k_init<T, Q>), grid, dim3(NT), 0, st, g, ph, tb, src,                     \
                           (const cpx<T> *)f, (cpx<T> *)w);                                          \
    }
    FIO_DISPATCH_Q(g.q, L_INIT)
#undef L_INIT
    return hipGetLastError();
}

template <typename T>
static hipError_t plevel_t(const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                           const void *win, void *wout, hipStream_t st) {
    const unsigned nblk = 1u << (2 * g.L - 2);
#define L_PL(Q)                                                                                      \
    hipLaunchKernelGGL((k_plevel<T, Q>), dim3(nblk), dim3(NT), 0, st, g, ph, tb, level,              \
                       (const cpx<T> *)win, (cpx<T> *)wout);
    FIO_DISPATCH_Q(g.q, L_PL)
#undef L_PL
    return hipGetLastError();
}

template <typename T>
static hipError_t xlevel_t(const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                           const void *win, void *wout, hipStream_t st) {
    const unsigned nblk = 1u << (2 * g.L - 2);
#define L_XL(Q)                                                                                      \
    hipLaunchKernelGGL((k_xlevel<T, Q>), dim3(nblk), dim3(NT), 0, st, g, ph, tb, level,              \
                       (const cpx<T> *)win, (cpx<T> *)wout);
    FIO_DISPATCH_Q(g.q, L_XL)
#undef L_XL
    return hipGetLastError();
}

template <typename T>
static hipError_t switch_t(const Geom &g, const PhaseDev &ph, const Tables &tb, void *w, hipStream_t st) {
    const size_t npairs = (size_t)1 << (2 * g.L);
#define L_SW(Q)                                                                                      \
    {                                                                                                \
        constexpr int PPB = NT / (Q * Q);                                                            \
        const unsigned nblk = (unsigned)((npairs + PPB - 1) / PPB);                                  \
        hipLaunchKernelGGL((k_switch<T, Q>), dim3(nblk), dim3(NT), 0, st, g, ph, tb, (cpx<T> *)w);   \
    }
    FIO_DISPATCH_Q(g.q, L_SW)
#undef L_SW
    return hipGetLastError();
}

template <typename T>
static hipError_t term_t(const Geom &g, const PhaseDev &ph, const Tables &tb, const void *win, void *u,
                         hipStream_t st) {
    const unsigned nA = 1u << (2 * (g.L - g.s));
#define L_TM(Q)                                                                                      \
    hipLaunchKernelGGL((k_term<T, Q>), dim3(nA), dim3(NT), 0, st, g, ph, tb, (const cpx<T> *)win,    \
                       (cpx<T> *)u);
    FIO_DISPATCH_Q(g.q, L_TM)
#undef L_TM
    return hipGetLastError();
}

template <typename T>
static hipError_t term_adj_t(const Geom &g, const PhaseDev &ph, const Tables &tb, const void *u, void *w,
                             hipStream_t st) {
    const unsigned nA = 1u << (2 * (g.L - g.s));
#define L_TMA(Q)                                                                                     \
    hipLaunchKernelGGL((k_term_adj<T, Q>), dim3(nA), dim3(NT), 0, st, g, ph, tb, (const cpx<T> *)u,  \
                       (cpx<T> *)w);
    FIO_DISPATCH_Q(g.q, L_TMA)
#undef L_TMA
    return hipGetLastError();
}

template <typename T>
static hipError_t xlevel_adj_t(const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                               const void *win, void *wout, hipStream_t st) {
    const unsigned nblk = 1u << (2 * g.L - 2);
#define L_XLA(Q)                                                                                     \
    hipLaunchKernelGGL((k_xlevel_adj<T, Q>), dim3(nblk), dim3(NT), 0, st, g, ph, tb, level,          \
                       (const cpx<T> *)win, (cpx<T> *)wout);
    FIO_DISPATCH_Q(g.q, L_XLA)
#undef L_XLA
    return hipGetLastError();
}

template <typename T>
static hipError_t switch_adj_t(const Geom &g, const PhaseDev &ph, const Tables &tb, void *w,
                               hipStream_t st) {
    const size_t npairs = (size_t)1 << (2 * g.L);
#define L_SWA(Q)                                                                                     \
    {                                                                                                \
        constexpr int PPB = swadj_ppb<T, Q>();                                                       \
        const unsigned nblk = (unsigned)((npairs + PPB - 1) / PPB);                                  \
        hipLaunchKernelGGL((k_switch_adj<T, Q>), dim3(nblk), dim3(NT), 0, st, g, ph, tb,             \
                           (cpx<T> *)w);                                                             \
    }
    FIO_DISPATCH_Q(g.q, L_SWA)
#undef L_SWA
    return hipGetLastError();
}

template <typename T>
static hipError_t plevel_adj_t(const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                               const void *win, void *wout, hipStream_t st) {
    const unsigned nblk = 1u << (2 * g.L - 2);
#define L_PLA(Q)                                                                                     \
    hipLaunchKernelGGL((k_plevel_adj<T, Q>), dim3(nblk), dim3(NT), 0, st, g, ph, tb, level,          \
                       (const cpx<T> *)win, (cpx<T> *)wout);
    FIO_DISPATCH_Q(g.q, L_PLA)
#undef L_PLA
    return hipGetLastError();
}

template <typename T>
static hipError_t init_adj_t(const Geom &g, const PhaseDev &ph, const Tables &tb, const Sources &src,
                             const void *w, void *f, hipStream_t st) {
    const unsigned nB = 1u << (2 * (g.L - g.s));
#define L_INA(Q)                                                                                     \
    hipLaunchKernelGGL((k_init_adj<T, Q>), dim3(nB), dim3(NT), 0, st, g, ph, tb, src,                \
                       (const cpx<T> *)w, (cpx<T> *)f);
    FIO_DISPATCH_Q(g.q, L_INA)
#undef L_INA
    return hipGetLastError();
}

#define FIO_BY_DTYPE(dtype, CALL) \
    ((dtype) == FIO_C128 ? CALL(double) : CALL(float))

hipError_t launch_init(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, const Sources &src,
                       const void *f, void *w, hipStream_t st) {
#define C(T) init_t<T>(g, ph, tb, src, f, w, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_plevel(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                         const void *win, void *wout, hipStream_t st) {
#define C(T) plevel_t<T>(g, ph, tb, level, win, wout, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_switch(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, void *w,
                         hipStream_t st) {
#define C(T) switch_t<T>(g, ph, tb, w, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_xlevel(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                         const void *win, void *wout, hipStream_t st) {
#define C(T) xlevel_t<T>(g, ph, tb, level, win, wout, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_term(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, const void *win,
                       void *u, hipStream_t st) {
#define C(T) term_t<T>(g, ph, tb, win, u, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_term_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, const void *u,
                           void *w, hipStream_t st) {
#define C(T) term_adj_t<T>(g, ph, tb, u, w, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_xlevel_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                             const void *win, void *wout, hipStream_t st) {
#define C(T) xlevel_adj_t<T>(g, ph, tb, level, win, wout, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_switch_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, void *w,
                             hipStream_t st) {
#define C(T) switch_adj_t<T>(g, ph, tb, w, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_plevel_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                             const void *win, void *wout, hipStream_t st) {
#define C(T) plevel_adj_t<T>(g, ph, tb, level, win, wout, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_init_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb,
                           const Sources &src, const void *w, void *f, hipStream_t st) {
#define C(T) init_adj_t<T>(g, ph, tb, src, w, f, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}

}  // namespace fio
