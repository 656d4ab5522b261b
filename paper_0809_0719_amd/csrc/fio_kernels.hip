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
// Butterfly blocks per workgroup for the level kernels: 8q threads per block
// (2q per output pair), limited so the block's LDS stays near 40 KB.
// ===========================================================================
template <typename T, int Q, int PERBB>
constexpr int blocks_per_wg() {
    constexpr int byT = NT / (8 * Q);
    constexpr int byL = 40960 / (PERBB * Q * Q * (int)sizeof(cpx<T>));
    constexpr int b = byT < byL ? byT : byL;
    return b < 1 ? 1 : b;
}

// ===========================================================================
// Step 3, p-recursion (eq:alg2b) at level l: block (A_p at l-1, B at L-l)
//   delta^{AB}_t = conj E(x0(A), p^B_t) sum_c sum_t' M_c1[t1][t'1] M_c2[t2][t'2]
//                     E(x0(A), p^{B_c}_t') delta^{A_p B_c}_t'
// for the four children A of A_p.  The q x q Kronecker sum over the four
// children B_c is done one dimension at a time (Sec. 4: 6 q^3 per pair).
// Each output pair gets 2q threads: in the first pass thread (c1, t'1)
// forms its prefactored row of the two children (c1, 0), (c1, 1) in
// registers and contracts it against M_c2 (read as LDS broadcasts); in the
// second pass thread (t2, half) takes column t2 and produces half the rows
// t1, remodulated and stored.
// ===========================================================================
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_plevel(Geom g, PhaseDev ph, Tables tb, int level,
                                               const cpx<T> *__restrict__ win,
                                               cpx<T> *__restrict__ wout, unsigned nblk) {
    constexpr int QQ = Q * Q;
    constexpr int TPO = 2 * Q;            // threads per output pair
    constexpr int TPB = 4 * TPO;          // threads per butterfly block
    constexpr int BPW = blocks_per_wg<T, Q, 8>();
    constexpr int H1 = (Q + 1) / 2;
    __shared__ T Mt[2][Q][Q];             // Mt[c][t'][t] = M_c[t][t']
    __shared__ T Ms[2][Q][Q];             // Ms[c][t][t'] = M_c[t][t']
    __shared__ double rc[BPW][2 * Q], ctc[BPW][2 * Q], stc[BPW][2 * Q];  // child nodes: rho(c1,t'), theta(c2,t')
    __shared__ double rb[BPW][Q], ctb[BPW][Q], stb[BPW][Q];              // B's nodes
    __shared__ double Gc[BPW][4][2 * Q], Gb[BPW][4][Q];
    __shared__ cpx<T> W[BPW][4][2 * QQ];  // first-pass rows [c1][t'1][t2]

    const int tid = threadIdx.x;
    const int bbl = tid / TPB, r = tid - bbl * TPB;
    const int j = r / TPO, rr = r - j * TPO;
    const size_t blk = (size_t)blockIdx.x * BPW + bbl;
    const bool active = bbl < BPW && blk < nblk;
    const int lB = g.L - level;
    const size_t nBl = (size_t)1 << (2 * lB);

    const T *Mg = pick_M<T>(tb);
    for (int i = tid; i < 2 * QQ; i += NT) {
        const int c = i / QQ, t = (i - c * QQ) / Q, tp = i - c * QQ - t * Q;
        Ms[c][t][tp] = Mg[i];
        Mt[c][tp][t] = Mg[i];
    }
    uint32_t mB = 0, mAp = 0;
    int b1 = 0, b2 = 0, ap1 = 0, ap2 = 0;
    if (active) {
        mB = (uint32_t)(blk & (nBl - 1));
        mAp = (uint32_t)(blk >> (2 * lB));
        morton_decode(mB, b1, b2);
        morton_decode(mAp, ap1, ap2);
        if (j == 0) {
            const int c = rr / Q, t = rr - c * Q;
            const double z = tb.z[t];
            rc[bbl][rr] = g.rho_scale * box_node(2 * b1 + c, lB + 1, z);
            double s_, c_;
            sincospi(2.0 * box_node(2 * b2 + c, lB + 1, z), &s_, &c_);
            ctc[bbl][rr] = c_;
            stc[bbl][rr] = s_;
        } else if (j == 1 && rr < Q) {
            const double z = tb.z[rr];
            rb[bbl][rr] = g.rho_scale * box_node(b1, lB, z);
            double s_, c_;
            sincospi(2.0 * box_node(b2, lB, z), &s_, &c_);
            ctb[bbl][rr] = c_;
            stb[bbl][rr] = s_;
        }
    }
    __syncthreads();
    const int a1 = 2 * ap1 + (j >> 1), a2 = 2 * ap2 + (j & 1);
    if (active) {
        const XP xp = make_xp(ph, box_centre(a1, level), box_centre(a2, level));
        Gc[bbl][j][rr] = phase_dir(xp, ctc[bbl][rr], stc[bbl][rr]);
        if (rr < Q) Gb[bbl][j][rr] = phase_dir(xp, ctb[bbl][rr], stb[bbl][rr]);
    }
    __syncthreads();
    if (active) {
        // first pass: row (c1, t'1)
        const int c1 = rr / Q, tp1 = rr - c1 * Q;
        const double rho = rc[bbl][rr];
        cpx<T> acc[Q];
#pragma unroll
        for (int t = 0; t < Q; ++t) acc[t] = {(T)0, (T)0};
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2) {
            const cpx<T> *src = win + (blk * 4 + 2 * c1 + c2) * QQ + tp1 * Q;
#pragma unroll
            for (int tp2 = 0; tp2 < Q; ++tp2) {
                const cpx<T> v = cmul(cis<T>(rho * Gc[bbl][j][c2 * Q + tp2]), src[tp2]);
#pragma unroll
                for (int t2 = 0; t2 < Q; ++t2) crfma(acc[t2], Mt[c2][tp2][t2], v);
            }
        }
#pragma unroll
        for (int t2 = 0; t2 < Q; ++t2) W[bbl][j][rr * Q + t2] = acc[t2];
    }
    __syncthreads();
    if (active) {
        // second pass: column t2, rows t1 of one half, then remodulation
        const int h = rr / Q, t2 = rr - h * Q;
        cpx<T> col[2 * Q];
#pragma unroll
        for (int k = 0; k < 2 * Q; ++k) col[k] = W[bbl][j][k * Q + t2];
        const double G = Gb[bbl][j][t2];
        cpx<T> *dst = wout + ((size_t)(4 * mAp + j) * nBl + mB) * QQ;
#pragma unroll
        for (int k = 0; k < H1; ++k) {
            const int t1 = h * H1 + k;
            if (t1 < Q) {
                cpx<T> o = {(T)0, (T)0};
#pragma unroll
                for (int c1 = 0; c1 < 2; ++c1)
#pragma unroll
                    for (int tp1 = 0; tp1 < Q; ++tp1) crfma(o, Ms[c1][t1][tp1], col[c1 * Q + tp1]);
                dst[t1 * Q + t2] = cmulc(o, cis<T>(rb[bbl][t1] * G));
            }
        }
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
// (A_p, B_c) and is applied once per block; the first (second-dimension)
// pass depends on A only through a2, so it is shared by the children with
// the same a2.  Threads: prefactor (c, t'1) rows; first pass (a2, c, t'1)
// rows; second pass (A, t2, half) columns with the remodulation per B_c.
// ===========================================================================
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_xlevel(Geom g, PhaseDev ph, Tables tb, int level,
                                               const cpx<T> *__restrict__ win,
                                               cpx<T> *__restrict__ wout, unsigned nblk) {
    constexpr int QQ = Q * Q;
    constexpr int TPB = 8 * Q;
    constexpr int BPW = blocks_per_wg<T, Q, 12>();
    constexpr int H1 = (Q + 1) / 2;
    __shared__ T Ms[2][Q][Q];                       // Ms[a][t'][t] = M_a[t'][t]
    __shared__ cpx<T> v[BPW][4][QQ];                // prefactored inputs [c][t'1][t'2]
    __shared__ cpx<T> Y[BPW][2][4][QQ];             // first pass [a2][c][t'1][t2]
    __shared__ double sp[BPW][2][Q], cp[BPW][2][Q];        // sin/cos(2 pi x) at A_p's nodes, per dim
    __shared__ double sj[BPW][2][2][Q], cj[BPW][2][2][Q];  // at the children's nodes [dim][a][t]
    __shared__ double r0c[BPW][2], ct0[BPW][2], st0[BPW][2];

    const int tid = threadIdx.x;
    const int bbl = tid / TPB, rr = tid - bbl * TPB;
    const size_t blk = (size_t)blockIdx.x * BPW + bbl;
    const bool active = bbl < BPW && blk < nblk;
    const int lB = g.L - level;
    const size_t nBl = (size_t)1 << (2 * lB);
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;

    const T *Mg = pick_M<T>(tb);
    for (int i = tid; i < 2 * QQ; i += NT) (&Ms[0][0][0])[i] = Mg[i];
    uint32_t mB = 0, mAp = 0;
    int b1 = 0, b2 = 0, ap1 = 0, ap2 = 0;
    if (active) {
        mB = (uint32_t)(blk & (nBl - 1));
        mAp = (uint32_t)(blk >> (2 * lB));
        morton_decode(mB, b1, b2);
        morton_decode(mAp, ap1, ap2);
        if (rr < 2 * Q) {                      // A_p's nodes, dim rr / Q
            const int d = rr / Q, t = rr - d * Q;
            double s_ = 0, c_ = 1;
            if (ell) sincospi(2.0 * box_node(d ? ap2 : ap1, level - 1, tb.z[t]), &s_, &c_);
            sp[bbl][d][t] = s_;
            cp[bbl][d][t] = c_;
        } else if (rr < 6 * Q) {               // children's nodes, [dim][a][t]
            const int k = rr - 2 * Q, d = k / (2 * Q), a = (k / Q) & 1, t = k % Q;
            double s_ = 0, c_ = 1;
            if (ell) sincospi(2.0 * box_node(2 * (d ? ap2 : ap1) + a, level, tb.z[t]), &s_, &c_);
            sj[bbl][d][a][t] = s_;
            cj[bbl][d][a][t] = c_;
        } else if (rr < 6 * Q + 2) {           // p0(B_c): rho by c1, theta by c2
            const int c = rr - 6 * Q;
            r0c[bbl][c] = g.rho_scale * box_centre(2 * b1 + c, lB + 1);
            double s_, c_;
            sincospi(2.0 * box_centre(2 * b2 + c, lB + 1), &s_, &c_);
            ct0[bbl][c] = c_;
            st0[bbl][c] = s_;
        }
    }
    __syncthreads();
    // prefactor conj E(x^{A_p}_t', p0(B_c)) delta^{A_p B_c}_t': row (c, t'1)
    if (active && rr < 4 * Q) {
        const int c = rr / Q, tp1 = rr - c * Q;
        const int c1 = c >> 1, c2 = c & 1;
        const cpx<T> *src = win + (blk * 4 + c) * QQ + tp1 * Q;
        const double xa1 = box_node(ap1, level - 1, tb.z[tp1]);
#pragma unroll
        for (int tp2 = 0; tp2 < Q; ++tp2) {
            const XP xp = make_xp_sc(ph, xa1, box_node(ap2, level - 1, tb.z[tp2]), sp[bbl][0][tp1],
                                     cp[bbl][0][tp1], sp[bbl][1][tp2], cp[bbl][1][tp2]);
            const double G = phase_dir(xp, ct0[bbl][c2], st0[bbl][c2]);
            v[bbl][c][tp1 * Q + tp2] = cmulc(src[tp2], cis<T>(r0c[bbl][c1] * G));
        }
    }
    __syncthreads();
    // first pass (second dimension): Y[a2][c][t'1][t2] = sum_t'2 M_a2[t'2][t2] v[c][t'1][t'2]
    if (active) {
        const int a2c = rr / (4 * Q), k = rr - a2c * 4 * Q;
        const int c = k / Q, tp1 = k - c * Q;
        cpx<T> acc[Q];
#pragma unroll
        for (int t = 0; t < Q; ++t) acc[t] = {(T)0, (T)0};
#pragma unroll
        for (int tp2 = 0; tp2 < Q; ++tp2) {
            const cpx<T> vv = v[bbl][c][tp1 * Q + tp2];
#pragma unroll
            for (int t2 = 0; t2 < Q; ++t2) crfma(acc[t2], Ms[a2c][tp2][t2], vv);
        }
#pragma unroll
        for (int t2 = 0; t2 < Q; ++t2) Y[bbl][a2c][c][tp1 * Q + t2] = acc[t2];
    }
    __syncthreads();
    // second pass (first dimension), remodulation E(x^A_t, p0(B_c)), sum over c
    if (active) {
        const int jj = rr / (2 * Q), k = rr - jj * 2 * Q;
        const int h = k / Q, t2 = k - h * Q;
        const int j1 = jj >> 1, j2 = jj & 1;
        const int a1 = 2 * ap1 + j1, a2 = 2 * ap2 + j2;
        double G0[H1], G1[H1];
        cpx<T> out[H1];
        const double xb2 = box_node(a2, level, tb.z[t2]);
#pragma unroll
        for (int kk = 0; kk < H1; ++kk) {
            const int t1 = min(h * H1 + kk, Q - 1);
            const XP xp = make_xp_sc(ph, box_node(a1, level, tb.z[t1]), xb2, sj[bbl][0][j1][t1],
                                     cj[bbl][0][j1][t1], sj[bbl][1][j2][t2], cj[bbl][1][j2][t2]);
            G0[kk] = phase_dir(xp, ct0[bbl][0], st0[bbl][0]);
            G1[kk] = phase_dir(xp, ct0[bbl][1], st0[bbl][1]);
            out[kk] = {(T)0, (T)0};
        }
#pragma unroll 1
        for (int c = 0; c < 4; ++c) {
            const int c1 = c >> 1, c2 = c & 1;
            cpx<T> col[Q];
#pragma unroll
            for (int tp1 = 0; tp1 < Q; ++tp1) col[tp1] = Y[bbl][j2][c][tp1 * Q + t2];
            const double rho = r0c[bbl][c1];
#pragma unroll
            for (int kk = 0; kk < H1; ++kk) {
                const int t1 = min(h * H1 + kk, Q - 1);
                cpx<T> z = {(T)0, (T)0};
#pragma unroll
                for (int tp1 = 0; tp1 < Q; ++tp1) crfma(z, Ms[j1][tp1][t1], col[tp1]);
                cfma(out[kk], cis<T>(rho * (c2 ? G1[kk] : G0[kk])), z);
            }
        }
        cpx<T> *dst = wout + ((size_t)(4 * mAp + jj) * nBl + mB) * QQ;
#pragma unroll
        for (int kk = 0; kk < H1; ++kk) {
            const int t1 = h * H1 + kk;
            if (t1 < Q) dst[t1 * Q + t2] = out[kk];
        }
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
// First pass: thread (j1, c2, t1, j2) forms row t1 of conj E delta for its
// child (j1, j2) and both c1, contracts over t2 with M_j2, and the two j2
// partial rows are added through a lane exchange.  Second pass: thread
// (c, t'2, half) contracts over t1 with M_j1, sums j1 and applies the factor
// E(x^{A_p}_t', p0(B_c)).
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_xlevel_adj(Geom g, PhaseDev ph, Tables tb, int level,
                                                   const cpx<T> *__restrict__ win,
                                                   cpx<T> *__restrict__ wout, unsigned nblk) {
    constexpr int QQ = Q * Q;
    constexpr int TPB = 8 * Q;
    constexpr int BPW = blocks_per_wg<T, Q, 8>();
    constexpr int H1 = (Q + 1) / 2;
    __shared__ T Ms[2][Q][Q];                       // Ms[a][t'][t] = M_a[t'][t]
    __shared__ cpx<T> Y[BPW][2][4][QQ];             // [j1][c][t1][t'2]
    __shared__ double sp[BPW][2][Q], cp[BPW][2][Q];
    __shared__ double sj[BPW][2][2][Q], cj[BPW][2][2][Q];
    __shared__ double r0c[BPW][2], ct0[BPW][2], st0[BPW][2];

    const int tid = threadIdx.x;
    const int bbl = tid / TPB, rr = tid - bbl * TPB;
    const size_t blk = (size_t)blockIdx.x * BPW + bbl;
    const bool active = bbl < BPW && blk < nblk;
    const int lB = g.L - level;
    const size_t nBl = (size_t)1 << (2 * lB);
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;

    const T *Mg = pick_M<T>(tb);
    for (int i = tid; i < 2 * QQ; i += NT) (&Ms[0][0][0])[i] = Mg[i];
    uint32_t mB = 0, mAp = 0;
    int b1 = 0, b2 = 0, ap1 = 0, ap2 = 0;
    if (active) {
        mB = (uint32_t)(blk & (nBl - 1));
        mAp = (uint32_t)(blk >> (2 * lB));
        morton_decode(mB, b1, b2);
        morton_decode(mAp, ap1, ap2);
        if (rr < 2 * Q) {
            const int d = rr / Q, t = rr - d * Q;
            double s_ = 0, c_ = 1;
            if (ell) sincospi(2.0 * box_node(d ? ap2 : ap1, level - 1, tb.z[t]), &s_, &c_);
            sp[bbl][d][t] = s_;
            cp[bbl][d][t] = c_;
        } else if (rr < 6 * Q) {
            const int k = rr - 2 * Q, d = k / (2 * Q), a = (k / Q) & 1, t = k % Q;
            double s_ = 0, c_ = 1;
            if (ell) sincospi(2.0 * box_node(2 * (d ? ap2 : ap1) + a, level, tb.z[t]), &s_, &c_);
            sj[bbl][d][a][t] = s_;
            cj[bbl][d][a][t] = c_;
        } else if (rr < 6 * Q + 2) {
            const int c = rr - 6 * Q;
            r0c[bbl][c] = g.rho_scale * box_centre(2 * b1 + c, lB + 1);
            double s_, c_;
            sincospi(2.0 * box_centre(2 * b2 + c, lB + 1), &s_, &c_);
            ct0[bbl][c] = c_;
            st0[bbl][c] = s_;
        }
    }
    __syncthreads();
    {
        // rr = ((j1 * 2 + c2) * Q + t1) * 2 + j2: the two j2 of a row are adjacent lanes
        const int j2 = rr & 1, k = rr >> 1;
        const int t1 = k % Q, jc = k / Q, c2 = jc & 1, j1 = jc >> 1;
        cpx<T> acc0[Q], acc1[Q];   // c1 = 0, 1
#pragma unroll
        for (int t = 0; t < Q; ++t) acc0[t] = acc1[t] = {(T)0, (T)0};
        if (active) {
            const int a1 = 2 * ap1 + j1, a2 = 2 * ap2 + j2;
            const cpx<T> *src = win + ((size_t)(4 * mAp + 2 * j1 + j2) * nBl + mB) * QQ + t1 * Q;
            const double xa1 = box_node(a1, level, tb.z[t1]);
#pragma unroll
            for (int t2 = 0; t2 < Q; ++t2) {
                const XP xp = make_xp_sc(ph, xa1, box_node(a2, level, tb.z[t2]), sj[bbl][0][j1][t1],
                                         cj[bbl][0][j1][t1], sj[bbl][1][j2][t2], cj[bbl][1][j2][t2]);
                const double G = phase_dir(xp, ct0[bbl][c2], st0[bbl][c2]);
                const cpx<T> d = src[t2];
                const cpx<T> v0 = cmulc(d, cis<T>(r0c[bbl][0] * G));
                const cpx<T> v1 = cmulc(d, cis<T>(r0c[bbl][1] * G));
#pragma unroll
                for (int tp2 = 0; tp2 < Q; ++tp2) {
                    const T m = Ms[j2][tp2][t2];
                    crfma(acc0[tp2], m, v0);
                    crfma(acc1[tp2], m, v1);
                }
            }
        }
        // add the partner lane's (other j2) partial rows
#pragma unroll
        for (int t = 0; t < Q; ++t) {
            acc0[t].re += __shfl_xor(acc0[t].re, 1);
            acc0[t].im += __shfl_xor(acc0[t].im, 1);
            acc1[t].re += __shfl_xor(acc1[t].re, 1);
            acc1[t].im += __shfl_xor(acc1[t].im, 1);
        }
        if (active && j2 == 0) {
#pragma unroll
            for (int tp2 = 0; tp2 < Q; ++tp2) {
                Y[bbl][j1][c2][t1 * Q + tp2] = acc0[tp2];        // c = 2*0 + c2
                Y[bbl][j1][2 + c2][t1 * Q + tp2] = acc1[tp2];    // c = 2*1 + c2
            }
        }
    }
    __syncthreads();
    if (active) {
        // second pass: thread (c, t'2, half)
        const int c = rr / (2 * Q), k = rr - c * 2 * Q;
        const int h = k / Q, tp2 = k - h * Q;
        const int c1 = c >> 1, c2 = c & 1;
        cpx<T> acc[H1];
#pragma unroll
        for (int kk = 0; kk < H1; ++kk) acc[kk] = {(T)0, (T)0};
#pragma unroll
        for (int j1 = 0; j1 < 2; ++j1) {
            cpx<T> col[Q];
#pragma unroll
            for (int t1 = 0; t1 < Q; ++t1) col[t1] = Y[bbl][j1][c][t1 * Q + tp2];
#pragma unroll
            for (int kk = 0; kk < H1; ++kk) {
                const int tp1 = min(h * H1 + kk, Q - 1);
#pragma unroll
                for (int t1 = 0; t1 < Q; ++t1) crfma(acc[kk], Ms[j1][tp1][t1], col[t1]);
            }
        }
        cpx<T> *dst = wout + (blk * 4 + c) * QQ;
        const double xa2 = box_node(ap2, level - 1, tb.z[tp2]);
#pragma unroll
        for (int kk = 0; kk < H1; ++kk) {
            const int tp1 = h * H1 + kk;
            if (tp1 < Q) {
                const XP xp = make_xp_sc(ph, box_node(ap1, level - 1, tb.z[tp1]), xa2, sp[bbl][0][tp1],
                                         cp[bbl][0][tp1], sp[bbl][1][tp2], cp[bbl][1][tp2]);
                const double G = phase_dir(xp, ct0[bbl][c2], st0[bbl][c2]);
                dst[tp1 * Q + tp2] = cmul(acc[kk], cis<T>(r0c[bbl][c1] * G));
            }
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
// First pass: thread (j, c2, t1) forms row t1 of E delta for output j and
// contracts it over t2 with M_c2.  Second pass: thread (c, t'2, half)
// contracts over t1 with M_c1, applies conj E(x0(A_j), p^{B_c}_t') and sums j.
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_plevel_adj(Geom g, PhaseDev ph, Tables tb, int level,
                                                   const cpx<T> *__restrict__ win,
                                                   cpx<T> *__restrict__ wout, unsigned nblk) {
    constexpr int QQ = Q * Q;
    constexpr int TPO = 2 * Q;
    constexpr int TPB = 4 * TPO;
    constexpr int BPW = blocks_per_wg<T, Q, 8>();
    constexpr int H1 = (Q + 1) / 2;
    __shared__ T Ms[2][Q][Q];             // Ms[c][t][t'] = M_c[t][t']
    __shared__ double rc[BPW][2 * Q], ctc[BPW][2 * Q], stc[BPW][2 * Q];
    __shared__ double rb[BPW][Q], ctb[BPW][Q], stb[BPW][Q];
    __shared__ double Gc[BPW][4][2 * Q], Gb[BPW][4][Q];
    __shared__ cpx<T> Y[BPW][4][2][QQ];   // [j][c2][t1][t'2]

    const int tid = threadIdx.x;
    const int bbl = tid / TPB, r = tid - bbl * TPB;
    const int j = r / TPO, rr = r - j * TPO;
    const size_t blk = (size_t)blockIdx.x * BPW + bbl;
    const bool active = bbl < BPW && blk < nblk;
    const int lB = g.L - level;
    const size_t nBl = (size_t)1 << (2 * lB);

    const T *Mg = pick_M<T>(tb);
    for (int i = tid; i < 2 * QQ; i += NT) (&Ms[0][0][0])[i] = Mg[i];
    uint32_t mB = 0, mAp = 0;
    int b1 = 0, b2 = 0, ap1 = 0, ap2 = 0;
    if (active) {
        mB = (uint32_t)(blk & (nBl - 1));
        mAp = (uint32_t)(blk >> (2 * lB));
        morton_decode(mB, b1, b2);
        morton_decode(mAp, ap1, ap2);
        if (j == 0) {
            const int c = rr / Q, t = rr - c * Q;
            const double z = tb.z[t];
            rc[bbl][rr] = g.rho_scale * box_node(2 * b1 + c, lB + 1, z);
            double s_, c_;
            sincospi(2.0 * box_node(2 * b2 + c, lB + 1, z), &s_, &c_);
            ctc[bbl][rr] = c_;
            stc[bbl][rr] = s_;
        } else if (j == 1 && rr < Q) {
            const double z = tb.z[rr];
            rb[bbl][rr] = g.rho_scale * box_node(b1, lB, z);
            double s_, c_;
            sincospi(2.0 * box_node(b2, lB, z), &s_, &c_);
            ctb[bbl][rr] = c_;
            stb[bbl][rr] = s_;
        }
    }
    __syncthreads();
    if (active) {
        const int a1 = 2 * ap1 + (j >> 1), a2 = 2 * ap2 + (j & 1);
        const XP xp = make_xp(ph, box_centre(a1, level), box_centre(a2, level));
        Gc[bbl][j][rr] = phase_dir(xp, ctc[bbl][rr], stc[bbl][rr]);
        if (rr < Q) Gb[bbl][j][rr] = phase_dir(xp, ctb[bbl][rr], stb[bbl][rr]);
    }
    __syncthreads();
    if (active) {
        // first pass: thread (j, c2, t1)
        const int c2 = rr / Q, t1 = rr - c2 * Q;
        const cpx<T> *src = win + ((size_t)(4 * mAp + j) * nBl + mB) * QQ + t1 * Q;
        const double rho = rb[bbl][t1];
        cpx<T> acc[Q];
#pragma unroll
        for (int t = 0; t < Q; ++t) acc[t] = {(T)0, (T)0};
#pragma unroll
        for (int t2 = 0; t2 < Q; ++t2) {
            const cpx<T> gv = cmul(src[t2], cis<T>(rho * Gb[bbl][j][t2]));
#pragma unroll
            for (int tp2 = 0; tp2 < Q; ++tp2) crfma(acc[tp2], Ms[c2][t2][tp2], gv);
        }
#pragma unroll
        for (int tp2 = 0; tp2 < Q; ++tp2) Y[bbl][j][c2][t1 * Q + tp2] = acc[tp2];
    }
    __syncthreads();
    if (active) {
        // second pass: thread (c, t'2, half); r = c * 2Q + h * Q + t'2
        const int c = r / (2 * Q), k = r - c * 2 * Q;
        const int h = k / Q, tp2 = k - h * Q;
        const int c1 = c >> 1, c2 = c & 1;
        cpx<T> acc[H1];
#pragma unroll
        for (int kk = 0; kk < H1; ++kk) acc[kk] = {(T)0, (T)0};
#pragma unroll 1
        for (int jj = 0; jj < 4; ++jj) {
            cpx<T> col[Q];
#pragma unroll
            for (int t1 = 0; t1 < Q; ++t1) col[t1] = Y[bbl][jj][c2][t1 * Q + tp2];
            const double G = Gc[bbl][jj][c2 * Q + tp2];
#pragma unroll
            for (int kk = 0; kk < H1; ++kk) {
                const int tp1 = min(h * H1 + kk, Q - 1);
                cpx<T> z = {(T)0, (T)0};
#pragma unroll
                for (int t1 = 0; t1 < Q; ++t1) crfma(z, Ms[c1][t1][tp1], col[t1]);
                const cpx<T> e = cis<T>(rc[bbl][c1 * Q + tp1] * G);
                const cpx<T> add = cmulc(z, e);
                acc[kk].re += add.re;
                acc[kk].im += add.im;
            }
        }
        cpx<T> *dst = wout + (blk * 4 + c) * QQ;
#pragma unroll
        for (int kk = 0; kk < H1; ++kk) {
            const int tp1 = h * H1 + kk;
            if (tp1 < Q) dst[tp1 * Q + tp2] = acc[kk];
        }
    }
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
    {                                                                                                \
        constexpr int BPW = blocks_per_wg<T, Q, 8>();                                                \
        hipLaunchKernelGGL((k_plevel<T, Q>), dim3((nblk + BPW - 1) / BPW), dim3(NT), 0, st, g, ph,   \
                           tb, level, (const cpx<T> *)win, (cpx<T> *)wout, nblk);                    \
    }
    FIO_DISPATCH_Q(g.q, L_PL)
#undef L_PL
    return hipGetLastError();
}

template <typename T>
static hipError_t xlevel_t(const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                           const void *win, void *wout, hipStream_t st) {
    const unsigned nblk = 1u << (2 * g.L - 2);
#define L_XL(Q)                                                                                      \
    {                                                                                                \
        constexpr int BPW = blocks_per_wg<T, Q, 12>();                                               \
        hipLaunchKernelGGL((k_xlevel<T, Q>), dim3((nblk + BPW - 1) / BPW), dim3(NT), 0, st, g, ph,   \
                           tb, level, (const cpx<T> *)win, (cpx<T> *)wout, nblk);                    \
    }
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
    {                                                                                                \
        constexpr int BPW = blocks_per_wg<T, Q, 8>();                                                \
        hipLaunchKernelGGL((k_xlevel_adj<T, Q>), dim3((nblk + BPW - 1) / BPW), dim3(NT), 0, st, g,   \
                           ph, tb, level, (const cpx<T> *)win, (cpx<T> *)wout, nblk);                \
    }
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
    {                                                                                                \
        constexpr int BPW = blocks_per_wg<T, Q, 8>();                                                \
        hipLaunchKernelGGL((k_plevel_adj<T, Q>), dim3((nblk + BPW - 1) / BPW), dim3(NT), 0, st, g,   \
                           ph, tb, level, (const cpx<T> *)win, (cpx<T> *)wout, nblk);                \
    }
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
