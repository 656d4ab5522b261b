// HIP kernels (gfx950) of the forward butterfly pass: the steps of Sec. 4
// (eq:alg2a, eq:alg2b, eq:alg2m, eq:alg2c, eq:alg2d).
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

#include "fio_kernels_common.h"

namespace fio {

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
    lds_barrier();
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
        lds_barrier();
        // kernel values E(x0(A), k) f(k) for this chunk, all A of the workgroup
        for (int it = tid; it < nAc * n; it += NT) {
            const int al = it / n, jj = it - al * n;
            const cpx<T> e = cis<T>(phase_cart(xA[al], kk[jj].x, kk[jj].y));
            gA[al][jj] = cmul(e, fs[jj]);
        }
        lds_barrier();
        if (active) {
            for (int jj = 0; jj < n; ++jj) {
                const cpx<T> gv = gA[aL][jj];
                const T l1 = lag1[jj][t1];
                const cpx<T> h = {l1 * gv.re, l1 * gv.im};
#pragma unroll
                for (int t2 = 0; t2 < Q; ++t2) crfma(acc[t2], lag2[jj][t2], h);
            }
        }
        lds_barrier();
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
// Each output pair gets 2q threads: in the first pass thread (c1, t'1)
// forms its prefactored row of the two children (c1, 0), (c1, 1) in
// registers and contracts it against M_c2 (read as LDS broadcasts); in the
// second pass thread (t2, half) takes column t2 and produces half the rows
// t1, remodulated and stored.
// ===========================================================================
template <typename T, int Q, bool HOIST>
__global__ __launch_bounds__(NT) void k_plevel(Geom g, PhaseDev ph, Tables tb, int level,
                                               const cpx<T> *__restrict__ win,
                                               cpx<T> *__restrict__ wout, unsigned nblk,
                                               int nrhs, size_t plane) {
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
    lds_barrier();
    const int a1 = 2 * ap1 + (j >> 1), a2 = 2 * ap2 + (j & 1);
    if (active) {
        const XP xp = make_xp(ph, box_centre(a1, level), box_centre(a2, level));
        Gc[bbl][j][rr] = phase_dir(xp, ctc[bbl][rr], stc[bbl][rr]);
        if (rr < Q) Gb[bbl][j][rr] = phase_dir(xp, ctb[bbl][rr], stb[bbl][rr]);
    }
    lds_barrier();
    // exponentials of this thread's row (first pass) and column (second
    // pass), shared by all right-hand sides
    const int c1 = rr / Q, tp1 = rr - c1 * Q;
    const int h = rr / Q, t2 = rr - h * Q;
    cpx<T> Ea[2 * Q], Eb[H1];
    const double rhoA = rc[bbl][rr], GB = Gb[bbl][j][t2];
    if constexpr (HOIST) {
        if (active) {
#pragma unroll
            for (int k = 0; k < 2 * Q; ++k) Ea[k] = cis<T>(rhoA * Gc[bbl][j][k]);
#pragma unroll
            for (int k = 0; k < H1; ++k) Eb[k] = cis<T>(rb[bbl][min(h * H1 + k, Q - 1)] * GB);
        }
    }
    // inputs of the thread's row, loaded one right-hand side ahead
    cpx<T> nx[2 * Q];
    auto load_row = [&](int r) {
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2) {
            const cpx<T> *src = win + r * plane + (blk * 4 + 2 * c1 + c2) * QQ + tp1 * Q;
#pragma unroll
            for (int tp2 = 0; tp2 < Q; ++tp2) nx[c2 * Q + tp2] = src[tp2];
        }
    };
    constexpr bool PF = HOIST && !(sizeof(T) == 8 && Q > 10);  // prefetch unless it spills
    if (PF && active) load_row(0);
    for (int r = 0; r < (HOIST ? nrhs : 1); ++r) {
        if (active) {
            if (!PF) load_row(r);
            const cpx<T>(&in)[2 * Q] = nx;
            // first pass: row (c1, t'1)
            cpx<T> acc[Q];
#pragma unroll
            for (int t = 0; t < Q; ++t) acc[t] = {(T)0, (T)0};
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2) {
#pragma unroll
                for (int tp2 = 0; tp2 < Q; ++tp2) {
                    const cpx<T> e = HOIST ? Ea[c2 * Q + tp2] : cis<T>(rhoA * Gc[bbl][j][c2 * Q + tp2]);
                    const cpx<T> v = cmul(e, in[c2 * Q + tp2]);
                    // M_c2[tt][t'2]: the same for every thread, read through the
                    // scalar cache (SGPR operands) rather than as LDS broadcasts
#pragma unroll
                    for (int tt = 0; tt < Q; ++tt) crfma(acc[tt], Mg[(c2 * Q + tt) * Q + tp2], v);
                }
            }
#pragma unroll
            for (int tt = 0; tt < Q; ++tt) W[bbl][j][rr * Q + tt] = acc[tt];
        }
        lds_barrier();
        // the next right-hand side's row is loaded during the second pass, once
        // the first pass has consumed this one
        if (PF && active && r + 1 < nrhs) load_row(r + 1);
        if (active) {
            // second pass: column t2, rows t1 of one half, then remodulation
            cpx<T> col[2 * Q];
#pragma unroll
            for (int k = 0; k < 2 * Q; ++k) col[k] = W[bbl][j][k * Q + t2];
            cpx<T> *dst = wout + r * plane + ((size_t)(4 * mAp + j) * nBl + mB) * QQ;
#pragma unroll
            for (int k = 0; k < H1; ++k) {
                const int t1 = h * H1 + k;
                if (t1 < Q) {
                    cpx<T> o = {(T)0, (T)0};
#pragma unroll
                    for (int cc = 0; cc < 2; ++cc)
#pragma unroll
                        for (int p1 = 0; p1 < Q; ++p1) crfma(o, Ms[cc][t1][p1], col[cc * Q + p1]);
                    dst[t1 * Q + t2] = cmulc(o, HOIST ? Eb[k] : cis<T>(rb[bbl][t1] * GB));
                }
            }
        }
        lds_barrier();
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
template <typename T, int Q, int RC, bool ONE>
__global__ __launch_bounds__(NT) void k_switch(Geom g, PhaseDev ph, Tables tb, cpx<T> *__restrict__ w,
                                               int nrhs, size_t plane) {
    constexpr int QQ = Q * Q;
    constexpr int H = Q / 2;
    constexpr int HH = H > 0 ? H : 1;
    constexpr int PPB = NT / QQ;  // pairs per workgroup
    // pair sums S and differences D, [rc][s2][j] per pair, the pair's block
    // padded by two values: unpadded, the block (RC q floor(q/2) values) is a
    // multiple of the 32 LDS banks at q = 9, and a wave that straddles two
    // pairs reads both pairs' values from one bank; two values (16 bytes) keep
    // the 16-byte alignment that lets S_j, S_j+1 load as one 128-bit read
    constexpr int SDB = RC * Q * HH + 2;
    __shared__ cpx<T> Sx[PPB][SDB];
    __shared__ cpx<T> Dx[PPB][SDB];
    __shared__ cpx<T> Mid[PPB][RC][Q];
    __shared__ double cth[PPB][Q], sth[PPB][Q];
    __shared__ double rho0[PPB], hz[PPB][HH];

    const int tid = threadIdx.x;
    const int pl = tid / QQ, t = tid - pl * QQ;
    const size_t npairs = (size_t)1 << (2 * g.L);
    const size_t pair = linear_block() * PPB + pl;
    const bool active = (pl < PPB) && (pair < npairs);
    const int lA = g.lm, lB = g.L - g.lm;
    const size_t nBl = (size_t)1 << (2 * lB);
    const uint32_t mB = active ? (uint32_t)(pair & (nBl - 1)) : 0;
    const uint32_t mA = active ? (uint32_t)(pair >> (2 * lB)) : 0;
    int b1, b2, a1, a2;
    morton_decode(mB, b1, b2);
    morton_decode(mA, a1, a2);
    const int t1 = t / Q, t2 = t - t1 * Q;

    if (active) {
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
    XP xp{};
    if (active) xp = make_xp(ph, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]));

    for (int r0 = 0; r0 < (ONE ? 1 : nrhs); r0 += RC) {
        const int nr = min(RC, nrhs - r0);
        lds_barrier();
        // pair sums / differences of rows j and q-1-j (thread (t1, t2): t1 plays j)
        if (active) {
            for (int rc = 0; rc < nr; ++rc) {
                const cpx<T> *wp = w + (size_t)(r0 + rc) * plane + pair * QQ;
                if (t1 < H) {
                    const cpx<T> a = wp[t1 * Q + t2], b = wp[(Q - 1 - t1) * Q + t2];
                    Sx[pl][(rc * Q + t2) * HH + t1] = {a.re + b.re, a.im + b.im};
                    Dx[pl][(rc * Q + t2) * HH + t1] = {a.re - b.re, a.im - b.im};
                } else if ((Q & 1) && t1 == H) {
                    Mid[pl][rc][t2] = wp[H * Q + t2];
                }
            }
        }
        lds_barrier();
        if (!active) continue;
        const double r0v = rho0[pl];
        cpx<T> acc[RC];
#pragma unroll
        for (int rc = 0; rc < RC; ++rc) acc[rc] = {(T)0, (T)0};
        for (int s2 = 0; s2 < Q; ++s2) {
            const double G = phase_dir(xp, cth[pl][s2], sth[pl][s2]);
            const cpx<T> base = cis<T>(r0v * G);
            cpx<T> d[HH];
#pragma unroll
            for (int j = 0; j < H; ++j) d[j] = cis<T>(hz[pl][j] * G);
#pragma unroll
            for (int rc = 0; rc < RC; ++rc) {
                if (rc < nr) {
                    cpx<T> inner = (Q & 1) ? Mid[pl][rc][s2] : cpx<T>{(T)0, (T)0};
#pragma unroll
                    for (int j = 0; j < H; ++j) {
                        const cpx<T> S = Sx[pl][(rc * Q + s2) * HH + j], D = Dx[pl][(rc * Q + s2) * HH + j];
                        inner.re = fma(d[j].re, S.re, fma(-d[j].im, D.im, inner.re));
                        inner.im = fma(d[j].re, S.im, fma(d[j].im, D.re, inner.im));
                    }
                    cfma(acc[rc], base, inner);
                }
            }
        }
#pragma unroll
        for (int rc = 0; rc < RC; ++rc)
            if (rc < nr) w[(size_t)(r0 + rc) * plane + pair * QQ + t] = acc[rc];
    }
}

// ===========================================================================
// Step 5, x-recursion (eq:alg2c) at level l: block (A_p at l-1, B at L-l)
//   delta^{AB}_t = sum_c E(x^A_t, p0(B_c)) sum_t' M_a1[t'1][t1] M_a2[t'2][t2]
//                    conj E(x^{A_p}_t', p0(B_c)) delta^{A_p B_c}_t'
// for the four children A = (a1, a2) of A_p.  The prefactor depends only on
// (A_p, B_c); the first (second-dimension) pass depends on A only through
// a2, so it is shared by the children with the same a2.  Threads: first pass
// (a2, c, t'1) rows; second pass (A, t2, half) columns with the remodulation
// per B_c.  One right-hand side: the prefactor is applied once per row
// (c, t'1) in a phase of its own.  Several: every first-pass thread applies
// its row's prefactor itself (kernel values hoisted for all right-hand
// sides), which saves a barrier per right-hand side.
// ===========================================================================
template <typename T, int Q, bool HOIST>
__global__ __launch_bounds__(NT) void k_xlevel(Geom g, PhaseDev ph, Tables tb, int level,
                                               const cpx<T> *__restrict__ win,
                                               cpx<T> *__restrict__ wout, unsigned nblk,
                                               int nrhs, size_t plane) {
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
    lds_barrier();
    // exponentials shared by all right-hand sides: the prefactor row (c, t'1)
    // of threads rr < 4q, and the remodulation E(x^A_t, p0(B_c)) of the
    // second-pass column (A, t2, half) of every thread
    const int pc = rr / Q, ptp1 = rr - pc * Q;          // prefactor row (rr < 4q)
    const int a2c = rr / (4 * Q), ak = rr - a2c * 4 * Q;
    const int ac = ak / Q, atp1 = ak - ac * Q;          // first-pass row
    const int jj = rr / (2 * Q), bk = rr - jj * 2 * Q;
    const int h = bk / Q, t2 = bk - h * Q;              // second-pass column
    const int j1 = jj >> 1, j2 = jj & 1;
    cpx<T> Ep[Q], E2[4][H1];
    auto pre_exp = [&](int tp2) -> cpx<T> {
        const int c2 = pc & 1, c1 = pc >> 1;
        const XP xp = make_xp_sc(ph, box_node(ap1, level - 1, tb.z[ptp1]), box_node(ap2, level - 1, tb.z[tp2]),
                                 sp[bbl][0][ptp1], cp[bbl][0][ptp1], sp[bbl][1][tp2], cp[bbl][1][tp2]);
        return cis<T>(r0c[bbl][c1] * phase_dir(xp, ct0[bbl][c2], st0[bbl][c2]));
    };
    // batched first pass: the child's a2 is the same for a pair of waves
    // (threads [128 a2, 128 a2 + 128)), row (block, c, t'1) within it, so the
    // factors M_a2[t'2][t2] are wave-uniform (scalar operands)
    // (fa2 is uniform over the wave: make that explicit for the compiler)
    const int fa2 = __builtin_amdgcn_readfirstlane(tid / (NT / 2)), fi = tid - fa2 * (NT / 2);
    const int fb = fi / (4 * Q), fk = fi - fb * (4 * Q), fac = fk / Q, fatp1 = fk - fac * Q;
    const size_t fblk = (size_t)blockIdx.x * BPW + fb;
    const bool factive = fb < BPW && fblk < nblk;
    int fap1 = 0, fap2 = 0;
    if (factive) morton_decode((uint32_t)(fblk >> (2 * lB)), fap1, fap2);
    if (HOIST && factive) {
        // every first-pass thread applies the prefactor of its own row (c, t'1)
        const int c2 = fac & 1, c1 = fac >> 1;
        const double xa1 = box_node(fap1, level - 1, tb.z[fatp1]);
#pragma unroll
        for (int tp2 = 0; tp2 < Q; ++tp2) {
            const XP xp = make_xp_sc(ph, xa1, box_node(fap2, level - 1, tb.z[tp2]), sp[fb][0][fatp1],
                                     cp[fb][0][fatp1], sp[fb][1][tp2], cp[fb][1][tp2]);
            Ep[tp2] = cis<T>(r0c[fb][c1] * phase_dir(xp, ct0[fb][c2], st0[fb][c2]));
        }
    }
    if (HOIST && active) {
        const int a1 = 2 * ap1 + j1, a2 = 2 * ap2 + j2;
        const double xb2 = box_node(a2, level, tb.z[t2]);
#pragma unroll
        for (int kk = 0; kk < H1; ++kk) {
            const int t1 = min(h * H1 + kk, Q - 1);
            const XP xp = make_xp_sc(ph, box_node(a1, level, tb.z[t1]), xb2, sj[bbl][0][j1][t1],
                                     cj[bbl][0][j1][t1], sj[bbl][1][j2][t2], cj[bbl][1][j2][t2]);
            const double G0 = phase_dir(xp, ct0[bbl][0], st0[bbl][0]);
            const double G1 = phase_dir(xp, ct0[bbl][1], st0[bbl][1]);
            E2[0][kk] = cis<T>(r0c[bbl][0] * G0);
            E2[1][kk] = cis<T>(r0c[bbl][0] * G1);
            E2[2][kk] = cis<T>(r0c[bbl][1] * G0);
            E2[3][kk] = cis<T>(r0c[bbl][1] * G1);
        }
    }
    if constexpr (HOIST) {
        // inputs of the first-pass row, loaded one right-hand side ahead, during
        // the second pass (issuing it before the first pass measured slower)
        cpx<T> nx[Q];
        auto load_row = [&](int r) {
            const cpx<T> *src = win + r * plane + (fblk * 4 + fac) * QQ + fatp1 * Q;
#pragma unroll
            for (int tp2 = 0; tp2 < Q; ++tp2) nx[tp2] = src[tp2];
        };
        if (factive) load_row(0);
        for (int r = 0; r < nrhs; ++r) {
            // first pass with the prefactor: Y[a2][c][t'1][t2] =
            //   sum_t'2 M_a2[t'2][t2] conj E(x^{A_p}_t', p0(B_c)) delta^{A_p B_c}_t'
            if (factive) {
                cpx<T> acc[Q];
#pragma unroll
                for (int t = 0; t < Q; ++t) acc[t] = {(T)0, (T)0};
#pragma unroll
                for (int tp2 = 0; tp2 < Q; ++tp2) {
                    const cpx<T> vv = cmulc(nx[tp2], Ep[tp2]);
#pragma unroll
                    for (int tt = 0; tt < Q; ++tt) crfma(acc[tt], Mg[(fa2 * Q + tp2) * Q + tt], vv);
                }
#pragma unroll
                for (int tt = 0; tt < Q; ++tt) Y[fb][fa2][fac][fatp1 * Q + tt] = acc[tt];
            }
            lds_barrier();
            if (factive && r + 1 < nrhs) load_row(r + 1);
            if (active) {
                cpx<T> out[H1];
#pragma unroll
                for (int kk = 0; kk < H1; ++kk) out[kk] = {(T)0, (T)0};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    cpx<T> col[Q];
#pragma unroll
                    for (int tp1 = 0; tp1 < Q; ++tp1) col[tp1] = Y[bbl][j2][c][tp1 * Q + t2];
#pragma unroll
                    for (int kk = 0; kk < H1; ++kk) {
                        const int t1 = min(h * H1 + kk, Q - 1);
                        cpx<T> z = {(T)0, (T)0};
#pragma unroll
                        for (int tp1 = 0; tp1 < Q; ++tp1) crfma(z, Ms[j1][tp1][t1], col[tp1]);
                        cfma(out[kk], E2[c][kk], z);
                    }
                }
                cpx<T> *dst = wout + r * plane + ((size_t)(4 * mAp + jj) * nBl + mB) * QQ;
#pragma unroll
                for (int kk = 0; kk < H1; ++kk) {
                    const int t1 = h * H1 + kk;
                    if (t1 < Q) dst[t1 * Q + t2] = out[kk];
                }
            }
            lds_barrier();
        }
        return;
    }
    // one right-hand side: prefactor conj E(x^{A_p}_t', p0(B_c)) delta^{A_p B_c}_t'
    // once per row (c, t'1)
    if (active && rr < 4 * Q) {
        const cpx<T> *src = win + (blk * 4 + pc) * QQ + ptp1 * Q;
#pragma unroll
        for (int tp2 = 0; tp2 < Q; ++tp2) v[bbl][pc][ptp1 * Q + tp2] = cmulc(src[tp2], pre_exp(tp2));
    }
    lds_barrier();
    // first pass (second dimension): Y[a2][c][t'1][t2] = sum_t'2 M_a2[t'2][t2] v[c][t'1][t'2]
    if (active) {
        cpx<T> acc[Q];
#pragma unroll
        for (int t = 0; t < Q; ++t) acc[t] = {(T)0, (T)0};
#pragma unroll
        for (int tp2 = 0; tp2 < Q; ++tp2) {
            const cpx<T> vv = v[bbl][ac][atp1 * Q + tp2];
#pragma unroll
            for (int tt = 0; tt < Q; ++tt) crfma(acc[tt], Ms[a2c][tp2][tt], vv);
        }
#pragma unroll
        for (int tt = 0; tt < Q; ++tt) Y[bbl][a2c][ac][atp1 * Q + tt] = acc[tt];
    }
    lds_barrier();
    // second pass (first dimension), remodulation E(x^A_t, p0(B_c)), sum over c
    if (active) {
        cpx<T> out[H1];
        const int a1 = 2 * ap1 + j1, a2 = 2 * ap2 + j2;
        double G0[H1], G1[H1];
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
        lds_barrier();
        // prefactor conj E(x^A_t, p0(B)) delta^{AB}_t
        for (int i = tid; i < nb * QQ; i += NT) {
            const int b = i / QQ, t = i - b * QQ;
            const int t1 = t / Q, t2 = t - t1 * Q;
            const XP xp = make_xp_sc(ph, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]),
                                     sx1[t1], cx1[t1], sx2[t2], cx2[t2]);
            const cpx<T> e = cis<T>(r0b[b] * phase_dir(xp, ctb[b], stb[b]));
            v[i] = cmulc(src[(size_t)(b0 + b) * QQ + t], e);
        }
        lds_barrier();
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
        lds_barrier();
        // pass 2 (first dimension) and the factor E(x, p0(B)), summed per grid point
        for (int i = tid; i < nb * np; i += NT) {
            const int b = i / np;  // i % np == jp since NT % np == 0
            cpx<T> acc = {(T)0, (T)0};
            const cpx<T> *yy = Y + b * Q * m + j2;
#pragma unroll
            for (int t1 = 0; t1 < Q; ++t1) crfma(acc, Tt[j1 * Q + t1], yy[t1 * m]);
            cfma(uacc, cis<T>(r0b[b] * phase_dir(xg, ctb[b], stb[b])), acc);
        }
        lds_barrier();
    }
    red[tid] = uacc;
    lds_barrier();
    if (tid < np) {
        cpx<T> sum = red[tid];
        for (int k = tid + np; k < NT; k += np) {
            sum.re += red[k].re;
            sum.im += red[k].im;
        }
        u[(size_t)(a1 * m + j1) * g.N + (a2 * m + j2)] = sum;
    }
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
                           const void *win, void *wout, int nrhs, size_t plane, hipStream_t st) {
    const unsigned nblk = 1u << (2 * g.L - 2);
#define L_PL(Q)                                                                                      \
    {                                                                                                \
        constexpr int BPW = blocks_per_wg<T, Q, 8>();                                                \
        const dim3 grid((nblk + BPW - 1) / BPW);                                                     \
        if (nrhs == 1)                                                                               \
            hipLaunchKernelGGL((k_plevel<T, Q, false>), grid, dim3(NT), 0, st, g, ph, tb, level,     \
                               (const cpx<T> *)win, (cpx<T> *)wout, nblk, nrhs, plane);              \
        else                                                                                         \
            hipLaunchKernelGGL((k_plevel<T, Q, true>), grid, dim3(NT), 0, st, g, ph, tb, level,      \
                               (const cpx<T> *)win, (cpx<T> *)wout, nblk, nrhs, plane);              \
    }
    FIO_DISPATCH_Q(g.q, L_PL)
#undef L_PL
    return hipGetLastError();
}

template <typename T>
static hipError_t xlevel_t(const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                           const void *win, void *wout, int nrhs, size_t plane, hipStream_t st) {
    const unsigned nblk = 1u << (2 * g.L - 2);
#define L_XL(Q)                                                                                      \
    {                                                                                                \
        constexpr int BPW = blocks_per_wg<T, Q, 12>();                                               \
        const dim3 grid((nblk + BPW - 1) / BPW);                                                     \
        if (nrhs == 1)                                                                               \
            hipLaunchKernelGGL((k_xlevel<T, Q, false>), grid, dim3(NT), 0, st, g, ph, tb, level,     \
                               (const cpx<T> *)win, (cpx<T> *)wout, nblk, nrhs, plane);              \
        else                                                                                         \
            hipLaunchKernelGGL((k_xlevel<T, Q, true>), grid, dim3(NT), 0, st, g, ph, tb, level,      \
                               (const cpx<T> *)win, (cpx<T> *)wout, nblk, nrhs, plane);              \
    }
    FIO_DISPATCH_Q(g.q, L_XL)
#undef L_XL
    return hipGetLastError();
}

template <typename T>
static hipError_t switch_t(const Geom &g, const PhaseDev &ph, const Tables &tb, void *w, int nrhs, size_t plane,
                           hipStream_t st) {
    if (sizeof(T) == 4 && switch_mfma_supported(g.q, nrhs)) return launch_switch_mfma(g, ph, tb, w, nrhs, plane, st);
    const size_t npairs = (size_t)1 << (2 * g.L);
#define L_SW(Q)                                                                                      \
    {                                                                                                \
        constexpr int PPB = NT / (Q * Q);                                                            \
        const unsigned nblk = (unsigned)((npairs + PPB - 1) / PPB);                                  \
        if (nrhs == 1)                                                                               \
            hipLaunchKernelGGL((k_switch<T, Q, 1, true>), grid_of(nblk), dim3(NT), 0, st, g, ph, tb, \
                               (cpx<T> *)w, nrhs, plane);                                            \
        else                                                                                         \
            hipLaunchKernelGGL((k_switch<T, Q, switch_rc<T>(), false>), grid_of(nblk), dim3(NT), 0,  \
                               st, g, ph, tb, (cpx<T> *)w, nrhs, plane);                             \
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

hipError_t launch_init(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, const Sources &src,
                       const void *f, void *w, hipStream_t st) {
#define C(T) init_t<T>(g, ph, tb, src, f, w, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_plevel(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                         const void *win, void *wout, int nrhs, size_t plane, hipStream_t st) {
#define C(T) plevel_t<T>(g, ph, tb, level, win, wout, nrhs, plane, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_switch(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, void *w, int nrhs,
                         size_t plane, hipStream_t st) {
#define C(T) switch_t<T>(g, ph, tb, w, nrhs, plane, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_xlevel(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                         const void *win, void *wout, int nrhs, size_t plane, hipStream_t st) {
#define C(T) xlevel_t<T>(g, ph, tb, level, win, wout, nrhs, plane, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_term(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, const void *win,
                       void *u, hipStream_t st) {
#define C(T) term_t<T>(g, ph, tb, win, u, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
}  // namespace fio
