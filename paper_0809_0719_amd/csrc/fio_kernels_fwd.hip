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
// children B_c is done one dimension at a time (Sec. 4), each 1-D pass
// summing two children: with M_1 = J M_0 J (the nodes are symmetric),
//   M_0 u + M_1 y = S (u + J y) + A (u - J y),
// S and A the symmetric and antisymmetric halves of M_0 by rows, whose rows
// n and q-1-n agree up to sign -- so P = S_n . a and D = A_n . b give both
// outputs n (P + D) and q-1-n (P - D): q MACs per output instead of 2q.
// First pass: thread (block, j, c1, t'1) forms its prefactored row of the
// two children (c1, 0), (c1, 1) in registers and contracts it against S
// and A.  Second pass: thread (h, block, j, t2) takes column t2 of output j
// and the row pairs n = h, h + 2, ...; h is the same for a half of the
// workgroup (two waves), so in both passes the factors are wave-uniform
// (SGPR operands through the scalar cache).
// ===========================================================================
template <typename T, int Q, bool HOIST>
__global__ __launch_bounds__(NT) void k_plevel(Geom g, PhaseDev ph, Tables tb, int level,
                                               const cpx<T> *__restrict__ win,
                                               cpx<T> *__restrict__ wout, unsigned nblk,
                                               int nrhs, size_t plane) {
    constexpr int QQ = Q * Q;
    constexpr int TPO = 2 * Q;            // first-pass threads per output pair
    constexpr int TPB = 4 * TPO;          // first-pass threads per butterfly block
    constexpr int BPW = blocks_per_wg<T, Q, 8>();
    static_assert(BPW * 4 * Q <= NT / 2, "second pass: a block's columns fit a half workgroup");
    constexpr int H1 = (Q + 1) / 2, H = Q / 2;
    constexpr int NK = (H1 + 1) / 2;      // row pairs per second-pass thread
    __shared__ double rc[BPW][2 * Q], ctc[BPW][2 * Q], stc[BPW][2 * Q];  // child nodes: rho(c1,t'), theta(c2,t')
    __shared__ double rb[BPW][Q], ctb[BPW][Q], stb[BPW][Q];              // B's nodes
    __shared__ double Gc[BPW][4][2 * Q], Gb[BPW][4][Q];
    constexpr int WJ = 2 * QQ + pad_plevel<T, Q>();
    __shared__ cpx<T> W[BPW][4][WJ];      // first-pass rows [c1][t'1][t2] (+ bank padding)
    constexpr int NE = BPW * 4 * QQ;      // the workgroup's inputs: BPW blocks x 4 children, contiguous
    __shared__ cpx<T> xin[stage_len<NE>()];

    const int tid = threadIdx.x;
    const int bbl = tid / TPB, r = tid - bbl * TPB;
    const int j = r / TPO, rr = r - j * TPO;
    const size_t blk = (size_t)blockIdx.x * BPW + bbl;
    const bool active = bbl < BPW && blk < nblk;
    const int lB = g.L - level;
    const size_t nBl = (size_t)1 << (2 * lB);
    cptr<T> SAg = to_constant(pick_SA<T>(tb));
    // inputs staged through LDS one right-hand side ahead
    cpx<T> stv[stage_per<NE>()];
    auto piece = [&](int e) __attribute__((always_inline)) {
        return (size_t)blockIdx.x * BPW + e / (4 * QQ) < nblk ? (size_t)blockIdx.x * NE + e : (size_t)0;
    };

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
    stage_fetch<NE>(stv, win, piece);  // after the node tables (their sine/cosine calls would save it to scratch)
    const int a1 = 2 * ap1 + (j >> 1), a2 = 2 * ap2 + (j & 1);
    if (active) {
        const XP xp = make_xp(ph, box_centre(a1, level), box_centre(a2, level));
        Gc[bbl][j][rr] = phase_dir(xp, ctc[bbl][rr], stc[bbl][rr]);
        if (rr < Q) Gb[bbl][j][rr] = phase_dir(xp, ctb[bbl][rr], stb[bbl][rr]);
    }
    stage_put<NE>(stv, xin);
    lds_barrier();
    // first-pass row (c1, t'1)
    const int c1 = rr / Q, tp1 = rr - c1 * Q;
    const double rhoA = rc[bbl][rr];
    // second-pass column: (h, block sb, output sj, column st2)
    const int h = __builtin_amdgcn_readfirstlane(tid / (NT / 2));
    const int si = tid - h * (NT / 2);
    const int sb = si / (4 * Q), sk = si - sb * (4 * Q), sj = sk / Q, st2 = sk - sj * Q;
    const size_t sblk = (size_t)blockIdx.x * BPW + sb;
    const bool sactive = sb < BPW && sblk < nblk;
    const double GB = sactive ? Gb[sb][sj][st2] : 0.0;
    // exponentials of the first-pass row and of the second-pass rows, shared
    // by all right-hand sides
    cpx<T> Ea[2 * Q], Eb[2 * NK];
    if constexpr (HOIST) {
        if (active) {
#pragma unroll
            for (int k = 0; k < 2 * Q; ++k) Ea[k] = cis<T>(rhoA * Gc[bbl][j][k]);
        }
        if (sactive) {
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const int n = min(h + 2 * k, H1 - 1);
                Eb[2 * k] = cis<T>(rb[sb][n] * GB);
                Eb[2 * k + 1] = cis<T>(rb[sb][Q - 1 - n] * GB);
            }
        }
    }
    cpx<T> *const dst0 = wout + ((size_t)(4 * (sblk >> (2 * lB)) + sj) * nBl + (sblk & (nBl - 1))) * QQ;
    const cpx<T> *const in = &xin[(bbl * 4 + 2 * c1) * QQ + tp1 * Q];  // row of child (c1, 0); + QQ: (c1, 1)
    for (int r = 0; r < (HOIST ? nrhs : 1); ++r) {
        opaque_sgpr(SAg);
        if (active) {
            // first pass: row (c1, t'1); a = v_0 + J v_1, b = v_0 - J v_1
            cpx<T> P[H1], D[H > 0 ? H : 1];
#pragma unroll
            for (int n = 0; n < H1; ++n) P[n] = {(T)0, (T)0};
#pragma unroll
            for (int n = 0; n < H; ++n) D[n] = {(T)0, (T)0};
#pragma unroll
            for (int m = 0; m < Q; ++m) {
                const cpx<T> e0 = HOIST ? Ea[m] : cis<T>(rhoA * Gc[bbl][j][m]);
                const cpx<T> e1 = HOIST ? Ea[2 * Q - 1 - m] : cis<T>(rhoA * Gc[bbl][j][2 * Q - 1 - m]);
                const cpx<T> v0 = cmul(e0, in[m]);
                const cpx<T> v1 = cmul(e1, in[QQ + Q - 1 - m]);
                const cpx<T> av = {v0.re + v1.re, v0.im + v1.im};
                const cpx<T> bv = {v0.re - v1.re, v0.im - v1.im};
#pragma unroll
                for (int n = 0; n < H1; ++n) crfma(P[n], SAg[n * Q + m], av);
#pragma unroll
                for (int n = 0; n < H; ++n) crfma(D[n], SAg[QQ + n * Q + m], bv);
            }
            cpx<T> *wr = &W[bbl][j][rr * Q];
#pragma unroll
            for (int n = 0; n < H; ++n) {
                wr[n] = {P[n].re + D[n].re, P[n].im + D[n].im};
                wr[Q - 1 - n] = {P[n].re - D[n].re, P[n].im - D[n].im};
            }
            if constexpr (Q & 1) wr[H] = P[H];
        }
        lds_barrier();
        // the next right-hand side's inputs are loaded during the second pass
        // and staged once it is done (the first pass has consumed this one's)
        // (unconditionally: the last one refetches the last right-hand side,
        // which keeps the staged values in registers rather than in scratch)
        if (HOIST) stage_fetch<NE>(stv, win + (size_t)min(r + 1, nrhs - 1) * plane, piece);
        if (sactive) with_uniform<0, 2>(h, [&](auto hc) __attribute__((always_inline)) {
            constexpr int hh = decltype(hc)::value;
            // second pass: column st2 over c1 (a = W_0 + J W_1, b = W_0 - J W_1),
            // row pairs n = hh + 2k, then remodulation
            cpx<T> Pn[NK], Dn[NK];
#pragma unroll
            for (int k = 0; k < NK; ++k) Pn[k] = Dn[k] = {(T)0, (T)0};
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                const cpx<T> x0 = W[sb][sj][p * Q + st2], x1 = W[sb][sj][(2 * Q - 1 - p) * Q + st2];
                const cpx<T> av = {x0.re + x1.re, x0.im + x1.im};
                const cpx<T> bv = {x0.re - x1.re, x0.im - x1.im};
#pragma unroll
                for (int k = 0; k < NK; ++k) {
                    constexpr int n0 = hh;
                    const int n = n0 + 2 * k;
                    if (n < H1) {
                        crfma(Pn[k], SAg[n * Q + p], av);
                        if (n < H) crfma(Dn[k], SAg[QQ + n * Q + p], bv);
                    }
                }
            }
            cpx<T> *dst = dst0 + r * plane;
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const int n = hh + 2 * k;
                if (n < H1) {
                    const cpx<T> o0 = {Pn[k].re + Dn[k].re, Pn[k].im + Dn[k].im};
                    dst[n * Q + st2] = cmulc(o0, HOIST ? Eb[2 * k] : cis<T>(rb[sb][n] * GB));
                    if (n < H) {
                        const cpx<T> o1 = {Pn[k].re - Dn[k].re, Pn[k].im - Dn[k].im};
                        dst[(Q - 1 - n) * Q + st2] =
                            cmulc(o1, HOIST ? Eb[2 * k + 1] : cis<T>(rb[sb][Q - 1 - n] * GB));
                    }
                }
            }
        });
        if (HOIST) stage_put<NE>(stv, xin);
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
// (A_p, B_c).  Each 1-D pass feeds one input to two children (a = 0, 1):
// with M_1 = J M_0 J, (M_1^T v)[q-1-n] = (M_0^T J v)[n], so splitting v into
// s = v + J v and d = v - J v (first half) gives P = ST_n . s and
// D = AT_n . d with (M_0^T v)[n] = P + D and (M_1^T v)[q-1-n] = P - D:
// q MACs for two outputs instead of 2q.
// First pass (second dimension): thread (h, block, c, t'1) forms the
// prefactored row (c, t'1) and produces the outputs n = h H1 + k of child
// a2 = 0 and q-1-n of a2 = 1; h is the same for two waves.  Second pass
// (first dimension): thread (g, block, a2, t2), g the wave, takes column t2
// of the first-pass rows of a2, produces rows n = g, g + 4, ... of child
// a1 = 0 and q-1-n of a1 = 1, remodulates by E(x^A_t, p0(B_c)) and sums
// over c.  The factors are wave-uniform in both passes (SGPR operands).
// One right-hand side: the prefactor is applied once per row (c, t'1) in a
// phase of its own.  Several: every first-pass thread applies its row's
// prefactor itself (kernel values hoisted for all right-hand sides), which
// saves a barrier per right-hand side.
// ===========================================================================
template <typename T, int Q, bool HOIST>
__global__ __launch_bounds__(NT) void k_xlevel(Geom g, PhaseDev ph, Tables tb, int level,
                                               const cpx<T> *__restrict__ win,
                                               cpx<T> *__restrict__ wout, unsigned nblk,
                                               int nrhs, size_t plane) {
    constexpr int QQ = Q * Q;
    constexpr int TPB = 8 * Q;
    constexpr int BPW = blocks_per_wg<T, Q, 12>();
    static_assert(BPW * 4 * Q <= NT / 2 && BPW * 2 * Q <= 64, "pass layouts fit the workgroup");
    constexpr int H1 = (Q + 1) / 2, H = Q / 2;
    constexpr int NG = (Q + 3) / 4;                 // second-pass rows per thread
    constexpr int NE = BPW * 4 * QQ;                // the workgroup's inputs: BPW blocks x 4 children, contiguous
    __shared__ cpx<T> xin[stage_len<NE>()];         // inputs (several RHS) or prefactored inputs (one)
    constexpr int YA = 4 * QQ + pad_sum_out<T, Q>();
    __shared__ cpx<T> Y[BPW][2][YA];                // first pass [a2][c][t'1][t2] (+ bank padding)
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
    cptr<T> SAg = to_constant(pick_SA<T>(tb));
    cptr<T> STg = SAg + 2 * QQ, ATg = SAg + 3 * QQ;  // re-derived per right-hand side

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
    // first pass: thread (fh, block fb, c fac, row fatp1); fh uniform over two waves
    const int fh = __builtin_amdgcn_readfirstlane(tid / (NT / 2)), fi = tid - fh * (NT / 2);
    const int fb = fi / (4 * Q), fk = fi - fb * (4 * Q), fac = fk / Q, fatp1 = fk - fac * Q;
    const size_t fblk = (size_t)blockIdx.x * BPW + fb;
    const bool factive = fb < BPW && fblk < nblk;
    int fap1 = 0, fap2 = 0;
    if (factive) morton_decode((uint32_t)(fblk >> (2 * lB)), fap1, fap2);
    // second pass: thread (wave sg, block sb, a2 sj2, column st2)
    const int sg = __builtin_amdgcn_readfirstlane(tid / 64), sl = tid & 63;
    const int sb = sl / (2 * Q), sk = sl - sb * (2 * Q), sj2 = sk / Q, st2 = sk - sj2 * Q;
    const size_t sblk = (size_t)blockIdx.x * BPW + sb;
    const bool sactive = sb < BPW && sblk < nblk;
    int sap1 = 0, sap2 = 0;
    if (sactive) morton_decode((uint32_t)(sblk >> (2 * lB)), sap1, sap2);
    // remodulation phases of this thread's outputs: (a1 = 0, row n), (a1 = 1, row q-1-n)
    // for n = sg + 4k, against theta0(B_c2); G[c2][2k + side]
    auto out_row = [&](int k, int side) __attribute__((always_inline)) {
        const int n = min(sg + 4 * k, Q - 1);
        return side ? Q - 1 - n : n;
    };
    auto remod_phase = [&](int k, int side, int c2) __attribute__((always_inline)) {
        const int a1 = 2 * sap1 + side, a2 = 2 * sap2 + sj2, t1 = out_row(k, side);
        const XP xp = make_xp_sc(ph, box_node(a1, level, tb.z[t1]), box_node(a2, level, tb.z[st2]),
                                 sj[sb][0][side][t1], cj[sb][0][side][t1], sj[sb][1][sj2][st2],
                                 cj[sb][1][sj2][st2]);
        return phase_dir(xp, ct0[sb][c2], st0[sb][c2]);
    };
    cpx<T> *const dst0 = wout + ((size_t)(4 * (sblk >> (2 * lB)) + sj2) * nBl + (sblk & (nBl - 1))) * QQ;
    cpx<T> *const dst1 = dst0 + 2 * nBl * QQ;  // child (1, a2)

    // first pass on the prefactored row vv (both children a2)
    auto first_pass = [&](const cpx<T> (&vv)[Q]) __attribute__((always_inline)) {
        with_uniform<0, 2>(fh, [&](auto hc) __attribute__((always_inline)) {
        constexpr int fhh = decltype(hc)::value;
        cpx<T> sv[H1], dv[H > 0 ? H : 1];
#pragma unroll
        for (int m = 0; m < H; ++m) {
            sv[m] = {vv[m].re + vv[Q - 1 - m].re, vv[m].im + vv[Q - 1 - m].im};
            dv[m] = {vv[m].re - vv[Q - 1 - m].re, vv[m].im - vv[Q - 1 - m].im};
        }
        if constexpr (Q & 1) sv[H] = vv[H];
#pragma unroll
        for (int k = 0; k < H1; ++k) {
            const int n = fhh * H1 + k;
            if (n < Q) {
                cpx<T> P = {(T)0, (T)0}, D = {(T)0, (T)0};
#pragma unroll
                for (int m = 0; m < H1; ++m) crfma(P, STg[n * Q + m], sv[m]);
#pragma unroll
                for (int m = 0; m < H; ++m) crfma(D, ATg[n * Q + m], dv[m]);
                Y[fb][0][fac * QQ + fatp1 * Q + n] = {P.re + D.re, P.im + D.im};
                Y[fb][1][fac * QQ + fatp1 * Q + Q - 1 - n] = {P.re - D.re, P.im - D.im};
            }
        }
        });
    };
    // second pass for one c, accumulated into out[2k + side]
    auto second_pass_c = [&](auto gc, int c, cpx<T> (&z)[2 * NG]) __attribute__((always_inline)) {
        constexpr int gg = decltype(gc)::value;
        cpx<T> sv[H1], dv[H > 0 ? H : 1];
        const cpx<T> *col = &Y[sb][sj2][c * QQ + st2];
#pragma unroll
        for (int m = 0; m < H; ++m) {
            const cpx<T> x0 = col[m * Q], x1 = col[(Q - 1 - m) * Q];
            sv[m] = {x0.re + x1.re, x0.im + x1.im};
            dv[m] = {x0.re - x1.re, x0.im - x1.im};
        }
        if constexpr (Q & 1) sv[H] = col[H * Q];
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const int n = gg + 4 * k;
            z[2 * k] = z[2 * k + 1] = {(T)0, (T)0};
            if (n < Q) {
                cpx<T> P = {(T)0, (T)0}, D = {(T)0, (T)0};
#pragma unroll
                for (int m = 0; m < H1; ++m) crfma(P, STg[n * Q + m], sv[m]);
#pragma unroll
                for (int m = 0; m < H; ++m) crfma(D, ATg[n * Q + m], dv[m]);
                z[2 * k] = {P.re + D.re, P.im + D.im};
                z[2 * k + 1] = {P.re - D.re, P.im - D.im};
            }
        }
    };
    auto store_outputs = [&](auto gc, const cpx<T> (&out)[2 * NG], size_t off) __attribute__((always_inline)) {
        constexpr int gg = decltype(gc)::value;
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const int n = gg + 4 * k;
            if (n < Q) {
                dst0[off + n * Q + st2] = out[2 * k];
                dst1[off + (Q - 1 - n) * Q + st2] = out[2 * k + 1];
            }
        }
    };

    if constexpr (HOIST) {
        cpx<T> stv[stage_per<NE>()];
        auto piece = [&](int e) __attribute__((always_inline)) {
            return (size_t)blockIdx.x * BPW + e / (4 * QQ) < nblk ? (size_t)blockIdx.x * NE + e : (size_t)0;
        };
        stage_fetch<NE>(stv, win, piece);
        // exponentials shared by all right-hand sides: the prefactor of the
        // first-pass row (every first-pass thread applies its own) and the
        // remodulation of the second-pass outputs
        cpx<T> Ep[Q], E2[4][2 * NG];
        if (factive) {
            const int c2 = fac & 1, c1 = fac >> 1;
            const double xa1 = box_node(fap1, level - 1, tb.z[fatp1]);
#pragma unroll
            for (int tp2 = 0; tp2 < Q; ++tp2) {
                const XP xp = make_xp_sc(ph, xa1, box_node(fap2, level - 1, tb.z[tp2]), sp[fb][0][fatp1],
                                         cp[fb][0][fatp1], sp[fb][1][tp2], cp[fb][1][tp2]);
                Ep[tp2] = cis<T>(r0c[fb][c1] * phase_dir(xp, ct0[fb][c2], st0[fb][c2]));
            }
        }
        if (sactive) {
#pragma unroll
            for (int o = 0; o < 2 * NG; ++o) {
                const double G0 = remod_phase(o >> 1, o & 1, 0), G1 = remod_phase(o >> 1, o & 1, 1);
                E2[0][o] = cis<T>(r0c[sb][0] * G0);
                E2[1][o] = cis<T>(r0c[sb][0] * G1);
                E2[2][o] = cis<T>(r0c[sb][1] * G0);
                E2[3][o] = cis<T>(r0c[sb][1] * G1);
            }
        }
        // inputs staged through LDS by coalesced loads, one right-hand side
        // ahead: loaded during the second pass, staged once it is done
        stage_put<NE>(stv, xin);
        lds_barrier();
        const cpx<T> *const in = &xin[(fb * 4 + fac) * QQ + fatp1 * Q];
        for (int r = 0; r < nrhs; ++r) {
            opaque_sgpr(SAg);
            STg = SAg + 2 * QQ;
            ATg = SAg + 3 * QQ;
            if (factive) {
                cpx<T> vv[Q];
#pragma unroll
                for (int tp2 = 0; tp2 < Q; ++tp2) vv[tp2] = cmulc(in[tp2], Ep[tp2]);
                first_pass(vv);
            }
            lds_barrier();
            // (the last one refetches the last right-hand side: unconditional
            // loads keep the staged values in registers)
            stage_fetch<NE>(stv, win + (size_t)min(r + 1, nrhs - 1) * plane, piece);
            if (sactive) with_uniform<0, 4>(sg, [&](auto gc) __attribute__((always_inline)) {
                cpx<T> out[2 * NG];
#pragma unroll
                for (int o = 0; o < 2 * NG; ++o) out[o] = {(T)0, (T)0};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    cpx<T> z[2 * NG];
                    second_pass_c(gc, c, z);
#pragma unroll
                    for (int o = 0; o < 2 * NG; ++o) cfma(out[o], E2[c][o], z[o]);
                }
                store_outputs(gc, out, r * plane);
            });
            stage_put<NE>(stv, xin);
            lds_barrier();
        }
        return;
    }
    // one right-hand side: prefactor conj E(x^{A_p}_t', p0(B_c)) delta^{A_p B_c}_t'
    // once per row (c, t'1)
    if (active && rr < 4 * Q) {
        const int pc = rr / Q, ptp1 = rr - pc * Q;
        const int c2 = pc & 1, c1 = pc >> 1;
        const cpx<T> *src = win + (blk * 4 + pc) * QQ + ptp1 * Q;
#pragma unroll
        for (int tp2 = 0; tp2 < Q; ++tp2) {
            const XP xp = make_xp_sc(ph, box_node(ap1, level - 1, tb.z[ptp1]),
                                     box_node(ap2, level - 1, tb.z[tp2]), sp[bbl][0][ptp1], cp[bbl][0][ptp1],
                                     sp[bbl][1][tp2], cp[bbl][1][tp2]);
            xin[(bbl * 4 + pc) * QQ + ptp1 * Q + tp2] =
                cmulc(src[tp2], cis<T>(r0c[bbl][c1] * phase_dir(xp, ct0[bbl][c2], st0[bbl][c2])));
        }
    }
    lds_barrier();
    if (factive) {
        cpx<T> vv[Q];
#pragma unroll
        for (int tp2 = 0; tp2 < Q; ++tp2) vv[tp2] = xin[(fb * 4 + fac) * QQ + fatp1 * Q + tp2];
        first_pass(vv);
    }
    lds_barrier();
    // second pass, remodulation E(x^A_t, p0(B_c)), sum over c
    if (sactive) {
        double G0[2 * NG], G1[2 * NG];
#pragma unroll
        for (int o = 0; o < 2 * NG; ++o) {
            G0[o] = remod_phase(o >> 1, o & 1, 0);
            G1[o] = remod_phase(o >> 1, o & 1, 1);
        }
        cpx<T> out[2 * NG];
#pragma unroll
        for (int o = 0; o < 2 * NG; ++o) out[o] = {(T)0, (T)0};
        with_uniform<0, 4>(sg, [&](auto gc) __attribute__((always_inline)) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int c1 = c >> 1, c2 = c & 1;
                cpx<T> z[2 * NG];
                second_pass_c(gc, c, z);
                const double rho = r0c[sb][c1];
#pragma unroll
                for (int o = 0; o < 2 * NG; ++o)
                    if (decltype(gc)::value + 4 * (o >> 1) < Q) cfma(out[o], cis<T>(rho * (c2 ? G1[o] : G0[o])), z[o]);
            }
            store_outputs(gc, out, 0);
        });
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
