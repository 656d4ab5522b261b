// HIP kernels (gfx950) of the adjoint butterfly pass: the exact conjugate
// transposes of the forward steps, applied in reverse order.  Same weight
// layout and launch conventions as fio_kernels_fwd.hip.
#include <hip/hip_runtime.h>

#include "fio_kernels_common.h"

namespace fio {

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
        lds_barrier();
        for (int i = tid; i < nb * np; i += NT) {
            const int b = i / np;
            U[b * np + jp] = cmulc(uv, cis<T>(r0b[b] * phase_dir(xg, ctb[b], stb[b])));
        }
        lds_barrier();
        // Y[b][t1][j2] = sum_j1 Tt[j1][t1] U[b][j1][j2]
        for (int i = tid; i < nb * Q * m; i += NT) {
            const int b = i / (Q * m), r = i - b * (Q * m);
            const int t1 = r / m, jj2 = r - t1 * m;
            cpx<T> acc = {(T)0, (T)0};
            for (int jj1 = 0; jj1 < m; ++jj1) crfma(acc, Tt[jj1 * Q + t1], U[b * np + jj1 * m + jj2]);
            Y[i] = acc;
        }
        lds_barrier();
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
        lds_barrier();
    }
}

// x-level^H at level l: from the outputs (A_j, B) back to the inputs (A_p, B_c)
//   delta^{A_p B_c}_t' = E(x^{A_p}_t', p0(B_c)) sum_j sum_t M_j1[t'1][t1] M_j2[t'2][t2]
//                          conj E(x^{A_j}_t, p0(B_c)) delta^{A_j B}_t
// Each 1-D pass sums two children j: with M_1 = J M_0 J,
//   M_0 u + M_1 y = S (u + J y) + A (u - J y),
// and rows n, q-1-n of S agree and of A differ in sign, so P = S_n . a and
// D = A_n . b give outputs n (P + D) and q-1-n (P - D): q MACs per output
// instead of 2q.  First pass: thread (j1, c, t1) takes row t1 of the two
// children (j1, 0), (j1, 1), applies conj E(x^{A_j}_t, p0(B_c)) and
// contracts over t2.  Second pass: thread (h, block, c, t'2) takes column
// t'2 of the first-pass rows of both j1, produces the row pairs n = h,
// h + 2, ... and applies E(x^{A_p}_t', p0(B_c)); h is the same for two
// waves.  The factors S, A are the same for every thread (SGPR operands).
template <typename T, int Q, bool HOIST>
__global__ __launch_bounds__(NT) void k_xlevel_adj(Geom g, PhaseDev ph, Tables tb, int level,
                                                   const cpx<T> *__restrict__ win,
                                                   cpx<T> *__restrict__ wout, unsigned nblk,
                                                   int nrhs, size_t plane) {
    constexpr int QQ = Q * Q;
    constexpr int TPB = 8 * Q;
    constexpr int BPW = blocks_per_wg<T, Q, 8>();
    static_assert(BPW * 4 * Q <= NT / 2, "second pass: a block's columns fit a half workgroup");
    constexpr int H1 = (Q + 1) / 2, H = Q / 2;
    constexpr int NK = (H1 + 1) / 2;                // row pairs per second-pass thread
    constexpr int YC = QQ + pad_xadj_c<T, Q>(), YJ = 4 * YC + pad_xadj_j<T, Q>();
    __shared__ cpx<T> Y[BPW][2][YJ];                // [j1][c][t1][t'2] (+ bank padding)
    constexpr int NE = BPW * 4 * QQ;                // the workgroup's inputs: BPW blocks x 4 outputs j
    __shared__ cpx<T> xin[stage_len<NE>()];
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
    cptr<T> SAg = to_constant(pick_SA<T>(tb));

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
    lds_barrier();
    // first pass: thread (block bbl, j1, c, t1)
    const int j1 = rr / (4 * Q), fc = (rr / Q) & 3, t1 = rr % Q;
    const int fc1 = fc >> 1, fc2 = fc & 1;
    // kernel value conj-applied to row t1 of child (j1, j2) at column t2
    auto row_exp = [&](int j2, int t2) __attribute__((always_inline)) {
        const int a1 = 2 * ap1 + j1, a2 = 2 * ap2 + j2;
        const XP xp = make_xp_sc(ph, box_node(a1, level, tb.z[t1]), box_node(a2, level, tb.z[t2]),
                                 sj[bbl][0][j1][t1], cj[bbl][0][j1][t1], sj[bbl][1][j2][t2], cj[bbl][1][j2][t2]);
        return cis<T>(r0c[bbl][fc1] * phase_dir(xp, ct0[bbl][fc2], st0[bbl][fc2]));
    };
    // second pass: thread (h, block sb, c sc, column tp2)
    const int h = __builtin_amdgcn_readfirstlane(tid / (NT / 2));
    const int si = tid - h * (NT / 2);
    const int sb = si / (4 * Q), sk = si - sb * (4 * Q), sc = sk / Q, tp2 = sk - sc * Q;
    const int sc1 = sc >> 1, sc2 = sc & 1;
    const size_t sblk = (size_t)blockIdx.x * BPW + sb;
    const bool sactive = sb < BPW && sblk < nblk;
    int sap1 = 0, sap2 = 0;
    if (sactive) morton_decode((uint32_t)(sblk >> (2 * lB)), sap1, sap2);
    auto pre_exp = [&](int tp1) __attribute__((always_inline)) {  // E(x^{A_p}_t', p0(B_c)) at t' = (tp1, tp2)
        const XP xp = make_xp_sc(ph, box_node(sap1, level - 1, tb.z[tp1]), box_node(sap2, level - 1, tb.z[tp2]),
                                 sp[sb][0][tp1], cp[sb][0][tp1], sp[sb][1][tp2], cp[sb][1][tp2]);
        return cis<T>(r0c[sb][sc1] * phase_dir(xp, ct0[sb][sc2], st0[sb][sc2]));
    };
    // exponentials shared by all right-hand sides
    cpx<T> E1[2][Q], E2[2 * NK];
    if (HOIST && active) {
#pragma unroll
        for (int t2 = 0; t2 < Q; ++t2) {
            E1[0][t2] = row_exp(0, t2);
            E1[1][t2] = row_exp(1, t2);
        }
    }
    if (HOIST && sactive) {
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int n = min(h + 2 * k, H1 - 1);
            E2[2 * k] = pre_exp(n);
            E2[2 * k + 1] = pre_exp(Q - 1 - n);
        }
    }
    // inputs staged through LDS by coalesced loads, one right-hand side ahead:
    // piece (block b, output j) is QQ values at ((4 A_p + j) nBl + B) QQ
    cpx<T> stv[stage_per<NE>()];
    auto piece = [&](int e) __attribute__((always_inline)) {
        const int b = e / (4 * QQ), rem = e - b * (4 * QQ), jj = rem / QQ, o = rem - jj * QQ;
        const size_t pb = (size_t)blockIdx.x * BPW + b;
        return pb < nblk ? ((4 * (pb >> (2 * lB)) + jj) * nBl + (pb & (nBl - 1))) * QQ + o : (size_t)0;
    };
    stage_fetch<NE>(stv, win, piece);
    stage_put<NE>(stv, xin);
    lds_barrier();
    const cpx<T> *const in0 = &xin[(bbl * 4 + 2 * j1) * QQ + t1 * Q];  // row t1 of child (j1, 0); + QQ: (j1, 1)
    cpx<T> *const dst0 = wout + (sblk * 4 + sc) * QQ;
    for (int r = 0; r < (HOIST ? nrhs : 1); ++r) {
        opaque_sgpr(SAg);
        if (active) {
            // a = v_0 + J v_1, b = v_0 - J v_1 with v_j2 = conj E . delta of child (j1, j2)
            cpx<T> P[H1], D[H > 0 ? H : 1];
#pragma unroll
            for (int n = 0; n < H1; ++n) P[n] = {(T)0, (T)0};
#pragma unroll
            for (int n = 0; n < H; ++n) D[n] = {(T)0, (T)0};
#pragma unroll
            for (int m = 0; m < Q; ++m) {
                const cpx<T> v0 = cmulc(in0[m], HOIST ? E1[0][m] : row_exp(0, m));
                const cpx<T> v1 = cmulc(in0[QQ + Q - 1 - m], HOIST ? E1[1][Q - 1 - m] : row_exp(1, Q - 1 - m));
                const cpx<T> av = {v0.re + v1.re, v0.im + v1.im};
                const cpx<T> bv = {v0.re - v1.re, v0.im - v1.im};
#pragma unroll
                for (int n = 0; n < H1; ++n) crfma(P[n], SAg[n * Q + m], av);
#pragma unroll
                for (int n = 0; n < H; ++n) crfma(D[n], SAg[QQ + n * Q + m], bv);
            }
            cpx<T> *wr = &Y[bbl][j1][fc * YC + t1 * Q];
#pragma unroll
            for (int n = 0; n < H; ++n) {
                wr[n] = {P[n].re + D[n].re, P[n].im + D[n].im};
                wr[Q - 1 - n] = {P[n].re - D[n].re, P[n].im - D[n].im};
            }
            if constexpr (Q & 1) wr[H] = P[H];
        }
        lds_barrier();
        // the next right-hand side's inputs are loaded during the second pass
        // (unconditionally: the last one refetches the last right-hand side,
        // which keeps the staged values in registers)
        if (HOIST) stage_fetch<NE>(stv, win + (size_t)min(r + 1, nrhs - 1) * plane, piece);
        if (sactive) with_uniform<0, 2>(h, [&](auto hc) __attribute__((always_inline)) {
            constexpr int hh = decltype(hc)::value;
            cpx<T> Pn[NK], Dn[NK];
#pragma unroll
            for (int k = 0; k < NK; ++k) Pn[k] = Dn[k] = {(T)0, (T)0};
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                const cpx<T> x0 = Y[sb][0][sc * YC + p * Q + tp2];
                const cpx<T> x1 = Y[sb][1][sc * YC + (Q - 1 - p) * Q + tp2];
                const cpx<T> av = {x0.re + x1.re, x0.im + x1.im};
                const cpx<T> bv = {x0.re - x1.re, x0.im - x1.im};
#pragma unroll
                for (int k = 0; k < NK; ++k) {
                    const int n = hh + 2 * k;
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
                    dst[n * Q + tp2] = cmul(o0, HOIST ? E2[2 * k] : pre_exp(n));
                    if (n < H) {
                        const cpx<T> o1 = {Pn[k].re - Dn[k].re, Pn[k].im - Dn[k].im};
                        dst[(Q - 1 - n) * Q + tp2] = cmul(o1, HOIST ? E2[2 * k + 1] : pre_exp(Q - 1 - n));
                    }
                }
            }
        });
        if (HOIST) stage_put<NE>(stv, xin);
        lds_barrier();
    }
}

// switch^H at level lm, in place: delta_s <- sum_t conj E(x^A_t, p^B_s) delta_t.
// Thread <-> (pair, s2) owns the q outputs s1 of its column.  With
// rho(s1) = rho0 + h_s1 and z_{q-1-j} = -z_j, the factor of (t, s) is
// conj(base) conj(d_j) for s1 = j and conj(base) d_j for s1 = q-1-j, where
// base = exp(2 pi i rho0 G), d_j = exp(2 pi i h_j G), G = G(x_t, theta_s2).
// So per t the thread forms b = conj(base) delta_t once per right-hand side
// and accumulates P_j = sum_t Re(d_j) b and Q_j = sum_t Im(d_j) b (4 FMA per
// pair of outputs); at the end out_j = P_j - i Q_j, out_{q-1-j} = P_j + i Q_j.
// The 1 + floor(q/2) exponentials of (t, s2) serve a chunk of RC right-hand
// sides.  The inputs of the workgroup's pairs are staged through LDS one row
// t1 at a time, double-buffered: the loads of row t1+1 are issued before the
// arithmetic of row t1 and land in LDS after it.
template <typename T, int Q, int RC, bool ONE>
__global__ __launch_bounds__(NT) void k_switch_adj(Geom g, PhaseDev ph, Tables tb, cpx<T> *__restrict__ w,
                                                   int nrhs, size_t plane) {
    constexpr int QQ = Q * Q;
    constexpr int H = Q / 2;
    constexpr int HH = H > 0 ? H : 1;
    constexpr int PPB = NT / Q;
    constexpr int ROW = PPB * RC * Q;             // staged values per row
    constexpr int LPT = (ROW + NT - 1) / NT;      // of which each thread loads LPT
    __shared__ cpx<T> rowbuf[2][RC][PPB][Q];
    __shared__ double sx[PPB][2][Q], cx[PPB][2][Q];

    const int tid = threadIdx.x;
    const int pl = tid / Q, s2 = tid - pl * Q;
    const size_t npairs = (size_t)1 << (2 * g.L);
    const size_t pair0 = (size_t)blockIdx.x * PPB;
    const size_t pair = pair0 + pl;
    const bool active = (pl < PPB) && (pair < npairs);
    const int lA = g.lm, lB = g.L - g.lm;
    const size_t nBl = (size_t)1 << (2 * lB);
    const uint32_t mB = active ? (uint32_t)(pair & (nBl - 1)) : 0;
    const uint32_t mA = active ? (uint32_t)(pair >> (2 * lB)) : 0;
    int b1, b2, a1, a2;
    morton_decode(mB, b1, b2);
    morton_decode(mA, a1, a2);
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;
    if (active) {
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
    double st = 0, ct = 1;
    if (active) sincospi(2.0 * box_node(b2, lB, tb.z[s2]), &st, &ct);
    const double r0 = g.rho_scale * box_centre(b1, lB);
    double hz[HH];
#pragma unroll
    for (int j = 0; j < H; ++j) hz[j] = g.rho_scale * ldexp(tb.z[j], -lB);

    for (int q0 = 0; q0 < (ONE ? 1 : nrhs); q0 += RC) {
        const int nr = min(RC, nrhs - q0);
        // staged element e = (rc * PPB + p) * Q + t2 of row t1
        auto fetch = [&](int t1, cpx<T> (&v)[LPT]) __attribute__((always_inline)) {
#pragma unroll
            for (int k = 0; k < LPT; ++k) {
                const int e = tid + k * NT;
                const int rc = e / (PPB * Q), rem = e - rc * (PPB * Q);
                const int p = rem / Q, t2 = rem - p * Q;
                if (e < ROW && rc < nr && pair0 + p < npairs)
                    v[k] = w[(size_t)(q0 + rc) * plane + (pair0 + p) * QQ + t1 * Q + t2];
            }
        };
        auto stash = [&](int buf, const cpx<T> (&v)[LPT]) __attribute__((always_inline)) {
#pragma unroll
            for (int k = 0; k < LPT; ++k) {
                const int e = tid + k * NT;
                const int rc = e / (PPB * Q), rem = e - rc * (PPB * Q);
                const int p = rem / Q, t2 = rem - p * Q;
                if (e < ROW) rowbuf[buf][rc][p][t2] = v[k];
            }
        };
        cpx<T> pre[LPT];
#pragma unroll
        for (int k = 0; k < LPT; ++k) pre[k] = {(T)0, (T)0};
        lds_barrier();  // the previous chunk's readers are done with rowbuf
        fetch(0, pre);
        stash(0, pre);
        lds_barrier();

        cpx<T> P[RC][HH], Qs[RC][HH], Mi[RC];
#pragma unroll
        for (int rc = 0; rc < RC; ++rc) {
            Mi[rc] = {(T)0, (T)0};
#pragma unroll
            for (int j = 0; j < HH; ++j) P[rc][j] = Qs[rc][j] = {(T)0, (T)0};
        }
        for (int t1 = 0; t1 < Q; ++t1) {
            const int buf = t1 & 1;
            if (t1 + 1 < Q) fetch(t1 + 1, pre);
            if (active) {
                for (int t2 = 0; t2 < Q; ++t2) {
                    const XP xp = make_xp_sc(ph, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]),
                                             sx[pl][0][t1], cx[pl][0][t1], sx[pl][1][t2], cx[pl][1][t2]);
                    const double G = phase_dir(xp, ct, st);
                    const cpx<T> base = cis<T>(r0 * G);
                    cpx<T> d[HH];
#pragma unroll
                    for (int j = 0; j < H; ++j) d[j] = cis<T>(hz[j] * G);
#pragma unroll
                    for (int rc = 0; rc < RC; ++rc) {
                        if (rc < nr) {
                            const cpx<T> bb = cmulc(rowbuf[buf][rc][pl][t2], base);
                            if (Q & 1) {
                                Mi[rc].re += bb.re;
                                Mi[rc].im += bb.im;
                            }
#pragma unroll
                            for (int j = 0; j < H; ++j) {
                                crfma(P[rc][j], d[j].re, bb);
                                crfma(Qs[rc][j], d[j].im, bb);
                            }
                        }
                    }
                }
            }
            if (t1 + 1 < Q) stash(buf ^ 1, pre);
            lds_barrier();
        }
        // every read of this chunk happened before the barrier above
        if (active) {
#pragma unroll
            for (int rc = 0; rc < RC; ++rc)
                if (rc < nr) {
                    cpx<T> *wp = w + (size_t)(q0 + rc) * plane + pair * QQ;
#pragma unroll
                    for (int j = 0; j < H; ++j) {
                        const cpx<T> p = P[rc][j], qq = Qs[rc][j];
                        wp[j * Q + s2] = {p.re + qq.im, p.im - qq.re};
                        wp[(Q - 1 - j) * Q + s2] = {p.re - qq.im, p.im + qq.re};
                    }
                    if (Q & 1) wp[H * Q + s2] = Mi[rc];
                }
        }
    }
}

// p-level^H at level l: from the outputs (A_j, B) back to the inputs (A_p, B_c)
//   delta^{A_p B_c}_t' = sum_j conj E(x0(A_j), p^{B_c}_t') sum_t M_c1[t1][t'1] M_c2[t2][t'2]
//                          E(x0(A_j), p^B_t) delta^{A_j B}_t
// Each 1-D pass feeds one input to two children c (the transposes M_c^T):
// with M_1 = J M_0 J, (M_1^T v)[q-1-n] = (M_0^T J v)[n], so s = v + J v and
// d = v - J v (first half) give P = ST_n . s and D = AT_n . d with
// (M_0^T v)[n] = P + D and (M_1^T v)[q-1-n] = P - D: q MACs for two outputs.
// First pass: thread (h, block, j, t1) forms row t1 of E delta for output j
// and produces the columns n = h H1 + k of child c2 = 0 and q-1-n of c2 = 1
// (h the same for two waves).  Second pass: thread (g, block, c2, t'2), g
// the wave, takes column t'2 of the first-pass rows of c2 and each output
// j, produces rows n = g, g + 4, ... of child c1 = 0 and q-1-n of c1 = 1,
// applies conj E(x0(A_j), p^{B_c}_t') and sums j.  The factors are
// wave-uniform in both passes (SGPR operands).
template <typename T, int Q, bool HOIST>
__global__ __launch_bounds__(NT) void k_plevel_adj(Geom g, PhaseDev ph, Tables tb, int level,
                                                   const cpx<T> *__restrict__ win,
                                                   cpx<T> *__restrict__ wout, unsigned nblk,
                                                   int nrhs, size_t plane) {
    constexpr int QQ = Q * Q;
    constexpr int TPO = 2 * Q;
    constexpr int TPB = 4 * TPO;
    constexpr int BPW = blocks_per_wg<T, Q, 8>();
    static_assert(BPW * 4 * Q <= NT / 2 && BPW * 2 * Q <= 64, "pass layouts fit the workgroup");
    constexpr int H1 = (Q + 1) / 2, H = Q / 2;
    constexpr int NG = (Q + 3) / 4;       // second-pass rows per thread
    __shared__ double rc[BPW][2 * Q], ctc[BPW][2 * Q], stc[BPW][2 * Q];
    __shared__ double rb[BPW][Q], ctb[BPW][Q], stb[BPW][Q];
    __shared__ double Gc[BPW][4][2 * Q], Gb[BPW][4][Q];
    constexpr int YA = 4 * QQ + pad_sum_out<T, Q>();
    __shared__ cpx<T> Y[BPW][2][YA];      // [c2][j][t1][t'2] (+ bank padding)
    constexpr int NE = BPW * 4 * QQ;      // the workgroup's inputs: BPW blocks x 4 outputs j
    __shared__ cpx<T> xin[stage_len<NE>()];

    const int tid = threadIdx.x;
    const int bbl = tid / TPB, r = tid - bbl * TPB;
    const int j = r / TPO, rr = r - j * TPO;
    const size_t blk = (size_t)blockIdx.x * BPW + bbl;
    const bool active = bbl < BPW && blk < nblk;
    const int lB = g.L - level;
    const size_t nBl = (size_t)1 << (2 * lB);
    cptr<T> SAg = to_constant(pick_SA<T>(tb));
    cptr<T> STg = SAg + 2 * QQ, ATg = SAg + 3 * QQ;  // re-derived per right-hand side

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
    if (active) {
        const int a1 = 2 * ap1 + (j >> 1), a2 = 2 * ap2 + (j & 1);
        const XP xp = make_xp(ph, box_centre(a1, level), box_centre(a2, level));
        Gc[bbl][j][rr] = phase_dir(xp, ctc[bbl][rr], stc[bbl][rr]);
        if (rr < Q) Gb[bbl][j][rr] = phase_dir(xp, ctb[bbl][rr], stb[bbl][rr]);
    }
    lds_barrier();
    // first pass: thread (fh, block fb, output fj, row t1); fh uniform over two waves
    const int fh = __builtin_amdgcn_readfirstlane(tid / (NT / 2)), fi = tid - fh * (NT / 2);
    const int fb = fi / (4 * Q), fk = fi - fb * (4 * Q), fj = fk / Q, t1 = fk - fj * Q;
    const size_t fblk = (size_t)blockIdx.x * BPW + fb;
    const bool factive = fb < BPW && fblk < nblk;
    uint32_t fmB = 0, fmAp = 0;
    if (factive) {
        fmB = (uint32_t)(fblk & (nBl - 1));
        fmAp = (uint32_t)(fblk >> (2 * lB));
    }
    // second pass: thread (wave sg, block sb, child column c2 sc2, column tp2)
    const int sg = __builtin_amdgcn_readfirstlane(tid / 64), sl = tid & 63;
    const int sb = sl / (2 * Q), sk = sl - sb * (2 * Q), sc2 = sk / Q, tp2 = sk - sc2 * Q;
    const size_t sblk = (size_t)blockIdx.x * BPW + sb;
    const bool sactive = sb < BPW && sblk < nblk;
    // this thread's outputs: (c1 = 0, row n), (c1 = 1, row q-1-n), n = sg + 4k
    auto out_row = [&](int o) __attribute__((always_inline)) {
        const int n = min(sg + 4 * (o >> 1), Q - 1);
        return (o & 1) ? Q - 1 - n : n;
    };
    cpx<T> *const dst0 = wout + (sblk * 4 + sc2) * QQ;  // child (0, c2); (1, c2) is 2 QQ further
    const double rhoB = factive ? rb[fb][t1] : 0.0;

    auto first_pass = [&](const cpx<T> (&gv)[Q]) __attribute__((always_inline)) {
        with_uniform<0, 2>(fh, [&](auto hc) __attribute__((always_inline)) {
        constexpr int fhh = decltype(hc)::value;
        cpx<T> sv[H1], dv[H > 0 ? H : 1];
#pragma unroll
        for (int m = 0; m < H; ++m) {
            sv[m] = {gv[m].re + gv[Q - 1 - m].re, gv[m].im + gv[Q - 1 - m].im};
            dv[m] = {gv[m].re - gv[Q - 1 - m].re, gv[m].im - gv[Q - 1 - m].im};
        }
        if constexpr (Q & 1) sv[H] = gv[H];
#pragma unroll
        for (int k = 0; k < H1; ++k) {
            const int n = fhh * H1 + k;
            if (n < Q) {
                cpx<T> P = {(T)0, (T)0}, D = {(T)0, (T)0};
#pragma unroll
                for (int m = 0; m < H1; ++m) crfma(P, STg[n * Q + m], sv[m]);
#pragma unroll
                for (int m = 0; m < H; ++m) crfma(D, ATg[n * Q + m], dv[m]);
                Y[fb][0][fj * QQ + t1 * Q + n] = {P.re + D.re, P.im + D.im};
                Y[fb][1][fj * QQ + t1 * Q + Q - 1 - n] = {P.re - D.re, P.im - D.im};
            }
        }
        });
    };
    // second pass for output jj: z[o] = (M_c1^T col)[row] of this thread's outputs
    auto second_pass_j = [&](auto gc, int jj, cpx<T> (&z)[2 * NG]) __attribute__((always_inline)) {
        constexpr int gg = decltype(gc)::value;
        cpx<T> sv[H1], dv[H > 0 ? H : 1];
        const cpx<T> *col = &Y[sb][sc2][jj * QQ + tp2];
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
    // exponentials shared by all right-hand sides
    cpx<T> E1[Q], E2[4][2 * NG];
    if (HOIST && factive) {
#pragma unroll
        for (int t2 = 0; t2 < Q; ++t2) E1[t2] = cis<T>(rhoB * Gb[fb][fj][t2]);
    }
    if (HOIST && sactive) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const double G = Gc[sb][jj][sc2 * Q + tp2];
#pragma unroll
            for (int o = 0; o < 2 * NG; ++o)
                if (sg + 4 * (o >> 1) < Q) E2[jj][o] = cis<T>(rc[sb][(o & 1) * Q + out_row(o)] * G);
        }
    }
    // inputs staged through LDS by coalesced loads, one right-hand side ahead:
    // piece (block b, output j) is QQ values at ((4 A_p + j) nBl + B) QQ
    cpx<T> stv[stage_per<NE>()];
    auto piece = [&](int e) __attribute__((always_inline)) {
        const int b = e / (4 * QQ), rem = e - b * (4 * QQ), jj = rem / QQ, o = rem - jj * QQ;
        const size_t pb = (size_t)blockIdx.x * BPW + b;
        return pb < nblk ? ((4 * (pb >> (2 * lB)) + jj) * nBl + (pb & (nBl - 1))) * QQ + o : (size_t)0;
    };
    stage_fetch<NE>(stv, win, piece);
    stage_put<NE>(stv, xin);
    lds_barrier();
    const cpx<T> *const in = &xin[(fb * 4 + fj) * QQ + t1 * Q];
    for (int ri = 0; ri < (HOIST ? nrhs : 1); ++ri) {
        opaque_sgpr(SAg);
        STg = SAg + 2 * QQ;
        ATg = SAg + 3 * QQ;
        if (factive) {
            cpx<T> gv[Q];
#pragma unroll
            for (int t2 = 0; t2 < Q; ++t2) gv[t2] = cmul(in[t2], HOIST ? E1[t2] : cis<T>(rhoB * Gb[fb][fj][t2]));
            first_pass(gv);
        }
        lds_barrier();
        // the next right-hand side's inputs are loaded during the second pass
        // (unconditionally: the last one refetches the last right-hand side,
        // which keeps the staged values in registers)
        if (HOIST) stage_fetch<NE>(stv, win + (size_t)min(ri + 1, nrhs - 1) * plane, piece);
        if (sactive) with_uniform<0, 4>(sg, [&](auto gc) __attribute__((always_inline)) {
            constexpr int gg = decltype(gc)::value;
            cpx<T> acc[2 * NG];
#pragma unroll
            for (int o = 0; o < 2 * NG; ++o) acc[o] = {(T)0, (T)0};
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                cpx<T> z[2 * NG];
                second_pass_j(gc, jj, z);
                const double G = Gc[sb][jj][sc2 * Q + tp2];
#pragma unroll
                for (int o = 0; o < 2 * NG; ++o)
                    if (gg + 4 * (o >> 1) < Q)
                        cfmac(acc[o], z[o], HOIST ? E2[jj][o] : cis<T>(rc[sb][(o & 1) * Q + out_row(o)] * G));
            }
            cpx<T> *dst = dst0 + ri * plane;
#pragma unroll
            for (int k = 0; k < NG; ++k) {
                const int n = gg + 4 * k;
                if (n < Q) {
                    dst[n * Q + tp2] = acc[2 * k];
                    dst[2 * QQ + (Q - 1 - n) * Q + tp2] = acc[2 * k + 1];
                }
            }
        });
        if (HOIST) stage_put<NE>(stv, xin);
        lds_barrier();
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
    lds_barrier();
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
            lds_barrier();
            if (tid < na) {
                int a1, a2;
                morton_decode((uint32_t)(a0 + tid), a1, a2);
                xA[tid] = make_xp(ph, box_centre(a1, g.s), box_centre(a2, g.s));
            }
            lds_barrier();
            for (int i = tid; i < na * QQ; i += NT) {
                const int al = i / QQ, t = i - al * QQ;
                const int t1 = t / Q, t2 = t - t1 * Q;
                const double rho = g.rho_scale * box_node(bp1, lB, zs[t1]);
                const cpx<T> e = cis<T>(rho * phase_dir(xA[al], ctb[t2], stb[t2]));
                gA[al][t] = cmul(win[((size_t)(a0 + al) * nBl + mB) * QQ + t], e);
            }
            lds_barrier();
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
                               const void *win, void *wout, int nrhs, size_t plane, hipStream_t st) {
    const unsigned nblk = 1u << (2 * g.L - 2);
#define L_XLA(Q)                                                                                     \
    {                                                                                                \
        constexpr int BPW = blocks_per_wg<T, Q, 8>();                                                \
        const dim3 grid((nblk + BPW - 1) / BPW);                                                     \
        if (nrhs == 1)                                                                               \
            hipLaunchKernelGGL((k_xlevel_adj<T, Q, false>), grid, dim3(NT), 0, st, g, ph, tb, level, \
                               (const cpx<T> *)win, (cpx<T> *)wout, nblk, nrhs, plane);              \
        else                                                                                         \
            hipLaunchKernelGGL((k_xlevel_adj<T, Q, true>), grid, dim3(NT), 0, st, g, ph, tb, level,  \
                               (const cpx<T> *)win, (cpx<T> *)wout, nblk, nrhs, plane);              \
    }
    FIO_DISPATCH_Q(g.q, L_XLA)
#undef L_XLA
    return hipGetLastError();
}

template <typename T>
static hipError_t switch_adj_t(const Geom &g, const PhaseDev &ph, const Tables &tb, void *w, int nrhs,
                               size_t plane, hipStream_t st) {
    if (sizeof(T) == 4 && switch_adj_mfma_supported(g.q, nrhs))
        return launch_switch_adj_mfma(g, ph, tb, w, nrhs, plane, st);
    const size_t npairs = (size_t)1 << (2 * g.L);
#define L_SWA(Q)                                                                                     \
    {                                                                                                \
        constexpr int PPB = NT / Q;                                                                  \
        if (nrhs == 1) {                                                                             \
            const unsigned nblk = (unsigned)((npairs + PPB - 1) / PPB);                              \
            hipLaunchKernelGGL((k_switch_adj<T, Q, 1, true>), dim3(nblk), dim3(NT), 0, st, g, ph, tb,\
                               (cpx<T> *)w, nrhs, plane);                                            \
        } else {                                                                                     \
            constexpr int RC = swadj_rc<T>();                                                        \
            const unsigned nblk = (unsigned)((npairs + PPB - 1) / PPB);                              \
            hipLaunchKernelGGL((k_switch_adj<T, Q, RC, false>), dim3(nblk), dim3(NT), 0, st, g, ph,  \
                               tb,                                                                   \
                               (cpx<T> *)w, nrhs, plane);                                            \
        }                                                                                            \
    }
    FIO_DISPATCH_Q(g.q, L_SWA)
#undef L_SWA
    return hipGetLastError();
}

template <typename T>
static hipError_t plevel_adj_t(const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                               const void *win, void *wout, int nrhs, size_t plane, hipStream_t st) {
    const unsigned nblk = 1u << (2 * g.L - 2);
#define L_PLA(Q)                                                                                     \
    {                                                                                                \
        constexpr int BPW = blocks_per_wg<T, Q, 8>();                                                \
        const dim3 grid((nblk + BPW - 1) / BPW);                                                     \
        if (nrhs == 1)                                                                               \
            hipLaunchKernelGGL((k_plevel_adj<T, Q, false>), grid, dim3(NT), 0, st, g, ph, tb, level, \
                               (const cpx<T> *)win, (cpx<T> *)wout, nblk, nrhs, plane);              \
        else                                                                                         \
            hipLaunchKernelGGL((k_plevel_adj<T, Q, true>), grid, dim3(NT), 0, st, g, ph, tb, level,  \
                               (const cpx<T> *)win, (cpx<T> *)wout, nblk, nrhs, plane);              \
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

hipError_t launch_term_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, const void *u,
                           void *w, hipStream_t st) {
#define C(T) term_adj_t<T>(g, ph, tb, u, w, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_xlevel_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                             const void *win, void *wout, int nrhs, size_t plane, hipStream_t st) {
#define C(T) xlevel_adj_t<T>(g, ph, tb, level, win, wout, nrhs, plane, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_switch_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, void *w,
                             int nrhs, size_t plane, hipStream_t st) {
#define C(T) switch_adj_t<T>(g, ph, tb, w, nrhs, plane, st)
    return FIO_BY_DTYPE(dtype, C);
#undef C
}
hipError_t launch_plevel_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                             const void *win, void *wout, int nrhs, size_t plane, hipStream_t st) {
#define C(T) plevel_adj_t<T>(g, ph, tb, level, win, wout, nrhs, plane, st)
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
