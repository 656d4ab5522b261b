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
// First pass: thread (j1, c2, t1, j2) forms row t1 of conj E delta for its
// child (j1, j2) and both c1 and contracts over t2 with M_j2; the partial
// rows of the two j2 are summed.  Second pass: thread (c, t'2, half)
// contracts over t1 with M_j1, sums j1 and applies the factor
// E(x^{A_p}_t', p0(B_c)).
// SPLIT (FP32): j2 is the same for a pair of waves (threads [128 j2,
// 128 j2 + 128)), so the first-pass factors are wave-uniform (SGPR
// operands); both partial rows go to LDS and the second pass adds them.
// Otherwise (FP64, whose doubled partial rows would not fit the LDS budget):
// the two j2 of a row are adjacent lanes and add their rows through a DPP
// lane exchange before one of them stores the sum.
template <typename T, int Q>
constexpr bool xadj_split() { return sizeof(T) == 4; }

template <typename T, int Q, bool HOIST>
__global__ __launch_bounds__(NT) void k_xlevel_adj(Geom g, PhaseDev ph, Tables tb, int level,
                                                   const cpx<T> *__restrict__ win,
                                                   cpx<T> *__restrict__ wout, unsigned nblk,
                                                   int nrhs, size_t plane) {
    constexpr int QQ = Q * Q;
    constexpr int TPB = 8 * Q;
    constexpr bool SPLIT = xadj_split<T, Q>();
    constexpr int NS = SPLIT ? 2 : 1;
    constexpr int BPW = blocks_per_wg<T, Q, 8 * NS>();
    constexpr int H1 = (Q + 1) / 2;
    __shared__ T Ms[2][Q][Q];                       // Ms[a][t'][t] = M_a[t'][t]
    // rows padded to q^2 + 9 for q = 9: an LDS bank model of both passes' access
    // patterns (32 banks, 16 lanes per 64-bit access cycle) finds 22% fewer cycles
    constexpr int YROW = QQ + (Q == 9 ? 9 : 0);
    __shared__ cpx<T> Y[BPW][NS][2][4][YROW];       // [j2 partial][j1][c][t1][t'2]
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
    lds_barrier();
    // first-pass item (block fb, j1, c2f, t1, j2)
    int fb, j1, c2f, t1, j2;
    if constexpr (SPLIT) {
        j2 = __builtin_amdgcn_readfirstlane(tid / (NT / 2));
        const int fi = tid - j2 * (NT / 2);
        fb = fi / (4 * Q);
        const int fk = fi - fb * (4 * Q);
        j1 = fk / (2 * Q);
        c2f = (fk / Q) & 1;
        t1 = fk % Q;
    } else {
        // rr = ((j1 * 2 + c2) * Q + t1) * 2 + j2: the two j2 of a row are adjacent lanes
        fb = bbl;
        j2 = rr & 1;
        const int k1 = rr >> 1;
        t1 = k1 % Q;
        const int jc = k1 / Q;
        c2f = jc & 1;
        j1 = jc >> 1;
    }
    const size_t fblk = (size_t)blockIdx.x * BPW + fb;
    const bool factive = fb < BPW && fblk < nblk;
    uint32_t fmB = 0, fmAp = 0;
    int fap1 = 0, fap2 = 0;
    if (factive) {
        fmB = (uint32_t)(fblk & (nBl - 1));
        fmAp = (uint32_t)(fblk >> (2 * lB));
        morton_decode(fmAp, fap1, fap2);
    }
    // second pass: thread (c, t'2, half) of its block
    const int c = rr / (2 * Q), k2 = rr - c * 2 * Q;
    const int h = k2 / Q, tp2 = k2 - h * Q;
    const int c1 = c >> 1, c2 = c & 1;
    // exponentials shared by all right-hand sides
    cpx<T> E1[2][Q], E2[H1];
    auto row_exp = [&](int t2, cpx<T> &e0, cpx<T> &e1) {
        const int a1 = 2 * fap1 + j1, a2 = 2 * fap2 + j2;
        const XP xp = make_xp_sc(ph, box_node(a1, level, tb.z[t1]), box_node(a2, level, tb.z[t2]),
                                 sj[fb][0][j1][t1], cj[fb][0][j1][t1], sj[fb][1][j2][t2], cj[fb][1][j2][t2]);
        const double G = phase_dir(xp, ct0[fb][c2f], st0[fb][c2f]);
        e0 = cis<T>(r0c[fb][0] * G);
        e1 = cis<T>(r0c[fb][1] * G);
    };
    if (HOIST && factive) {
#pragma unroll
        for (int t2 = 0; t2 < Q; ++t2) row_exp(t2, E1[0][t2], E1[1][t2]);
    }
    if (HOIST && active) {
        const double xa2 = box_node(ap2, level - 1, tb.z[tp2]);
#pragma unroll
        for (int kk = 0; kk < H1; ++kk) {
            const int tp1 = min(h * H1 + kk, Q - 1);
            const XP xp = make_xp_sc(ph, box_node(ap1, level - 1, tb.z[tp1]), xa2, sp[bbl][0][tp1],
                                     cp[bbl][0][tp1], sp[bbl][1][tp2], cp[bbl][1][tp2]);
            E2[kk] = cis<T>(r0c[bbl][c1] * phase_dir(xp, ct0[bbl][c2], st0[bbl][c2]));
        }
    }
    // inputs of the thread's row, loaded one right-hand side ahead
    cpx<T> nx[Q];
    auto load_row = [&](int r) {
        const cpx<T> *src = win + r * plane + ((size_t)(4 * fmAp + 2 * j1 + j2) * nBl + fmB) * QQ + t1 * Q;
#pragma unroll
        for (int t2 = 0; t2 < Q; ++t2) nx[t2] = src[t2];
    };
    constexpr bool PF = HOIST && !(sizeof(T) == 8 && Q > 10);  // prefetch unless it spills
    if (PF && factive) load_row(0);
    for (int r = 0; r < (HOIST ? nrhs : 1); ++r) {
        {
            cpx<T> acc0[Q], acc1[Q];   // c1 = 0, 1
#pragma unroll
            for (int t = 0; t < Q; ++t) acc0[t] = acc1[t] = {(T)0, (T)0};
            if (factive) {
                if (!PF) load_row(r);
                cpx<T> in[Q];
#pragma unroll
                for (int k = 0; k < Q; ++k) in[k] = nx[k];
                if (PF && r + 1 < nrhs) load_row(r + 1);
#pragma unroll
                for (int t2 = 0; t2 < Q; ++t2) {
                    cpx<T> e0, e1;
                    if constexpr (HOIST) {
                        e0 = E1[0][t2];
                        e1 = E1[1][t2];
                    } else {
                        row_exp(t2, e0, e1);
                    }
                    const cpx<T> d = in[t2];
                    const cpx<T> v0 = cmulc(d, e0);
                    const cpx<T> v1 = cmulc(d, e1);
#pragma unroll
                    for (int p2 = 0; p2 < Q; ++p2) {
                        const T m = SPLIT ? Mg[(j2 * Q + p2) * Q + t2] : Ms[j2][p2][t2];
                        crfma(acc0[p2], m, v0);
                        crfma(acc1[p2], m, v1);
                    }
                }
            }
            if constexpr (SPLIT) {
                if (factive) {
#pragma unroll
                    for (int p2 = 0; p2 < Q; ++p2) {
                        Y[fb][j2][j1][c2f][t1 * Q + p2] = acc0[p2];        // c = 2*0 + c2
                        Y[fb][j2][j1][2 + c2f][t1 * Q + p2] = acc1[p2];    // c = 2*1 + c2
                    }
                }
            } else {
                // add the partner lane's (other j2) partial rows
#pragma unroll
                for (int t = 0; t < Q; ++t) {
                    acc0[t].re += swap_adjacent_lanes(acc0[t].re);
                    acc0[t].im += swap_adjacent_lanes(acc0[t].im);
                    acc1[t].re += swap_adjacent_lanes(acc1[t].re);
                    acc1[t].im += swap_adjacent_lanes(acc1[t].im);
                }
                if (factive && j2 == 0) {
#pragma unroll
                    for (int p2 = 0; p2 < Q; ++p2) {
                        Y[fb][0][j1][c2f][t1 * Q + p2] = acc0[p2];
                        Y[fb][0][j1][2 + c2f][t1 * Q + p2] = acc1[p2];
                    }
                }
            }
        }
        lds_barrier();
        if (active) {
            cpx<T> acc[H1];
#pragma unroll
            for (int kk = 0; kk < H1; ++kk) acc[kk] = {(T)0, (T)0};
#pragma unroll
            for (int jj1 = 0; jj1 < 2; ++jj1) {
                cpx<T> col[Q];
#pragma unroll
                for (int tt = 0; tt < Q; ++tt) {
                    col[tt] = Y[bbl][0][jj1][c][tt * Q + tp2];
                    if constexpr (SPLIT) {
                        const cpx<T> o = Y[bbl][NS - 1][jj1][c][tt * Q + tp2];
                        col[tt].re += o.re;
                        col[tt].im += o.im;
                    }
                }
#pragma unroll
                for (int kk = 0; kk < H1; ++kk) {
                    const int tp1 = min(h * H1 + kk, Q - 1);
#pragma unroll
                    for (int tt = 0; tt < Q; ++tt) crfma(acc[kk], Ms[jj1][tp1][tt], col[tt]);
                }
            }
            cpx<T> *dst = wout + r * plane + (blk * 4 + c) * QQ;
            const double xa2 = box_node(ap2, level - 1, tb.z[tp2]);
#pragma unroll
            for (int kk = 0; kk < H1; ++kk) {
                const int tp1 = h * H1 + kk;
                if (tp1 < Q) {
                    cpx<T> e;
                    if constexpr (HOIST) {
                        e = E2[kk];
                    } else {
                        const XP xp = make_xp_sc(ph, box_node(ap1, level - 1, tb.z[tp1]), xa2, sp[bbl][0][tp1],
                                                 cp[bbl][0][tp1], sp[bbl][1][tp2], cp[bbl][1][tp2]);
                        e = cis<T>(r0c[bbl][c1] * phase_dir(xp, ct0[bbl][c2], st0[bbl][c2]));
                    }
                    dst[tp1 * Q + tp2] = cmul(acc[kk], e);
                }
            }
        }
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
        auto fetch = [&](int t1, cpx<T> (&v)[LPT]) {
#pragma unroll
            for (int k = 0; k < LPT; ++k) {
                const int e = tid + k * NT;
                const int rc = e / (PPB * Q), rem = e - rc * (PPB * Q);
                const int p = rem / Q, t2 = rem - p * Q;
                if (e < ROW && rc < nr && pair0 + p < npairs)
                    v[k] = w[(size_t)(q0 + rc) * plane + (pair0 + p) * QQ + t1 * Q + t2];
            }
        };
        auto stash = [&](int buf, const cpx<T> (&v)[LPT]) {
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
// First pass: thread (j, c2, t1) forms row t1 of E delta for output j and
// contracts it over t2 with M_c2.  Second pass: thread (c, t'2, half)
// contracts over t1 with M_c1, applies conj E(x0(A_j), p^{B_c}_t') and sums j.
template <typename T, int Q, bool HOIST>
__global__ __launch_bounds__(NT) void k_plevel_adj(Geom g, PhaseDev ph, Tables tb, int level,
                                                   const cpx<T> *__restrict__ win,
                                                   cpx<T> *__restrict__ wout, unsigned nblk,
                                                   int nrhs, size_t plane) {
    constexpr int QQ = Q * Q;
    constexpr int TPO = 2 * Q;
    constexpr int TPB = 4 * TPO;
    constexpr int BPW = blocks_per_wg<T, Q, 8>();
    constexpr int H1 = (Q + 1) / 2;
    __shared__ T Ms[2][Q][Q];             // Ms[c][t][t'] = M_c[t][t']
    __shared__ double rc[BPW][2 * Q], ctc[BPW][2 * Q], stc[BPW][2 * Q];
    __shared__ double rb[BPW][Q], ctb[BPW][Q], stb[BPW][Q];
    __shared__ double Gc[BPW][4][2 * Q], Gb[BPW][4][Q];
    __shared__ cpx<T> Y[BPW][2][4][QQ];   // [c2][j][t1][t'2] (c2 outside j: fewer LDS bank conflicts)

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
    lds_barrier();
    if (active) {
        const int a1 = 2 * ap1 + (j >> 1), a2 = 2 * ap2 + (j & 1);
        const XP xp = make_xp(ph, box_centre(a1, level), box_centre(a2, level));
        Gc[bbl][j][rr] = phase_dir(xp, ctc[bbl][rr], stc[bbl][rr]);
        if (rr < Q) Gb[bbl][j][rr] = phase_dir(xp, ctb[bbl][rr], stb[bbl][rr]);
    }
    lds_barrier();
    // first pass: the child index c2 is the same for a pair of waves (threads
    // [128 c2, 128 c2 + 128)), row (block, j, t1) within it, so the factors
    // M_c2[t2][t'2] are wave-uniform (scalar operands); second pass: thread
    // (c, t'2, half) of its block, r = c * 2q + h * q + t'2
    const int fc2 = __builtin_amdgcn_readfirstlane(tid / (NT / 2)), fi = tid - fc2 * (NT / 2);
    const int fb = fi / (4 * Q), fk = fi - fb * (4 * Q), fj = fk / Q, t1 = fk - fj * Q;
    const size_t fblk = (size_t)blockIdx.x * BPW + fb;
    const bool factive = fb < BPW && fblk < nblk;
    uint32_t fmB = 0, fmAp = 0;
    if (factive) {
        fmB = (uint32_t)(fblk & (nBl - 1));
        fmAp = (uint32_t)(fblk >> (2 * lB));
    }
    const int c = r / (2 * Q), k = r - c * 2 * Q;
    const int h = k / Q, tp2 = k - h * Q;
    const int c1 = c >> 1, c2 = c & 1;
    // exponentials shared by all right-hand sides
    cpx<T> E1[Q], E2[4][H1];
    const double rhoB = factive ? rb[fb][t1] : 0.0;
    if (HOIST && factive) {
#pragma unroll
        for (int t2 = 0; t2 < Q; ++t2) E1[t2] = cis<T>(rhoB * Gb[fb][fj][t2]);
    }
    if (HOIST && active) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const double G = Gc[bbl][jj][c2 * Q + tp2];
#pragma unroll
            for (int kk = 0; kk < H1; ++kk) E2[jj][kk] = cis<T>(rc[bbl][c1 * Q + min(h * H1 + kk, Q - 1)] * G);
        }
    }
    // inputs of the thread's row, loaded one right-hand side ahead
    cpx<T> nx[Q];
    auto load_row = [&](int ri) {
        const cpx<T> *src = win + ri * plane + ((size_t)(4 * fmAp + fj) * nBl + fmB) * QQ + t1 * Q;
#pragma unroll
        for (int t2 = 0; t2 < Q; ++t2) nx[t2] = src[t2];
    };
    constexpr bool PF = HOIST && !(sizeof(T) == 8 && Q > 10);  // prefetch unless it spills
    if (PF && factive) load_row(0);
    for (int ri = 0; ri < (HOIST ? nrhs : 1); ++ri) {
        if (factive) {
            if (!PF) load_row(ri);
            cpx<T> in[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) in[k] = nx[k];
            cpx<T> acc[Q];
#pragma unroll
            for (int t = 0; t < Q; ++t) acc[t] = {(T)0, (T)0};
#pragma unroll
            for (int t2 = 0; t2 < Q; ++t2) {
                const cpx<T> gv = cmul(in[t2], HOIST ? E1[t2] : cis<T>(rhoB * Gb[fb][fj][t2]));
#pragma unroll
                for (int p2 = 0; p2 < Q; ++p2) crfma(acc[p2], Mg[(fc2 * Q + t2) * Q + p2], gv);
            }
#pragma unroll
            for (int p2 = 0; p2 < Q; ++p2) Y[fb][fc2][fj][t1 * Q + p2] = acc[p2];
        }
        lds_barrier();
        // the next right-hand side's row is loaded during the (longer) second
        // pass (issuing it before the first pass measured slower)
        if (PF && factive && ri + 1 < nrhs) load_row(ri + 1);
        if (active) {
            cpx<T> acc[H1];
#pragma unroll
            for (int kk = 0; kk < H1; ++kk) acc[kk] = {(T)0, (T)0};
#pragma unroll(HOIST ? 4 : 1)
            for (int jj = 0; jj < 4; ++jj) {
                cpx<T> col[Q];
#pragma unroll
                for (int tt = 0; tt < Q; ++tt) col[tt] = Y[bbl][c2][jj][tt * Q + tp2];
                const double G = Gc[bbl][jj][c2 * Q + tp2];
#pragma unroll
                for (int kk = 0; kk < H1; ++kk) {
                    const int tp1 = min(h * H1 + kk, Q - 1);
                    cpx<T> z = {(T)0, (T)0};
#pragma unroll
                    for (int tt = 0; tt < Q; ++tt) crfma(z, Ms[c1][tt][tp1], col[tt]);
                    const cpx<T> add = cmulc(z, HOIST ? E2[jj][kk] : cis<T>(rc[bbl][c1 * Q + tp1] * G));
                    acc[kk].re += add.re;
                    acc[kk].im += add.im;
                }
            }
            cpx<T> *dst = wout + ri * plane + (blk * 4 + c) * QQ;
#pragma unroll
            for (int kk = 0; kk < H1; ++kk) {
                const int tp1 = h * H1 + kk;
                if (tp1 < Q) dst[tp1 * Q + tp2] = acc[kk];
            }
        }
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
        constexpr int BPW = blocks_per_wg<T, Q, 8 * (xadj_split<T, Q>() ? 2 : 1)>();               \
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
