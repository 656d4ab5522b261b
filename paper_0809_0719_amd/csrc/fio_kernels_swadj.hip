// Adjoint switch (the conjugate transpose of eq:alg2m) for batches of
// right-hand sides on the matrix cores, complex64.
//
// For a pair (A, B) at the switch level the polar nodes of B are
// p_s = (rho0 + h_s1, theta_s2) with h_{q-1-j} = -h_j (Chebyshev symmetry), and
// with G(t, s2) = Phi(x^A_t, e(theta_s2)) homogeneity gives
//     E(x^A_t, p_s) = b(t, s2) d_s1(t, s2),  b = e^{2 pi i rho0 G},  d_j = e^{2 pi i h_j G},
// d_{q-1-j} = conj d_j and d_H = 1 for odd q (H = floor(q/2)).  The adjoint
//     delta'_s = sum_t conj E(x^A_t, p_s) delta_t
// is therefore, for each direction node s2 and with y_t = conj b(t, s2) delta_t,
//     delta'_(j, s2)     = P_j - i Q_j,   delta'_(q-1-j, s2) = P_j + i Q_j,
//     delta'_(H, s2)     = sum_t y_t (odd q),
//     P_j = sum_t Re d_j(t, s2) y_t,   Q_j = sum_t Im d_j(t, s2) y_t:
// a real (q x q^2) matrix R_s2 = [Re d_j; Im d_j; 1] times the (q^2 x nrhs)
// complex matrix y.  That product runs as v_mfma_f32_16x16x4_f32 tiles: rows
// k of R (q <= 16, one tile), reduction over t in steps of 4, columns the
// real and imaginary parts of 8 right-hand sides per wave.
//
// A workgroup (4 waves) takes 16 (pair, 64-RHS chunk) items in turn, each as
// two halves of 32 right-hand sides.  Per half: the weights are staged
// through LDS (coalesced rows in, then each lane keeps its operand column,
// q^2/4 values, in registers for all q direction nodes), the outputs of
// every s2 go back to the staging buffer and leave as coalesced rows; the
// tables R and conj b (one phase and 1 + floor(q/2) exponentials per (t, s2),
// as in the vector kernel) are built in LDS once per pair.  The next half's
// weights are loaded into registers while the current one computes.  In
// place: a half's stores go to the rows its own loads read.  The forward
// switch below shares the tables, the items and the staging.
//
// MFMA lane layout (16x16x4, 64 lanes): A operand lane l holds A[l%16][l/16],
// B operand B[l/16][l%16], accumulator element v of lane l is D[4(l/16)+v][l%16].
#include <hip/hip_runtime.h>

#include "fio_kernels_common.h"

namespace fio {

namespace {

using f32x4 = __attribute__((ext_vector_type(4))) float;

constexpr int SA_RC = 64;   // right-hand sides per item (16 per wave)

template <int Q>
constexpr int sa_srow() { return (Q * Q) | 1; }  // odd row stride (complex) of the staging buffer
template <int Q>
constexpr int sa_kt() { return (Q * Q + 3) / 4; }  // reduction steps over t
template <int Q>
constexpr int sa_lpt() { return (SA_RC * Q * Q + NT - 1) / NT; }  // staged values per thread

}  // namespace

bool switch_adj_mfma_supported(int q, int nrhs) { return q >= QMIN && q <= 9 && nrhs >= 32; }

// The adjoint takes each item in two halves of 32 right-hand sides (8 per
// wave, real and imaginary parts of one right-hand side in adjacent columns,
// so a lane forms only its part of y), with the pair's tables built once for
// both halves: the smaller staging buffer lets three workgroups share a CU.
constexpr int SH_RC = SA_RC / 2;  // right-hand sides per half item

template <int Q>
constexpr int sh_lpt() { return (SH_RC * Q * Q + NT - 1) / NT; }

template <int Q, int PPW>
__global__ __launch_bounds__(NT, 3) void k_switch_adj_mm(Geom g, PhaseDev ph, Tables tb, cpx<float> *__restrict__ w,
                                                         int nrhs, size_t plane, size_t nitems, int nchunk) {
    constexpr int QQ = Q * Q, H = Q / 2;
    constexpr int KT = sa_kt<Q>(), SROW = sa_srow<Q>(), LPT = sh_lpt<Q>();
    __shared__ float Rt[Q][QQ][Q];          // [s2][t][k]: Re d_j (k = 2j), Im d_j (k = 2j + 1), 1 (k = 2H)
    __shared__ cpx<float> Bt[Q][QQ];        // conj b(t, s2)
    __shared__ cpx<float> stage[SH_RC][SROW];
    __shared__ double sx[2][Q], cx[2][Q], cth[Q], sth[Q];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lo = lane & 15, hi = lane >> 4;
    const int lA = g.lm, lB = g.L - g.lm;
    const size_t nBl = (size_t)1 << (2 * lB);
    // half items h = 2 item + half; a workgroup takes 2 PPW of them in turn
    const size_t nhalf = 2 * nitems;
    const size_t h0 = linear_block() * (2 * PPW);
    if (h0 >= nhalf) return;  // whole workgroup
    const int nh = (int)min((size_t)(2 * PPW), nhalf - h0);
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;
    double hz[H > 0 ? H : 1];
#pragma unroll
    for (int j = 0; j < H; ++j) hz[j] = g.rho_scale * ldexp(tb.z[j], -lB);

    // staged element e = tid + k NT = r q^2 + t of a half (right-hand side r,
    // node t), walked incrementally: NT = DR q^2 + DT
    constexpr int DR = NT / QQ, DT = NT - DR * QQ;
    const int r_0 = tid / QQ, t_0 = tid - r_0 * QQ;
    auto first_rhs = [&](size_t h, size_t &pair) {
        const size_t item = h >> 1;
        pair = item / nchunk;
        return (int)(item - pair * nchunk) * SA_RC + (int)(h & 1) * SH_RC;
    };
    cpx<float> pf[LPT];
    auto fetch = [&](size_t h) {
        size_t pair;
        const int q0 = first_rhs(h, pair);
        const cpx<float> *src = w + (size_t)(q0 + r_0) * plane + pair * QQ + t_0;
        int r = r_0, t = t_0;
#pragma unroll
        for (int k = 0; k < LPT; ++k) {
            pf[k] = (r < SH_RC && q0 + r < nrhs) ? *src : cpx<float>{0.f, 0.f};
            r += DR;
            t += DT;
            src += DR * plane + DT;
            if (t >= QQ) {
                t -= QQ;
                ++r;
                src += plane - QQ;
            }
        }
    };
    if (Q & 1)  // the middle row of R: d_H = 1 for every (s2, t)
        for (int i = tid; i < Q * QQ; i += NT) (&Rt[0][0][0])[i * Q + 2 * H] = 1.f;
    // this lane's column: right-hand side rl of the half, part 0 (real) or 1
    // (imaginary); its row k = lo of R (rows k >= q read row q - 1: they only
    // feed accumulator rows that are never stored)
    const int rl = 8 * wv + (lo >> 1), part = lo & 1;
    const int kr = lo < Q ? lo : Q - 1;
    fetch(h0);
    size_t built = ~(size_t)0;  // the pair whose tables are in LDS
    for (int ih = 0; ih < nh; ++ih) {
        const size_t h = h0 + ih;
        size_t pair;
        const int q0 = first_rhs(h, pair);

        lds_barrier();  // the previous half's stores (and, for a new pair, table readers) are done
        {
            int r = r_0, t = t_0;
#pragma unroll
            for (int k = 0; k < LPT; ++k) {
                if (r < SH_RC) stage[r][t] = pf[k];
                r += DR;
                t += DT;
                if (t >= QQ) {
                    t -= QQ;
                    ++r;
                }
            }
        }
        if (ih + 1 < nh) fetch(h + 1);
        const bool newpair = pair != built;  // uniform
        built = pair;
        const uint32_t mB = (uint32_t)(pair & (nBl - 1)), mA = (uint32_t)(pair >> (2 * lB));
        int b1, b2, a1, a2;
        morton_decode(mB, b1, b2);
        morton_decode(mA, a1, a2);
        if (newpair) {
            if (tid < 2 * Q) {  // A's nodes per dimension
                const int d = tid / Q, t = tid - d * Q;
                double s_ = 0, c_ = 1;
                if (ell) sincospi(2.0 * box_node(d ? a2 : a1, lA, tb.z[t]), &s_, &c_);
                sx[d][t] = s_;
                cx[d][t] = c_;
            } else if (tid < 3 * Q) {  // B's direction nodes
                const int t = tid - 2 * Q;
                double s_, c_;
                sincospi(2.0 * box_node(b2, lB, tb.z[t]), &s_, &c_);
                cth[t] = c_;
                sth[t] = s_;
            }
        }
        lds_barrier();  // the staged weights (and a new pair's node data) are complete
        if (newpair) {
            // thread (t, group of SG direction nodes): A's node data once per t
            constexpr int SG = (QQ * Q + NT - 1) / NT > 1 ? (Q + (NT / QQ) - 1) / (NT / QQ) : 1;
            const double r0 = g.rho_scale * box_centre(b1, lB);
            for (int i = tid; i < QQ * ((Q + SG - 1) / SG); i += NT) {
                const int sg = i / QQ, t = i - sg * QQ, t1 = t / Q, t2 = t - t1 * Q;
                const XP xp = make_xp_sc(ph, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]), sx[0][t1],
                                         cx[0][t1], sx[1][t2], cx[1][t2]);
#pragma unroll 1
                for (int u = 0; u < SG; ++u) {
                    const int s2 = sg * SG + u;
                    if (s2 < Q) {
                        const double G = phase_dir(xp, cth[s2], sth[s2]);
                        const cpx<float> b = cis<float>(r0 * G);
                        Bt[s2][t] = {b.re, -b.im};
#pragma unroll
                        for (int j = 0; j < H; ++j) {
                            const cpx<float> d = cis<float>(hz[j] * G);
                            Rt[s2][t][2 * j] = d.re;
                            Rt[s2][t][2 * j + 1] = d.im;
                        }
                    }
                }
            }
        }
        // this lane's weights d (right-hand side rl, nodes t = 4 ks + hi) as the
        // pair (dp, dq) with part(c d) = c.re dp + c.im dq: (d.re, -d.im) for
        // the real part, (d.im, d.re) for the imaginary part
        float dp[KT], dq[KT];
#pragma unroll
        for (int ks = 0; ks < KT; ++ks) {
            const int t = 4 * ks + hi;
            const cpx<float> d = t < QQ ? stage[rl][t] : cpx<float>{0.f, 0.f};
            dp[ks] = part ? d.im : d.re;
            dq[ks] = part ? d.re : -d.im;
        }
        lds_barrier();  // tables built; every operand read from the staging buffer is done
        float *const srow = &stage[rl][0].re;  // the lane's output row, as floats
#pragma unroll 1
        for (int s2 = 0; s2 < Q; ++s2) {
            f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KT; ++ks) {
                const int t = 4 * ks + hi, tc = t < QQ ? t : QQ - 1;
                const float a = Rt[s2][tc][kr];
                const cpx<float> c = Bt[s2][tc];  // y = c d, zero where t >= q^2
                const float y = fmaf(c.re, dp[ks], c.im * dq[ks]);
                z = __builtin_amdgcn_mfma_f32_16x16x4f32(a, y, z, 0, 0, 0);
            }
            // rows k = 4 hi + v of this lane's column: P_j (v = 0, 2) and Q_j
            // (v = 1, 3) in this lane's part; the partner lane holds the other
#pragma unroll
            for (int v = 0; v < 4; v += 2) {
                const int k = 4 * hi + v, j = k >> 1;
                const float qo = __shfl_xor(z[v + 1], 1);  // the other part of Q_j
                if (j < H) {
                    // real parts: P_j.re +- Q_j.im; imaginary parts: P_j.im -+ Q_j.re
                    const float p = z[v];
                    srow[2 * (j * Q + s2) + part] = part ? p - qo : p + qo;
                    srow[2 * ((Q - 1 - j) * Q + s2) + part] = part ? p + qo : p - qo;
                } else if ((Q & 1) && k == 2 * H) {
                    srow[2 * (H * Q + s2) + part] = z[v];
                }
            }
        }
        lds_barrier();
        {
            cpx<float> *dst = w + (size_t)(q0 + r_0) * plane + pair * QQ + t_0;
            int r = r_0, t = t_0;
#pragma unroll
            for (int k = 0; k < LPT; ++k) {
                if (r < SH_RC && q0 + r < nrhs) *dst = stage[r][t];
                r += DR;
                t += DT;
                dst += DR * plane + DT;
                if (t >= QQ) {
                    t -= QQ;
                    ++r;
                    dst += plane - QQ;
                }
            }
        }
    }
}

// Forward switch on the matrix cores, complex64: with the same R and
//     X_s2 = [S_j; i D_j; delta_H],  S_j = delta_(j, s2) + delta_(q-1-j, s2),
//     D_j = delta_(j, s2) - delta_(q-1-j, s2),
// delta'_t = sum_s2 b(t, s2) (R_s2 X_s2)_t: per direction node a real
// (q^2 x q) by complex (q x nrhs) product on the matrix cores (rows t padded
// to a multiple of 16, reduction k padded to a multiple of 4 with zero rows of
// X), then the remodulation by b and the sum over s2 on the vector ALUs, in
// registers.  Items, staging and prefetch as in the adjoint above; the staged
// inputs stay in LDS for the whole item (X is formed from them per node) and
// the outputs go back through the same buffer once every node is done.
bool switch_mfma_supported(int q, int nrhs) { return q >= QMIN && q <= 9 && nrhs >= 32; }

template <int Q, int PPW>
__global__ __launch_bounds__(NT, 2) void k_switch_mm(Geom g, PhaseDev ph, Tables tb, cpx<float> *__restrict__ w,
                                                     int nrhs, size_t plane, size_t nitems, int nchunk) {
    constexpr int QQ = Q * Q, H = Q / 2;
    constexpr int SROW = sa_srow<Q>(), LPT = sa_lpt<Q>();
    constexpr int TT = (QQ + 15) / 16;  // row tiles of t
    constexpr int KS = (Q + 3) / 4;     // reduction steps over k
    constexpr int TH = (TT + 1) / 2;    // row tiles per accumulator group
    __shared__ float Rt[Q][QQ][Q];      // [s2][t][k] as in the adjoint
    __shared__ cpx<float> Bt[Q][QQ];    // b(t, s2)
    __shared__ cpx<float> stage[SA_RC][SROW];
    __shared__ double sx[2][Q], cx[2][Q], cth[Q], sth[Q];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lo = lane & 15, hi = lane >> 4;
    const int lA = g.lm, lB = g.L - g.lm;
    const size_t nBl = (size_t)1 << (2 * lB);
    const size_t item0 = linear_block() * PPW;
    if (item0 >= nitems) return;  // whole workgroup
    const int nit = (int)min((size_t)PPW, nitems - item0);
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;
    double hz[H > 0 ? H : 1];
#pragma unroll
    for (int j = 0; j < H; ++j) hz[j] = g.rho_scale * ldexp(tb.z[j], -lB);

    constexpr int DR = NT / QQ, DT = NT - DR * QQ;
    const int r_0 = tid / QQ, t_0 = tid - r_0 * QQ;
    cpx<float> pf[LPT];
    auto fetch = [&](size_t item) {
        const size_t pair = item / nchunk;
        const int q0 = (int)(item - pair * nchunk) * SA_RC;
        const cpx<float> *src = w + (size_t)(q0 + r_0) * plane + pair * QQ + t_0;
        int r = r_0, t = t_0;
#pragma unroll
        for (int k = 0; k < LPT; ++k) {
            pf[k] = (r < SA_RC && q0 + r < nrhs) ? *src : cpx<float>{0.f, 0.f};
            r += DR;
            t += DT;
            src += DR * plane + DT;
            if (t >= QQ) {
                t -= QQ;
                ++r;
                src += plane - QQ;
            }
        }
    };
    if (Q & 1)  // the middle column of R: d_H = 1 for every (s2, t)
        for (int i = tid; i < Q * QQ; i += NT) (&Rt[0][0][0])[i * Q + 2 * H] = 1.f;
    // this lane's reduction rows k = 4 ks + hi of X: the pair j = k / 2 (S_j for
    // even k, i D_j for odd k), the middle row k = 2H, zero past q
    const int rl = 16 * wv + lo;
    fetch(item0);
    for (int it = 0; it < nit; ++it) {
        const size_t item = item0 + it, pair = item / nchunk;
        const int q0 = (int)(item - pair * nchunk) * SA_RC;
        const uint32_t mB = (uint32_t)(pair & (nBl - 1)), mA = (uint32_t)(pair >> (2 * lB));
        int b1, b2, a1, a2;
        morton_decode(mB, b1, b2);
        morton_decode(mA, a1, a2);

        lds_barrier();  // the previous item's stores and table readers are done
        {
            int r = r_0, t = t_0;
#pragma unroll
            for (int k = 0; k < LPT; ++k) {
                if (r < SA_RC) stage[r][t] = pf[k];
                r += DR;
                t += DT;
                if (t >= QQ) {
                    t -= QQ;
                    ++r;
                }
            }
        }
        if (it + 1 < nit) fetch(item + 1);
        if (tid < 2 * Q) {  // A's nodes per dimension
            const int d = tid / Q, t = tid - d * Q;
            double s_ = 0, c_ = 1;
            if (ell) sincospi(2.0 * box_node(d ? a2 : a1, lA, tb.z[t]), &s_, &c_);
            sx[d][t] = s_;
            cx[d][t] = c_;
        } else if (tid < 3 * Q) {  // B's direction nodes
            const int t = tid - 2 * Q;
            double s_, c_;
            sincospi(2.0 * box_node(b2, lB, tb.z[t]), &s_, &c_);
            cth[t] = c_;
            sth[t] = s_;
        }
        lds_barrier();
        {
            constexpr int SG = (QQ * Q + NT - 1) / NT > 1 ? (Q + (NT / QQ) - 1) / (NT / QQ) : 1;
            const double r0 = g.rho_scale * box_centre(b1, lB);
            for (int i = tid; i < QQ * ((Q + SG - 1) / SG); i += NT) {
                const int sg = i / QQ, t = i - sg * QQ, t1 = t / Q, t2 = t - t1 * Q;
                const XP xp = make_xp_sc(ph, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]), sx[0][t1],
                                         cx[0][t1], sx[1][t2], cx[1][t2]);
#pragma unroll 1
                for (int u = 0; u < SG; ++u) {
                    const int s2 = sg * SG + u;
                    if (s2 < Q) {
                        const double G = phase_dir(xp, cth[s2], sth[s2]);
                        Bt[s2][t] = cis<float>(r0 * G);
#pragma unroll
                        for (int j = 0; j < H; ++j) {
                            const cpx<float> d = cis<float>(hz[j] * G);
                            Rt[s2][t][2 * j] = d.re;
                            Rt[s2][t][2 * j + 1] = d.im;
                        }
                    }
                }
            }
        }
        lds_barrier();  // tables built
        cpx<float> acc[TT][4];
#pragma unroll
        for (int tt = 0; tt < TT; ++tt)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[tt][v] = {0.f, 0.f};
#pragma unroll 1
        for (int s2 = 0; s2 < Q; ++s2) {
            // B operand: X[k][rl] for k = 4 ks + hi
            float xr[KS], xi[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int k = 4 * ks + hi, j = k >> 1;
                const int ja = j < H ? j : H, jb = j < H ? Q - 1 - j : H;  // (H, H): the middle row
                const cpx<float> da = stage[rl][ja * Q + s2], db = stage[rl][jb * Q + s2];
                float vr, vi;
                if (k < 2 * H) {
                    if (k & 1) {  // i D_j
                        vr = db.im - da.im;
                        vi = da.re - db.re;
                    } else {  // S_j
                        vr = da.re + db.re;
                        vi = da.im + db.im;
                    }
                } else {
                    const bool mid = (Q & 1) && k == 2 * H;
                    vr = mid ? da.re : 0.f;
                    vi = mid ? da.im : 0.f;
                }
                xr[ks] = vr;
                xi[ks] = vi;
            }
            // row tiles in groups of TH (fewer accumulators live at once)
#pragma unroll
            for (int t0 = 0; t0 < TT; t0 += TH) {
                f32x4 zr[TH], zi[TH];
#pragma unroll
                for (int u = 0; u < TH; ++u) zr[u] = zi[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    // A operand R[t][k] for t = 16 tt + lo, k = 4 ks + hi: clamped reads
                    // (rows t >= q^2 feed accumulator rows that are never used; columns
                    // k >= q meet zero rows of X)
                    const int kc = 4 * ks + hi < Q ? 4 * ks + hi : Q - 1;
#pragma unroll
                    for (int u = 0; u < TH; ++u) {
                        if (t0 + u < TT) {
                            const int t = 16 * (t0 + u) + lo, tc = t < QQ ? t : QQ - 1;
                            const float a = Rt[s2][tc][kc];
                            zr[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, xr[ks], zr[u], 0, 0, 0);
                            zi[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, xi[ks], zi[u], 0, 0, 0);
                        }
                    }
                }
                // remodulate: rows t = 16 tt + 4 hi + v of column rl
#pragma unroll
                for (int u = 0; u < TH; ++u)
                    if (t0 + u < TT) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int t = 16 * (t0 + u) + 4 * hi + v, tc = t < QQ ? t : QQ - 1;
                            cfma(acc[t0 + u][v], Bt[s2][tc], cpx<float>{zr[u][v], zi[u][v]});
                        }
                    }
            }
        }
        lds_barrier();  // every read of the staged inputs is done
#pragma unroll
        for (int tt = 0; tt < TT; ++tt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int t = 16 * tt + 4 * hi + v;
                if (t < QQ) stage[rl][t] = acc[tt][v];
            }
        lds_barrier();
        {
            cpx<float> *dst = w + (size_t)(q0 + r_0) * plane + pair * QQ + t_0;
            int r = r_0, t = t_0;
#pragma unroll
            for (int k = 0; k < LPT; ++k) {
                if (r < SA_RC && q0 + r < nrhs) *dst = stage[r][t];
                r += DR;
                t += DT;
                dst += DR * plane + DT;
                if (t >= QQ) {
                    t -= QQ;
                    ++r;
                    dst += plane - QQ;
                }
            }
        }
    }
}

bool switch_ppw_supported(int ppw) { return ppw == 8 || ppw == 16 || ppw == 32; }

hipError_t launch_switch_mfma(const Geom &g, const PhaseDev &ph, const Tables &tb, void *w, int nrhs,
                              size_t plane, hipStream_t st) {
    if (!switch_mfma_supported(g.q, nrhs) || !switch_ppw_supported(g.sw_ppw)) return hipErrorInvalidValue;
    const size_t npairs = (size_t)1 << (2 * g.L);
    const int nchunk = (nrhs + SA_RC - 1) / SA_RC;
    const size_t nitems = npairs * (size_t)nchunk;
    const size_t nblk = (nitems + g.sw_ppw - 1) / g.sw_ppw;
#define L_SFP(Q, P)                                                                                           \
    hipLaunchKernelGGL((k_switch_mm<Q, P>), grid_of(nblk), dim3(NT), 0, st, g, ph, tb, (cpx<float> *)w, nrhs, \
                       plane, nitems, nchunk);
#define L_SFM(Q)                                   \
    {                                              \
        if (g.sw_ppw == 8) L_SFP(Q, 8)             \
        else if (g.sw_ppw == 16) L_SFP(Q, 16)      \
        else L_SFP(Q, 32)                          \
    }
    switch (g.q) {
        case 3: L_SFM(3) break;
        case 4: L_SFM(4) break;
        case 5: L_SFM(5) break;
        case 6: L_SFM(6) break;
        case 7: L_SFM(7) break;
        case 8: L_SFM(8) break;
        case 9: L_SFM(9) break;
        default: return hipErrorInvalidValue;
    }
#undef L_SFM
#undef L_SFP
    return hipGetLastError();
}

hipError_t launch_switch_adj_mfma(const Geom &g, const PhaseDev &ph, const Tables &tb, void *w, int nrhs,
                                  size_t plane, hipStream_t st) {
    if (!switch_adj_mfma_supported(g.q, nrhs) || !switch_ppw_supported(g.sw_ppw)) return hipErrorInvalidValue;
    const size_t npairs = (size_t)1 << (2 * g.L);
    const int nchunk = (nrhs + SA_RC - 1) / SA_RC;
    const size_t nitems = npairs * (size_t)nchunk;
    const size_t nblk = (nitems + g.sw_ppw - 1) / g.sw_ppw;
#define L_SAP(Q, P)                                                                                               \
    hipLaunchKernelGGL((k_switch_adj_mm<Q, P>), grid_of(nblk), dim3(NT), 0, st, g, ph, tb, (cpx<float> *)w, nrhs, \
                       plane, nitems, nchunk);
#define L_SAM(Q)                                   \
    {                                              \
        if (g.sw_ppw == 8) L_SAP(Q, 8)             \
        else if (g.sw_ppw == 16) L_SAP(Q, 16)      \
        else L_SAP(Q, 32)                          \
    }
    switch (g.q) {
        case 3: L_SAM(3) break;
        case 4: L_SAM(4) break;
        case 5: L_SAM(5) break;
        case 6: L_SAM(6) break;
        case 7: L_SAM(7) break;
        case 8: L_SAM(8) break;
        case 9: L_SAM(9) break;
        default: return hipErrorInvalidValue;
    }
#undef L_SAM
#undef L_SAP
    return hipGetLastError();
}

}  // namespace fio
