// Forward-mode derivatives of the butterfly with respect to the phase's
// velocity scalings (a1, a2): every kernel here carries three weight planes
// through one step of Sec. 4 -- the primal delta and its derivatives
// d delta / d a1, d delta / d a2 -- sharing the kernel values.  A kernel
// value E = exp(2 pi i Phi) contributes dE/da = 2 pi i (dPhi/da) E, so a
// step out = F(in) with factors E gives
//     d out = F(d in) + (the same step with one E replaced by dE/da) (in),
// summed over its factors (product rule).  The weights are recomputed for
// every call, never stored.
//
// For the ellipse phase Phi(x, e) = x.e + sqrt(C1 e1^2 + C2 e2^2) with
// C_j = (a_j c_j(x))^2: dPhi/da1 = C1 e1^2 / (a1 sqrt(.)), dPhi/da2 =
// C2 e2^2 / (a2 sqrt(.)); the Fourier phase does not depend on a (C = 0).
#include <hip/hip_runtime.h>

#include "fio_kernels_common.h"

namespace fio {

struct G3 {
    double g, d1, d2;  // Phi and its derivatives with respect to a1, a2
};

__device__ __forceinline__ G3 phase_dir3(const XP &x, const PhaseDev &ph, double ct, double st) {
    const double S = sqrt(fma(x.C1 * ct, ct, x.C2 * st * st));
    G3 r;
    r.g = fma(x.x1, ct, x.x2 * st) + S;
    r.d1 = (S > 0.0 && x.C1 > 0.0) ? x.C1 * ct * ct / (ph.a1 * S) : 0.0;
    r.d2 = (S > 0.0 && x.C2 > 0.0) ? x.C2 * st * st / (ph.a2 * S) : 0.0;
    return r;
}

__device__ __forceinline__ G3 phase_cart3(const XP &x, const PhaseDev &ph, double k1, double k2) {
    const double S = sqrt(fma(x.C1 * k1, k1, x.C2 * k2 * k2));
    G3 r;
    r.g = fma(x.x1, k1, x.x2 * k2) + S;
    r.d1 = (S > 0.0 && x.C1 > 0.0) ? x.C1 * k1 * k1 / (ph.a1 * S) : 0.0;
    r.d2 = (S > 0.0 && x.C2 > 0.0) ? x.C2 * k2 * k2 / (ph.a2 * S) : 0.0;
    return r;
}

// 2 pi i phi z
template <typename T>
__device__ __forceinline__ cpx<T> i2pi(double phi, cpx<T> z) {
    const T s = (T)(6.283185307179586476925286766559 * phi);
    return {-s * z.im, s * z.re};
}
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) {
    return {a.re - b.re, a.im - b.im};
}

// Sources per chunk in the tangent initialisation: 64 (a whole box B at
// s = 3, on average) where the chunk's products for all ACH boxes A fit in
// 48 KB of LDS, else 32 or 16.  A chunk costs one pass of Lagrange rows and
// three workgroup barriers.
template <typename T, int Q>
constexpr int init_tan_sct() {
    constexpr int ACH = (NT / Q) < 64 ? (NT / Q) : 64;
    constexpr int per = 3 * ACH * 2 * (int)sizeof(T);
    return 64 * per <= 48 * 1024 ? 64 : 32 * per <= 48 * 1024 ? 32 : 16;
}

// ===========================================================================
// initialisation (eq:alg2a) with derivatives:
//   out   = conj Er . acc0,  acc0 = sum_p L(p) E(x0,p) f(p)
//   d out = conj Er . acc_k - 2 pi i rho dG_k . out,  acc_k = sum_p L(p) 2 pi i dPhi_k(x0,p) E(x0,p) f(p)
// ===========================================================================
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_init_tan(Geom g, PhaseDev ph, Tables tb, Sources src,
                                                 const cpx<T> *__restrict__ f, cpx<T> *__restrict__ w,
                                                 size_t plane) {
    constexpr int ACH = (NT / Q) < 64 ? (NT / Q) : 64;
    constexpr int SCT = init_tan_sct<T, Q>();
    __shared__ T lag1[SCT][Q];
    __shared__ T lag2[SCT][Q];
    __shared__ cpx<T> gA[3][ACH][SCT];
    __shared__ double2 kk[SCT];
    __shared__ cpx<T> fs[SCT];
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

    cpx<T> acc[3][Q];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int t = 0; t < Q; ++t) acc[k][t] = {(T)0, (T)0};

    const int beg = src.off[mB], end = src.off[mB + 1];
    __syncthreads();
    for (int c0 = beg; c0 < end; c0 += SCT) {
        const int n = min(SCT, end - c0);
        // the two Lagrange rows of a source on two threads (SCT <= 64 < NT / 2)
        if (tid < n) {
            const int j = c0 + tid;
            const int idx = src.idx[j];
            const double2 p = src.p[j];
            lagrange_row<T, Q>(p.x * scale - ((double)bp1 + 0.5), zs, ls, lag1[tid]);
            kk[tid] = make_double2((double)(idx / g.N - g.N / 2), (double)(idx % g.N - g.N / 2));
            fs[tid] = f[idx];
        } else if (tid >= 64 && tid < 64 + n) {
            const double2 p = src.p[c0 + tid - 64];
            lagrange_row<T, Q>(p.y * scale - ((double)bp2 + 0.5), zs, ls, lag2[tid - 64]);
        }
        __syncthreads();
        for (int it = tid; it < nAc * n; it += NT) {
            const int al = it / n, jj = it - al * n;
            const G3 ph3 = phase_cart3(xA[al], ph, kk[jj].x, kk[jj].y);
            const cpx<T> g0 = cmul(cis<T>(ph3.g), fs[jj]);
            gA[0][al][jj] = g0;
            gA[1][al][jj] = i2pi(ph3.d1, g0);
            gA[2][al][jj] = i2pi(ph3.d2, g0);
        }
        __syncthreads();
        if (active) {
            for (int jj = 0; jj < n; ++jj) {
                const T l1 = lag1[jj][t1];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const cpx<T> gv = gA[k][aL][jj];
                    const cpx<T> h = {l1 * gv.re, l1 * gv.im};
#pragma unroll
                    for (int t2 = 0; t2 < Q; ++t2) crfma(acc[k][t2], lag2[jj][t2], h);
                }
            }
        }
        __syncthreads();
    }
    if (!active) return;
    const uint32_t mA = a0 + aL;
    const XP xp = xA[aL];
    const double rho = g.rho_scale * box_node(bp1, lB, zs[t1]);
    cpx<T> *out = w + ((size_t)mA * ((size_t)1 << (2 * lB)) + mB) * (Q * Q) + t1 * Q;
#pragma unroll
    for (int t2 = 0; t2 < Q; ++t2) {
        double st, ct;
        sincospi(2.0 * box_node(bp2, lB, zs[t2]), &st, &ct);
        const G3 gr = phase_dir3(xp, ph, ct, st);
        const cpx<T> e = cis<T>(rho * gr.g);
        const cpx<T> o0 = cmulc(acc[0][t2], e);
        out[t2] = o0;
        out[plane + t2] = csub(cmulc(acc[1][t2], e), i2pi(rho * gr.d1, o0));
        out[2 * plane + t2] = csub(cmulc(acc[2][t2], e), i2pi(rho * gr.d2, o0));
    }
}

// A thread's elements tid + n NT (n < ceil(NE / NT)) of three planes `plane`
// values apart: every load is issued (indices past NE clamped to NE - 1, so
// no element is conditional), their waits fall where the values are used.
template <typename T, int NE, int NP = (NE + NT - 1) / NT>
__device__ __forceinline__ void fetch_planes(cpx<T> (&d)[3][NP], const cpx<T> *src, size_t plane, int tid) {
#pragma unroll
    for (int n = 0; n < NP; ++n) {
        const int i = min(tid + n * NT, NE - 1);
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k][n] = src[k * plane + i];
    }
}

// Outputs (children j) a tangent level kernel takes per pass: two while two
// workgroups still share a CU's 160 KB of LDS, else one.  Two halve the
// workgroup barriers per right-hand side and keep about twice the threads
// busy in every pass (at q = 9, FP32: 52 KB, three workgroups per CU, a third
// less time than one output per pass at four).
template <typename T, int Q>
constexpr int plevel_tan_lds(int jp) {
    constexpr int QQ = Q * Q, C = 2 * (int)sizeof(T), S = (int)sizeof(T);
    return jp * 18 * QQ * C + 20 * QQ * C + 40 * QQ * S + 9 * Q * 8 + 12 * Q * 24;
}
template <typename T, int Q>
constexpr int xlevel_tan_lds(int jp) {
    constexpr int QQ = Q * Q, C = 2 * (int)sizeof(T), S = (int)sizeof(T);
    return (12 + jp * 12) * QQ * C + 20 * QQ * C + 40 * QQ * S + 12 * Q * 8 + 6 * 8;
}
template <typename T, int Q>
constexpr int plevel_tan_jp() { return plevel_tan_lds<T, Q>(2) <= 80 * 1024 ? 2 : 1; }
template <typename T, int Q>
constexpr int xlevel_tan_jp() { return xlevel_tan_lds<T, Q>(2) <= 80 * 1024 ? 2 : 1; }

// ===========================================================================
// p-recursion (eq:alg2b) with derivatives, one workgroup per block (A_p, B),
// the four outputs one after another:
//   v   = Ep . in,       d v = Ep . (d in + 2 pi i dPhi_p . in)
//   out = conj Er . K v, d out = conj Er . K d v - 2 pi i dPhi_r . out
// The kernel values of the four outputs (Ep, Er and the factors
// 2 pi dPhi of the derivative terms) are made once per block in LDS and
// serve nrhs right-hand sides, whose three planes start rstride values apart.
// ===========================================================================
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_plevel_tan(Geom g, PhaseDev ph, Tables tb, int level,
                                                   const cpx<T> *__restrict__ win,
                                                   cpx<T> *__restrict__ wout, size_t plane, int nrhs,
                                                   size_t rstride) {
    constexpr int QQ = Q * Q;
    constexpr double TWO_PI = 6.283185307179586476925286766559;
    constexpr int JP = plevel_tan_jp<T, Q>();
    __shared__ cpx<T> v[JP][3][4 * QQ];
    __shared__ cpx<T> W[JP][3][2 * QQ];
    __shared__ double rc[2 * Q], ctc[2 * Q], stc[2 * Q];
    __shared__ double rb[Q], ctb[Q], stb[Q];
    __shared__ G3 Gc[4][2 * Q], Gb[4][Q];
    __shared__ cpx<T> Ep[4][4 * QQ];  // E(x0(A_j), p^{B_c}_t')
    __shared__ T Sp[2][4][4 * QQ];    // 2 pi rho dPhi_k(x0(A_j), .) at p^{B_c}_t'
    __shared__ cpx<T> Er[4][QQ];      // E(x0(A_j), p^B_t)
    __shared__ T Sr[2][4][QQ];

    const int tid = threadIdx.x;
    const int lB = g.L - level;
    const size_t blk = linear_block();  // exact grid: the block count is a power of two
    const size_t nBl = (size_t)1 << (2 * lB);
    const uint32_t mB = (uint32_t)(blk & (nBl - 1));
    const uint32_t mAp = (uint32_t)(blk >> (2 * lB));
    int b1, b2, ap1, ap2;
    morton_decode(mB, b1, b2);
    morton_decode(mAp, ap1, ap2);

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
    // kernel values of the four outputs, all four at once
    for (int it = tid; it < 4 * 3 * Q; it += NT) {
        const int j = it / (3 * Q), u = it - j * (3 * Q);
        const int a1 = 2 * ap1 + (j >> 1), a2 = 2 * ap2 + (j & 1);
        const XP xp = make_xp(ph, box_centre(a1, level), box_centre(a2, level));
        if (u < 2 * Q)
            Gc[j][u] = phase_dir3(xp, ph, ctc[u], stc[u]);
        else
            Gb[j][u - 2 * Q] = phase_dir3(xp, ph, ctb[u - 2 * Q], stb[u - 2 * Q]);
    }
    __syncthreads();
    for (int it = tid; it < 4 * 4 * QQ; it += NT) {
        const int j = it / (4 * QQ), i = it - j * (4 * QQ);
        const int c = i / QQ, t = i - c * QQ;
        const int c1 = c >> 1, c2 = c & 1;
        const int tp1 = t / Q, tp2 = t - tp1 * Q;
        const double rho = rc[c1 * Q + tp1];
        const G3 gg = Gc[j][c2 * Q + tp2];
        Ep[j][i] = cis<T>(rho * gg.g);
        Sp[0][j][i] = (T)(TWO_PI * (rho * gg.d1));
        Sp[1][j][i] = (T)(TWO_PI * (rho * gg.d2));
    }
    for (int it = tid; it < 4 * QQ; it += NT) {
        const int j = it / QQ, i = it - j * QQ;
        const int t1 = i / Q, t2 = i - t1 * Q;
        const G3 gg = Gb[j][t2];
        Er[j][i] = cis<T>(rb[t1] * gg.g);
        Sr[0][j][i] = (T)(TWO_PI * (rb[t1] * gg.d1));
        Sr[1][j][i] = (T)(TWO_PI * (rb[t1] * gg.d2));
    }
    __syncthreads();
    // the two contractions go row by row: a thread loads one row of its
    // operand into registers once and makes a run of outputs from it, with
    // the interpolation matrix read through the scalar cache (wave-uniform
    // offsets).  JP outputs j = JP jp + jj per pass.  Pass 1, rows
    // (jj, k, c1, t'1), outputs t2 in half (w & 1); pass 2, rows (jj, k, t2),
    // outputs t1 in quarter w.
    constexpr int HA = (Q + 1) / 2, HB = (Q + 3) / 4, NPT = (4 * QQ + NT - 1) / NT;
    cptr<T> Mg = to_constant(pick_M<T>(tb));
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    // a thread's share of the block's three input planes sits in registers,
    // the next right-hand side's loads in flight while this one computes
    cpx<T> xin[3][NPT], xnx[3][NPT];
    fetch_planes<T, 4 * QQ>(xin, win + blk * (4 * QQ), plane, tid);
    for (int r = 0; r < nrhs; ++r) {
        fetch_planes<T, 4 * QQ>(xnx, win + (size_t)min(r + 1, nrhs - 1) * rstride + blk * (4 * QQ), plane, tid);
        for (int jp = 0; jp < 4 / JP; ++jp) {
            opaque_sgpr(Mg);
#pragma unroll
            for (int n = 0; n < NPT; ++n) {
                const int i = tid + n * NT;
                if (i < 4 * QQ) {
                    const cpx<T> in0 = xin[0][n];
#pragma unroll
                    for (int jj = 0; jj < JP; ++jj) {
                        const int j = JP * jp + jj;
                        const cpx<T> e = Ep[j][i];
                        const T s1 = Sp[0][j][i], s2 = Sp[1][j][i];
                        v[jj][0][i] = cmul(e, in0);
                        v[jj][1][i] = cmul(e, cadd(xin[1][n], cpx<T>{-s1 * in0.im, s1 * in0.re}));
                        v[jj][2][i] = cmul(e, cadd(xin[2][n], cpx<T>{-s2 * in0.im, s2 * in0.re}));
                    }
                }
            }
            __syncthreads();
            // W[k][c1][t'1][t2] = sum_{c2, t'2} M_c2[t2][t'2] v[k][2 c1 + c2][t'1][t'2]
            with_uniform<0, 2>(w & 1, [&](auto hc) {
                constexpr int t0 = decltype(hc)::value * HA, nt = Q - t0 < HA ? Q - t0 : HA;
                for (int row = (w >> 1) * 64 + lane; row < JP * 6 * Q; row += 128) {
                    const int jj = row / (6 * Q), rj = row - jj * 6 * Q;
                    const int k = rj / (2 * Q), rem = rj - k * 2 * Q;
                    const int c1 = rem / Q, tp1 = rem - c1 * Q;
                    cpx<T> acc[nt];
#pragma unroll
                    for (int u = 0; u < nt; ++u) acc[u] = {(T)0, (T)0};
#pragma unroll
                    for (int c2 = 0; c2 < 2; ++c2) {
                        const cpx<T> *vv = v[jj][k] + (2 * c1 + c2) * QQ + tp1 * Q;
#pragma unroll
                        for (int tp2 = 0; tp2 < Q; ++tp2) {
                            const cpx<T> x = vv[tp2];
#pragma unroll
                            for (int u = 0; u < nt; ++u) crfma(acc[u], Mg[c2 * QQ + (t0 + u) * Q + tp2], x);
                        }
                    }
                    cpx<T> *ww = W[jj][k] + c1 * QQ + tp1 * Q + t0;
#pragma unroll
                    for (int u = 0; u < nt; ++u) ww[u] = acc[u];
                }
            });
            __syncthreads();
            // o[k][t1][t2] = sum_{c1, t'1} M_c1[t1][t'1] W[k][c1][t'1][t2], into v[jj][k][0, QQ)
            with_uniform<0, 4>(w, [&](auto pc) {
                constexpr int t0 = decltype(pc)::value * HB;
                constexpr int nt = Q - t0 >= HB ? HB : (Q - t0 > 0 ? Q - t0 : 0);
                if constexpr (nt > 0) {
                    for (int row = lane; row < JP * 3 * Q; row += 64) {
                        const int jj = row / (3 * Q), rj = row - jj * 3 * Q;
                        const int k = rj / Q, t2 = rj - k * Q;
                        cpx<T> acc[nt];
#pragma unroll
                        for (int u = 0; u < nt; ++u) acc[u] = {(T)0, (T)0};
#pragma unroll
                        for (int c1 = 0; c1 < 2; ++c1) {
#pragma unroll
                            for (int tp1 = 0; tp1 < Q; ++tp1) {
                                const cpx<T> x = W[jj][k][c1 * QQ + tp1 * Q + t2];
#pragma unroll
                                for (int u = 0; u < nt; ++u) crfma(acc[u], Mg[c1 * QQ + (t0 + u) * Q + tp1], x);
                            }
                        }
#pragma unroll
                        for (int u = 0; u < nt; ++u) v[jj][k][(t0 + u) * Q + t2] = acc[u];
                    }
                }
            });
            __syncthreads();
            for (int it = tid; it < JP * QQ; it += NT) {
                const int jj = it / QQ, i = it - jj * QQ;
                const int j = JP * jp + jj;
                cpx<T> *dst = wout + r * rstride + ((size_t)(4 * mAp + j) * nBl + mB) * QQ;
                const cpx<T> e = Er[j][i];
                const cpx<T> o0 = cmulc(v[jj][0][i], e);
                const T s1 = Sr[0][j][i], s2 = Sr[1][j][i];
                dst[i] = o0;
                dst[plane + i] = csub(cmulc(v[jj][1][i], e), cpx<T>{-s1 * o0.im, s1 * o0.re});
                dst[2 * plane + i] = csub(cmulc(v[jj][2][i], e), cpx<T>{-s2 * o0.im, s2 * o0.re});
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int n = 0; n < NPT; ++n) xin[k][n] = xnx[k][n];
    }
}

// ===========================================================================
// switch (eq:alg2m) with derivatives, in place on three planes:
//   out   = sum_s E[t,s] in[s]
//   d out = sum_s E[t,s] (d in[s] + 2 pi i rho(s1) dG(x_t, theta_s2) in[s])
// With the same node symmetry as the forward switch; the derivative term
// uses the weighted plane in'(s) = rho(s1) in(s).
// ===========================================================================
template <typename T, int Q, bool HOLD>
__global__ __launch_bounds__(NT) void k_switch_tan(Geom g, PhaseDev ph, Tables tb, cpx<T> *__restrict__ w,
                                                   size_t plane, int nrhs, size_t rstride) {
    constexpr int QQ = Q * Q;
    constexpr int H = Q / 2;
    constexpr int HH = H > 0 ? H : 1;
    constexpr int PPB = NT / QQ;
    constexpr double TWO_PI = 6.283185307179586476925286766559;
    // HOLD (FP32, a chunk of right-hand sides): a thread's kernel values
    // against every s2 stay in registers for the whole chunk and the next
    // right-hand side's inputs load while this one computes.  Otherwise
    // (one right-hand side, or FP64, whose tables would not fit) the values
    // are made again for each right-hand side, with fewer registers.
    static_assert(!HOLD || sizeof(T) == 4, "register-held tables are FP32 only");
    constexpr int NS = HOLD ? Q : 1;
    __shared__ cpx<T> Sx[PPB][4][Q][HH];
    __shared__ cpx<T> Dx[PPB][4][Q][HH];
    __shared__ cpx<T> Mid[PPB][4][Q];
    __shared__ double cth[PPB][Q], sth[PPB][Q], rhos[PPB][Q];
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
            rhos[pl][t] = g.rho_scale * box_node(b1, lB, tb.z[t]);
        } else if (t == Q) {
            rho0[pl] = g.rho_scale * box_centre(b1, lB);
        } else if (t > Q && t <= Q + H) {
            hz[pl][t - Q - 1] = g.rho_scale * ldexp(tb.z[t - Q - 1], -lB);
        }
    }
    __syncthreads();
    XP xp{};
    double r0 = 0.0;
    cpx<T> base[NS], d[NS][HH];
    T f1[NS], f2[NS];
    if (active) {
        xp = make_xp(ph, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]));
        r0 = rho0[pl];
        if constexpr (HOLD) {
#pragma unroll
            for (int s2 = 0; s2 < Q; ++s2) {
                const G3 G = phase_dir3(xp, ph, cth[pl][s2], sth[pl][s2]);
                base[s2] = cis<T>(r0 * G.g);
#pragma unroll
                for (int j = 0; j < H; ++j) d[s2][j] = cis<T>(hz[pl][j] * G.g);
                f1[s2] = (T)(TWO_PI * G.d1);
                f2[s2] = (T)(TWO_PI * G.d2);
            }
        }
    }
    // rows t1 and Q - 1 - t1 of the three planes at (., t2), every active
    // thread (the rows of t1 >= H are loaded and not used: in bounds)
    constexpr int NA = HOLD ? 3 : 1;
    cpx<T> A[NA], B[NA], An[NA], Bn[NA];
    auto fetch = [&](cpx<T> (&a)[NA], cpx<T> (&b)[NA], int r) __attribute__((always_inline)) {
        const cpx<T> *wp = w + r * rstride + pair * QQ;
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            a[k] = wp[k * plane + t1 * Q + t2];
            b[k] = wp[k * plane + (Q - 1 - t1) * Q + t2];
        }
    };
    if constexpr (HOLD)
        if (active) fetch(A, B, 0);
    for (int r = 0; r < nrhs; ++r) {
        cpx<T> *wp = w + r * rstride + pair * QQ;
        if constexpr (HOLD)
            if (active) fetch(An, Bn, min(r + 1, nrhs - 1));
        if (active) {
            // planes 0, 1, 2 and the weighted primal rho(s1) in0(s); thread (t1, t2): t1 plays j
            if (t1 < H) {
                const double ra = rhos[pl][t1], rbv = rhos[pl][Q - 1 - t1];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const size_t off = (k < 3 ? k : 0) * plane;
                    cpx<T> a, b;
                    if constexpr (HOLD) {
                        a = A[k < 3 ? k : 0];
                        b = B[k < 3 ? k : 0];
                    } else {
                        a = wp[off + t1 * Q + t2];
                        b = wp[off + (Q - 1 - t1) * Q + t2];
                    }
                    if (k == 3) {
                        a = {(T)(ra * a.re), (T)(ra * a.im)};
                        b = {(T)(rbv * b.re), (T)(rbv * b.im)};
                    }
                    Sx[pl][k][t2][t1] = cadd(a, b);
                    Dx[pl][k][t2][t1] = csub(a, b);
                }
            } else if ((Q & 1) && t1 == H) {
                const double rm = rhos[pl][H];
                if constexpr (HOLD) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) Mid[pl][k][t2] = A[k];
                } else {
#pragma unroll
                    for (int k = 0; k < 3; ++k) Mid[pl][k][t2] = wp[k * plane + H * Q + t2];
                }
                const cpx<T> a = Mid[pl][0][t2];
                Mid[pl][3][t2] = {(T)(rm * a.re), (T)(rm * a.im)};
            }
        }
        __syncthreads();
        if (active) {
            cpx<T> acc[3] = {{(T)0, (T)0}, {(T)0, (T)0}, {(T)0, (T)0}};
            auto step = [&](int s2, const cpx<T> &bs, const cpx<T> *ds, T g1, T g2) __attribute__((always_inline)) {
                cpx<T> inner[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    cpx<T> in = (Q & 1) ? Mid[pl][k][s2] : cpx<T>{(T)0, (T)0};
#pragma unroll
                    for (int j = 0; j < H; ++j) {
                        const cpx<T> S = Sx[pl][k][s2][j], D = Dx[pl][k][s2][j];
                        in.re = fma(ds[j].re, S.re, fma(-ds[j].im, D.im, in.re));
                        in.im = fma(ds[j].re, S.im, fma(ds[j].im, D.re, in.im));
                    }
                    inner[k] = in;
                }
                cfma(acc[0], bs, inner[0]);
                cfma(acc[1], bs, cadd(inner[1], cpx<T>{-g1 * inner[3].im, g1 * inner[3].re}));
                cfma(acc[2], bs, cadd(inner[2], cpx<T>{-g2 * inner[3].im, g2 * inner[3].re}));
            };
            if constexpr (HOLD) {
#pragma unroll
                for (int s2 = 0; s2 < Q; ++s2) step(s2, base[s2], d[s2], f1[s2], f2[s2]);
            } else {
#pragma unroll 1
                for (int s2 = 0; s2 < Q; ++s2) {
                    const G3 G = phase_dir3(xp, ph, cth[pl][s2], sth[pl][s2]);
                    cpx<T> dd[HH];
#pragma unroll
                    for (int j = 0; j < H; ++j) dd[j] = cis<T>(hz[pl][j] * G.g);
                    step(s2, cis<T>(r0 * G.g), dd, (T)(TWO_PI * G.d1), (T)(TWO_PI * G.d2));
                }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) wp[k * plane + t] = acc[k];
        }
        __syncthreads();
        if constexpr (HOLD) {
#pragma unroll
            for (int k = 0; k < NA; ++k) {
                A[k] = An[k];
                B[k] = Bn[k];
            }
        }
    }
}

// ===========================================================================
// x-recursion (eq:alg2c) with derivatives, one workgroup per block:
//   v   = conj Ep . in,  d v = conj Ep . (d in - 2 pi i dPhi_p . in)
//   out = sum_c Er_c . z_c, z_c = K_A v_c;  d out = sum_c Er_c . (d z_c + 2 pi i dPhi_r,c . z_c)
// The kernel values (Ep of the inputs, Er of the four outputs, and the
// factors 2 pi dPhi of the derivative terms) are made once per block in LDS
// and serve nrhs right-hand sides, whose three planes start rstride apart.
// ===========================================================================
template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_xlevel_tan(Geom g, PhaseDev ph, Tables tb, int level,
                                                   const cpx<T> *__restrict__ win,
                                                   cpx<T> *__restrict__ wout, size_t plane, int nrhs,
                                                   size_t rstride) {
    constexpr int QQ = Q * Q;
    constexpr double TWO_PI = 6.283185307179586476925286766559;
    constexpr int JP = xlevel_tan_jp<T, Q>();
    __shared__ cpx<T> v[3][4 * QQ];
    __shared__ cpx<T> Y[JP][3][4 * QQ];
    __shared__ double sx1[Q], cx1[Q], sx2[Q], cx2[Q];
    __shared__ double sxa[2][Q], cxa[2][Q], sxb[2][Q], cxb[2][Q];  // nodes of the children's boxes
    __shared__ double r0c[2], ct0[2], st0[2];
    __shared__ cpx<T> Ep[4 * QQ];       // E(x^{A_p}_t', p0(B_c)) [c][t']
    __shared__ T Sp[2][4 * QQ];         // 2 pi rho dPhi_k of the same
    __shared__ cpx<T> Er[4][4][QQ];    // E(x^{A_j}_t, p0(B_c)) [j][c][t]
    __shared__ T Sr[2][4][4][QQ];

    const int tid = threadIdx.x;
    const int lB = g.L - level;
    const size_t blk = linear_block();  // exact grid: the block count is a power of two
    const size_t nBl = (size_t)1 << (2 * lB);
    const uint32_t mB = (uint32_t)(blk & (nBl - 1));
    const uint32_t mAp = (uint32_t)(blk >> (2 * lB));
    int b1, b2, ap1, ap2;
    morton_decode(mB, b1, b2);
    morton_decode(mAp, ap1, ap2);
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;

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
    } else if (tid >= 160 && tid < 160 + 4 * Q) {
        // child boxes 2 ap + h in either coordinate (e = 0: x1, 1: x2)
        const int u = tid - 160, e = u / (2 * Q), h = (u - e * 2 * Q) / Q, t = u - e * 2 * Q - h * Q;
        double s_ = 0, c_ = 1;
        if (ell) sincospi(2.0 * box_node(2 * (e ? ap2 : ap1) + h, level, tb.z[t]), &s_, &c_);
        if (e) {
            sxb[h][t] = s_;
            cxb[h][t] = c_;
        } else {
            sxa[h][t] = s_;
            cxa[h][t] = c_;
        }
    }
    __syncthreads();
    // prefactor kernel values of the inputs
    for (int i = tid; i < 2 * QQ; i += NT) {
        const int c2 = i / QQ, tp = i - c2 * QQ;
        const int tp1 = tp / Q, tp2 = tp - tp1 * Q;
        const XP xp = make_xp_sc(ph, box_node(ap1, level - 1, tb.z[tp1]), box_node(ap2, level - 1, tb.z[tp2]),
                                 sx1[tp1], cx1[tp1], sx2[tp2], cx2[tp2]);
        const G3 G = phase_dir3(xp, ph, ct0[c2], st0[c2]);
#pragma unroll
        for (int c1 = 0; c1 < 2; ++c1) {
            const int c = 2 * c1 + c2;
            const double rho = r0c[c1];
            Ep[c * QQ + tp] = cis<T>(rho * G.g);
            Sp[0][c * QQ + tp] = (T)(TWO_PI * (rho * G.d1));
            Sp[1][c * QQ + tp] = (T)(TWO_PI * (rho * G.d2));
        }
    }
    __syncthreads();
    // remodulation kernel values of the four outputs, all four at once
    for (int it = tid; it < 4 * QQ; it += NT) {
        const int j = it / QQ, i = it - j * QQ;
        const int j1 = j >> 1, j2 = j & 1;
        const int a1 = 2 * ap1 + j1, a2 = 2 * ap2 + j2;
        const int t1 = i / Q, t2 = i - t1 * Q;
        const XP xp = make_xp_sc(ph, box_node(a1, level, tb.z[t1]), box_node(a2, level, tb.z[t2]), sxa[j1][t1],
                                 cxa[j1][t1], sxb[j2][t2], cxb[j2][t2]);
        const G3 G0 = phase_dir3(xp, ph, ct0[0], st0[0]);
        const G3 G1 = phase_dir3(xp, ph, ct0[1], st0[1]);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int c1 = c >> 1, c2 = c & 1;
            const G3 &G = c2 ? G1 : G0;
            const double rho = r0c[c1];
            Er[j][c][i] = cis<T>(rho * G.g);
            Sr[0][j][c][i] = (T)(TWO_PI * (rho * G.d1));
            Sr[1][j][c][i] = (T)(TWO_PI * (rho * G.d2));
        }
    }
    __syncthreads();
    // the two contractions go row by row (a thread loads one row of its
    // operand into registers once, the interpolation matrix comes through
    // the scalar cache), JP outputs j = JP jp + jj per pass: pass 1, rows
    // (k, c, t'1); pass 2 in place, one thread per column (jj, k, c, t2), all t1.
    constexpr int HA = (Q + 1) / 2, NPT = (4 * QQ + NT - 1) / NT;
    cptr<T> Mg = to_constant(pick_M<T>(tb));
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    // the next right-hand side's inputs load into registers while this one computes
    cpx<T> xin[3][NPT], xnx[3][NPT];
    fetch_planes<T, 4 * QQ>(xin, win + blk * (4 * QQ), plane, tid);
    for (int r = 0; r < nrhs; ++r) {
        fetch_planes<T, 4 * QQ>(xnx, win + (size_t)min(r + 1, nrhs - 1) * rstride + blk * (4 * QQ), plane, tid);
#pragma unroll
        for (int n = 0; n < NPT; ++n) {
            const int i = tid + n * NT;
            if (i < 4 * QQ) {
                const cpx<T> e = Ep[i];
                const cpx<T> in0 = xin[0][n];
                const T s1 = Sp[0][i], s2 = Sp[1][i];
                v[0][i] = cmulc(in0, e);
                v[1][i] = cmulc(csub(xin[1][n], cpx<T>{-s1 * in0.im, s1 * in0.re}), e);
                v[2][i] = cmulc(csub(xin[2][n], cpx<T>{-s2 * in0.im, s2 * in0.re}), e);
            }
        }
        __syncthreads();
        for (int jp = 0; jp < 4 / JP; ++jp) {
            const int j1 = (JP * jp) >> 1;  // the same for the JP outputs of this pass
            opaque_sgpr(Mg);
            // Y[jj][k][c][t'1][t2] = sum_{t'2} M_j2[t'2][t2] v[k][c][t'1][t'2], j2 = (JP jp + jj) & 1.
            // JP = 2: jj = w >> 1 (wave-uniform j2), every t2; JP = 1: t2 in half (w & 1)
            with_uniform<0, 2>(JP == 2 ? 0 : (w & 1), [&](auto hc) {
                constexpr int HO = JP == 2 ? Q : HA;
                constexpr int t0 = decltype(hc)::value * HO, nt = Q - t0 < HO ? Q - t0 : HO;
                const int jj = JP == 2 ? (w >> 1) : 0;
                const int j2 = (JP * jp + jj) & 1;
                const int rg = JP == 2 ? (w & 1) : (w >> 1);
                if constexpr (nt > 0) {
                    for (int row = rg * 64 + lane; row < 12 * Q; row += 128) {
                        const int k = row / (4 * Q), rem = row - k * 4 * Q;
                        const int c = rem / Q, tp1 = rem - c * Q;
                        const cpx<T> *vv = v[k] + c * QQ + tp1 * Q;
                        cpx<T> acc[nt];
#pragma unroll
                        for (int u = 0; u < nt; ++u) acc[u] = {(T)0, (T)0};
#pragma unroll
                        for (int tp2 = 0; tp2 < Q; ++tp2) {
                            const cpx<T> x = vv[tp2];
#pragma unroll
                            for (int u = 0; u < nt; ++u) crfma(acc[u], Mg[j2 * QQ + tp2 * Q + t0 + u], x);
                        }
                        cpx<T> *yy = Y[jj][k] + c * QQ + tp1 * Q + t0;
#pragma unroll
                        for (int u = 0; u < nt; ++u) yy[u] = acc[u];
                    }
                }
            });
            __syncthreads();
            // z[k][c][t1][t2] = sum_{t'1} M_j1[t'1][t1] Y[k][c][t'1][t2], in place
            for (int row = tid; row < JP * 12 * Q; row += NT) {
                const int jj = row / (12 * Q), rj = row - jj * 12 * Q;
                const int k = rj / (4 * Q), rem = rj - k * 4 * Q;
                const int c = rem / Q, t2 = rem - c * Q;
                cpx<T> *yy = Y[jj][k] + c * QQ + t2;
                cpx<T> x[Q];
#pragma unroll
                for (int tp1 = 0; tp1 < Q; ++tp1) x[tp1] = yy[tp1 * Q];
                cptr<T> Mj = Mg + j1 * QQ;
#pragma unroll
                for (int t1 = 0; t1 < Q; ++t1) {
                    opaque_sgpr(Mj);  // one column of M live at a time
                    cpx<T> acc = {(T)0, (T)0};
#pragma unroll
                    for (int tp1 = 0; tp1 < Q; ++tp1) crfma(acc, Mj[tp1 * Q + t1], x[tp1]);
                    yy[t1 * Q] = acc;
                }
            }
            __syncthreads();
            for (int it = tid; it < JP * QQ; it += NT) {
                const int jj = it / QQ, i = it - jj * QQ;
                const int j = JP * jp + jj;
                cpx<T> *dst = wout + r * rstride + ((size_t)(4 * mAp + j) * nBl + mB) * QQ;
                cpx<T> out[3] = {{(T)0, (T)0}, {(T)0, (T)0}, {(T)0, (T)0}};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const cpx<T> z0 = Y[jj][0][c * QQ + i], z1 = Y[jj][1][c * QQ + i], z2 = Y[jj][2][c * QQ + i];
                    const cpx<T> e = Er[j][c][i];
                    const T s1 = Sr[0][j][c][i], s2 = Sr[1][j][c][i];
                    cfma(out[0], e, z0);
                    cfma(out[1], e, cadd(z1, cpx<T>{-s1 * z0.im, s1 * z0.re}));
                    cfma(out[2], e, cadd(z2, cpx<T>{-s2 * z0.im, s2 * z0.re}));
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) dst[k * plane + i] = out[k];
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int n = 0; n < NPT; ++n) xin[k][n] = xnx[k][n];
    }
}

// ===========================================================================
// termination (eq:alg2d) with derivatives:
//   v = conj Et . delta, d v = conj Et . (d delta - 2 pi i dPhi_t . delta)
//   u = sum_B Ex . U,   U = T_x v;   d u = sum_B Ex . (d U + 2 pi i dPhi_x . U)
// ===========================================================================
template <typename T, int Q>
constexpr int bch3() {
    return bch<T, Q>() / 3 < 1 ? 1 : bch<T, Q>() / 3;
}

template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_term_tan(Geom g, PhaseDev ph, Tables tb, const cpx<T> *__restrict__ win,
                                                 size_t plane, cpx<T> *u0, cpx<T> *u1, cpx<T> *u2) {
    constexpr int QQ = Q * Q;
    constexpr int BC = bch3<T, Q>();
    __shared__ cpx<T> v[3][BC * QQ];
    __shared__ cpx<T> Y[3][BC * Q * 8];
    __shared__ cpx<T> red[NT];
    __shared__ double sx1[Q], cx1[Q], sx2[Q], cx2[Q];
    __shared__ double r0b[BC], ctb[BC], stb[BC];

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
    cpx<T> uacc[3] = {{(T)0, (T)0}, {(T)0, (T)0}, {(T)0, (T)0}};

    const cpx<T> *src = win + (size_t)mA * nBt * QQ;
    for (int b0 = 0; b0 < nBt; b0 += BC) {
        const int nb = min(BC, nBt - b0);
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
        for (int i = tid; i < nb * QQ; i += NT) {
            const int b = i / QQ, t = i - b * QQ;
            const int t1 = t / Q, t2 = t - t1 * Q;
            const XP xp = make_xp_sc(ph, box_node(a1, lA, tb.z[t1]), box_node(a2, lA, tb.z[t2]), sx1[t1], cx1[t1],
                                     sx2[t2], cx2[t2]);
            const G3 G = phase_dir3(xp, ph, ctb[b], stb[b]);
            const double rho = r0b[b];
            const cpx<T> e = cis<T>(rho * G.g);
            const size_t o = (size_t)(b0 + b) * QQ + t;
            const cpx<T> d0 = src[o];
            v[0][i] = cmulc(d0, e);
            v[1][i] = cmulc(csub(src[plane + o], i2pi(rho * G.d1, d0)), e);
            v[2][i] = cmulc(csub(src[2 * plane + o], i2pi(rho * G.d2, d0)), e);
        }
        __syncthreads();
        for (int i = tid; i < 3 * nb * Q * m; i += NT) {
            const int k = i / (nb * Q * m), ii = i - k * nb * Q * m;
            const int b = ii / (Q * m), r = ii - b * (Q * m);
            const int t1 = r / m, jj2 = r - t1 * m;
            const cpx<T> *vv = v[k] + b * QQ + t1 * Q;
            cpx<T> acc = {(T)0, (T)0};
#pragma unroll
            for (int t2 = 0; t2 < Q; ++t2) crfma(acc, Tt[jj2 * Q + t2], vv[t2]);
            Y[k][ii] = acc;
        }
        __syncthreads();
        for (int i = tid; i < nb * np; i += NT) {
            const int b = i / np;
            cpx<T> U[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                cpx<T> acc = {(T)0, (T)0};
                const cpx<T> *yy = Y[k] + b * Q * m + j2;
#pragma unroll
                for (int t1 = 0; t1 < Q; ++t1) crfma(acc, Tt[j1 * Q + t1], yy[t1 * m]);
                U[k] = acc;
            }
            const G3 G = phase_dir3(xg, ph, ctb[b], stb[b]);
            const double rho = r0b[b];
            const cpx<T> e = cis<T>(rho * G.g);
            cfma(uacc[0], e, U[0]);
            cfma(uacc[1], e, cadd(U[1], i2pi(rho * G.d1, U[0])));
            cfma(uacc[2], e, cadd(U[2], i2pi(rho * G.d2, U[0])));
        }
        __syncthreads();
    }
    cpx<T> *const dst[3] = {u0, u1, u2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        red[tid] = uacc[k];
        __syncthreads();
        if (tid < np && dst[k] != nullptr) {
            cpx<T> sum = red[tid];
            for (int kk = tid + np; kk < NT; kk += np) sum = cadd(sum, red[kk]);
            dst[k][(size_t)(a1 * m + j1) * g.N + (a2 * m + j2)] = sum;
        }
        __syncthreads();
    }
}

// ===========================================================================
// Launchers
// ===========================================================================
#define FIO_DISPATCH_QT(q, MACRO)  \
    switch (q) {                   \
        case 3: MACRO(3); break;   \
        case 4: MACRO(4); break;   \
        case 5: MACRO(5); break;   \
        case 6: MACRO(6); break;   \
        case 7: MACRO(7); break;   \
        case 8: MACRO(8); break;   \
        case 9: MACRO(9); break;   \
        case 10: MACRO(10); break; \
        case 11: MACRO(11); break; \
        case 12: MACRO(12); break; \
        default: return hipErrorInvalidValue; \
    }

bool tangent_supported_q(int q) { return q >= QMIN && q <= 12; }

template <typename T>
static hipError_t tan_t(int step, const Geom &g, const PhaseDev &ph, const Tables &tb, const Sources &src,
                        int level, const void *in, void *out, size_t plane, void *u1, void *u2, int nrhs,
                        hipStream_t st) {
    if (step == 0) {
        const unsigned nB = 1u << (2 * (g.L - g.s));
        const int nA = 1 << (2 * g.s);
#define L_IT(Q)                                                                                          \
    {                                                                                                    \
        constexpr int ACH = (NT / Q) < 64 ? (NT / Q) : 64;                                               \
        hipLaunchKernelGGL((k_init_tan<T, Q>), dim3(nB, (nA + ACH - 1) / ACH), dim3(NT), 0, st, g, ph, tb, \
                           src, (const cpx<T> *)in, (cpx<T> *)out, plane);                               \
    }
        FIO_DISPATCH_QT(g.q, L_IT)
#undef L_IT
    } else if (step == 1 || step == 3) {
        const unsigned nblk = 1u << (2 * g.L - 2);
#define L_LT(Q)                                                                                          \
    if (step == 1)                                                                                       \
        hipLaunchKernelGGL((k_plevel_tan<T, Q>), grid_of(nblk), dim3(NT), 0, st, g, ph, tb, level,       \
                           (const cpx<T> *)in, (cpx<T> *)out, plane, nrhs, 3 * plane);                   \
    else                                                                                                 \
        hipLaunchKernelGGL((k_xlevel_tan<T, Q>), grid_of(nblk), dim3(NT), 0, st, g, ph, tb, level,       \
                           (const cpx<T> *)in, (cpx<T> *)out, plane, nrhs, 3 * plane);
        FIO_DISPATCH_QT(g.q, L_LT)
#undef L_LT
    } else if (step == 2) {
        const size_t npairs = (size_t)1 << (2 * g.L);
#define L_ST(Q)                                                                                          \
    {                                                                                                    \
        constexpr int PPB = NT / (Q * Q);                                                                \
        if (sizeof(T) == 4 && nrhs > 1)                                                                  \
            hipLaunchKernelGGL((k_switch_tan<T, Q, sizeof(T) == 4>), grid_of((npairs + PPB - 1) / PPB),  \
                               dim3(NT), 0, st, g, ph, tb, (cpx<T> *)out, plane, nrhs, 3 * plane);       \
        else                                                                                             \
            hipLaunchKernelGGL((k_switch_tan<T, Q, false>), grid_of((npairs + PPB - 1) / PPB), dim3(NT), \
                               0, st, g, ph, tb, (cpx<T> *)out, plane, nrhs, 3 * plane);                 \
    }
        FIO_DISPATCH_QT(g.q, L_ST)
#undef L_ST
    } else {
        const unsigned nA = 1u << (2 * (g.L - g.s));
#define L_TT(Q)                                                                                          \
    hipLaunchKernelGGL((k_term_tan<T, Q>), dim3(nA), dim3(NT), 0, st, g, ph, tb, (const cpx<T> *)in,     \
                       plane, (cpx<T> *)out, (cpx<T> *)u1, (cpx<T> *)u2);
        FIO_DISPATCH_QT(g.q, L_TT)
#undef L_TT
    }
    return hipGetLastError();
}

hipError_t launch_tangent_step(int dtype, int step, const Geom &g, const PhaseDev &ph, const Tables &tb,
                               const Sources &src, int level, const void *in, void *out, size_t plane,
                               void *u1, void *u2, int nrhs, hipStream_t st) {
    return dtype == FIO_C128 ? tan_t<double>(step, g, ph, tb, src, level, in, out, plane, u1, u2, nrhs, st)
                             : tan_t<float>(step, g, ph, tb, src, level, in, out, plane, u1, u2, nrhs, st);
}

}  // namespace fio
