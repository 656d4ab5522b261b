// Termination (eq:alg2d) and its adjoint for several right-hand sides at
// once: the kernel values of a box pair (A, B) -- E(x^A_t, p0(B)) at the q^2
// Chebyshev nodes of A and E(x, p0(B)) at the 4^s grid points x of A --
// are computed once per workgroup and serve every right-hand side.
//
// One workgroup per box A (level L-s) takes the boxes B in chunks of BC:
// the chunk's kernel values go to LDS (all 256 threads), then each wave runs
// its own right-hand sides through the chunk with wave-local LDS scratch
// (lanes in lockstep, so only wave-level ordering is needed between the
// passes).  Forward, per right-hand side and B:
//   v[t]       = conj E(x^A_t, p0(B)) delta^{AB}_t,
//   Y[t1][j2]  = sum_t2 T[j2][t2] v[t1][t2],
//   u(x_j)    += E(x_j, p0(B)) sum_t1 T[j1][t1] Y[t1][j2],
// the lane of grid point j keeping u(x_j) of the wave's right-hand sides in
// registers over all B.  Adjoint, the transposed steps in reverse order.
#include <hip/hip_runtime.h>

#include "fio_kernels_common.h"

namespace fio {

namespace {

constexpr int TW = NT / 64;  // waves per workgroup
constexpr int TRW = 16;      // right-hand sides per wave and pass (registers)
// batches of at least this many right-hand sides take the one-lane-per-RHS kernels
constexpr int TERM_WIDE_MIN_RHS = 32;

// LDS ordering between the lanes of one wave: a compiler barrier; the LDS
// operations of a wave complete in order.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// B boxes per chunk: the chunk's kernel values and the waves' scratch within ~56 KB of LDS
template <typename T, int Q>
constexpr int term_bc() {
    constexpr int scratch = Q * Q > 64 ? Q * Q : 64;  // forward v (q^2) or adjoint U (4^s <= 64)
    constexpr int per_b = (Q * Q + 64 + TW * (scratch + 8 * Q)) * (int)sizeof(cpx<T>);
    constexpr int b = 57344 / per_b;
    return b < 1 ? 1 : (b > 8 ? 8 : b);
}

// Shared set-up of a box A: sin/cos of its nodes, the interpolation table at
// its grid points and the phase data of the grid points.
struct TermBox {
    int s, m, np, nBt, lA, a1, a2;
    uint32_t mA;
};

__device__ __forceinline__ TermBox term_box(const Geom &g) {
    TermBox b;
    b.s = g.s;
    b.m = 1 << b.s;
    b.np = b.m * b.m;
    b.nBt = 1 << (2 * b.s);
    b.lA = g.L - b.s;
    b.mA = blockIdx.x;
    morton_decode(b.mA, b.a1, b.a2);
    return b;
}

template <typename T, int Q>
__device__ __forceinline__ void term_setup(const Geom &g, const PhaseDev &ph, const Tables &tb, const TermBox &bx,
                                           double *sx1, double *cx1, double *sx2, double *cx2, T (*Ts)[Q],
                                           XP *xg) {
    const int tid = threadIdx.x;
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;
    if (tid < Q) {
        double s_ = 0, c_ = 1;
        if (ell) sincospi(2.0 * box_node(bx.a1, bx.lA, tb.z[tid]), &s_, &c_);
        sx1[tid] = s_;
        cx1[tid] = c_;
    } else if (tid >= 64 && tid < 64 + Q) {
        const int t = tid - 64;
        double s_ = 0, c_ = 1;
        if (ell) sincospi(2.0 * box_node(bx.a2, bx.lA, tb.z[t]), &s_, &c_);
        sx2[t] = s_;
        cx2[t] = c_;
    }
    const T *Tt = pick_T<T>(tb);
    for (int i = tid; i < bx.m * Q; i += NT) (&Ts[0][0])[i] = Tt[i];
    if (tid >= 128 && tid < 128 + bx.np) {
        const int jp = tid - 128, j1 = jp / bx.m, j2 = jp - j1 * bx.m;
        xg[jp] = make_xp(ph, (double)(bx.a1 * bx.m + j1) / g.N, (double)(bx.a2 * bx.m + j2) / g.N);
    }
}

// Kernel values of B boxes [b0, b0 + nb): Epre[b][t] = E(x^A_t, p0(B)),
// Ex[b][j] = E(x_j, p0(B)).
// `between` runs after the centres are in LDS and before the kernel values
// are computed (loads issued there overlap that computation).
template <typename T, int Q, int BC, typename F>
__device__ __forceinline__ void term_chunk(const Geom &g, const PhaseDev &ph, const Tables &tb, const TermBox &bx,
                                           int b0, int nb, const double *sx1, const double *cx1,
                                           const double *sx2, const double *cx2, const XP *xg, double *r0b,
                                           double *ctb, double *stb, cpx<T> (*Epre)[Q * Q], cpx<T> (*Ex)[64],
                                           F between) {
    constexpr int QQ = Q * Q;
    const int tid = threadIdx.x;
    if (tid < nb) {
        int bb1, bb2;
        morton_decode((uint32_t)(b0 + tid), bb1, bb2);
        r0b[tid] = g.rho_scale * box_centre(bb1, bx.s);
        double s_, c_;
        sincospi(2.0 * box_centre(bb2, bx.s), &s_, &c_);
        ctb[tid] = c_;
        stb[tid] = s_;
    }
    lds_barrier();
    between();
    for (int i = tid; i < nb * QQ; i += NT) {
        const int b = i / QQ, t = i - b * QQ, t1 = t / Q, t2 = t - t1 * Q;
        const XP xp = make_xp_sc(ph, box_node(bx.a1, bx.lA, tb.z[t1]), box_node(bx.a2, bx.lA, tb.z[t2]), sx1[t1],
                                 cx1[t1], sx2[t2], cx2[t2]);
        Epre[b][t] = cis<T>(r0b[b] * phase_dir(xp, ctb[b], stb[b]));
    }
    for (int i = tid; i < nb * bx.np; i += NT) {
        const int b = i / bx.np, j = i - b * bx.np;
        Ex[b][j] = cis<T>(r0b[b] * phase_dir(xg[j], ctb[b], stb[b]));
    }
}

}  // namespace

template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_term_b(Geom g, PhaseDev ph, Tables tb, const cpx<T> *__restrict__ win,
                                               cpx<T> *__restrict__ u, int nrhs, size_t plane, size_t uplane) {
    constexpr int QQ = Q * Q;
    constexpr int BC = term_bc<T, Q>();
    __shared__ cpx<T> Epre[BC][QQ];
    __shared__ cpx<T> Ex[BC][64];
    __shared__ cpx<T> vw[TW][BC][QQ];
    __shared__ cpx<T> Yw[TW][BC][Q * 8];
    __shared__ T Ts[8][Q];
    __shared__ XP xg[64];
    __shared__ double sx1[Q], cx1[Q], sx2[Q], cx2[Q];
    __shared__ double r0b[BC], ctb[BC], stb[BC];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const TermBox bx = term_box(g);
    const int m = bx.m, np = bx.np;
    term_setup<T, Q>(g, ph, tb, bx, sx1, cx1, sx2, cx2, Ts, xg);
    const int j1 = lane / m, j2 = lane - (lane / m) * m;
    // the rows of T this lane uses: pass 1 items i = lane + 64 k all have
    // j2 = lane % m (m divides 64), pass 2 is the lane's own grid point
    lds_barrier();
    T t_p1[Q], t_p2[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t) {
        t_p1[t] = Ts[j2][t];
        t_p2[t] = lane < np ? Ts[j1][t] : (T)0;
    }

    // a wave's weights of one right-hand side and chunk, loaded one
    // right-hand side ahead
    constexpr int PL = (BC * QQ + 63) / 64;
    cpx<T> nx[PL];
    auto load = [&](int r, int b0, int nb) {
        const cpx<T> *src = win + (size_t)r * plane + ((size_t)bx.mA * bx.nBt + b0) * QQ;
#pragma unroll
        for (int k = 0; k < PL; ++k) {
            const int i = lane + 64 * k;
            if (i < nb * QQ) nx[k] = src[i];
        }
    };
    for (int rp = 0; rp < nrhs; rp += TW * TRW) {
        cpx<T> acc[TRW];
#pragma unroll
        for (int k = 0; k < TRW; ++k) acc[k] = {(T)0, (T)0};
        for (int b0 = 0; b0 < bx.nBt; b0 += BC) {
            const int nb = min(BC, bx.nBt - b0);
            lds_barrier();  // set-up done; the previous chunk's readers are finished
            term_chunk<T, Q, BC>(g, ph, tb, bx, b0, nb, sx1, cx1, sx2, cx2, xg, r0b, ctb, stb, Epre, Ex, [&]() {
                if (rp + wv < nrhs) load(rp + wv, b0, nb);
            });
            lds_barrier();
#pragma unroll
            for (int k = 0; k < TRW; ++k) {
                const int r = rp + k * TW + wv;
                if (r >= nrhs) continue;  // uniform over the wave
#pragma unroll
                for (int kk = 0; kk < PL; ++kk) {
                    const int i = lane + 64 * kk;
                    if (i < nb * QQ) {
                        const int b = i / QQ, t = i - b * QQ;
                        vw[wv][b][t] = cmulc(nx[kk], Epre[b][t]);
                    }
                }
                if (k + 1 < TRW && r + TW < nrhs) load(r + TW, b0, nb);
                wave_sync();
                for (int i = lane; i < nb * Q * m; i += 64) {
                    const int b = i / (Q * m), rr = i - b * (Q * m), t1 = rr / m, jj2 = rr - t1 * m;
                    cpx<T> y = {(T)0, (T)0};
#pragma unroll
                    for (int t2 = 0; t2 < Q; ++t2) crfma(y, t_p1[t2], vw[wv][b][t1 * Q + t2]);
                    Yw[wv][b][t1 * m + jj2] = y;
                }
                wave_sync();
                if (lane < np) {
                    for (int b = 0; b < nb; ++b) {
                        cpx<T> U = {(T)0, (T)0};
#pragma unroll
                        for (int t1 = 0; t1 < Q; ++t1) crfma(U, t_p2[t1], Yw[wv][b][t1 * m + j2]);
                        cfma(acc[k], Ex[b][lane], U);
                    }
                }
                wave_sync();  // the next right-hand side rewrites vw and Yw
            }
        }
        if (lane < np) {
#pragma unroll
            for (int k = 0; k < TRW; ++k) {
                const int r = rp + k * TW + wv;
                if (r < nrhs)
                    u[(size_t)r * uplane + (size_t)(bx.a1 * m + j1) * g.N + (bx.a2 * m + j2)] = acc[k];
            }
        }
    }
}

template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_term_adj_b(Geom g, PhaseDev ph, Tables tb, const cpx<T> *__restrict__ u,
                                                   cpx<T> *__restrict__ wout, int nrhs, size_t plane,
                                                   size_t uplane) {
    constexpr int QQ = Q * Q;
    constexpr int BC = term_bc<T, Q>();
    __shared__ cpx<T> Epre[BC][QQ];
    __shared__ cpx<T> Ex[BC][64];
    __shared__ cpx<T> Uw[TW][BC][64];
    __shared__ cpx<T> Yw[TW][BC][Q * 8];
    __shared__ T Ts[8][Q];
    __shared__ XP xg[64];
    __shared__ double sx1[Q], cx1[Q], sx2[Q], cx2[Q];
    __shared__ double r0b[BC], ctb[BC], stb[BC];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const TermBox bx = term_box(g);
    const int m = bx.m, np = bx.np;
    term_setup<T, Q>(g, ph, tb, bx, sx1, cx1, sx2, cx2, Ts, xg);
    const int j1 = lane / m, j2 = lane - (lane / m) * m;

    for (int rp = 0; rp < nrhs; rp += TW * TRW) {
        // the wave's right-hand sides at this lane's grid point
        cpx<T> uu[TRW];
#pragma unroll
        for (int k = 0; k < TRW; ++k) {
            const int r = rp + k * TW + wv;
            uu[k] = (r < nrhs && lane < np)
                        ? u[(size_t)r * uplane + (size_t)(bx.a1 * m + j1) * g.N + (bx.a2 * m + j2)]
                        : cpx<T>{(T)0, (T)0};
        }
        for (int b0 = 0; b0 < bx.nBt; b0 += BC) {
            const int nb = min(BC, bx.nBt - b0);
            lds_barrier();
            term_chunk<T, Q, BC>(g, ph, tb, bx, b0, nb, sx1, cx1, sx2, cx2, xg, r0b, ctb, stb, Epre, Ex, []() {});
            lds_barrier();
#pragma unroll
            for (int k = 0; k < TRW; ++k) {
                const int r = rp + k * TW + wv;
                if (r >= nrhs) continue;  // uniform over the wave
                if (lane < np)
                    for (int b = 0; b < nb; ++b) Uw[wv][b][lane] = cmulc(uu[k], Ex[b][lane]);
                wave_sync();
                // Y[b][t1][j2] = sum_j1 T[j1][t1] U[b][j1][j2]
                for (int i = lane; i < nb * Q * m; i += 64) {
                    const int b = i / (Q * m), rr = i - b * (Q * m), t1 = rr / m, jj2 = rr - t1 * m;
                    cpx<T> y = {(T)0, (T)0};
                    for (int jj1 = 0; jj1 < m; ++jj1) crfma(y, Ts[jj1][t1], Uw[wv][b][jj1 * m + jj2]);
                    Yw[wv][b][t1 * m + jj2] = y;
                }
                wave_sync();
                // delta[b][t1][t2] = E(x^A_t, p0(B)) sum_j2 T[j2][t2] Y[b][t1][j2]
                cpx<T> *dst = wout + (size_t)r * plane + ((size_t)bx.mA * bx.nBt + b0) * QQ;
                for (int i = lane; i < nb * QQ; i += 64) {
                    const int b = i / QQ, t = i - b * QQ, t1 = t / Q, t2 = t - t1 * Q;
                    cpx<T> acc = {(T)0, (T)0};
                    for (int jj2 = 0; jj2 < m; ++jj2) crfma(acc, Ts[jj2][t2], Yw[wv][b][t1 * m + jj2]);
                    dst[i] = cmul(acc, Epre[b][t]);
                }
                wave_sync();  // the next right-hand side rewrites Uw and Yw
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Wide batches: 64 right-hand sides per workgroup of 64 q threads, one box
// A.  Node side: thread i holds row t1 = i % q of right-hand side i / q, so
// a wave's loads (stores, adjoint) cover about 64/q consecutive rows of a
// few right-hand sides (coalesced, few pages per instruction).  Grid side:
// wave w is grid column j2 = w (+ q, ...) and lane r is right-hand side r,
// so the kernel values and interpolation coefficients it uses are the same
// for all lanes (LDS broadcasts).  The only per-right-hand-side LDS traffic
// is one write and one read of the 2^s x q intermediate Y[j2][t1].  Each
// thread's next row of weights is loaded during the current box B; the
// barriers order LDS only, so that load stays in flight across them.
// ---------------------------------------------------------------------------
constexpr int TR_BCH = 8;   // boxes B whose kernel values are staged together
constexpr int TR_YS = 68;   // row stride of Y over right-hand sides (== 4 mod 32: conflict-free node side)

template <int Q>
constexpr int term_r_jw() { return (8 + Q - 1) / Q; }  // grid columns per wave (2^s <= 8)

template <typename T, int Q>
constexpr int term_r_lds(int nbuf) {
    return (nbuf * 8 * Q * TR_YS + TR_BCH * (Q * Q + 64)) * (int)sizeof(cpx<T>) + 8 * Q * (int)sizeof(T) +
           64 * (int)sizeof(XP) + (4 * Q + 3 * TR_BCH) * 8;
}

// Y buffers: two (one barrier per box B) where they fit in 144 KB of LDS.
// The kernels' registers allow one workgroup per CU, so LDS is not what
// limits their occupancy.
template <typename T, int Q>
constexpr int term_r_nbuf() { return term_r_lds<T, Q>(2) <= 144 * 1024 ? 2 : 1; }

template <typename T, int Q>
constexpr bool term_r_fits() { return term_r_lds<T, Q>(1) <= 96 * 1024 && Q <= (sizeof(T) == 4 ? 12 : 8); }

// Kernel values of B boxes [b0, b0 + nb) with all 64 q threads.
template <typename T, int Q>
__device__ __forceinline__ void term_values_r(const Geom &g, const PhaseDev &ph, const Tables &tb,
                                              const TermBox &bx, int b0, int nb, const double *sx1,
                                              const double *cx1, const double *sx2, const double *cx2,
                                              const XP *xg, double *r0b, double *ctb, double *stb,
                                              cpx<T> (*Epre)[Q * Q], cpx<T> (*Ex)[64]) {
    constexpr int QQ = Q * Q, NTR = 64 * Q;
    const int tid = threadIdx.x;
    if (tid < nb) {
        int bb1, bb2;
        morton_decode((uint32_t)(b0 + tid), bb1, bb2);
        r0b[tid] = g.rho_scale * box_centre(bb1, bx.s);
        double s_, c_;
        sincospi(2.0 * box_centre(bb2, bx.s), &s_, &c_);
        ctb[tid] = c_;
        stb[tid] = s_;
    }
    lds_barrier();
    for (int i = tid; i < nb * QQ; i += NTR) {
        const int b = i / QQ, t = i - b * QQ, t1 = t / Q, t2 = t - t1 * Q;
        const XP xp = make_xp_sc(ph, box_node(bx.a1, bx.lA, tb.z[t1]), box_node(bx.a2, bx.lA, tb.z[t2]), sx1[t1],
                                 cx1[t1], sx2[t2], cx2[t2]);
        Epre[b][t] = cis<T>(r0b[b] * phase_dir(xp, ctb[b], stb[b]));
    }
    for (int i = tid; i < nb * bx.np; i += NTR) {
        const int b = i / bx.np, j = i - b * bx.np;
        Ex[b][j] = cis<T>(r0b[b] * phase_dir(xg[j], ctb[b], stb[b]));
    }
}

template <typename T, int Q>
__global__ __launch_bounds__(64 * Q) void k_term_r(Geom g, PhaseDev ph, Tables tb, const cpx<T> *__restrict__ win,
                                                   cpx<T> *__restrict__ u, int nrhs, size_t plane, size_t uplane) {
    constexpr int QQ = Q * Q, JW = term_r_jw<Q>(), NBUF = term_r_nbuf<T, Q>();
    __shared__ cpx<T> Ys[NBUF][8][Q][TR_YS];
    __shared__ cpx<T> Epre[TR_BCH][QQ];
    __shared__ cpx<T> Ex[TR_BCH][64];
    __shared__ T Ts[8][Q];
    __shared__ XP xg[64];
    __shared__ double sx1[Q], cx1[Q], sx2[Q], cx2[Q];
    __shared__ double r0b[TR_BCH], ctb[TR_BCH], stb[TR_BCH];

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TermBox bx = term_box(g);
    const int m = bx.m;
    term_setup<T, Q>(g, ph, tb, bx, sx1, cx1, sx2, cx2, Ts, xg);
    const int r0 = blockIdx.y * 64;
    // node side: right-hand side rn, row tn of delta^{AB}
    const int rn = threadIdx.x / Q, tn = threadIdx.x - rn * Q;
    const cpx<T> *src =
        win + (size_t)(r0 + rn < nrhs ? r0 + rn : 0) * plane + (size_t)bx.mA * bx.nBt * QQ + tn * Q;
    cpx<T> nx[Q];
    auto load = [&](int b) {
#pragma unroll
        for (int t = 0; t < Q; ++t) nx[t] = src[(size_t)b * QQ + t];
    };
    load(0);
    cpx<T> acc[JW][8];
#pragma unroll
    for (int jw = 0; jw < JW; ++jw)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[jw][j] = {(T)0, (T)0};

    int buf = 0;
    for (int b0 = 0; b0 < bx.nBt; b0 += TR_BCH) {
        const int nb = min(TR_BCH, bx.nBt - b0);
        lds_barrier();  // set-up done; the previous chunk's readers are finished
        term_values_r<T, Q>(g, ph, tb, bx, b0, nb, sx1, cx1, sx2, cx2, xg, r0b, ctb, stb, Epre, Ex);
        lds_barrier();
        for (int bb = 0; bb < nb; ++bb) {
            // With two Y buffers the barrier after this box's node side also
            // orders the previous box's grid-side reads of the buffer
            // rewritten next; with one, a second barrier closes each box.
            // node side: v = conj E(x^A_t, p0(B)) delta_t;  Y[j2][tn] = sum_t2 T[j2][t2] v[tn][t2]
            cpx<T> v[Q];
#pragma unroll
            for (int t2 = 0; t2 < Q; ++t2) v[t2] = cmulc(nx[t2], Epre[bb][tn * Q + t2]);
            if (b0 + bb + 1 < bx.nBt) load(b0 + bb + 1);
#pragma unroll
            for (int j2 = 0; j2 < 8; ++j2) {
                if (j2 < m) {
                    cpx<T> y = {(T)0, (T)0};
#pragma unroll
                    for (int t2 = 0; t2 < Q; ++t2) crfma(y, Ts[j2][t2], v[t2]);
                    Ys[buf][j2][tn][rn] = y;
                }
            }
            lds_barrier();
            // grid side: u(x_{j1 j2}) += E(x, p0(B)) sum_t1 T[j1][t1] Y[j2][t1]
#pragma unroll
            for (int jw = 0; jw < JW; ++jw) {
                const int j2 = w + jw * Q;
                if (j2 < m) {
                    cpx<T> y[Q];
#pragma unroll
                    for (int t1 = 0; t1 < Q; ++t1) y[t1] = Ys[buf][j2][t1][lane];
#pragma unroll
                    for (int j1 = 0; j1 < 8; ++j1) {
                        if (j1 < m) {
                            cpx<T> U = {(T)0, (T)0};
#pragma unroll
                            for (int t1 = 0; t1 < Q; ++t1) crfma(U, Ts[j1][t1], y[t1]);
                            cfma(acc[jw][j1], Ex[bb][j1 * m + j2], U);
                        }
                    }
                }
            }
            if (NBUF == 1) lds_barrier();
            buf = NBUF - 1 - buf;
        }
    }
    const int r = r0 + lane;
    if (r < nrhs) {
        cpx<T> *dst = u + (size_t)r * uplane + (size_t)(bx.a1 * m) * g.N + bx.a2 * m;
#pragma unroll
        for (int jw = 0; jw < JW; ++jw) {
            const int j2 = w + jw * Q;
            if (j2 < m) {
#pragma unroll
                for (int j1 = 0; j1 < 8; ++j1)
                    if (j1 < m) dst[(size_t)j1 * g.N + j2] = acc[jw][j1];
            }
        }
    }
}

template <typename T, int Q>
__global__ __launch_bounds__(64 * Q) void k_term_adj_r(Geom g, PhaseDev ph, Tables tb, const cpx<T> *__restrict__ u,
                                                       cpx<T> *__restrict__ wout, int nrhs, size_t plane,
                                                       size_t uplane) {
    constexpr int QQ = Q * Q, JW = term_r_jw<Q>(), NBUF = term_r_nbuf<T, Q>();
    __shared__ cpx<T> Ys[NBUF][8][Q][TR_YS];
    __shared__ cpx<T> Epre[TR_BCH][QQ];
    __shared__ cpx<T> Ex[TR_BCH][64];
    __shared__ T Ts[8][Q];
    __shared__ XP xg[64];
    __shared__ double sx1[Q], cx1[Q], sx2[Q], cx2[Q];
    __shared__ double r0b[TR_BCH], ctb[TR_BCH], stb[TR_BCH];

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TermBox bx = term_box(g);
    const int m = bx.m;
    term_setup<T, Q>(g, ph, tb, bx, sx1, cx1, sx2, cx2, Ts, xg);
    const int r0 = blockIdx.y * 64, r = r0 + lane;
    // grid side: u at the grid columns of this wave, for right-hand side r
    cpx<T> uu[JW][8];
    {
        const cpx<T> *us = u + (size_t)(r < nrhs ? r : 0) * uplane + (size_t)(bx.a1 * m) * g.N + bx.a2 * m;
#pragma unroll
        for (int jw = 0; jw < JW; ++jw) {
            const int j2 = w + jw * Q;
#pragma unroll
            for (int j1 = 0; j1 < 8; ++j1)
                uu[jw][j1] = (j2 < m && j1 < m) ? us[(size_t)j1 * g.N + j2] : cpx<T>{(T)0, (T)0};
        }
    }
    // node side: right-hand side rn, row tn of delta^{AB}
    const int rn = threadIdx.x / Q, tn = threadIdx.x - rn * Q;
    const bool live_n = r0 + rn < nrhs;
    cpx<T> *dst = wout + (size_t)(live_n ? r0 + rn : 0) * plane + (size_t)bx.mA * bx.nBt * QQ + tn * Q;

    int buf = 0;
    for (int b0 = 0; b0 < bx.nBt; b0 += TR_BCH) {
        const int nb = min(TR_BCH, bx.nBt - b0);
        lds_barrier();
        term_values_r<T, Q>(g, ph, tb, bx, b0, nb, sx1, cx1, sx2, cx2, xg, r0b, ctb, stb, Epre, Ex);
        lds_barrier();
        for (int bb = 0; bb < nb; ++bb) {
            // grid side: Y[j2][t1] = sum_j1 T[j1][t1] conj E(x_{j1 j2}, p0(B)) u(x_{j1 j2})
#pragma unroll
            for (int jw = 0; jw < JW; ++jw) {
                const int j2 = w + jw * Q;
                if (j2 < m) {
                    cpx<T> U[8];
#pragma unroll
                    for (int j1 = 0; j1 < 8; ++j1)
                        U[j1] = j1 < m ? cmulc(uu[jw][j1], Ex[bb][j1 * m + j2]) : cpx<T>{(T)0, (T)0};
#pragma unroll
                    for (int t1 = 0; t1 < Q; ++t1) {
                        cpx<T> y = {(T)0, (T)0};
#pragma unroll
                        for (int j1 = 0; j1 < 8; ++j1)
                            if (j1 < m) crfma(y, Ts[j1][t1], U[j1]);
                        Ys[buf][j2][t1][lane] = y;
                    }
                }
            }
            lds_barrier();
            // node side: delta[tn][t2] = E(x^A_t, p0(B)) sum_j2 T[j2][t2] Y[j2][tn]
            cpx<T> y[8];
#pragma unroll
            for (int j2 = 0; j2 < 8; ++j2) y[j2] = j2 < m ? Ys[buf][j2][tn][rn] : cpx<T>{(T)0, (T)0};
            if (live_n) {
                cpx<T> *d = dst + (size_t)(b0 + bb) * QQ;
#pragma unroll
                for (int t2 = 0; t2 < Q; ++t2) {
                    cpx<T> a = {(T)0, (T)0};
#pragma unroll
                    for (int j2 = 0; j2 < 8; ++j2)
                        if (j2 < m) crfma(a, Ts[j2][t2], y[j2]);
                    d[t2] = cmul(a, Epre[bb][tn * Q + t2]);
                }
            }
            if (NBUF == 1) lds_barrier();  // Ys is rewritten for the next B
            buf = NBUF - 1 - buf;
        }
    }
}

template <typename T, int Q>
static void term_b_q(bool adjoint, const Geom &g, const PhaseDev &ph, const Tables &tb, const void *in, void *out,
                     int nrhs, size_t plane, size_t uplane, hipStream_t st) {
    const unsigned nA = 1u << (2 * (g.L - g.s));
    if constexpr (term_r_fits<T, Q>()) {
        if (nrhs >= TERM_WIDE_MIN_RHS) {
            const dim3 grid(nA, (unsigned)((nrhs + 63) / 64));
            if (adjoint)
                hipLaunchKernelGGL((k_term_adj_r<T, Q>), grid, dim3(64 * Q), 0, st, g, ph, tb, (const cpx<T> *)in,
                                   (cpx<T> *)out, nrhs, plane, uplane);
            else
                hipLaunchKernelGGL((k_term_r<T, Q>), grid, dim3(64 * Q), 0, st, g, ph, tb, (const cpx<T> *)in,
                                   (cpx<T> *)out, nrhs, plane, uplane);
            return;
        }
    }
    if (adjoint)
        hipLaunchKernelGGL((k_term_adj_b<T, Q>), dim3(nA), dim3(NT), 0, st, g, ph, tb, (const cpx<T> *)in,
                           (cpx<T> *)out, nrhs, plane, uplane);
    else
        hipLaunchKernelGGL((k_term_b<T, Q>), dim3(nA), dim3(NT), 0, st, g, ph, tb, (const cpx<T> *)in,
                           (cpx<T> *)out, nrhs, plane, uplane);
}

template <typename T>
static hipError_t term_b_t(bool adjoint, const Geom &g, const PhaseDev &ph, const Tables &tb, const void *in,
                           void *out, int nrhs, size_t plane, size_t uplane, hipStream_t st) {
#define L_TB(Q) term_b_q<T, Q>(adjoint, g, ph, tb, in, out, nrhs, plane, uplane, st);
    FIO_DISPATCH_Q(g.q, L_TB)
#undef L_TB
    return hipGetLastError();
}

hipError_t launch_term_batch(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, const void *w_in,
                             void *u, int nrhs, size_t plane, size_t uplane, hipStream_t st) {
    return dtype == FIO_C128 ? term_b_t<double>(false, g, ph, tb, w_in, u, nrhs, plane, uplane, st)
                             : term_b_t<float>(false, g, ph, tb, w_in, u, nrhs, plane, uplane, st);
}

hipError_t launch_term_adj_batch(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, const void *u,
                                 void *w_out, int nrhs, size_t plane, size_t uplane, hipStream_t st) {
    return dtype == FIO_C128 ? term_b_t<double>(true, g, ph, tb, u, w_out, nrhs, plane, uplane, st)
                             : term_b_t<float>(true, g, ph, tb, u, w_out, nrhs, plane, uplane, st);
}

}  // namespace fio
