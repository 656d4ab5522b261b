// Initialisation (eq:alg2a) and its adjoint on the matrix cores, complex64
// weights, s = 3 (the 64 boxes A of level 3 share every box B of level L-3),
// q <= 9 (the per-box remodulation table fills most of the workgroup's LDS).
//
// For one box B and one right-hand side r the initialisation is a dense
// contraction over the sources p of B,
//     D_r[t][A] = sum_p K[t][p] E(x0(A), k_p) f_r(k_p),   K[t][p] = L_t1(p1) L_t2(p2),
//     delta_r^{AB}_t = conj E(x0(A), p^B_t) D_r[t][A],
// a real (q^2 x n_p) matrix times a complex (n_p x 64) one.  It runs as FP32
// MFMA tiles v_mfma_f32_16x16x4_f32 with t as the row dimension (padded to a
// multiple of 16), the sources as the reduction dimension (in steps of 4)
// and the columns (r, A, re/im) -- the complex operand split into its real
// and imaginary parts.  The adjoint is the transposed contraction
//     Y_r[A][p] = sum_t (E(x0(A), p^B_t) delta_r^{AB}_t) K[t][p],
//     f_r(k_p)  = sum_A conj E(x0(A), k_p) Y_r[A][p],
// with (r, A, re/im) as rows, t as the reduction dimension and the sources
// as columns, followed by the sum over A.
//
// Both operands of the contraction are read from two tables in source order
// (sources sorted by their box B, as the plan's CSR): K[j][t] (the Lagrange
// products; they depend only on the plan and are made once) and
// E[j][A] = E(x0(A), k_j) (the kernel values; they depend on the phase and
// are remade when it changes).  The right-hand sides are gathered into source
// order first.  One workgroup (4 waves) per box B; per box, once, the
// remodulation factors E(x0(A), p^B_t) for all 64 A and q^2 nodes t go to
// LDS.  Wave w owns the column tiles [w CTW, (w+1) CTW).
//
// MFMA lane layout (16x16x4, 64 lanes): A operand lane l holds A[l%16][l/16],
// B operand B[l/16][l%16], accumulator element v of lane l is D[4(l/16)+v][l%16].
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fio_kernels_common.h"

namespace fio {

using f32x4 = __attribute__((ext_vector_type(4))) float;

constexpr int IM_NA = 64;  // A boxes at level 3

bool init_mfma_supported(int q, int s) { return s == 3 && q >= QMIN && q <= 9; }

// Workgroups per box: the right-hand sides of a box are split into up to
// IM_CH chunks of passes, one workgroup each.  Workgroup w runs on XCD
// w mod 8 (round-robin dispatch); numbering boxes so that the chunks of one
// box are the workgroups k*8 + x, ..., (k + IM_CH - 1)*8 + x of one XCD x
// puts them on that XCD at about the same time, so the box's rows of the K
// and E tables are fetched from HBM once and then served by that XCD's L2
// (with every chunk of every box in flight at once, the tables of the boxes
// active on an XCD exceed its L2 and are re-read from HBM per pass).
constexpr int IM_CH = 8;
__device__ __forceinline__ void im_box_chunk(int nch, uint32_t &box, int &chunk) {
    const uint32_t w = blockIdx.x, x = w & 7u, k = w >> 3;
    box = (k / (uint32_t)nch) * 8u + x;
    chunk = (int)(k % (uint32_t)nch);
}

// Row length of the K table: q^2 padded to the forward kernel's row tiles.
constexpr int im_ks(int q) { return (q * q + 15) / 16 * 16; }
int init_mfma_ktab_row(int q) { return im_ks(q); }

// Nodes, the 64 centres x0(A) and the remodulation factors
// Er[A][t] = E(x0(A), p^B_t) of box B = (bp1, bp2).
template <int Q>
__device__ __forceinline__ void init_mm_setup(const Geom &g, const PhaseDev &ph, const Tables &tb, int bp1,
                                              int bp2, double *zs, XP *xA, cpx<float> (*Er)[Q * Q]) {
    constexpr int QQ = Q * Q;
    const int tid = threadIdx.x;
    const int lB = g.L - g.s;
    if (tid < Q) zs[tid] = tb.z[tid];
    if (tid < IM_NA) {
        int a1, a2;
        morton_decode((uint32_t)tid, a1, a2);
        xA[tid] = make_xp(ph, box_centre(a1, g.s), box_centre(a2, g.s));
    }
    lds_barrier();
    for (int i = tid; i < IM_NA * QQ; i += NT) {
        const int a = i / QQ, t = i - a * QQ, t1 = t / Q, t2 = t - t1 * Q;
        double st, ct;
        sincospi(2.0 * box_node(bp2, lB, zs[t2]), &st, &ct);
        Er[a][t] = cis<float>(g.rho_scale * box_node(bp1, lB, zs[t1]) * phase_dir(xA[a], ct, st));
    }
    lds_barrier();
}

// K[j][t] = L_t1(u1(p_j)) L_t2(u2(p_j)) for the j-th source in sorted order
// (u the coordinates of p in its level-(L-s) box, scaled to [-1/2, 1/2]),
// product form in FP64, zero for t >= q^2.
template <int Q>
__global__ __launch_bounds__(NT) void k_init_ktab(Geom g, Tables tb, const double2 *__restrict__ sp,
                                                  float *__restrict__ K, int n2) {
    constexpr int QQ = Q * Q, KS = im_ks(Q);
    const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
    if (i >= (size_t)n2 * KS) return;
    const int j = (int)(i / KS), t = (int)(i - (size_t)j * KS);
    float v = 0.f;
    if (t < QQ) {
        const int nb = 1 << (g.L - g.s);
        const double2 p = sp[j];
        const double x1 = p.x * nb, x2 = p.y * nb;
        const double u1 = x1 - ((double)min((int)floor(x1), nb - 1) + 0.5);
        const double u2 = x2 - ((double)min((int)floor(x2), nb - 1) + 0.5);
        const int t1 = t / Q, t2 = t - t1 * Q;
        double l1 = tb.lam[t1], l2 = tb.lam[t2];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const double zk = tb.z[k];
            if (k != t1) l1 *= (u1 - zk);
            if (k != t2) l2 *= (u2 - zk);
        }
        v = (float)(l1 * l2);
    }
    K[i] = v;
}

// E[j][A] = E(x0(A), k_j) for the j-th source in sorted order.  A workgroup
// takes 64 consecutive sources; thread (jl, A) with jl = tid / 64 steps by 4.
__global__ __launch_bounds__(NT) void k_init_etab(Geom g, PhaseDev ph, const int32_t *__restrict__ idx,
                                                  cpx<float> *__restrict__ E, int n2) {
    __shared__ XP xA[IM_NA];
    const int tid = threadIdx.x;
    if (tid < IM_NA) {
        int a1, a2;
        morton_decode((uint32_t)tid, a1, a2);
        xA[tid] = make_xp(ph, box_centre(a1, g.s), box_centre(a2, g.s));
    }
    lds_barrier();
    const int A = tid & (IM_NA - 1);
    for (int jl = tid >> 6; jl < 64; jl += NT / IM_NA) {
        const int j = blockIdx.x * 64 + jl;
        if (j >= n2) break;
        const int k = idx[j];
        E[(size_t)j * IM_NA + A] =
            cis<float>(phase_cart(xA[A], (double)(k / g.N - g.N / 2), (double)(k % g.N - g.N / 2)));
    }
}

// fs[r][j] = f[r][idx[j]]: right-hand sides in sorted source order.
__global__ __launch_bounds__(NT) void k_gather_sorted(const cpx<float> *__restrict__ f,
                                                      const int32_t *__restrict__ idx,
                                                      cpx<float> *__restrict__ fs, int n2, int nrhs) {
    const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
    if (i >= (size_t)n2 * nrhs) return;
    const size_t r = i / n2, j = i - r * n2;
    fs[i] = f[r * n2 + idx[j]];
}

template <int Q, int RCI>
__global__ __launch_bounds__(NT, 2) void k_init_mm(Geom g, PhaseDev ph, Tables tb, Sources src,
                                                   const float *__restrict__ Kt, const cpx<float> *__restrict__ Et,
                                                   const cpx<float> *__restrict__ fsrt, cpx<float> *__restrict__ w,
                                                   int nrhs, size_t plane, int nch, int ppc) {
    constexpr int QQ = Q * Q;
    constexpr int TT = (QQ + 15) / 16;  // row tiles of t
    constexpr int KS = im_ks(Q);
    constexpr int CTW = 2 * RCI;        // column tiles per wave: 64 A x 2 x RCI / 16 / 4 waves
    constexpr int WPR = 4 / RCI;        // waves per right-hand side
    __shared__ cpx<float> Er[IM_NA][QQ];
    __shared__ double zs[Q];
    __shared__ XP xA[IM_NA];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int cl = lane & 15, kq = lane >> 4;
    uint32_t mB;
    int chunk;
    im_box_chunk(nch, mB, chunk);  // passes [chunk ppc, (chunk + 1) ppc) of box mB
    int bp1, bp2;
    morton_decode(mB, bp1, bp2);
    const int n2 = g.N * g.N;
    const size_t nBl = (size_t)1 << (2 * (g.L - g.s));
    const int beg = src.off[mB], np = src.off[mB + 1] - beg;
    init_mm_setup<Q>(g, ph, tb, bp1, bp2, zs, xA, Er);

    // this lane's column cl of tile wv*CTW + ct: A = acol[ct], c = cl & 1
    const int rl = wv / WPR, c = cl & 1;
    int acol[CTW];
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) acol[ct] = ((((wv * CTW + ct) * 16 + cl) >> 1)) & (IM_NA - 1);

    const int rend = min(nrhs, (chunk + 1) * ppc * RCI);
    for (int r0 = chunk * ppc * RCI; r0 < rend; r0 += RCI) {
        const int r = r0 + rl;
        const bool rok = r < nrhs;
        const cpx<float> *fr = fsrt + (size_t)min(r, nrhs - 1) * n2 + beg;
        f32x4 acc[CTW][TT];
#pragma unroll
        for (int ct = 0; ct < CTW; ++ct)
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) acc[ct][tt] = f32x4{0.f, 0.f, 0.f, 0.f};
        // operands of one reduction step (4 sources): K column and E f
        float a[TT];
        cpx<float> e[CTW], fv;
        auto load = [&](int k0) {
            const int j = k0 + kq;
            const bool ok = j < np;
            const float *kr = Kt + (size_t)(ok ? beg + j : 0) * KS + cl;
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) a[tt] = ok ? kr[16 * tt] : 0.f;
            const cpx<float> *er = Et + (size_t)(ok ? beg + j : 0) * IM_NA;
#pragma unroll
            for (int ct = 0; ct < CTW; ++ct) e[ct] = ok ? er[acol[ct]] : cpx<float>{0.f, 0.f};
            fv = (ok && rok) ? fr[j] : cpx<float>{0.f, 0.f};
        };
        load(0);
        for (int k0 = 0; k0 < np; k0 += 4) {
            float ac[TT];
            cpx<float> ec[CTW], fc = fv;
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) ac[tt] = a[tt];
#pragma unroll
            for (int ct = 0; ct < CTW; ++ct) ec[ct] = e[ct];
            if (k0 + 4 < np) load(k0 + 4);
#pragma unroll
            for (int ct = 0; ct < CTW; ++ct) {
                const float b = c ? fmaf(ec[ct].re, fc.im, ec[ct].im * fc.re)
                                  : fmaf(ec[ct].re, fc.re, -ec[ct].im * fc.im);
#pragma unroll
                for (int tt = 0; tt < TT; ++tt)
                    acc[ct][tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[tt], b, acc[ct][tt], 0, 0, 0);
            }
        }
        // remodulate and store: the even lane of a (re, im) column pair takes
        // rows v = 0, 1 of its 4, the odd lane rows 2, 3
        if (rok) {
#pragma unroll
            for (int ct = 0; ct < CTW; ++ct) {
                const int A = acol[ct];
                cpx<float> *dst = w + (size_t)r * plane + ((size_t)A * nBl + mB) * QQ;
#pragma unroll
                for (int tt = 0; tt < TT; ++tt) {
                    const f32x4 d = acc[ct][tt];
                    const float s0 = c ? d[0] : d[2], s1 = c ? d[1] : d[3];
                    const float g0 = __shfl_xor(s0, 1), g1 = __shfl_xor(s1, 1);
                    const int t = 16 * tt + 4 * kq + (c ? 2 : 0);
                    const cpx<float> y0 = c ? cpx<float>{g0, d[2]} : cpx<float>{d[0], g0};
                    const cpx<float> y1 = c ? cpx<float>{g1, d[3]} : cpx<float>{d[1], g1};
                    if (t < QQ) dst[t] = cmulc(y0, Er[A][t]);
                    if (t + 1 < QQ) dst[t + 1] = cmulc(y1, Er[A][t + 1]);
                }
            }
        }
    }
}

// Adjoint, one right-hand side per pass over the box.  Its A operand, the
// remodulated weights W = Er delta (KT values per lane and row tile), stays in
// registers across the source tiles of 16.  Each tile's rows of the K and E
// tables (contiguous in source order) are copied to LDS with coalesced loads,
// issued one tile ahead into registers.
template <int Q>
__global__ __launch_bounds__(NT, 2) void k_init_adj_mm(Geom g, PhaseDev ph, Tables tb, Sources src,
                                                       const float *__restrict__ Kt,
                                                       const cpx<float> *__restrict__ Et,
                                                       const cpx<float> *__restrict__ win,
                                                       cpx<float> *__restrict__ f, int nrhs, size_t plane, int nch,
                                                       int ppc) {
    constexpr int QQ = Q * Q;
    constexpr int KT = (QQ + 3) / 4;   // reduction steps over t (t = 4 ks + lane / 16)
    constexpr int KS = im_ks(Q);
    constexpr int KP = 4 * KT + 1;     // LDS row of K (odd: the 16 sources' rows hit distinct banks)
    constexpr int CTW = 2;             // row tiles of (A, re/im) per wave
    constexpr int KL = (16 * KS / 4 + NT - 1) / NT;        // float4 loads of a K tile per thread
    constexpr int EL = (16 * IM_NA / 2 + NT - 1) / NT;     // float4 loads (2 complex) of an E tile
    __shared__ cpx<float> Er[IM_NA][QQ];
    __shared__ float Kc[16][KP];
    __shared__ cpx<float> Es[16][IM_NA + 1];
    __shared__ cpx<float> part[4][16];
    __shared__ double zs[Q];
    __shared__ XP xA[IM_NA];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int cl = lane & 15, kq = lane >> 4;
    uint32_t mB;
    int chunk;
    im_box_chunk(nch, mB, chunk);  // right-hand sides [chunk ppc, (chunk + 1) ppc) of box mB
    int bp1, bp2;
    morton_decode(mB, bp1, bp2);
    const int n2 = g.N * g.N;
    const size_t nBl = (size_t)1 << (2 * (g.L - g.s));
    const int beg = src.off[mB], np = src.off[mB + 1] - beg;
    init_mm_setup<Q>(g, ph, tb, bp1, bp2, zs, xA, Er);

    // tile loads: thread's float4 pieces of the K rows and the E rows of
    // sources [c0, c0 + 16) (rows beyond np are not read)
    float4 kpre[KL], epre[EL];
    auto fetch = [&](int c0) {
        const int nrow = min(16, np - c0);
        const float4 *k4 = (const float4 *)(Kt + (size_t)(beg + c0) * KS);
#pragma unroll
        for (int u = 0; u < KL; ++u) {
            const int i = tid + u * NT;
            if (i < nrow * (KS / 4)) kpre[u] = k4[i];
        }
        const float4 *e4 = (const float4 *)(Et + (size_t)(beg + c0) * IM_NA);
#pragma unroll
        for (int u = 0; u < EL; ++u) {
            const int i = tid + u * NT;
            if (i < nrow * (IM_NA / 2)) epre[u] = e4[i];
        }
    };
    auto stash = [&](int c0) {
        const int nrow = min(16, np - c0);
#pragma unroll
        for (int u = 0; u < KL; ++u) {
            const int i = tid + u * NT;
            if (i < 16 * (KS / 4)) {
                const int row = i / (KS / 4), col = 4 * (i - row * (KS / 4));
                const float4 v = row < nrow ? kpre[u] : float4{0.f, 0.f, 0.f, 0.f};
                // K row in the reduction order t = 4 ks + kq: Kc[row][t]
                if (col + 0 < 4 * KT) Kc[row][col + 0] = v.x;
                if (col + 1 < 4 * KT) Kc[row][col + 1] = v.y;
                if (col + 2 < 4 * KT) Kc[row][col + 2] = v.z;
                if (col + 3 < 4 * KT) Kc[row][col + 3] = v.w;
            }
        }
#pragma unroll
        for (int u = 0; u < EL; ++u) {
            const int i = tid + u * NT;
            if (i < 16 * (IM_NA / 2)) {
                const int row = i / (IM_NA / 2), a = 2 * (i - row * (IM_NA / 2));
                const float4 v = row < nrow ? epre[u] : float4{0.f, 0.f, 0.f, 0.f};
                Es[row][a] = {v.x, v.y};
                Es[row][a + 1] = {v.z, v.w};
            }
        }
    };

    const int c = cl & 1;
    int arow[CTW];
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) arow[ct] = (((wv * CTW + ct) * 16 + cl) >> 1) & (IM_NA - 1);
    const int rend = min(nrhs, (chunk + 1) * ppc);
    for (int r = chunk * ppc; r < rend; ++r) {
        float wa[CTW][KT];
#pragma unroll
        for (int ct = 0; ct < CTW; ++ct) {
            const int A = arow[ct];
            const cpx<float> *dp = win + (size_t)r * plane + ((size_t)A * nBl + mB) * QQ;
#pragma unroll
            for (int ks = 0; ks < KT; ++ks) {
                const int t = 4 * ks + kq;
                float v = 0.f;
                if (t < QQ) {
                    const cpx<float> d = dp[t], e = Er[A][t];
                    v = c ? fmaf(e.re, d.im, e.im * d.re) : fmaf(e.re, d.re, -e.im * d.im);
                }
                wa[ct][ks] = v;
            }
        }
        if (np > 0) fetch(0);
        for (int c0 = 0; c0 < np; c0 += 16) {
            lds_barrier();  // the previous tile's readers of Kc, Es and part are finished
            stash(c0);
            lds_barrier();
            if (c0 + 16 < np) fetch(c0 + 16);
            f32x4 acc[CTW];
#pragma unroll
            for (int ct = 0; ct < CTW; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KT; ++ks) {
                const float b = Kc[cl][4 * ks + kq];
#pragma unroll
                for (int ct = 0; ct < CTW; ++ct)
                    acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[ct][ks], b, acc[ct], 0, 0, 0);
            }
            // rows 4 kq + v of a tile: (A, re) for v = 0, 2 and (A, im) for v = 1, 3
            cpx<float> sacc = {0.f, 0.f};
#pragma unroll
            for (int ct = 0; ct < CTW; ++ct) {
                const int row0 = (wv * CTW + ct) * 16 + 4 * kq;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int A = ((row0 + 2 * h) >> 1) & (IM_NA - 1);
                    const cpx<float> y = {acc[ct][2 * h], acc[ct][2 * h + 1]};
                    const cpx<float> e = Es[cl][A];
                    sacc.re = fmaf(e.re, y.re, fmaf(e.im, y.im, sacc.re));  // conj(e) y
                    sacc.im = fmaf(e.re, y.im, fmaf(-e.im, y.re, sacc.im));
                }
            }
            sacc.re += __shfl_xor(sacc.re, 16);
            sacc.im += __shfl_xor(sacc.im, 16);
            sacc.re += __shfl_xor(sacc.re, 32);
            sacc.im += __shfl_xor(sacc.im, 32);
            if (kq == 0) part[wv][cl] = sacc;
            lds_barrier();
            if (tid < 16 && c0 + tid < np) {
                cpx<float> v = part[0][tid];
#pragma unroll
                for (int k = 1; k < 4; ++k) {
                    v.re += part[k][tid].re;
                    v.im += part[k][tid].im;
                }
                f[(size_t)r * n2 + src.idx[beg + c0 + tid]] = v;
            }
        }
    }
}

#define FIO_DISPATCH_QI(q, MACRO)             \
    switch (q) {                              \
        case 3: MACRO(3); break;              \
        case 4: MACRO(4); break;              \
        case 5: MACRO(5); break;              \
        case 6: MACRO(6); break;              \
        case 7: MACRO(7); break;              \
        case 8: MACRO(8); break;              \
        case 9: MACRO(9); break;              \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_init_tables(const Geom &g, const Tables &tb, const Sources &src, void *ktab,
                              hipStream_t st) {
    if (!init_mfma_supported(g.q, g.s)) return hipErrorInvalidValue;
    const int n2 = g.N * g.N;
    const unsigned nblk = (unsigned)(((size_t)n2 * im_ks(g.q) + NT - 1) / NT);
#define L_KT(Q) hipLaunchKernelGGL((k_init_ktab<Q>), dim3(nblk), dim3(NT), 0, st, g, tb, src.p, (float *)ktab, n2);
    FIO_DISPATCH_QI(g.q, L_KT)
#undef L_KT
    return hipGetLastError();
}

hipError_t launch_init_etab(const Geom &g, const PhaseDev &ph, const Sources &src, void *etab, hipStream_t st) {
    const int n2 = g.N * g.N;
    hipLaunchKernelGGL(k_init_etab, dim3((n2 + 63) / 64), dim3(NT), 0, st, g, ph, src.idx, (cpx<float> *)etab,
                       n2);
    return hipGetLastError();
}

hipError_t launch_init_mfma(const Geom &g, const PhaseDev &ph, const Tables &tb, const Sources &src,
                            const void *ktab, const void *etab, const void *f, void *fsorted, void *w, int nrhs,
                            size_t plane, hipStream_t st) {
    if (!init_mfma_supported(g.q, g.s)) return hipErrorInvalidValue;
    const int n2 = g.N * g.N;
    hipLaunchKernelGGL(k_gather_sorted, dim3((unsigned)(((size_t)n2 * nrhs + NT - 1) / NT)), dim3(NT), 0, st,
                       (const cpx<float> *)f, src.idx, (cpx<float> *)fsorted, n2, nrhs);
    const unsigned nB = 1u << (2 * (g.L - g.s));  // a multiple of 8 (s = 3, N >= 64)
    if (nB % 8) return hipErrorInvalidValue;
    const int rci = nrhs == 1 ? 1 : 2, npass = (nrhs + rci - 1) / rci;
    const int nch = std::min(IM_CH, npass), ppc = (npass + nch - 1) / nch;
#define L_IMM(Q)                                                                                          \
    if (nrhs == 1)                                                                                        \
        hipLaunchKernelGGL((k_init_mm<Q, 1>), dim3(nB * nch), dim3(NT), 0, st, g, ph, tb, src,            \
                           (const float *)ktab, (const cpx<float> *)etab, (const cpx<float> *)fsorted,    \
                           (cpx<float> *)w, nrhs, plane, nch, ppc);                                       \
    else                                                                                                  \
        hipLaunchKernelGGL((k_init_mm<Q, 2>), dim3(nB * nch), dim3(NT), 0, st, g, ph, tb, src,            \
                           (const float *)ktab, (const cpx<float> *)etab, (const cpx<float> *)fsorted,    \
                           (cpx<float> *)w, nrhs, plane, nch, ppc);
    FIO_DISPATCH_QI(g.q, L_IMM)
#undef L_IMM
    return hipGetLastError();
}

hipError_t launch_init_adj_mfma(const Geom &g, const PhaseDev &ph, const Tables &tb, const Sources &src,
                                const void *ktab, const void *etab, const void *w, void *f, int nrhs,
                                size_t plane, hipStream_t st) {
    if (!init_mfma_supported(g.q, g.s)) return hipErrorInvalidValue;
    const unsigned nB = 1u << (2 * (g.L - g.s));  // a multiple of 8 (s = 3, N >= 64)
    if (nB % 8) return hipErrorInvalidValue;
    const int nch = std::min(IM_CH, nrhs), ppc = (nrhs + nch - 1) / nch;
#define L_IAMM(Q)                                                                                         \
    hipLaunchKernelGGL((k_init_adj_mm<Q>), dim3(nB * nch), dim3(NT), 0, st, g, ph, tb, src,               \
                       (const float *)ktab, (const cpx<float> *)etab, (const cpx<float> *)w, (cpx<float> *)f, \
                       nrhs, plane, nch, ppc);
    FIO_DISPATCH_QI(g.q, L_IAMM)
#undef L_IAMM
    return hipGetLastError();
}

}  // namespace fio
