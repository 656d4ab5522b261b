// Batched level kernels with the interpolation contractions on the matrix
// cores (gfx950 v_mfma_f32_16x16x32_bf16): BF16 operands, FP32 accumulation.
//
// The weights stay complex64 in HBM (planes of one right-hand side each);
// the kernel values (FP64 phases, FP32 exponentials) are computed once per
// output pair and applied in FP32; only the operands of the two 1-D passes
// of the Kronecker sum (Sec. 4) are rounded to BF16.  Right-hand sides are
// processed in tiles of 16 (the MFMA's M dimension); a ragged last tile is
// masked.
#include <hip/hip_runtime.h>

#include "fio_kernels_common.h"

namespace fio {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int RT = 16;  // right-hand sides per MFMA tile

// B operand of both passes: Bk[k][n] = M_{k / q}[n][k % q] for k < 2q, n < q
// (zero elsewhere), i.e. the two Kronecker factors stacked along k.  Lane l
// holds k = 8 (l / 16) + e, n = l % 16, e = 0..7.
template <int Q>
__device__ __forceinline__ bf16x8 mcat_operand(const float *Mg, int lane) {
    bf16x8 b;
    const int n = lane & 15, g = lane >> 4;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = 8 * g + e;
        float v = 0.0f;
        if (k < 2 * Q && n < Q) {
            const int c = k / Q, tp = k - c * Q;
            v = Mg[(c * Q + n) * Q + tp];
        }
        b[e] = (__bf16)v;
    }
    return b;
}

// ===========================================================================
// p-recursion (eq:alg2b) at level l, batched, contractions on MFMA.
// One workgroup per butterfly block (A_p, B); wave j <-> output A_j.
// First pass per row k' = (c1, t'1):  C[r][t2] = sum_k V[r][k] Bk[k][t2],
//   V[r][(c2,t'2)] = E(x0(A_j), p^{B_c}_t') delta_r^{A_p B_c}_{t'1 t'2}, c = (c1,c2);
// second pass per column t2:           D[r][t1] = sum_k' W[r][k'] Bk[k'][t1],
//   W[r][k'] = C_{k'}[r][t2]; then conj E(x0(A_j), p^B_t) and store.
// ===========================================================================
template <int Q, bool STG>
__global__ __launch_bounds__(256) void k_plevel_mfma(Geom g, PhaseDev ph, Tables tb, int level,
                                                    const cpx<float> *__restrict__ win,
                                                    cpx<float> *__restrict__ wout, int nrhs, size_t plane) {
    constexpr int QQ = Q * Q;
    constexpr int KP = 24;                 // padded k' extent of the staged rows (>= 2q, multiple of 8)
    static_assert(2 * Q <= KP, "q too large for the MFMA p-level");
    __shared__ double rc[2 * Q], ctc[2 * Q], stc[2 * Q];
    __shared__ double rb[Q], ctb[Q], stb[Q];
    __shared__ cpx<float> Epre[4][4 * QQ];           // per output: E(x0(A_j), p^{B_c}_t') [c][t'1][t'2]
    __shared__ cpx<float> Erem[4][QQ];               // per output: E(x0(A_j), p^B_t)
    __shared__ __bf16 Wre[4][Q][RT][KP], Wim[4][Q][RT][KP];   // per output: first-pass rows [t2][r][k']
    // the block's inputs for one tile of right-hand sides, staged by coalesced
    // loads and read by all four waves (row r padded by one value: the 16
    // lanes that read one offset of 16 rows fall on different banks).  For
    // q > 7 the buffer would leave one workgroup per CU (measured slower at
    // q = 9), and a tile of fewer than RT / 2 right-hand sides gains nothing
    // from it: there each lane loads its own right-hand side's inputs from
    // global memory
    constexpr bool STAGE = STG && Q <= 7;  // STG: the launch has RT / 2 or more right-hand sides
    __shared__ cpx<float> xs[STAGE ? RT : 1][STAGE ? 4 * QQ + 1 : 1];

    const int tid = threadIdx.x;
    const int j = tid >> 6, lane = tid & 63;
    const int lB = g.L - level;
    const size_t nBl = (size_t)1 << (2 * lB);
    const size_t blk = blockIdx.x;
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
    // zero the padding k' in [2q, KP) of the staged rows once (none when 2q = KP)
    if constexpr (KP > 2 * Q) {
        for (int i = tid; i < 4 * Q * RT * (KP - 2 * Q); i += 256) {
            const int kp = 2 * Q + i % (KP - 2 * Q), rest = i / (KP - 2 * Q);
            const int r = rest % RT, rest2 = rest / RT;
            const int t2 = rest2 % Q, jj = rest2 / Q;
            Wre[jj][t2][r][kp] = (__bf16)0.0f;
            Wim[jj][t2][r][kp] = (__bf16)0.0f;
        }
    }
    __syncthreads();
    // kernel values of output j, shared by all right-hand sides
    {
        const int a1 = 2 * ap1 + (j >> 1), a2 = 2 * ap2 + (j & 1);
        const XP xp = make_xp(ph, box_centre(a1, level), box_centre(a2, level));
        for (int i = lane; i < 4 * QQ; i += 64) {
            const int c = i / QQ, t = i - c * QQ, tp1 = t / Q, tp2 = t - tp1 * Q;
            const int c1 = c >> 1, c2 = c & 1;
            Epre[j][i] = cis<float>(rc[c1 * Q + tp1] * phase_dir(xp, ctc[c2 * Q + tp2], stc[c2 * Q + tp2]));
        }
        for (int i = lane; i < QQ; i += 64) {
            const int t1 = i / Q, t2 = i - t1 * Q;
            Erem[j][i] = cis<float>(rb[t1] * phase_dir(xp, ctb[t2], stb[t2]));
        }
    }
    const bf16x8 Bk = mcat_operand<Q>(tb.Mf, lane);
    const int ln = lane & 15, lg = lane >> 4;
    cpx<float> *dst_pair = wout + ((size_t)(4 * mAp + j) * nBl + mB) * QQ;
    __syncthreads();

    for (int r0 = 0; r0 < nrhs; r0 += RT) {
        // stage the tile's inputs (4 q^2 consecutive values per right-hand
        // side; zero past nrhs); the previous tile's readers finished at the
        // barrier that closed it
        const bool staged = STAGE && nrhs - r0 >= RT / 2;  // uniform
        if (staged) {
            for (int i = tid; i < RT * 4 * QQ; i += 256) {
                const int r = i / (4 * QQ), o = i - r * (4 * QQ);
                xs[STAGE ? r : 0][STAGE ? o : 0] =
                    r0 + r < nrhs ? win[(size_t)(r0 + r) * plane + blk * 4 * QQ + o] : cpx<float>{0.f, 0.f};
            }
            __syncthreads();
        }
        // ---- first pass: rows k' = (c1, t'1); lane holds r = r0 + ln, k = 8 lg + e
        const int rA = r0 + ln;
        const bool rok = staged || rA < nrhs;  // staged rows past nrhs are zero
        const cpx<float> *src = staged ? &xs[STAGE ? ln : 0][0] : win + (size_t)min(rA, nrhs - 1) * plane + blk * 4 * QQ;
#pragma unroll 1
        for (int kr = 0; kr < 2 * Q; ++kr) {
            const int c1 = kr / Q, tp1 = kr - c1 * Q;
            bf16x8 are, aim;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * lg + e;
                float vr = 0.0f, vi = 0.0f;
                if (k < 2 * Q && rok) {
                    const int c2 = k / Q, tp2 = k - c2 * Q;
                    const int c = 2 * c1 + c2;
                    const cpx<float> d = src[c * QQ + tp1 * Q + tp2];
                    const cpx<float> v = cmul(Epre[j][c * QQ + tp1 * Q + tp2], d);
                    vr = v.re;
                    vi = v.im;
                }
                are[e] = (__bf16)vr;
                aim[e] = (__bf16)vi;
            }
            f32x4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
            cre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(are, Bk, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aim, Bk, cim, 0, 0, 0);
            // lane holds C[r = 4 lg + v][t2 = ln]
            if (ln < Q) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    Wre[j][ln][4 * lg + v][kr] = (__bf16)cre[v];
                    Wim[j][ln][4 * lg + v][kr] = (__bf16)cim[v];
                }
            }
        }
        __syncthreads();
        // ---- second pass: per column t2; lane holds r = ln, k' = 8 lg + e
#pragma unroll 1
        for (int t2 = 0; t2 < Q; ++t2) {
            bf16x8 are, aim;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int kp = 8 * lg + e;
                are[e] = kp < KP ? Wre[j][t2][ln][kp] : (__bf16)0.0f;
                aim[e] = kp < KP ? Wim[j][t2][ln][kp] : (__bf16)0.0f;
            }
            f32x4 dre = {0.f, 0.f, 0.f, 0.f}, dim = {0.f, 0.f, 0.f, 0.f};
            dre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(are, Bk, dre, 0, 0, 0);
            dim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aim, Bk, dim, 0, 0, 0);
            // lane holds D[r = 4 lg + v][t1 = ln]
            if (ln < Q) {
                const cpx<float> e = Erem[j][ln * Q + t2];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = r0 + 4 * lg + v;
                    if (r < nrhs) {
                        const cpx<float> o = {dre[v], dim[v]};
                        dst_pair[(size_t)r * plane + ln * Q + t2] = cmulc(o, e);
                    }
                }
            }
        }
        __syncthreads();
    }
}

template <int Q>
static hipError_t plevel_mfma_q(const Geom &g, const PhaseDev &ph, const Tables &tb, int level, const void *win,
                                void *wout, int nrhs, size_t plane, hipStream_t st) {
    const unsigned nblk = 1u << (2 * g.L - 2);
    // the staging buffer only where a tile can use it (its LDS would lower
    // the occupancy of a launch of a few right-hand sides for nothing)
    if (nrhs >= RT / 2)
        hipLaunchKernelGGL((k_plevel_mfma<Q, true>), dim3(nblk), dim3(256), 0, st, g, ph, tb, level,
                           (const cpx<float> *)win, (cpx<float> *)wout, nrhs, plane);
    else
        hipLaunchKernelGGL((k_plevel_mfma<Q, false>), dim3(nblk), dim3(256), 0, st, g, ph, tb, level,
                           (const cpx<float> *)win, (cpx<float> *)wout, nrhs, plane);
    return hipGetLastError();
}

bool mfma_supported_q(int q) { return q >= QMIN && q <= 12; }

hipError_t launch_plevel_mfma(const Geom &g, const PhaseDev &ph, const Tables &tb, int level, const void *win,
                              void *wout, int nrhs, size_t plane, hipStream_t st) {
    switch (g.q) {
        case 3: return plevel_mfma_q<3>(g, ph, tb, level, win, wout, nrhs, plane, st);
        case 4: return plevel_mfma_q<4>(g, ph, tb, level, win, wout, nrhs, plane, st);
        case 5: return plevel_mfma_q<5>(g, ph, tb, level, win, wout, nrhs, plane, st);
        case 6: return plevel_mfma_q<6>(g, ph, tb, level, win, wout, nrhs, plane, st);
        case 7: return plevel_mfma_q<7>(g, ph, tb, level, win, wout, nrhs, plane, st);
        case 8: return plevel_mfma_q<8>(g, ph, tb, level, win, wout, nrhs, plane, st);
        case 9: return plevel_mfma_q<9>(g, ph, tb, level, win, wout, nrhs, plane, st);
        case 10: return plevel_mfma_q<10>(g, ph, tb, level, win, wout, nrhs, plane, st);
        case 11: return plevel_mfma_q<11>(g, ph, tb, level, win, wout, nrhs, plane, st);
        case 12: return plevel_mfma_q<12>(g, ph, tb, level, win, wout, nrhs, plane, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fio
