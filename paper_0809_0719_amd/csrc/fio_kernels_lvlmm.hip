// Butterfly levels on the matrix cores for batches of complex64 right-hand
// sides (q <= 9); weights plane by plane as everywhere else,
// w[r plane + pair q^2 + t].
//
// Two steps share one structure: every output box pair of a butterfly block
// sums, inside one contraction, over the four input pairs of the block,
// after an input- and output-dependent prefactor, and is then remodulated:
//   p-level (eq:alg2b), block (A_p, B), outputs o = children A_j of A_p,
//     inputs i = children B_c of B:
//       Z_o[n] = sum_{i, k} M_i1[n1][k1] M_i2[n2][k2] E(x0(A_o), p^{B_i}_k) delta_i[k],
//       delta'_o[n] = conj E(x0(A_o), p^B_n) Z_o[n];
//   adjoint x-level (conjugate transpose of eq:alg2c), block (A_p, B),
//     outputs o = children B_c of B, inputs i = children A_a of A_p:
//       Z_o[n] = sum_{i, k} M_i1[n1][k1] M_i2[n2][k2] conj E(x^{A_i}_k, p0(B_o)) delta_i[k],
//       delta'_o[n] = E(x^{A_p}_n, p0(B_o)) Z_o[n],
// with M_c[n][k] = L_n((z_k + c - 1/2)/2) (Sec. 4: the Lagrange values of a
// parent basis at a child's nodes, the same for every pair and level).
//
// The Kronecker sum runs one dimension at a time (Sec. 4), and each
// one-dimensional pass uses the symmetry of the Chebyshev nodes,
// z_{q-1-k} = -z_k, which gives M_1 = J M_0 J (J reverses the order): for two
// inputs u (child 0) and y (child 1),
//     M_0 u + M_1 y = S (u + v) + A (u - v),  v = J y,
//     S[n] = (M_0[n] + M_0[q-1-n]) / 2,  A[n] = (M_0[n] - M_0[q-1-n]) / 2,
// where S[q-1-n] = S[n] and A[q-1-n] = -A[n]: only rows n < ceil(q/2) of S
// and n < floor(q/2) of A are needed, half the multiply-adds of [M_0 M_1].
// Both halves run as v_mfma_f32_4x4x1_16b_f32 (16 independent 4x4x1
// products per instruction; lane l = 4 b + x supplies row x of block b's
// A operand and column x of its B operand, and receives column x of its
// result): the A operand holds rows 0..3 of S or A (the row of lane l & 3),
// the B operand one value per lane -- every lane is one column, the real or
// the imaginary part of one right-hand side, so each K step is one MFMA over
// 32 right-hand sides.  At q = 9 the middle row of S (n = 4) is the one row
// outside the 4-row tiles; it runs on the vector ALUs.
//
// Per butterfly block one workgroup (4 waves: wave o computes output o);
// the prefactor and remodulation values of the block are made once in LDS
// (FP64 phases reduced mod 1, FP32 sine and cosine) and shared by every
// right-hand side.  A wave takes 16 right-hand sides at a time: lane
// (h, r, part), h the half of the wave.  For each row pair p the lower half
// runs pass 1 (the second dimension) of input row (0, p), the upper half of
// row (1, q-1-p); the halves exchange their results (v_permlane32_swap) and
// run pass 2 (the first dimension) with them as one K step -- the lower half
// accumulating the S rows, the upper half the A rows -- so no pass-1 result
// leaves the registers and a lane holds 4q + q accumulators.  The four input
// rows of a row pair (16 right-hand sides) are loaded once per workgroup
// with coalesced loads (consecutive threads, consecutive nodes of one
// plane), two row pairs ahead of their use, and pass through an LDS stage
// laid out right-hand side innermost, from which every wave reads its
// operands.
//
// Measured at N = 1024, q = 9, 64 right-hand sides: 35.6 ms per p-level
// against 26.7 ms for the vector-ALU kernel -- the 2-D accumulators and the
// prefetch buffers hold a wave at ~230 registers, two waves per SIMD, which
// leaves the LDS and matrix-core latencies exposed; the kernel is therefore
// an option of the plan (contraction FIO_CONTRACT_MFMA), not the default.
#include <hip/hip_runtime.h>

#include "fio_kernels_common.h"

namespace fio {

namespace {

using f32x4 = __attribute__((ext_vector_type(4))) float;

constexpr int LV_RG = 16;  // right-hand sides per wave step

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// (alpha, beta) with part(e d) = alpha d.re + beta d.im: part 0 is the real
// part, part 1 the imaginary part of the product.
__device__ __forceinline__ float2 part_coef(cpx<float> e, int part) {
    return part ? make_float2(e.im, e.re) : make_float2(e.re, -e.im);
}

// Lane-dependent choice between two values (never between two arrays: a
// select of addresses would move the arrays to private memory).
__device__ __forceinline__ float pick(bool c, float a, float b) { return c ? a : b; }
__device__ __forceinline__ f32x4 pick4(bool c, f32x4 a, f32x4 b) {
    return f32x4{pick(c, a[0], b[0]), pick(c, a[1], b[1]), pick(c, a[2], b[2]), pick(c, a[3], b[3])};
}

// The value of lane l ^ 32, `upper` = (l >= 32): v_permlane32_swap(a, b)
// leaves a = [a lower half, b lower half] and b = [a upper half, b upper half].
__device__ __forceinline__ float other_half(float x, bool upper) {
    const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, x),
                                                    false, false);
    return __builtin_bit_cast(float, upper ? r[0] : r[1]);
}

}  // namespace

bool level_mfma_supported(int q) { return q >= QMIN && q <= 9; }

template <int Q, bool ADJX>
__global__ __launch_bounds__(NT, 2) void k_level_mm(Geom g, PhaseDev ph, Tables tb, int level,
                                                    const float2 *__restrict__ win, float2 *__restrict__ wout,
                                                    int nrhs, size_t plane) {
    constexpr int QQ = Q * Q;
    constexpr int H = Q / 2, HS = (Q + 1) / 2, MID = (Q - 1) / 2;
    constexpr bool MIDV = (Q & 1) && MID >= 4;  // the middle row of S outside the tiles (q = 9)
    // one row pair: 4 input rows (segments) of Q nodes for LV_RG right-hand sides
    constexpr int PAIR_ELEMS = 4 * Q * LV_RG, LPT = (PAIR_ELEMS + NT - 1) / NT;
    constexpr int SROW = LV_RG + 1;      // stage row (one node of one segment) padded against bank conflicts
    constexpr int SPARE = (64 + SROW - 1) / SROW;  // rows taking the elements past a row pair (one per lane)
    __shared__ float2 stage[2][4 * Q + SPARE][SROW];  // [slot][segment, node][r]
    // prefactor and remodulation coefficients per lane part
    __shared__ float2 pre[2][4][4][QQ];  // [part][o][i][k]
    __shared__ float2 post[2][4][QQ];    // [part][o][n]
    __shared__ double rho_i[2][Q], cth_i[2][Q], sth_i[2][Q];  // p-level: the children's nodes
    __shared__ double rho_b[Q], cth_b[Q], sth_b[Q];           // p-level: B's nodes
    __shared__ double Gi[4][2][Q], Gb[4][Q];                   // p-level: direction phases
    __shared__ double sx[2][2][Q], cx[2][2][Q];                // x-level: sin/cos 2 pi x at the children's nodes
    __shared__ double spx[2][Q], cpx_[2][Q];                   // x-level: at A_p's nodes
    __shared__ double r0c[2], ct0[2], st0[2];                  // x-level: p0(B_c)

    const int tid = threadIdx.x, lane = tid & 63;
    const int o = __builtin_amdgcn_readfirstlane(tid >> 6);
    // lane: right-hand side rl of the step, part (real, imaginary), half h:
    // pass 1 of row (0, p) in the lower half, of row (1, q-1-p) in the upper;
    // pass 2 accumulates the S rows in the lower half, the A rows in the upper
    const int part = lane & 1, rl = (lane >> 1) & (LV_RG - 1), i4 = lane & 3;
    const bool hup = lane >= 32;
    const size_t blk = blockIdx.x;
    const int lB = g.L - level;
    const size_t nBl = (size_t)1 << (2 * lB);
    const uint32_t mB = (uint32_t)(blk & (nBl - 1)), mAp = (uint32_t)(blk >> (2 * lB));
    int b1, b2, ap1, ap2;
    morton_decode(mB, b1, b2);
    morton_decode(mAp, ap1, ap2);
    const bool ell = ph.kind == FIO_PHASE_ELLIPSE;

    // ---- kernel values of the block ---------------------------------------
    if constexpr (!ADJX) {
        if (tid < 2 * Q) {  // children's nodes: rho by (c1, k1), direction by (c2, k2)
            const int c = tid / Q, k = tid - c * Q;
            const double z = tb.z[k];
            rho_i[c][k] = g.rho_scale * box_node(2 * b1 + c, lB + 1, z);
            double s_, c_;
            sincospi(2.0 * box_node(2 * b2 + c, lB + 1, z), &s_, &c_);
            cth_i[c][k] = c_;
            sth_i[c][k] = s_;
        } else if (tid < 3 * Q) {  // B's nodes
            const int k = tid - 2 * Q;
            const double z = tb.z[k];
            rho_b[k] = g.rho_scale * box_node(b1, lB, z);
            double s_, c_;
            sincospi(2.0 * box_node(b2, lB, z), &s_, &c_);
            cth_b[k] = c_;
            sth_b[k] = s_;
        }
        lds_barrier();
        if (tid < 4 * 3 * Q) {  // direction phases G(x0(A_o), theta): children's (2q) and B's (q)
            const int oo = tid / (3 * Q), k = tid - oo * 3 * Q;
            const XP xp = make_xp(ph, box_centre(2 * ap1 + (oo >> 1), level), box_centre(2 * ap2 + (oo & 1), level));
            if (k < 2 * Q) {
                const int c = k / Q, kk = k - c * Q;
                Gi[oo][c][kk] = phase_dir(xp, cth_i[c][kk], sth_i[c][kk]);
            } else {
                Gb[oo][k - 2 * Q] = phase_dir(xp, cth_b[k - 2 * Q], sth_b[k - 2 * Q]);
            }
        }
        lds_barrier();
        for (int e = tid; e < 16 * QQ; e += NT) {  // prefactor E(x0(A_o), p^{B_i}_k)
            const int oo = e / (4 * QQ), r = e - oo * 4 * QQ, ii = r / QQ, k = r - ii * QQ;
            const int k1 = k / Q, k2 = k - k1 * Q;
            const cpx<float> v = cis<float>(rho_i[ii >> 1][k1] * Gi[oo][ii & 1][k2]);
            pre[0][oo][ii][k] = part_coef(v, 0);
            pre[1][oo][ii][k] = part_coef(v, 1);
        }
        for (int e = tid; e < 4 * QQ; e += NT) {  // remodulation conj E(x0(A_o), p^B_n)
            const int oo = e / QQ, n = e - oo * QQ, n1 = n / Q, n2 = n - n1 * Q;
            const cpx<float> v0 = cis<float>(rho_b[n1] * Gb[oo][n2]);
            const cpx<float> v = {v0.re, -v0.im};
            post[0][oo][n] = part_coef(v, 0);
            post[1][oo][n] = part_coef(v, 1);
        }
    } else {
        if (tid < 4 * Q) {  // sin/cos 2 pi x at the children's nodes [dim][a][k]
            const int d = tid / (2 * Q), a = (tid / Q) & 1, k = tid % Q;
            double s_ = 0, c_ = 1;
            if (ell) sincospi(2.0 * box_node(2 * (d ? ap2 : ap1) + a, level, tb.z[k]), &s_, &c_);
            sx[d][a][k] = s_;
            cx[d][a][k] = c_;
        } else if (tid < 6 * Q) {  // at A_p's nodes [dim][k]
            const int d = (tid - 4 * Q) / Q, k = (tid - 4 * Q) % Q;
            double s_ = 0, c_ = 1;
            if (ell) sincospi(2.0 * box_node(d ? ap2 : ap1, level - 1, tb.z[k]), &s_, &c_);
            spx[d][k] = s_;
            cpx_[d][k] = c_;
        } else if (tid < 6 * Q + 2) {  // p0(B_c): rho by c1, direction by c2
            const int c = tid - 6 * Q;
            r0c[c] = g.rho_scale * box_centre(2 * b1 + c, lB + 1);
            double s_, c_;
            sincospi(2.0 * box_centre(2 * b2 + c, lB + 1), &s_, &c_);
            ct0[c] = c_;
            st0[c] = s_;
        }
        lds_barrier();
        for (int e = tid; e < 4 * QQ; e += NT) {  // prefactor conj E(x^{A_i}_k, p0(B_o)), all o
            const int ii = e / QQ, k = e - ii * QQ, k1 = k / Q, k2 = k - k1 * Q;
            const int a1 = ii >> 1, a2 = ii & 1;
            const XP xp = make_xp_sc(ph, box_node(2 * ap1 + a1, level, tb.z[k1]), box_node(2 * ap2 + a2, level, tb.z[k2]),
                                     sx[0][a1][k1], cx[0][a1][k1], sx[1][a2][k2], cx[1][a2][k2]);
            const double G0 = phase_dir(xp, ct0[0], st0[0]), G1 = phase_dir(xp, ct0[1], st0[1]);
#pragma unroll
            for (int oo = 0; oo < 4; ++oo) {
                const cpx<float> v0 = cis<float>(r0c[oo >> 1] * ((oo & 1) ? G1 : G0));
                const cpx<float> v = {v0.re, -v0.im};
                pre[0][oo][ii][k] = part_coef(v, 0);
                pre[1][oo][ii][k] = part_coef(v, 1);
            }
        }
        for (int e = tid; e < QQ; e += NT) {  // remodulation E(x^{A_p}_n, p0(B_o)), all o
            const int n1 = e / Q, n2 = e - n1 * Q;
            const XP xp = make_xp_sc(ph, box_node(ap1, level - 1, tb.z[n1]), box_node(ap2, level - 1, tb.z[n2]),
                                     spx[0][n1], cpx_[0][n1], spx[1][n2], cpx_[1][n2]);
            const double G0 = phase_dir(xp, ct0[0], st0[0]), G1 = phase_dir(xp, ct0[1], st0[1]);
#pragma unroll
            for (int oo = 0; oo < 4; ++oo) {
                const cpx<float> v = cis<float>(r0c[oo >> 1] * ((oo & 1) ? G1 : G0));
                post[0][oo][e] = part_coef(v, 0);
                post[1][oo][e] = part_coef(v, 1);
            }
        }
    }

    // ---- the symmetric halves of M_0 for this lane's A-operand row --------
    const float *M0 = tb.Mf;  // M_0[n][k] = M0[n Q + k]
    __shared__ float Scol[2][4][Q];  // [S or A][row][k]: the pass-2 operands, read per row pair
    __shared__ float Smid[Q];        // the middle row of S (q = 9)
    float Sv[Q], Av[Q], Sm[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const float top = i4 < Q ? M0[min(i4, Q - 1) * Q + k] : 0.f;
        const float bot = i4 < Q ? M0[(Q - 1 - min(i4, Q - 1)) * Q + k] : 0.f;
        Sv[k] = i4 < HS ? 0.5f * (top + bot) : 0.f;
        Av[k] = i4 < H ? 0.5f * (top - bot) : 0.f;
        Sm[k] = MIDV ? M0[MID * Q + k] : 0.f;
        if (tid < 4) {
            Scol[0][i4][k] = Sv[k];
            Scol[1][i4][k] = Av[k];
        }
        if (tid == 0) Smid[k] = Sm[k];
    }
    lds_barrier();

    // ---- inputs and outputs of this block ---------------------------------
    // p-level: inputs (A_p, B_i) at blk 4 + i, outputs (A_o, B) at (4 mAp + o) nBl + mB;
    // adjoint x-level: inputs (A_i, B) at (4 mAp + i) nBl + mB, outputs (A_p, B_o) at blk 4 + o.
    auto in_pair = [&](int i) -> size_t { return ADJX ? (size_t)(4 * mAp + i) * nBl + mB : blk * 4 + i; };
    const size_t out_pair = ADJX ? blk * 4 + o : (size_t)(4 * mAp + o) * nBl + mB;
    const float2(*const prv)[QQ] = pre[part][o];
    const float2 *const pov = post[part][o];
    const int ngrp = (nrhs + LV_RG - 1) / LV_RG;

    // Row pair s: segment sg = (i1, i2) = (sg >> 1, sg & 1) at row k1 = p (i1 = 0)
    // or q - 1 - p (i1 = 1), nodes k2, right-hand sides grp 32 + r.  Element
    // e = (r 4 + sg) Q + k2 of the pair: consecutive threads read consecutive
    // nodes of one segment of one plane.  A thread's elements are the same in
    // every row pair; their offsets are made once.  Elements past the pair
    // (the last of the thread's LPT) go to a spare stage row.
    // (offsets within a plane fit 32 bits: N^2 q^2 < 2^32 for the q <= 9 served here)
    uint32_t gofs[LPT];
    int lofs[LPT], rkh[LPT];  // rkh: right-hand side r, plus 64 when the segment is a row q-1-p
#pragma unroll
    for (int k = 0; k < LPT; ++k) {
        const int e = tid + k * NT;
        const int r = e / (4 * Q), rem = e - r * 4 * Q, sg = rem / Q, k2 = rem - sg * Q;
        const bool ok = e < PAIR_ELEMS;
        rkh[k] = (ok ? r : 0) + ((sg >> 1) ? 64 : 0);
        gofs[k] = (uint32_t)(ok ? in_pair(sg & 3) * QQ + k2 : in_pair(0) * QQ);
        lofs[k] = ok ? (sg * Q + k2) * SROW + r : 4 * Q * SROW + (tid & 63);  // element offset in a stage slot
    }
    // Right-hand sides past nrhs load the last one's values (their columns'
    // results are never stored), so every load is in bounds and its value is
    // used as loaded.
    auto fetch = [&](int grp, int p, float2 (&buf)[LPT]) {
#pragma unroll
        for (int k = 0; k < LPT; ++k) {
            const size_t rg = (size_t)min(grp * LV_RG + (rkh[k] & 63), nrhs - 1);
            buf[k] = win[rg * plane + gofs[k] + ((rkh[k] & 64) ? Q - 1 - p : p) * Q];
        }
    };
    auto put = [&](int slot, const float2 (&buf)[LPT]) {
#pragma unroll
        for (int k = 0; k < LPT; ++k) (&stage[slot][0][0])[lofs[k]] = buf[k];
    };

    // pass 2 accumulators: S rows (lower half) or A rows (upper half) of the
    // lane's column for every n2, and the middle S row on the vector ALUs
    f32x4 ZC[Q];
    float Zm[Q];
    // pass 1 of this lane's input row at row pair p: children (i1, 0), (i1, 1)
    // (segments 2 i1, 2 i1 + 1) at row k1, i1 = h, k1 = p or q-1-p:
    // W[n2] = sum_{i2, k2} M_i2[n2][k2] y_(i1,i2)[k1][k2]
    auto pass1 = [&](int slot, int p, float (&W)[Q]) {
        const int iu = hup ? 2 : 0, k1 = hup ? Q - 1 - p : p;
        // per-lane row bases; the node offsets below are compile-time constants
        const float2 *const su = &stage[slot][iu * Q][rl];
        const float2 *const sv = &stage[slot][(iu + 1) * Q][rl];
        const float2 *const pu = &prv[iu][k1 * Q];
        const float2 *const pv = &prv[iu + 1][k1 * Q];
        f32x4 aS = {0.f, 0.f, 0.f, 0.f}, aA = {0.f, 0.f, 0.f, 0.f};
        float sm = 0.f;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const float2 du = su[k * SROW], dv = sv[(Q - 1 - k) * SROW];
            const float2 cu = pu[k], cv = pv[Q - 1 - k];
            const float yu = fmaf(cu.x, du.x, cu.y * du.y), yv = fmaf(cv.x, dv.x, cv.y * dv.y);
            const float a = yu + yv, b = yu - yv;
            aS = mfma4(Sv[k], a, aS);
            aA = mfma4(Av[k], b, aA);
            if (MIDV) sm = fmaf(Sm[k], a, sm);
            if (k % 3 == 2) __builtin_amdgcn_sched_barrier(0);  // bound the operand reads in flight
        }
#pragma unroll
        for (int n = 0; n < H; ++n) {
            W[n] = aS[n] + aA[n];
            W[Q - 1 - n] = aS[n] - aA[n];
        }
        if constexpr (Q & 1) W[MID] = MIDV ? sm : aS[MID & 3];
    };
    auto compute = [&](int p, int slot) {
        float W[Q];
        pass1(slot, p, W);
        // pass 2, K step p: Z[n1][n2] += S[n1][p] (W0 + W1)[n2] + A[n1][p] (W0 - W1)[n2],
        // W0 in the lower half, W1 in the upper half of the wave
        const float cp = Scol[hup ? 1 : 0][i4][p];
        const float mp = MIDV ? Smid[p] : 0.f;
#pragma unroll
        for (int n2 = 0; n2 < Q; ++n2) {
            const float wo = other_half(W[n2], hup);
            const float x = hup ? wo - W[n2] : W[n2] + wo;  // (W0 - W1) or (W0 + W1)
            ZC[n2] = mfma4(cp, x, ZC[n2]);
            if (MIDV) Zm[n2] = fmaf(mp, x, Zm[n2]);
        }
    };
    // Z[n1][n2] of this lane's part: S rows from the lower half, A rows from
    // the upper half (lane ^ 32), the middle row from the lower half.
    // The four lanes of a right-hand side (h, part) store a quarter of the
    // nodes each, as whole remodulated complex values: nodes 4m + 2h + part,
    // the part lanes exchanging the other part of each (DPP).
    auto store_group = [&](int grp) {
        const int rg = grp * LV_RG + rl;
        float2 *dst = wout + (size_t)min(rg, nrhs - 1) * plane + out_pair * QQ;
        f32x4 ZO[Q];
        float Zmo[Q];
#pragma unroll
        for (int n2 = 0; n2 < Q; ++n2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) ZO[n2][v] = other_half(ZC[n2][v], hup);
            Zmo[n2] = MIDV ? other_half(Zm[n2], hup) : 0.f;
        }
        auto zval = [&](int n) -> float {
            const int n1 = n / Q, n2 = n - n1 * Q;
            const f32x4 zc = ZC[n2], zo = ZO[n2];
            const f32x4 zs = pick4(hup, zo, zc), za = pick4(hup, zc, zo);
            if (n1 < H) return zs[n1] + za[n1];
            if ((Q & 1) && n1 == MID) return MIDV ? pick(hup, Zmo[n2], Zm[n2]) : zs[MID & 3];
            return zs[Q - 1 - n1] - za[Q - 1 - n1];
        };
        // right-hand sides past nrhs keep their lanes busy and store nothing
        auto store_all = [&](bool guarded) {
#pragma unroll
            for (int m = 0; m < (QQ + 3) / 4; ++m) {
                // nodes (4m, 4m + 1) in the lower half, (4m + 2, 4m + 3) in the upper;
                // the register indices stay compile-time constants
                const int a0 = min(4 * m, QQ - 1), a1 = min(4 * m + 1, QQ - 1);
                const int b0 = min(4 * m + 2, QQ - 1), b1 = min(4 * m + 3, QQ - 1);
                const float za0 = zval(a0), za1 = zval(a1), zb0 = zval(b0), zb1 = zval(b1);
                const int n0 = hup ? b0 : a0, n1 = hup ? b1 : a1;
                const float z0 = pick(hup, zb0, za0), z1 = pick(hup, zb1, za1);  // own part of nodes n0, n1
                // part 0 keeps node n0 and needs its imaginary part from part 1;
                // part 1 keeps node n1 and needs its real part from part 0
                const float got = swap_adjacent_lanes(part ? z0 : z1);
                const int n = part ? n1 : n0;
                const float zr = part ? got : z0, zi = part ? z1 : got;
                const float2 c = post[0][o][n];  // (E.re, -E.im)
                const float2 v = make_float2(fmaf(c.x, zr, c.y * zi), fmaf(c.x, zi, -c.y * zr));
                if (!guarded || rg < nrhs) dst[n] = v;
            }
        };
        if (grp * LV_RG + LV_RG <= nrhs)  // uniform
            store_all(false);
        else
            store_all(true);
    };

    // Pipeline per group of 16 right-hand sides, row pairs p = 0 .. q-1: the
    // loads of row pair p + 3 are issued while row pair p is computed, row pair
    // p + 1 goes from registers to its LDS slot before (past the last row pair
    // both repeat it); row pairs 0 and 1 of the next group are loaded before
    // this group's outputs are stored (past the last group they repeat its
    // first ones).  Every step issues the same loads, so the loads in flight
    // are the same on every path.  Register buffers: bufA holds the even row
    // pairs, bufB the odd ones.
    float2 bufA[LPT], bufB[LPT];
    auto step = [&](int grp, int p, float2 (&nxt)[LPT]) {
        lds_barrier();  // slot p & 1 complete; every read of slot (p + 1) & 1 (row pair p - 1) done
        put((p + 1) & 1, nxt);
        fetch(grp, min(p + 3, Q - 1), nxt);
        compute(p, p & 1);
    };
    fetch(0, 0, bufA);
    fetch(0, 1, bufB);
#pragma unroll 1
    for (int grp = 0; grp < ngrp; ++grp) {
        lds_barrier();  // the previous group's reads of slot 0 are done
        put(0, bufA);
        fetch(grp, min(2, Q - 1), bufA);
#pragma unroll
        for (int n = 0; n < Q; ++n) {
            ZC[n] = f32x4{0.f, 0.f, 0.f, 0.f};
            Zm[n] = 0.f;
        }
#pragma unroll 1
        for (int p = 0; p + 1 < Q; p += 2) {
            step(grp, p, bufB);
            step(grp, p + 1, bufA);
        }
        if (Q & 1) step(grp, Q - 1, bufB);
        const int gn = min(grp + 1, ngrp - 1);
        fetch(gn, 0, bufA);
        fetch(gn, 1, bufB);
        store_group(grp);
    }
}

// One workgroup per butterfly block (N^2 / 4 blocks), right-hand sides in
// steps of 32, weights planes `plane` complex values apart.
hipError_t launch_level_mm(bool adjoint_x, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                           const void *w_in, void *w_out, int nrhs, size_t plane, hipStream_t st) {
    const size_t nblk = (size_t)g.N * g.N / 4;
    if (nrhs < 1 || nblk > 0x7fffffffu) return hipErrorInvalidValue;
#define L_LV(Q)                                                                                                \
    if (adjoint_x)                                                                                             \
        hipLaunchKernelGGL((k_level_mm<Q, true>), dim3((unsigned)nblk), dim3(NT), 0, st, g, ph, tb, level,    \
                           (const float2 *)w_in, (float2 *)w_out, nrhs, plane);                                \
    else                                                                                                       \
        hipLaunchKernelGGL((k_level_mm<Q, false>), dim3((unsigned)nblk), dim3(NT), 0, st, g, ph, tb, level,   \
                           (const float2 *)w_in, (float2 *)w_out, nrhs, plane);
    switch (g.q) {
        case 3: L_LV(3); break;
        case 4: L_LV(4); break;
        case 5: L_LV(5); break;
        case 6: L_LV(6); break;
        case 7: L_LV(7); break;
        case 8: L_LV(8); break;
        case 9: L_LV(9); break;
        default: return hipErrorInvalidValue;
    }
#undef L_LV
    return hipGetLastError();
}

}  // namespace fio
