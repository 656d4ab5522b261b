// Shared device helpers and launch-shape constants of the butterfly kernels
// (forward kernels in fio_kernels_fwd.hip, adjoints in fio_kernels_adj.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fio_device.h"

namespace fio {

constexpr int NT = 256;  // threads per workgroup for every kernel here

// ---------------------------------------------------------------------------
// Shared helpers
// ---------------------------------------------------------------------------

// Lagrange basis values L_t(u), t < Q, on the Chebyshev grid z (barycentric
// form of the second kind, with lam the barycentric weights).
template <typename T, int Q>
__device__ __forceinline__ void lagrange_row(double u, const double *z, const double *lam, T *out) {
    int exact = -1;
    double ssum = 0.0;
    double tmp[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t) {
        const double d = u - z[t];
        if (d == 0.0) exact = t;
        tmp[t] = lam[t] / d;
        ssum += tmp[t];
    }
    if (exact >= 0) {
#pragma unroll
        for (int t = 0; t < Q; ++t) out[t] = (T)(t == exact ? 1.0 : 0.0);
    } else {
        const double inv = 1.0 / ssum;
#pragma unroll
        for (int t = 0; t < Q; ++t) out[t] = (T)(tmp[t] * inv);
    }
}

template <typename T>
__device__ __forceinline__ const T *pick_M(const Tables &tb);
template <>
__device__ __forceinline__ const float *pick_M<float>(const Tables &tb) { return tb.Mf; }
template <>
__device__ __forceinline__ const double *pick_M<double>(const Tables &tb) { return tb.M; }

template <typename T>
__device__ __forceinline__ const T *pick_SA(const Tables &tb);
template <>
__device__ __forceinline__ const float *pick_SA<float>(const Tables &tb) { return tb.SAf; }
template <>
__device__ __forceinline__ const double *pick_SA<double>(const Tables &tb) { return tb.SA; }

template <typename T>
__device__ __forceinline__ const T *pick_T(const Tables &tb);
template <>
__device__ __forceinline__ const float *pick_T<float>(const Tables &tb) { return tb.Ttf; }
template <>
__device__ __forceinline__ const double *pick_T<double>(const Tables &tb) { return tb.Tt; }

// ===========================================================================
// Butterfly blocks per workgroup for the level kernels: 8q threads per block
// (2q per output pair), limited so the block's LDS stays near 40 KB.
// ===========================================================================
template <typename T, int Q, int PERBB>
constexpr int blocks_per_wg() {
    constexpr int byT = NT / (8 * Q);
    constexpr int byL = 40960 / (PERBB * Q * Q * (int)sizeof(cpx<T>));
    constexpr int b = byT < byL ? byT : byL;
    return b < 1 ? 1 : b;
}

// B boxes per chunk: keeps the chunk's weights and partial sums within 32 KB of LDS.
template <typename T, int Q>
constexpr int bch() {
    return (32768 / (Q * Q * 2 * (int)sizeof(T))) < 16 ? (32768 / (Q * Q * 2 * (int)sizeof(T))) : 16;
}

// right-hand sides per chunk of the switch kernels
template <typename T>
constexpr int switch_rc() { return sizeof(T) == 4 ? 8 : 4; }

template <typename T>
constexpr int swadj_rc() { return sizeof(T) == 4 ? 4 : 2; }


// Padding (complex64 elements) of the level kernels' LDS buffers, chosen per
// q with a model of the LDS banks (32 banks of 4 bytes, 64-bit accesses
// served 16 lanes at a time) over both passes' lane-to-address maps:
//   pad_sum_out: after each child's 4 q^2 first-pass rows in the kernels
//     whose passes feed one input to two children (x-level, p-level^H);
//   pad_plevel: after each output's 2 q^2 first-pass rows of the p-level;
//   pad_xadj_c, pad_xadj_j: after each q^2 block of c, and after each j1
//     block, of the x-level^H.
// Complex128 buffers are not padded.
template <typename T, int Q>
constexpr int pad_sum_out() {
    constexpr int t[17] = {0, 0, 0, 15, 4, 1, 6, 3, 8, 5, 10, 7, 12, 9, 14, 11, 0};
    return sizeof(T) == 4 ? t[Q] : 0;
}
template <typename T, int Q>
constexpr int pad_plevel() {
    constexpr int t[17] = {0, 0, 0, 0, 2, 3, 14, 5, 8, 7, 2, 9, 12, 11, 6, 13, 0};
    return sizeof(T) == 4 ? t[Q] : 0;
}
template <typename T, int Q>
constexpr int pad_xadj_c() {
    constexpr int t[17] = {0, 0, 0, 10, 3, 0, 2, 6, 1, 8, 6, 2, 12, 4, 10, 14, 0};
    return sizeof(T) == 4 ? t[Q] : 0;
}
template <typename T, int Q>
constexpr int pad_xadj_j() {
    constexpr int t[17] = {0, 0, 0, 2, 0, 0, 4, 10, 0, 14, 4, 10, 0, 6, 4, 2, 0};
    return sizeof(T) == 4 ? t[Q] : 0;
}

// Coalesced staging of a workgroup's input weights for one right-hand side:
// NE complex values made of pieces of consecutive values of a weight plane
// (piece(e) gives the plane offset of staged element e), copied through
// registers into an LDS buffer of stage_len<NE>() values in element order.
// Thread tid moves elements tid, tid + NT, ...: consecutive lanes read
// consecutive addresses, so a load instruction reads 64 adjacent values
// instead of 64 rows q values apart.  Elements past NE read element 0 of the
// plane and land in the buffer's tail, which nothing reads.  The offsets are
// recomputed per fetch (a few integer operations) rather than held in
// registers for the whole kernel.
template <int NE>
constexpr int stage_len() {
    return ((NE + NT - 1) / NT) * NT;
}
template <int NE>
constexpr int stage_per() {
    return (NE + NT - 1) / NT;
}
template <int NE, typename T, typename F>
__device__ __forceinline__ void stage_fetch(cpx<T> (&v)[stage_per<NE>()], const cpx<T> *plane, F &&piece) {
#pragma unroll
    for (int k = 0; k < stage_per<NE>(); ++k) {
        const int e = (int)threadIdx.x + k * NT;
        v[k] = plane[e < NE ? piece(e) : (size_t)0];
    }
}
template <int NE, typename T>
__device__ __forceinline__ void stage_put(const cpx<T> (&v)[stage_per<NE>()], cpx<T> *stage) {
#pragma unroll
    for (int k = 0; k < stage_per<NE>(); ++k) stage[threadIdx.x + k * NT] = v[k];
}

// Grids of more than 2^32 / NT workgroups (the work-item limit of one grid
// dimension): the workgroups are laid out over (x, y) with x at most 2^16,
// and kernels take their linear index.  Workgroups past the count the
// launcher asked for are the kernel's to skip.
__device__ __forceinline__ size_t linear_block() { return (size_t)blockIdx.y * gridDim.x + blockIdx.x; }
inline dim3 grid_of(size_t nblocks) {
    const size_t gx = nblocks < 65536 ? nblocks : 65536;
    return dim3((unsigned)gx, (unsigned)((nblocks + gx - 1) / gx));
}

// Workgroup barrier that orders LDS accesses only: global loads still in
// flight stay in flight across it (__syncthreads also waits for them), so a
// register prefetch may be issued anywhere.  For kernels whose threads do
// not exchange data through global memory within the workgroup.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The value of the neighbouring lane (lane ^ 1), through a DPP quad
// permutation [1,0,3,2] on the vector ALU (no LDS-pipe shuffle).
__device__ __forceinline__ float swap_adjacent_lanes(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ double swap_adjacent_lanes(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0xB1, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// f(std::integral_constant<int, v>) for a wave-uniform v in [I, N): code that
// indexes wave-uniform tables by v is then compiled once per value, with the
// table offsets known (batched scalar loads, no per-element branches).
template <int I, int N, typename F>
__device__ __forceinline__ void with_uniform(int v, F &&f) {
    if constexpr (I < N) {
        if (v == I)
            f(std::integral_constant<int, I>{});
        else
            with_uniform<I + 1, N>(v, f);
    }
}

// A pointer into the constant address space: wave-uniform loads through it
// are scalar loads (s_load, through the scalar cache) whatever the stores
// around them.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ cptr<T> to_constant(const T *p) {
    return (cptr<T>)p;
}

// Makes a wave-uniform pointer opaque to the optimiser (an empty asm that
// claims to update the SGPR pair holding it).  Called once per right-hand
// side on the interpolation-table pointer, it keeps the table's scalar
// loads (scalar-cache hits) inside the loop: as loop invariants the compiler
// would hoist them, and with more table values than SGPRs it parks them in
// VGPRs for the whole loop, costing waves per SIMD.
template <typename T>
__device__ __forceinline__ void opaque_sgpr(cptr<T> &p) {
    asm volatile("" : "+s"(p));
}

#define FIO_DISPATCH_Q(q, MACRO) \
    switch (q) {                 \
        case 3: MACRO(3); break; \
        case 4: MACRO(4); break; \
        case 5: MACRO(5); break; \
        case 6: MACRO(6); break; \
        case 7: MACRO(7); break; \
        case 8: MACRO(8); break; \
        case 9: MACRO(9); break; \
        case 10: MACRO(10); break; \
        case 11: MACRO(11); break; \
        case 12: MACRO(12); break; \
        case 13: MACRO(13); break; \
        case 14: MACRO(14); break; \
        case 15: MACRO(15); break; \
        case 16: MACRO(16); break; \
        default: return hipErrorInvalidValue; \
    }

#define FIO_BY_DTYPE(dtype, CALL) \
    ((dtype) == FIO_C128 ? CALL(double) : CALL(float))

}  // namespace fio
