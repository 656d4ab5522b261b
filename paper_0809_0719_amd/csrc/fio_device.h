// Device-side building blocks of the butterfly kernels: complex arithmetic,
// the FP64 phase with its exact mod-1 reduction, the polar / Cartesian
// geometry of the two quadtrees, and Morton index helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fio_internal.h"

namespace fio {

template <typename T>
struct cpx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T>
__device__ __forceinline__ void cfma(cpx<T> &acc, cpx<T> a, cpx<T> b) {
    acc.re = fma(a.re, b.re, fma(-a.im, b.im, acc.re));
    acc.im = fma(a.re, b.im, fma(a.im, b.re, acc.im));
}
// acc += a * conj(b)
template <typename T>
__device__ __forceinline__ void cfmac(cpx<T> &acc, cpx<T> a, cpx<T> b) {
    acc.re = fma(a.re, b.re, fma(a.im, b.im, acc.re));
    acc.im = fma(a.im, b.re, fma(-a.re, b.im, acc.im));
}
// acc += r * a  (r real)
template <typename T>
__device__ __forceinline__ void crfma(cpx<T> &acc, T r, cpx<T> a) {
    acc.re = fma(r, a.re, acc.re);
    acc.im = fma(r, a.im, acc.im);
}

// exp(2 pi i phi) for a phase given in cycles.  The argument is reduced
// mod 1 in FP64 (exact: |phi| << 2^52); the exponential of the reduced
// r in [-1/2, 1/2] is taken in the weight precision.  The FP32 version uses
// the hardware sine/cosine, whose argument is in revolutions.
template <typename T>
__device__ __forceinline__ cpx<T> cis(double phi);

template <>
__device__ __forceinline__ cpx<float> cis<float>(double phi) {
    const float r = (float)(phi - rint(phi));
    return {__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r)};
}
template <>
__device__ __forceinline__ cpx<double> cis<double>(double phi) {
    const double r = phi - rint(phi);
    double s, c;
    sincospi(2.0 * r, &s, &c);
    return {c, s};
}

// Per-target-point data of the phase: x and the squared ellipse axes
// C_j = c_j(x)^2 (zero for the Fourier phase, which removes the root term).
struct XP {
    double x1, x2, C1, C2;
};

__device__ __forceinline__ XP make_xp_sc(const PhaseDev &ph, double x1, double x2,
                                         double s1, double c1, double s2, double c2) {
    XP r{x1, x2, 0.0, 0.0};
    if (ph.kind == FIO_PHASE_ELLIPSE) {
        const double v1 = ph.a1 * (2.0 + (1.0 + ph.eta1) * s1 * s2) * (1.0 / 3.0);
        const double v2 = ph.a2 * (2.0 + (1.0 + ph.eta2) * c1 * c2) * (1.0 / 3.0);
        r.C1 = v1 * v1;
        r.C2 = v2 * v2;
    }
    return r;
}

__device__ __forceinline__ XP make_xp(const PhaseDev &ph, double x1, double x2) {
    double s1 = 0, c1 = 1, s2 = 0, c2 = 1;
    if (ph.kind == FIO_PHASE_ELLIPSE) {
        sincospi(2.0 * x1, &s1, &c1);
        sincospi(2.0 * x2, &s2, &c2);
    }
    return make_xp_sc(ph, x1, x2, s1, c1, s2, c2);
}

// Phi(x, e) for a unit direction e = (ct, st).  By homogeneity,
// Phi(x, k) = |k| * Phi(x, k/|k|), so a polar node p costs one product
// rho(p1) * G(x, theta(p2)) once G is known.
__device__ __forceinline__ double phase_dir(const XP &x, double ct, double st) {
    return fma(x.x1, ct, x.x2 * st) + sqrt(fma(x.C1 * ct, ct, x.C2 * st * st));
}

// Phi(x, k) for a Cartesian frequency k (the sources' own phases).
__device__ __forceinline__ double phase_cart(const XP &x, double k1, double k2) {
    return fma(x.x1, k1, x.x2 * k2) + sqrt(fma(x.C1 * k1, k1, x.C2 * k2 * k2));
}

// Box geometry: box b (per-dimension index) at `level` of a tree on [0,1].
__device__ __forceinline__ double box_centre(int b, int level) {
    return ((double)b + 0.5) * ldexp(1.0, -level);
}
__device__ __forceinline__ double box_node(int b, int level, double z) {
    return ((double)b + 0.5 + z) * ldexp(1.0, -level);
}

// Morton helpers: m = interleave(b1 at odd bits, b2 at even bits).
__device__ __forceinline__ uint32_t compact_even(uint32_t x) {
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return x;
}
__device__ __forceinline__ void morton_decode(uint32_t m, int &b1, int &b2) {
    b2 = (int)compact_even(m);
    b1 = (int)compact_even(m >> 1);
}

}  // namespace fio
