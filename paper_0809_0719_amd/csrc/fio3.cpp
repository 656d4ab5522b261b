// Host side of the three-dimensional butterfly: the plan (spherical images
// of the frequencies sorted by their level-(L-s) box, interpolation tables,
// two weight buffers) and the level schedule driving fio_kernels_3d.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "fio_internal.h"

using namespace fio;

struct fio3_plan_s {
    Geom3 g{};
    int dtype = FIO_C64, device = 0;
    size_t plane = 0;  // N^3 q^3
    void *w0 = nullptr, *w1 = nullptr, *tab = nullptr, *srcbuf = nullptr;
    Tab3 tb{};
    Src3 src{};
};

namespace {

void free3(fio3_plan_s *p) {
    if (!p) return;
    (void)hipFree(p->w0);
    (void)hipFree(p->w1);
    (void)hipFree(p->tab);
    (void)hipFree(p->srcbuf);
    delete p;
}

double lagrange1(const std::vector<double> &z, int t, double u) {
    double v = 1.0;
    for (size_t j = 0; j < z.size(); ++j)
        if ((int)j != t) v *= (u - z[j]) / (z[t] - z[j]);
    return v;
}

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

}  // namespace

extern "C" {

int fio3_plan(int N, int q, int phase_kind, int s, int lm, int dtype, fio3_plan_t *out) {
    clear_error();
    if (!out) return set_error(FIO_EINVAL, "out is NULL");
    *out = nullptr;
    int L = 0;
    while ((1 << L) < N) ++L;
    if ((1 << L) != N || N < 4 || N > 256) return set_error(FIO_EINVAL, "N must be a power of two in [4, 256] (got %d)", N);
    if (q < 3 || q > 8) return set_error(FIO_EINVAL, "q must be in [3, 8] for three dimensions (got %d)", q);
    if (phase_kind != FIO3_PHASE_FOURIER && phase_kind != FIO3_PHASE_SPHERES)
        return set_error(FIO_EINVAL, "unknown three-dimensional phase kind %d", phase_kind);
    if (dtype != FIO_C64 && dtype != FIO_C128) return set_error(FIO_EINVAL, "unknown dtype %d", dtype);
    if (s < 0) s = std::min(3, L / 2);
    if (lm < 0) lm = L / 2;
    if (s > 3 || !(s <= lm && lm <= L - s))
        return set_error(FIO_EINVAL, "need 0 <= s <= 3 and s <= lm <= L - s (s=%d, lm=%d, L=%d)", s, lm, L);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_hip_error(e, "hipGetDevice");

    fio3_plan_s *p = new fio3_plan_s;
    p->dtype = dtype;
    p->device = dev;
    p->g = Geom3{N, L, q, s, lm, phase_kind, std::sqrt(3.0) / 2.0 * N};
    const size_t n3 = (size_t)N * N * N;
    p->plane = n3 * q * q * q;
    const size_t esz = dtype == FIO_C128 ? 16 : 8;

    // tables
    std::vector<double> z(q), lam(q);
    for (int i = 0; i < q; ++i) z[i] = 0.5 * std::cos(i * M_PI / (q - 1));
    if (q % 2) z[q / 2] = 0.0;
    for (int i = 0; i < q; ++i) z[q - 1 - i] = -z[i];  // exact symmetry (the nodes are symmetric)
    for (int i = 0; i < q; ++i) {
        double d = 1.0;
        for (int j = 0; j < q; ++j)
            if (j != i) d *= z[i] - z[j];
        lam[i] = 1.0 / d;
    }
    const int m = 1 << s;
    std::vector<double> Md(2 * q * q), Td(m * q);
    for (int c = 0; c < 2; ++c)
        for (int t = 0; t < q; ++t)
            for (int j = 0; j < q; ++j) Md[(c * q + t) * q + j] = lagrange1(z, t, (z[j] + c - 0.5) / 2.0);
    for (int j = 0; j < m; ++j)
        for (int t = 0; t < q; ++t) Td[j * q + t] = lagrange1(z, t, (double)j / m - 0.5);
    std::vector<float> Mf(Md.begin(), Md.end()), Tf(Td.begin(), Td.end());
    const size_t o_z = 0, o_lam = align256(q * 8), o_Md = o_lam + align256(q * 8), o_Td = o_Md + align256(Md.size() * 8),
                 o_Mf = o_Td + align256(Td.size() * 8), o_Tf = o_Mf + align256(Mf.size() * 4),
                 tbytes = o_Tf + align256(Tf.size() * 4);

    // sources: spherical images, sorted (stably) by their level-(L-s) box
    const int lB = L - s, nB = 1 << lB;
    const size_t nB3 = (size_t)nB * nB * nB;
    std::vector<double> pp(3 * n3);
    std::vector<int32_t> box(n3), idx(n3), off(nB3 + 1, 0);
    const double rs = std::sqrt(3.0) / 2.0 * N;
    for (size_t kk = 0; kk < n3; ++kk) {
        const double k1 = (double)(kk / ((size_t)N * N)) - N / 2, k2 = (double)((kk / N) % N) - N / 2,
                     k3 = (double)(kk % N) - N / 2;
        const double r = std::sqrt(k1 * k1 + k2 * k2 + k3 * k3);
        double p1 = r / rs, p2 = 0.0, p3 = 0.0;
        if (r > 0) {
            p2 = std::acos(std::min(1.0, std::max(-1.0, k3 / r))) / M_PI;
            p3 = std::atan2(k2, k1) / (2.0 * M_PI);
            if (p3 < 0) p3 += 1.0;
        }
        pp[3 * kk] = p1;
        pp[3 * kk + 1] = p2;
        pp[3 * kk + 2] = p3;
        int b[3];
        for (int d = 0; d < 3; ++d) b[d] = std::min((int)std::floor(pp[3 * kk + d] * nB), nB - 1);
        box[kk] = (b[0] * nB + b[1]) * nB + b[2];
        ++off[box[kk] + 1];
    }
    for (size_t i = 0; i < nB3; ++i) off[i + 1] += off[i];
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    std::vector<double> ps(3 * n3);
    for (size_t kk = 0; kk < n3; ++kk) {
        const int j = fill[box[kk]]++;
        idx[j] = (int32_t)kk;
        for (int d = 0; d < 3; ++d) ps[3 * j + d] = pp[3 * kk + d];
    }
    const size_t o_idx = 0, o_p = align256(n3 * 4), o_off = o_p + align256(n3 * 24), sbytes = o_off + align256((nB3 + 1) * 4);

    e = hipMalloc(&p->tab, tbytes);
    if (e == hipSuccess) e = hipMalloc(&p->srcbuf, sbytes);
    if (e == hipSuccess) e = hipMalloc(&p->w0, p->plane * esz);
    if (e == hipSuccess) e = hipMalloc(&p->w1, p->plane * esz);
    char *tb = (char *)p->tab, *sb = (char *)p->srcbuf;
    if (e == hipSuccess) e = hipMemcpy(tb + o_z, z.data(), q * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(tb + o_lam, lam.data(), q * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(tb + o_Md, Md.data(), Md.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(tb + o_Td, Td.data(), Td.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(tb + o_Mf, Mf.data(), Mf.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(tb + o_Tf, Tf.data(), Tf.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(sb + o_idx, idx.data(), n3 * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(sb + o_p, ps.data(), n3 * 24, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(sb + o_off, off.data(), (nB3 + 1) * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free3(p);
        return set_hip_error(e, "three-dimensional plan");
    }
    p->tb = Tab3{(const double *)(tb + o_z), (const double *)(tb + o_lam), (const double *)(tb + o_Md),
                 (const double *)(tb + o_Td), (const float *)(tb + o_Mf), (const float *)(tb + o_Tf)};
    p->src = Src3{(const int32_t *)(sb + o_idx), (const double *)(sb + o_p), (const int32_t *)(sb + o_off)};
    *out = p;
    return FIO_OK;
}

int fio3_apply(fio3_plan_t plan, const void *f, void *u, void *stream) {
    clear_error();
    if (!plan) return set_error(FIO_EINVAL, "plan is NULL");
    if (!f || !u || f == u) return set_error(FIO_EINVAL, "f and u must be distinct non-NULL device pointers");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != plan->device) e = hipSetDevice(plan->device);
    if (e != hipSuccess) return set_hip_error(e, "device");
    const Geom3 &g = plan->g;
    hipStream_t st = (hipStream_t)stream;
    void *a = plan->w0, *b = plan->w1;
    e = launch_step3(plan->dtype, 0, g, plan->tb, plan->src, g.s, f, a, st);
    for (int l = g.s + 1; e == hipSuccess && l <= g.lm; ++l) {
        e = launch_step3(plan->dtype, 1, g, plan->tb, plan->src, l, a, b, st);
        std::swap(a, b);
    }
    if (e == hipSuccess) e = launch_step3(plan->dtype, 2, g, plan->tb, plan->src, g.lm, nullptr, a, st);
    for (int l = g.lm + 1; e == hipSuccess && l <= g.L - g.s; ++l) {
        e = launch_step3(plan->dtype, 3, g, plan->tb, plan->src, l, a, b, st);
        std::swap(a, b);
    }
    if (e == hipSuccess) e = launch_step3(plan->dtype, 4, g, plan->tb, plan->src, g.L - g.s, a, u, st);
    return e == hipSuccess ? FIO_OK : set_hip_error(e, "three-dimensional launch");
}

int fio3_apply_adjoint(fio3_plan_t plan, const void *u, void *f, void *stream) {
    clear_error();
    if (!plan) return set_error(FIO_EINVAL, "plan is NULL");
    if (!f || !u || f == u) return set_error(FIO_EINVAL, "u and f must be distinct non-NULL device pointers");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != plan->device) e = hipSetDevice(plan->device);
    if (e != hipSuccess) return set_hip_error(e, "device");
    const Geom3 &g = plan->g;
    hipStream_t st = (hipStream_t)stream;
    void *a = plan->w0, *b = plan->w1;
    e = launch_step3_adj(plan->dtype, 4, g, plan->tb, plan->src, g.L - g.s, u, a, st);
    for (int l = g.L - g.s; e == hipSuccess && l > g.lm; --l) {
        e = launch_step3_adj(plan->dtype, 3, g, plan->tb, plan->src, l, a, b, st);
        std::swap(a, b);
    }
    if (e == hipSuccess) e = launch_step3_adj(plan->dtype, 2, g, plan->tb, plan->src, g.lm, nullptr, a, st);
    for (int l = g.lm; e == hipSuccess && l > g.s; --l) {
        e = launch_step3_adj(plan->dtype, 1, g, plan->tb, plan->src, l, a, b, st);
        std::swap(a, b);
    }
    if (e == hipSuccess) e = launch_step3_adj(plan->dtype, 0, g, plan->tb, plan->src, g.s, a, f, st);
    return e == hipSuccess ? FIO_OK : set_hip_error(e, "three-dimensional adjoint launch");
}

int fio3_destroy(fio3_plan_t plan) {
    clear_error();
    if (!plan) return FIO_OK;
    free3(plan);
    return FIO_OK;
}

}  // extern "C"
