// Host side of the C ABI: argument validation, the plan (trees of Sec. 4
// step 1, interpolation tables, workspace), and the level schedule that
// drives the kernels of fio_kernels_fwd.hip, fio_kernels_adj.hip,
// fio_kernels_init.hip, fio_kernels_term.hip, fio_kernels_mfma.hip,
// fio_kernels_tan.hip and fio_kernels_amp.hip.  Batches of plans, the
// direct evaluation at sampled targets and the choice of q are in
// fio_batch.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fio_internal.h"

using namespace fio;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? FIO_ENOMEM : FIO_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int ilog2_exact(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return ((1 << l) == n) ? l : -1;
}

uint32_t morton(uint32_t b1, uint32_t b2) {
    uint32_t m = 0;
    for (int i = 0; i < 16; ++i) {
        m |= ((b2 >> i) & 1u) << (2 * i);
        m |= ((b1 >> i) & 1u) << (2 * i + 1);
    }
    return m;
}

int validate_phase(const fio_phase_t *ph) {
    if (!ph) return fail(FIO_EINVAL, "phase is NULL");
    if (ph->kind != FIO_PHASE_FOURIER && ph->kind != FIO_PHASE_ELLIPSE)
        return fail(FIO_EINVAL, "unknown phase kind %d", ph->kind);
    if (ph->kind == FIO_PHASE_ELLIPSE) {
        if (!(ph->a1 > 0.0) || !(ph->a2 > 0.0) || !std::isfinite(ph->a1) || !std::isfinite(ph->a2))
            return fail(FIO_EINVAL, "ellipse phase needs a1, a2 > 0 (got %g, %g)", ph->a1, ph->a2);
        if (!(ph->eta1 >= -1.0 && ph->eta1 <= 1.0) || !(ph->eta2 >= -1.0 && ph->eta2 <= 1.0))
            return fail(FIO_EINVAL, "ellipse phase needs -1 <= eta1, eta2 <= 1 (got %g, %g)", ph->eta1, ph->eta2);
    }
    return FIO_OK;
}

PhaseDev to_dev(const fio_phase_t *ph) {
    PhaseDev d;
    d.kind = ph->kind;
    d.a1 = ph->a1;
    d.a2 = ph->a2;
    d.eta1 = ph->eta1;
    d.eta2 = ph->eta2;
    return d;
}

// Lagrange basis L_t(u) on nodes z (product form), for the host tables.
double lagrange(const std::vector<double> &z, int t, double u) {
    double v = 1.0;
    for (size_t j = 0; j < z.size(); ++j)
        if ((int)j != t) v *= (u - z[j]) / (z[t] - z[j]);
    return v;
}

}  // namespace

struct fio_plan_s {
    int N = 0, q = 0, L = 0, s = 0, lm = 0, dtype = FIO_C64, device = 0, nrhs_max = 1;
    int chunk = 1;  // right-hand sides per pass (<= nrhs_max; tuned)
    int contract = FIO_CONTRACT_FP;
    fio_phase_t phase{};
    int max_box = 0;
    size_t wbytes = 0;       // bytes of one right-hand side's weights (one plane)
    size_t plane = 0;        // complex values per plane = N^2 q^2
    size_t total_bytes = 0;  // all device memory of the plan
    void *w0 = nullptr, *w1 = nullptr;
    void *t0 = nullptr, *t1 = nullptr;  // tangent workspace (3 planes each), when nrhs_max < 3
    bool init_mm = false;               // initialisation on the matrix cores
    void *ktab = nullptr, *etab = nullptr;
    bool etab_ok = false;               // etab holds the kernel values of the current phase
    void *amp0 = nullptr, *amp1 = nullptr;  // separated-amplitude workspace, amp_cap planes each
    int amp_cap = 0;
    void *dtab = nullptr;    // tables
    int32_t *d_idx = nullptr, *d_off = nullptr;
    double2 *d_p = nullptr;
    Tables tb{};
    Geom geom{};
    // profiling: event pairs recorded around each launch
    bool prof = false;
    std::vector<hipEvent_t> ev;      // 2 per recorded launch
    std::vector<int> ev_kind;
    size_t ev_used = 0;
};

namespace {

void free_plan(fio_plan_s *p) {
    if (!p) return;
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    (void)hipFree(p->w0);
    (void)hipFree(p->w1);
    (void)hipFree(p->t0);
    (void)hipFree(p->t1);
    (void)hipFree(p->ktab);
    (void)hipFree(p->etab);
    (void)hipFree(p->amp0);
    (void)hipFree(p->amp1);
    (void)hipFree(p->dtab);
    (void)hipFree(p->d_idx);
    (void)hipFree(p->d_off);
    (void)hipFree(p->d_p);
    delete p;
}

int dmalloc(void **ptr, size_t bytes, size_t *total, const char *what) {
    hipError_t e = hipMalloc(ptr, bytes ? bytes : 16);
    if (e != hipSuccess) {
        *ptr = nullptr;
        return hip_fail(e, what);
    }
    *total += bytes;
    return FIO_OK;
}

// With FIO_CONTRACT_MFMA, chunks of at least this many right-hand sides take
// the p-levels and the adjoint x-levels on the matrix cores.
constexpr int LVL_MM_MIN_RHS = 32;

int check_plan(fio_plan_t plan) {
    if (!plan) return fail(FIO_EINVAL, "plan is NULL");
    return FIO_OK;
}

// Whether the byte ranges [a, a + na) and [b, b + nb) share a byte.
bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

// Arguments of fio_apply / fio_apply_adjoint: non-NULL, nrhs >= 1, the
// caller's dtype equal to the plan's, and input and output ranges (nrhs
// planes of N^2 complex values each) disjoint.
int check_apply_args(fio_plan_t plan, const void *in, void *out, int nrhs, int dtype, const char *names) {
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!in || !out) return fail(FIO_EINVAL, "%s must be non-NULL device pointers", names);
    if (nrhs < 1) return fail(FIO_EINVAL, "nrhs must be >= 1 (got %d)", nrhs);
    if (dtype != plan->dtype)
        return fail(FIO_EINVAL, "dtype %d does not match the plan's dtype %d (%s)", dtype, plan->dtype,
                    plan->dtype == FIO_C64 ? "FIO_C64" : "FIO_C128");
    const size_t bytes = (size_t)nrhs * plan->N * plan->N * (plan->dtype == FIO_C128 ? 16 : 8);
    if (overlaps(in, bytes, out, bytes)) return fail(FIO_EINVAL, "%s must not overlap", names);
    return FIO_OK;
}

int set_device(fio_plan_t plan) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != plan->device) {
        e = hipSetDevice(plan->device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    }
    return FIO_OK;
}

// Bracket one launch with events when profiling is on.
struct Timed {
    fio_plan_s *p;
    int kind;
    hipStream_t st;
    size_t slot = (size_t)-1;
    Timed(fio_plan_s *p_, int kind_, hipStream_t st_) : p(p_), kind(kind_), st(st_) {
        if (!p->prof) return;
        if (p->ev_used * 2 + 2 > p->ev.size()) {
            for (int i = 0; i < 64; ++i) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                p->ev.push_back(e);
            }
            p->ev_kind.resize(p->ev.size() / 2);
        }
        slot = p->ev_used++;
        p->ev_kind[slot] = kind;
        (void)hipEventRecord(p->ev[2 * slot], st);
    }
    ~Timed() {
        if (slot != (size_t)-1) (void)hipEventRecord(p->ev[2 * slot + 1], st);
    }
};

}  // namespace

namespace fio {

int set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int set_hip_error(hipError_t e, const char *what) { return hip_fail(e, what); }

void clear_error() { g_last_error.clear(); }

int plan_view(fio_plan_t plan, PlanView *v) {
    int rc = check_plan(plan);
    if (rc) return rc;
    v->N = plan->N;
    v->q = plan->q;
    v->dtype = plan->dtype;
    v->device = plan->device;
    v->ph = to_dev(&plan->phase);
    return FIO_OK;
}

}  // namespace fio

extern "C" {

const char *fio_last_error(void) { return g_last_error.c_str(); }

int fio_plan(int N, int q, const fio_phase_t *phase, fio_plan_t *out) {
    return fio_plan_ex(N, q, phase, nullptr, out);
}

int fio_plan_ex(int N, int q, const fio_phase_t *phase, const fio_plan_opts_t *opts, fio_plan_t *out) {
    g_last_error.clear();
    if (!out) return fail(FIO_EINVAL, "out is NULL");
    *out = nullptr;
    const int L = ilog2_exact(N);
    if (L < 0 || N < 8 || N > 8192) return fail(FIO_EINVAL, "N must be a power of two in [8, 8192] (got %d)", N);
    if (q < QMIN || q > QMAX) return fail(FIO_EINVAL, "q must be in [%d, %d] (got %d)", QMIN, QMAX, q);
    int rc = validate_phase(phase);
    if (rc) return rc;
    int s = std::min(3, L / 2), lm = L / 2, dtype = FIO_C64, nrhs_max = 1, contract = FIO_CONTRACT_FP;
    if (opts) {
        if (opts->contract != -1) contract = opts->contract;
        if (opts->s != -1) s = opts->s;
        if (opts->lm != -1) lm = opts->lm;
        if (opts->dtype != -1) dtype = opts->dtype;
        if (opts->nrhs_max != -1) {
            if (opts->nrhs_max < 1 || opts->nrhs_max > 4096)
                return fail(FIO_EINVAL, "nrhs_max must be in [1, 4096] (got %d)", opts->nrhs_max);
            nrhs_max = opts->nrhs_max;
        }
    }
    if (s < 0 || s > 3) return fail(FIO_EINVAL, "s must be in [0, 3] (got %d)", s);
    if (!(s <= lm && lm <= L - s)) return fail(FIO_EINVAL, "need s <= lm <= L - s (s=%d, lm=%d, L=%d)", s, lm, L);
    if (dtype != FIO_C64 && dtype != FIO_C128) return fail(FIO_EINVAL, "unknown dtype %d", dtype);
    if (contract != FIO_CONTRACT_FP && contract != FIO_CONTRACT_BF16 && contract != FIO_CONTRACT_MFMA)
        return fail(FIO_EINVAL, "unknown contraction precision %d", contract);
    if (contract == FIO_CONTRACT_MFMA && (dtype != FIO_C64 || !level_mfma_supported(q)))
        return fail(FIO_EINVAL, "FP32 matrix-core levels need dtype FIO_C64 and q <= 9 (dtype %d, q %d)", dtype, q);
    if (contract == FIO_CONTRACT_BF16 && (dtype != FIO_C64 || !mfma_supported_q(q)))
        return fail(FIO_EINVAL, "BF16 contractions need dtype FIO_C64 and q <= 12 (dtype %d, q %d)", dtype, q);

    fio_plan_s *p = new fio_plan_s();
    p->N = N;
    p->q = q;
    p->L = L;
    p->s = s;
    p->lm = lm;
    p->dtype = dtype;
    p->nrhs_max = nrhs_max;
    p->chunk = nrhs_max;
    p->contract = contract;
    p->phase = *phase;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDevice");
    }

    // ---- T_P: polar images of Omega (eq:polar), sorted by level-(L-s) box
    const int lB = L - s;
    const int nb1 = 1 << lB;
    const size_t n2 = (size_t)N * N;
    const size_t nboxes = (size_t)1 << (2 * lB);
    std::vector<double2> pp(n2);
    std::vector<uint32_t> boxof(n2);
    std::vector<int32_t> count(nboxes + 1, 0);
    const double two_pi = 2.0 * M_PI;
    for (int j1 = 0; j1 < N; ++j1) {
        for (int j2 = 0; j2 < N; ++j2) {
            const double k1 = j1 - N / 2, k2 = j2 - N / 2;
            double p1 = std::sqrt(2.0 * (k1 * k1 + k2 * k2)) / N;
            double p2 = std::atan2(k2, k1) / two_pi;
            if (p2 < 0.0) p2 += 1.0;
            const size_t idx = (size_t)j1 * N + j2;
            pp[idx] = make_double2(p1, p2);
            const int b1 = std::min((int)std::floor(p1 * nb1), nb1 - 1);
            const int b2 = std::min((int)std::floor(p2 * nb1), nb1 - 1);
            const uint32_t m = morton((uint32_t)b1, (uint32_t)b2);
            boxof[idx] = m;
            count[m + 1]++;
        }
    }
    for (size_t b = 0; b < nboxes; ++b) {
        p->max_box = std::max(p->max_box, count[b + 1]);
        count[b + 1] += count[b];
    }
    std::vector<int32_t> sidx(n2);
    std::vector<double2> sp(n2);
    {
        std::vector<int32_t> fillp(count.begin(), count.end() - 1);
        for (size_t idx = 0; idx < n2; ++idx) {  // stable: Omega order within a box
            const int32_t dst = fillp[boxof[idx]]++;
            sidx[dst] = (int32_t)idx;
            sp[dst] = pp[idx];
        }
    }

    // ---- tables (Sec. 3 Chebyshev grid; Sec. 4 Kronecker factors)
    std::vector<double> z(q), lam(q);
    for (int i = 0; i < q; ++i) z[i] = 0.5 * std::cos(i * M_PI / (q - 1));
    for (int i = 0; i < q / 2; ++i) z[q - 1 - i] = -z[i];  // exact symmetry z_{q-1-i} = -z_i
    if (q & 1) z[q / 2] = 0.0;
    for (int i = 0; i < q; ++i) {
        double d = 1.0;
        for (int j = 0; j < q; ++j)
            if (j != i) d *= (z[i] - z[j]);
        lam[i] = 1.0 / d;
    }
    const int m = 1 << s;
    std::vector<double> M(2 * q * q), Tt((size_t)m * q);
    for (int c = 0; c < 2; ++c)
        for (int t = 0; t < q; ++t)
            for (int j = 0; j < q; ++j) M[(c * q + t) * q + j] = lagrange(z, t, (z[j] + c - 0.5) / 2.0);
    for (int jj = 0; jj < m; ++jj)
        for (int t = 0; t < q; ++t) Tt[jj * q + t] = lagrange(z, t, (double)jj / m - 0.5);
    // symmetric and antisymmetric halves of M_0 (the kernels use M_1 = J M_0 J)
    std::vector<double> SA(4 * q * q, 0.0);
    const int hq = q / 2;
    for (int n = 0; n < q; ++n)
        for (int m = 0; m < q; ++m) {
            SA[(0 * q + n) * q + m] = 0.5 * (M[n * q + m] + M[(q - 1 - n) * q + m]);
            SA[(1 * q + n) * q + m] = 0.5 * (M[n * q + m] - M[(q - 1 - n) * q + m]);
            if (m < hq) {
                SA[(2 * q + n) * q + m] = 0.5 * (M[m * q + n] + M[(q - 1 - m) * q + n]);
                SA[(3 * q + n) * q + m] = 0.5 * (M[m * q + n] - M[(q - 1 - m) * q + n]);
            } else if (m == hq && (q & 1)) {
                SA[(2 * q + n) * q + m] = M[m * q + n];
            }
        }
    std::vector<float> Mf(M.begin(), M.end()), Ttf(Tt.begin(), Tt.end()), SAf(SA.begin(), SA.end());

    // table blob: z | lam | M | Tt | Mf | Ttf | SA | SAf  (256-byte aligned pieces)
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t oz = 0, olam = al(oz + q * 8), oM = al(olam + q * 8), oT = al(oM + M.size() * 8),
                 oMf = al(oT + Tt.size() * 8), oTf = al(oMf + Mf.size() * 4), oSA = al(oTf + Ttf.size() * 4),
                 oSAf = al(oSA + SA.size() * 8), tbytes = al(oSAf + SAf.size() * 4);
    std::vector<unsigned char> blob(tbytes, 0);
    memcpy(&blob[oz], z.data(), q * 8);
    memcpy(&blob[olam], lam.data(), q * 8);
    memcpy(&blob[oM], M.data(), M.size() * 8);
    memcpy(&blob[oT], Tt.data(), Tt.size() * 8);
    memcpy(&blob[oMf], Mf.data(), Mf.size() * 4);
    memcpy(&blob[oTf], Ttf.data(), Ttf.size() * 4);
    memcpy(&blob[oSA], SA.data(), SA.size() * 8);
    memcpy(&blob[oSAf], SAf.data(), SAf.size() * 4);

    // ---- device memory
    const size_t csize = dtype == FIO_C128 ? 16 : 8;
    p->plane = n2 * (size_t)q * q;
    p->wbytes = p->plane * csize;
    size_t tot = 0;
    const size_t wall = p->wbytes * (size_t)nrhs_max;
    if ((rc = dmalloc(&p->w0, wall, &tot, "weights 0")) || (rc = dmalloc(&p->w1, wall, &tot, "weights 1")) ||
        (rc = dmalloc(&p->dtab, tbytes, &tot, "tables")) ||
        (rc = dmalloc((void **)&p->d_idx, n2 * 4, &tot, "source index")) ||
        (rc = dmalloc((void **)&p->d_p, n2 * sizeof(double2), &tot, "source p")) ||
        (rc = dmalloc((void **)&p->d_off, (nboxes + 1) * 4, &tot, "box offsets"))) {
        free_plan(p);
        return rc;
    }
    p->total_bytes = tot;
    if ((e = hipMemcpy(p->dtab, blob.data(), tbytes, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_idx, sidx.data(), n2 * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_p, sp.data(), n2 * sizeof(double2), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_off, count.data(), (nboxes + 1) * 4, hipMemcpyHostToDevice)) != hipSuccess) {
        free_plan(p);
        return hip_fail(e, "plan upload");
    }
    unsigned char *base = (unsigned char *)p->dtab;
    p->tb.z = (const double *)(base + oz);
    p->tb.lam = (const double *)(base + olam);
    p->tb.M = (const double *)(base + oM);
    p->tb.Tt = (const double *)(base + oT);
    p->tb.Mf = (const float *)(base + oMf);
    p->tb.Ttf = (const float *)(base + oTf);
    p->tb.SA = (const double *)(base + oSA);
    p->tb.SAf = (const float *)(base + oSAf);
    p->geom.N = N;
    p->geom.L = L;
    p->geom.q = q;
    p->geom.s = s;
    p->geom.lm = lm;
    p->geom.rho_scale = std::sqrt(2.0) / 2.0 * N;
    p->geom.sw_ppw = 16;

    // tables of the initialisation on the matrix cores
    p->init_mm = dtype == FIO_C64 && init_mfma_supported(q, s);
    if (p->init_mm) {
        const size_t kbytes = n2 * (size_t)init_mfma_ktab_row(q) * 4, ebytes = n2 * 64 * 8;
        if ((rc = dmalloc(&p->ktab, kbytes, &p->total_bytes, "init K table")) ||
            (rc = dmalloc(&p->etab, ebytes, &p->total_bytes, "init kernel-value table"))) {
            free_plan(p);
            return rc;
        }
        Sources srcs{p->d_idx, p->d_p, p->d_off};
        if ((e = launch_init_tables(p->geom, p->tb, srcs, p->ktab, nullptr)) != hipSuccess ||
            (e = hipDeviceSynchronize()) != hipSuccess) {
            free_plan(p);
            return hip_fail(e, "init K table");
        }
    }
    *out = p;
    return FIO_OK;
}

int fio_set_phase(fio_plan_t plan, const fio_phase_t *phase) {
    int rc = check_plan(plan);
    if (rc) return rc;
    if ((rc = validate_phase(phase))) return rc;
    if (phase->kind != plan->phase.kind || phase->a1 != plan->phase.a1 || phase->a2 != plan->phase.a2 ||
        phase->eta1 != plan->phase.eta1 || phase->eta2 != plan->phase.eta2)
        plan->etab_ok = false;
    plan->phase = *phase;
    return FIO_OK;
}

int fio_plan_autotune(fio_plan_t plan, int nrhs, fio_tune_t *out) {
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (nrhs < 1) return fail(FIO_EINVAL, "nrhs must be >= 1 (got %d)", nrhs);
    if ((rc = set_device(plan))) return rc;
    fio_tune_t res{};
    res.chunk = plan->chunk;
    res.switch_items = plan->geom.sw_ppw;
    // candidates: chunks of >= 32 right-hand sides (the same kernels for every
    // chunk), items per workgroup of the matrix-core switches
    // A chunk shape c is a candidate when it gives every right-hand side of a
    // call of nrhs the kernels the plan's current shape gives it: chunks of
    // >= 32 take the same kernels, so both shapes must leave no remainder
    // below 32, or the same one.
    auto same_kernels = [&](int c) {
        const int tc = nrhs % c, td = nrhs % plan->chunk;
        return tc == td || ((tc == 0 || tc >= 32) && (td == 0 || td >= 32));
    };
    std::vector<int> chunks;
    const int cmax = std::min(plan->nrhs_max, nrhs);
    if (plan->dtype == FIO_C64 && plan->q <= 9 && plan->chunk >= 32) {
        for (int c = 32; c <= cmax; c *= 2)
            if (same_kernels(c)) chunks.push_back(c);
        if (cmax >= 32 && (chunks.empty() || chunks.back() != cmax) && same_kernels(cmax)) chunks.push_back(cmax);
    }
    if (chunks.empty()) {
        if (out) *out = res;
        return FIO_OK;
    }
    const size_t bytes = (size_t)nrhs * plan->N * plan->N * 8;
    void *f = nullptr, *u = nullptr;
    hipError_t e = hipMalloc(&f, bytes);
    if (e == hipSuccess) e = hipMalloc(&u, bytes);
    if (e == hipSuccess) e = hipMemset(f, 0, bytes);
    if (e == hipSuccess) e = hipMemset(u, 0, bytes);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    const int keep_chunk = plan->chunk, keep_ppw = plan->geom.sw_ppw;
    double best = 1e300, dflt = 0.0;
    int best_chunk = keep_chunk, best_ppw = keep_ppw, ncand = 0;
    auto timed = [&](double *ms) -> int {
        int r2 = FIO_OK;
        for (int rep = 0; rep < 3 && !r2; ++rep) {  // one warm-up, then the faster of two
            hipError_t e2 = hipEventRecord(t0, nullptr);
            if (e2 != hipSuccess) return hip_fail(e2, "autotune event");
            if ((r2 = fio_apply(plan, f, u, nrhs, FIO_C64, nullptr))) break;
            if ((r2 = fio_apply_adjoint(plan, u, f, nrhs, FIO_C64, nullptr))) break;
            if ((e2 = hipEventRecord(t1, nullptr)) != hipSuccess || (e2 = hipEventSynchronize(t1)) != hipSuccess)
                return hip_fail(e2, "autotune event");
            float m = 0.f;
            if ((e2 = hipEventElapsedTime(&m, t0, t1)) != hipSuccess) return hip_fail(e2, "autotune event");
            if (rep > 0 && m < *ms) *ms = m;
        }
        return r2;
    };
    if (e != hipSuccess) {
        rc = hip_fail(e, "autotune buffers");
    } else {
        for (int c : chunks) {
            for (int ppw : {8, 16, 32}) {
                plan->chunk = c;
                plan->geom.sw_ppw = ppw;
                double ms = 1e300;
                if ((rc = timed(&ms))) break;
                ++ncand;
                if (c == keep_chunk && ppw == keep_ppw) dflt = ms;
                if (ms < best) {
                    best = ms;
                    best_chunk = c;
                    best_ppw = ppw;
                }
            }
            if (rc) break;
        }
    }
    plan->chunk = rc ? keep_chunk : best_chunk;
    plan->geom.sw_ppw = rc ? keep_ppw : best_ppw;
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipFree(f);
    (void)hipFree(u);
    if (rc) return rc;
    res.chunk = plan->chunk;
    res.switch_items = plan->geom.sw_ppw;
    res.candidates = ncand;
    res.best_ms = best;
    res.default_ms = dflt;
    if (out) *out = res;
    return FIO_OK;
}

int fio_plan_set_shape(fio_plan_t plan, int chunk, int switch_items) {
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (chunk < 1 || chunk > plan->nrhs_max)
        return fail(FIO_EINVAL, "chunk must be in [1, %d] (got %d)", plan->nrhs_max, chunk);
    if (!switch_ppw_supported(switch_items))
        return fail(FIO_EINVAL, "switch_items must be 8, 16 or 32 (got %d)", switch_items);
    plan->chunk = chunk;
    plan->geom.sw_ppw = switch_items;
    return FIO_OK;
}

int fio_plan_get_info(fio_plan_t plan, fio_plan_info_t *info) {
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!info) return fail(FIO_EINVAL, "info is NULL");
    info->N = plan->N;
    info->q = plan->q;
    info->L = plan->L;
    info->s = plan->s;
    info->lm = plan->lm;
    info->dtype = plan->dtype;
    info->contract = plan->contract;
    info->n_pairs = (int64_t)plan->N * plan->N;
    info->weights_per_level = (int64_t)plan->N * plan->N * plan->q * plan->q;
    info->workspace_bytes = (int64_t)plan->total_bytes;
    info->nrhs_max = plan->nrhs_max;
    info->max_box_sources = plan->max_box;
    info->chunk = plan->chunk;
    info->switch_items = plan->geom.sw_ppw;
    return FIO_OK;
}

// Whether a chunk of nr right-hand sides takes the matrix-core levels.
static bool level_mm(fio_plan_t p, int nr) { return p->contract == FIO_CONTRACT_MFMA && nr >= LVL_MM_MIN_RHS; }

// The kernel-value table of the matrix-core initialisation, remade after a
// phase change (on the stream of the call that needs it).
static hipError_t ensure_etab(fio_plan_t p, const PhaseDev &ph, const Sources &src, hipStream_t st) {
    if (p->etab_ok) return hipSuccess;
    Timed tm(p, FIO_K_TABLES, st);
    hipError_t e = launch_init_etab(p->geom, ph, src, p->etab, st);
    if (e == hipSuccess) p->etab_ok = true;
    return e;
}

// Forward pipeline for `nr` <= nrhs_max right-hand sides (f, u: nr planes of
// N^2); stops after `last_stage` (-1: run to the potentials) and returns the
// buffer holding that stage's weights through *wlast.
static int run_forward(fio_plan_t p, const void *f, void *u, int nr, int last_stage, void **wlast,
                       hipStream_t st) {
    const PhaseDev ph = to_dev(&p->phase);
    Sources src{p->d_idx, p->d_p, p->d_off};
    const size_t csize = p->dtype == FIO_C128 ? 16 : 8;
    const size_t fstep = (size_t)p->N * p->N * csize;
    char *a = (char *)p->w0, *b = (char *)p->w1;
    int stage = 0;
    hipError_t e = hipSuccess;
    if (p->init_mm) {
        e = ensure_etab(p, ph, src, st);
        if (e == hipSuccess) {
            Timed tm(p, FIO_K_INIT, st);
            e = launch_init_mfma(p->geom, ph, p->tb, src, p->ktab, p->etab, f, b, a, nr, p->plane, st);
        }
    } else {
        for (int r = 0; r < nr && e == hipSuccess; ++r) {
            Timed tm(p, FIO_K_INIT, st);
            e = launch_init(p->dtype, p->geom, ph, p->tb, src, (const char *)f + r * fstep, a + r * p->wbytes,
                            st);
        }
    }
    if (e != hipSuccess) return hip_fail(e, "init launch");
    if (last_stage == stage) {
        *wlast = a;
        return FIO_OK;
    }
    for (int l = p->s + 1; l <= p->lm; ++l) {
        ++stage;
        {
            Timed tm(p, FIO_K_PLEVEL, st);
            e = p->contract == FIO_CONTRACT_BF16
                    ? launch_plevel_mfma(p->geom, ph, p->tb, l, a, b, nr, p->plane, st)
                : level_mm(p, nr) ? launch_level_mm(false, p->geom, ph, p->tb, l, a, b, nr, p->plane, st)
                                  : launch_plevel(p->dtype, p->geom, ph, p->tb, l, a, b, nr, p->plane, st);
        }
        if (e != hipSuccess) return hip_fail(e, "p-level launch");
        std::swap(a, b);
        if (last_stage == stage) {
            *wlast = a;
            return FIO_OK;
        }
    }
    ++stage;
    {
        Timed tm(p, FIO_K_SWITCH, st);
        e = launch_switch(p->dtype, p->geom, ph, p->tb, a, nr, p->plane, st);
    }
    if (e != hipSuccess) return hip_fail(e, "switch launch");
    if (last_stage == stage) {
        *wlast = a;
        return FIO_OK;
    }
    for (int l = p->lm + 1; l <= p->L - p->s; ++l) {
        ++stage;
        {
            Timed tm(p, FIO_K_XLEVEL, st);
            e = launch_xlevel(p->dtype, p->geom, ph, p->tb, l, a, b, nr, p->plane, st);
        }
        if (e != hipSuccess) return hip_fail(e, "x-level launch");
        std::swap(a, b);
        if (last_stage == stage) {
            *wlast = a;
            return FIO_OK;
        }
    }
    if (last_stage >= 0) return fail(FIO_EINVAL, "stage %d out of range (last is %d)", last_stage, stage);
    if (nr > 1) {
        Timed tm(p, FIO_K_TERM, st);
        e = launch_term_batch(p->dtype, p->geom, ph, p->tb, a, u, nr, p->plane, (size_t)p->N * p->N, st);
    } else {
        Timed tm(p, FIO_K_TERM, st);
        e = launch_term(p->dtype, p->geom, ph, p->tb, a, u, st);
    }
    if (e != hipSuccess) return hip_fail(e, "termination launch");
    return FIO_OK;
}

static int run_adjoint(fio_plan_t p, const void *u, void *f, int nr, hipStream_t st) {
    const PhaseDev ph = to_dev(&p->phase);
    Sources src{p->d_idx, p->d_p, p->d_off};
    const size_t csize = p->dtype == FIO_C128 ? 16 : 8;
    const size_t fstep = (size_t)p->N * p->N * csize;
    char *a = (char *)p->w0, *b = (char *)p->w1;
    hipError_t e = hipSuccess;
    if (nr > 1) {
        Timed tm(p, FIO_K_TERM_ADJ, st);
        e = launch_term_adj_batch(p->dtype, p->geom, ph, p->tb, u, a, nr, p->plane, (size_t)p->N * p->N, st);
    } else {
        Timed tm(p, FIO_K_TERM_ADJ, st);
        e = launch_term_adj(p->dtype, p->geom, ph, p->tb, u, a, st);
    }
    if (e != hipSuccess) return hip_fail(e, "termination^H launch");
    for (int l = p->L - p->s; l >= p->lm + 1; --l) {
        {
            Timed tm(p, FIO_K_XLEVEL_ADJ, st);
            e = level_mm(p, nr) ? launch_level_mm(true, p->geom, ph, p->tb, l, a, b, nr, p->plane, st)
                                : launch_xlevel_adj(p->dtype, p->geom, ph, p->tb, l, a, b, nr, p->plane, st);
        }
        if (e != hipSuccess) return hip_fail(e, "x-level^H launch");
        std::swap(a, b);
    }
    {
        Timed tm(p, FIO_K_SWITCH_ADJ, st);
        e = launch_switch_adj(p->dtype, p->geom, ph, p->tb, a, nr, p->plane, st);
    }
    if (e != hipSuccess) return hip_fail(e, "switch^H launch");
    for (int l = p->lm; l >= p->s + 1; --l) {
        {
            Timed tm(p, FIO_K_PLEVEL_ADJ, st);
            e = launch_plevel_adj(p->dtype, p->geom, ph, p->tb, l, a, b, nr, p->plane, st);
        }
        if (e != hipSuccess) return hip_fail(e, "p-level^H launch");
        std::swap(a, b);
    }
    if (p->init_mm) {
        e = ensure_etab(p, ph, src, st);
        if (e == hipSuccess) {
            Timed tm(p, FIO_K_INIT_ADJ, st);
            e = launch_init_adj_mfma(p->geom, ph, p->tb, src, p->ktab, p->etab, a, f, nr, p->plane, st);
        }
    } else {
        for (int r = 0; r < nr && e == hipSuccess; ++r) {
            Timed tm(p, FIO_K_INIT_ADJ, st);
            e = launch_init_adj(p->dtype, p->geom, ph, p->tb, src, a + r * p->wbytes, (char *)f + r * fstep,
                                st);
        }
    }
    if (e != hipSuccess) return hip_fail(e, "initialisation^H launch");
    return FIO_OK;
}

// Primal and the two phase tangents of nr right-hand sides through the
// whole pass (kernels of fio_kernels_tan.hip).  Right-hand side r keeps its
// three weight planes at 3r, 3r + 1 and 3r + 2 of the plan's buffers; the
// level and switch kernels take all nr in one launch and make their kernel
// values once, the initialisation and termination go one right-hand side a
// launch.
static int run_tangent(fio_plan_t p, const char *f, char *u, char *d1, char *d2, int nr, size_t fstep,
                       hipStream_t st) {
    const PhaseDev ph = to_dev(&p->phase);
    Sources src{p->d_idx, p->d_p, p->d_off};
    char *a = (char *)(p->nrhs_max >= 3 ? p->w0 : p->t0), *b = (char *)(p->nrhs_max >= 3 ? p->w1 : p->t1);
    const size_t rb = 3 * p->wbytes;
    Timed tm(p, FIO_K_TANGENT, st);
    hipError_t e = hipSuccess;
    for (int r = 0; r < nr && e == hipSuccess; ++r)
        e = launch_tangent_step(p->dtype, 0, p->geom, ph, p->tb, src, 0, f + r * fstep, a + r * rb, p->plane,
                                nullptr, nullptr, 1, st);
    for (int l = p->s + 1; l <= p->lm && e == hipSuccess; ++l) {
        e = launch_tangent_step(p->dtype, 1, p->geom, ph, p->tb, src, l, a, b, p->plane, nullptr, nullptr, nr,
                                st);
        std::swap(a, b);
    }
    if (e == hipSuccess)
        e = launch_tangent_step(p->dtype, 2, p->geom, ph, p->tb, src, p->lm, a, a, p->plane, nullptr, nullptr, nr,
                                st);
    for (int l = p->lm + 1; l <= p->L - p->s && e == hipSuccess; ++l) {
        e = launch_tangent_step(p->dtype, 3, p->geom, ph, p->tb, src, l, a, b, p->plane, nullptr, nullptr, nr,
                                st);
        std::swap(a, b);
    }
    for (int r = 0; r < nr && e == hipSuccess; ++r)
        e = launch_tangent_step(p->dtype, 4, p->geom, ph, p->tb, src, 0, a + r * rb, u ? u + r * fstep : nullptr,
                                p->plane, d1 + r * fstep, d2 + r * fstep, 1, st);
    if (e != hipSuccess) return hip_fail(e, "tangent launch");
    return FIO_OK;
}

int fio_apply_dphase(fio_plan_t plan, const void *f, void *u, void *du_da1, void *du_da2, int nrhs,
                     void *stream) {
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!f || !du_da1 || !du_da2) return fail(FIO_EINVAL, "f, du_da1 and du_da2 must be non-NULL device pointers");
    if (nrhs < 1) return fail(FIO_EINVAL, "nrhs must be >= 1 (got %d)", nrhs);
    if (!tangent_supported_q(plan->q)) return fail(FIO_EINVAL, "phase derivatives need q <= 12 (got %d)", plan->q);
    {
        const size_t nb = (size_t)nrhs * plan->N * plan->N * (plan->dtype == FIO_C128 ? 16 : 8);
        const void *arr[4] = {f, du_da1, du_da2, u};
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j)
                if (arr[i] && arr[j] && overlaps(arr[i], nb, arr[j], nb))
                    return fail(FIO_EINVAL, "f, u, du_da1 and du_da2 must not overlap");
    }
    if ((rc = set_device(plan))) return rc;
    if (plan->nrhs_max < 3 && !plan->t0) {
        size_t tot = plan->total_bytes;
        if ((rc = dmalloc(&plan->t0, 3 * plan->wbytes, &tot, "tangent weights 0")) ||
            (rc = dmalloc(&plan->t1, 3 * plan->wbytes, &tot, "tangent weights 1"))) {
            (void)hipFree(plan->t0);
            plan->t0 = nullptr;
            return rc;
        }
        plan->total_bytes = tot;
    }
    const size_t step = (size_t)plan->N * plan->N * (plan->dtype == FIO_C128 ? 16 : 8);
    // chunks of at most nrhs_max / 3 right-hand sides, as even as they come
    const int cmax = plan->nrhs_max >= 3 ? plan->nrhs_max / 3 : 1;
    const int nchunks = (nrhs + cmax - 1) / cmax;
    const int chunk = (nrhs + nchunks - 1) / nchunks;
    hipStream_t st = (hipStream_t)stream;
    for (int r = 0; r < nrhs; r += chunk) {
        const int nr = std::min(chunk, nrhs - r);
        rc = run_tangent(plan, (const char *)f + r * step, u ? (char *)u + r * step : nullptr,
                         (char *)du_da1 + r * step, (char *)du_da2 + r * step, nr, step, st);
        if (rc) return rc;
    }
    return FIO_OK;
}

// Workspace of the separated-amplitude applies: two buffers of `rank`
// planes of N^2 complex values, grown on demand.
static int ensure_amp(fio_plan_t p, int rank) {
    if (rank <= p->amp_cap) return FIO_OK;
    const size_t bytes = (size_t)rank * p->N * p->N * (p->dtype == FIO_C128 ? 16 : 8);
    if (p->amp0) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        (void)hipFree(p->amp0);
        (void)hipFree(p->amp1);
        p->total_bytes -= 2 * (size_t)p->amp_cap * p->N * p->N * (p->dtype == FIO_C128 ? 16 : 8);
        p->amp0 = p->amp1 = nullptr;
        p->amp_cap = 0;
    }
    int rc;
    if ((rc = dmalloc(&p->amp0, bytes, &p->total_bytes, "amplitude workspace 0")) ||
        (rc = dmalloc(&p->amp1, bytes, &p->total_bytes, "amplitude workspace 1"))) {
        (void)hipFree(p->amp0);
        p->amp0 = nullptr;
        return rc;
    }
    p->amp_cap = rank;
    return FIO_OK;
}

static int amp_args(fio_plan_t plan, const void *in, const void *g, const void *h, int rank, void *out) {
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!in || !g || !h || !out) return fail(FIO_EINVAL, "all array arguments must be non-NULL device pointers");
    if (rank < 1 || rank > 4096) return fail(FIO_EINVAL, "rank must be in [1, 4096] (got %d)", rank);
    {
        const size_t plane = (size_t)plan->N * plan->N * (plan->dtype == FIO_C128 ? 16 : 8);
        if (overlaps(in, plane, out, plane) || overlaps(g, rank * plane, out, plane) ||
            overlaps(h, rank * plane, out, plane))
            return fail(FIO_EINVAL, "the output must not overlap the inputs");
    }
    return set_device(plan);
}

// The separated-amplitude pass with its two staging buffers given: buf0
// receives the rank scaled inputs, buf1 the rank butterfly outputs (rank
// planes of N^2 complex values each).
static int amp_run(fio_plan_t plan, bool adjoint, const void *in, const void *g, const void *h, int rank, void *out,
                   void *buf0, void *buf1, hipStream_t st) {
    const size_t n2 = (size_t)plan->N * plan->N, step = n2 * (plan->dtype == FIO_C128 ? 16 : 8);
    // forward: buf0 = h_t . f, buf1 = B buf0, u = sum_t g_t . buf1;
    // adjoint: buf0 = conj(g_t) . u, buf1 = B^H buf0, f = sum_t conj(h_t) . buf1
    hipError_t e = launch_scale_planes(plan->dtype, adjoint, adjoint ? g : h, in, buf0, n2, rank, st);
    if (e != hipSuccess) return hip_fail(e, "amplitude scale launch");
    for (int r = 0; r < rank; r += plan->nrhs_max) {
        const int nr = std::min(plan->nrhs_max, rank - r);
        const int rc = adjoint ? run_adjoint(plan, (const char *)buf0 + r * step, (char *)buf1 + r * step, nr, st)
                               : run_forward(plan, (const char *)buf0 + r * step, (char *)buf1 + r * step, nr, -1,
                                             nullptr, st);
        if (rc) return rc;
    }
    e = launch_combine_planes(plan->dtype, adjoint, adjoint ? h : g, buf1, out, n2, rank, st);
    if (e != hipSuccess) return hip_fail(e, "amplitude combine launch");
    return FIO_OK;
}

}  // extern "C"

namespace fio {

int amplitude_apply_in(fio_plan_t plan, const void *f, const void *g, const void *h, int rank, void *u,
                       size_t scratch_bytes, void *(*scratch_of_device)(int device), void *stream) {
    g_last_error.clear();
    int rc = amp_args(plan, f, g, h, rank, u);
    if (rc) return rc;
    const size_t need = 2 * (size_t)rank * plan->N * plan->N * (plan->dtype == FIO_C128 ? 16 : 8);
    if (need > scratch_bytes)
        return fail(FIO_EINVAL,
                    "rank %d at N = %d needs %zu bytes of staging, more than the %zu bytes of the static scratch "
                    "array (at most 2 rank N^2 complex values)",
                    rank, plan->N, need, scratch_bytes);
    char *base = (char *)scratch_of_device(plan->device);
    if (!base) return FIO_EDEVICE;  // the message is set by scratch_of_device
    return amp_run(plan, false, f, g, h, rank, u, base, base + need / 2, (hipStream_t)stream);
}

}  // namespace fio

extern "C" {

int fio_apply_amplitude(fio_plan_t plan, const void *f, const void *g, const void *h, int rank, void *u,
                        void *stream) {
    g_last_error.clear();
    int rc = amp_args(plan, f, g, h, rank, u);
    if (rc || (rc = ensure_amp(plan, rank))) return rc;
    return amp_run(plan, false, f, g, h, rank, u, plan->amp0, plan->amp1, (hipStream_t)stream);
}

int fio_apply_amplitude_adjoint(fio_plan_t plan, const void *u, const void *g, const void *h, int rank, void *f,
                                void *stream) {
    g_last_error.clear();
    int rc = amp_args(plan, u, g, h, rank, f);
    if (rc || (rc = ensure_amp(plan, rank))) return rc;
    return amp_run(plan, true, u, g, h, rank, f, plan->amp0, plan->amp1, (hipStream_t)stream);
}

int fio_apply(fio_plan_t plan, const void *f, void *u, int nrhs, int dtype, void *stream) {
    g_last_error.clear();
    int rc = check_apply_args(plan, f, u, nrhs, dtype, "f and u");
    if (rc) return rc;
    if ((rc = set_device(plan))) return rc;
    const size_t step = (size_t)plan->N * plan->N * (plan->dtype == FIO_C128 ? 16 : 8);
    hipStream_t st = (hipStream_t)stream;
    for (int r = 0; r < nrhs; r += plan->chunk) {
        const int nr = std::min(plan->chunk, nrhs - r);
        rc = run_forward(plan, (const char *)f + r * step, (char *)u + r * step, nr, -1, nullptr, st);
        if (rc) return rc;
    }
    return FIO_OK;
}

int fio_apply_adjoint(fio_plan_t plan, const void *u, void *f, int nrhs, int dtype, void *stream) {
    g_last_error.clear();
    int rc = check_apply_args(plan, u, f, nrhs, dtype, "u and f");
    if (rc) return rc;
    if ((rc = set_device(plan))) return rc;
    const size_t step = (size_t)plan->N * plan->N * (plan->dtype == FIO_C128 ? 16 : 8);
    hipStream_t st = (hipStream_t)stream;
    for (int r = 0; r < nrhs; r += plan->chunk) {
        const int nr = std::min(plan->chunk, nrhs - r);
        rc = run_adjoint(plan, (const char *)u + r * step, (char *)f + r * step, nr, st);
        if (rc) return rc;
    }
    return FIO_OK;
}

int fio_debug_stage(fio_plan_t plan, const void *f, int stage, void *weights, void *stream) {
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!f || !weights) return fail(FIO_EINVAL, "f and weights must be non-NULL device pointers");
    const int nstages = plan->L - 2 * plan->s + 2;
    if (stage < 0 || stage >= nstages) return fail(FIO_EINVAL, "stage must be in [0, %d) (got %d)", nstages, stage);
    if ((rc = set_device(plan))) return rc;
    hipStream_t st = (hipStream_t)stream;
    void *wl = nullptr;
    if ((rc = run_forward(plan, f, nullptr, 1, stage, &wl, st))) return rc;
    hipError_t e = hipMemcpyAsync(weights, wl, plan->wbytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "weights copy");
    return FIO_OK;
}

int fio_profile_enable(fio_plan_t plan, int enable) {
    int rc = check_plan(plan);
    if (rc) return rc;
    plan->prof = enable != 0;
    return FIO_OK;
}

int fio_profile_read(fio_plan_t plan, double *ms, int64_t *launches, int n) {
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!ms || !launches || n < 0) return fail(FIO_EINVAL, "ms and launches must be non-NULL");
    for (int k = 0; k < n; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (size_t i = 0; i < plan->ev_used; ++i) {
        hipError_t e = hipEventSynchronize(plan->ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float t = 0.0f;
        e = hipEventElapsedTime(&t, plan->ev[2 * i], plan->ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        const int k = plan->ev_kind[i];
        if (k < n) {
            ms[k] += t;
            launches[k] += 1;
        }
    }
    plan->ev_used = 0;
    return FIO_OK;
}

int fio_destroy(fio_plan_t plan) {
    if (!plan) return FIO_OK;
    const int dev = plan->device;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != dev) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    free_plan(plan);
    if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    return FIO_OK;
}

}  // extern "C"
