// Host side of the batch of plans (uneven problem sizes side by side on
// internal streams, capturable as one graph), the direct evaluation of
// eq:dfio at sampled targets, and the choice of q by the estimated error
// eq:err (Sec. 5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include "fio_internal.h"

using namespace fio;

struct fio_batch_s {
    std::vector<fio_plan_t> plans;
    std::vector<int> dtypes;     // each plan's dtype
    std::vector<int> order;      // plans by decreasing work
    std::vector<int> stream_of;  // internal stream of each plan
    std::vector<hipStream_t> streams;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    int device = 0;
};

namespace {

void free_batch(fio_batch_s *b) {
    if (!b) return;
    for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
    delete b;
}

int use_device(int dev) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return set_hip_error(e, "hipGetDevice");
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return set_hip_error(e, "hipSetDevice");
    return FIO_OK;
}

uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Fork from `st` onto the batch's streams, run `fn(plan index, stream)` for
// every plan, and join back; the joins are recorded even after a failure so
// that `st` still orders everything that was launched.
template <typename F>
int run_batch(fio_batch_s *b, hipStream_t st, F fn) {
    hipError_t e = hipEventRecord(b->fork, st);
    if (e != hipSuccess) return set_hip_error(e, "hipEventRecord");
    for (hipStream_t s : b->streams)
        if ((e = hipStreamWaitEvent(s, b->fork, 0)) != hipSuccess) return set_hip_error(e, "hipStreamWaitEvent");
    int rc = FIO_OK;
    for (int i : b->order) {
        rc = fn(i, b->streams[b->stream_of[i]]);
        if (rc) break;
    }
    for (size_t j = 0; j < b->streams.size(); ++j) {
        hipError_t e1 = hipEventRecord(b->join[j], b->streams[j]);
        hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(st, b->join[j], 0) : e1;
        if (e2 != hipSuccess && !rc) rc = set_hip_error(e2, "batch join");
    }
    return rc;
}

}  // namespace

extern "C" {

int fio_batch_create(const fio_plan_t *plans, int n, int nstreams, fio_batch_t *out) {
    clear_error();
    if (!out) return set_error(FIO_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plans || n < 1 || n > 4096) return set_error(FIO_EINVAL, "need 1 <= n <= 4096 plans (got %d)", n);
    if (nstreams < 1 || nstreams > 16) return set_error(FIO_EINVAL, "nstreams must be in [1, 16] (got %d)", nstreams);
    std::vector<double> cost(n);
    std::vector<int> dtypes(n);
    int dev = -1;
    for (int i = 0; i < n; ++i) {
        PlanView v;
        if (plan_view(plans[i], &v)) return set_error(FIO_EINVAL, "plan %d is NULL", i);
        if (dev < 0) dev = v.device;
        if (v.device != dev) return set_error(FIO_EINVAL, "plans %d and 0 are on different devices", i);
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return set_error(FIO_EINVAL, "plan %d appears twice (plans %d and %d)", i, j, i);
        cost[i] = (double)v.N * v.N * v.q * v.q * v.q;  // work per level ~ N^2 q^3
        dtypes[i] = v.dtype;
    }
    int rc = use_device(dev);
    if (rc) return rc;
    fio_batch_s *b = new fio_batch_s;
    b->device = dev;
    b->plans.assign(plans, plans + n);
    b->dtypes = dtypes;
    const int ns = std::min(nstreams, n);
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int j = 0; e == hipSuccess && j < ns; ++j) {
        hipStream_t s = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) b->streams.push_back(s);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) b->join.push_back(ev);
    }
    if (e != hipSuccess) {
        free_batch(b);
        return set_hip_error(e, "batch streams and events");
    }
    // largest work first, each to the stream with the least work so far
    b->order.resize(n);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    b->stream_of.assign(n, 0);
    std::vector<double> load(ns, 0.0);
    for (int i : b->order) {
        const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        b->stream_of[i] = j;
        load[j] += cost[i];
    }
    *out = b;
    return FIO_OK;
}

int fio_batch_apply(fio_batch_t batch, const void *const *f, void *const *u, void *stream) {
    clear_error();
    if (!batch) return set_error(FIO_EINVAL, "batch is NULL");
    if (!f || !u) return set_error(FIO_EINVAL, "f and u must be non-NULL host arrays of device pointers");
    for (size_t i = 0; i < batch->plans.size(); ++i)
        if (!f[i] || !u[i] || f[i] == u[i])
            return set_error(FIO_EINVAL, "f[%zu], u[%zu] must be distinct non-NULL device pointers", i, i);
    int rc = use_device(batch->device);
    if (rc) return rc;
    return run_batch(batch, (hipStream_t)stream,
                     [&](int i, hipStream_t s) { return fio_apply(batch->plans[i], f[i], u[i], 1, batch->dtypes[i], s); });
}

int fio_batch_apply_adjoint(fio_batch_t batch, const void *const *u, void *const *f, void *stream) {
    clear_error();
    if (!batch) return set_error(FIO_EINVAL, "batch is NULL");
    if (!f || !u) return set_error(FIO_EINVAL, "u and f must be non-NULL host arrays of device pointers");
    for (size_t i = 0; i < batch->plans.size(); ++i)
        if (!f[i] || !u[i] || f[i] == u[i])
            return set_error(FIO_EINVAL, "u[%zu], f[%zu] must be distinct non-NULL device pointers", i, i);
    int rc = use_device(batch->device);
    if (rc) return rc;
    return run_batch(batch, (hipStream_t)stream,
                     [&](int i, hipStream_t s) {
                         return fio_apply_adjoint(batch->plans[i], u[i], f[i], 1, batch->dtypes[i], s);
                     });
}

int fio_batch_destroy(fio_batch_t batch) {
    clear_error();
    if (!batch) return set_error(FIO_EINVAL, "batch is NULL");
    (void)use_device(batch->device);
    free_batch(batch);
    return FIO_OK;
}

int fio_direct_rows(fio_plan_t plan, const void *f, const int64_t *rows, int nrows, void *out, void *stream) {
    clear_error();
    PlanView v;
    int rc = plan_view(plan, &v);
    if (rc) return rc;
    if (!f || !rows || !out) return set_error(FIO_EINVAL, "f, rows and out must be non-NULL device pointers");
    if (nrows < 1 || nrows > (1 << 20)) return set_error(FIO_EINVAL, "nrows must be in [1, 2^20] (got %d)", nrows);
    if ((rc = use_device(v.device))) return rc;
    hipError_t e = launch_direct_rows(v.dtype, v.N, v.ph, f, rows, nrows, out, (hipStream_t)stream);
    return e == hipSuccess ? FIO_OK : set_hip_error(e, "direct rows launch");
}

int fio_select_q(int N, const fio_phase_t *phase, const fio_plan_opts_t *opts, double tol, int qmin, int qmax,
                 int nrows, uint64_t seed, int *q_out, double *err_out, double *errs) {
    clear_error();
    if (!q_out || !err_out) return set_error(FIO_EINVAL, "q_out and err_out must be non-NULL");
    if (qmin < QMIN || qmax > QMAX || qmin > qmax)
        return set_error(FIO_EINVAL, "need %d <= qmin <= qmax <= %d (got %d, %d)", QMIN, QMAX, qmin, qmax);
    if (!(tol > 0.0)) return set_error(FIO_EINVAL, "tol must be > 0");
    if (nrows < 1 || nrows > 4096) return set_error(FIO_EINVAL, "nrows must be in [1, 4096] (got %d)", nrows);
    if (errs)
        for (int q = qmin; q <= qmax; ++q) errs[q - qmin] = NAN;
    // the first plan validates N, the phase and the options
    fio_plan_t plan = nullptr;
    int rc = fio_plan_ex(N, qmin, phase, opts, &plan);
    if (rc) return rc;
    PlanView v;
    plan_view(plan, &v);
    const size_t n2 = (size_t)N * N, esz = v.dtype == FIO_C128 ? 16 : 8;
    std::vector<int64_t> rows(nrows);
    for (int i = 0; i < nrows; ++i) rows[i] = (int64_t)(splitmix64(seed ^ 0x5851F42D4C957F2Dull, (uint64_t)i) % n2);
    void *f = nullptr, *u = nullptr, *ud = nullptr, *dr = nullptr;
    hipError_t e = hipMalloc(&f, n2 * esz);
    if (e == hipSuccess) e = hipMalloc(&u, n2 * esz);
    if (e == hipSuccess) e = hipMalloc(&ud, nrows * esz);
    if (e == hipSuccess) e = hipMalloc(&dr, nrows * sizeof(int64_t));
    if (e == hipSuccess) e = hipMemcpy(dr, rows.data(), nrows * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_probe(v.dtype, N, seed, f, nullptr);
    if (e == hipSuccess) e = launch_direct_rows(v.dtype, N, v.ph, f, (const int64_t *)dr, nrows, ud, nullptr);
    std::vector<double> ref(2 * nrows), got(2 * nrows);
    auto to_host = [&](const void *d, std::vector<double> &h) -> hipError_t {
        if (v.dtype == FIO_C128) return hipMemcpy(h.data(), d, nrows * 16, hipMemcpyDeviceToHost);
        std::vector<float> tmp(2 * nrows);
        hipError_t r = hipMemcpy(tmp.data(), d, nrows * 8, hipMemcpyDeviceToHost);
        for (int i = 0; i < 2 * nrows; ++i) h[i] = tmp[i];
        return r;
    };
    if (e == hipSuccess) e = to_host(ud, ref);
    double err = INFINITY;
    int q = qmin;
    for (; e == hipSuccess && !rc; ++q) {
        if (q > qmin) {
            fio_destroy(plan);
            plan = nullptr;
            if ((rc = fio_plan_ex(N, q, phase, opts, &plan))) break;
        }
        if ((rc = fio_apply(plan, f, u, 1, v.dtype, nullptr))) break;
        // the butterfly at the sampled targets: gather on the host
        std::vector<double> full;
        {
            std::vector<char> hb(n2 * esz);
            if ((e = hipMemcpy(hb.data(), u, n2 * esz, hipMemcpyDeviceToHost)) != hipSuccess) break;
            for (int i = 0; i < nrows; ++i) {
                if (v.dtype == FIO_C128) {
                    const double *p = (const double *)hb.data() + 2 * rows[i];
                    got[2 * i] = p[0];
                    got[2 * i + 1] = p[1];
                } else {
                    const float *p = (const float *)hb.data() + 2 * rows[i];
                    got[2 * i] = p[0];
                    got[2 * i + 1] = p[1];
                }
            }
        }
        double num = 0.0, den = 0.0;
        for (int i = 0; i < 2 * nrows; ++i) {
            num += (got[i] - ref[i]) * (got[i] - ref[i]);
            den += ref[i] * ref[i];
        }
        err = den > 0.0 ? std::sqrt(num / den) : std::sqrt(num);
        if (errs) errs[q - qmin] = err;
        if (err <= tol) break;
        if (q == qmax) break;
    }
    const int qsel = std::min(q, qmax);
    if (plan) fio_destroy(plan);
    (void)hipFree(f);
    (void)hipFree(u);
    (void)hipFree(ud);
    (void)hipFree(dr);
    if (rc) return rc;
    if (e != hipSuccess) return set_hip_error(e, "q selection");
    *q_out = qsel;
    *err_out = err;
    return FIO_OK;
}

}  // extern "C"
