// Variable amplitude through a separated approximation a(x,k) = sum_t g_t(x)
// h_t(k) (end of Sec. 4): the butterfly is applied to the rank inputs
// h_t f together (they share every kernel value), and the outputs are
// multiplied by g_t and summed.  The two elementwise steps are here; both are
// plain streaming kernels (bandwidth-bound).
#include <hip/hip_runtime.h>

#include <mutex>

#include "fio_kernels_common.h"

namespace fio {

// out[t][i] = op(a[t][i]) * b[i], op = conj if CONJ; t < rank, i < n
template <typename T, bool CONJ>
__global__ __launch_bounds__(NT) void k_scale_planes(const cpx<T> *__restrict__ a, const cpx<T> *__restrict__ b,
                                                     cpx<T> *__restrict__ out, size_t n, int rank) {
    const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const cpx<T> bv = b[i];
    for (int t = 0; t < rank; ++t) {
        const cpx<T> av = a[(size_t)t * n + i];
        out[(size_t)t * n + i] = CONJ ? cmulc(bv, av) : cmul(av, bv);
    }
}

// out[i] = sum_t op(a[t][i]) * b[t][i]
template <typename T, bool CONJ>
__global__ __launch_bounds__(NT) void k_combine_planes(const cpx<T> *__restrict__ a, const cpx<T> *__restrict__ b,
                                                       cpx<T> *__restrict__ out, size_t n, int rank) {
    const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    cpx<T> acc = {(T)0, (T)0};
    for (int t = 0; t < rank; ++t) {
        const cpx<T> av = a[(size_t)t * n + i], bv = b[(size_t)t * n + i];
        cfma(acc, CONJ ? cpx<T>{av.re, -av.im} : av, bv);
    }
    out[i] = acc;
}

template <typename T>
static hipError_t amp_t(bool combine, bool conj, const void *a, const void *b, void *out, size_t n, int rank,
                        hipStream_t st) {
    const dim3 grid((unsigned)((n + NT - 1) / NT));
    if (!combine) {
        if (conj)
            hipLaunchKernelGGL((k_scale_planes<T, true>), grid, dim3(NT), 0, st, (const cpx<T> *)a,
                               (const cpx<T> *)b, (cpx<T> *)out, n, rank);
        else
            hipLaunchKernelGGL((k_scale_planes<T, false>), grid, dim3(NT), 0, st, (const cpx<T> *)a,
                               (const cpx<T> *)b, (cpx<T> *)out, n, rank);
    } else {
        if (conj)
            hipLaunchKernelGGL((k_combine_planes<T, true>), grid, dim3(NT), 0, st, (const cpx<T> *)a,
                               (const cpx<T> *)b, (cpx<T> *)out, n, rank);
        else
            hipLaunchKernelGGL((k_combine_planes<T, false>), grid, dim3(NT), 0, st, (const cpx<T> *)a,
                               (const cpx<T> *)b, (cpx<T> *)out, n, rank);
    }
    return hipGetLastError();
}

hipError_t launch_scale_planes(int dtype, bool conj, const void *a, const void *b, void *out, size_t n, int rank,
                               hipStream_t st) {
    return dtype == FIO_C128 ? amp_t<double>(false, conj, a, b, out, n, rank, st)
                             : amp_t<float>(false, conj, a, b, out, n, rank, st);
}

hipError_t launch_combine_planes(int dtype, bool conj, const void *a, const void *b, void *out, size_t n, int rank,
                                 hipStream_t st) {
    return dtype == FIO_C128 ? amp_t<double>(true, conj, a, b, out, n, rank, st)
                             : amp_t<float>(true, conj, a, b, out, n, rank, st);
}

// ---------------------------------------------------------------------------
// Staging of the allocation-free amplitude apply: a file-scope device array
// (each device that loads the library holds its own copy until the process
// ends).  Host code never passes the array's name to a kernel -- on the host
// that name is only a stand-in -- but the address hipGetSymbolAddress gives
// for it on each device, looked up once per device with that device current.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES];

// Address of `scratch` on `device` (which must be current); NULL on failure.
static void *scratch_of_device(int device) {
    if (device < 0 || device >= MAX_DEVICES) {
        set_error(FIO_EDEVICE, "device %d beyond the %d devices the scratch table covers", device, MAX_DEVICES);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
            return nullptr;
        }
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}

}  // namespace fio

extern "C" int fio_apply_amplitude_noalloc(fio_plan_t plan, const void *f, const void *g, const void *h, int rank,
                                           void *u, void *stream) {
    return fio::amplitude_apply_in(plan, f, g, h, rank, u, fio::NOALLOC_SCRATCH_BYTES, fio::scratch_of_device,
                                   stream);
}
