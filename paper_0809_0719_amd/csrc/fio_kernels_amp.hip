// Variable amplitude through a separated approximation a(x,k) = sum_t g_t(x)
// h_t(k) (end of Sec. 4): the butterfly is applied to the rank inputs
// h_t f together (they share every kernel value), and the outputs are
// multiplied by g_t and summed.  The two elementwise steps are here; both are
// plain streaming kernels (bandwidth-bound).
#include <hip/hip_runtime.h>

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

}  // namespace fio
