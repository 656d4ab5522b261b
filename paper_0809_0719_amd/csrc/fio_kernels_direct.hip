// Direct evaluation of eq:dfio at a few target points, and the random probe
// input of the q selector.
//
// k_direct_rows: u(x_i) = sum_k e^{2 pi i Phi(x_i, k)} f(k) for the listed
// targets, one workgroup per target, the N^2 sources strided over its
// threads.  The phase is FP64, reduced mod 1 exactly, the exponential and
// the sum FP64 whatever the storage type, so the result is the definition to
// rounding: the reference the error estimate eq:err (Sec. 5) compares the
// butterfly against on a sample of targets.
//
// k_probe: f(k) = e^{2 pi i v_k}, v_k uniform in [0, 1) from the SplitMix64
// generator (Steele, Lea and Flood, 2014) at counter k: unit-modulus random
// phases, so E|f|^2 = 1 and every frequency is excited.
#include <hip/hip_runtime.h>

#include "fio_kernels_common.h"

namespace fio {

template <typename T>
__global__ __launch_bounds__(NT) void k_direct_rows(int N, PhaseDev ph, const cpx<T> *__restrict__ f,
                                                    const int64_t *__restrict__ rows, int nrows,
                                                    cpx<T> *__restrict__ out) {
    __shared__ double red[2][NT / 64];
    const int i = blockIdx.x;
    const int64_t row = rows[i];
    const int i1 = (int)(row / N), i2 = (int)(row - (int64_t)i1 * N);
    const XP xp = make_xp(ph, (double)i1 / N, (double)i2 / N);
    const int n2 = N * N, h = N / 2;
    double sr = 0.0, si = 0.0;
    for (int k = threadIdx.x; k < n2; k += NT) {
        const int j1 = k / N, j2 = k - j1 * N;
        const cpx<double> e = cis<double>(phase_cart(xp, (double)(j1 - h), (double)(j2 - h)));
        const cpx<T> v = f[k];
        sr = fma(e.re, (double)v.re, fma(-e.im, (double)v.im, sr));
        si = fma(e.re, (double)v.im, fma(e.im, (double)v.re, si));
    }
    // wave sums, then across the waves
    for (int o = 32; o > 0; o >>= 1) {
        sr += __shfl_xor(sr, o);
        si += __shfl_xor(si, o);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = sr;
        red[1][wv] = si;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < NT / 64; ++w) {
            a += red[0][w];
            b += red[1][w];
        }
        out[i] = {(T)a, (T)b};
    }
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_probe(int n2, uint64_t seed, cpx<T> *__restrict__ f) {
    const int k = blockIdx.x * NT + threadIdx.x;
    if (k >= n2) return;
    const double v = (double)(splitmix64(seed, (uint64_t)k) >> 11) * 0x1.0p-53;
    double s, c;
    sincospi(2.0 * v, &s, &c);
    f[k] = {(T)c, (T)s};
}

hipError_t launch_direct_rows(int dtype, int N, const PhaseDev &ph, const void *f, const int64_t *rows, int nrows,
                              void *out, hipStream_t st) {
    if (dtype == FIO_C128)
        hipLaunchKernelGGL((k_direct_rows<double>), dim3(nrows), dim3(NT), 0, st, N, ph, (const cpx<double> *)f, rows,
                           nrows, (cpx<double> *)out);
    else
        hipLaunchKernelGGL((k_direct_rows<float>), dim3(nrows), dim3(NT), 0, st, N, ph, (const cpx<float> *)f, rows,
                           nrows, (cpx<float> *)out);
    return hipGetLastError();
}

hipError_t launch_probe(int dtype, int N, uint64_t seed, void *f, hipStream_t st) {
    const int n2 = N * N;
    const dim3 grid((unsigned)((n2 + NT - 1) / NT));
    if (dtype == FIO_C128)
        hipLaunchKernelGGL((k_probe<double>), grid, dim3(NT), 0, st, n2, seed, (cpx<double> *)f);
    else
        hipLaunchKernelGGL((k_probe<float>), grid, dim3(NT), 0, st, n2, seed, (cpx<float> *)f);
    return hipGetLastError();
}

}  // namespace fio
