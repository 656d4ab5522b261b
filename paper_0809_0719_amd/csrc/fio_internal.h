// Internal definitions shared by the host plan (fio_plan.cpp) and the HIP
// kernels (fio_kernels_fwd.hip, fio_kernels_adj.hip, fio_kernels_init.hip,
// fio_kernels_term.hip, fio_kernels_mfma.hip, fio_kernels_tan.hip,
// fio_kernels_amp.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fio.h"

namespace fio {

constexpr int QMIN = 3;
constexpr int QMAX = 16;

// Phase parameters as the kernels see them.  For FOURIER the ellipse
// coefficients are zero, which makes the square-root term vanish exactly.
struct PhaseDev {
    int kind;
    double a1, a2, eta1, eta2;
};

// Geometry of a plan, passed by value to every kernel.
struct Geom {
    int N;       // grid side
    int L;       // log2 N
    int q;       // Chebyshev points per dimension
    int s;       // levels skipped at each end
    int lm;      // switch level
    double rho_scale;  // (sqrt(2)/2) N : |k| = rho_scale * p1 (eq:polar)
    int sw_ppw;        // items per workgroup of the matrix-core switches (8, 16 or 32; tuned)
};

// Device-resident tables of a plan (all FP64 except where a float copy is kept).
//   z[q]            Chebyshev nodes cos(i pi/(q-1))/2 (middle node exactly 0 for odd q)
//   lam[q]          barycentric weights 1/prod_{j!=i}(z_i - z_j)
//   M[2][q][q]      M_c[t][j] = L_t((z_j + c - 1/2)/2): parent basis t at child node j
//   Tt[2^s][q]      Tt[j][t] = L_t(j 2^-s - 1/2): basis t at the 2^s grid points of a leaf-level box
struct Tables {
    const double *z;
    const double *lam;
    const double *M;    // FP64 copy
    const float  *Mf;   // FP32 copy
    const double *Tt;
    const float  *Ttf;
    // Chebyshev-symmetric halves of M_0 (M_1 = J M_0 J, J the reversal), four
    // q x q matrices: [0] S[n][m] = (M_0[n][m] + M_0[q-1-n][m]) / 2 and
    // [1] A[n][m] = (M_0[n][m] - M_0[q-1-n][m]) / 2 for contractions that sum
    // two children into one output; [2] ST[n][m] = (M_0[m][n] + M_0[q-1-m][n]) / 2
    // and [3] AT[n][m] = (M_0[m][n] - M_0[q-1-m][n]) / 2 for m < q/2
    // (ST[n][(q-1)/2] = M_0[(q-1)/2][n] for odd q, zero past) for contractions
    // that feed one input to two children.
    const double *SA;   // FP64
    const float  *SAf;  // FP32
};

// Sources of T_P sorted by their box at level L-s (a CSR over Morton order).
struct Sources {
    const int32_t *idx;     // Omega index (k1+N/2)*N + (k2+N/2) of the j-th sorted source
    const double2 *p;       // (p1, p2) of the j-th sorted source
    const int32_t *off;     // off[mB] .. off[mB+1]: sources of the box with Morton index mB
};

// Kernel launchers (defined in fio_kernels_fwd.hip / fio_kernels_adj.hip).  All return hipError_t of the launch.
// `dtype` selects FP64 (FIO_C128) or FP32 (FIO_C64) weights.  The level and
// switch launchers process `nrhs` right-hand sides whose weights are planes
// `plane` complex values apart; initialisation and termination take one.
hipError_t launch_init(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb,
                       const Sources &src, const void *f, void *w_out, hipStream_t st);
hipError_t launch_plevel(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                         const void *w_in, void *w_out, int nrhs, size_t plane, hipStream_t st);
hipError_t launch_switch(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb,
                         void *w, int nrhs, size_t plane, hipStream_t st);
hipError_t launch_xlevel(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                         const void *w_in, void *w_out, int nrhs, size_t plane, hipStream_t st);
hipError_t launch_term(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb,
                       const void *w_in, void *u, hipStream_t st);

// Batched level kernels with BF16 MFMA contractions (fio_kernels_mfma.hip),
// complex64 weights; mfma_supported_q tells which q they are built for.
bool mfma_supported_q(int q);
hipError_t launch_plevel_mfma(const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                              const void *w_in, void *w_out, int nrhs, size_t plane, hipStream_t st);

// Initialisation and its adjoint on the matrix cores (fio_kernels_init.hip),
// complex64, s = 3, q <= 9.  They read two tables in sorted source order:
// ktab (N^2 rows of init_mfma_ktab_row(q) floats, the Lagrange products; made
// once per plan by launch_init_tables) and etab (N^2 rows of 64 complex64,
// E(x0(A), k); made by launch_init_etab whenever the phase changes).  The
// forward gathers the `nrhs` right-hand sides (f planes N^2 apart) into
// sorted order in `fsorted` (nrhs N^2 complex64) first; weights are planes
// `plane` apart.
bool init_mfma_supported(int q, int s);
int init_mfma_ktab_row(int q);
hipError_t launch_init_tables(const Geom &g, const Tables &tb, const Sources &src, void *ktab, hipStream_t st);
hipError_t launch_init_etab(const Geom &g, const PhaseDev &ph, const Sources &src, void *etab, hipStream_t st);
hipError_t launch_init_mfma(const Geom &g, const PhaseDev &ph, const Tables &tb, const Sources &src,
                            const void *ktab, const void *etab, const void *f, void *fsorted, void *w, int nrhs,
                            size_t plane, hipStream_t st);
hipError_t launch_init_adj_mfma(const Geom &g, const PhaseDev &ph, const Tables &tb, const Sources &src,
                                const void *ktab, const void *etab, const void *w, void *f, int nrhs,
                                size_t plane, hipStream_t st);

// Switch and adjoint switch on the matrix cores (fio_kernels_swadj.hip),
// complex64, q <= 9 and nrhs >= 32: in place on the weights at level lm,
// planes `plane` apart; the same operators as the vector kernels of
// launch_switch and launch_switch_adj.
bool switch_mfma_supported(int q, int nrhs);
bool switch_ppw_supported(int ppw);
hipError_t launch_switch_mfma(const Geom &g, const PhaseDev &ph, const Tables &tb, void *w, int nrhs, size_t plane,
                              hipStream_t st);
bool switch_adj_mfma_supported(int q, int nrhs);
hipError_t launch_switch_adj_mfma(const Geom &g, const PhaseDev &ph, const Tables &tb, void *w, int nrhs,
                                  size_t plane, hipStream_t st);

// Levels on the matrix cores (fio_kernels_lvlmm.hip, complex64, q <= 9): the
// p-level (adjoint_x false; eq:alg2b, level l from level l - 1) or the
// adjoint x-level (adjoint_x true; the transpose of eq:alg2c at level l, from
// level l to level l - 1), `nrhs` right-hand sides whose weights are planes
// `plane` complex values apart.
bool level_mfma_supported(int q);
hipError_t launch_level_mm(bool adjoint_x, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                           const void *w_in, void *w_out, int nrhs, size_t plane, hipStream_t st);

// Termination and its adjoint for `nrhs` > 1 right-hand sides in one launch
// (fio_kernels_term.hip): weights planes `plane` apart, potentials `uplane`.
hipError_t launch_term_batch(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, const void *w_in,
                             void *u, int nrhs, size_t plane, size_t uplane, hipStream_t st);
hipError_t launch_term_adj_batch(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, const void *u,
                                 void *w_out, int nrhs, size_t plane, size_t uplane, hipStream_t st);

// Elementwise steps of the separated-amplitude applies (fio_kernels_amp.hip):
// scale:   out[t][i] = op(a[t][i]) b[i];   combine: out[i] = sum_t op(a[t][i]) b[t][i],
// op = conj if `conj`, t < rank, i < n.
hipError_t launch_scale_planes(int dtype, bool conj, const void *a, const void *b, void *out, size_t n, int rank,
                               hipStream_t st);
hipError_t launch_combine_planes(int dtype, bool conj, const void *a, const void *b, void *out, size_t n, int rank,
                                 hipStream_t st);

// Adjoint launchers: exact conjugate transposes of the above.
hipError_t launch_term_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb,
                           const void *u, void *w_out, hipStream_t st);
hipError_t launch_xlevel_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                             const void *w_in, void *w_out, int nrhs, size_t plane, hipStream_t st);
hipError_t launch_switch_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb,
                             void *w, int nrhs, size_t plane, hipStream_t st);
hipError_t launch_plevel_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb, int level,
                             const void *w_in, void *w_out, int nrhs, size_t plane, hipStream_t st);
hipError_t launch_init_adj(int dtype, const Geom &g, const PhaseDev &ph, const Tables &tb,
                           const Sources &src, const void *w_in, void *f, hipStream_t st);

// Forward pass with the derivatives with respect to the phase's velocity
// scalings (fio_kernels_tan.hip): the weights of one right-hand side are
// three planes `plane` complex values apart (primal, d/da1, d/da2).  `step`:
// 0 initialisation (in = f), 1 p-level, 2 switch (in place on out),
// 3 x-level, 4 termination (out = u or NULL, u1 = du/da1, u2 = du/da2).
// The level and switch steps (1, 2, 3) take `nrhs` right-hand sides whose
// planes start 3 * plane apart; the others take one and ignore `nrhs`.
bool tangent_supported_q(int q);
hipError_t launch_tangent_step(int dtype, int step, const Geom &g, const PhaseDev &ph, const Tables &tb,
                               const Sources &src, int level, const void *in, void *out, size_t plane,
                               void *u1, void *u2, int nrhs, hipStream_t st);

// Direct sum of eq:dfio at listed targets (FP64 phase, exponentials and sums)
// and the SplitMix64 unit-modulus probe (fio_kernels_direct.hip).
hipError_t launch_direct_rows(int dtype, int N, const PhaseDev &ph, const void *f, const int64_t *rows, int nrows,
                              void *out, hipStream_t st);
hipError_t launch_probe(int dtype, int N, uint64_t seed, void *f, hipStream_t st);

// Three dimensions (fio_kernels_3d.hip, host side fio3.cpp).
struct Geom3 {
    int N, L, q, s, lm, kind;
    double rho_scale;  // (sqrt(3)/2) N : |k| = rho_scale * p1
};
//   z[q], lam[q]   Chebyshev nodes and barycentric weights 1/prod_{j!=i}(z_i - z_j)
//   M[2][q][q]     M_c[t][j] = L_t((z_j + c - 1/2)/2), FP64 and FP32
//   T[2^s][q]      T[j][t] = L_t(j 2^-s - 1/2), FP64 and FP32
struct Tab3 {
    const double *z, *lam, *Md, *Td;
    const float *Mf, *Tf;
};
// Sources sorted by their level-(L-s) box: Omega index, p (3 per source), CSR offsets.
struct Src3 {
    const int32_t *idx;
    const double *p;
    const int32_t *off;
};
// step: 0 initialisation (in = f), 1 p-level, 2 switch (in place on out),
// 3 x-level, 4 termination (out = u).
hipError_t launch_step3(int dtype, int step, const Geom3 &g, const Tab3 &tb, const Src3 &src, int level,
                        const void *in, void *out, hipStream_t st);
// The conjugate transposes: step 4 termination^H (in = u), 3 x-level^H
// (outputs at `level` -> inputs at level - 1), 2 switch^H (in place on out),
// 1 p-level^H (likewise), 0 initialisation^H (out = f).
hipError_t launch_step3_adj(int dtype, int step, const Geom3 &g, const Tab3 &tb, const Src3 &src, int level,
                            const void *in, void *out, hipStream_t st);

// Host helpers shared by the host sources (defined in fio_plan.cpp): the
// calling thread's error message, and the parts of a plan other host code
// needs.
int set_error(int code, const char *fmt, ...);
int set_hip_error(hipError_t e, const char *what);
void clear_error();
// fio_apply_amplitude with its two staging buffers (2 rank N^2 complex
// values) taken from a caller-provided device array instead of the plan's
// workspace: scratch_of_device(d) returns the array's address on device d
// (NULL after setting the error message on failure); FIO_EINVAL when the
// staging needs more than scratch_bytes.  Allocates nothing.
int amplitude_apply_in(fio_plan_t plan, const void *f, const void *g, const void *h, int rank, void *u,
                       size_t scratch_bytes, void *(*scratch_of_device)(int device), void *stream);

struct PlanView {
    int N, q, dtype, device;
    PhaseDev ph;
};
int plan_view(fio_plan_t plan, PlanView *v);

}  // namespace fio
