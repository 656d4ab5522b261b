/*
 * fio.h -- C ABI of the MI355X butterfly evaluator for 2-D discrete Fourier
 * integral operators (Candes, Demanet & Ying, "A fast butterfly algorithm
 * for the computation of Fourier integral operators").
 *
 * The operator (eq:dfio, Sec. 1):
 *
 *     u(x) = sum_{k in Omega} exp(2 pi i Phi(x,k)) f(k),   x in X,
 *     X     = {(i1/N, i2/N) : 0 <= i1,i2 < N},
 *     Omega = {(k1,k2)      : -N/2 <= k1,k2 < N/2},
 *
 * is approximated by the butterfly of Sec. 4: the sources are mapped to
 * polar coordinates p (eq:polar), the quadtrees T_X and T_P are paired level
 * by level with l(A) + l(B) = L = log2 N, and per box pair (A,B) a q x q
 * tensor Chebyshev expansion delta^{AB}_t is carried from the leaves of T_P
 * (initialisation, eq:alg2a) through the p-interpolation levels (eq:alg2b),
 * the switch (eq:alg2m) and the x-interpolation levels (eq:alg2c) to the
 * potentials (termination, eq:alg2d).  As in the numerical section, the
 * recursion starts s levels above the leaves of T_P and stops s levels
 * below its root (pairs (A at level s, B at level L-s) first, (A at level
 * L-s, B at level s) last, the potentials summing over the 4^s boxes B).
 *
 * All compute runs in HIP kernels on the current device.  Every pointer
 * marked "device" must be device memory on that device; the library never
 * reads or writes host copies of the data.  Calls are asynchronous on the
 * given stream (a hipStream_t passed as void*, NULL = the null stream).
 *
 * Error behaviour: every function returns FIO_OK (0) or a negative code;
 * argument errors are detected before any launch.  fio_last_error() gives a
 * human-readable message for the calling thread's last failure.
 *
 * Thread-safety: distinct plans may be used concurrently; one plan owns one
 * workspace, so concurrent applies on the same plan must be serialised by
 * the caller (e.g. by issuing them on one stream).
 *
 * Graph capture: fio_apply and fio_apply_adjoint only launch kernels on the
 * given stream (no allocation, memset or synchronisation), so a capture of
 * them into a HIP graph replays the pass.  The replay uses the phase that
 * was current at capture time.  fio_apply_dphase allocates its tangent
 * workspace on its first call when nrhs_max < 3; call it once before
 * capturing it.
 */
#ifndef FIO_H
#define FIO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define FIO_OK        0
#define FIO_EINVAL   (-1)  /* bad argument (N, q, s, lm, nrhs, pointer, ...) */
#define FIO_ENOMEM   (-2)  /* device or host allocation failed               */
#define FIO_EDEVICE  (-3)  /* a HIP runtime call or kernel launch failed     */

/* ---- phase functions ----------------------------------------------------
 * Phi must be smooth for k != 0 and homogeneous of degree 1 in k (Sec. 1).
 *
 * FIO_PHASE_FOURIER:  Phi(x,k) = x . k   (the 2-D DFT; the closed-form check)
 * FIO_PHASE_ELLIPSE:  Phi(x,k) = x . k + sqrt(c1(x)^2 k1^2 + c2(x)^2 k2^2),
 *     c1(x) = a1 (2 + (1+eta1) sin(2 pi x1) sin(2 pi x2)) / 3,
 *     c2(x) = a2 (2 + (1+eta2) cos(2 pi x1) cos(2 pi x2)) / 3,
 *   which is eq:ex1 (Sec. 5) for a1 = a2 = 1, eta1 = eta2 = 0.  a1, a2 are
 *   velocity scalings (e.g. learnable), eta1, eta2 perturb the modulation.
 *   Requires a1, a2 > 0 and -1 <= eta1, eta2 <= 1 (so c_j > 0).         */
#define FIO_PHASE_FOURIER 0
#define FIO_PHASE_ELLIPSE 1

typedef struct {
    int    kind;       /* FIO_PHASE_*                     */
    double a1, a2;     /* ELLIPSE velocity scalings (> 0) */
    double eta1, eta2; /* ELLIPSE modulation amplitudes   */
} fio_phase_t;

/* ---- precision ----------------------------------------------------------
 * Phases Phi are always evaluated in FP64 and reduced mod 1 in FP64 (their
 * magnitude reaches ~N cycles, so single precision would lose the phase).
 *
 * FIO_C128: f, u are complex128; weights, exponentials and contractions FP64.
 * FIO_C64:  f, u are complex64; the reduced phase feeds an FP32 exponential,
 *           weights and interpolation contractions are FP32.              */
#define FIO_C128 0
#define FIO_C64  1

/* Contraction precision of the interpolation passes (FIO_C64 plans only):
 * FIO_CONTRACT_FP:   FP32 on the vector ALUs (default);
 * FIO_CONTRACT_BF16: operands rounded to BF16, products accumulated in FP32
 *                    on the matrix cores (MFMA), right-hand sides in tiles
 *                    of 16; kernel values and all other steps stay FP32/FP64.
 *                    Requires q <= 12.                                     */
#define FIO_CONTRACT_FP   0
#define FIO_CONTRACT_BF16 1
/* FIO_CONTRACT_MFMA: the p-levels and the adjoint x-levels of chunks of 32 or
 *                    more right-hand sides run their interpolation passes as
 *                    FP32 matrix-core products (v_mfma_f32_4x4x1f32) with
 *                    the Chebyshev-symmetric halves of the interpolation
 *                    matrices; every other step as FIO_CONTRACT_FP.  Results
 *                    agree with FIO_CONTRACT_FP to FP32 rounding.  Requires
 *                    FIO_C64 and q <= 9.                                     */
#define FIO_CONTRACT_MFMA 2

typedef struct fio_plan_s *fio_plan_t;

/* Options for fio_plan_ex.  Any field set to -1 takes its default. */
typedef struct {
    int s;        /* levels skipped at each end of the trees; default min(3, L/2)
                     (the numerical section starts at level log2N-3 of T_P and
                     stops at level 3); s = 0 is Sec. 4 verbatim               */
    int lm;       /* switch level (eq:alg2m); default floor(L/2); must satisfy
                     s <= lm <= L - s                                          */
    int dtype;    /* FIO_C64 (default) or FIO_C128                             */
    int nrhs_max; /* right-hand sides processed together (default 1, at most
                     4096): the plan holds two weight buffers of nrhs_max
                     N^2 q^2 complex values, and fio_apply / fio_apply_adjoint
                     take nrhs in chunks of nrhs_max, computing every kernel
                     value of the levels and the switch once per chunk (the
                     vectorised butterfly of Sec. 4, last paragraphs)        */
    int contract; /* FIO_CONTRACT_FP (default), FIO_CONTRACT_BF16 or
                     FIO_CONTRACT_MFMA                                        */
} fio_plan_opts_t;

/* Geometry and sizes of a plan. */
typedef struct {
    int N, q, L, s, lm, dtype, contract;
    int64_t n_pairs;          /* box pairs per level = N^2                        */
    int64_t weights_per_level;/* complex weights per level per RHS = N^2 q^2      */
    int64_t workspace_bytes;  /* device memory owned by the plan                  */
    int max_box_sources;      /* largest number of sources in a level-(L-s) box */
    int nrhs_max;             /* right-hand sides the weight buffers hold          */
    int chunk;                /* right-hand sides per pass (nrhs_max unless tuned) */
    int switch_items;         /* pair items per workgroup of the matrix-core
                                 switches (16 unless tuned)                        */
} fio_plan_info_t;

/* Create a plan for an N x N problem with q Chebyshev points per dimension
 * (r = q^2 expansion terms per box pair, Sec. 3).
 *   N:     power of two, 8 <= N <= 8192 (N = 2^L).
 *   q:     3 <= q <= 16.
 *   phase: host pointer, copied into the plan.
 *   out:   host pointer receiving the plan handle.
 * Builds T_P for the polar images of Omega (Sec. 4 step 1; sources sorted by
 * their level-(L-s) box) and the interpolation tables (the Lagrange values
 * L^B_t(p^{B_c}_t') are the same for every pair and level, Sec. 4), and
 * allocates two weight buffers of nrhs_max x N^2 q^2 complex values each
 * (only two consecutive levels of weights are ever live, Sec. 4) on the
 * current device.  Returns FIO_OK, FIO_EINVAL, FIO_ENOMEM or FIO_EDEVICE. */
int fio_plan(int N, int q, const fio_phase_t *phase, fio_plan_t *out);
int fio_plan_ex(int N, int q, const fio_phase_t *phase,
                const fio_plan_opts_t *opts, fio_plan_t *out);

/* Replace the phase parameters of a plan (e.g. after a gradient step on
 * a1, a2).  The trees and tables do not depend on the phase. */
int fio_set_phase(fio_plan_t plan, const fio_phase_t *phase);

int fio_plan_get_info(fio_plan_t plan, fio_plan_info_t *info);

/* Launch-shape autotuner (end of Sec. 4: the vectorised butterfly; the
 * shapes are this library's own).  Times a forward and an adjoint apply of
 * nrhs right-hand sides on the plan's device for each candidate pair
 *   switch_items in {8, 16, 32}   (pair items per workgroup of the
 *                                  matrix-core switches),
 *   chunk in {32, 64, ..., nrhs_max} (right-hand sides per pass),
 * and keeps the fastest in the plan for every later apply.  Every candidate
 * runs the same arithmetic on each right-hand side (the kernels each chunk
 * takes do not change while chunk >= 32), so results do not depend on the
 * choice; a chunk shape is a candidate only when it leaves each right-hand
 * side of a call of nrhs in a pass of >= 32 (or in the same last pass) as
 * the current shape does.  Plans where nothing applies (complex128, q > 9,
 * nrhs_max, nrhs or the current chunk below 32) keep their shape and report
 * it with candidates = 0.
 *   nrhs: right-hand sides per call to tune for (inputs are zero-filled
 *         device buffers the call allocates and frees: 2 nrhs N^2 complex).
 *   out:  host pointer or NULL; receives the choice and the measured times
 *         (milliseconds per forward + adjoint pair; best and default shape).
 * Synchronises the device.  FIO_EINVAL on bad arguments, FIO_ENOMEM,
 * FIO_EDEVICE. */
typedef struct {
    int chunk, switch_items;   /* the shape kept                          */
    int candidates;            /* shapes timed (0: nothing to tune)       */
    double best_ms;            /* forward + adjoint at the kept shape     */
    double default_ms;         /* forward + adjoint at the default shape  */
} fio_tune_t;
int fio_plan_autotune(fio_plan_t plan, int nrhs, fio_tune_t *out);
/* Set the launch shape directly: chunk in [1, nrhs_max], switch_items in
 * {8, 16, 32} (the shapes fio_plan_autotune chooses among).  FIO_EINVAL
 * otherwise. */
int fio_plan_set_shape(fio_plan_t plan, int chunk, int switch_items);

/* Forward butterfly u = B f (approximates eq:dfio).
 *   f: device, nrhs x N x N complex (plan dtype), f[r][k1+N/2][k2+N/2].
 *      Read only.
 *   u: device, nrhs x N x N complex (plan dtype), u[r][i1][i2] = u_r(i1/N,
 *      i2/N).  Fully overwritten.  The byte ranges of f and u (nrhs N^2
 *      complex values each) must not share a byte.
 *   nrhs >= 1 right-hand sides, processed in chunks of the plan's chunk
 *   (nrhs_max unless fio_plan_autotune chose fewer);
 *   within a chunk the kernel values of the levels and the switch are
 *   computed once and applied to every right-hand side.
 *   dtype: FIO_C64 or FIO_C128, the element type of f and u as the caller
 *      holds them; it must equal the plan's dtype (the weight buffers, the
 *      tables and the kernels are sized and compiled for the plan's precision
 *      when the plan is made, so a call cannot switch it).
 * Asynchronous on `stream`; FIO_EINVAL before any launch on bad arguments
 * (NULL pointers, nrhs < 1, a dtype other than the plan's, overlapping
 * ranges). */
int fio_apply(fio_plan_t plan, const void *f, void *u, int nrhs, int dtype, void *stream);

/* Adjoint butterfly f = B^H u: the exact conjugate transpose of the
 * forward pipeline (termination^H, x-levels^H, switch^H, p-levels^H,
 * initialisation^H), which approximates f(k) = sum_x exp(-2 pi i Phi(x,k))
 * u(x).  Same layouts and rules as fio_apply with the roles of f, u swapped.
 * Chunks of 32 or more complex64 right-hand sides at q <= 9 take the switch^H
 * on the matrix cores, as fio_apply takes the switch (FP32 products and sums
 * in another order: the results agree with the single-right-hand-side path
 * to FP32 rounding). */
int fio_apply_adjoint(fio_plan_t plan, const void *u, void *f, int nrhs, int dtype, void *stream);

/* Forward butterfly with its derivatives with respect to the velocity
 * scalings a1, a2 of the ellipse phase (Sec. 5, eq:ex1 family), at the
 * plan's current phase: for every right-hand side r
 *     u[r]      = B f[r]                (as fio_apply, to rounding),
 *     du_da1[r] = d(B f[r]) / d a1,     du_da2[r] = d(B f[r]) / d a2,
 * the exact derivatives of the butterfly approximation itself (every kernel
 * value E = exp(2 pi i Phi) of Sec. 4 differentiated, the Chebyshev grids
 * and tables held fixed), by forward-mode propagation of two tangent weight
 * sets beside the primal one.  For FIO_PHASE_FOURIER both derivatives are 0.
 *   f: device, nrhs x N x N complex (plan dtype), read only.
 *   u: device, nrhs x N x N, or NULL (then the primal output is not stored).
 *   du_da1, du_da2: device, nrhs x N x N each; fully overwritten.
 *   The outputs must not overlap f or each other.  Requires q <= 12.
 * Workspace: three N^2 q^2 planes per right-hand side in each of two
 * buffers -- the plan's own weight buffers when nrhs_max >= 3, else two
 * buffers of three planes that the first call allocates and the plan keeps
 * until fio_destroy (FIO_ENOMEM if that fails).  The right-hand sides go in
 * chunks of at most nrhs_max / 3 (at least one), split as evenly as they
 * come; the level kernels of a chunk share their kernel values and
 * derivative factors, so a chunk's results equal those of one right-hand
 * side at a time bit for bit.  Asynchronous on `stream`; FIO_EINVAL before
 * any launch on bad arguments. */
int fio_apply_dphase(fio_plan_t plan, const void *f, void *u, void *du_da1, void *du_da2, int nrhs,
                     void *stream);

/* Variable amplitude (eq:allfio) through a separated approximation
 *     a(x,k) = sum_{t < rank} g_t(x) h_t(k)       (end of Sec. 4):
 *   fio_apply_amplitude:         u = sum_t g_t . B(h_t . f)
 *                                  ~ sum_k a(x,k) exp(2 pi i Phi(x,k)) f(k),
 *   fio_apply_amplitude_adjoint: f = sum_t conj(h_t) . B^H(conj(g_t) . u)
 *                                  ~ sum_x conj(a(x,k)) exp(-2 pi i Phi(x,k)) u(x)
 * ('.' is the elementwise product).  The rank butterfly applications run
 * as right-hand sides of one batched apply (chunks of nrhs_max), sharing
 * every kernel value, as the end of Sec. 4 recommends.
 *   f, u: device, N x N complex (plan dtype), layouts as fio_apply; the input
 *         is read only, the output fully overwritten and must not overlap
 *         the inputs.
 *   g: device, rank x N x N complex, g[t][i1][i2] = g_t(i1/N, i2/N).
 *   h: device, rank x N x N complex, h[t][k1+N/2][k2+N/2] = h_t(k).
 *   1 <= rank <= 4096.
 * Workspace: two buffers of rank N^2 complex values, allocated by the plan
 * on first use and regrown (after a device synchronisation) when a larger
 * rank comes; FIO_ENOMEM if that fails.  Asynchronous on `stream` otherwise;
 * FIO_EINVAL before any launch on bad arguments. */
int fio_apply_amplitude(fio_plan_t plan, const void *f, const void *g, const void *h, int rank, void *u,
                        void *stream);
int fio_apply_amplitude_adjoint(fio_plan_t plan, const void *u, const void *g, const void *h, int rank,
                                void *f, void *stream);

/* fio_apply_amplitude for callers that cannot allocate device memory during
 * the call -- code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc: the same computation with the same kernels, but its
 * two staging buffers (the rank scaled inputs h_t . f and the rank butterfly
 * outputs) live in a static device array of 64 MiB that the library holds
 * on every device it is loaded on, instead of the plan's workspace, which
 * fio_apply_amplitude allocates on first use and regrows (after a device
 * synchronisation) for a larger rank.  This call allocates nothing, frees
 * nothing and synchronises nothing.
 *   Limit: 2 rank N^2 complex values of the plan dtype must fit in 64 MiB
 *   (complex64: rank N^2 <= 4194304, e.g. rank 64 at N = 256, 4 at N = 1024);
 *   larger requests return FIO_EINVAL before any launch.
 *   Every call on one device shares that device's array and leaves the last
 *   call's values in it (each call fully overwrites what it reads, nothing
 *   needs to start at zero): calls that may overlap in time on one device --
 *   on different streams, or from different threads -- race; serialise them
 *   (e.g. on one stream).  The plan's own weight buffers are used as by
 *   fio_apply.
 *   Arguments, layouts and errors otherwise as fio_apply_amplitude. */
int fio_apply_amplitude_noalloc(fio_plan_t plan, const void *f, const void *g, const void *h, int rank, void *u,
                                void *stream);

/* ---- uneven batches ------------------------------------------------------
 * A batch applies several plans (any N, q, phase, dtype) as one unit, the
 * mixed-size workload of many small and large problems: fio_batch_apply
 * forks from `stream` onto the batch's internal streams (events only, no
 * host synchronisation), runs each plan's fio_apply there -- the largest work
 * (N^2 q^3) first, each on the stream with the least work so far -- and
 * joins back into `stream`, so problems too small to fill the device run
 * side by side.  Since the fork and the join are events, a stream capture of
 * fio_batch_apply records the whole batch as one HIP graph (call it once
 * before capturing: plans make their initialisation tables on first use).
 *   plans:    host array of n distinct plans on one device.  The batch keeps
 *             the handles, not copies: destroy the batch before its plans,
 *             and do not use a plan elsewhere while a batch apply that
 *             includes it may be running.
 *   1 <= n <= 4096; 1 <= nstreams <= 16 (internal streams, default priority).
 *   f, u:     host arrays of n device pointers; f[i], u[i] are plan i's input
 *             and output for one right-hand side, laid out as for fio_apply.
 * FIO_EINVAL before any launch on bad arguments. */
typedef struct fio_batch_s *fio_batch_t;
int fio_batch_create(const fio_plan_t *plans, int n, int nstreams, fio_batch_t *out);
int fio_batch_apply(fio_batch_t batch, const void *const *f, void *const *u, void *stream);
int fio_batch_apply_adjoint(fio_batch_t batch, const void *const *u, void *const *f, void *stream);
int fio_batch_destroy(fio_batch_t batch);

/* Direct evaluation of eq:dfio at sampled targets, by the definition:
 *     out[i] = sum_k exp(2 pi i Phi(x_i, k)) f(k),  x_i = (r / N, r % N) / N,
 * r = rows[i], with the plan's N, phase and dtype.  Phases, exponentials and
 * sums are FP64 whatever the dtype (the output is stored in the plan dtype).
 * This is the reference of the error measure eq:err (Sec. 5) on a sample of
 * targets; it costs nrows N^2 phase evaluations.
 *   f:    device, N x N complex (plan dtype), as for fio_apply.
 *   rows: device, nrows int64 flat target indices i1 N + i2 in [0, N^2) (an
 *         index outside that range evaluates a point outside X; no memory is
 *         addressed by it).
 *   out:  device, nrows complex (plan dtype).
 *   1 <= nrows <= 2^20.  Asynchronous on `stream`. */
int fio_direct_rows(fio_plan_t plan, const void *f, const int64_t *rows, int nrows, void *out, void *stream);

/* Choice of q by the estimated error (Sec. 5: q is raised until the error
 * estimate is small enough).  For q = qmin, qmin + 1, ..., qmax: builds a
 * plan (N, phase and opts as given), applies it to the probe
 *     f(k) = exp(2 pi i v_k),  v_k = (SplitMix64(seed, k) >> 11) 2^-53,
 * with k the flat index k1' N + k2' (k' = k + N/2), and estimates eq:err
 * against fio_direct_rows on nrows targets rows[i] = SplitMix64(seed ^
 * 0x5851F42D4C957F2D, i) mod N^2, where SplitMix64(s, i) is the output of the
 * generator of Steele, Lea and Flood (2014) with state s + (i + 1) 0x9E3779B97F4A7C15.
 * Stops at the first q whose estimate is <= tol.
 *   q_out, err_out: host; the chosen q and its estimate.  When no q reaches
 *                   tol they receive qmax and its estimate (compare *err_out
 *                   with tol).
 *   errs:           host array of qmax - qmin + 1 doubles, or NULL; receives
 *                   every estimate made (NaN for the q not tried).
 *   3 <= qmin <= qmax <= 16, tol > 0, 1 <= nrows <= 4096.
 * Synchronous; allocates and frees its plans and buffers on the current
 * device (null stream). */
int fio_select_q(int N, const fio_phase_t *phase, const fio_plan_opts_t *opts, double tol, int qmin, int qmax,
                 int nrows, uint64_t seed, int *q_out, double *err_out, double *errs);

/* ---- three dimensions (Sec. 5, last example) -----------------------------
 * u(x) = sum_{k in Omega} exp(2 pi i Phi(x,k)) f(k) on X = {i/N}^3,
 * Omega = {-N/2 <= k_j < N/2}, by the butterfly with q x q x q tensor
 * Chebyshev grids and octrees (eight children per box), l(A) + l(B) = L.
 * The frequencies are mapped to spherical coordinates
 *     p = (|k| / (sqrt(3) N / 2), theta / pi, phi / (2 pi) mod 1),
 * theta = arccos(k3/|k|), phi = atan2(k2, k1), k = 0 -> p = 0, the analogue
 * of eq:polar, so that Phi(x, k(p)) = |k| Phi(x, k/|k|) is evaluated from
 * one direction phase per node.  Forward apply, one right-hand side.
 *   FIO3_PHASE_FOURIER: Phi = x . k
 *   FIO3_PHASE_SPHERES: eq:ex3, Phi = x . k + c(x)|k|,
 *                       c(x) = (3 + sin 2 pi x1 sin 2 pi x2 sin 2 pi x3)/4
 * fio3_plan: N power of two, 4 <= N <= 256; 3 <= q <= 8; s, lm as in
 *   fio_plan_opts_t (-1: min(3, L/2) and L/2; s <= lm <= L - s); dtype
 *   FIO_C64 or FIO_C128.  Holds two weight buffers of N^3 q^3 complex values
 *   and the sorted sources; FIO_ENOMEM if they do not fit.
 * fio3_apply: f device N x N x N complex (plan dtype),
 *   f[k1+N/2][k2+N/2][k3+N/2]; u device N x N x N, u[i1][i2][i3] = u(i/N);
 *   u must not overlap f.  Asynchronous on `stream`. */
#define FIO3_PHASE_FOURIER 0
#define FIO3_PHASE_SPHERES 1
typedef struct fio3_plan_s *fio3_plan_t;
int fio3_plan(int N, int q, int phase_kind, int s, int lm, int dtype, fio3_plan_t *out);
int fio3_apply(fio3_plan_t plan, const void *f, void *u, void *stream);
/* fio3_apply_adjoint: f = B^H u, the exact conjugate transpose of fio3_apply
 * (every step transposed, in reverse order); layouts as fio3_apply, f must
 * not overlap u.  Asynchronous on `stream`. */
int fio3_apply_adjoint(fio3_plan_t plan, const void *u, void *f, void *stream);
int fio3_destroy(fio3_plan_t plan);

/* Diagnostics: run the forward pipeline for one right-hand side up to and
 * including stage `stage` and copy that stage's weights to `weights`.
 *   stage 0                 : initialisation, level s
 *   stage 1 .. lm-s         : p-level s+stage
 *   stage lm-s+1            : after the switch, level lm
 *   stage lm-s+1+j (j >= 1) : x-level lm+j, up to level L-s
 *   weights: device, N^2 q^2 complex (plan dtype), laid out as
 *     weights[(mA * 4^(L-l) + mB) * q^2 + t1*q + t2]
 *   with l the stage's level, mA the Morton index of A at level l of T_X
 *   (bits of the x1 box index at odd positions, of the x2 index at even
 *   positions), mB the Morton index of B at level L-l of T_P (p1 bits odd,
 *   p2 bits even), and (t1, t2) the Chebyshev node of z_t1 in the first and
 *   z_t2 in the second coordinate. */
int fio_debug_stage(fio_plan_t plan, const void *f, int stage, void *weights, void *stream);

/* ---- per-kernel timing ----------------------------------------------------
 * With profiling enabled, every kernel launch of the plan is bracketed by
 * two HIP events recorded on the launch stream.  fio_profile_read waits for
 * those events, writes per kernel kind the summed elapsed milliseconds and
 * the number of launches since the last read (arrays of length n, n <= 
 * FIO_KERNEL_KINDS, host memory), and resets the counters.               */
#define FIO_K_INIT        0
#define FIO_K_PLEVEL      1
#define FIO_K_SWITCH      2
#define FIO_K_XLEVEL      3
#define FIO_K_TERM        4
#define FIO_K_TERM_ADJ    5
#define FIO_K_XLEVEL_ADJ  6
#define FIO_K_SWITCH_ADJ  7
#define FIO_K_PLEVEL_ADJ  8
#define FIO_K_INIT_ADJ    9
#define FIO_K_TANGENT    10  /* every kernel of fio_apply_dphase */
#define FIO_K_TABLES     11  /* kernel-value table, remade after a phase change */
#define FIO_KERNEL_KINDS 12

int fio_profile_enable(fio_plan_t plan, int enable);
int fio_profile_read(fio_plan_t plan, double *ms, int64_t *launches, int n);

/* Free the plan and its device workspace (synchronises the device first). */
int fio_destroy(fio_plan_t plan);

/* Message describing the calling thread's last error ("" if none). */
const char *fio_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FIO_H */
