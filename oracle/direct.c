/*
 * Direct-sum oracle for the discrete Fourier integral operator (TEST
 * INFRASTRUCTURE ONLY: nothing on the product path may link or call this).
 *
 *   u(x) = sum_{k in Omega} exp(2 pi i Phi(x,k)) f(k),   x in X        (eq:dfio, Sec. 1)
 *   X     = {(i1/N, i2/N) : 0 <= i1,i2 < N}
 *   Omega = {(k1,k2)      : -N/2 <= k1,k2 < N/2}
 *
 * Plain O(N^2) work per output row, accumulated in FP64 in natural order.
 * The phase is evaluated in Cartesian k straight from its definition
 * (eq:ex1, Sec. 5), reduced mod 1 in FP64 (|Phi| << 2^52, so the reduction
 * is exact), and the exponential is taken with libm sin/cos.
 *
 * Array conventions (interleaved complex, re/im as consecutive doubles):
 *   f[(k1+N/2)*N + (k2+N/2)]   sources
 *   u[i1*N + i2]               potentials
 */
#include <math.h>
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_FOURIER 0
#define ORC_ELLIPSE 1

typedef struct {
    int kind;        /* ORC_FOURIER: Phi = x.k ; ORC_ELLIPSE: eq:ex1 (generalised) */
    double a1, a2;   /* velocity scalings of c1, c2 (1 for eq:ex1)           */
    double eta1, eta2; /* amplitude of the x-modulation perturbation (0 for eq:ex1) */
} orc_phase_t;

static const double ORC_PI = 3.14159265358979323846264338327950288;

/* Phi(x,k) from its definition.  For ELLIPSE:
 *   Phi = x.k + sqrt( (a1 c1(x))^2 k1^2 + (a2 c2(x))^2 k2^2 )
 *   c1 = (2 + (1+eta1) sin(2 pi x1) sin(2 pi x2)) / 3
 *   c2 = (2 + (1+eta2) cos(2 pi x1) cos(2 pi x2)) / 3
 * which is eq:ex1 for a1=a2=1, eta1=eta2=0.  Homogeneous of degree 1 in k. */
double orc_phi(const orc_phase_t *ph, double x1, double x2, double k1, double k2)
{
    double v = x1 * k1 + x2 * k2;
    if (ph->kind == ORC_ELLIPSE) {
        double c1 = (2.0 + (1.0 + ph->eta1) * sin(2.0 * ORC_PI * x1) * sin(2.0 * ORC_PI * x2)) / 3.0;
        double c2 = (2.0 + (1.0 + ph->eta2) * cos(2.0 * ORC_PI * x1) * cos(2.0 * ORC_PI * x2)) / 3.0;
        c1 *= ph->a1;
        c2 *= ph->a2;
        v += sqrt(c1 * c1 * k1 * k1 + c2 * c2 * k2 * k2);
    }
    return v;
}

/* exp(2 pi i phi) with an exact FP64 mod-1 reduction first. */
static void orc_cis(double phi, double *re, double *im)
{
    double r = phi - rint(phi);
    *re = cos(2.0 * ORC_PI * r);
    *im = sin(2.0 * ORC_PI * r);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Forward: u at the listed rows (flat index i1*N+i2), all N^2 sources. */
void orc_direct_forward(int N, const orc_phase_t *ph, const double *f,
                        int nrows, const int64_t *rows, double *u)
{
    const int h = N / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < nrows; ++r) {
        const int64_t idx = rows[r];
        const double x1 = (double)(idx / N) / N;
        const double x2 = (double)(idx % N) / N;
        double sr = 0.0, si = 0.0;
        for (int j1 = 0; j1 < N; ++j1) {
            for (int j2 = 0; j2 < N; ++j2) {
                const double k1 = (double)(j1 - h), k2 = (double)(j2 - h);
                double er, ei;
                orc_cis(orc_phi(ph, x1, x2, k1, k2), &er, &ei);
                const double fr = f[2 * ((int64_t)j1 * N + j2)];
                const double fi = f[2 * ((int64_t)j1 * N + j2) + 1];
                sr += er * fr - ei * fi;
                si += er * fi + ei * fr;
            }
        }
        u[2 * r] = sr;
        u[2 * r + 1] = si;
    }
}

/* Adjoint: f(k) = sum_x exp(-2 pi i Phi(x,k)) u(x) at the listed source
 * indices (flat (k1+N/2)*N + (k2+N/2)), all N^2 potentials. */
void orc_direct_adjoint(int N, const orc_phase_t *ph, const double *u,
                        int ncols, const int64_t *cols, double *f)
{
    const int h = N / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < ncols; ++c) {
        const int64_t idx = cols[c];
        const double k1 = (double)(idx / N - h);
        const double k2 = (double)(idx % N - h);
        double sr = 0.0, si = 0.0;
        for (int i1 = 0; i1 < N; ++i1) {
            for (int i2 = 0; i2 < N; ++i2) {
                const double x1 = (double)i1 / N, x2 = (double)i2 / N;
                double er, ei;
                orc_cis(orc_phi(ph, x1, x2, k1, k2), &er, &ei);
                const double ur = u[2 * ((int64_t)i1 * N + i2)];
                const double ui = u[2 * ((int64_t)i1 * N + i2) + 1];
                /* conj(e) * u */
                sr += er * ur + ei * ui;
                si += er * ui - ei * ur;
            }
        }
        f[2 * c] = sr;
        f[2 * c + 1] = si;
    }
}
