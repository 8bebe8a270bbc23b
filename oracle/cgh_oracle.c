/*
 * FP64 CPU oracle for the direct point-source hologram sum.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * What it computes (Shimobaba et al., Section 1, Eq. (1)):
 *
 *     I(x_h, y_h) = sum_j A_j cos( P_j ((x_h - x_j)^2 + (y_h - y_j)^2) ),
 *     P_j = pi p^2 / (lambda z_j),
 *
 * with all coordinates in units of the sampling pitch p (the paper normalises
 * them by p), pixel (i, k) of an Nx x Ny hologram sitting at x_h = i,
 * y_h = k, and the hologram stored row-major (x fastest).
 *
 * The adjoint is the chain rule applied to Eq. (1).  With theta = P_j r^2,
 * d(theta)/dx_j = -2 P_j (x_h - x_j) and d(theta)/dz_j = -theta / z_j, so for
 * an upstream gradient G = dL/dI:
 *
 *     dL/dA_j = sum_h G cos(theta)
 *     dL/dx_j = 2 A_j P_j sum_h G sin(theta) (x_h - x_j)
 *     dL/dy_j = 2 A_j P_j sum_h G sin(theta) (y_h - y_j)
 *     dL/dz_j = (A_j P_j / z_j) sum_h G sin(theta) r^2
 *
 * Everything is double precision, in radians, with the C library cos/sin.
 * No blocking, no reordering: every pixel sums its points in ascending j,
 * every point sums its pixels in row-major order.  The optional threads split
 * whole rows (forward) or whole points (adjoint) between workers, so each
 * output is produced by exactly the serial instruction sequence and the
 * result is bitwise identical to the single-threaded run.
 *
 * Parity status: pinned (single point closed form, Fresnel zone radii,
 * symmetry, linearity, superposition, high-precision brute force, integer
 * translation, the separable identity, the recurrence of Eq. (2), and
 * central finite differences / dot-product tests for the adjoint).
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ENOMEM 2
#define ORACLE_ETHREAD 3

/* P_j = pi p^2 / (lambda z_j), Section 1 (definition below Eq. (1)). */
static double phase_coefficient(double pitch, double wavelength, double z) {
    return M_PI * pitch * pitch / (wavelength * z);
}

/* One hologram value, Eq. (1), summed over j in ascending order. */
static double intensity_at(const double *x, const double *y, const double *a,
                           const double *P, long n, double xh, double yh) {
    double s = 0.0;
    for (long j = 0; j < n; ++j) {
        double dx = xh - x[j];
        double dy = yh - y[j];
        s += a[j] * cos(P[j] * (dx * dx + dy * dy));
    }
    return s;
}

typedef struct {
    const double *x, *y, *z, *a, *P, *g;
    long n;
    int nx, ny;
    /* forward on the full grid */
    double *out;
    /* forward on a pixel list */
    const long *px, *py;
    long m;
    /* adjoint */
    const long *idx;
    double *gx, *gy, *gz, *ga;
    /* work split */
    int tid, nthreads;
} job_t;

static void *forward_rows(void *arg) {
    job_t *J = (job_t *)arg;
    for (int k = J->tid; k < J->ny; k += J->nthreads)
        for (int i = 0; i < J->nx; ++i)
            J->out[(long)k * J->nx + i] =
                intensity_at(J->x, J->y, J->a, J->P, J->n, (double)i, (double)k);
    return NULL;
}

static void *forward_list(void *arg) {
    job_t *J = (job_t *)arg;
    for (long t = J->tid; t < J->m; t += J->nthreads)
        J->out[t] = intensity_at(J->x, J->y, J->a, J->P, J->n, (double)J->px[t],
                                 (double)J->py[t]);
    return NULL;
}

/* The four pixel sums of the adjoint for point j, row-major pixel order. */
static void *adjoint_points(void *arg) {
    job_t *J = (job_t *)arg;
    for (long t = J->tid; t < J->m; t += J->nthreads) {
        long j = J->idx ? J->idx[t] : t;
        double Pj = J->P[j];
        double Sc = 0.0, Sx = 0.0, Sy = 0.0, Sr = 0.0;
        for (int k = 0; k < J->ny; ++k) {
            for (int i = 0; i < J->nx; ++i) {
                double G = J->g[(long)k * J->nx + i];
                double dx = (double)i - J->x[j];
                double dy = (double)k - J->y[j];
                double r2 = dx * dx + dy * dy;
                double th = Pj * r2;
                double s = sin(th);
                Sc += G * cos(th);
                Sx += G * s * dx;
                Sy += G * s * dy;
                Sr += G * s * r2;
            }
        }
        J->ga[t] = Sc;
        J->gx[t] = 2.0 * J->a[j] * Pj * Sx;
        J->gy[t] = 2.0 * J->a[j] * Pj * Sy;
        J->gz[t] = J->a[j] * Pj / J->z[j] * Sr;
    }
    return NULL;
}

static int run_threads(job_t *base, int nthreads, void *(*fn)(void *)) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads == 1) {
        base->tid = 0;
        base->nthreads = 1;
        fn(base);
        return ORACLE_OK;
    }
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    job_t *jobs = (job_t *)malloc(sizeof(job_t) * (size_t)nthreads);
    if (!th || !jobs) {
        free(th);
        free(jobs);
        return ORACLE_ENOMEM;
    }
    int started = 0, rc = ORACLE_OK;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *base;
        jobs[t].tid = t;
        jobs[t].nthreads = nthreads;
        if (pthread_create(&th[t], NULL, fn, &jobs[t]) != 0) {
            rc = ORACLE_ETHREAD;
            break;
        }
        ++started;
    }
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    if (rc != ORACLE_OK && started < nthreads) {
        /* finish the shares of the workers that never started, serially */
        for (int t = started; t < nthreads; ++t) fn(&jobs[t]);
        rc = ORACLE_OK;
    }
    free(th);
    free(jobs);
    return rc;
}

static int common_checks(const double *x, const double *y, const double *z,
                         const double *a, long n, int nx, int ny, double pitch,
                         double wavelength) {
    if (n < 0 || nx < 1 || ny < 1) return ORACLE_EINVAL;
    if (n > 0 && (!x || !y || !z || !a)) return ORACLE_EINVAL;
    if (!(pitch > 0.0) || !(wavelength > 0.0) || isinf(pitch) || isinf(wavelength))
        return ORACLE_EINVAL;
    return ORACLE_OK;
}

static double *coefficients(const double *z, long n, double pitch, double wavelength) {
    double *P = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!P) return NULL;
    for (long j = 0; j < n; ++j) P[j] = phase_coefficient(pitch, wavelength, z[j]);
    return P;
}

/* Full hologram, out[ny*nx] row-major. */
int cgh_oracle_forward(const double *x, const double *y, const double *z, const double *a,
                       long n, int nx, int ny, double pitch, double wavelength, double *out,
                       int threads) {
    int rc = common_checks(x, y, z, a, n, nx, ny, pitch, wavelength);
    if (rc) return rc;
    if (!out) return ORACLE_EINVAL;
    double *P = coefficients(z, n, pitch, wavelength);
    if (!P) return ORACLE_ENOMEM;
    job_t J = {0};
    J.x = x; J.y = y; J.z = z; J.a = a; J.P = P; J.n = n; J.nx = nx; J.ny = ny; J.out = out;
    rc = run_threads(&J, threads, forward_rows);
    free(P);
    return rc;
}

/* Hologram values at m listed pixels (px[t], py[t]); out[m]. */
int cgh_oracle_forward_at(const double *x, const double *y, const double *z, const double *a,
                          long n, int nx, int ny, double pitch, double wavelength,
                          const long *px, const long *py, long m, double *out, int threads) {
    int rc = common_checks(x, y, z, a, n, nx, ny, pitch, wavelength);
    if (rc) return rc;
    if (m < 0 || (m > 0 && (!px || !py || !out))) return ORACLE_EINVAL;
    for (long t = 0; t < m; ++t)
        if (px[t] < 0 || px[t] >= nx || py[t] < 0 || py[t] >= ny) return ORACLE_EINVAL;
    double *P = coefficients(z, n, pitch, wavelength);
    if (!P) return ORACLE_ENOMEM;
    job_t J = {0};
    J.x = x; J.y = y; J.z = z; J.a = a; J.P = P; J.n = n; J.nx = nx; J.ny = ny;
    J.px = px; J.py = py; J.m = m; J.out = out;
    rc = run_threads(&J, threads, forward_list);
    free(P);
    return rc;
}

/* Adjoint for m points (indices idx[t], or 0..m-1 when idx is NULL), given the
 * full upstream gradient g[ny*nx]; writes gx, gy, gz, ga [m]. */
int cgh_oracle_adjoint(const double *x, const double *y, const double *z, const double *a,
                       long n, int nx, int ny, double pitch, double wavelength,
                       const double *g, const long *idx, long m, double *gx, double *gy,
                       double *gz, double *ga, int threads) {
    int rc = common_checks(x, y, z, a, n, nx, ny, pitch, wavelength);
    if (rc) return rc;
    if (m < 0 || (m > 0 && (!g || !gx || !gy || !gz || !ga))) return ORACLE_EINVAL;
    if (!idx && m > n) return ORACLE_EINVAL;
    if (idx)
        for (long t = 0; t < m; ++t)
            if (idx[t] < 0 || idx[t] >= n) return ORACLE_EINVAL;
    double *P = coefficients(z, n, pitch, wavelength);
    if (!P) return ORACLE_ENOMEM;
    job_t J = {0};
    J.x = x; J.y = y; J.z = z; J.a = a; J.P = P; J.n = n; J.nx = nx; J.ny = ny;
    J.g = g; J.idx = idx; J.m = m; J.gx = gx; J.gy = gy; J.gz = gz; J.ga = ga;
    rc = run_threads(&J, threads, adjoint_points);
    free(P);
    return rc;
}
