/*
 * oracle.c -- plain CPU reference of the explicit 3-D diffusion step, its halo
 * update, its adjoint and its staggered flux form, in FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant with the
 * HIP path.
 *
 * Paper: Omlin, Raess, Utkin, "Distributed Parallelization of xPU Stencil
 * Computations in Julia" (arXiv 2211.15716).  The step is the `step!` kernel
 * of Fig. 1; the halo update is `update_halo!` (Fig. 1 and Sec. 2); the global
 * grid size follows the implicit-global-grid rule of Sec. 2.
 *
 * Conventions (all functions):
 *   - arrays are dense, x fastest: A[i + nx*(j + ny*k)], 0-based indices;
 *   - "inner" points are 1..n-2 in every dimension (the `@inn` selection of
 *     Fig. 1); index 0 and n-1 are halo planes;
 *   - arithmetic follows the order written in Fig. 1, left to right, and the
 *     file is compiled with -ffp-contract=off so no multiply-add is fused.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(A, i, j, k, nx, ny) ((A)[(size_t)(i) + (size_t)(nx) * ((size_t)(j) + (size_t)(ny) * (size_t)(k))])

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Halo update of one field on a single-process grid (Fig. 1 `update_halo!`,
 * Sec. 2).  Neighbouring local grids share ol planes, so plane ol-1 is the
 * last plane of the lower neighbour and plane n-ol the first plane of the
 * upper one; with one process, a periodic dimension is its own neighbour on
 * both sides and the halo planes take plane ol-1 (last plane) and plane n-ol
 * (first plane) of the same array.  Dimensions are processed in the
 * order x, y, z and each copy moves the full plane, so edge and corner halo
 * points end up as images in every periodic dimension.  A non-periodic
 * dimension has no neighbour and is left untouched.
 *   ol[d] is the overlap of THIS field in dimension d (a field one point
 *   larger than the grid, a staggered face field, has overlap ol+1).
 */
void oracle_halo(double *A, int64_t nx, int64_t ny, int64_t nz,
                 const int ol[3], const int periods[3])
{
    if (periods[0]) {
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j) {
                AT(A, nx - 1, j, k, nx, ny) = AT(A, ol[0] - 1, j, k, nx, ny);
                AT(A, 0, j, k, nx, ny) = AT(A, nx - ol[0], j, k, nx, ny);
            }
    }
    if (periods[1]) {
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t i = 0; i < nx; ++i) {
                AT(A, i, ny - 1, k, nx, ny) = AT(A, i, ol[1] - 1, k, nx, ny);
                AT(A, i, 0, k, nx, ny) = AT(A, i, ny - ol[1], k, nx, ny);
            }
    }
    if (periods[2]) {
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                AT(A, i, j, nz - 1, nx, ny) = AT(A, i, j, ol[2] - 1, nx, ny);
                AT(A, i, j, 0, nx, ny) = AT(A, i, j, nz - ol[2], nx, ny);
            }
    }
}

/*
 * One explicit step on the inner points (Fig. 1, `step!`):
 *   T2 = T + dt*( lam*Ci*( d2x(T)/dx^2 + d2y(T)/dy^2 + d2z(T)/dz^2 ) )
 * with d2x(T) = (T[i+1]-T[i]) - (T[i]-T[i-1]), the second difference taken
 * as the difference of the two neighbouring first differences.  Halo points
 * of T2 are not written.
 */
void oracle_step(double *T2, const double *T, const double *Ci,
                 int64_t nx, int64_t ny, int64_t nz,
                 double lam, double dt, double dx, double dy, double dz)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k < nz - 1; ++k)
        for (int64_t j = 1; j < ny - 1; ++j)
            for (int64_t i = 1; i < nx - 1; ++i) {
                double c = AT(T, i, j, k, nx, ny);
                double d2x = (AT(T, i + 1, j, k, nx, ny) - c) - (c - AT(T, i - 1, j, k, nx, ny));
                double d2y = (AT(T, i, j + 1, k, nx, ny) - c) - (c - AT(T, i, j - 1, k, nx, ny));
                double d2z = (AT(T, i, j, k + 1, nx, ny) - c) - (c - AT(T, i, j, k - 1, nx, ny));
                AT(T2, i, j, k, nx, ny) =
                    c + dt * (lam * AT(Ci, i, j, k, nx, ny) *
                              (d2x / (dx * dx) + d2y / (dy * dy) + d2z / (dz * dz)));
            }
}

/* Largest value over every point of the array (Fig. 1, `maximum(Ci)`). */
double oracle_max(const double *A, int64_t n)
{
    double m = -INFINITY;
    for (int64_t p = 0; p < n; ++p)
        if (A[p] > m) m = A[p];
    return m;
}

/* Stable time step of Fig. 1: min(dx^2,dy^2,dz^2)/lam/maximum(Ci)/6.1. */
double oracle_dt(double dx, double dy, double dz, double lam, double max_ci)
{
    double m = dx * dx;
    if (dy * dy < m) m = dy * dy;
    if (dz * dz < m) m = dz * dz;
    return m / lam / max_ci / 6.1;
}

/*
 * nt steps of the Fig. 1 time loop: step, halo update of T2, swap.
 * T holds the initial state on entry and the final state on exit; W is a
 * work array of the same size whose halo and inner contents are overwritten.
 */
void oracle_run(double *T, double *W, const double *Ci,
                int64_t nx, int64_t ny, int64_t nz,
                const int ol[3], const int periods[3],
                double lam, double dt, double dx, double dy, double dz, int nt)
{
    size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
    double *cur = T, *nxt = W;
    /* the step writes inner points only: the halo of the new buffer comes
       from the halo update, and non-periodic halo planes keep the values
       they had in the initial state */
    memcpy(W, T, n * sizeof(double));
    for (int it = 0; it < nt; ++it) {
        oracle_step(nxt, cur, Ci, nx, ny, nz, lam, dt, dx, dy, dz);
        oracle_halo(nxt, nx, ny, nz, ol, periods);
        double *t = cur; cur = nxt; nxt = t;
    }
    if (cur != T) memcpy(T, cur, n * sizeof(double));
}

/*
 * Adjoint of one step with respect to the state and to Ci.
 * The step maps T_n to T_{n+1} = T_n + a*Ci.*(L T_n) on the inner points,
 * with a = dt*lam and L the symmetric second-difference operator
 * sum_d d2_d(.)/dd^2.  Its transpose applied to the incoming adjoint
 * lp = dLoss/dT_{n+1} gives
 *   lam_n = lp + a * L(Ci .* lp)
 *   gCi  += a * lp .* (L T_n)
 * on the inner points.  Ci .* lp is needed at the six neighbours too, so lp
 * and Ci must carry up-to-date halos; lam_n's halo is not written.
 */
void oracle_adjoint_step(double *lam_n, const double *lp, const double *Tn,
                         const double *Ci, double *gCi,
                         int64_t nx, int64_t ny, int64_t nz,
                         double lam, double dt, double dx, double dy, double dz)
{
    double a = dt * lam;
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k < nz - 1; ++k)
        for (int64_t j = 1; j < ny - 1; ++j)
            for (int64_t i = 1; i < nx - 1; ++i) {
#define MU(ii, jj, kk) (AT(Ci, ii, jj, kk, nx, ny) * AT(lp, ii, jj, kk, nx, ny))
                double m = MU(i, j, k);
                double mx = (MU(i + 1, j, k) - m) - (m - MU(i - 1, j, k));
                double my = (MU(i, j + 1, k) - m) - (m - MU(i, j - 1, k));
                double mz = (MU(i, j, k + 1) - m) - (m - MU(i, j, k - 1));
#undef MU
                double c = AT(Tn, i, j, k, nx, ny);
                double tx = (AT(Tn, i + 1, j, k, nx, ny) - c) - (c - AT(Tn, i - 1, j, k, nx, ny));
                double ty = (AT(Tn, i, j + 1, k, nx, ny) - c) - (c - AT(Tn, i, j - 1, k, nx, ny));
                double tz = (AT(Tn, i, j, k + 1, nx, ny) - c) - (c - AT(Tn, i, j, k - 1, nx, ny));
                double l = AT(lp, i, j, k, nx, ny);
                AT(lam_n, i, j, k, nx, ny) =
                    l + a * (mx / (dx * dx) + my / (dy * dy) + mz / (dz * dz));
                AT(gCi, i, j, k, nx, ny) +=
                    a * l * (tx / (dx * dx) + ty / (dy * dy) + tz / (dz * dz));
            }
}

/*
 * Staggered-grid flux form of the same step.  Cell-centred T and Ci have
 * (nx,ny,nz) points; the face fluxes are qx (nx+1,ny,nz), qy (nx,ny+1,nz),
 * qz (nx,ny,nz+1).  Face f of a dimension lies between cells f-1 and f, so
 *   qx[f,j,k] = -lam*(T[f,j,k]-T[f-1,j,k])/dx   for f = 1..nx-1,
 * on the inner j,k, and likewise for qy, qz.  Faces 0 and n and the
 * halo rows of the other dimensions are left to the halo update.
 */
void oracle_flux(double *qx, double *qy, double *qz, const double *T,
                 int64_t nx, int64_t ny, int64_t nz,
                 double lam, double dx, double dy, double dz)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k < nz - 1; ++k)
        for (int64_t j = 1; j < ny - 1; ++j)
            for (int64_t f = 1; f < nx; ++f)
                AT(qx, f, j, k, nx + 1, ny) =
                    -lam * (AT(T, f, j, k, nx, ny) - AT(T, f - 1, j, k, nx, ny)) / dx;
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k < nz - 1; ++k)
        for (int64_t f = 1; f < ny; ++f)
            for (int64_t i = 1; i < nx - 1; ++i)
                AT(qy, i, f, k, nx, ny + 1) =
                    -lam * (AT(T, i, f, k, nx, ny) - AT(T, i, f - 1, k, nx, ny)) / dy;
#pragma omp parallel for schedule(static)
    for (int64_t f = 1; f < nz; ++f)
        for (int64_t j = 1; j < ny - 1; ++j)
            for (int64_t i = 1; i < nx - 1; ++i)
                AT(qz, i, j, f, nx, ny) =
                    -lam * (AT(T, i, j, f, nx, ny) - AT(T, i, j, f - 1, nx, ny)) / dz;
}

/*
 * Cell update of the flux form: cell i lies between faces i and i+1, so
 *   T2 = T - dt*Ci*( (qx[i+1]-qx[i])/dx + (qy[j+1]-qy[j])/dy + (qz[k+1]-qz[k])/dz )
 * on the inner cells.
 */
void oracle_flux_update(double *T2, const double *T, const double *Ci,
                        const double *qx, const double *qy, const double *qz,
                        int64_t nx, int64_t ny, int64_t nz,
                        double dt, double dx, double dy, double dz)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k < nz - 1; ++k)
        for (int64_t j = 1; j < ny - 1; ++j)
            for (int64_t i = 1; i < nx - 1; ++i) {
                double div = (AT(qx, i + 1, j, k, nx + 1, ny) - AT(qx, i, j, k, nx + 1, ny)) / dx +
                             (AT(qy, i, j + 1, k, nx, ny + 1) - AT(qy, i, j, k, nx, ny + 1)) / dy +
                             (AT(qz, i, j, k + 1, nx, ny) - AT(qz, i, j, k, nx, ny)) / dz;
                AT(T2, i, j, k, nx, ny) = AT(T, i, j, k, nx, ny) - dt * AT(Ci, i, j, k, nx, ny) * div;
            }
}

/*
 * Adjoint of one flux-form step.  With mu = Ci .* lp (lp carrying a valid
 * halo) the transposed chain is: a face "flux" of mu, pmu = -lam*grad(mu)
 * on faces 1..n-1, then lam_n = lp - dt*div(pmu) on the inner cells.
 * The Ci gradient is gCi += -dt * lp .* div(q_n) with q_n the forward face
 * fluxes of step n (their values on faces 1..n-1 of the inner rows).
 *   pm* are work arrays of the face-field sizes.
 */
void oracle_flux_adjoint_step(double *lam_n, const double *lp, const double *Ci,
                              const double *qx, const double *qy, const double *qz,
                              double *pmx, double *pmy, double *pmz, double *gCi,
                              int64_t nx, int64_t ny, int64_t nz,
                              double lam, double dt, double dx, double dy, double dz)
{
    size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
    double *mu = (double *)malloc(n * sizeof(double));
    for (size_t p = 0; p < n; ++p) mu[p] = Ci[p] * lp[p];
    oracle_flux(pmx, pmy, pmz, mu, nx, ny, nz, lam, dx, dy, dz);
    free(mu);
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k < nz - 1; ++k)
        for (int64_t j = 1; j < ny - 1; ++j)
            for (int64_t i = 1; i < nx - 1; ++i) {
                double divp = (AT(pmx, i + 1, j, k, nx + 1, ny) - AT(pmx, i, j, k, nx + 1, ny)) / dx +
                              (AT(pmy, i, j + 1, k, nx, ny + 1) - AT(pmy, i, j, k, nx, ny + 1)) / dy +
                              (AT(pmz, i, j, k + 1, nx, ny) - AT(pmz, i, j, k, nx, ny)) / dz;
                double divq = (AT(qx, i + 1, j, k, nx + 1, ny) - AT(qx, i, j, k, nx + 1, ny)) / dx +
                              (AT(qy, i, j + 1, k, nx, ny + 1) - AT(qy, i, j, k, nx, ny + 1)) / dy +
                              (AT(qz, i, j, k + 1, nx, ny) - AT(qz, i, j, k, nx, ny)) / dz;
                double l = AT(lp, i, j, k, nx, ny);
                AT(lam_n, i, j, k, nx, ny) = l - dt * divp;
                AT(gCi, i, j, k, nx, ny) += -dt * l * divq;
            }
}
