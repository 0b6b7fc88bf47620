/*
 * Plain FP64 CPU oracle for the Helmholtz pressure-correction solve  A x = b.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it; the GPU library never links, includes or calls it, and it shares
 * no code with the GPU library.
 *
 * Paper: C. M. Maynard and D. N. Walters, "Precision of the ENDGame: Mixed-precision
 * arithmetic in the iterative solver of the Unified Model" (arXiv:1811.03852).
 *
 *   orc_apply      Sec. 2, Eq. 4 and the text after it: A is a 7-band matrix over a
 *                  lon-lat-height grid (Laplacian-like, non-symmetric, variable coefficient).
 *                  Written as the plain row definition  y = C x - sum_nb a_nb x_nb.
 *   orc_thomas     Sec. 2, Eq. 6-7 and the text after them: T is the vertical tridiagonal
 *                  part of A, inverted per horizontal point with no vertical decomposition.
 *                  Plain LU (Thomas) without pivoting.
 *   orc_rbsor      Sec. 2, Eq. 6-7: the tri_sor preconditioner (a few over-relaxed sweeps of
 *                  vertical-line Gauss-Seidel in which T takes the place of the diagonal),
 *                  with the columns visited in red-black order instead of lexicographically.
 *   orc_lexsor     the same sweeps in the natural (lexicographic) column order of Eq. 7's L, U.
 *   orc_bicgstab   Sec. 2 (post-conditioned BiCGStab, Eq. 5; van der Vorst's method with the
 *                  preconditioner applied on the right) and Sec. 3 (halting on
 *                  R = ||r_i|| / ||b|| of the unpreconditioned residual, Eq. 8-9), with the
 *                  breakdown guard and the optional fixed-interval restart of Sec. 4.
 *
 * Conventions (shared with the GPU library as a *specification*, not as code):
 *   coef[7][nlev][nlat][nlon], direction order W, E, S, N, D, U, C, lon fastest,
 *   idx = i + nlon*(j + nlat*k).  W/E couple to i-1 / i+1 (periodic), S/N to j-1 / j+1,
 *   D/U to k-1 / k+1.  Couplings are magnitudes (entries of A are -coef[d]); C is the
 *   diagonal.  Couplings across the poles, the bottom and the top must be zero; the oracle
 *   simply omits those neighbours.
 *
 * Floating point: FP64 throughout, sums left to right, built with -ffp-contract=off.
 * Parity status: every function here is pinned by tests (closed-form eigenpairs, symmetry of
 * the finite-volume operator, dense LU, banded LAPACK solve, manufactured solutions and
 * special cases that terminate at the first half step).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Multi-threaded build (-fopenmp -DORC_OPENMP, liboracle_omp.so): the same arithmetic with the
 * grid loops shared among threads.  Every loop writes disjoint elements, so each result is
 * bitwise the single-threaded one, except the inner products, which add the partial sums of a
 * fixed partition into ORC_DOT_BLOCKS contiguous blocks (each left to right, then the block
 * sums left to right): deterministic for any thread count, but summed in another order than
 * the single-threaded build. */
#ifdef ORC_OPENMP
#include <omp.h>
#define ORC_PARFOR _Pragma("omp parallel for schedule(static)")
#define ORC_PARFOR2 _Pragma("omp parallel for collapse(2) schedule(static)")
#define ORC_PARALLEL _Pragma("omp parallel")
#define ORC_FOR _Pragma("omp for schedule(static)")
#else
#define ORC_PARFOR
#define ORC_PARFOR2
#define ORC_PARALLEL
#define ORC_FOR
#endif
#define ORC_DOT_BLOCKS 256

#define ORC_W 0
#define ORC_E 1
#define ORC_S 2
#define ORC_N 3
#define ORC_D 4
#define ORC_U 5
#define ORC_C 6

typedef struct {
    int iterations;          /* iterations performed; an exit at the half step counts as one */
    int restarts;            /* breakdown, periodic and residual-gap restarts                 */
    int status;              /* 0 converged, 1 iteration limit, 3 stalled above tol           */
    int half_step_exit;      /* 1 if the final exit happened at the half step                 */
    double rel_residual;     /* recursive ||r|| / ||b|| at exit                               */
    double true_rel_residual;/* ||b - A x|| / ||b|| at exit                                   */
    int sigma_restarts;      /* restarts taken because <rhat, v> was near zero                 */
    int rho_restarts;        /* restarts taken because <rhat, r> was near zero                 */
} orc_info;

/* y = A x, plain row definition (Sec. 2: 7-band operator). */
void orc_apply(int nlon, int nlat, int nlev, const double *coef, const double *x, double *y)
{
    const long P = (long)nlon * nlat;
    const long n = P * nlev;
    const double *aW = coef + ORC_W * n, *aE = coef + ORC_E * n, *aS = coef + ORC_S * n;
    const double *aN = coef + ORC_N * n, *aD = coef + ORC_D * n, *aU = coef + ORC_U * n;
    const double *C = coef + ORC_C * n;
    ORC_PARFOR2
    for (int k = 0; k < nlev; ++k)
        for (int j = 0; j < nlat; ++j)
            for (int i = 0; i < nlon; ++i) {
                long c = i + (long)nlon * (j + (long)nlat * k);
                int iw = (i == 0) ? nlon - 1 : i - 1;
                int ie = (i == nlon - 1) ? 0 : i + 1;
                double acc = C[c] * x[c];
                acc = acc - aW[c] * x[iw + (long)nlon * (j + (long)nlat * k)];
                acc = acc - aE[c] * x[ie + (long)nlon * (j + (long)nlat * k)];
                if (j > 0) acc = acc - aS[c] * x[c - nlon];
                if (j < nlat - 1) acc = acc - aN[c] * x[c + nlon];
                if (k > 0) acc = acc - aD[c] * x[c - P];
                if (k < nlev - 1) acc = acc - aU[c] * x[c + P];
                y[c] = acc;
            }
}

/* (A x)[idx[p]] for a sample of points (the same definition, one row at a time). */
void orc_apply_points(int nlon, int nlat, int nlev, const double *coef, const double *x,
                      const long *idx, long npts, double *y)
{
    const long P = (long)nlon * nlat;
    const long n = P * nlev;
    for (long p = 0; p < npts; ++p) {
        long c = idx[p];
        int i = (int)(c % nlon);
        int j = (int)((c / nlon) % nlat);
        int k = (int)(c / P);
        int iw = (i == 0) ? nlon - 1 : i - 1;
        int ie = (i == nlon - 1) ? 0 : i + 1;
        double acc = coef[ORC_C * n + c] * x[c];
        acc = acc - coef[ORC_W * n + c] * x[c - i + iw];
        acc = acc - coef[ORC_E * n + c] * x[c - i + ie];
        if (j > 0) acc = acc - coef[ORC_S * n + c] * x[c - nlon];
        if (j < nlat - 1) acc = acc - coef[ORC_N * n + c] * x[c + nlon];
        if (k > 0) acc = acc - coef[ORC_D * n + c] * x[c - P];
        if (k < nlev - 1) acc = acc - coef[ORC_U * n + c] * x[c + P];
        y[p] = acc;
    }
}

/*
 * z = T^{-1} q per column, T = tridiag(-aD, C, -aU) (Sec. 2, the tridiagonal T of Eq. 6 that
 * replaces the diagonal in Eq. 7; its LU factors per horizontal point).  T keeps the full
 * diagonal C of A.  Textbook Thomas recurrences, no pivoting (T is strictly diagonally
 * dominant because every row of A is).
 */
void orc_thomas(int nlon, int nlat, int nlev, const double *coef, const double *q, double *z)
{
    const long P = (long)nlon * nlat;
    const long n = P * nlev;
    const double *aD = coef + ORC_D * n, *aU = coef + ORC_U * n, *C = coef + ORC_C * n;
#ifdef ORC_OPENMP
    /* the same recurrences for blocks of ORC_TB adjacent columns at a time, level by level,
     * so that each level of a block is one contiguous run of memory */
#define ORC_TB 64
#pragma omp parallel
    {
        double *cp = (double *)malloc(sizeof(double) * (size_t)nlev * ORC_TB);
        double *yy = (double *)malloc(sizeof(double) * (size_t)nlev * ORC_TB);
#pragma omp for schedule(static)
        for (long c0 = 0; c0 < P; c0 += ORC_TB) {
            const int nb = (int)(P - c0 < ORC_TB ? P - c0 : ORC_TB);
            for (int m = 0; m < nb; ++m) {
                const long col = c0 + m;
                cp[m] = -aU[col] / C[col];
                yy[m] = q[col] / C[col];
            }
            for (int k = 1; k < nlev; ++k)
                for (int m = 0; m < nb; ++m) {
                    const long c = c0 + m + k * P;
                    const double den = C[c] - (-aD[c]) * cp[(k - 1) * ORC_TB + m];
                    cp[k * ORC_TB + m] = -aU[c] / den;
                    yy[k * ORC_TB + m] = (q[c] - (-aD[c]) * yy[(k - 1) * ORC_TB + m]) / den;
                }
            for (int m = 0; m < nb; ++m) z[c0 + m + (long)(nlev - 1) * P] = yy[(nlev - 1) * ORC_TB + m];
            for (int k = nlev - 2; k >= 0; --k)
                for (int m = 0; m < nb; ++m)
                    z[c0 + m + k * P] = yy[k * ORC_TB + m] - cp[k * ORC_TB + m] * z[c0 + m + (k + 1) * P];
        }
        free(cp);
        free(yy);
    }
    return;
#endif
    ORC_PARALLEL
    {
        double *cp = (double *)malloc(sizeof(double) * (size_t)nlev);
        double *yy = (double *)malloc(sizeof(double) * (size_t)nlev);
        ORC_FOR
        for (long col = 0; col < P; ++col) {
            /* forward elimination: T = L U with unit-upper U having superdiagonal cp */
            cp[0] = -aU[col] / C[col];
            yy[0] = q[col] / C[col];
            for (int k = 1; k < nlev; ++k) {
                long c = col + k * P;
                double den = C[c] - (-aD[c]) * cp[k - 1];
                cp[k] = -aU[c] / den;
                yy[k] = (q[c] - (-aD[c]) * yy[k - 1]) / den;
            }
            /* back substitution */
            z[col + (long)(nlev - 1) * P] = yy[nlev - 1];
            for (int k = nlev - 2; k >= 0; --k)
                z[col + k * P] = yy[k] - cp[k] * z[col + (k + 1) * P];
        }
        free(cp);
        free(yy);
    }
}

/*
 * Red-black vertical-line SOR (Sec. 2, Eq. 6-7).  The paper writes the scaled operator as
 * T + L + U (T the vertical tridiagonal part, L and U the couplings to columns visited before
 * and after a column) and applies a few sweeps of
 *     (T + omega L) x_n = (1 - omega) T x_{n-1} + omega (r - U x_{n-1}),   x_0 = 0.
 * Solved column by column this is: x_c <- (1 - omega) x_c + omega T_c^{-1} (r_c + sum of the
 * horizontal couplings times the newest neighbour values).  Here the columns are visited in
 * red-black order (red: i + j even, then black), so "before" means "of the other colour and
 * already updated in this sweep".  Within one colour all columns use the values at the start
 * of the half-sweep (with even nlon no column has a neighbour of its own colour).
 * nhalf = number of half-sweeps (two per sweep: red, then black).  z receives x.
 */
void orc_rbsor(int nlon, int nlat, int nlev, const double *coef, const double *q, double *z, int nhalf,
               double omega)
{
    const long P = (long)nlon * nlat;
    const long n = P * nlev;
    const double *aW = coef + ORC_W * n, *aE = coef + ORC_E * n, *aS = coef + ORC_S * n, *aN = coef + ORC_N * n;
    const double *aD = coef + ORC_D * n, *aU = coef + ORC_U * n, *C = coef + ORC_C * n;
    double *old = (double *)malloc(sizeof(double) * (size_t)n);
    double *rhs = (double *)malloc(sizeof(double) * (size_t)nlev);
    double *cp = (double *)malloc(sizeof(double) * (size_t)nlev);
    double *yy = (double *)malloc(sizeof(double) * (size_t)nlev);
    double *col = (double *)malloc(sizeof(double) * (size_t)nlev);
    for (long c = 0; c < n; ++c) z[c] = 0.0;
    for (int h = 0; h < nhalf; ++h) {
        const int colour = h % 2;
        memcpy(old, z, sizeof(double) * (size_t)n);
        for (int j = 0; j < nlat; ++j)
            for (int i = 0; i < nlon; ++i) {
                if ((i + j) % 2 != colour) continue;
                const int iw = (i == 0) ? nlon - 1 : i - 1;
                const int ie = (i == nlon - 1) ? 0 : i + 1;
                for (int k = 0; k < nlev; ++k) {
                    const long c = i + (long)nlon * (j + (long)nlat * k);
                    double acc = q[c];
                    acc = acc + aW[c] * old[c - i + iw];
                    acc = acc + aE[c] * old[c - i + ie];
                    if (j > 0) acc = acc + aS[c] * old[c - nlon];
                    if (j < nlat - 1) acc = acc + aN[c] * old[c + nlon];
                    rhs[k] = acc;
                }
                /* T_c y = rhs, plain Thomas as in orc_thomas */
                const long c0 = i + (long)nlon * j;
                cp[0] = -aU[c0] / C[c0];
                yy[0] = rhs[0] / C[c0];
                for (int k = 1; k < nlev; ++k) {
                    const long c = c0 + k * P;
                    const double den = C[c] - (-aD[c]) * cp[k - 1];
                    cp[k] = -aU[c] / den;
                    yy[k] = (rhs[k] - (-aD[c]) * yy[k - 1]) / den;
                }
                col[nlev - 1] = yy[nlev - 1];
                for (int k = nlev - 2; k >= 0; --k) col[k] = yy[k] - cp[k] * col[k + 1];
                for (int k = 0; k < nlev; ++k) {
                    const long c = c0 + k * P;
                    z[c] = (1.0 - omega) * old[c] + omega * col[k];
                }
            }
    }
    free(old);
    free(rhs);
    free(cp);
    free(yy);
    free(col);
}

/*
 * The same SOR in the natural column order of the splitting A = L + T + U of Sec. 2, Eq. 7
 * (L, U the lower and upper triangles with i fastest, then j): columns visited in that order,
 * each using the newest values of all its neighbours (x_c <- (1 - omega) x_c + omega
 * T_c^{-1}(q_c + sum_nb a_nb x_nb)); nsweeps sweeps from x = 0.  Kept for comparing the
 * orderings; the GPU builds the red-black one.
 */
void orc_lexsor(int nlon, int nlat, int nlev, const double *coef, const double *q, double *z, int nsweeps,
                double omega)
{
    const long P = (long)nlon * nlat;
    const long n = P * nlev;
    const double *aW = coef + ORC_W * n, *aE = coef + ORC_E * n, *aS = coef + ORC_S * n, *aN = coef + ORC_N * n;
    const double *aD = coef + ORC_D * n, *aU = coef + ORC_U * n, *C = coef + ORC_C * n;
    double *rhs = (double *)malloc(sizeof(double) * (size_t)nlev);
    double *cp = (double *)malloc(sizeof(double) * (size_t)nlev);
    double *yy = (double *)malloc(sizeof(double) * (size_t)nlev);
    for (long c = 0; c < n; ++c) z[c] = 0.0;
    for (int sw = 0; sw < nsweeps; ++sw)
        for (int j = 0; j < nlat; ++j)
            for (int i = 0; i < nlon; ++i) {
                const int iw = (i == 0) ? nlon - 1 : i - 1;
                const int ie = (i == nlon - 1) ? 0 : i + 1;
                for (int k = 0; k < nlev; ++k) {
                    const long c = i + (long)nlon * (j + (long)nlat * k);
                    double acc = q[c];
                    acc = acc + aW[c] * z[c - i + iw];
                    acc = acc + aE[c] * z[c - i + ie];
                    if (j > 0) acc = acc + aS[c] * z[c - nlon];
                    if (j < nlat - 1) acc = acc + aN[c] * z[c + nlon];
                    rhs[k] = acc;
                }
                const long c0 = i + (long)nlon * j;
                cp[0] = -aU[c0] / C[c0];
                yy[0] = rhs[0] / C[c0];
                for (int k = 1; k < nlev; ++k) {
                    const long c = c0 + k * P;
                    const double den = C[c] - (-aD[c]) * cp[k - 1];
                    cp[k] = -aU[c] / den;
                    yy[k] = (rhs[k] - (-aD[c]) * yy[k - 1]) / den;
                }
                double znext = yy[nlev - 1];
                z[c0 + (long)(nlev - 1) * P] = (1.0 - omega) * z[c0 + (long)(nlev - 1) * P] + omega * znext;
                for (int k = nlev - 2; k >= 0; --k) {
                    const double y = yy[k] - cp[k] * znext;
                    const long c = c0 + k * P;
                    z[c] = (1.0 - omega) * z[c] + omega * y;
                    znext = y;
                }
            }
    free(rhs);
    free(cp);
    free(yy);
}

double orc_dot(long n, const double *a, const double *b)
{
#ifdef ORC_OPENMP
    double part[ORC_DOT_BLOCKS];
    ORC_PARFOR
    for (int blk = 0; blk < ORC_DOT_BLOCKS; ++blk) {
        const long lo = n * blk / ORC_DOT_BLOCKS, hi = n * (blk + 1) / ORC_DOT_BLOCKS;
        double s = 0.0;
        for (long i = lo; i < hi; ++i) s = s + a[i] * b[i];
        part[blk] = s;
    }
    double s = 0.0;
    for (int blk = 0; blk < ORC_DOT_BLOCKS; ++blk) s = s + part[blk];
    return s;
#else
    double s = 0.0;
    for (long i = 0; i < n; ++i) s = s + a[i] * b[i];
    return s;
#endif
}

static double nrm2(long n, const double *a) { return sqrt(orc_dot(n, a, a)); }

/* Breakdown threshold of BiCGStab (relative cosine), 2^-52 unless a test sets another to force
 * the restart paths. */
static double g_eps_bd = 2.220446049250313e-16;
void orc_set_eps_bd(double eps) { g_eps_bd = eps; }

/* preconditioner choice of orc_bicgstab: 0 = identity, 1 = vertical tridiagonal (T^{-1}),
 * 2 = red-black line SOR (orc_rbsor), 3 = lexicographic line SOR (orc_lexsor), both with
 * sor_sweeps sweeps and relaxation sor_omega (orc_bicgstab_sor) */
static int g_sor_sweeps = 3;
static double g_sor_omega = 1.5;

static void apply_m(int precond, int nlon, int nlat, int nlev, const double *coef,
                    const double *q, double *z, long n)
{
    if (precond == 1)
        orc_thomas(nlon, nlat, nlev, coef, q, z);
    else if (precond == 2)
        orc_rbsor(nlon, nlat, nlev, coef, q, z, 2 * g_sor_sweeps, g_sor_omega);
    else if (precond == 3)
        orc_lexsor(nlon, nlat, nlev, coef, q, z, g_sor_sweeps, g_sor_omega);
    else
        memcpy(z, q, sizeof(double) * (size_t)n);
}

/*
 * Right-preconditioned BiCGStab (Sec. 2, Eq. 5: the solver iterates on A M y = b with x = M y,
 * so the residual it tracks is the unpreconditioned b - A x that the halting test of Sec. 3,
 * Eq. 8-9, measures).  Steps of one iteration, in van der Vorst's notation:
 *
 *   rho = <rhat, r>; beta = (rho / rho_prev) (alpha / omega); p = r + beta (p - omega v)
 *   phat = M p; v = A phat; alpha = rho / <rhat, v>; s = r - alpha v
 *   (stop here with x += alpha phat if ||s|| / ||b|| <= tol)
 *   shat = M s; t = A shat; omega = <t, s> / <t, t>
 *   x += alpha phat + omega shat; r = s - omega t
 *
 * Guards (Sec. 4: near-zero scalar weights break the iteration; a mandatory restart after a
 * fixed number of iterations restores the Krylov basis):
 *   |rho| or |<rhat, v>| below eps_bd times the product of the norms -> restart with rhat = r;
 *   <t, t> = 0 or omega = 0 -> take the half step, then restart;
 *   restart_every > 0 -> every restart_every iterations recompute r = b - A x and restart;
 *   on exit the true residual is checked; if it exceeds tol the iteration restarts from the
 *   current x (at most 3 times, then status 3: the true residual is stuck above tol).
 *
 * x holds the initial guess on entry and the solution on exit.  hist (may be NULL) receives
 * the recursive ||r|| / ||b|| after each iteration.  Returns info->status.
 */
int orc_bicgstab(int nlon, int nlat, int nlev, const double *coef, const double *b, double *x,
                 double tol, int maxit, int restart_every, int precond, double *hist,
                 int hist_cap, orc_info *info)
{
    const long n = (long)nlon * nlat * nlev;
    const double eps_bd = g_eps_bd;
    orc_info loc;
    if (!info) info = &loc;
    memset(info, 0, sizeof(*info));
    int it = 0;

    double *r = (double *)calloc((size_t)n, sizeof(double));
    double *rh = (double *)calloc((size_t)n, sizeof(double));
    double *p = (double *)calloc((size_t)n, sizeof(double));
    double *ph = (double *)calloc((size_t)n, sizeof(double));
    double *v = (double *)calloc((size_t)n, sizeof(double));
    double *s = (double *)calloc((size_t)n, sizeof(double));
    double *sh = (double *)calloc((size_t)n, sizeof(double));
    double *t = (double *)calloc((size_t)n, sizeof(double));

    double nb = nrm2(n, b);
    if (nb == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        info->status = 0;
        goto done;
    }

    /* r = b - A x */
    orc_apply(nlon, nlat, nlev, coef, x, r);
    ORC_PARFOR
    for (long i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double rnorm = nrm2(n, r);
    info->rel_residual = rnorm / nb;
    info->true_rel_residual = rnorm / nb;
    if (rnorm / nb <= tol) {
        info->status = 0;
        goto done;
    }

    int gap_restarts = 0;
    int fresh = 1; /* 1: (re)start state — rhat = r, p = v = 0, scalars = 1 */
    double rho_prev = 1.0, alpha = 1.0, omega = 1.0, rhnorm = 0.0;
    info->status = 1;
    while (it < maxit) {
        if (fresh) {
            memcpy(rh, r, sizeof(double) * (size_t)n);
            memset(p, 0, sizeof(double) * (size_t)n);
            memset(v, 0, sizeof(double) * (size_t)n);
            rho_prev = alpha = omega = 1.0;
            rhnorm = nrm2(n, rh);
            fresh = 0;
        }
        ++it;
        double rho = orc_dot(n, rh, r);
        if (fabs(rho) <= eps_bd * rhnorm * rnorm) {
            /* rhat has become orthogonal to r: restart the shadow space */
            memcpy(rh, r, sizeof(double) * (size_t)n);
            memset(p, 0, sizeof(double) * (size_t)n);
            memset(v, 0, sizeof(double) * (size_t)n);
            rho_prev = alpha = omega = 1.0;
            rhnorm = rnorm;
            rho = orc_dot(n, rh, r);
            info->restarts++;
            info->rho_restarts++;
        }
        double beta = (rho / rho_prev) * (alpha / omega);
        ORC_PARFOR
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        apply_m(precond, nlon, nlat, nlev, coef, p, ph, n);
        orc_apply(nlon, nlat, nlev, coef, ph, v);
        double sigma = orc_dot(n, rh, v);
        if (fabs(sigma) <= eps_bd * rhnorm * nrm2(n, v)) {
            info->restarts++;
            info->sigma_restarts++;
            fresh = 1;
            if (hist && it <= hist_cap) hist[it - 1] = rnorm / nb;
            continue;
        }
        alpha = rho / sigma;
        ORC_PARFOR
        for (long i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        double snorm = nrm2(n, s);
        if (snorm / nb <= tol) {
            ORC_PARFOR
            for (long i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i];
            info->rel_residual = snorm / nb;
            if (hist && it <= hist_cap) hist[it - 1] = snorm / nb;
            info->half_step_exit = 1;
            info->status = 0;
        } else {
            apply_m(precond, nlon, nlat, nlev, coef, s, sh, n);
            orc_apply(nlon, nlat, nlev, coef, sh, t);
            double tt = orc_dot(n, t, t);
            double ts = orc_dot(n, t, s);
            if (tt == 0.0 || ts == 0.0) {
                /* omega would be zero or undefined: keep the half step and restart */
                ORC_PARFOR
                for (long i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i];
                memcpy(r, s, sizeof(double) * (size_t)n);
                rnorm = snorm;
                info->restarts++;
                fresh = 1;
                if (hist && it <= hist_cap) hist[it - 1] = rnorm / nb;
                continue;
            }
            omega = ts / tt;
            ORC_PARFOR
            for (long i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i] + omega * sh[i];
            ORC_PARFOR
            for (long i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
            rho_prev = rho;
            rnorm = nrm2(n, r);
            info->rel_residual = rnorm / nb;
            if (hist && it <= hist_cap) hist[it - 1] = rnorm / nb;
            info->half_step_exit = 0;
            if (rnorm / nb <= tol) info->status = 0;
        }
        if (info->status == 0) {
            /* residual-gap check on the true residual */
            orc_apply(nlon, nlat, nlev, coef, x, t);
            ORC_PARFOR
            for (long i = 0; i < n; ++i) r[i] = b[i] - t[i];
            rnorm = nrm2(n, r);
            info->true_rel_residual = rnorm / nb;
            if (rnorm / nb <= tol) goto done;
            if (gap_restarts >= 3) {
                /* the true residual cannot be driven below tol (attainable-accuracy floor) */
                info->status = 3;
                goto done;
            }
            gap_restarts++;
            info->restarts++;
            info->status = 1;
            fresh = 1;
            continue;
        }
        if (restart_every > 0 && it % restart_every == 0) {
            orc_apply(nlon, nlat, nlev, coef, x, t);
            ORC_PARFOR
            for (long i = 0; i < n; ++i) r[i] = b[i] - t[i];
            rnorm = nrm2(n, r);
            info->restarts++;
            fresh = 1;
        }
    }
    if (info->status != 0) {
        /* iteration limit: report the true residual of the returned x */
        orc_apply(nlon, nlat, nlev, coef, x, t);
        ORC_PARFOR
        for (long i = 0; i < n; ++i) r[i] = b[i] - t[i];
        info->true_rel_residual = nrm2(n, r) / nb;
    }
done:
    info->iterations = it;
    free(r); free(rh); free(p); free(ph); free(v); free(s); free(sh); free(t);
    return info->status;
}

/* orc_bicgstab with a line-SOR preconditioner (precond 2 red-black, 3 lexicographic) and its
 * parameters. */
int orc_bicgstab_sor(int nlon, int nlat, int nlev, const double *coef, const double *b, double *x,
                     double tol, int maxit, int restart_every, int precond, int sweeps, double omega,
                     double *hist, int hist_cap, orc_info *info)
{
    g_sor_sweeps = sweeps;
    g_sor_omega = omega;
    const int st = orc_bicgstab(nlon, nlat, nlev, coef, b, x, tol, maxit, restart_every, precond, hist, hist_cap,
                                info);
    g_sor_sweeps = 3;
    g_sor_omega = 1.5;
    return st;
}
