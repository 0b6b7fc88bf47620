/* Driver for the sanitizer test of the oracle: builds a small diagonally dominant 7-point
 * operator with its own tiny generator (no solver arithmetic), then calls every oracle routine
 * on odd-sized grids (ragged in every direction, one-level and one-row cases included).  Built
 * with AddressSanitizer and UndefinedBehaviorSanitizer; any out-of-bounds access, leak or
 * undefined operation makes the run fail.  Test code only. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int iterations, restarts, status, half_step_exit;
    double rel_residual, true_rel_residual;
    int sigma_restarts, rho_restarts;
} orc_info;

void orc_apply(int, int, int, const double *, const double *, double *);
void orc_apply_points(int, int, int, const double *, const double *, const long *, long, double *);
void orc_thomas(int, int, int, const double *, const double *, double *);
void orc_rbsor(int, int, int, const double *, const double *, double *, int, double);
void orc_lexsor(int, int, int, const double *, const double *, double *, int, double);
double orc_dot(long, const double *, const double *);
void orc_set_eps_bd(double);
int orc_bicgstab(int, int, int, const double *, const double *, double *, double, int, int, int, double *, int,
                 orc_info *);
int orc_bicgstab_sor(int, int, int, const double *, const double *, double *, double, int, int, int, int, double,
                     double *, int, orc_info *);

static unsigned long long st = 12345;
static double unif(void)
{
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(st >> 11) / 9007199254740992.0;
}

static int run(int nlon, int nlat, int nlev)
{
    const long P = (long)nlon * nlat, n = P * nlev;
    double *coef = calloc(7 * (size_t)n, sizeof(double));
    double *b = malloc(sizeof(double) * (size_t)n), *x = calloc((size_t)n, sizeof(double));
    double *y = malloc(sizeof(double) * (size_t)n), *hist = malloc(sizeof(double) * 64);
    long *idx = malloc(sizeof(long) * 5);
    for (int k = 0; k < nlev; ++k)
        for (int j = 0; j < nlat; ++j)
            for (int i = 0; i < nlon; ++i) {
                const long c = i + nlon * ((long)j + (long)nlat * k);
                double s = 0.0;
                for (int d = 0; d < 6; ++d) {
                    double a = 0.1 + unif();
                    if ((d == 2 && j == 0) || (d == 3 && j == nlat - 1) || (d == 4 && k == 0) || (d == 5 && k == nlev - 1))
                        a = 0.0;
                    coef[d * n + c] = a;
                    s += a;
                }
                coef[6 * n + c] = s + 1e-2;
                b[c] = unif() - 0.5;
            }
    orc_apply(nlon, nlat, nlev, coef, b, y);
    for (int p = 0; p < 5; ++p) idx[p] = (p * 7919L) % n;
    orc_apply_points(nlon, nlat, nlev, coef, b, idx, 5, y);
    orc_thomas(nlon, nlat, nlev, coef, b, y);
    if (nlon % 2 == 0) orc_rbsor(nlon, nlat, nlev, coef, b, y, 5, 1.5);
    orc_lexsor(nlon, nlat, nlev, coef, b, y, 2, 1.5);
    double d = orc_dot(n, b, y);
    orc_info info;
    int bad = 0;
    for (int pc = 0; pc <= 1; ++pc) {
        for (long c = 0; c < n; ++c) x[c] = 0.0;
        orc_bicgstab(nlon, nlat, nlev, coef, b, x, 1e-10, 500, 7, pc, hist, 64, &info);
        bad |= info.status != 0;
    }
    orc_set_eps_bd(1e-2);
    for (long c = 0; c < n; ++c) x[c] = 0.0;
    orc_bicgstab(nlon, nlat, nlev, coef, b, x, 1e-10, 500, 0, 1, hist, 64, &info);
    orc_set_eps_bd(2.220446049250313e-16);
    bad |= info.status != 0;
    if (nlon % 2 == 0) {
        for (long c = 0; c < n; ++c) x[c] = 0.0;
        orc_bicgstab_sor(nlon, nlat, nlev, coef, b, x, 1e-10, 500, 0, 2, 2, 1.2, hist, 64, &info);
        bad |= info.status != 0;
    }
    for (long c = 0; c < n; ++c) x[c] = 0.0;
    orc_bicgstab_sor(nlon, nlat, nlev, coef, b, x, 1e-10, 500, 0, 3, 2, 1.2, hist, 64, &info);
    bad |= info.status != 0;
    printf("%dx%dx%d: dot %.6f, last solve %d iterations, status %d\n", nlon, nlat, nlev, d, info.iterations,
           info.status);
    free(coef); free(b); free(x); free(y); free(hist); free(idx);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= run(7, 5, 3);
    bad |= run(6, 1, 4);
    bad |= run(10, 3, 1);
    bad |= run(3, 2, 9);
    return bad;
}
