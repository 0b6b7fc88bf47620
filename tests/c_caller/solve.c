/*
 * A plain C99 caller of the solver library, for the GPU test of the boundary: no Python, no
 * torch.  It reads a coefficient file (double[7][nlev][nlat][nlon], planes W, E, S, N, D, U, C)
 * and a right-hand side (double[n]), copies them to the device with the HIP runtime, solves
 * A x = b from x = 0 through eg_create_operator / eg_solve, and writes x (double[n]).
 *
 *   solve COEFFS B X_OUT NLON NLAT NLEV TOL MAXIT MODE
 *
 * Prints "status iterations outer_steps true_rel_residual" on success; exits 1 on any error.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "endgame.h"

static int read_doubles(const char *path, double *buf, long count)
{
    FILE *f = fopen(path, "rb");
    long got;
    if (!f) return -1;
    got = (long)fread(buf, sizeof(double), (size_t)count, f);
    fclose(f);
    return got == count ? 0 : -1;
}

#define HIP_OK(call)                                                                \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));              \
            return 1;                                                               \
        }                                                                           \
    } while (0)

int main(int argc, char **argv)
{
    int nlon, nlat, nlev, maxit, mode, status;
    long n;
    double tol, *hc, *hb, *hx, *dc = NULL, *db = NULL, *dx = NULL;
    eg_operator *op = NULL;
    eg_info info;
    FILE *f;
    if (argc != 10) {
        fprintf(stderr, "usage: solve COEFFS B X_OUT NLON NLAT NLEV TOL MAXIT MODE\n");
        return 1;
    }
    nlon = atoi(argv[4]);
    nlat = atoi(argv[5]);
    nlev = atoi(argv[6]);
    tol = atof(argv[7]);
    maxit = atoi(argv[8]);
    mode = atoi(argv[9]);
    if (nlon <= 0 || nlat <= 0 || nlev <= 0) {
        fprintf(stderr, "bad shape\n");
        return 1;
    }
    n = (long)nlon * nlat * nlev;
    hc = malloc(7 * n * sizeof(double));
    hb = malloc(n * sizeof(double));
    hx = calloc((size_t)n, sizeof(double));
    if (!hc || !hb || !hx) return 1;
    if (read_doubles(argv[1], hc, 7 * n) || read_doubles(argv[2], hb, n)) {
        fprintf(stderr, "cannot read the inputs\n");
        return 1;
    }
    HIP_OK(hipMalloc((void **)&dc, 7 * n * sizeof(double)));
    HIP_OK(hipMalloc((void **)&db, n * sizeof(double)));
    HIP_OK(hipMalloc((void **)&dx, n * sizeof(double)));
    HIP_OK(hipMemcpy(dc, hc, 7 * n * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(db, hb, n * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dx, hx, n * sizeof(double), hipMemcpyHostToDevice));
    if (eg_create_operator(dc, nlon, nlat, nlev, &op) < 0) {
        fprintf(stderr, "eg_create_operator: %s\n", eg_last_error());
        return 1;
    }
    HIP_OK(hipFree(dc));   /* the library keeps its own copy */
    status = eg_solve(op, db, dx, tol, maxit, mode);
    if (status < 0 || eg_get_info(op, &info) < 0) {
        fprintf(stderr, "eg_solve: %s\n", eg_last_error());
        return 1;
    }
    HIP_OK(hipMemcpy(hx, dx, n * sizeof(double), hipMemcpyDeviceToHost));
    eg_destroy_operator(op);
    HIP_OK(hipFree(db));
    HIP_OK(hipFree(dx));
    f = fopen(argv[3], "wb");
    if (!f || fwrite(hx, sizeof(double), (size_t)n, f) != (size_t)n) return 1;
    fclose(f);
    printf("%d %d %d %.17g\n", status, info.iterations, info.outer_steps, info.true_rel_residual);
    free(hc);
    free(hb);
    free(hx);
    return 0;
}
