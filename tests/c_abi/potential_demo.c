/* The C ABI used from plain C: a 2D Coulomb potential of rho = exp(-|x|^2) on a 64^2 grid of
 * [-8,8)^2 through nlf_plan_create / nlf_potential, with HIP runtime calls for device memory.
 * Writes u (64*64 doubles, row-major) to the file named by argv[1] and prints u at the origin
 * next to the closed form sqrt(pi)/2 of the continuum potential (Example 2.2, sigma = 1).
 * Exit status: 0 on success, 1 on any library or runtime error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "nlf.h"

#define N 64

static int check(int st, const char* what) {
    if (st != NLF_OK) {
        fprintf(stderr, "%s failed: %s (%s)\n", what, nlf_strerror(st), nlf_last_error());
        return 1;
    }
    return 0;
}

int main(int argc, char** argv) {
    if (argc < 2) {
        fprintf(stderr, "usage: %s output.bin\n", argv[0]);
        return 1;
    }
    static double rho[N * N], u[N * N];
    const double L = 8.0, h = 2.0 * L / N;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            const double x = -L + i * h, y = -L + j * h;
            rho[i * N + j] = exp(-(x * x + y * y));
        }
    nlf_box box = {2, {N, N, 1}, {L, L, 0.0}};
    nlf_plan* plan = NULL;
    if (check(nlf_plan_create(&box, NLF_COULOMB2D, NULL, NULL, &plan), "nlf_plan_create")) return 1;
    void *rho_dev = NULL, *u_dev = NULL;
    if (hipMalloc(&rho_dev, sizeof rho) != hipSuccess || hipMalloc(&u_dev, sizeof u) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    if (hipMemcpy(rho_dev, rho, sizeof rho, hipMemcpyHostToDevice) != hipSuccess) return 1;
    if (check(nlf_potential(plan, rho_dev, u_dev), "nlf_potential")) return 1;
    if (hipMemcpy(u, u_dev, sizeof u, hipMemcpyDeviceToHost) != hipSuccess) return 1;
    /* the origin is grid point (N/2, N/2) */
    const double u0 = u[(N / 2) * N + N / 2], want = 0.5 * sqrt(3.14159265358979323846);
    printf("u(0) = %.15f  closed form %.15f  rel err %.3e\n", u0, want, fabs(u0 - want) / want);
    FILE* f = fopen(argv[1], "wb");
    if (!f || fwrite(u, sizeof(double), N * N, f) != N * N) return 1;
    fclose(f);
    (void)hipFree(rho_dev);
    (void)hipFree(u_dev);
    return check(nlf_plan_destroy(plan), "nlf_plan_destroy");
}
