/* Runs the FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
 * every boundary kind (periodic, halfway bounce-back with a lid, on-node walls),
 * a porosity field with Ergun K and F_phi, a free-fluid cell (K = infinity),
 * a per-node J plane, and the D2Q5 thermal coupling, on small odd-sized
 * domains, a few steps each, plus the macroscopic output and the reductions.
 * Exits 0 when every run finishes with finite outputs; the sanitizers abort
 * on any invalid access or undefined operation. Built and run by
 * tests/test_sanitize_cpu.py with gcc -fsanitize=address,undefined. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static int run_case(int nx, int ny, int bc_x, int bc_y, double lid, int thermal, int jplane)
{
    orc_params p;
    orc_default_params(&p);
    p.nx = nx; p.ny = ny; p.bc_x = bc_x; p.bc_y = bc_y; p.lid_ux = lid;
    p.nu = 0.05; p.ax = 1e-5; p.ay = -2e-6; p.nthreads = 1;
    const long n = (long)nx * ny;
    double *phi = malloc(sizeof(double) * n), *K = malloc(sizeof(double) * n),
           *F = malloc(sizeof(double) * n), *Jc = malloc(sizeof(double) * n);
    for (long k = 0; k < n; ++k) {
        phi[k] = 0.3 + 0.6 * (double)((k * 7919) % 101) / 100.0;
        Jc[k] = 1.0 + (double)(k % 3);
    }
    phi[n / 2] = 1.0;   /* a free-fluid cell: K = infinity */
    orc_ergun(n, phi, 3.0, K, F);
    if (jplane) p.Jcell = Jc;
    if (thermal) {
        p.thermal = 1; p.sigma = 1.0; p.tau_T = 0.8; p.Th = 2.0; p.Tc = 0.0; p.T0 = 1.0; p.gbeta = 1e-4;
    }
    double *f = malloc(sizeof(double) * n * 8), *g = thermal ? malloc(sizeof(double) * n * 5) : NULL;
    orc_rest_state(&p, n, 0.6, f);
    if (thermal) {
        double *T0 = malloc(sizeof(double) * n);
        for (long k = 0; k < n; ++k) T0[k] = 1.0 + 0.5 * sin(0.3 * (double)k);
        orc_thermal_rest_state(&p, n, T0, g);
        free(T0);
    }
    int rc = orc_run(&p, phi, K, F, f, g, 7);
    double *ux = malloc(sizeof(double) * n), *uy = malloc(sizeof(double) * n),
           *pr = malloc(sizeof(double) * n), *T = malloc(sizeof(double) * n);
    orc_macroscopic(&p, phi, K, F, f, g, ux, uy, pr, thermal ? T : NULL);
    double s = 0.0;
    for (long k = 0; k < 8 * n; ++k) s += f[k];
    for (long k = 0; k < n; ++k) s += ux[k] + uy[k] + pr[k] + (thermal ? T[k] : 0.0);
    free(phi); free(K); free(F); free(Jc); free(f); free(g); free(ux); free(uy); free(pr); free(T);
    if (rc != 0 || !isfinite(s)) {
        fprintf(stderr, "case %dx%d bc %d/%d thermal %d: rc %d sum %g\n", nx, ny, bc_x, bc_y, thermal, rc, s);
        return 1;
    }
    return 0;
}

int main(void)
{
    int bad = 0;
    bad += run_case(13, 9, ORC_PERIODIC, ORC_PERIODIC, 0.0, 0, 0);
    bad += run_case(11, 7, ORC_PERIODIC, ORC_WALLS, 0.05, 0, 1);
    bad += run_case(9, 10, ORC_WALLS, ORC_WALLS, 0.05, 1, 0);
    bad += run_case(8, 6, ORC_NEE, ORC_NEE, 0.05, 1, 0);
    bad += run_case(5, 12, ORC_PERIODIC, ORC_NEE, 0.02, 0, 1);
    bad += run_case(1, 3, ORC_PERIODIC, ORC_WALLS, 0.0, 0, 0);
    printf("oracle sanitizer driver: %d failing cases\n", bad);
    return bad != 0;
}
