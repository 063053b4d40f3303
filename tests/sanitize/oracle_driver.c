/* Exercises every entry point of the C oracle on small random sets (brute
 * force and tree searches, all targets and a subset, degenerate boxes of one
 * to three particles), for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Exits 0 when every call returns 0; the
 * sanitizers abort on the first invalid access or undefined operation. */
#include "../../oracle/crk_oracle.c"

#include <stdio.h>
#include <stdlib.h>

static double urand(unsigned long long *s) {
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0;
}

static int run(int64_t ng, int64_t nd, unsigned long long seed, int brute) {
    const int64_t n = ng + nd;
    double *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n),
           *z = malloc(sizeof(double) * n), *m = malloc(sizeof(double) * n);
    double *h = malloc(sizeof(double) * (ng ? ng : 1));
    double *v[3], *u = malloc(sizeof(double) * (ng ? ng : 1));
    for (int a = 0; a < 3; ++a) v[a] = malloc(sizeof(double) * (ng ? ng : 1));
    for (int64_t i = 0; i < n; ++i) {
        x[i] = 1.0 + urand(&seed);
        y[i] = 1.0 + urand(&seed);
        z[i] = 1.0 + urand(&seed);
        m[i] = (0.5 + urand(&seed)) / (double)n;
    }
    for (int64_t i = 0; i < ng; ++i) {
        h[i] = 0.06 + 0.02 * urand(&seed);
        u[i] = 1.0 + 0.1 * urand(&seed);
        for (int a = 0; a < 3; ++a) v[a][i] = 0.1 * (urand(&seed) - 0.5);
    }
    /* (at least 3: the subset calls below write three targets) */
    const int64_t g1 = ng > 3 ? ng : 3;
    const int64_t n1 = n > 3 ? n : 3;
    double *V = calloc(g1, sizeof(double)), *rt = calloc(g1, sizeof(double));
    double *A = calloc(g1, sizeof(double)), *B = calloc(3 * g1, sizeof(double));
    double *gA = calloc(3 * g1, sizeof(double)), *gB = calloc(9 * g1, sizeof(double));
    double *rho = calloc(g1, sizeof(double)), *P = calloc(g1, sizeof(double));
    double *cs = calloc(g1, sizeof(double)), *dv = calloc(9 * g1, sizeof(double));
    double *ax = calloc(n1, sizeof(double)), *ay = calloc(n1, sizeof(double));
    double *az = calloc(n1, sizeof(double)), *du = calloc(g1, sizeof(double));
    int *deg = calloc(g1, sizeof(int));
    int64_t *counts = calloc(g1, sizeof(int64_t)), *off = calloc(g1 + 1, sizeof(int64_t));
    int64_t sub[3] = {0, ng > 1 ? ng - 1 : 0, ng / 2};
    int rc = 0;
    if (ng) {
        for (int mode = 0; mode < 2; ++mode) {
            rc |= orc_neighbours(ng, x, y, z, h, mode, ng, NULL, brute, counts, NULL, NULL);
            for (int64_t i = 0; i < ng; ++i) off[i + 1] = off[i] + counts[i];
            int64_t *idx = malloc(sizeof(int64_t) * (off[ng] ? off[ng] : 1));
            rc |= orc_neighbours(ng, x, y, z, h, mode, ng, NULL, brute, counts, off, idx);
            free(idx);
        }
        rc |= orc_density(ng, x, y, z, h, m, ng, NULL, brute, V, rt);
        rc |= orc_coefficients(ng, x, y, z, h, m, V, u, 5.0 / 3.0, ng, NULL, brute,
                               A, B, gA, gB, rho, P, cs, deg);
        rc |= orc_velocity_gradient(ng, x, y, z, v[0], v[1], v[2], h, V, A, B, gA, gB,
                                    ng, NULL, brute, dv);
        rc |= orc_hydro(ng, x, y, z, v[0], v[1], v[2], h, m, V, rho, P, cs, A, B, gA, gB,
                        1.0, 2.0, 0.01, NULL, 0.8, 0.2, NULL, NULL, NULL, ng, NULL,
                        brute, ax, ay, az, du);
        rc |= orc_hydro(ng, x, y, z, v[0], v[1], v[2], h, m, V, rho, P, cs, A, B, gA, gB,
                        1.0, 2.0, 0.01, dv, 0.8, 0.2, v[0], v[1], v[2], 3, sub,
                        brute, ax, ay, az, du);
        rc |= orc_density(ng, x, y, z, h, m, 3, sub, brute, V, rt);
    }
    if (n) rc |= orc_gravity(n, x, y, z, m, 0.09, 0.0015, 1.0, n, NULL, brute, ax, ay, az);
    free(x); free(y); free(z); free(m); free(h); free(u);
    for (int a = 0; a < 3; ++a) free(v[a]);
    free(V); free(rt); free(A); free(B); free(gA); free(gB); free(rho); free(P);
    free(cs); free(dv); free(ax); free(ay); free(az); free(du); free(deg);
    free(counts); free(off);
    return rc;
}

int main(void) {
    int rc = 0;
    const int64_t sizes[][2] = {{500, 400}, {1, 0}, {2, 1}, {3, 0}, {0, 7}, {60, 0}};
    for (int b = 0; b < 2; ++b)
        for (unsigned k = 0; k < sizeof(sizes) / sizeof(sizes[0]); ++k)
            rc |= run(sizes[k][0], sizes[k][1], 1234567ULL + k, b);
    double W, dW;
    orc_kernel(0.0, 0.1, &W, &dW);
    orc_kernel(0.15, 0.1, &W, &dW);
    (void)orc_s2_force(0.01, 0.05);
    (void)orc_grav_g(0.0, 0.05, 0.001);
    printf("oracle driver: %s\n", rc ? "a call failed" : "all calls returned 0");
    return rc ? 1 : 0;
}
