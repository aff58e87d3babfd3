/*
 * oracle_sanitize_driver.c -- drives every entry point of the FP64 oracle on
 * small lattices, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py compiles and runs
 * it).  Test infrastructure only.
 *
 * It walks both lattices, both stages, the two-step solid initialisation,
 * the density/viscosity contrast, both readings of the confining potential
 * and of the surface-tension force, population get/set and the
 * post-collision entry, the observables, the wall fraction of every link,
 * the argument checks and the refusal of a non-finite state, and exits
 * non-zero if an invariant of the scheme fails (the liquid amount is conserved by every fluid step; the solid
 * amount by every solid step).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/dsm_oracle.h"

static int failures = 0;

#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            fprintf(stderr, "check failed: " __VA_ARGS__); \
            fprintf(stderr, "\n");                         \
            ++failures;                                    \
        }                                                  \
    } while (0)

/* a flat wall along the last axis plus a ball: C1 from the tanh of the
 * signed distance, the mask its C1 > 1/2 set, a drop of liquid beside it */
static void geometry(int dim, const int n[3], double* C1, double* C2, unsigned char* mask) {
    int nz = dim == 3 ? n[2] : 1;
    /* ball centre: x = 0.4 nx, 7 nodes above the bottom (and y = ny / 2 in 3D) */
    double cx = 0.4 * n[0], cy = dim == 3 ? 0.5 * n[1] : 7.0, cz = 7.0;
    long k = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x, ++k) {
                double h = dim == 3 ? z : y;
                double d_wall = 2.5 - h;
                double dx = x - cx, dy = y - cy, dz = dim == 3 ? z - cz : 0.0;
                double r = sqrt(dx * dx + (dim == 3 ? dy * dy + dz * dz : dy * dy));
                double d = fmax(d_wall, 2.5 - r);
                C1[k] = 0.5 + 0.5 * tanh(d / 2.0);
                mask[k] = C1[k] > 0.5;
                double rd = sqrt((x - 0.75 * n[0]) * (x - 0.75 * n[0]) + (h - 3.0) * (h - 3.0));
                C2[k] = (0.5 + 0.5 * tanh((4.0 - rd) / 2.0)) * (1.0 - C1[k]);
            }
}

static void run_case(int dim, const int n[3], int contrast, int force_reading, int confine_reading) {
    dsmo_params p;
    memset(&p, 0, sizeof(p));
    p.dim = dim;
    p.nx = n[0];
    p.ny = n[1];
    p.nz = dim == 3 ? n[2] : 1;
    p.kappa[0] = 0.01;
    p.kappa[1] = 0.006;
    p.kappa[2] = 0.009;
    p.alpha = 1.0;
    p.tau = 1.0;
    p.mobility = 0.1;
    p.gravity[0] = 1e-5;
    p.gravity[1] = dim == 3 ? -2e-6 : 0.0;
    p.confine_reading = confine_reading;
    p.threads = 2;
    p.rho_liquid = 1.0;
    p.rho_gas = contrast ? 0.5 : 1.0;
    p.tau_gas = contrast ? 0.7 : 1.0;
    p.force_reading = force_reading;
    long N = (long)p.nx * p.ny * p.nz;
    int Q = dim == 2 ? 9 : 19;
    double* C1 = malloc(N * sizeof(double));
    double* C2 = malloc(N * sizeof(double));
    double* C3 = malloc(N * sizeof(double));
    double* u = malloc(3 * N * sizeof(double));
    double* pr = malloc(N * sizeof(double));
    double* mu = malloc(N * sizeof(double));
    double* f = malloc((size_t)Q * N * sizeof(double));
    double* g = malloc((size_t)Q * N * sizeof(double));
    unsigned char* mask = malloc(N);
    unsigned char* S = malloc(N);
    geometry(dim, n, C1, C2, mask);

    dsmo_sim* s = NULL;
    CHECK(dsmo_create(&p, mask, &s) == DSMO_OK, "create");
    if (!s) return;
    CHECK(dsmo_num_directions(s) == Q, "Q");
    CHECK(dsmo_step(s, 1) == DSMO_ESTATE, "step before a liquid");

    /* solid stage, two-step */
    double m_s0[3], m_s1[3], F, E;
    CHECK(dsmo_init_solid(s, 20, 1e-2, 2e-3, 1.0, 1.0 / 6.0, DSMO_SOLID_RESET | DSMO_SOLID_REMASK) == DSMO_OK,
          "solid stage 1");
    CHECK(dsmo_mass(s, m_s0) == DSMO_OK, "mass");
    CHECK(dsmo_get_mask(s, S) == DSMO_OK, "mask");
    CHECK(dsmo_init_solid(s, 20, 1e-3, 2e-4, 1.0, 1.0 / 6.0, 0) == DSMO_OK, "solid stage 2");
    CHECK(dsmo_mass(s, m_s1) == DSMO_OK, "mass");
    CHECK(fabs(m_s1[0] - m_s0[0]) <= 1e-12 * fabs(m_s0[0]), "solid amount %g -> %g", m_s0[0], m_s1[0]);
    CHECK(dsmo_free_energy(s, &F, &E) == DSMO_OK && isfinite(F) && isfinite(E), "solid free energy");

    /* fluid stage on the given solid */
    CHECK(dsmo_set_solid_field(s, C1) == DSMO_OK, "set solid");
    CHECK(dsmo_set_liquid(s, C2) == DSMO_OK, "set liquid");
    double m0[3], m1[3];
    CHECK(dsmo_mass(s, m0) == DSMO_OK, "mass");
    CHECK(dsmo_step(s, 12) == DSMO_OK, "steps");
    CHECK(dsmo_mass(s, m1) == DSMO_OK, "mass");
    CHECK(fabs(m1[1] - m0[1]) <= 1e-12 * fabs(m0[1]), "liquid amount %g -> %g", m0[1], m1[1]);
    CHECK(dsmo_fields(s, C1, C2, C3, u, pr) == DSMO_OK, "fields");
    CHECK(dsmo_fields(s, NULL, NULL, NULL, NULL, NULL) == DSMO_OK, "fields, all skipped");
    CHECK(dsmo_chemical_potential(s, mu) == DSMO_OK, "mu");
    CHECK(dsmo_free_energy(s, &F, &E) == DSMO_OK && isfinite(F) && isfinite(E), "free energy");
    CHECK(dsmo_get_populations(s, f, g) == DSMO_OK, "get populations");
    CHECK(dsmo_set_populations(s, f, g) == DSMO_OK, "set populations");
    CHECK(dsmo_set_postcollision(s, f, g) == DSMO_OK, "set post-collision");
    const double grav[3] = {0.0, 1e-6, 0.0};
    CHECK(dsmo_set_gravity(s, grav) == DSMO_OK, "gravity");
    CHECK(dsmo_step(s, 3) == DSMO_OK, "steps");
    for (long k = 0; k < N; ++k) {
        CHECK(isfinite(C2[k]) && isfinite(u[k]), "finite fields at %ld", k);
        if (C1[k] < 0.5)
            for (int i = 1; i < Q; ++i) {
                double q = dsmo_link_q(s, k, i);
                CHECK(q >= 0.0 && q <= 1.0, "q(%ld, %d) = %g", k, i, q);
            }
    }
    /* argument checks */
    CHECK(dsmo_link_q(s, -1, 1) == -1.0 && dsmo_link_q(s, N, 1) == -1.0 && dsmo_link_q(s, 0, Q) == -1.0,
          "link_q bounds");
    CHECK(dsmo_step(s, -1) == DSMO_EINVAL, "negative steps");
    CHECK(dsmo_init_solid(s, 1, -1.0, 0.0, 1.0, 0.1, 0) == DSMO_EINVAL, "negative beta");
    CHECK(dsmo_set_liquid(s, NULL) == DSMO_EINVAL, "NULL liquid");
    dsmo_destroy(s);

    double w[19], feq[19], geq[19], Fi[19];
    int ci[57];
    const double uu[3] = {0.01, -0.02, 0.005}, gr[3] = {0.1, 0.0, -0.1}, FF[3] = {1e-5, 0.0, 2e-5};
    CHECK(dsmo_lattice(dim, ci, w) == Q, "lattice");
    dsmo_equilibrium_f(dim, 0.3, 1.2, uu, feq);
    dsmo_equilibrium_g(dim, 0.4, 1e-3, uu, geq);
    dsmo_forcing(dim, 0.8, 1.2, uu, gr, FF, Fi);
    free(C1);
    free(C2);
    free(C3);
    free(u);
    free(pr);
    free(mu);
    free(f);
    free(g);
    free(mask);
    free(S);
}

/* a body force far beyond the scheme's range: the oracle refuses the step
 * that starts from the non-finite state, and again after that */
static void unstable_case(const int n[3]) {
    dsmo_params p;
    memset(&p, 0, sizeof(p));
    p.dim = 2;
    p.nx = n[0];
    p.ny = n[1];
    p.nz = 1;
    p.kappa[0] = 0.01;
    p.kappa[1] = 0.006;
    p.kappa[2] = 0.009;
    p.alpha = 1.0;
    p.tau = 1.0;
    p.mobility = 0.1;
    p.gravity[0] = 50.0;
    p.threads = 2;
    p.rho_liquid = 1.0;
    p.rho_gas = 1.0;
    p.tau_gas = 1.0;
    long N = (long)p.nx * p.ny;
    double* C1 = malloc(N * sizeof(double));
    double* C2 = malloc(N * sizeof(double));
    unsigned char* mask = malloc(N);
    geometry(2, n, C1, C2, mask);
    dsmo_sim* s = NULL;
    CHECK(dsmo_create(&p, mask, &s) == DSMO_OK, "create (unstable case)");
    if (s) {
        CHECK(dsmo_set_solid_field(s, C1) == DSMO_OK && dsmo_set_liquid(s, C2) == DSMO_OK, "set (unstable)");
        CHECK(dsmo_step(s, 500) == DSMO_EUNSTABLE, "step under a body force of 50");
        CHECK(dsmo_step(s, 1) == DSMO_EUNSTABLE, "step after the state went non-finite");
        dsmo_destroy(s);
    }
    free(C1);
    free(C2);
    free(mask);
}

int main(void) {
    const int n2[3] = {20, 14, 1}, n3[3] = {12, 9, 10};
    dsmo_params bad;
    memset(&bad, 0, sizeof(bad));
    dsmo_sim* s = NULL;
    CHECK(dsmo_create(&bad, NULL, &s) == DSMO_EINVAL && s == NULL, "invalid params");
    CHECK(dsmo_create(NULL, NULL, &s) == DSMO_EINVAL, "NULL params");
    for (int contrast = 0; contrast < 2; ++contrast)
        for (int fr = 0; fr < 2; ++fr) {
            run_case(2, n2, contrast, fr, contrast);
            run_case(3, n3, contrast, fr, 1 - contrast);
        }
    unstable_case(n2);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: all checks passed\n");
    return 0;
}
