/*
 * host_sanitize_driver.c -- drives the host side of libdsm.so (argument
 * checks, buffer sizing, the error strings, the NULL-handle paths of every
 * entry point, the batch calls) on a build whose host code runs under
 * AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers.py builds and runs it).  Test infrastructure only.
 * Nothing here reaches the device: every call fails its host-side checks
 * before any HIP call, which is what it verifies.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "dsm.h"

static int failures = 0;

#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            fprintf(stderr, "check failed: " __VA_ARGS__); \
            fprintf(stderr, "\n");                         \
            ++failures;                                    \
        }                                                  \
    } while (0)

static dsm_params good(int dim, int nx, int ny, int nz, int storage) {
    dsm_params p;
    memset(&p, 0, sizeof(p));
    p.dim = dim;
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.kappa[0] = 0.01;
    p.kappa[1] = 0.005;
    p.kappa[2] = 0.01;
    p.alpha = 1.0;
    p.tau = 1.0;
    p.mobility = 0.1;
    p.storage = storage;
    return p;
}

static void invalid(dsm_params p, const char* what) {
    dsm_sim* s = (dsm_sim*)0;
    CHECK(dsm_required_bytes(&p) == 0, "%s: sized", what);
    int rc = dsm_create(&p, NULL, (void*)(uintptr_t)4096, (size_t)1 << 40, NULL, &s);
    CHECK(rc == DSM_EINVAL && s == NULL, "%s: created (rc %d)", what, rc);
    CHECK(strlen(dsm_last_error()) > 0, "%s: no message", what);
}

int main(void) {
    /* sizing over both lattices, both storages, ragged and padded rows */
    for (int storage = 0; storage < 2; ++storage)
        for (int nx = 4; nx < 140; nx += 17) {
            dsm_params p3 = good(3, nx, 6, 5, storage), p2 = good(2, nx, 9, 1, storage);
            size_t n3 = dsm_required_bytes(&p3), n2 = dsm_required_bytes(&p2);
            CHECK(n3 > (size_t)nx * 30 * 19 * 4 * (storage ? 2 : 4), "3D size %d", nx);
            CHECK(n2 > (size_t)nx * 9 * 9 * 4 * (storage ? 2 : 4), "2D size %d", nx);
        }
    /* every parameter check */
    dsm_params p;
    p = good(3, 32, 24, 16, 0); p.dim = 4; invalid(p, "dim");
    p = good(3, 3, 24, 16, 0); invalid(p, "nx");
    p = good(2, 32, 24, 2, 0); invalid(p, "nz in 2D");
    p = good(3, 32, 24, 16, 0); p.tau = 0.5; invalid(p, "tau");
    p = good(3, 32, 24, 16, 0); p.tau = NAN; invalid(p, "tau nan");
    p = good(3, 32, 24, 16, 0); p.mobility = 0.0; invalid(p, "mobility");
    p = good(3, 32, 24, 16, 0); p.alpha = 0.0; invalid(p, "alpha");
    p = good(3, 32, 24, 16, 0); p.reduce_every = -1; invalid(p, "reduce_every");
    p = good(3, 32, 24, 16, 0); p.kernel = 7; invalid(p, "kernel");
    p = good(3, 32, 24, 16, 3); invalid(p, "storage");
    p = good(3, 32, 24, 16, 0); p.kappa[0] = -1.0; invalid(p, "kappa_1");
    p = good(3, 32, 24, 16, 0); p.kappa[1] = p.kappa[2] = 0.0; invalid(p, "fluid kappas");
    p = good(3, 32, 24, 16, 0); p.rho[0] = -1.0; invalid(p, "rho");
    p = good(3, 32, 24, 16, 0); p.tau_gas = 0.4; invalid(p, "tau_gas");
    p = good(2, 32, 24, 1, 0); p.gravity[2] = 1e-5; invalid(p, "gravity along z in 2D");
    /* buffer checks */
    p = good(3, 32, 24, 16, 0);
    size_t need = dsm_required_bytes(&p);
    dsm_sim* s = NULL;
    CHECK(dsm_create(&p, NULL, (void*)(uintptr_t)4096, need - 1, NULL, &s) == DSM_ENOMEM, "small buffer");
    CHECK(dsm_create(&p, NULL, (void*)(uintptr_t)4104, need, NULL, &s) == DSM_EINVAL, "misaligned buffer");
    CHECK(dsm_create(&p, NULL, NULL, need, NULL, &s) == DSM_EINVAL, "NULL buffer");
    CHECK(dsm_create(NULL, NULL, (void*)(uintptr_t)4096, need, NULL, &s) == DSM_EINVAL, "NULL params");
    CHECK(dsm_create(&p, NULL, (void*)(uintptr_t)4096, need, NULL, NULL) == DSM_EINVAL, "NULL out");
    /* NULL handles on every entry point */
    double d3[3] = {0, 0, 0}, F = 0, E = 0;
    dsm_diag dg;
    uint8_t m8[4];
    char img[16];
    int v = 0, pl = 0;
    CHECK(dsm_init_solid(NULL, 1, 0.1, 0.1, 1.0, 0.1, DSM_SOLID_RESET) == DSM_EINVAL, "init_solid");
    CHECK(dsm_set_solid_field(NULL, d3) == DSM_EINVAL, "set_solid_field");
    CHECK(dsm_set_liquid(NULL, d3) == DSM_EINVAL, "set_liquid");
    CHECK(dsm_set_gravity(NULL, d3) == DSM_EINVAL, "set_gravity");
    CHECK(dsm_step(NULL, 1) == DSM_EINVAL, "step");
    CHECK(dsm_step_timed(NULL, 1, &F, &E) == DSM_EINVAL, "step_timed");
    CHECK(dsm_free_energy(NULL, &F, &E) == DSM_EINVAL, "free_energy");
    CHECK(dsm_mass(NULL, d3) == DSM_EINVAL, "mass");
    CHECK(dsm_diagnostics(NULL, &dg) == DSM_EINVAL, "diagnostics");
    CHECK(dsm_diagnostics_noalloc(NULL, &dg) == DSM_EINVAL, "diagnostics_noalloc");
    CHECK(dsm_solid_region(NULL, m8) == DSM_EINVAL, "solid_region");
    CHECK(dsm_fields(NULL, d3, d3, d3, d3, d3) == DSM_EINVAL, "fields");
    CHECK(dsm_chemical_potential(NULL, d3) == DSM_EINVAL, "chemical_potential");
    CHECK(dsm_get_populations(NULL, d3, d3) == DSM_EINVAL, "get_populations");
    CHECK(dsm_set_populations(NULL, d3, d3) == DSM_EINVAL, "set_populations");
    CHECK(dsm_set_postcollision(NULL, d3, d3) == DSM_EINVAL, "set_postcollision");
    CHECK(dsm_state_bytes(NULL) == 0, "state_bytes");
    CHECK(dsm_get_state(NULL, img, sizeof(img)) == DSM_EINVAL, "get_state");
    CHECK(dsm_set_state(NULL, img, sizeof(img)) == DSM_EINVAL, "set_state");
    CHECK(dsm_step_count(NULL) < 0, "step_count");
    CHECK(dsm_set_tiling(NULL, 0, 16) == DSM_EINVAL, "set_tiling");
    CHECK(dsm_get_tiling(NULL, &v, &pl) == DSM_EINVAL, "get_tiling");
    CHECK(dsm_tune_tiling(NULL, 3, &F) == DSM_EINVAL, "tune_tiling");
    CHECK(dsm_tiling_variants(3) >= 1 && dsm_tiling_variants(2) >= 1 && dsm_tiling_variants(5) == 0, "variants");
    CHECK(dsm_destroy(NULL) == DSM_EINVAL, "destroy");
    /* batch calls */
    dsm_sim* members[2] = {NULL, NULL};
    dsm_batch* b = NULL;
    dsm_batch_schedule sc = {0, 16, 0};
    double cost[2];
    CHECK(dsm_batch_required_bytes(NULL, 3) == 0, "batch size NULL");
    CHECK(dsm_batch_required_bytes(members, 0) == 0, "batch size empty");
    CHECK(dsm_batch_required_bytes(members, 2) == 0, "batch size NULL members");
    CHECK(dsm_batch_create(members, 2, (void*)(uintptr_t)4096, 1 << 20, NULL, &b) == DSM_EINVAL && !b,
          "batch create");
    CHECK(dsm_batch_set_schedule(NULL, 2, &sc) == DSM_EINVAL, "batch set schedule");
    CHECK(dsm_batch_get_schedule(NULL, 2, &sc) == DSM_EINVAL, "batch get schedule");
    CHECK(dsm_batch_tune(NULL, 0, cost) == DSM_EINVAL, "batch tune");
    CHECK(dsm_batch_step(NULL, 1) == DSM_EINVAL, "batch step");
    CHECK(dsm_batch_step_timed(NULL, 1, &F) == DSM_EINVAL, "batch step timed");
    CHECK(dsm_batch_size(NULL) == -1 && dsm_batch_items(NULL, 2) == -1, "batch size/items");
    CHECK(dsm_batch_destroy(NULL) == DSM_EINVAL, "batch destroy");
    CHECK(strlen(dsm_last_error()) > 0, "last error");
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("host sanitizer run: all checks passed\n");
    return 0;
}
