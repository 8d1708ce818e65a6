/* Host sanitizer run of libmsf.so's C ABI (library built with host-side
 * -fsanitize=address,undefined): the validation paths that run before any
 * device work, i.e. invalid and oversize geometries, null handles on every
 * entry point, network parameter checks and option defaults.  No GPU is
 * needed.  Exit status 0 = every call returned what the header promises. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "msf.h"

static int failures = 0;
static void expect(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s (last error: %s)\n", what, msf_last_error());
        failures++;
    }
}

static msf_geometry base_geom(int64_t *vo, double *an)
{
    msf_geometry g;
    memset(&g, 0, sizeof g);
    g.nx = g.ny = g.nz = 8;
    g.n_frames = 1;
    g.nu = g.nv = 12;
    g.du = g.dv = 2.0;
    g.src_iso = 50.0;
    g.src_det = 100.0;
    vo[0] = 0;
    vo[1] = 2;
    an[0] = 0.1;
    an[1] = 0.2;
    g.view_offset = vo;
    g.angles = an;
    return g;
}

int main(void)
{
    int64_t vo[2];
    double an[2];
    msf_plan *plan = NULL;

    /* invalid geometries: EINVAL, *out untouched, a message */
    for (int c = 0; c < 10; c++) {
        msf_geometry g = base_geom(vo, an);
        switch (c) {
        case 0: g.nx = 0; break;
        case 1: g.n_frames = 0; break;
        case 2: g.du = -1.0; break;
        case 3: g.src_iso = 4.0; break;
        case 4: g.src_det = 55.0; break;
        case 5: g.dv = NAN; break;
        case 6: vo[0] = 1; break;
        case 7: an[1] = NAN; break;
        case 8: g.angles = NULL; break;
        case 9: g.nx = 1 << 11; g.ny = 1 << 11; g.nz = 1 << 10; g.src_iso = 3000.0; g.src_det = 6000.0; break;
        }
        plan = NULL;
        expect(msf_plan_create(&g, &plan) == MSF_EINVAL && plan == NULL, "plan_create rejects bad geometry");
        expect(strlen(msf_last_error()) > 0, "plan_create sets a message");
    }
    expect(msf_plan_create(NULL, &plan) == MSF_EINVAL, "plan_create rejects NULL geometry");

    /* null handles */
    msf_tiles t;
    msf_timing tm;
    msf_mace_opts mo;
    msf_mace_opts_default(&mo);
    expect(msf_project(NULL, NULL, NULL, NULL) == MSF_EINVAL, "project");
    expect(msf_backproject(NULL, NULL, NULL, NULL) == MSF_EINVAL, "backproject");
    expect(msf_prox_solve(NULL, NULL, NULL, NULL, 0.5, NULL, NULL, NULL, NULL) == MSF_EINVAL, "prox_solve");
    expect(msf_prox_features(NULL, NULL, NULL, NULL, 0.5, NULL, NULL) == MSF_EINVAL, "prox_features");
    expect(msf_plan_set_tiles(NULL, &t) == MSF_EINVAL, "set_tiles");
    expect(msf_plan_get_tiles(NULL, &t) == MSF_EINVAL, "get_tiles");
    expect(msf_plan_sizes(NULL, NULL, NULL, NULL) == MSF_EINVAL, "sizes");
    expect(msf_plan_set_timing(NULL, 1) == MSF_EINVAL, "set_timing");
    expect(msf_plan_get_timing(NULL, &tm) == MSF_EINVAL, "get_timing");
    expect(msf_plan_autotune(NULL, NULL, NULL, NULL) == MSF_EINVAL, "autotune");
    expect(msf_count_intersections(NULL, NULL, NULL) == MSF_EINVAL, "count_intersections");
    expect(msf_fixture_correct(NULL, NULL, NULL, 10.0, 1.0, NULL, NULL, NULL) == MSF_EINVAL, "fixture_correct");
    expect(msf_fixture_correct_noalloc(NULL, NULL, NULL, 10.0, 1.0, NULL, NULL, NULL) == MSF_EINVAL,
           "fixture_correct_noalloc");
    expect(msf_mace_run(NULL, NULL, NULL, NULL, 0.5, &mo, NULL, NULL, NULL) == MSF_EINVAL, "mace_run");
    expect(msf_cnn_get_params(NULL, NULL) == MSF_EINVAL, "cnn_get_params");
    expect(msf_cnn_infer(NULL, NULL, NULL, 1, 1, 8, 8, NULL, NULL) == MSF_EINVAL, "cnn_infer");
    expect(msf_cnn_train_step(NULL, NULL, NULL, NULL, 1, 1, 8, 8, 1e-3, 1, NULL, NULL, NULL) == MSF_EINVAL,
           "cnn_train_step");
    expect(msf_denoise25(NULL, NULL, 1, 8, 8, 8, 1, NULL, NULL) == MSF_EINVAL, "denoise25");
    expect(msf_cnn_kind(NULL) == -1 && msf_cnn_n_params(NULL) == 0, "cnn kind / count of NULL");
    msf_plan_destroy(NULL);
    msf_cnn_destroy(NULL);

    /* network parameter validation: wrong count, scale <= 0, non-finite weight */
    const int64_t counts[2] = {15169, 5521};
    const int nsc[2] = {3, 2};
    for (int k = 0; k < 2; k++) {
        const int64_t n = counts[k];
        float *p = calloc((size_t)n, sizeof(float));
        float sc[3] = {1.0f, 1.0f, 1.0f};
        msf_cnn *net = NULL;
        msf_status (*create)(const float *, int64_t, const float *, msf_cnn **) =
            k == 0 ? msf_cnn_create : msf_cnn_create_denoiser;
        expect(create(p, n - 1, sc, &net) == MSF_EINVAL && net == NULL, "network: wrong count");
        sc[nsc[k] - 1] = 0.0f;
        expect(create(p, n, sc, &net) == MSF_EINVAL && net == NULL, "network: scale <= 0");
        sc[nsc[k] - 1] = 1.0f;
        p[n / 2] = NAN;
        expect(create(p, n, sc, &net) == MSF_EINVAL && net == NULL, "network: non-finite weight");
        expect(create(NULL, n, sc, &net) == MSF_EINVAL, "network: NULL parameters");
        free(p);
    }

    /* option defaults */
    msf_solve_opts so;
    msf_solve_opts_default(&so);
    expect(so.tol == 1e-6 && so.max_iter == 1000 && so.check_every == 8 && so.use_graph == 1, "solve defaults");
    expect(mo.n_iter == 10 && mo.rho == 0.5 && mo.beta == 1.0, "mace defaults");
    expect(strncmp(msf_version(), "msf", 3) == 0, "version");
    if (failures) return 1;
    printf("C ABI sanitizer run: clean\n");
    return 0;
}
