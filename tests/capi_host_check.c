/* Host-only paths of the liblb C ABI, run by tests/test_host_sanitizers.py
 * against a build of the library whose host code is instrumented with
 * AddressSanitizer and UndefinedBehaviorSanitizer (no GPU is needed: every
 * call below is refused or fails before touching a device, or is a host
 * helper).  Exit status 0 when every call returned what it should. */
#include <stdio.h>
#include <string.h>

#include "lb.h"

static int failures = 0;

static void expect(int cond, const char* what) {
    if (!cond) {
        fprintf(stderr, "FAILED: %s (last error: %s)\n", what, lb_last_error());
        ++failures;
    }
}

static lb_params base(void) {
    lb_params p;
    memset(&p, 0, sizeof p);
    p.nx = 16;
    p.ny = 16;
    p.scheme = LB_FV_HEUN;
    p.storage = LB_F32;
    p.dt = 1.0;
    p.tau = 0.5;
    p.tau_g = 0.5;
    p.rho_ref = 1.0;
    p.rho_x0 = 1.0;
    p.rho_x1 = 1.0;
    return p;
}

int main(void) {
    double f[1025];
    /* grid helpers: every face written, ends exact, bad arguments refused */
    expect(lb_grid_uniform(1024, 3.0, f) == LB_OK && f[0] == 0.0 && f[1024] == 3.0, "uniform grid");
    expect(lb_grid_tanh(1024, 100.0, 2.5, f) == LB_OK && f[0] == 0.0 && f[1024] == 100.0, "tanh grid");
    expect(lb_grid_sinh(1024, 64.0, 6.5, f) == LB_OK && f[512] > 31.999 && f[512] < 32.001, "sinh grid");
    expect(lb_grid_sinh(1023, 64.0, 6.5, f) == LB_EINVAL, "sinh grid, odd n");
    expect(lb_grid_chebyshev(1024, 2.0, f) == LB_OK && f[1024] == 2.0, "chebyshev grid");
    expect(lb_grid_uniform(0, 1.0, f) == LB_EINVAL, "uniform grid, n = 0");
    expect(lb_grid_tanh(8, 1.0, 2.0, NULL) == LB_EINVAL, "tanh grid, NULL output");

    /* creation: every bad parameter refused with its message */
    lb_sim* sim = NULL;
    lb_params p = base();
    expect(lb_create(NULL, &sim) == LB_EINVAL, "create, NULL params");
    expect(lb_create(&p, NULL) == LB_EINVAL, "create, NULL output");
    p.nx = 2; expect(lb_create(&p, &sim) == LB_EINVAL && sim == NULL, "create, nx = 2"); p = base();
    p.tau = 0.0; expect(lb_create(&p, &sim) == LB_EINVAL, "create, tau = 0"); p = base();
    p.dt = -1.0; expect(lb_create(&p, &sim) == LB_EINVAL, "create, dt < 0"); p = base();
    p.storage = 9; expect(lb_create(&p, &sim) == LB_EINVAL, "create, storage code"); p = base();
    p.scheme = 7; expect(lb_create(&p, &sim) == LB_EINVAL, "create, scheme code"); p = base();
    p.bc_y = LB_DENSITY; expect(lb_create(&p, &sim) == LB_EINVAL, "create, density on y"); p = base();
    p.scheme = LB_ST; p.storage = LB_BF16S; expect(lb_create(&p, &sim) == LB_EINVAL, "create, split ST"); p = base();
    p.nx = p.ny = 12000; p.storage = LB_F64; p.thermal = 1;
    expect(lb_create(&p, &sim) == LB_EINVAL && strstr(lb_last_error(), "4 GiB") != NULL, "create, 4 GiB state");
    p = base();

    /* NULL handles and outputs */
    double out[8];
    expect(lb_step(NULL, 1) == LB_EINVAL, "step, NULL handle");
    expect(lb_sync(NULL) == LB_EINVAL, "sync, NULL handle");
    expect(lb_diagnostics(NULL, out) == LB_EINVAL, "diagnostics, NULL handle");
    expect(lb_diagnostics_noalloc(NULL, out) == LB_EINVAL, "diagnostics_noalloc, NULL handle");
    expect(lb_nusselt(NULL, out, out + 1, out + 2) == LB_EINVAL, "nusselt, NULL handle");
    expect(lb_set_fv_fused(NULL, 1) == LB_EINVAL, "set_fv_fused, NULL handle");
    expect(lb_set_rebase(NULL, 3) == LB_EINVAL, "set_rebase, NULL handle");
    expect(lb_state_bytes(NULL) == 0, "state_bytes, NULL handle");
    expect(lb_device_bytes(NULL) == 0, "device_bytes, NULL handle");
    lb_destroy(NULL);
    expect(lb_stream_probe(1 << 20, NULL, out) == LB_EINVAL, "stream probe, small buffer");
    expect(lb_stream_probe(64 << 20, NULL, NULL) == LB_EINVAL, "stream probe, NULL output");

    /* groups */
    lb_group* g = NULL;
    expect(lb_group_create(0, NULL, &g) == LB_EINVAL, "group, 0 slots");
    expect(lb_group_create(70000, NULL, &g) == LB_EINVAL, "group, too many slots");
    expect(lb_group_step(NULL, 1) == LB_EINVAL, "group step, NULL");
    expect(lb_group_set_chunk(NULL, 8) == LB_EINVAL, "group chunk, NULL");
    expect(lb_group_remove(NULL, 0) == LB_EINVAL, "group remove, NULL");
    lb_group_destroy(NULL);

    /* 3D */
    lb3_sim* s3 = NULL;
    expect(lb3_create(NULL, &s3) == LB_EINVAL, "3D create, NULL params");
    expect(lb3_step(NULL, 1) == LB_EINVAL, "3D step, NULL handle");
    lb3_destroy(NULL);

    if (failures) fprintf(stderr, "%d failures\n", failures);
    else printf("host checks passed\n");
    return failures ? 1 : 0;
}
