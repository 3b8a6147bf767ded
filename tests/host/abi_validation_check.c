/* Host-side validation of the C ABI (include/iblb.h), built with AddressSanitizer
 * and UndefinedBehaviorSanitizer on the host code: iblb_workspace_size validates
 * a configuration and lays out the workspace without touching a device.  Each
 * case states the status it must return; a mismatch or a sanitizer report makes
 * the program fail. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "iblb.h"

static int failures = 0;

/* a closed tetrahedron, counter-clockwise seen from outside */
static const double TET[4][3] = {{10, 10, 3}, {14, 10, 3}, {10, 14, 3}, {10, 10, 7}};
static const int32_t TET_T[4][3] = {{0, 2, 1}, {0, 1, 3}, {0, 3, 2}, {1, 2, 3}};

static void expect(const char *name, const iblb_config *cfg, iblb_status want) {
    size_t bytes = 0;
    const iblb_status got = iblb_workspace_size(cfg, &bytes);
    const char *msg = iblb_last_error(NULL);
    if (got != want || msg == NULL || (got != IBLB_OK && strlen(msg) == 0) || (got == IBLB_OK && bytes == 0)) {
        printf("FAIL %s: status %d, want %d (%s)\n", name, got, want, msg ? msg : "(null)");
        ++failures;
    } else {
        printf("ok   %s: %d %s\n", name, got, got == IBLB_OK ? "" : msg);
    }
}

int main(void) {
    double nodes[4][3];
    int32_t tris[4][3];
    memcpy(nodes, TET, sizeof nodes);
    memcpy(tris, TET_T, sizeof tris);
    iblb_box box;
    memset(&box, 0, sizeof box);
    box.nx = 24; box.ny = 20; box.nz = 16; box.zbc = IBLB_Z_WALLS;
    box.tau = 0.8; box.rho0 = 1.0;
    iblb_droplet d;
    memset(&d, 0, sizeof d);
    d.box = 0; d.n_nodes = 4; d.n_tris = 4; d.n_exp = 9; d.m_exp = 3;
    d.nodes = &nodes[0][0]; d.tris = &tris[0][0];
    d.sigma = 0.01; d.theta_eq = 1.0; d.xi = 0.4;
    iblb_config cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.n_boxes = 1; cfg.n_droplets = 1; cfg.boxes = &box; cfg.droplets = &d;
    cfg.storage = IBLB_F32; cfg.dev_scale = 1.0;

    expect("valid", &cfg, IBLB_OK);
    expect("null config", NULL, IBLB_E_INVAL);
    { iblb_config c = cfg; c.storage = 7; expect("storage", &c, IBLB_E_INVAL); }
    { iblb_config c = cfg; c.flags = 64u; expect("flags", &c, IBLB_E_INVAL); }
    { iblb_config c = cfg; c.storage = IBLB_F16DEV; c.dev_scale = 3.0; expect("dev_scale", &c, IBLB_E_INVAL); }
    { iblb_box b = box; iblb_config c = cfg; c.boxes = &b; b.tau = 0.5; expect("tau", &c, IBLB_E_INVAL); }
    { iblb_box b = box; iblb_config c = cfg; c.boxes = &b; b.tau_in = 0.3; expect("tau_in", &c, IBLB_E_INVAL); }
    { iblb_box b = box; iblb_config c = cfg; c.boxes = &b; b.wall_lo[0] = 0.5; expect("wall speed", &c, IBLB_E_INVAL); }
    { iblb_box b = box; iblb_config c = cfg; c.boxes = &b; b.body_force[1] = NAN; expect("body force", &c, IBLB_E_INVAL); }
    { iblb_box b = box; iblb_config c = cfg; c.boxes = &b; b.nx = 3; expect("box too small for a droplet", &c, IBLB_E_INVAL); }
    { iblb_box b = box; iblb_config c = cfg; c.boxes = &b; b.nx = 4096; b.ny = 4096; b.nz = 64;
      c.n_droplets = 0; expect("box beyond 4 GiB of planes", &c, IBLB_E_INVAL); }
    { iblb_droplet e = d; iblb_config c = cfg; c.droplets = &e; e.box = 2; expect("droplet box index", &c, IBLB_E_INVAL); }
    { iblb_droplet e = d; iblb_config c = cfg; c.droplets = &e; e.n_exp = 3; expect("exponents", &c, IBLB_E_INVAL); }
    { iblb_droplet e = d; iblb_config c = cfg; c.droplets = &e; e.xi = 0.0; expect("xi", &c, IBLB_E_INVAL); }
    { iblb_droplet e = d; iblb_config c = cfg; c.droplets = &e; e.n_tris = 3; expect("too few triangles", &c, IBLB_E_INVAL); }
    {
        int32_t t2[4][3];
        memcpy(t2, tris, sizeof t2);
        t2[3][0] = 1; t2[3][1] = 2; t2[3][2] = 0;  /* repeats the directed edge 2 -> 0 */
        iblb_droplet e = d; iblb_config c = cfg; c.droplets = &e; e.tris = &t2[0][0];
        expect("non-manifold mesh", &c, IBLB_E_MESH);
    }
    {
        int32_t t2[4][3];
        memcpy(t2, tris, sizeof t2);
        t2[1][2] = 9;
        iblb_droplet e = d; iblb_config c = cfg; c.droplets = &e; e.tris = &t2[0][0];
        expect("node index out of range", &c, IBLB_E_MESH);
        t2[1][2] = t2[1][1];
        expect("degenerate triangle", &c, IBLB_E_MESH);
    }
    {
        int32_t t2[4][3];
        for (int k = 0; k < 4; ++k) { t2[k][0] = tris[k][0]; t2[k][1] = tris[k][2]; t2[k][2] = tris[k][1]; }
        iblb_droplet e = d; iblb_config c = cfg; c.droplets = &e; e.tris = &t2[0][0];
        expect("inward orientation", &c, IBLB_E_MESH);
    }
    {
        double n2[4][3];
        memcpy(n2, nodes, sizeof n2);
        n2[0][2] = 0.0;
        iblb_droplet e = d; iblb_config c = cfg; c.droplets = &e; e.nodes = &n2[0][0];
        expect("node on the wall", &c, IBLB_E_MESH);
        n2[0][2] = NAN;
        expect("node not finite", &c, IBLB_E_INVAL);
    }
    {
        int32_t cv[19 * 3];
        double w[19];
        int32_t shape[3];
        if (iblb_velocity_set(cv, w) != IBLB_OK || iblb_band_tile(shape) != IBLB_OK ||
            shape[0] * shape[1] * shape[2] != 64) {
            printf("FAIL velocity set / band tile\n");
            ++failures;
        }
        double sw = 0.0;
        for (int i = 0; i < 19; ++i) sw += w[i];
        if (fabs(sw - 1.0) > 1e-15) { printf("FAIL weights sum %.17g\n", sw); ++failures; }
    }
    printf("%s: %d failures\n", failures ? "FAILED" : "passed", failures);
    return failures ? 1 : 0;
}
