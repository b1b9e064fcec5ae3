/*
 * sanitize_check.c -- TEST INFRASTRUCTURE ONLY: a driver that runs the oracle's entry points on
 * small boxes so that the oracle can be built and run under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py builds it with
 * -fsanitize=address,undefined and fails on any report or non-zero exit).
 *
 * For each body (sphere, rotated ellipsoid, z-slab between EB walls, y-axis cylinder, fluid
 * cavity) on a 16^3 box (the cylinder and the slab periodic in some directions), and a small
 * cavity on a 12^3 box whose wall stencils take the covered-node fallback: geometry,
 * viscosity, one RK2 step with each end-of-stage projection, the drag with each pressure, the
 * nodal operators, the step adjoint and the drag adjoint, with the yield stress multiplied by a
 * per-cell field.  Inputs are deterministic (a fixed linear congruential sequence).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "eb_oracle.h"

static unsigned long long lcg_state = 12345;
static double lcg_uniform(void) {  /* in [-1, 1) */
    lcg_state = lcg_state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg_state >> 11) / 4503599627370496.0 - 1.0;
}

static void *xcalloc(size_t n, size_t sz) {
    void *p = calloc(n, sz);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static int run_case(const char *name, const or_box *box, const or_body *body) {
    int err = 0;
    or_geom *g = or_geom_build(box, body, &err);
    if (!g || err) {
        fprintf(stderr, "%s: geometry error %d\n", name, err);
        return 1;
    }
    int nx = box->n[0], ny = box->n[1], nz = box->n[2];
    long N = (long)nx * ny * nz;
    long NN = (long)(nx + 1) * (ny + 1) * (nz + 1);
    int ncut = or_geom_ncut(g);
    double *u = xcalloc(3 * N, sizeof(double)), *p = xcalloc(N, sizeof(double));
    double *theta = xcalloc(N, sizeof(double)), *eta = xcalloc(N, sizeof(double));
    double *eta_eb = xcalloc(ncut > 0 ? ncut : 1, sizeof(double));
    double *sr = xcalloc(N, sizeof(double));
    double *u0 = xcalloc(3 * N, sizeof(double)), *p0 = xcalloc(N, sizeof(double));
    double *ub = xcalloc(3 * N, sizeof(double)), *pb = xcalloc(N, sizeof(double));
    double *tau0b = xcalloc(N, sizeof(double));
    double *pn = xcalloc(NN, sizeof(double)), *dn = xcalloc(NN, sizeof(double));
    double *bn = xcalloc(NN, sizeof(double)), *yn = xcalloc(NN, sizeof(double));
    double *gp = xcalloc(3 * N, sizeof(double));
    for (long c = 0; c < N; c++) {
        theta[c] = 1.0 + 0.05 * lcg_uniform();
        for (int m = 0; m < 3; m++) u[m * N + c] = body->u_eb[m] + 0.01 * lcg_uniform();
    }
    or_rheo rh;
    memset(&rh, 0, sizeof rh);
    rh.law = OR_LAW_BINGHAM_REG;
    rh.mu = 1.0;
    rh.tau0 = 1.0;
    rh.eps = 1e-6;
    rh.rho = 1.0;
    or_opts o;
    memset(&o, 0, sizeof o);
    o.rtol_visc = o.rtol_mac = o.rtol_proj = 1e-10;
    o.max_iter = 200;
    o.nu1 = o.nu2 = 2;
    o.nbottom = 16;
    o.projection = OR_PROJ_CELL;
    double dt = 1e-3;
    int rc = 0;
    or_viscosity(g, &rh, u, theta, eta, eta_eb, sr);
    memcpy(u0, u, 3 * N * sizeof(double));
    or_stats st;
    int e = or_rk2_step(g, &rh, theta, dt, &o, u, p, &st);
    if (e != OR_OK) {
        fprintf(stderr, "%s: cell-projection step returned %d\n", name, e);
        rc = 1;
    }
    double F[3], Fb[3] = {0.0, 0.0, 1.0};
    or_drag(g, &rh, theta, u, p, F);
    /* the step adjoint of the drag after one step */
    or_drag_adj(g, &rh, theta, u, Fb, ub, pb, tau0b);
    e = or_rk2_step_adjoint(g, &rh, theta, dt, &o, u0, p0, ub, pb, tau0b, &st);
    if (e != OR_OK) {
        fprintf(stderr, "%s: step adjoint returned %d\n", name, e);
        rc = 1;
    }
    /* nodal operators and a step with the nodal projection */
    or_nodal_div(g, u, dn);
    or_nodal_bflux(g, bn);
    for (long q = 0; q < NN; q++) pn[q] = 0.1 * lcg_uniform();
    or_nodal_apply(g, pn, yn);
    or_nodal_grad(g, pn, gp);
    memset(pn, 0, NN * sizeof(double));
    memcpy(u, u0, 3 * N * sizeof(double));
    o.projection = OR_PROJ_NODAL;
    o.max_iter = 2000;
    e = or_rk2_step(g, &rh, theta, dt, &o, u, pn, &st);
    if (e != OR_OK) {
        fprintf(stderr, "%s: nodal-projection step returned %d\n", name, e);
        rc = 1;
    }
    or_drag_nodal(g, &rh, theta, u, pn, F);
    printf("%s: ncut %d, nfallback %d, drag (%.6e, %.6e, %.6e)\n", name, ncut,
           or_geom_nfallback(g), F[0], F[1], F[2]);
    free(u); free(p); free(theta); free(eta); free(eta_eb); free(sr); free(u0); free(p0);
    free(ub); free(pb); free(tau0b); free(pn); free(dn); free(bn); free(yn); free(gp);
    or_geom_free(g);
    return rc;
}

int main(void) {
    int n = 16, rc = 0;
    or_box box;
    memset(&box, 0, sizeof box);
    for (int d = 0; d < 3; d++) box.n[d] = n;
    box.h = 1.0 / n;
    for (int f = 0; f < 6; f++) box.wall_u[f][2] = -1.0;
    or_body b;

    memset(&b, 0, sizeof b);
    b.kind = OR_BODY_SPHERE;
    b.center[0] = b.center[1] = b.center[2] = 0.5;
    b.radii[0] = 0.23;
    rc |= run_case("sphere", &box, &b);

    memset(&b, 0, sizeof b);
    b.kind = OR_BODY_ELLIPSOID;
    b.center[0] = b.center[1] = b.center[2] = 0.5;
    b.radii[0] = 0.3; b.radii[1] = 0.2; b.radii[2] = 0.16;
    b.euler_zyx[0] = 0.4; b.euler_zyx[1] = -0.3; b.euler_zyx[2] = 0.7;
    rc |= run_case("ellipsoid", &box, &b);

    or_box pbox = box;
    pbox.periodic[0] = pbox.periodic[1] = 1;
    for (int f = 0; f < 6; f++) pbox.wall_u[f][2] = 0.0;
    memset(&b, 0, sizeof b);
    b.kind = OR_BODY_ZSLAB;
    b.zlo = 0.1171875;
    b.zhi = 0.8828125;
    rc |= run_case("zslab", &pbox, &b);

    or_box cbox = box;
    cbox.periodic[1] = 1;
    memset(&b, 0, sizeof b);
    b.kind = OR_BODY_CYLINDER;
    b.center[0] = b.center[1] = b.center[2] = 0.5;
    b.radii[0] = 0.2;
    rc |= run_case("cylinder", &cbox, &b);

    or_box vbox = box;
    for (int f = 0; f < 6; f++) vbox.wall_u[f][2] = 0.0;
    memset(&b, 0, sizeof b);
    b.kind = OR_BODY_CAVITY;
    b.center[0] = b.center[1] = b.center[2] = 0.5;
    b.radii[0] = 0.37;
    b.u_eb[0] = 1.0;
    rc |= run_case("cavity", &vbox, &b);

    /* a small cavity on a coarse box: its wall stencils take the covered-node fallback */
    or_box fbox = vbox;
    for (int d = 0; d < 3; d++) fbox.n[d] = 12;
    fbox.h = 1.0 / 12;
    memset(&b, 0, sizeof b);
    b.kind = OR_BODY_CAVITY;
    b.center[0] = 0.5; b.center[1] = 0.53; b.center[2] = 0.46;
    b.radii[0] = 0.15;
    b.u_eb[0] = 1.0;
    rc |= run_case("cavity_fallback", &fbox, &b);
    return rc;
}
