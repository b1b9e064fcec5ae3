/*
 * eb_oracle.c -- plain FP64 CPU oracle for the embedded-boundary viscoplastic RK2 step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, the smoke check and the CPU-baseline leg of the
 * bench, never by the product path.  Shares no code with the HIP library.
 *
 * Written for readability, not speed: every step is a plain loop over cells or faces in the
 * order the paper states it.  Floating point is IEEE binary64 throughout; build with
 * -ffp-contract=off so no fused multiply-add changes a rounding.
 *
 * Parity unpinned (no external value or closed form fixes them; they follow the written readings
 * and are checked only against the HIP path and through convergence rates): the covered-node
 * fallback of the wall stencil, the slope limiter and upwind tie rules, the face average of the
 * viscosity, and the coarse-level operators and smoother of the multigrid preconditioner.
 */
#include "eb_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXLEV 16

/* ------------------------------------------------------------------------------------------ */
/* grid helpers                                                                                */
/* ------------------------------------------------------------------------------------------ */
static long cidx(const int n[3], int i, int j, int k) {
    return (long)i + (long)n[0] * ((long)j + (long)n[1] * (long)k);
}
static long fidx(const int n[3], int d, int i, int j, int k) {
    long m0 = n[0] + (d == 0), m1 = n[1] + (d == 1);
    return (long)i + m0 * ((long)j + m1 * (long)k);
}
static long nfaces(const int n[3], int d) {
    return (long)(n[0] + (d == 0)) * (n[1] + (d == 1)) * (n[2] + (d == 2));
}
/* cell at integer position q (wrapped in periodic directions); -1 when outside a wall */
static long cell_at(const int n[3], const int per[3], const int q_in[3]) {
    int q[3] = {q_in[0], q_in[1], q_in[2]};
    for (int d = 0; d < 3; d++) {
        if (q[d] < 0 || q[d] >= n[d]) {
            if (!per[d]) return -1;
            q[d] = ((q[d] % n[d]) + n[d]) % n[d];
        }
    }
    return cidx(n, q[0], q[1], q[2]);
}
static void cell_ijk(const int n[3], long c, int q[3]) {
    q[0] = (int)(c % n[0]);
    q[1] = (int)((c / n[0]) % n[1]);
    q[2] = (int)(c / ((long)n[0] * n[1]));
}
/* the two directions other than d, in increasing order */
static void others(int d, int* t1, int* t2) {
    *t1 = (d == 0) ? 1 : 0;
    *t2 = (d == 2) ? 1 : 2;
}

/* ------------------------------------------------------------------------------------------ */
/* geometry (Sec. III.B: planar cut per cell, continuous at faces; fraction, apertures, normal) */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int n[3];
    long N;
    double h;
    double* alpha;
    double* ap[3];
    uint8_t* mask; /* alpha > 0 */
    /* operator built per solve */
    double* K[3];
    double* S;
    double* D;
} level_t;

struct or_geom {
    or_box box;
    or_body body;
    long N;
    uint8_t* flag;
    double* alpha;
    double* ap[3];
    int ncut;
    long* cut;    /* cell of each cut cell */
    long* cutid;  /* per cell: position in the cut list, or -1 */
    double* nrm;  /* [ncut][3] unit normal, into the fluid */
    double* aeb;  /* [ncut] EB area in units of h^2 */
    double* bc;   /* [ncut][3] EB centroid, relative to the cell centre, units of h */
    double* delta;/* [ncut] distance of the cell centre from the EB plane, units of h */
    double* dd;   /* [ncut][2] d1, d2 */
    int* nfb;     /* [ncut] planes whose stencil needed the covered-node fallback */
    long* sidx;   /* [ncut][2][9] stencil cells; -1 means "use the EB wall velocity" */
    double* sw;   /* [ncut][2][9] biquadratic weights */
    int nfallback;
    int nlev;
    level_t lev[MAXLEV];
    double R[3][3];
};

static void rotation_zyx(const double e[3], double R[3][3]) {
    double ca = cos(e[0]), sa = sin(e[0]), cb = cos(e[1]), sb = sin(e[1]);
    double cc = cos(e[2]), sc = sin(e[2]);
    double Rz[3][3] = {{ca, -sa, 0}, {sa, ca, 0}, {0, 0, 1}};
    double Ry[3][3] = {{cb, 0, sb}, {0, 1, 0}, {-sb, 0, cb}};
    double Rx[3][3] = {{1, 0, 0}, {0, cc, -sc}, {0, sc, cc}};
    double T[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            T[a][b] = 0;
            for (int c = 0; c < 3; c++) T[a][b] += Rz[a][c] * Ry[c][b];
        }
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            R[a][b] = 0;
            for (int c = 0; c < 3; c++) R[a][b] += T[a][c] * Rx[c][b];
        }
}

/* level set: > 0 in the fluid, <= 0 in the body */
static double levelset(const or_geom* g, const double x[3]) {
    const or_body* b = &g->body;
    switch (b->kind) {
    case OR_BODY_SPHERE: {
        double s = 0;
        for (int d = 0; d < 3; d++) s += (x[d] - b->center[d]) * (x[d] - b->center[d]);
        return s - b->radii[0] * b->radii[0];
    }
    case OR_BODY_ELLIPSOID: {
        double s = 0;
        for (int a = 0; a < 3; a++) {
            double y = 0;
            for (int d = 0; d < 3; d++) y += g->R[d][a] * (x[d] - b->center[d]);
            s += (y / b->radii[a]) * (y / b->radii[a]);
        }
        return s - 1.0;
    }
    case OR_BODY_ZSLAB:
        return (x[2] - b->zlo) * (b->zhi - x[2]);
    case OR_BODY_PLANE:
        return b->plane_n[0] * x[0] + b->plane_n[1] * x[1] + b->plane_n[2] * x[2] - b->plane_d;
    case OR_BODY_CYLINDER: /* axis along y through the centre */
        return (x[0] - b->center[0]) * (x[0] - b->center[0]) +
               (x[2] - b->center[2]) * (x[2] - b->center[2]) - b->radii[0] * b->radii[0];
    case OR_BODY_CAVITY: { /* fluid inside the sphere, body outside */
        double s = 0;
        for (int d = 0; d < 3; d++) s += (x[d] - b->center[d]) * (x[d] - b->center[d]);
        return b->radii[0] * b->radii[0] - s;
    }
    default:
        return 1.0;
    }
}

/* the level set along x0 + t*h*e_d is the quadratic A t^2 + B t + psi(x0) */
static void levelset_edge(const or_geom* g, const double x0[3], int d, double* A, double* B) {
    const or_body* b = &g->body;
    double h = g->box.h;
    *A = 0;
    *B = 0;
    switch (b->kind) {
    case OR_BODY_SPHERE:
        *A = h * h;
        *B = 2 * h * (x0[d] - b->center[d]);
        break;
    case OR_BODY_ELLIPSOID:
        for (int a = 0; a < 3; a++) {
            double y = 0;
            for (int e = 0; e < 3; e++) y += g->R[e][a] * (x0[e] - b->center[e]);
            double ra2 = b->radii[a] * b->radii[a];
            *A += h * h * g->R[d][a] * g->R[d][a] / ra2;
            *B += 2 * h * y * g->R[d][a] / ra2;
        }
        break;
    case OR_BODY_ZSLAB:
        if (d == 2) {
            *A = -h * h;
            *B = h * (b->zhi + b->zlo - 2 * x0[2]);
        }
        break;
    case OR_BODY_PLANE:
        *B = h * b->plane_n[d];
        break;
    case OR_BODY_CYLINDER:
        if (d != 1) {
            *A = h * h;
            *B = 2 * h * (x0[d] - b->center[d]);
        }
        break;
    case OR_BODY_CAVITY:
        *A = -h * h;
        *B = -2 * h * (x0[d] - b->center[d]);
        break;
    default:
        break;
    }
}

/* root in [0,1] of A t^2 + B t + C, given psi(0) = C and psi(1) = C1 of different fluid state */
static double edge_root(double A, double B, double C, double C1) {
    if (C == 0.0) return 0.0;
    if (C1 == 0.0) return 1.0;
    double t;
    if (A == 0.0) {
        t = -C / B;
    } else {
        double disc = B * B - 4 * A * C;
        if (disc < 0) disc = 0;
        double q = -0.5 * (B + (B >= 0 ? sqrt(disc) : -sqrt(disc)));
        double r1 = q / A;
        double r2 = (q != 0.0) ? C / q : r1;
        int in1 = (r1 >= 0.0 && r1 <= 1.0), in2 = (r2 >= 0.0 && r2 <= 1.0);
        if (in1 && !in2) t = r1;
        else if (in2 && !in1) t = r2;
        else if (in1 && in2) t = (fabs(r1 - 0.5) <= fabs(r2 - 0.5)) ? r1 : r2;
        else {
            double e1 = r1 < 0 ? -r1 : r1 - 1, e2 = r2 < 0 ? -r2 : r2 - 1;
            t = (e1 <= e2) ? r1 : r2;
        }
    }
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    return t;
}

static long node_idx(const int n[3], int i, int j, int k) {
    return (long)i + (long)(n[0] + 1) * ((long)j + (long)(n[1] + 1) * (long)k);
}

/* is the edge from node q along d cut?  If so return 1 and the fraction t of the cut point */
static int edge_cut(const or_geom* g, const double* psi, const int q[3], int d, double* t) {
    const int* n = g->box.n;
    int q1[3] = {q[0], q[1], q[2]};
    q1[d] += 1;
    double p0 = psi[node_idx(n, q[0], q[1], q[2])];
    double p1 = psi[node_idx(n, q1[0], q1[1], q1[2])];
    if ((p0 > 0) == (p1 > 0)) return 0;
    double x0[3];
    for (int e = 0; e < 3; e++) x0[e] = g->box.lo[e] + q[e] * g->box.h;
    double A, B;
    levelset_edge(g, x0, d, &A, &B);
    *t = edge_root(A, B, p0, p1);
    return 1;
}

/* fluid area fraction of the face normal to d whose lower corner is node q (Sec. III.B) */
static double face_area(const or_geom* g, const double* psi, int d, const int q[3], int* amb) {
    const int* n = g->box.n;
    int t1, t2;
    others(d, &t1, &t2);
    int c[4][3];
    for (int m = 0; m < 4; m++)
        for (int e = 0; e < 3; e++) c[m][e] = q[e];
    c[1][t1] += 1;
    c[2][t1] += 1;
    c[2][t2] += 1;
    c[3][t2] += 1;
    int f[4];
    for (int m = 0; m < 4; m++) f[m] = psi[node_idx(n, c[m][0], c[m][1], c[m][2])] > 0;
    if (f[0] && f[1] && f[2] && f[3]) return 1.0;
    if (!f[0] && !f[1] && !f[2] && !f[3]) return 0.0;
    double px[12], py[12];
    int np = 0, ncut = 0;
    double t;
    static const double cx[4] = {0, 1, 1, 0}, cy[4] = {0, 0, 1, 1};
    /* walk corners 0 -> 1 -> 2 -> 3 -> 0, adding fluid corners and cut points */
    for (int m = 0; m < 4; m++) {
        if (f[m]) {
            px[np] = cx[m];
            py[np] = cy[m];
            np++;
        }
        int m2 = (m + 1) & 3;
        if (f[m] != f[m2]) {
            /* each edge is evaluated from its lower node in the positive direction */
            if (m == 0) { edge_cut(g, psi, c[0], t1, &t); px[np] = t; py[np] = 0; }
            else if (m == 1) { edge_cut(g, psi, c[1], t2, &t); px[np] = 1; py[np] = t; }
            else if (m == 2) { edge_cut(g, psi, c[3], t1, &t); px[np] = t; py[np] = 1; }
            else { edge_cut(g, psi, c[0], t2, &t); px[np] = 0; py[np] = t; }
            np++;
            ncut++;
        }
    }
    if (ncut > 2) *amb = 1;
    double a = 0;
    for (int m = 0; m < np; m++) {
        int m2 = (m + 1) % np;
        a += px[m] * py[m2] - px[m2] * py[m];
    }
    return 0.5 * fabs(a);
}

/* centroid of the polygon where the plane n.x = s cuts the cube [-1/2,1/2]^3 */
static void plane_cube_centroid(const double nv[3], double s, double b[3]) {
    double pts[12][3];
    int np = 0;
    for (int d = 0; d < 3; d++) {
        int t1, t2;
        others(d, &t1, &t2);
        if (nv[d] == 0.0) continue;
        for (int o1 = 0; o1 < 2; o1++)
            for (int o2 = 0; o2 < 2; o2++) {
                double x[3];
                x[t1] = o1 - 0.5;
                x[t2] = o2 - 0.5;
                x[d] = (s - nv[t1] * x[t1] - nv[t2] * x[t2]) / nv[d];
                if (x[d] >= -0.5 && x[d] <= 0.5) {
                    for (int e = 0; e < 3; e++) pts[np][e] = x[e];
                    np++;
                }
            }
    }
    if (np == 0) {
        for (int e = 0; e < 3; e++) b[e] = s * nv[e];
        return;
    }
    double m0[3] = {0, 0, 0};
    for (int k = 0; k < np; k++)
        for (int e = 0; e < 3; e++) m0[e] += pts[k][e] / np;
    /* in-plane basis */
    double a0[3] = {0, 0, 0};
    int dmin = 0;
    for (int e = 1; e < 3; e++)
        if (fabs(nv[e]) < fabs(nv[dmin])) dmin = e;
    a0[dmin] = 1.0;
    double dot = a0[0] * nv[0] + a0[1] * nv[1] + a0[2] * nv[2];
    double u1[3], u2[3];
    for (int e = 0; e < 3; e++) u1[e] = a0[e] - dot * nv[e];
    double l = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
    for (int e = 0; e < 3; e++) u1[e] /= l;
    u2[0] = nv[1] * u1[2] - nv[2] * u1[1];
    u2[1] = nv[2] * u1[0] - nv[0] * u1[2];
    u2[2] = nv[0] * u1[1] - nv[1] * u1[0];
    double ang[12];
    for (int k = 0; k < np; k++) {
        double x = 0, y = 0;
        for (int e = 0; e < 3; e++) {
            x += (pts[k][e] - m0[e]) * u1[e];
            y += (pts[k][e] - m0[e]) * u2[e];
        }
        ang[k] = atan2(y, x);
    }
    for (int k = 1; k < np; k++) { /* insertion sort by angle */
        double a = ang[k], p[3] = {pts[k][0], pts[k][1], pts[k][2]};
        int m = k - 1;
        while (m >= 0 && ang[m] > a) {
            ang[m + 1] = ang[m];
            for (int e = 0; e < 3; e++) pts[m + 1][e] = pts[m][e];
            m--;
        }
        ang[m + 1] = a;
        for (int e = 0; e < 3; e++) pts[m + 1][e] = p[e];
    }
    double area = 0, c[3] = {0, 0, 0};
    for (int k = 0; k < np; k++) {
        int k2 = (k + 1) % np;
        double v1[3], v2[3];
        for (int e = 0; e < 3; e++) {
            v1[e] = pts[k][e] - m0[e];
            v2[e] = pts[k2][e] - m0[e];
        }
        double cr[3] = {v1[1] * v2[2] - v1[2] * v2[1], v1[2] * v2[0] - v1[0] * v2[2],
                        v1[0] * v2[1] - v1[1] * v2[0]};
        double at = 0.5 * (cr[0] * nv[0] + cr[1] * nv[1] + cr[2] * nv[2]);
        area += at;
        for (int e = 0; e < 3; e++) c[e] += at * (m0[e] + pts[k][e] + pts[k2][e]) / 3.0;
    }
    if (fabs(area) < 1e-300) {
        for (int e = 0; e < 3; e++) b[e] = m0[e];
    } else {
        for (int e = 0; e < 3; e++) b[e] = c[e] / area;
    }
}

/* Lagrange weights on nodes -1, 0, +1 at position x (App. A, Eq. lagrange_polynomial) */
static void lagrange3(double x, double w[3]) {
    w[0] = (x - 0.0) * (x - 1.0) / ((-1.0 - 0.0) * (-1.0 - 1.0));
    w[1] = (x + 1.0) * (x - 1.0) / ((0.0 + 1.0) * (0.0 - 1.0));
    w[2] = (x + 1.0) * (x - 0.0) / ((1.0 + 1.0) * (1.0 - 0.0));
}

/* wall-flux stencil of one cut cell (Sec. III.B.3, Eqs. interpolation_distances, dudn) */
static int build_wall_stencil(or_geom* g, int cid) {
    const int* n = g->box.n;
    const int* per = g->box.periodic;
    long cell = g->cut[cid];
    int q[3];
    cell_ijk(n, cell, q);
    const double* nv = &g->nrm[3 * cid];
    const double* b = &g->bc[3 * cid];
    int ds = 0;
    for (int d = 1; d < 3; d++)
        if (fabs(nv[d]) > fabs(nv[ds])) ds = d;
    int s = nv[ds] > 0 ? 1 : -1;
    int t1, t2;
    others(ds, &t1, &t2);
    for (int kk = 1; kk <= 2; kk++) {
        double dk = (kk * s - b[ds]) / nv[ds];
        g->dd[2 * cid + kk - 1] = dk;
        double p[3];
        for (int e = 0; e < 3; e++) p[e] = b[e] + dk * nv[e];
        int c1 = (int)floor(p[t1] + 0.5), c2 = (int)floor(p[t2] + 0.5);
        int ok = 0;
        for (int attempt = 0; attempt < 2 && !ok; attempt++) {
            if (attempt == 1) {
                c1 += (nv[t1] > 0) - (nv[t1] < 0);
                c2 += (nv[t2] > 0) - (nv[t2] < 0);
            }
            ok = 1;
            for (int m1 = -1; m1 <= 1; m1++)
                for (int m2 = -1; m2 <= 1; m2++) {
                    int r[3];
                    r[ds] = q[ds] + kk * s;
                    r[t1] = q[t1] + c1 + m1;
                    r[t2] = q[t2] + c2 + m2;
                    long cc = cell_at(n, per, r);
                    if (cc < 0) return OR_EGEOM;
                    if (g->alpha[cc] <= 0.0) ok = 0;
                }
        }
        double w1[3], w2[3];
        lagrange3(p[t1] - c1, w1);
        lagrange3(p[t2] - c2, w2);
        for (int m1 = -1; m1 <= 1; m1++)
            for (int m2 = -1; m2 <= 1; m2++) {
                int r[3];
                r[ds] = q[ds] + kk * s;
                r[t1] = q[t1] + c1 + m1;
                r[t2] = q[t2] + c2 + m2;
                long cc = cell_at(n, per, r);
                long slot = ((long)cid * 2 + (kk - 1)) * 9 + (m1 + 1) * 3 + (m2 + 1);
                g->sw[slot] = w1[m1 + 1] * w2[m2 + 1];
                g->sidx[slot] = (g->alpha[cc] > 0.0) ? cc : -1;
            }
        if (!ok) {
            g->nfallback++;
            g->nfb[cid]++;
        }
    }
    return OR_OK;
}

static void build_levels(or_geom* g) {
    level_t* L0 = &g->lev[0];
    memcpy(L0->n, g->box.n, sizeof(L0->n));
    L0->N = g->N;
    L0->h = g->box.h;
    L0->alpha = g->alpha;
    for (int d = 0; d < 3; d++) L0->ap[d] = g->ap[d];
    g->nlev = 1;
    for (;;) {
        level_t* F = &g->lev[g->nlev - 1];
        int can = g->nlev < MAXLEV;
        for (int d = 0; d < 3; d++)
            if (F->n[d] % 4 != 0) can = 0;
        if (!can) break;
        level_t* Cl = &g->lev[g->nlev];
        for (int d = 0; d < 3; d++) Cl->n[d] = F->n[d] / 2;
        Cl->N = (long)Cl->n[0] * Cl->n[1] * Cl->n[2];
        Cl->h = 2 * F->h;
        Cl->alpha = calloc(Cl->N, sizeof(double));
        for (int k = 0; k < Cl->n[2]; k++)
            for (int j = 0; j < Cl->n[1]; j++)
                for (int i = 0; i < Cl->n[0]; i++) {
                    double s = 0;
                    for (int c = 0; c < 8; c++)
                        s += F->alpha[cidx(F->n, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1),
                                           2 * k + ((c >> 2) & 1))];
                    Cl->alpha[cidx(Cl->n, i, j, k)] = s / 8.0;
                }
        for (int d = 0; d < 3; d++) {
            int t1, t2;
            others(d, &t1, &t2);
            Cl->ap[d] = calloc(nfaces(Cl->n, d), sizeof(double));
            int m[3] = {Cl->n[0] + (d == 0), Cl->n[1] + (d == 1), Cl->n[2] + (d == 2)};
            for (int k = 0; k < m[2]; k++)
                for (int j = 0; j < m[1]; j++)
                    for (int i = 0; i < m[0]; i++) {
                        int q[3] = {i, j, k};
                        double s = 0;
                        for (int o1 = 0; o1 < 2; o1++)
                            for (int o2 = 0; o2 < 2; o2++) {
                                int r[3];
                                r[d] = 2 * q[d];
                                r[t1] = 2 * q[t1] + o1;
                                r[t2] = 2 * q[t2] + o2;
                                s += F->ap[d][fidx(F->n, d, r[0], r[1], r[2])];
                            }
                        Cl->ap[d][fidx(Cl->n, d, i, j, k)] = s / 4.0;
                    }
        }
        g->nlev++;
    }
    for (int l = 0; l < g->nlev; l++) {
        level_t* L = &g->lev[l];
        L->mask = calloc(L->N, 1);
        for (long c = 0; c < L->N; c++) L->mask[c] = L->alpha[c] > 0.0;
        for (int d = 0; d < 3; d++) L->K[d] = calloc(nfaces(L->n, d), sizeof(double));
        L->S = calloc(L->N, sizeof(double));
        L->D = calloc(L->N, sizeof(double));
    }
}

or_geom* or_geom_build(const or_box* box, const or_body* body, int* err) {
    *err = OR_OK;
    for (int d = 0; d < 3; d++)
        if (box->n[d] < 2 || box->n[d] % 2 != 0) {
            *err = OR_EINVAL;
            return NULL;
        }
    if (!(box->h > 0)) {
        *err = OR_EINVAL;
        return NULL;
    }
    or_geom* g = calloc(1, sizeof(or_geom));
    g->box = *box;
    g->body = *body;
    if (body->kind == OR_BODY_ELLIPSOID) rotation_zyx(body->euler_zyx, g->R);
    const int* n = box->n;
    g->N = (long)n[0] * n[1] * n[2];
    long nn = (long)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
    double* psi = malloc(nn * sizeof(double));
    for (int k = 0; k <= n[2]; k++)
        for (int j = 0; j <= n[1]; j++)
            for (int i = 0; i <= n[0]; i++) {
                double x[3] = {box->lo[0] + i * box->h, box->lo[1] + j * box->h,
                               box->lo[2] + k * box->h};
                psi[node_idx(n, i, j, k)] = levelset(g, x);
            }
    /* face apertures */
    int amb = 0;
    for (int d = 0; d < 3; d++) {
        g->ap[d] = calloc(nfaces(n, d), sizeof(double));
        int m[3] = {n[0] + (d == 0), n[1] + (d == 1), n[2] + (d == 2)};
        for (int k = 0; k < m[2]; k++)
            for (int j = 0; j < m[1]; j++)
                for (int i = 0; i < m[0]; i++) {
                    int q[3] = {i, j, k};
                    g->ap[d][fidx(n, d, i, j, k)] = face_area(g, psi, d, q, &amb);
                }
        if (box->periodic[d]) { /* the last face is the first one */
            for (int k = 0; k < m[2]; k++)
                for (int j = 0; j < m[1]; j++)
                    for (int i = 0; i < m[0]; i++) {
                        int q[3] = {i, j, k};
                        if (q[d] != n[d]) continue;
                        int q0[3] = {i, j, k};
                        q0[d] = 0;
                        g->ap[d][fidx(n, d, i, j, k)] = g->ap[d][fidx(n, d, q0[0], q0[1], q0[2])];
                    }
        }
    }
    /* cells */
    g->flag = calloc(g->N, 1);
    g->alpha = calloc(g->N, sizeof(double));
    g->cutid = malloc(g->N * sizeof(long));
    double* tmp_n = malloc(g->N * 3 * sizeof(double)); /* sized generously, trimmed below */
    double* tmp_a = malloc(g->N * sizeof(double));
    double* tmp_b = malloc(g->N * 3 * sizeof(double));
    double* tmp_s = malloc(g->N * sizeof(double));
    long* tmp_c = malloc(g->N * sizeof(long));
    int ncut = 0;
    for (int k = 0; k < n[2]; k++)
        for (int j = 0; j < n[1]; j++)
            for (int i = 0; i < n[0]; i++) {
                long c = cidx(n, i, j, k);
                int q[3] = {i, j, k};
                double a[3][2];
                int all1 = 1, all0 = 1;
                double sumA = 0;
                for (int d = 0; d < 3; d++)
                    for (int s = 0; s < 2; s++) {
                        int r[3] = {i, j, k};
                        r[d] += s;
                        a[d][s] = g->ap[d][fidx(n, d, r[0], r[1], r[2])];
                        if (a[d][s] != 1.0) all1 = 0;
                        if (a[d][s] != 0.0) all0 = 0;
                        sumA += a[d][s];
                    }
                g->cutid[c] = -1;
                if (all1) {
                    g->flag[c] = 2;
                    g->alpha[c] = 1.0;
                    continue;
                }
                if (all0) {
                    g->flag[c] = 0;
                    g->alpha[c] = 0.0;
                    continue;
                }
                double m[3], aeb = 0;
                for (int d = 0; d < 3; d++) {
                    m[d] = a[d][1] - a[d][0];
                    aeb += m[d] * m[d];
                }
                aeb = sqrt(aeb);
                if (aeb == 0.0) {
                    *err = OR_EGEOM;
                    continue;
                }
                double nv[3] = {m[0] / aeb, m[1] / aeb, m[2] / aeb};
                /* plane offset: mean of n.p over the cut points on the 12 cell edges */
                double ssum = 0;
                int npt = 0;
                for (int d = 0; d < 3; d++) {
                    int t1, t2;
                    others(d, &t1, &t2);
                    for (int o1 = 0; o1 < 2; o1++)
                        for (int o2 = 0; o2 < 2; o2++) {
                            int r[3] = {q[0], q[1], q[2]};
                            r[t1] += o1;
                            r[t2] += o2;
                            double t;
                            if (edge_cut(g, psi, r, d, &t)) {
                                double p[3];
                                p[d] = t - 0.5;
                                p[t1] = o1 - 0.5;
                                p[t2] = o2 - 0.5;
                                ssum += nv[0] * p[0] + nv[1] * p[1] + nv[2] * p[2];
                                npt++;
                            }
                        }
                }
                double s = npt > 0 ? ssum / npt : 0.0;
                /* divergence theorem with x.n: 3V = sum_f A_f/2 - s A_EB (cell units) */
                double al = (0.5 * sumA - s * aeb) / 3.0;
                if (al > 1.0) al = 1.0;
                if (al < 1e-12) al = 1e-12;
                g->flag[c] = 1;
                g->alpha[c] = al;
                g->cutid[c] = ncut;
                tmp_c[ncut] = c;
                for (int e = 0; e < 3; e++) tmp_n[3 * ncut + e] = nv[e];
                tmp_a[ncut] = aeb;
                double b[3];
                plane_cube_centroid(nv, s, b);
                for (int e = 0; e < 3; e++) tmp_b[3 * ncut + e] = b[e];
                tmp_s[ncut] = -s;
                ncut++;
            }
    if (amb) *err = OR_EGEOM;
    g->ncut = ncut;
    long nc = ncut > 0 ? ncut : 1;
    g->cut = malloc(nc * sizeof(long));
    g->nrm = malloc(nc * 3 * sizeof(double));
    g->aeb = malloc(nc * sizeof(double));
    g->bc = malloc(nc * 3 * sizeof(double));
    g->delta = malloc(nc * sizeof(double));
    memcpy(g->cut, tmp_c, ncut * sizeof(long));
    memcpy(g->nrm, tmp_n, ncut * 3 * sizeof(double));
    memcpy(g->aeb, tmp_a, ncut * sizeof(double));
    memcpy(g->bc, tmp_b, ncut * 3 * sizeof(double));
    memcpy(g->delta, tmp_s, ncut * sizeof(double));
    free(tmp_c);
    free(tmp_n);
    free(tmp_a);
    free(tmp_b);
    free(tmp_s);
    free(psi);
    g->dd = calloc(nc * 2, sizeof(double));
    g->sidx = calloc(nc * 18, sizeof(long));
    g->sw = calloc(nc * 18, sizeof(double));
    g->nfb = calloc(nc, sizeof(int));
    for (int c = 0; c < ncut; c++) {
        int e = build_wall_stencil(g, c);
        if (e != OR_OK) *err = e;
    }
    build_levels(g);
    return g;
}

void or_geom_free(or_geom* g) {
    if (!g) return;
    for (int l = 0; l < g->nlev; l++) {
        level_t* L = &g->lev[l];
        if (l > 0) {
            free(L->alpha);
            for (int d = 0; d < 3; d++) free(L->ap[d]);
        }
        free(L->mask);
        for (int d = 0; d < 3; d++) free(L->K[d]);
        free(L->S);
        free(L->D);
    }
    free(g->flag);
    free(g->alpha);
    for (int d = 0; d < 3; d++) free(g->ap[d]);
    free(g->cut);
    free(g->cutid);
    free(g->nrm);
    free(g->aeb);
    free(g->bc);
    free(g->delta);
    free(g->dd);
    free(g->sidx);
    free(g->sw);
    free(g->nfb);
    free(g);
}

int or_geom_ncut(const or_geom* g) { return g->ncut; }
int or_geom_nlevels(const or_geom* g) { return g->nlev; }
int or_geom_nfallback(const or_geom* g) { return g->nfallback; }

void or_geom_export(const or_geom* g, uint8_t* flag, double* alpha, double* ax, double* ay,
                    double* az) {
    memcpy(flag, g->flag, g->N);
    memcpy(alpha, g->alpha, g->N * sizeof(double));
    memcpy(ax, g->ap[0], nfaces(g->box.n, 0) * sizeof(double));
    memcpy(ay, g->ap[1], nfaces(g->box.n, 1) * sizeof(double));
    memcpy(az, g->ap[2], nfaces(g->box.n, 2) * sizeof(double));
}

void or_cut_export(const or_geom* g, int64_t* cell, double* data) {
    for (int c = 0; c < g->ncut; c++) {
        cell[c] = g->cut[c];
        for (int e = 0; e < 3; e++) data[9 * c + e] = g->nrm[3 * c + e];
        data[9 * c + 3] = g->aeb[c];
        for (int e = 0; e < 3; e++) data[9 * c + 4 + e] = g->bc[3 * c + e];
        data[9 * c + 7] = g->delta[c];
        data[9 * c + 8] = g->nfb[c];
    }
}

/* ------------------------------------------------------------------------------------------ */
/* wall gradient (Eq. dudn) and cell gradients (one-sided quadratic differences, Sec. III.B.4)  */
/* ------------------------------------------------------------------------------------------ */
/* normal derivative of component j at the EB centroid of cut cell cid */
static double wall_dudn(const or_geom* g, int cid, const double* uj, double ueb) {
    double ui[2];
    for (int kk = 0; kk < 2; kk++) {
        double s = 0;
        for (int m = 0; m < 9; m++) {
            long slot = ((long)cid * 2 + kk) * 9 + m;
            long cc = g->sidx[slot];
            s += g->sw[slot] * (cc >= 0 ? uj[cc] : ueb);
        }
        ui[kk] = s;
    }
    double d1 = g->dd[2 * cid], d2 = g->dd[2 * cid + 1];
    return (d2 * d2 * (ui[0] - ueb) - d1 * d1 * (ui[1] - ueb)) / (d1 * d2 * (d2 - d1) * g->box.h);
}

void or_wall_gradient(const or_geom* g, const double* u, double* gw) {
    for (int c = 0; c < g->ncut; c++)
        for (int j = 0; j < 3; j++)
            gw[3 * c + j] = wall_dudn(g, c, u + (long)j * g->N, g->body.u_eb[j]);
}

void or_cell_gradient(const or_geom* g, const double* u, const double* gw, double* G) {
    const int* n = g->box.n;
    const int* per = g->box.periodic;
    long N = g->N;
    double h = g->box.h;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; c++) {
        for (int a = 0; a < 9; a++) G[a * N + c] = 0.0;
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int d = 0; d < 3; d++) {
            int r[3];
            memcpy(r, q, sizeof(r));
            r[d] = q[d] - 1;
            long lo = cell_at(n, per, r);
            r[d] = q[d] - 2;
            long lo2 = cell_at(n, per, r);
            r[d] = q[d] + 1;
            long hi = cell_at(n, per, r);
            r[d] = q[d] + 2;
            long hi2 = cell_at(n, per, r);
            int lo_wall = lo < 0, hi_wall = hi < 0;
            int lo_open = !lo_wall && g->alpha[lo] > 0.0;
            int hi_open = !hi_wall && g->alpha[hi] > 0.0;
            int lo2_open = lo2 >= 0 && g->alpha[lo2] > 0.0;
            int hi2_open = hi2 >= 0 && g->alpha[hi2] > 0.0;
            for (int j = 0; j < 3; j++) {
                const double* uj = u + (long)j * N;
                double uc = uj[c];
                /* Dirichlet domain walls enter through the ghost value 2 u_wall - u_c */
                double vlo = lo_open ? uj[lo] : 2.0 * g->box.wall_u[2 * d][j] - uc;
                double vhi = hi_open ? uj[hi] : 2.0 * g->box.wall_u[2 * d + 1][j] - uc;
                int lo_ok = lo_open || lo_wall, hi_ok = hi_open || hi_wall;
                double gr;
                if (lo_ok && hi_ok) {
                    gr = (vhi - vlo) / (2.0 * h);
                } else if (hi_ok) {
                    if (hi_open && hi2_open)
                        gr = (-1.5 * uc + 2.0 * vhi - 0.5 * uj[hi2]) / h;
                    else
                        gr = (vhi - uc) / h;
                } else if (lo_ok) {
                    if (lo_open && lo2_open)
                        gr = (1.5 * uc - 2.0 * vlo + 0.5 * uj[lo2]) / h;
                    else
                        gr = (uc - vlo) / h;
                } else {
                    long cid = g->cutid[c];
                    gr = (cid >= 0) ? g->nrm[3 * cid + d] * gw[3 * cid + j] : 0.0;
                }
                G[(d * 3 + j) * N + c] = gr;
            }
        }
    }
}

/* scaled Frobenius norm of gamma = G + G^T (Sec. II.A) */
static double strain_norm(const double Gm[3][3]) {
    double s = 0;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double y = Gm[a][b] + Gm[b][a];
            s += y * y;
        }
    return sqrt(0.5 * s);
}

/* the power-law term kappa s^(n-1) of Table rheology (Ostwald-de Waele); for n < 1 it grows
 * without bound as the strain rate goes to zero, and s = max(sr, eps) caps it (a reading: the
 * paper does not say how its code bounds the term); for n >= 1, s = sr */
static double power_term(const or_rheo* r, double sr) {
    double s = (r->n < 1.0 && sr < r->eps) ? r->eps : sr;
    return r->kappa * pow(s, r->n - 1.0);
}

/* apparent viscosity laws (Table rheology, Eq. papabing:viscosity).  The Papanastasiou factor
 * (1 - exp(-x))/sr is written -expm1(-x)/sr, with its limit at sr = 0; Herschel-Bulkley adds it
 * (x = sr/eps) to the power-law term, Souza Mendes-Dutra uses x = eta0 sr/tau0 (limit eta0). */
static double law_eta(const or_rheo* r, double tau0, double sr) {
    switch (r->law) {
    case OR_LAW_NEWTONIAN:
        return r->mu;
    case OR_LAW_BINGHAM_REG:
        if (tau0 == 0.0) return r->mu;
        return r->mu + tau0 / (sr + r->eps);
    case OR_LAW_PAPANASTASIOU:
        if (tau0 == 0.0) return r->mu;
        if (sr == 0.0) return r->mu + tau0 / r->eps;
        return r->mu + tau0 * (-expm1(-sr / r->eps)) / sr;
    case OR_LAW_POWER:
        return power_term(r, sr);
    case OR_LAW_HERSCHEL_BULKLEY: {
        double pw = power_term(r, sr);
        if (tau0 == 0.0) return pw;
        if (sr == 0.0) return pw + tau0 / r->eps;
        return pw + tau0 * (-expm1(-sr / r->eps)) / sr;
    }
    default: { /* OR_LAW_SOUZA_MENDES_DUTRA */
        double pw = power_term(r, sr);
        if (tau0 == 0.0) return pw;
        if (sr == 0.0) return pw + r->eta0;
        return pw + tau0 * (-expm1(-r->eta0 * sr / tau0)) / sr;
    }
    }
}

static void viscosity_from(const or_geom* g, const or_rheo* r, const double* theta,
                           const double* G, const double* gw, double* eta, double* eta_eb,
                           double* sr) {
    long N = g->N;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; c++) {
        if (g->alpha[c] <= 0.0) {
            eta[c] = r->mu;
            if (sr) sr[c] = 0.0;
            continue;
        }
        double Gm[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Gm[a][b] = G[(a * 3 + b) * N + c];
        double s = strain_norm(Gm);
        double t0 = r->tau0 * (theta ? theta[c] : 1.0);
        eta[c] = law_eta(r, t0, s);
        if (sr) sr[c] = s;
    }
    for (int cid = 0; cid < g->ncut; cid++) {
        long c = g->cut[cid];
        double Gm[3][3]; /* gradient at the wall: (grad u)_ab = n_a du_b/dn */
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Gm[a][b] = g->nrm[3 * cid + a] * gw[3 * cid + b];
        double s = strain_norm(Gm);
        double t0 = r->tau0 * (theta ? theta[c] : 1.0);
        eta_eb[cid] = law_eta(r, t0, s);
    }
}

void or_viscosity(const or_geom* g, const or_rheo* r, const double* u, const double* theta,
                  double* eta, double* eta_eb, double* sr) {
    double* gw = calloc(3 * (g->ncut + 1), sizeof(double));
    double* G = malloc(9 * g->N * sizeof(double));
    or_wall_gradient(g, u, gw);
    or_cell_gradient(g, u, gw, G);
    viscosity_from(g, r, theta, G, gw, eta, eta_eb, sr);
    free(G);
    free(gw);
}

/* ------------------------------------------------------------------------------------------ */
/* redistribution (Eqs. divergence_nonconservative ... divergence_final)                        */
/* ------------------------------------------------------------------------------------------ */
void or_redistribute(const or_geom* g, int ncomp, const double* DC, double* D) {
    const int* n = g->box.n;
    const int* per = g->box.periodic;
    long N = g->N;
    double* S = calloc(N, sizeof(double));
    double* dD = calloc((long)ncomp * N, sizeof(double));
    double* DH = calloc((long)ncomp * N, sizeof(double));
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; c++) {
        if (g->alpha[c] <= 0.0) continue;
        double a = g->alpha[c];
        if (g->flag[c] != 1) {
            for (int m = 0; m < ncomp; m++) DH[m * N + c] = DC[m * N + c];
            continue;
        }
        int q[3];
        cell_ijk(n, c, q);
        double s = 0, acc[3] = {0, 0, 0};
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    if (!dx && !dy && !dz) continue;
                    int r[3] = {q[0] + dx, q[1] + dy, q[2] + dz};
                    long cc = cell_at(n, per, r);
                    if (cc < 0 || g->alpha[cc] <= 0.0) continue;
                    s += g->alpha[cc];
                    for (int m = 0; m < ncomp; m++) acc[m] += g->alpha[cc] * DC[m * N + cc];
                }
        S[c] = s;
        for (int m = 0; m < ncomp; m++) {
            double dnc = s > 0 ? acc[m] / s : DC[m * N + c];
            DH[m * N + c] = a * DC[m * N + c] + (1.0 - a) * dnc;
            dD[m * N + c] = a * (1.0 - a) * (DC[m * N + c] - dnc);
        }
    }
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; c++) {
        for (int m = 0; m < ncomp; m++) D[m * N + c] = 0.0;
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        double acc[3] = {0, 0, 0};
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    if (!dx && !dy && !dz) continue;
                    int r[3] = {q[0] + dx, q[1] + dy, q[2] + dz};
                    long cc = cell_at(n, per, r);
                    if (cc < 0 || g->flag[cc] != 1 || S[cc] <= 0.0) continue;
                    for (int m = 0; m < ncomp; m++) acc[m] += dD[m * N + cc] / S[cc];
                }
        for (int m = 0; m < ncomp; m++) D[m * N + c] = DH[m * N + c] + acc[m];
    }
    free(S);
    free(dD);
    free(DH);
}

/* ------------------------------------------------------------------------------------------ */
/* explicit viscous term  V = div(eta (grad u)^T)  (Eq. explicit-viscous, Sec. III.B.3)         */
/* ------------------------------------------------------------------------------------------ */
static void transpose_term_dc(const or_geom* g, const double* eta, const double* eta_eb,
                              const double* u, const double* G, const double* gw, double* DC) {
    const int* n = g->box.n;
    const int* per = g->box.periodic;
    long N = g->N;
    double h = g->box.h;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; c++) {
        for (int j = 0; j < 3; j++) DC[j * N + c] = 0.0;
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int j = 0; j < 3; j++) {
            double acc = 0;
            for (int d = 0; d < 3; d++)
                for (int side = -1; side <= 1; side += 2) {
                    int f[3] = {q[0], q[1], q[2]};
                    if (side > 0) f[d] += 1;
                    double A = g->ap[d][fidx(n, d, f[0], f[1], f[2])];
                    if (A == 0.0) continue;
                    int r[3] = {q[0], q[1], q[2]};
                    r[d] += side;
                    long nb = cell_at(n, per, r);
                    const double* ud = u + (long)d * N;
                    double F;
                    if (nb >= 0) {
                        double ef = 0.5 * (eta[c] + eta[nb]);
                        double der;
                        if (j == d)
                            der = side > 0 ? (ud[nb] - ud[c]) / h : (ud[c] - ud[nb]) / h;
                        else
                            der = 0.5 * (G[(j * 3 + d) * N + c] + G[(j * 3 + d) * N + nb]);
                        F = ef * der;
                    } else {
                        double uw = g->box.wall_u[2 * d + (side > 0)][d];
                        double der = 0.0;
                        if (j == d)
                            der = side > 0 ? (uw - ud[c]) / (0.5 * h) : (ud[c] - uw) / (0.5 * h);
                        F = eta[c] * der;
                    }
                    acc += side * A * F;
                }
            long cid = g->cutid[c];
            if (cid >= 0) {
                const double* nv = &g->nrm[3 * cid];
                double ng = nv[0] * gw[3 * cid] + nv[1] * gw[3 * cid + 1] + nv[2] * gw[3 * cid + 2];
                acc -= g->aeb[cid] * eta_eb[cid] * nv[j] * ng;
            }
            DC[j * N + c] = acc / (g->alpha[c] * h);
        }
    }
}

void or_transpose_term(const or_geom* g, const double* eta, const double* eta_eb,
                       const double* u, double* V) {
    long N = g->N;
    double* gw = calloc(3 * (g->ncut + 1), sizeof(double));
    double* G = malloc(9 * N * sizeof(double));
    double* DC = malloc(3 * N * sizeof(double));
    or_wall_gradient(g, u, gw);
    or_cell_gradient(g, u, gw, G);
    transpose_term_dc(g, eta, eta_eb, u, G, gw, DC);
    or_redistribute(g, 3, DC, V);
    free(DC);
    free(G);
    free(gw);
}

/* ------------------------------------------------------------------------------------------ */
/* slopes, face extrapolation and upwinding (Sec. III.A.3, Alg. derived lines 1-2)              */
/* ------------------------------------------------------------------------------------------ */
/* monotonised-central limited slope of component j along d at cell c (0 next to walls/covered) */
static double mc_slope(const or_geom* g, const double* uj, long c, int d) {
    const int* n = g->box.n;
    int q[3];
    cell_ijk(n, c, q);
    int r[3];
    memcpy(r, q, sizeof(r));
    r[d] = q[d] - 1;
    long lo = cell_at(n, g->box.periodic, r);
    r[d] = q[d] + 1;
    long hi = cell_at(n, g->box.periodic, r);
    if (lo < 0 || hi < 0) return 0.0;
    if (g->alpha[lo] <= 0.0 || g->alpha[hi] <= 0.0) return 0.0;
    double dl = uj[c] - uj[lo], dr = uj[hi] - uj[c], dc = 0.5 * (uj[hi] - uj[lo]);
    if (dl * dr <= 0.0) return 0.0;
    double m = fmin(fabs(dc), fmin(2.0 * fabs(dl), 2.0 * fabs(dr)));
    return dc > 0 ? m : -m;
}

/* left/right extrapolated states of component j on face (d, f) between cells lo and hi */
static void face_states(const or_geom* g, const double* uj, long lo, long hi, int d, double* uL,
                        double* uR) {
    *uL = uj[lo] + 0.5 * mc_slope(g, uj, lo, d);
    *uR = uj[hi] - 0.5 * mc_slope(g, uj, hi, d);
}

/* cells on either side of face (d, i,j,k); -1 where the face is a domain wall */
static void face_cells(const or_geom* g, int d, const int f[3], long* lo, long* hi) {
    int r[3] = {f[0], f[1], f[2]};
    r[d] = f[d] - 1;
    *lo = cell_at(g->box.n, g->box.periodic, r);
    r[d] = f[d];
    *hi = cell_at(g->box.n, g->box.periodic, r);
}

void or_face_extrap(const or_geom* g, const double* u, double* fx, double* fy, double* fz) {
    const int* n = g->box.n;
    double* fo[3] = {fx, fy, fz};
    for (int d = 0; d < 3; d++) {
        int m[3] = {n[0] + (d == 0), n[1] + (d == 1), n[2] + (d == 2)};
        for (int k = 0; k < m[2]; k++)
            for (int j = 0; j < m[1]; j++)
                for (int i = 0; i < m[0]; i++) {
                    int f[3] = {i, j, k};
                    long fi = fidx(n, d, i, j, k);
                    long lo, hi;
                    face_cells(g, d, f, &lo, &hi);
                    double A = g->ap[d][fi];
                    double val = 0.0;
                    if (lo < 0 || hi < 0) {
                        val = g->box.wall_u[2 * d + (lo >= 0)][d];
                    } else if (A > 0.0) {
                        double uL, uR;
                        face_states(g, u + (long)d * g->N, lo, hi, d, &uL, &uR);
                        if (uL > 0.0 && uL + uR > 0.0) val = uL;
                        else if (uR < 0.0 && uL + uR < 0.0) val = uR;
                        else val = 0.0;
                    }
                    fo[d][fi] = val;
                }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* convective term C = -div(u (x) u^F) with upwinding by the projected face velocity            */
/* ------------------------------------------------------------------------------------------ */
static void conv_dc(const or_geom* g, const double* u, double* const uf[3], double* DC) {
    const int* n = g->box.n;
    long N = g->N;
    double h = g->box.h;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; c++) {
        for (int j = 0; j < 3; j++) DC[j * N + c] = 0.0;
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int j = 0; j < 3; j++) {
            double acc = 0;
            for (int d = 0; d < 3; d++)
                for (int side = -1; side <= 1; side += 2) {
                    int f[3] = {q[0], q[1], q[2]};
                    if (side > 0) f[d] += 1;
                    long fi = fidx(n, d, f[0], f[1], f[2]);
                    double A = g->ap[d][fi];
                    if (A == 0.0) continue;
                    long lo, hi;
                    face_cells(g, d, f, &lo, &hi);
                    double w = uf[d][fi], up;
                    if (lo < 0 || hi < 0) {
                        up = g->box.wall_u[2 * d + (lo >= 0)][j];
                    } else {
                        double uL, uR;
                        face_states(g, u + (long)j * N, lo, hi, d, &uL, &uR);
                        up = w > 0.0 ? uL : (w < 0.0 ? uR : 0.5 * (uL + uR));
                    }
                    acc += side * A * w * up;
                }
            long cid = g->cutid[c];
            if (cid >= 0) { /* flux through a moving wall: u_EB (u_EB . n_out), n_out = -n */
                const double* nv = &g->nrm[3 * cid];
                const double* ue = g->body.u_eb;
                double un = -(ue[0] * nv[0] + ue[1] * nv[1] + ue[2] * nv[2]);
                acc += g->aeb[cid] * un * ue[j];
            }
            DC[j * N + c] = -acc / (g->alpha[c] * h);
        }
    }
}

void or_conv_term(const or_geom* g, const double* u, const double* uf_x, const double* uf_y,
                  const double* uf_z, double* C) {
    double* DC = malloc(3 * g->N * sizeof(double));
    double* uf[3] = {(double*)uf_x, (double*)uf_y, (double*)uf_z};
    conv_dc(g, u, uf, DC);
    or_redistribute(g, 3, DC, C);
    free(DC);
}

/* ------------------------------------------------------------------------------------------ */
/* divergence of a face field, cell-centred pressure gradient                                   */
/* ------------------------------------------------------------------------------------------ */
void or_divergence(const or_geom* g, const double* fx, const double* fy, const double* fz,
                   double* div) {
    const int* n = g->box.n;
    const double* fo[3] = {fx, fy, fz};
    double h = g->box.h;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < g->N; c++) {
        div[c] = 0.0;
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        double acc = 0;
        for (int d = 0; d < 3; d++) {
            int f[3] = {q[0], q[1], q[2]};
            long f0 = fidx(n, d, f[0], f[1], f[2]);
            f[d] += 1;
            long f1 = fidx(n, d, f[0], f[1], f[2]);
            acc += g->ap[d][f1] * fo[d][f1] - g->ap[d][f0] * fo[d][f0];
        }
        long cid = g->cutid[c];
        if (cid >= 0) {
            const double* nv = &g->nrm[3 * cid];
            const double* ue = g->body.u_eb;
            acc += -g->aeb[cid] * (ue[0] * nv[0] + ue[1] * nv[1] + ue[2] * nv[2]);
        }
        div[c] = acc / h;
    }
}

/* aperture-weighted average of the two face gradients in each direction */
void or_gcc(const or_geom* g, const double* p, double* gp) {
    const int* n = g->box.n;
    long N = g->N;
    double h = g->box.h;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; c++) {
        for (int d = 0; d < 3; d++) gp[d * N + c] = 0.0;
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int d = 0; d < 3; d++) {
            double num = 0, den = 0;
            for (int side = -1; side <= 1; side += 2) {
                int f[3] = {q[0], q[1], q[2]};
                if (side > 0) f[d] += 1;
                double A = g->ap[d][fidx(n, d, f[0], f[1], f[2])];
                if (A == 0.0) continue;
                long lo, hi;
                face_cells(g, d, f, &lo, &hi);
                double gf = (lo >= 0 && hi >= 0) ? (p[hi] - p[lo]) / h : 0.0;
                num += A * gf;
                den += A;
            }
            gp[d * N + c] = den > 0 ? num / den : 0.0;
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* 7-point operators and the multigrid preconditioner                                           */
/* ------------------------------------------------------------------------------------------ */
enum { SYS_POISSON = 0, SYS_VISC = 1 };

/* The viscous system's coarse face coefficient for one of the four fine faces f2 (at fine face
 * position r) that make up a coarse face normal to d.  The line of fine faces normal to the coarse
 * face through the two coarse cells it separates, f1 (inside the lower coarse cell), f2 and f3
 * (inside the upper one), joins the two coarse centres, so its viscosity acts in series: the
 * weighted harmonic mean H = W / sum(w_i / g_i), W = sum(w_i), of g_i = K_i / A_i (the face
 * coefficient without its aperture) over the open faces of the line, with weights 1/2, 1, 1/2
 * for the half of f1, all of f2 and the half of f3 that lie between the two centres.  A domain
 * wall face f2 has the inner face only, weights 1/2 and 1/2, and g_2 = K_2 / (2 A_2) (the ghost
 * factor of the wall flux removed).  The line contributes K_2 H / g_2: its aperture and spacing
 * as before, its viscosity in series.  With a uniform viscosity every g_i is g_2 and the line
 * contributes K_2, the plain sum of the four fine faces. */
static double series_line(const or_geom* g, const level_t* F, int d, const int r[3], int wall) {
    long f2 = fidx(F->n, d, r[0], r[1], r[2]);
    double K2 = F->K[d][f2], A2 = F->ap[d][f2];
    if (K2 == 0.0 || A2 == 0.0) return K2;
    double g2 = wall ? K2 / (2.0 * A2) : K2 / A2;
    double W = wall ? 0.5 : 1.0, R = W / g2;
    int per = g->box.periodic[d];
    for (int side = -1; side <= 1; side += 2) {
        int q[3] = {r[0], r[1], r[2]};
        q[d] += side;
        if (q[d] < 0 || q[d] > F->n[d]) {
            if (!per) continue; /* beyond a domain wall: the wall face has no outer neighbour */
            q[d] = q[d] < 0 ? q[d] + F->n[d] : q[d] - F->n[d];
        }
        long fi = fidx(F->n, d, q[0], q[1], q[2]);
        double K = F->K[d][fi], A = F->ap[d][fi];
        if (K > 0.0 && A > 0.0) {
            W += 0.5;
            R += 0.5 / (K / A);
        }
    }
    return K2 * (W / R) / g2;
}

/* level-0 face coefficients and cell shifts, then coarse levels by averaging */
static void build_operator(or_geom* g, int sys, double beta, double rho, double dt,
                           const double* eta, const double* eta_eb) {
    level_t* L0 = &g->lev[0];
    const int* n = g->box.n;
    double h = g->box.h;
    for (int d = 0; d < 3; d++) {
        int m[3] = {n[0] + (d == 0), n[1] + (d == 1), n[2] + (d == 2)};
        for (int k = 0; k < m[2]; k++)
            for (int j = 0; j < m[1]; j++)
                for (int i = 0; i < m[0]; i++) {
                    int f[3] = {i, j, k};
                    long fi = fidx(n, d, i, j, k);
                    long lo, hi;
                    face_cells(g, d, f, &lo, &hi);
                    double A = g->ap[d][fi], K = 0.0;
                    if (A > 0.0) {
                        if (sys == SYS_POISSON) {
                            K = (lo >= 0 && hi >= 0) ? beta * A / (h * h) : 0.0;
                        } else {
                            if (lo >= 0 && hi >= 0)
                                K = dt * A * 0.5 * (eta[lo] + eta[hi]) / (h * h);
                            else
                                K = 2.0 * dt * A * eta[lo >= 0 ? lo : hi] / (h * h);
                        }
                    }
                    L0->K[d][fi] = K;
                }
    }
    for (long c = 0; c < g->N; c++) {
        double s = 0.0;
        if (sys == SYS_VISC && g->alpha[c] > 0.0) {
            s = g->alpha[c] * rho;
            long cid = g->cutid[c];
            if (cid >= 0)  /* the wall flux of a linear profile seen two cells from the wall */
                s += dt * g->aeb[cid] * eta_eb[cid] / (2.0 * h * h);
        }
        L0->S[c] = s;
    }
    for (int l = 1; l < g->nlev; l++) {
        level_t* F = &g->lev[l - 1];
        level_t* C = &g->lev[l];
        for (int d = 0; d < 3; d++) {
            int t1, t2;
            others(d, &t1, &t2);
            int m[3] = {C->n[0] + (d == 0), C->n[1] + (d == 1), C->n[2] + (d == 2)};
            for (int k = 0; k < m[2]; k++)
                for (int j = 0; j < m[1]; j++)
                    for (int i = 0; i < m[0]; i++) {
                        int q[3] = {i, j, k};
                        double s = 0;
                        int wall = !g->box.periodic[d] && (q[d] == 0 || q[d] == C->n[d]);
                        for (int o1 = 0; o1 < 2; o1++)
                            for (int o2 = 0; o2 < 2; o2++) {
                                int r[3];
                                r[d] = 2 * q[d];
                                r[t1] = 2 * q[t1] + o1;
                                r[t2] = 2 * q[t2] + o2;
                                s += sys == SYS_VISC ? series_line(g, F, d, r, wall)
                                                     : F->K[d][fidx(F->n, d, r[0], r[1], r[2])];
                            }
                        C->K[d][fidx(C->n, d, i, j, k)] = s / 16.0;
                    }
        }
        for (int k = 0; k < C->n[2]; k++)
            for (int j = 0; j < C->n[1]; j++)
                for (int i = 0; i < C->n[0]; i++) {
                    double s = 0;
                    for (int c = 0; c < 8; c++)
                        s += F->S[cidx(F->n, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1),
                                       2 * k + ((c >> 2) & 1))];
                    C->S[cidx(C->n, i, j, k)] = s / 8.0;
                }
    }
    for (int l = 0; l < g->nlev; l++) {
        level_t* L = &g->lev[l];
        for (int k = 0; k < L->n[2]; k++)
            for (int j = 0; j < L->n[1]; j++)
                for (int i = 0; i < L->n[0]; i++) {
                    long c = cidx(L->n, i, j, k);
                    double dsum = L->S[c];
                    for (int d = 0; d < 3; d++) {
                        int f[3] = {i, j, k};
                        dsum += L->K[d][fidx(L->n, d, f[0], f[1], f[2])];
                        f[d] += 1;
                        dsum += L->K[d][fidx(L->n, d, f[0], f[1], f[2])];
                    }
                    L->D[c] = L->mask[c] ? dsum : 0.0;
                }
    }
}

/* sum over interior faces of K_f x_nb (domain-wall faces only enter the diagonal) */
static double offdiag_sum(const or_geom* g, const level_t* L, const double* x, int i, int j,
                          int k) {
    const int* per = g->box.periodic;
    double s = 0;
    for (int d = 0; d < 3; d++)
        for (int side = -1; side <= 1; side += 2) {
            int f[3] = {i, j, k};
            if (side > 0) f[d] += 1;
            double K = L->K[d][fidx(L->n, d, f[0], f[1], f[2])];
            if (K == 0.0) continue;
            int r[3] = {i, j, k};
            r[d] += side;
            long nb = cell_at(L->n, per, r);
            if (nb < 0) continue;
            s += K * x[nb];
        }
    return s;
}

static void level_apply(const or_geom* g, const level_t* L, int ncomp, const double* x,
                        double* y) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < L->n[2]; k++)
        for (int j = 0; j < L->n[1]; j++)
            for (int i = 0; i < L->n[0]; i++) {
                long c = cidx(L->n, i, j, k);
                for (int m = 0; m < ncomp; m++) {
                    const double* xm = x + (long)m * L->N;
                    y[(long)m * L->N + c] =
                        L->mask[c] ? L->D[c] * xm[c] - offdiag_sum(g, L, xm, i, j, k) : 0.0;
                }
            }
}

/* one Gauss-Seidel half sweep over the cells of colour (i+j+k) mod 2 == col */
static void smooth_colour(const or_geom* g, const level_t* L, int ncomp, const double* b,
                          double* x, int col) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < L->n[2]; k++)
        for (int j = 0; j < L->n[1]; j++)
            for (int i = 0; i < L->n[0]; i++) {
                if (((i + j + k) & 1) != col) continue;
                long c = cidx(L->n, i, j, k);
                if (!L->mask[c] || L->D[c] <= 0.0) continue;
                for (int m = 0; m < ncomp; m++) {
                    double* xm = x + (long)m * L->N;
                    xm[c] = (b[(long)m * L->N + c] + offdiag_sum(g, L, xm, i, j, k)) / L->D[c];
                }
            }
}

static void vcycle_level(const or_geom* g, int l, int ncomp, const double* b, double* x,
                         const or_opts* o) {
    const level_t* L = &g->lev[l];
    long N = L->N;
    memset(x, 0, (size_t)ncomp * N * sizeof(double));
    if (l == g->nlev - 1) {
        for (int s = 0; s < o->nbottom; s++) {
            smooth_colour(g, L, ncomp, b, x, 0);
            smooth_colour(g, L, ncomp, b, x, 1);
        }
        for (int s = 0; s < o->nbottom; s++) {
            smooth_colour(g, L, ncomp, b, x, 1);
            smooth_colour(g, L, ncomp, b, x, 0);
        }
        return;
    }
    for (int s = 0; s < o->nu1; s++) {
        smooth_colour(g, L, ncomp, b, x, 0);
        smooth_colour(g, L, ncomp, b, x, 1);
    }
    const level_t* C = &g->lev[l + 1];
    double* r = malloc((size_t)ncomp * N * sizeof(double));
    level_apply(g, L, ncomp, x, r);
    for (long t = 0; t < (long)ncomp * N; t++) r[t] = b[t] - r[t];
    double* bc = calloc((size_t)ncomp * C->N, sizeof(double));
    double* ec = malloc((size_t)ncomp * C->N * sizeof(double));
    /* restriction: mean of the eight children (rows are already volume-fraction weighted) */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < C->n[2]; k++)
        for (int j = 0; j < C->n[1]; j++)
            for (int i = 0; i < C->n[0]; i++) {
                long cc = cidx(C->n, i, j, k);
                for (int m = 0; m < ncomp; m++) {
                    double s = 0;
                    for (int q = 0; q < 8; q++) {
                        long fc = cidx(L->n, 2 * i + (q & 1), 2 * j + ((q >> 1) & 1),
                                       2 * k + ((q >> 2) & 1));
                        if (L->mask[fc]) s += r[(long)m * N + fc];
                    }
                    bc[(long)m * C->N + cc] = C->mask[cc] ? s / 8.0 : 0.0;
                }
            }
    vcycle_level(g, l + 1, ncomp, bc, ec, o);
    /* piecewise-constant prolongation to uncovered children */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < L->n[2]; k++)
        for (int j = 0; j < L->n[1]; j++)
            for (int i = 0; i < L->n[0]; i++) {
                long fc = cidx(L->n, i, j, k);
                if (!L->mask[fc]) continue;
                long cc = cidx(C->n, i / 2, j / 2, k / 2);
                for (int m = 0; m < ncomp; m++) x[(long)m * N + fc] += ec[(long)m * C->N + cc];
            }
    for (int s = 0; s < o->nu2; s++) {
        smooth_colour(g, L, ncomp, b, x, 1);
        smooth_colour(g, L, ncomp, b, x, 0);
    }
    free(r);
    free(bc);
    free(ec);
}

void or_vcycle(const or_geom* g_in, int system, double beta, double rho, double dt,
               const double* eta, const double* eta_eb, const double* r, double* e,
               const or_opts* o) {
    or_geom* g = (or_geom*)g_in;
    build_operator(g, system, beta, rho, dt, eta, eta_eb);
    vcycle_level(g, 0, system == SYS_VISC ? 3 : 1, r, e, o);
}

void or_poisson_apply(const or_geom* g_in, double beta, const double* p, double* out) {
    or_geom* g = (or_geom*)g_in;
    build_operator(g, SYS_POISSON, beta, 0, 0, NULL, NULL);
    level_apply(g, &g->lev[0], 1, p, out);
}

/* exact viscous Helmholtz operator (Eq. implicit-viscous) with the EB wall flux of Eq. dudn,
 * rows multiplied by the volume fraction: alpha rho u - dt * (flux sum)/(h^2) + dt A_EB eta_EB g/h */
void or_visc_apply(const or_geom* g, double rho, double dt, const double* eta,
                   const double* eta_eb, const double* u, double* out, int homogeneous) {
    const int* n = g->box.n;
    const int* per = g->box.periodic;
    long N = g->N;
    double h = g->box.h;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; c++) {
        for (int j = 0; j < 3; j++) out[j * N + c] = 0.0;
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        long cid = g->cutid[c];
        for (int j = 0; j < 3; j++) {
            const double* uj = u + (long)j * N;
            double acc = g->alpha[c] * rho * uj[c];
            for (int d = 0; d < 3; d++)
                for (int side = -1; side <= 1; side += 2) {
                    int f[3] = {q[0], q[1], q[2]};
                    if (side > 0) f[d] += 1;
                    double A = g->ap[d][fidx(n, d, f[0], f[1], f[2])];
                    if (A == 0.0) continue;
                    int r[3] = {q[0], q[1], q[2]};
                    r[d] += side;
                    long nb = cell_at(n, per, r);
                    if (nb >= 0) {
                        double K = dt * A * 0.5 * (eta[c] + eta[nb]) / (h * h);
                        acc -= K * (uj[nb] - uj[c]);
                    } else {
                        double uw = homogeneous ? 0.0 : g->box.wall_u[2 * d + (side > 0)][j];
                        double K = 2.0 * dt * A * eta[c] / (h * h);
                        acc -= K * (uw - uj[c]);
                    }
                }
            if (cid >= 0) {
                double ueb = homogeneous ? 0.0 : g->body.u_eb[j];
                acc += dt * g->aeb[cid] * eta_eb[cid] * wall_dudn(g, (int)cid, uj, ueb) / h;
            }
            out[j * N + c] = acc;
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Krylov drivers around the V-cycle                                                            */
/* ------------------------------------------------------------------------------------------ */
/* max |x|, or NaN when any entry is NaN (a non-finite residual must reach the stop test) */
static double vmaxabs(const double* x, long n) {
    double m = 0;
    for (long t = 0; t < n; t++) {
        if (isnan(x[t])) return NAN;
        if (fabs(x[t]) > m) m = fabs(x[t]);
    }
    return m;
}
static double vdot(const double* x, const double* y, long n) {
    double s = 0;
    for (long t = 0; t < n; t++) s += x[t] * y[t];
    return s;
}

/* z minus its mean over open cells.  The Poisson system is singular (constants on the fluid are
 * its null space) and the V-cycle's output carries a constant component, which in exact
 * arithmetic only adds a constant to the iterate (removed by the final normalisation) and changes
 * no CG coefficient (the residual is mean-free).  In floating point, once the residual is near
 * the tolerance that component dominates the search direction, whose A-product is then rounding
 * noise times a huge step, and CG breaks down; removing it keeps the iteration in the range. */
static void open_mean_free(const or_geom* g, double* z) {
    double s = 0;
    long cnt = 0;
    for (long c = 0; c < g->N; c++)
        if (g->alpha[c] > 0.0) {
            s += z[c];
            cnt++;
        }
    double mean = cnt ? s / cnt : 0.0;
    for (long c = 0; c < g->N; c++)
        if (g->alpha[c] > 0.0) z[c] -= mean;
}

/* preconditioned CG on the symmetric Poisson system M p = b (operator already built); the
 * preconditioned residual is made mean-free over open cells after every V-cycle */
static int pcg(or_geom* g, const double* b, double* x, double rtol, double scale, int maxit,
               const or_opts* o, int* iters) {
    long N = g->N;
    level_t* L = &g->lev[0];
    double* r = malloc(N * sizeof(double));
    double* z = malloc(N * sizeof(double));
    double* p = malloc(N * sizeof(double));
    double* q = malloc(N * sizeof(double));
    int ret = OR_ENOCONV;
    *iters = 0;
    level_apply(g, L, 1, x, r);
    for (long t = 0; t < N; t++) r[t] = b[t] - r[t];
    double bn = vmaxabs(b, N);
    if (scale > bn) bn = scale;
    double rn0 = vmaxabs(r, N);
    if (!isfinite(rn0) || !isfinite(bn)) {
        ret = OR_ENAN;
        goto done;
    }
    if (bn == 0.0 || rn0 <= rtol * bn) {
        ret = OR_OK;
        goto done;
    }
    vcycle_level(g, 0, 1, r, z, o);
    open_mean_free(g, z);
    memcpy(p, z, N * sizeof(double));
    double rz = vdot(r, z, N);
    for (int it = 1; it <= maxit; it++) {
        level_apply(g, L, 1, p, q);
        double a = rz / vdot(p, q, N);
        for (long t = 0; t < N; t++) {
            x[t] += a * p[t];
            r[t] -= a * q[t];
        }
        *iters = it;
        double rn = vmaxabs(r, N);
        if (!isfinite(rn)) {
            ret = OR_ENAN;
            break;
        }
        if (rn <= rtol * bn) {
            ret = OR_OK;
            break;
        }
        vcycle_level(g, 0, 1, r, z, o);
        open_mean_free(g, z);
        double rzn = vdot(r, z, N);
        double be = rzn / rz;
        rz = rzn;
        for (long t = 0; t < N; t++) p[t] = z[t] + be * p[t];
    }
done:
    free(r);
    free(z);
    free(p);
    free(q);
    return ret;
}

/* Poisson solve for the projections: M p = -(D w - mean), then p normalised to zero mean.
 * Stop when max|r| <= rtol * max(max|b|, scale); scale is the largest face flux |A w|/h, the
 * size of the terms that make up the divergence (so an already solenoidal field stops at once). */
static int poisson_solve(or_geom* g, double beta, const double* divw, double* p, double rtol,
                         double scale, int maxit, const or_opts* o, int* iters) {
    long N = g->N;
    build_operator(g, SYS_POISSON, beta, 0, 0, NULL, NULL);
    double* b = malloc(N * sizeof(double));
    double s = 0;
    long cnt = 0;
    for (long c = 0; c < N; c++)
        if (g->alpha[c] > 0.0) {
            s += divw[c];
            cnt++;
        }
    double mean = cnt ? s / cnt : 0.0;
    for (long c = 0; c < N; c++) b[c] = g->alpha[c] > 0.0 ? -(divw[c] - mean) : 0.0;
    int ret = pcg(g, b, p, rtol, scale, maxit, o, iters);
    s = 0;
    for (long c = 0; c < N; c++)
        if (g->alpha[c] > 0.0) s += p[c];
    mean = cnt ? s / cnt : 0.0;
    for (long c = 0; c < N; c++) p[c] = g->alpha[c] > 0.0 ? p[c] - mean : 0.0;
    free(b);
    return ret;
}

int or_visc_solve(const or_geom* g_in, double rho, double dt, const double* eta,
                  const double* eta_eb, const double* psi, double* x, double rtol, int maxit,
                  const or_opts* o, int* iters) {
    or_geom* g = (or_geom*)g_in;
    long N = g->N, N3 = 3 * N;
    build_operator(g, SYS_VISC, 0, rho, dt, eta, eta_eb);
    double* r = malloc(N3 * sizeof(double));
    double* rh = malloc(N3 * sizeof(double));
    double* p = calloc(N3, sizeof(double));
    double* v = calloc(N3, sizeof(double));
    double* ph = malloc(N3 * sizeof(double));
    double* s = malloc(N3 * sizeof(double));
    double* sh = malloc(N3 * sizeof(double));
    double* t = malloc(N3 * sizeof(double));
    double* zero = calloc(N3, sizeof(double));
    int ret = OR_ENOCONV;
    *iters = 0;
    /* effective right-hand side b = alpha psi - A(0) (boundary values moved to the right) */
    or_visc_apply(g, rho, dt, eta, eta_eb, zero, t, 0);
    for (long q = 0; q < N3; q++) {
        long c = q % N;
        double b = g->alpha[c] > 0.0 ? g->alpha[c] * psi[q] : 0.0;
        s[q] = b - t[q];
    }
    double bn = vmaxabs(s, N3);
    double tol = rtol * bn;
    or_visc_apply(g, rho, dt, eta, eta_eb, x, t, 0);
    for (long q = 0; q < N3; q++) {
        long c = q % N;
        double b = g->alpha[c] > 0.0 ? g->alpha[c] * psi[q] : 0.0;
        r[q] = b - t[q];
    }
    double rn0 = vmaxabs(r, N3);
    if (!isfinite(rn0) || !isfinite(bn)) {
        ret = OR_ENAN;
        goto done;
    }
    if (bn == 0.0 || rn0 <= tol) {
        ret = OR_OK;
        goto done;
    }
    memcpy(rh, r, N3 * sizeof(double));
    double rho_old = 1, al = 1, om = 1;
    for (int it = 1; it <= maxit; it++) {
        double rr = vdot(rh, r, N3);
        double be = (rr / rho_old) * (al / om);
        for (long q = 0; q < N3; q++) p[q] = r[q] + be * (p[q] - om * v[q]);
        vcycle_level(g, 0, 3, p, ph, o);
        or_visc_apply(g, rho, dt, eta, eta_eb, ph, v, 1);
        al = rr / vdot(rh, v, N3);
        for (long q = 0; q < N3; q++) s[q] = r[q] - al * v[q];
        *iters = it;
        double sn = vmaxabs(s, N3);
        if (!isfinite(sn)) {
            ret = OR_ENAN;
            break;
        }
        if (sn <= tol) {
            for (long q = 0; q < N3; q++) x[q] += al * ph[q];
            ret = OR_OK;
            break;
        }
        vcycle_level(g, 0, 3, s, sh, o);
        or_visc_apply(g, rho, dt, eta, eta_eb, sh, t, 1);
        om = vdot(t, s, N3) / vdot(t, t, N3);
        for (long q = 0; q < N3; q++) {
            x[q] += al * ph[q] + om * sh[q];
            r[q] = s[q] - om * t[q];
        }
        double rn = vmaxabs(r, N3);
        if (!isfinite(rn)) {
            ret = OR_ENAN;
            break;
        }
        if (rn <= tol) {
            ret = OR_OK;
            break;
        }
        rho_old = rr;
    }
done:
    free(r);
    free(rh);
    free(p);
    free(v);
    free(ph);
    free(s);
    free(sh);
    free(t);
    free(zero);
    return ret;
}

/* ------------------------------------------------------------------------------------------ */
/* projections                                                                                  */
/* ------------------------------------------------------------------------------------------ */
/* face correction w -= beta (p_hi - p_lo)/h on open interior faces */
static void face_correct(const or_geom* g, double beta, const double* p, double* const fo[3]) {
    const int* n = g->box.n;
    double h = g->box.h;
    for (int d = 0; d < 3; d++) {
        int m[3] = {n[0] + (d == 0), n[1] + (d == 1), n[2] + (d == 2)};
        for (int k = 0; k < m[2]; k++)
            for (int j = 0; j < m[1]; j++)
                for (int i = 0; i < m[0]; i++) {
                    int f[3] = {i, j, k};
                    long fi = fidx(n, d, i, j, k);
                    long lo, hi;
                    face_cells(g, d, f, &lo, &hi);
                    if (lo < 0 || hi < 0 || g->ap[d][fi] == 0.0) continue;
                    fo[d][fi] -= beta * (p[hi] - p[lo]) / h;
                }
    }
}

/* cell-centred (MAC) projection of a face field (Eq. helmholtz and the Poisson problem) */
int or_mac_project(const or_geom* g_in, double beta, double* fx, double* fy, double* fz,
                   double* phi, double rtol, int maxit, const or_opts* o, double* div_inf,
                   int* iters) {
    or_geom* g = (or_geom*)g_in;
    long N = g->N;
    double* div = malloc(N * sizeof(double));
    double* fo[3] = {fx, fy, fz};
    or_divergence(g, fx, fy, fz, div);
    double scale = 0;
    for (int d = 0; d < 3; d++)
        for (long f = 0; f < nfaces(g->box.n, d); f++) {
            double a = fabs(g->ap[d][f] * fo[d][f]) / g->box.h;
            if (a > scale) scale = a;
        }
    int ret = poisson_solve(g, beta, div, phi, rtol, scale, maxit, o, iters);
    face_correct(g, beta, phi, fo);
    or_divergence(g, fx, fy, fz, div);
    if (div_inf) *div_inf = vmaxabs(div, N);
    free(div);
    return ret;
}

/* end-of-stage projection with cell-centred pressure (reading of the approximate projection):
 * add back beta*G p_old, average to faces, project the faces exactly, correct the cells with
 * the averaged face gradients of the new pressure. */
int or_cc_project(const or_geom* g_in, double beta, double* u, double* p, double rtol,
                  int maxit, const or_opts* o, double* div_inf, int* iters) {
    or_geom* g = (or_geom*)g_in;
    const int* n = g->box.n;
    long N = g->N;
    double* gp = malloc(3 * N * sizeof(double));
    double* fo[3];
    for (int d = 0; d < 3; d++) fo[d] = calloc(nfaces(n, d), sizeof(double));
    or_gcc(g, p, gp);
    for (long q = 0; q < 3 * N; q++)
        if (g->alpha[q % N] > 0.0) u[q] += beta * gp[q];
    for (int d = 0; d < 3; d++) {
        int m[3] = {n[0] + (d == 0), n[1] + (d == 1), n[2] + (d == 2)};
        for (int k = 0; k < m[2]; k++)
            for (int j = 0; j < m[1]; j++)
                for (int i = 0; i < m[0]; i++) {
                    int f[3] = {i, j, k};
                    long fi = fidx(n, d, i, j, k);
                    long lo, hi;
                    face_cells(g, d, f, &lo, &hi);
                    double v = 0.0;
                    if (lo < 0 || hi < 0)
                        v = g->box.wall_u[2 * d + (lo >= 0)][d];
                    else if (g->ap[d][fi] > 0.0)
                        v = 0.5 * (u[(long)d * N + lo] + u[(long)d * N + hi]);
                    fo[d][fi] = v;
                }
    }
    int ret = or_mac_project(g, beta, fo[0], fo[1], fo[2], p, rtol, maxit, o, div_inf, iters);
    or_gcc(g, p, gp);
    for (long q = 0; q < 3 * N; q++)
        if (g->alpha[q % N] > 0.0) u[q] -= beta * gp[q];
    for (int d = 0; d < 3; d++) free(fo[d]);
    free(gp);
    return ret;
}

/* ------------------------------------------------------------------------------------------ */
/* DerivedQuantities (Alg. derived) and the RK2 step (Alg. advance)                             */
/* ------------------------------------------------------------------------------------------ */
/* uf_keep (nullable): receives the projected face velocities used for the upwinding */
static int derived_impl(const or_geom* g_in, const or_rheo* rh, const double* theta,
                        const double* u, const or_opts* o, double* C, double* eta,
                        double* eta_eb, double* V, int* iters, double* const uf_keep[3]) {
    or_geom* g = (or_geom*)g_in;
    const int* n = g->box.n;
    long N = g->N;
    double* uf[3];
    for (int d = 0; d < 3; d++) uf[d] = calloc(nfaces(n, d), sizeof(double));
    double* phi = calloc(N, sizeof(double));
    or_face_extrap(g, u, uf[0], uf[1], uf[2]);
    int ret = or_mac_project(g, 1.0, uf[0], uf[1], uf[2], phi, o->rtol_mac, o->max_iter, o,
                             NULL, iters);
    or_conv_term(g, u, uf[0], uf[1], uf[2], C);
    double* gw = calloc(3 * (g->ncut + 1), sizeof(double));
    double* G = malloc(9 * N * sizeof(double));
    double* DC = malloc(3 * N * sizeof(double));
    or_wall_gradient(g, u, gw);
    or_cell_gradient(g, u, gw, G);
    viscosity_from(g, rh, theta, G, gw, eta, eta_eb, NULL);
    transpose_term_dc(g, eta, eta_eb, u, G, gw, DC);
    or_redistribute(g, 3, DC, V);
    if (uf_keep)
        for (int d = 0; d < 3; d++) memcpy(uf_keep[d], uf[d], nfaces(n, d) * sizeof(double));
    free(DC);
    free(G);
    free(gw);
    free(phi);
    for (int d = 0; d < 3; d++) free(uf[d]);
    return ret;
}

int or_derived(const or_geom* g, const or_rheo* rh, const double* theta, const double* u,
               const or_opts* o, double* C, double* eta, double* eta_eb, double* V,
               int* iters) {
    return derived_impl(g, rh, theta, u, o, C, eta, eta_eb, V, iters, NULL);
}

/* intermediate fields of one step, kept for the reverse sweep */
typedef struct {
    double* ufm[3]; /* projected face velocities of the predictor */
    double* em;     /* viscosity at u^m (predictor operator) */
    double* ebm;
    double* us1;    /* predictor solve, before its projection */
    double* u1;     /* projected predictor velocity u* */
    double* uf1[3]; /* projected face velocities of the corrector */
    double* ea;     /* averaged viscosity (corrector operator) */
    double* eba;
    double* us2;    /* corrector solve, before its projection */
} rk2_tape;

static long nd_count(const or_geom* g); /* nodes of the nodal projection (below) */

static int rk2_impl(const or_geom* g_in, const or_rheo* rh, const double* theta, double dt,
                    const or_opts* o, double* u, double* p, or_stats* st, rk2_tape* tp) {
    or_geom* g = (or_geom*)g_in;
    long N = g->N, N3 = 3 * N;
    int nc = g->ncut + 1;
    double rho = rh->rho, beta = dt / rh->rho;
    double *Cm = malloc(N3 * 8), *Vm = malloc(N3 * 8), *em = malloc(N * 8), *ebm = malloc(nc * 8);
    double *Cs = malloc(N3 * 8), *Vs = malloc(N3 * 8), *es = malloc(N * 8), *ebs = malloc(nc * 8);
    double *psi = malloc(N3 * 8), *gp = malloc(N3 * 8), *ut = malloc(N3 * 8);
    int nodal = o->projection == OR_PROJ_NODAL;
    long NP = nodal ? nd_count(g) : N; /* the pressure's storage: nodes or cells */
    double *ps = malloc(NP * 8);
    int err = OR_OK, e, it;
    or_stats loc;
    memset(&loc, 0, sizeof(loc));
    /* predictor */
    e = derived_impl(g, rh, theta, u, o, Cm, em, ebm, Vm, &it, tp ? tp->ufm : NULL);
    loc.it_mac[0] = it;
    if (e) err = e;
    if (nodal) or_nodal_grad(g, p, gp);
    else or_gcc(g, p, gp);
    for (long q = 0; q < N3; q++) {
        int d = (int)(q / N);
        psi[q] = rho * u[q] + dt * (rho * Cm[q] + Vm[q] - gp[q] + o->force[d]);
    }
    memcpy(ut, u, N3 * 8);
    e = or_visc_solve(g, rho, dt, em, ebm, psi, ut, o->rtol_visc, o->max_iter, o, &it);
    loc.it_visc[0] = it;
    if (e) err = e;
    if (tp) {
        memcpy(tp->em, em, N * 8);
        memcpy(tp->ebm, ebm, nc * 8);
        memcpy(tp->us1, ut, N3 * 8);
    }
    memcpy(ps, p, NP * 8);
    if (nodal)
        e = or_nodal_project(g, beta, ut, ps, o->rtol_proj, o->max_iter, &loc.div_proj[0], &it);
    else
        e = or_cc_project(g, beta, ut, ps, o->rtol_proj, o->max_iter, o, &loc.div_proj[0], &it);
    loc.it_proj[0] = it;
    if (e) err = e;
    /* corrector: derived quantities at u*, averaged with those at u^m */
    if (tp) memcpy(tp->u1, ut, N3 * 8);
    e = derived_impl(g, rh, theta, ut, o, Cs, es, ebs, Vs, &it, tp ? tp->uf1 : NULL);
    loc.it_mac[1] = it;
    if (e) err = e;
    for (long q = 0; q < N3; q++) {
        Cm[q] = 0.5 * (Cm[q] + Cs[q]);
        Vm[q] = 0.5 * (Vm[q] + Vs[q]);
    }
    for (long c = 0; c < N; c++) em[c] = 0.5 * (em[c] + es[c]);
    for (int c = 0; c < g->ncut; c++) ebm[c] = 0.5 * (ebm[c] + ebs[c]);
    if (nodal) or_nodal_grad(g, ps, gp);
    else or_gcc(g, ps, gp);
    for (long q = 0; q < N3; q++) {
        int d = (int)(q / N);
        psi[q] = rho * u[q] + dt * (rho * Cm[q] + Vm[q] - gp[q] + o->force[d]);
    }
    e = or_visc_solve(g, rho, dt, em, ebm, psi, ut, o->rtol_visc, o->max_iter, o, &it);
    loc.it_visc[1] = it;
    if (e) err = e;
    if (tp) {
        memcpy(tp->ea, em, N * 8);
        memcpy(tp->eba, ebm, nc * 8);
        memcpy(tp->us2, ut, N3 * 8);
    }
    if (nodal)
        e = or_nodal_project(g, beta, ut, ps, o->rtol_proj, o->max_iter, &loc.div_proj[1], &it);
    else
        e = or_cc_project(g, beta, ut, ps, o->rtol_proj, o->max_iter, o, &loc.div_proj[1], &it);
    loc.it_proj[1] = it;
    if (e) err = e;
    for (long q = 0; q < N3; q++) {
        long c = q % N;
        u[q] = g->alpha[c] > 0.0 ? ut[q] : g->body.u_eb[q / N];
    }
    if (nodal) memcpy(p, ps, NP * 8);
    else
        for (long c = 0; c < N; c++) p[c] = g->alpha[c] > 0.0 ? ps[c] : 0.0;
    if (st) *st = loc;
    free(Cm); free(Vm); free(em); free(ebm);
    free(Cs); free(Vs); free(es); free(ebs);
    free(psi); free(gp); free(ut); free(ps);
    return err;
}

int or_rk2_step(const or_geom* g, const or_rheo* rh, const double* theta, double dt,
                const or_opts* o, double* u, double* p, or_stats* st) {
    return rk2_impl(g, rh, theta, dt, o, u, p, st, NULL);
}

/* ------------------------------------------------------------------------------------------ */
/* nodal projection (Sec. III.A.4 "Incompressibility constraint"; Alg. advance NodalProjection):  */
/* velocities on cell centres, the pressure on the nodes (cell corners), an approximate          */
/* projection.  The paper leaves the discrete operators to its library's nodal solver; this is   */
/* the trilinear finite-element form of that projection, each cell weighted by its volume        */
/* fraction:                                                                                     */
/*  - D(w)_n: the weak divergence of a cell field w against the hat function of node n,          */
/*    sum over the cells c at n of alpha_c h^2/4 sum_d s_d w_{d,c} (s_d = +1 when n is on c's    */
/*    upper side in d, else -1), minus the boundary flux B_n of the given normal velocity:       */
/*    A_f h^2/4 (u_wall . n_out) per domain-wall face at n, A_EB h^2/8 (u_EB . n_out) per cut    */
/*    cell at n (n_out = -n_EB, the EB area shared equally by the cell's 8 nodes);               */
/*  - L: the stiffness matrix of those elements, L_nm = sum_c alpha_c h Khat(a, b);              */
/*  - G(q)_c: the cell average of the gradient of the trilinear interpolant of q;                */
/*  - solve L phi = D(w) - B on the nodes of open cells, CG with the diagonal as preconditioner  */
/*    (mean-free over those nodes: L is singular), phi normalised to zero mean there.            */
/* ------------------------------------------------------------------------------------------ */
static long nd_index(const or_geom* g, int i, int j, int k) {
    const int* n = g->box.n;
    return (long)i + (long)(n[0] + 1) * ((long)j + (long)(n[1] + 1) * (long)k);
}
static long nd_count(const or_geom* g) {
    const int* n = g->box.n;
    return (long)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
}
/* node of corner a (bit d set: upper side in d) of cell (i, j, k); in a periodic direction the
 * last node is the first */
static long nd_corner(const or_geom* g, const int q[3], int a) {
    int r[3];
    for (int d = 0; d < 3; d++) {
        r[d] = q[d] + ((a >> d) & 1);
        if (g->box.periodic[d] && r[d] == g->box.n[d]) r[d] = 0;
    }
    return nd_index(g, r[0], r[1], r[2]);
}
/* the trilinear stiffness of the unit cube between corners a and b: sum over d of the 1D
 * derivative term (+1 same side, -1 opposite) times the 1D mass terms of the other two
 * directions (1/3 same side, 1/6 opposite) */
static double khat(int a, int b) {
    double s = 0.0;
    for (int d = 0; d < 3; d++) {
        double t = (((a ^ b) >> d) & 1) ? -1.0 : 1.0;
        for (int e = 0; e < 3; e++)
            if (e != d) t *= (((a ^ b) >> e) & 1) ? 1.0 / 6.0 : 1.0 / 3.0;
        s += t;
    }
    return s;
}
/* periodic copies: the last node of a periodic direction takes the first node's value */
static void nd_sync(const or_geom* g, double* x) {
    const int* n = g->box.n;
    for (int k = 0; k <= n[2]; k++)
        for (int j = 0; j <= n[1]; j++)
            for (int i = 0; i <= n[0]; i++) {
                int r[3] = {i, j, k};
                for (int d = 0; d < 3; d++)
                    if (g->box.periodic[d] && r[d] == n[d]) r[d] = 0;
                x[nd_index(g, i, j, k)] = x[nd_index(g, r[0], r[1], r[2])];
            }
}

void or_nodal_div(const or_geom* g, const double* w, double* dn) {
    const int* n = g->box.n;
    long N = g->N, M = nd_count(g);
    double h = g->box.h;
    memset(dn, 0, M * sizeof(double));
    for (long c = 0; c < N; c++) {
        double al = g->alpha[c];
        if (al <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int a = 0; a < 8; a++) {
            double s = 0.0;
            for (int d = 0; d < 3; d++) s += (((a >> d) & 1) ? 1.0 : -1.0) * w[d * N + c];
            dn[nd_corner(g, q, a)] += al * h * h / 4.0 * s;
        }
    }
    nd_sync(g, dn);
}

void or_nodal_bflux(const or_geom* g, double* bn) {
    const int* n = g->box.n;
    long N = g->N, M = nd_count(g);
    double h = g->box.h;
    memset(bn, 0, M * sizeof(double));
    for (int d = 0; d < 3; d++) {
        if (g->box.periodic[d]) continue;
        for (int side = 0; side < 2; side++) {
            double un = g->box.wall_u[2 * d + side][d] * (side ? 1.0 : -1.0);
            for (long c = 0; c < N; c++) {
                int q[3];
                cell_ijk(n, c, q);
                if (q[d] != (side ? n[d] - 1 : 0)) continue;
                int f[3] = {q[0], q[1], q[2]};
                f[d] += side;
                double A = g->ap[d][fidx(n, d, f[0], f[1], f[2])];
                if (A == 0.0) continue;
                for (int a = 0; a < 8; a++)
                    if (((a >> d) & 1) == side) bn[nd_corner(g, q, a)] += A * h * h / 4.0 * un;
            }
        }
    }
    for (int cid = 0; cid < g->ncut; cid++) {
        int q[3];
        cell_ijk(n, g->cut[cid], q);
        double un = 0.0;
        for (int d = 0; d < 3; d++) un -= g->body.u_eb[d] * g->nrm[3 * cid + d];
        for (int a = 0; a < 8; a++) bn[nd_corner(g, q, a)] += g->aeb[cid] * h * h / 8.0 * un;
    }
    nd_sync(g, bn);
}

void or_nodal_apply(const or_geom* g, const double* x, double* y) {
    const int* n = g->box.n;
    long N = g->N, M = nd_count(g);
    double h = g->box.h;
    memset(y, 0, M * sizeof(double));
    for (long c = 0; c < N; c++) {
        double al = g->alpha[c];
        if (al <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        long nodes[8];
        for (int a = 0; a < 8; a++) nodes[a] = nd_corner(g, q, a);
        for (int a = 0; a < 8; a++) {
            double s = 0.0;
            for (int b = 0; b < 8; b++) s += khat(a, b) * x[nodes[b]];
            y[nodes[a]] += al * h * s;
        }
    }
    nd_sync(g, y);
}

void or_nodal_grad(const or_geom* g, const double* qn, double* gp) {
    const int* n = g->box.n;
    long N = g->N;
    double h = g->box.h;
    for (long c = 0; c < N; c++) {
        int q[3];
        cell_ijk(n, c, q);
        for (int d = 0; d < 3; d++) {
            double s = 0.0;
            for (int a = 0; a < 8; a++)
                s += (((a >> d) & 1) ? 1.0 : -1.0) * qn[nd_corner(g, q, a)];
            gp[d * N + c] = g->alpha[c] > 0.0 ? s / (4.0 * h) : 0.0;
        }
    }
}

/* nodes touching an open cell (the unknowns of the nodal solve) */
static void nd_active(const or_geom* g, uint8_t* act) {
    const int* n = g->box.n;
    memset(act, 0, nd_count(g));
    for (long c = 0; c < g->N; c++) {
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int a = 0; a < 8; a++) act[nd_corner(g, q, a)] = 1;
    }
}
static void nd_mean_free(const or_geom* g, const uint8_t* act, double* x) {
    long M = nd_count(g);
    double s = 0.0;
    long cnt = 0;
    for (long m = 0; m < M; m++)
        if (act[m]) {
            s += x[m];
            cnt++;
        }
    double mean = cnt ? s / cnt : 0.0;
    for (long m = 0; m < M; m++) x[m] = act[m] ? x[m] - mean : 0.0;
}

/* CG for L x = b on the active nodes, the diagonal as preconditioner and the preconditioned
 * residual mean-free; stop when max|r| <= rtol max(max|b|, scale) */
static int nd_cg(const or_geom* g, const uint8_t* act, const double* b, double* x, double rtol,
                 double scale, int maxit, int* iters) {
    const int* n = g->box.n;
    long M = nd_count(g);
    double h = g->box.h;
    double *r = malloc(M * 8), *z = malloc(M * 8), *p = malloc(M * 8), *q = malloc(M * 8);
    double* dg = calloc(M, 8);
    for (long c = 0; c < g->N; c++) {
        if (g->alpha[c] <= 0.0) continue;
        int qq[3];
        cell_ijk(n, c, qq);
        for (int a = 0; a < 8; a++) dg[nd_corner(g, qq, a)] += g->alpha[c] * h * khat(a, a);
    }
    int ret = OR_ENOCONV;
    *iters = 0;
    or_nodal_apply(g, x, q);
    for (long m = 0; m < M; m++) r[m] = act[m] ? b[m] - q[m] : 0.0;
    double bn = vmaxabs(b, M);
    if (scale > bn) bn = scale;
    double rn0 = vmaxabs(r, M);
    if (!isfinite(rn0) || !isfinite(bn)) {
        ret = OR_ENAN;
        goto done;
    }
    if (bn == 0.0 || rn0 <= rtol * bn) {
        ret = OR_OK;
        goto done;
    }
    for (long m = 0; m < M; m++) z[m] = act[m] ? r[m] / dg[m] : 0.0;
    nd_mean_free(g, act, z);
    memcpy(p, z, M * 8);
    double rz = vdot(r, z, M);
    for (int it = 1; it <= maxit; it++) {
        or_nodal_apply(g, p, q);
        for (long m = 0; m < M; m++)
            if (!act[m]) q[m] = 0.0;
        double al = rz / vdot(p, q, M);
        for (long m = 0; m < M; m++) {
            x[m] += al * p[m];
            r[m] -= al * q[m];
        }
        *iters = it;
        double rn = vmaxabs(r, M);
        if (!isfinite(rn)) {
            ret = OR_ENAN;
            break;
        }
        if (rn <= rtol * bn) {
            ret = OR_OK;
            break;
        }
        for (long m = 0; m < M; m++) z[m] = act[m] ? r[m] / dg[m] : 0.0;
        nd_mean_free(g, act, z);
        double rzn = vdot(r, z, M);
        double be = rzn / rz;
        rz = rzn;
        for (long m = 0; m < M; m++) p[m] = z[m] + be * p[m];
    }
done:
    free(r);
    free(z);
    free(p);
    free(q);
    free(dg);
    return ret;
}

int or_nodal_project(const or_geom* g, double beta, double* u, double* pn, double rtol,
                     int maxit, double* div_inf, int* iters) {
    const int* n = g->box.n;
    long N = g->N, N3 = 3 * N, M = nd_count(g);
    double h = g->box.h;
    double *w = malloc(N3 * 8), *gp = malloc(N3 * 8), *rhs = malloc(M * 8), *bf = malloc(M * 8);
    double *phi = malloc(M * 8), *tsum = calloc(M, 8);
    uint8_t* act = malloc(M);
    nd_active(g, act);
    /* w = u + beta G p_old */
    or_nodal_grad(g, pn, gp);
    for (long t = 0; t < N3; t++) w[t] = u[t] + beta * gp[t];
    or_nodal_div(g, w, rhs);
    or_nodal_bflux(g, bf);
    for (long m = 0; m < M; m++) rhs[m] = act[m] ? rhs[m] - bf[m] : 0.0;
    /* the size of the terms summed into D(w)_n: the stop test's second scale */
    for (long c = 0; c < N; c++) {
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        double s = 0.0;
        for (int d = 0; d < 3; d++) s += fabs(w[d * N + c]);
        for (int a = 0; a < 8; a++) tsum[nd_corner(g, q, a)] += g->alpha[c] * h * h / 4.0 * s;
    }
    double scale = vmaxabs(tsum, M);
    nd_mean_free(g, act, rhs); /* the rounding part of an incompatible right-hand side */
    for (long m = 0; m < M; m++) phi[m] = act[m] ? beta * pn[m] : 0.0;
    int ret = nd_cg(g, act, rhs, phi, rtol, scale, maxit, iters);
    nd_mean_free(g, act, phi);
    nd_sync(g, phi);
    or_nodal_grad(g, phi, gp);
    for (long t = 0; t < N3; t++) {
        long c = t % N;
        u[t] = g->alpha[c] > 0.0 ? w[t] - gp[t] : g->body.u_eb[t / N];
    }
    for (long m = 0; m < M; m++) pn[m] = phi[m] / beta;
    if (div_inf) { /* the weak divergence left in the projected field (not zero: approximate) */
        or_nodal_div(g, u, rhs);
        for (long m = 0; m < M; m++) rhs[m] = act[m] ? rhs[m] - bf[m] : 0.0;
        *div_inf = vmaxabs(rhs, M);
    }
    free(w);
    free(gp);
    free(rhs);
    free(bf);
    free(phi);
    free(tsum);
    free(act);
    return ret;
}

void or_drag_nodal(const or_geom* g, const or_rheo* r, const double* theta, const double* u,
                   const double* pn, double F[3]) {
    const int* n = g->box.n;
    double h = g->box.h;
    double* gw = calloc(3 * (g->ncut + 1), sizeof(double));
    or_wall_gradient(g, u, gw);
    F[0] = F[1] = F[2] = 0.0;
    for (int cid = 0; cid < g->ncut; cid++) {
        long c = g->cut[cid];
        int q[3];
        cell_ijk(n, c, q);
        const double* nv = &g->nrm[3 * cid];
        const double* gg = &gw[3 * cid];
        double Gm[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Gm[a][b] = nv[a] * gg[b];
        double eeb = law_eta(r, r->tau0 * (theta ? theta[c] : 1.0), strain_norm(Gm));
        /* trilinear interpolation of the nodal pressure at the wall centroid */
        double pe = 0.0;
        for (int a = 0; a < 8; a++) {
            double wgt = 1.0;
            for (int d = 0; d < 3; d++) {
                double xi = g->bc[3 * cid + d] + 0.5;
                wgt *= ((a >> d) & 1) ? xi : 1.0 - xi;
            }
            pe += wgt * pn[nd_corner(g, q, a)];
        }
        for (int a = 0; a < 3; a++) {
            double tn = 0;
            for (int b = 0; b < 3; b++) tn += eeb * (Gm[a][b] + Gm[b][a]) * nv[b];
            F[a] += g->aeb[cid] * h * h * (tn - pe * nv[a]);
        }
    }
    free(gw);
}

/* ------------------------------------------------------------------------------------------ */
/* drag on the embedded body (Eq. drag-force): sum over cut cells of (tau - p I) n A_EB h^2     */
/* ------------------------------------------------------------------------------------------ */
/* Time step of the stability rule (Sec. II.C.1): the convective coefficient (Eq.
 * cfl:convective) is the largest |u|/dx + |v|/dy + |w|/dz over fluid cells, the forcing one
 * (Eq. cfl:forcing) sqrt(sum_d |f_d| / dx_d), the viscous one (Eq. cfl:viscous:new)
 * 2 mu (Bi + 1) / rho * sum_d 1/dx_d^2 with the regularisation left out, and they combine by
 * Eq. cfl:dt.  Bi is the largest yield stress tau0 * theta_c over fluid cells (tau0 itself is
 * the Bingham number when mu, U and L are 1); a Newtonian law has Bi = 0.  The rule is stated
 * for the Newtonian and Bingham laws; for the power-law laws this returns 0. */
double or_stable_dt(const or_geom* g, const or_rheo* r, const double* theta, const double* u,
                    const double force[3], double c_cfl) {
    long N = g->N;
    double h = g->box.h;
    double cc = 0.0, bi = 0.0;
    if (r->law >= OR_LAW_POWER) return 0.0;
    for (long c = 0; c < N; c++) {
        if (!(g->alpha[c] > 0.0)) continue;
        double s = (fabs(u[c]) + fabs(u[N + c]) + fabs(u[2 * N + c])) / h;
        if (s > cc) cc = s;
        double t = r->law == OR_LAW_NEWTONIAN ? 0.0 : r->tau0 * (theta ? theta[c] : 1.0);
        if (t > bi) bi = t;
    }
    double cf = sqrt((fabs(force[0]) + fabs(force[1]) + fabs(force[2])) / h);
    double cv = 2.0 * r->mu / r->rho * (bi + 1.0) * (3.0 / (h * h));
    double a = cc + cv;
    return c_cfl / (0.5 * (a + sqrt(a * a + 4.0 * cf * cf)));
}

void or_drag(const or_geom* g, const or_rheo* r, const double* theta, const double* u,
             const double* p, double F[3]) {
    long N = g->N;
    double h = g->box.h;
    double* gw = calloc(3 * (g->ncut + 1), sizeof(double));
    double* gp = malloc(3 * N * sizeof(double));
    or_wall_gradient(g, u, gw);
    or_gcc(g, p, gp);
    F[0] = F[1] = F[2] = 0.0;
    for (int cid = 0; cid < g->ncut; cid++) {
        long c = g->cut[cid];
        const double* nv = &g->nrm[3 * cid];
        const double* gg = &gw[3 * cid];
        double Gm[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Gm[a][b] = nv[a] * gg[b];
        double eeb = law_eta(r, r->tau0 * (theta ? theta[c] : 1.0), strain_norm(Gm));
        double pe = p[c];
        for (int d = 0; d < 3; d++) pe += h * g->bc[3 * cid + d] * gp[d * N + c];
        for (int a = 0; a < 3; a++) {
            double tn = 0;
            for (int b = 0; b < 3; b++) tn += eeb * (Gm[a][b] + Gm[b][a]) * nv[b];
            F[a] += g->aeb[cid] * h * h * (tn - pe * nv[a]);
        }
    }
    free(gw);
    free(gp);
}

/* ------------------------------------------------------------------------------------------ */
/* adjoint (reverse mode) of the step.  Each routine is the exact transpose of the linearised  */
/* forward routine above it in the file, with                                                   */
/*   - every iterative solve taken as exact (implicit-function rule: the transposed system is  */
/*     solved, not the iteration differentiated),                                               */
/*   - every switch frozen at its forward value: upwind side, limiter branch, one-sided        */
/*     stencil choice, largest normal component, covered-node fallback.                        */
/* Adjoint arguments named *b hold d(loss)/d(that quantity) and are accumulated (+=) unless a   */
/* comment says otherwise.                                                                      */
/* ------------------------------------------------------------------------------------------ */
static void wall_dudn_adj(const or_geom* g, int cid, double gb, double* ubj) {
    double d1 = g->dd[2 * cid], d2 = g->dd[2 * cid + 1];
    double den = d1 * d2 * (d2 - d1) * g->box.h;
    for (int kk = 0; kk < 2; kk++) {
        double cf = kk == 0 ? d2 * d2 / den : -d1 * d1 / den;
        for (int m = 0; m < 9; m++) {
            long slot = ((long)cid * 2 + kk) * 9 + m;
            long cc = g->sidx[slot];
            if (cc >= 0) ubj[cc] += g->sw[slot] * cf * gb;
        }
    }
}

void or_wall_gradient_adj(const or_geom* g, const double* gwb, double* ub) {
    for (int c = 0; c < g->ncut; c++)
        for (int j = 0; j < 3; j++) wall_dudn_adj(g, c, gwb[3 * c + j], ub + (long)j * g->N);
}

void or_cell_gradient_adj(const or_geom* g, const double* Gb, double* ub, double* gwb) {
    const int* n = g->box.n;
    const int* per = g->box.periodic;
    long N = g->N;
    double h = g->box.h;
    for (long c = 0; c < N; c++) {
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int d = 0; d < 3; d++) {
            int r[3];
            memcpy(r, q, sizeof(r));
            r[d] = q[d] - 1;
            long lo = cell_at(n, per, r);
            r[d] = q[d] - 2;
            long lo2 = cell_at(n, per, r);
            r[d] = q[d] + 1;
            long hi = cell_at(n, per, r);
            r[d] = q[d] + 2;
            long hi2 = cell_at(n, per, r);
            int lo_wall = lo < 0, hi_wall = hi < 0;
            int lo_open = !lo_wall && g->alpha[lo] > 0.0;
            int hi_open = !hi_wall && g->alpha[hi] > 0.0;
            int lo2_open = lo2 >= 0 && g->alpha[lo2] > 0.0;
            int hi2_open = hi2 >= 0 && g->alpha[hi2] > 0.0;
            int lo_ok = lo_open || lo_wall, hi_ok = hi_open || hi_wall;
            for (int j = 0; j < 3; j++) {
                double gb = Gb[(d * 3 + j) * N + c];
                double* u = ub + (long)j * N;
                if (lo_ok && hi_ok) {
                    double w = gb / (2.0 * h); /* ghost values 2 u_wall - u_c at walls */
                    if (hi_open) u[hi] += w;
                    else u[c] -= w;
                    if (lo_open) u[lo] -= w;
                    else u[c] += w;
                } else if (hi_ok) {
                    if (hi_open && hi2_open) {
                        u[c] += -1.5 * gb / h;
                        u[hi] += 2.0 * gb / h;
                        u[hi2] += -0.5 * gb / h;
                    } else {
                        if (hi_open) u[hi] += gb / h;
                        else u[c] -= gb / h;
                        u[c] -= gb / h;
                    }
                } else if (lo_ok) {
                    if (lo_open && lo2_open) {
                        u[c] += 1.5 * gb / h;
                        u[lo] += -2.0 * gb / h;
                        u[lo2] += 0.5 * gb / h;
                    } else {
                        u[c] += gb / h;
                        if (lo_open) u[lo] -= gb / h;
                        else u[c] += gb / h;
                    }
                } else {
                    long cid = g->cutid[c];
                    if (cid >= 0) gwb[3 * cid + j] += g->nrm[3 * cid + d] * gb;
                }
            }
        }
    }
}

/* g'(x) for g(x) = (1 - e^-x)/x: (x e^-x + expm1(-x))/x^2, or below x = 1e-2 its Taylor series
 * -1/2 + x/3 - x^2/8 + x^3/30 - x^4/144, which avoids the cancellation */
static double gexp_prime(double x) {
    if (x < 1e-2) return -0.5 + x * (1.0 / 3.0 + x * (-1.0 / 8.0 + x * (1.0 / 30.0 - x / 144.0)));
    return (x * exp(-x) + expm1(-x)) / (x * x);
}

/* d eta / d(strain-rate norm) and d eta / d tau0 of the law in law_eta.  Where the strain
 * rate is zero (|.| is not differentiable there) or below the power-law cap, the power-law
 * term's derivative is taken as 0. */
static void law_deriv(const or_rheo* r, double tau0, double sr, double* d_sr, double* d_tau0) {
    *d_sr = 0.0;
    *d_tau0 = 0.0;
    if (r->law == OR_LAW_NEWTONIAN) return;
    if (r->law == OR_LAW_BINGHAM_REG) {
        double q = 1.0 / (sr + r->eps);
        *d_tau0 = q;
        *d_sr = -tau0 * q * q;
        return;
    }
    if (r->law >= OR_LAW_POWER && sr > 0.0 && !(r->n < 1.0 && sr < r->eps) && r->n != 1.0)
        *d_sr = r->kappa * (r->n - 1.0) * pow(sr, r->n - 2.0);
    if (r->law == OR_LAW_POWER) return;
    if (r->law == OR_LAW_SOUZA_MENDES_DUTRA) {
        /* tau0 (1 - e^-x)/sr = eta0 g(x) with x = eta0 sr/tau0: d/d sr = eta0^2 g'(x)/tau0 and
         * d/d tau0 = -eta0 x g'(x)/tau0; at tau0 = 0 the term is 0 and its tau0-derivative is
         * the limit 1/sr (0 at sr = 0) */
        if (tau0 == 0.0) {
            *d_tau0 = sr > 0.0 ? 1.0 / sr : 0.0;
            return;
        }
        double x = r->eta0 * sr / tau0, gp = gexp_prime(x);
        *d_sr += r->eta0 * r->eta0 * gp / tau0;
        *d_tau0 = -r->eta0 * x * gp / tau0;
        return;
    }
    /* Papanastasiou and Herschel-Bulkley: tau0 f(sr), f(s) = (1 - exp(-s/eps))/s; with
     * x = s/eps, f'(s) = g'(x)/eps^2 */
    double e = r->eps, x = sr / e;
    *d_tau0 = sr == 0.0 ? 1.0 / e : -expm1(-x) / sr;
    *d_sr += tau0 * gexp_prime(x) / (e * e);
}

/* strain_norm backward: d sr / d G_ab = (G_ab + G_ba)/sr (zero at sr = 0) */
static void strain_norm_adj(const double Gm[3][3], double sr, double srb, double Gmb[3][3]) {
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) Gmb[a][b] = sr > 0.0 ? srb * (Gm[a][b] + Gm[b][a]) / sr : 0.0;
}

static void viscosity_adj(const or_geom* g, const or_rheo* r, const double* theta,
                          const double* G, const double* gw, const double* etab,
                          const double* etaebb, double* Gb, double* gwb, double* tau0b) {
    long N = g->N;
    for (long c = 0; c < N; c++) {
        if (g->alpha[c] <= 0.0) continue;
        double Gm[3][3], Gmb[3][3], dsr, dt0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Gm[a][b] = G[(a * 3 + b) * N + c];
        double s = strain_norm(Gm);
        law_deriv(r, r->tau0 * (theta ? theta[c] : 1.0), s, &dsr, &dt0);
        tau0b[c] += dt0 * etab[c];
        strain_norm_adj(Gm, s, dsr * etab[c], Gmb);
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Gb[(a * 3 + b) * N + c] += Gmb[a][b];
    }
    for (int cid = 0; cid < g->ncut; cid++) {
        long c = g->cut[cid];
        const double* nv = &g->nrm[3 * cid];
        double Gm[3][3], Gmb[3][3], dsr, dt0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Gm[a][b] = nv[a] * gw[3 * cid + b];
        double s = strain_norm(Gm);
        law_deriv(r, r->tau0 * (theta ? theta[c] : 1.0), s, &dsr, &dt0);
        tau0b[c] += dt0 * etaebb[cid];
        strain_norm_adj(Gm, s, dsr * etaebb[cid], Gmb);
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) gwb[3 * cid + b] += nv[a] * Gmb[a][b];
    }
}

void or_redistribute_adj(const or_geom* g, int ncomp, const double* Db, double* DCb) {
    const int* n = g->box.n;
    const int* per = g->box.periodic;
    long N = g->N;
    double* S = calloc(N, sizeof(double));
    double* dDb = calloc((long)ncomp * N, sizeof(double));
    for (long c = 0; c < N; c++) {
        if (g->alpha[c] <= 0.0 || g->flag[c] != 1) continue;
        int q[3];
        cell_ijk(n, c, q);
        double s = 0;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    if (!dx && !dy && !dz) continue;
                    int r[3] = {q[0] + dx, q[1] + dy, q[2] + dz};
                    long cc = cell_at(n, per, r);
                    if (cc < 0 || g->alpha[cc] <= 0.0) continue;
                    s += g->alpha[cc];
                }
        S[c] = s;
    }
    /* the second pass adds dD_k / S_k of every cut neighbour k to each open cell */
    for (long c = 0; c < N; c++) {
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    if (!dx && !dy && !dz) continue;
                    int r[3] = {q[0] + dx, q[1] + dy, q[2] + dz};
                    long cc = cell_at(n, per, r);
                    if (cc < 0 || g->flag[cc] != 1 || S[cc] <= 0.0) continue;
                    for (int m = 0; m < ncomp; m++) dDb[m * N + cc] += Db[m * N + c] / S[cc];
                }
    }
    /* the first pass: DH = a DC + (1-a) DNC and dD = a (1-a) (DC - DNC) on cut cells */
    for (long c = 0; c < N; c++) {
        if (g->alpha[c] <= 0.0) continue;
        if (g->flag[c] != 1) {
            for (int m = 0; m < ncomp; m++) DCb[m * N + c] += Db[m * N + c];
            continue;
        }
        double a = g->alpha[c];
        int q[3];
        cell_ijk(n, c, q);
        for (int m = 0; m < ncomp; m++) {
            double dhb = Db[m * N + c], ddb = dDb[m * N + c];
            DCb[m * N + c] += a * dhb + a * (1.0 - a) * ddb;
            double dncb = (1.0 - a) * dhb - a * (1.0 - a) * ddb;
            if (S[c] <= 0.0) {
                DCb[m * N + c] += dncb;
                continue;
            }
            for (int dz = -1; dz <= 1; dz++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        if (!dx && !dy && !dz) continue;
                        int r[3] = {q[0] + dx, q[1] + dy, q[2] + dz};
                        long cc = cell_at(n, per, r);
                        if (cc < 0 || g->alpha[cc] <= 0.0) continue;
                        DCb[m * N + cc] += g->alpha[cc] / S[c] * dncb;
                    }
        }
    }
    free(S);
    free(dDb);
}

static void transpose_term_adj(const or_geom* g, const double* eta, const double* eta_eb,
                               const double* u, const double* G, const double* gw,
                               const double* DCb, double* etab, double* etaebb, double* ub,
                               double* Gb, double* gwb) {
    const int* n = g->box.n;
    const int* per = g->box.periodic;
    long N = g->N;
    double h = g->box.h;
    for (long c = 0; c < N; c++) {
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int j = 0; j < 3; j++) {
            double wj = DCb[j * N + c] / (g->alpha[c] * h);
            for (int d = 0; d < 3; d++)
                for (int side = -1; side <= 1; side += 2) {
                    int f[3] = {q[0], q[1], q[2]};
                    if (side > 0) f[d] += 1;
                    double A = g->ap[d][fidx(n, d, f[0], f[1], f[2])];
                    if (A == 0.0) continue;
                    int r[3] = {q[0], q[1], q[2]};
                    r[d] += side;
                    long nb = cell_at(n, per, r);
                    const double* ud = u + (long)d * N;
                    double cf = side * A * wj; /* adjoint of the face flux F */
                    if (nb >= 0) {
                        double ef = 0.5 * (eta[c] + eta[nb]);
                        double der;
                        if (j == d)
                            der = side > 0 ? (ud[nb] - ud[c]) / h : (ud[c] - ud[nb]) / h;
                        else
                            der = 0.5 * (G[(j * 3 + d) * N + c] + G[(j * 3 + d) * N + nb]);
                        etab[c] += 0.5 * cf * der;
                        etab[nb] += 0.5 * cf * der;
                        if (j == d) {
                            double t = cf * ef / h;
                            ub[d * N + nb] += side > 0 ? t : -t;
                            ub[d * N + c] += side > 0 ? -t : t;
                        } else {
                            Gb[(j * 3 + d) * N + c] += 0.5 * cf * ef;
                            Gb[(j * 3 + d) * N + nb] += 0.5 * cf * ef;
                        }
                    } else if (j == d) {
                        double uw = g->box.wall_u[2 * d + (side > 0)][d];
                        double der = side > 0 ? (uw - ud[c]) / (0.5 * h) : (ud[c] - uw) / (0.5 * h);
                        etab[c] += cf * der;
                        double t = cf * eta[c] / (0.5 * h);
                        ub[d * N + c] += side > 0 ? -t : t;
                    }
                }
            long cid = g->cutid[c];
            if (cid >= 0) {
                const double* nv = &g->nrm[3 * cid];
                double ng = nv[0] * gw[3 * cid] + nv[1] * gw[3 * cid + 1] + nv[2] * gw[3 * cid + 2];
                etaebb[cid] += -g->aeb[cid] * nv[j] * ng * wj;
                for (int b = 0; b < 3; b++)
                    gwb[3 * cid + b] += -g->aeb[cid] * eta_eb[cid] * nv[j] * nv[b] * wj;
            }
        }
    }
}

/* limited slope backward with the branch of the forward frozen: the slope equals the central
 * difference, twice the left or twice the right difference, or zero */
static void mc_slope_adj(const or_geom* g, const double* uj, long c, int d, double sb,
                         double* ubj) {
    const int* n = g->box.n;
    int q[3];
    cell_ijk(n, c, q);
    int r[3];
    memcpy(r, q, sizeof(r));
    r[d] = q[d] - 1;
    long lo = cell_at(n, g->box.periodic, r);
    r[d] = q[d] + 1;
    long hi = cell_at(n, g->box.periodic, r);
    if (lo < 0 || hi < 0) return;
    if (g->alpha[lo] <= 0.0 || g->alpha[hi] <= 0.0) return;
    double dl = uj[c] - uj[lo], dr = uj[hi] - uj[c], dc = 0.5 * (uj[hi] - uj[lo]);
    if (dl * dr <= 0.0) return;
    double adc = fabs(dc), al = 2.0 * fabs(dl), ar = 2.0 * fabs(dr);
    if (adc <= fmin(al, ar)) {
        ubj[hi] += 0.5 * sb;
        ubj[lo] -= 0.5 * sb;
    } else if (al <= ar) {
        ubj[c] += 2.0 * sb;
        ubj[lo] -= 2.0 * sb;
    } else {
        ubj[hi] += 2.0 * sb;
        ubj[c] -= 2.0 * sb;
    }
}

static void face_states_adj(const or_geom* g, const double* uj, long lo, long hi, int d,
                            double uLb, double uRb, double* ubj) {
    ubj[lo] += uLb;
    mc_slope_adj(g, uj, lo, d, 0.5 * uLb, ubj);
    ubj[hi] += uRb;
    mc_slope_adj(g, uj, hi, d, -0.5 * uRb, ubj);
}

void or_face_extrap_adj(const or_geom* g, const double* u, const double* fbx,
                        const double* fby, const double* fbz, double* ub) {
    const int* n = g->box.n;
    const double* fb[3] = {fbx, fby, fbz};
    for (int d = 0; d < 3; d++) {
        int m[3] = {n[0] + (d == 0), n[1] + (d == 1), n[2] + (d == 2)};
        for (int k = 0; k < m[2]; k++)
            for (int j = 0; j < m[1]; j++)
                for (int i = 0; i < m[0]; i++) {
                    int f[3] = {i, j, k};
                    long fi = fidx(n, d, i, j, k);
                    long lo, hi;
                    face_cells(g, d, f, &lo, &hi);
                    if (lo < 0 || hi < 0 || g->ap[d][fi] <= 0.0) continue;
                    const double* ud = u + (long)d * g->N;
                    double uL, uR;
                    face_states(g, ud, lo, hi, d, &uL, &uR);
                    if (uL > 0.0 && uL + uR > 0.0)
                        face_states_adj(g, ud, lo, hi, d, fb[d][fi], 0.0, ub + (long)d * g->N);
                    else if (uR < 0.0 && uL + uR < 0.0)
                        face_states_adj(g, ud, lo, hi, d, 0.0, fb[d][fi], ub + (long)d * g->N);
                }
    }
}

static void conv_adj(const or_geom* g, const double* u, double* const uf[3], const double* DCb,
                     double* ub, double* const ufb[3]) {
    const int* n = g->box.n;
    long N = g->N;
    double h = g->box.h;
    for (long c = 0; c < N; c++) {
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int j = 0; j < 3; j++) {
            double wj = -DCb[j * N + c] / (g->alpha[c] * h);
            for (int d = 0; d < 3; d++)
                for (int side = -1; side <= 1; side += 2) {
                    int f[3] = {q[0], q[1], q[2]};
                    if (side > 0) f[d] += 1;
                    long fi = fidx(n, d, f[0], f[1], f[2]);
                    double A = g->ap[d][fi];
                    if (A == 0.0) continue;
                    long lo, hi;
                    face_cells(g, d, f, &lo, &hi);
                    double w = uf[d][fi], cf = side * A * wj;
                    if (lo < 0 || hi < 0) {
                        ufb[d][fi] += cf * g->box.wall_u[2 * d + (lo >= 0)][j];
                        continue;
                    }
                    double uL, uR;
                    face_states(g, u + (long)j * N, lo, hi, d, &uL, &uR);
                    double up = w > 0.0 ? uL : (w < 0.0 ? uR : 0.5 * (uL + uR));
                    ufb[d][fi] += cf * up;
                    double upb = cf * w;
                    double uLb = w > 0.0 ? upb : (w < 0.0 ? 0.0 : 0.5 * upb);
                    double uRb = w > 0.0 ? 0.0 : (w < 0.0 ? upb : 0.5 * upb);
                    face_states_adj(g, u + (long)j * N, lo, hi, d, uLb, uRb, ub + (long)j * N);
                }
        }
    }
}

/* transpose of the face gradient G_f (open interior faces) applied to a face field */
static void face_grad_T(const or_geom* g, double* const fb[3], double* y) {
    const int* n = g->box.n;
    double h = g->box.h;
    memset(y, 0, g->N * sizeof(double));
    for (int d = 0; d < 3; d++) {
        int m[3] = {n[0] + (d == 0), n[1] + (d == 1), n[2] + (d == 2)};
        for (int k = 0; k < m[2]; k++)
            for (int j = 0; j < m[1]; j++)
                for (int i = 0; i < m[0]; i++) {
                    int f[3] = {i, j, k};
                    long fi = fidx(n, d, i, j, k);
                    long lo, hi;
                    face_cells(g, d, f, &lo, &hi);
                    if (lo < 0 || hi < 0 || g->ap[d][fi] == 0.0) continue;
                    y[hi] += fb[d][fi] / h;
                    y[lo] -= fb[d][fi] / h;
                }
    }
}

/* face field t = D^T z, the transpose of the linear part of or_divergence.  Along a periodic
 * direction faces 0 and n are stored twice; face 0 enters only the divergence of the cell above
 * it and face n only that of the cell below it. */
static void div_T(const or_geom* g, const double* z, double* const t[3]) {
    const int* n = g->box.n;
    double h = g->box.h;
    for (int d = 0; d < 3; d++) {
        int m[3] = {n[0] + (d == 0), n[1] + (d == 1), n[2] + (d == 2)};
        for (int k = 0; k < m[2]; k++)
            for (int j = 0; j < m[1]; j++)
                for (int i = 0; i < m[0]; i++) {
                    int f[3] = {i, j, k};
                    long fi = fidx(n, d, i, j, k);
                    long lo, hi;
                    face_cells(g, d, f, &lo, &hi);
                    double s = 0.0;
                    if (f[d] > 0 && lo >= 0 && g->alpha[lo] > 0.0) s += z[lo];
                    if (f[d] < n[d] && hi >= 0 && g->alpha[hi] > 0.0) s -= z[hi];
                    t[d][fi] = g->ap[d][fi] * s / h;
                }
    }
}

/* MAC projection backward.  Forward (exact solve): w' = w + beta G_f L^+ D w + const, with
 * L the Poisson matrix (symmetric) and L^+ its pseudo-inverse on the open cells (the mean
 * removal makes the right-hand side consistent).  Backward: wb += beta D^T L^+ G_f^T wb. */
int or_mac_project_adj(const or_geom* g_in, double beta, double* fbx, double* fby, double* fbz,
                       double rtol, int maxit, const or_opts* o, int* iters) {
    or_geom* g = (or_geom*)g_in;
    const int* n = g->box.n;
    long N = g->N;
    double* fb[3] = {fbx, fby, fbz};
    double* y = malloc(N * sizeof(double));
    double* z = calloc(N, sizeof(double));
    double* t[3];
    for (int d = 0; d < 3; d++) t[d] = malloc(nfaces(n, d) * sizeof(double));
    face_grad_T(g, fb, y);
    double scale = vmaxabs(y, N); /* stop rule: max|r| <= rtol * max|G_f^T wb| */
    for (long c = 0; c < N; c++) y[c] = -y[c];
    /* poisson_solve solves L z = -(div - mean(div)) with zero-mean z: here div = -y */
    int ret = poisson_solve(g, beta, y, z, rtol, scale, maxit, o, iters);
    div_T(g, z, t);
    for (int d = 0; d < 3; d++)
        for (long f = 0; f < nfaces(n, d); f++) fb[d][f] += beta * t[d][f];
    for (int d = 0; d < 3; d++) free(t[d]);
    free(y);
    free(z);
    return ret;
}

/* transpose of or_gcc, accumulated into pb */
void or_gcc_adj(const or_geom* g, const double* gpb, double* pb) {
    const int* n = g->box.n;
    long N = g->N;
    double h = g->box.h;
    for (long c = 0; c < N; c++) {
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int d = 0; d < 3; d++) {
            double den = 0;
            for (int side = -1; side <= 1; side += 2) {
                int f[3] = {q[0], q[1], q[2]};
                if (side > 0) f[d] += 1;
                den += g->ap[d][fidx(n, d, f[0], f[1], f[2])];
            }
            if (den <= 0.0) continue;
            for (int side = -1; side <= 1; side += 2) {
                int f[3] = {q[0], q[1], q[2]};
                if (side > 0) f[d] += 1;
                double A = g->ap[d][fidx(n, d, f[0], f[1], f[2])];
                if (A == 0.0) continue;
                long lo, hi;
                face_cells(g, d, f, &lo, &hi);
                if (lo < 0 || hi < 0) continue;
                double tt = gpb[d * N + c] * A / (den * h);
                pb[hi] += tt;
                pb[lo] -= tt;
            }
        }
    }
}

/* end-of-stage projection backward.  Forward: u1 = u + beta Gcc p_old, w = F u1 + const,
 * phi = -L^+ D w, u_new = u1 - beta Gcc phi, p_new = phi.  On entry ub, pb hold the adjoints
 * of u_new, p_new; on exit those of u and p_old (overwritten, open cells only). */
int or_cc_project_adj(const or_geom* g_in, double beta, double* ub, double* pb, double rtol,
                      int maxit, const or_opts* o, int* iters) {
    or_geom* g = (or_geom*)g_in;
    const int* n = g->box.n;
    long N = g->N;
    double* phib = calloc(N, sizeof(double));
    double* gpb = malloc(3 * N * sizeof(double));
    double* z = calloc(N, sizeof(double));
    double* t[3];
    for (int d = 0; d < 3; d++) t[d] = malloc(nfaces(n, d) * sizeof(double));
    for (long q = 0; q < 3 * N; q++) gpb[q] = g->alpha[q % N] > 0.0 ? -beta * ub[q] : 0.0;
    for (long c = 0; c < N; c++) phib[c] = g->alpha[c] > 0.0 ? pb[c] : 0.0;
    or_gcc_adj(g, gpb, phib);
    double scale = vmaxabs(phib, N);
    for (long c = 0; c < N; c++) phib[c] = -phib[c];
    /* z = L^+ phib (poisson_solve with div = -phib) */
    int ret = poisson_solve(g, beta, phib, z, rtol, scale, maxit, o, iters);
    div_T(g, z, t);
    /* ub1 = ub - F^T D^T z */
    for (int d = 0; d < 3; d++) {
        int m[3] = {n[0] + (d == 0), n[1] + (d == 1), n[2] + (d == 2)};
        for (int k = 0; k < m[2]; k++)
            for (int j = 0; j < m[1]; j++)
                for (int i = 0; i < m[0]; i++) {
                    int f[3] = {i, j, k};
                    long fi = fidx(n, d, i, j, k);
                    long lo, hi;
                    face_cells(g, d, f, &lo, &hi);
                    if (lo < 0 || hi < 0 || g->ap[d][fi] <= 0.0) continue;
                    ub[(long)d * N + lo] -= 0.5 * t[d][fi];
                    ub[(long)d * N + hi] -= 0.5 * t[d][fi];
                }
    }
    for (long q = 0; q < 3 * N; q++) {
        if (g->alpha[q % N] <= 0.0) ub[q] = 0.0;
        gpb[q] = beta * ub[q];
    }
    memset(pb, 0, N * sizeof(double));
    or_gcc_adj(g, gpb, pb);
    for (int d = 0; d < 3; d++) free(t[d]);
    free(phib);
    free(gpb);
    free(z);
    return ret;
}

/* transpose of the homogeneous viscous operator of or_visc_apply: the 7-point part is
 * symmetric, the wall-flux rows of the cut cells are scattered back onto their stencils */
static void visc_apply_T(const or_geom* g, double rho, double dt, const double* eta,
                         const double* eta_eb, const double* lam, double* out) {
    long N = g->N;
    const int* n = g->box.n;
    const int* per = g->box.periodic;
    double h = g->box.h;
    for (long c = 0; c < N; c++) {
        for (int j = 0; j < 3; j++) out[j * N + c] = 0.0;
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int j = 0; j < 3; j++) {
            const double* lj = lam + (long)j * N;
            double acc = g->alpha[c] * rho * lj[c];
            for (int d = 0; d < 3; d++)
                for (int side = -1; side <= 1; side += 2) {
                    int f[3] = {q[0], q[1], q[2]};
                    if (side > 0) f[d] += 1;
                    double A = g->ap[d][fidx(n, d, f[0], f[1], f[2])];
                    if (A == 0.0) continue;
                    int r[3] = {q[0], q[1], q[2]};
                    r[d] += side;
                    long nb = cell_at(n, per, r);
                    if (nb >= 0) acc -= dt * A * 0.5 * (eta[c] + eta[nb]) / (h * h) * (lj[nb] - lj[c]);
                    else acc += 2.0 * dt * A * eta[c] / (h * h) * lj[c];
                }
            out[j * N + c] = acc;
        }
    }
    for (int cid = 0; cid < g->ncut; cid++) {
        long c = g->cut[cid];
        for (int j = 0; j < 3; j++)
            wall_dudn_adj(g, cid, dt * g->aeb[cid] * eta_eb[cid] * lam[j * N + c] / h,
                          out + (long)j * N);
    }
}

/* BiCGSTAB on A^T lam = rhs, right-preconditioned by the same (symmetric) V-cycle; the
 * viscous operator of the multigrid levels must already be built */
static int visc_solve_T(or_geom* g, double rho, double dt, const double* eta,
                        const double* eta_eb, const double* rhs, double* x, double rtol,
                        int maxit, const or_opts* o, int* iters) {
    long N3 = 3 * g->N;
    double* r = malloc(N3 * sizeof(double));
    double* rh = malloc(N3 * sizeof(double));
    double* p = calloc(N3, sizeof(double));
    double* v = calloc(N3, sizeof(double));
    double* ph = malloc(N3 * sizeof(double));
    double* s = malloc(N3 * sizeof(double));
    double* sh = malloc(N3 * sizeof(double));
    double* t = malloc(N3 * sizeof(double));
    int ret = OR_ENOCONV;
    *iters = 0;
    memset(x, 0, N3 * sizeof(double));
    memcpy(r, rhs, N3 * sizeof(double));
    double bn = vmaxabs(rhs, N3), tol = rtol * bn;
    if (!isfinite(bn)) {
        ret = OR_ENAN;
        goto done;
    }
    if (bn == 0.0) {
        ret = OR_OK;
        goto done;
    }
    memcpy(rh, r, N3 * sizeof(double));
    double rho_old = 1, al = 1, om = 1;
    for (int it = 1; it <= maxit; it++) {
        double rr = vdot(rh, r, N3);
        double be = (rr / rho_old) * (al / om);
        for (long q = 0; q < N3; q++) p[q] = r[q] + be * (p[q] - om * v[q]);
        vcycle_level(g, 0, 3, p, ph, o);
        visc_apply_T(g, rho, dt, eta, eta_eb, ph, v);
        al = rr / vdot(rh, v, N3);
        for (long q = 0; q < N3; q++) s[q] = r[q] - al * v[q];
        *iters = it;
        double sn = vmaxabs(s, N3);
        if (!isfinite(sn)) {
            ret = OR_ENAN;
            break;
        }
        if (sn <= tol) {
            for (long q = 0; q < N3; q++) x[q] += al * ph[q];
            ret = OR_OK;
            break;
        }
        vcycle_level(g, 0, 3, s, sh, o);
        visc_apply_T(g, rho, dt, eta, eta_eb, sh, t);
        om = vdot(t, s, N3) / vdot(t, t, N3);
        for (long q = 0; q < N3; q++) {
            x[q] += al * ph[q] + om * sh[q];
            r[q] = s[q] - om * t[q];
        }
        double rn = vmaxabs(r, N3);
        if (!isfinite(rn)) {
            ret = OR_ENAN;
            break;
        }
        if (rn <= tol) {
            ret = OR_OK;
            break;
        }
        rho_old = rr;
    }
done:
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t);
    return ret;
}

/* viscosity backward of the viscous residual R(u; eta) = or_visc_apply(u) (with boundary
 * values): etab -= (dR/deta)^T lam, etaebb -= (dR/deta_EB)^T lam at the solution u */
static void visc_coef_adj(const or_geom* g, double dt, const double* u, const double* lam,
                          double* etab, double* etaebb) {
    const int* n = g->box.n;
    const int* per = g->box.periodic;
    long N = g->N;
    double h = g->box.h;
    for (long c = 0; c < N; c++) {
        if (g->alpha[c] <= 0.0) continue;
        int q[3];
        cell_ijk(n, c, q);
        for (int d = 0; d < 3; d++)
            for (int side = -1; side <= 1; side += 2) {
                int f[3] = {q[0], q[1], q[2]};
                if (side > 0) f[d] += 1;
                double A = g->ap[d][fidx(n, d, f[0], f[1], f[2])];
                if (A == 0.0) continue;
                int r[3] = {q[0], q[1], q[2]};
                r[d] += side;
                long nb = cell_at(n, per, r);
                for (int j = 0; j < 3; j++) {
                    const double* uj = u + (long)j * N;
                    double lc = lam[j * N + c];
                    if (nb >= 0) {
                        double t = dt * A / (2.0 * h * h) * (uj[nb] - uj[c]) * lc;
                        etab[c] += t;
                        etab[nb] += t;
                    } else {
                        double uw = g->box.wall_u[2 * d + (side > 0)][j];
                        etab[c] += 2.0 * dt * A / (h * h) * (uw - uj[c]) * lc;
                    }
                }
            }
    }
    for (int cid = 0; cid < g->ncut; cid++) {
        long c = g->cut[cid];
        for (int j = 0; j < 3; j++)
            etaebb[cid] -= dt * g->aeb[cid] / h *
                           wall_dudn(g, cid, u + (long)j * N, g->body.u_eb[j]) * lam[j * N + c];
    }
}

/* backward of the implicit viscous solve R(x; eta) = alpha psi: lam = A^-T xb,
 * psib += alpha lam, and the viscosity adjoints accumulate */
static int visc_solve_adj(or_geom* g, double rho, double dt, const double* eta,
                          const double* eta_eb, const double* x, const double* xb, double rtol,
                          int maxit, const or_opts* o, double* psib, double* etab,
                          double* etaebb, int* iters) {
    long N = g->N, N3 = 3 * N;
    double* rhs = malloc(N3 * sizeof(double));
    double* lam = malloc(N3 * sizeof(double));
    for (long q = 0; q < N3; q++) rhs[q] = g->alpha[q % N] > 0.0 ? xb[q] : 0.0;
    build_operator(g, SYS_VISC, 0, rho, dt, eta, eta_eb);
    int ret = visc_solve_T(g, rho, dt, eta, eta_eb, rhs, lam, rtol, maxit, o, iters);
    for (long q = 0; q < N3; q++) psib[q] += g->alpha[q % N] * lam[q];
    visc_coef_adj(g, dt, x, lam, etab, etaebb);
    free(rhs);
    free(lam);
    return ret;
}

int or_visc_solve_adj(const or_geom* g, double rho, double dt, const double* eta,
                      const double* eta_eb, const double* x, const double* xb, double rtol,
                      int maxit, const or_opts* o, double* psib, double* etab, double* etaebb,
                      int* iters) {
    return visc_solve_adj((or_geom*)g, rho, dt, eta, eta_eb, x, xb, rtol, maxit, o, psib, etab,
                          etaebb, iters);
}

/* backward of the derived quantities (C, eta, eta_EB, V) at u; uf: the projected face
 * velocities of the forward (nullable: recomputed) */
int or_derived_adj(const or_geom* g_in, const or_rheo* rh, const double* theta, const double* u,
                   const double* const uf_in[3], const or_opts* o, const double* Cb,
                   const double* etab_in, const double* etaebb_in, const double* Vb, double* ub,
                   double* tau0b, int* iters) {
    or_geom* g = (or_geom*)g_in;
    const int* n = g->box.n;
    long N = g->N;
    int nc = g->ncut + 1;
    double* uf[3];
    double* ufb[3];
    for (int d = 0; d < 3; d++) {
        uf[d] = malloc(nfaces(n, d) * sizeof(double));
        ufb[d] = calloc(nfaces(n, d), sizeof(double));
    }
    int ret = OR_OK, it = 0;
    if (uf_in) {
        for (int d = 0; d < 3; d++) memcpy(uf[d], uf_in[d], nfaces(n, d) * sizeof(double));
    } else {
        double* phi = calloc(N, sizeof(double));
        or_face_extrap(g, u, uf[0], uf[1], uf[2]);
        ret = or_mac_project(g, 1.0, uf[0], uf[1], uf[2], phi, o->rtol_mac, o->max_iter, o,
                             NULL, &it);
        free(phi);
    }
    double* gw = calloc(3 * nc, sizeof(double));
    double* G = malloc(9 * N * sizeof(double));
    double* eta = malloc(N * sizeof(double));
    double* eta_eb = calloc(nc, sizeof(double));
    double* etab = malloc(N * sizeof(double));
    double* etaebb = calloc(nc, sizeof(double));
    double* DCb = calloc(3 * N, sizeof(double));
    double* Gb = calloc(9 * N, sizeof(double));
    double* gwb = calloc(3 * nc, sizeof(double));
    or_wall_gradient(g, u, gw);
    or_cell_gradient(g, u, gw, G);
    viscosity_from(g, rh, theta, G, gw, eta, eta_eb, NULL);
    memcpy(etab, etab_in, N * sizeof(double));
    memcpy(etaebb, etaebb_in, g->ncut * sizeof(double));
    /* V = R(DC_V) */
    or_redistribute_adj(g, 3, Vb, DCb);
    transpose_term_adj(g, eta, eta_eb, u, G, gw, DCb, etab, etaebb, ub, Gb, gwb);
    viscosity_adj(g, rh, theta, G, gw, etab, etaebb, Gb, gwb, tau0b);
    or_cell_gradient_adj(g, Gb, ub, gwb);
    or_wall_gradient_adj(g, gwb, ub);
    /* C = R(DC_C(u, P uf(u))) */
    memset(DCb, 0, 3 * N * sizeof(double));
    or_redistribute_adj(g, 3, Cb, DCb);
    conv_adj(g, u, uf, DCb, ub, ufb);
    int e = or_mac_project_adj(g, 1.0, ufb[0], ufb[1], ufb[2], o->rtol_mac, o->max_iter, o,
                               iters);
    if (e) ret = e;
    or_face_extrap_adj(g, u, ufb[0], ufb[1], ufb[2], ub);
    for (int d = 0; d < 3; d++) {
        free(uf[d]);
        free(ufb[d]);
    }
    free(gw); free(G); free(eta); free(eta_eb); free(etab); free(etaebb);
    free(DCb); free(Gb); free(gwb);
    return ret;
}

/* backward of psi = rho u + dt (rho C + V - Gcc p + f) */
static void psi_adj(const or_geom* g, double rho, double dt, const double* psib, double* ub,
                    double* Cb, double* Vb, double* pb) {
    long N3 = 3 * g->N;
    double* gpb = malloc(N3 * sizeof(double));
    for (long q = 0; q < N3; q++) {
        ub[q] += rho * psib[q];
        Cb[q] += dt * rho * psib[q];
        Vb[q] += dt * psib[q];
        gpb[q] = -dt * psib[q];
    }
    or_gcc_adj(g, gpb, pb);
    free(gpb);
}

int or_rk2_step_adjoint(const or_geom* g_in, const or_rheo* rh, const double* theta, double dt,
                        const or_opts* o, const double* u0, const double* p0, double* ub,
                        double* pb, double* tau0b, or_stats* st) {
    or_geom* g = (or_geom*)g_in;
    const int* n = g->box.n;
    long N = g->N, N3 = 3 * N;
    int nc = g->ncut + 1;
    double rho = rh->rho, beta = dt / rh->rho;
    int err = OR_OK, e, it;
    or_stats loc;
    memset(&loc, 0, sizeof(loc));
    /* replay the forward step, keeping its intermediate fields */
    rk2_tape tp;
    for (int d = 0; d < 3; d++) {
        tp.ufm[d] = malloc(nfaces(n, d) * 8);
        tp.uf1[d] = malloc(nfaces(n, d) * 8);
    }
    tp.em = malloc(N * 8);
    tp.ea = malloc(N * 8);
    tp.ebm = calloc(nc, 8);
    tp.eba = calloc(nc, 8);
    tp.us1 = malloc(N3 * 8);
    tp.u1 = malloc(N3 * 8);
    tp.us2 = malloc(N3 * 8);
    double* u = malloc(N3 * 8);
    double* p = malloc(N * 8);
    memcpy(u, u0, N3 * 8);
    memcpy(p, p0, N * 8);
    e = rk2_impl(g, rh, theta, dt, o, u, p, NULL, &tp);
    if (e) err = e;
    /* reverse sweep */
    double* ubm = calloc(N3, 8); /* adjoint of u^m, accumulated */
    double* x = malloc(N3 * 8);
    double* pbs = malloc(N * 8);
    double* psib = calloc(N3, 8);
    double* Cb = calloc(N3, 8);
    double* Vb = calloc(N3, 8);
    double* etab = calloc(N, 8);
    double* etaebb = calloc(nc, 8);
    double* Ch = malloc(N3 * 8);
    double* Vh = malloc(N3 * 8);
    double* eh = malloc(N * 8);
    double* ebh = calloc(nc, 8);
    for (long q = 0; q < N3; q++) x[q] = g->alpha[q % N] > 0.0 ? ub[q] : 0.0;
    for (long c = 0; c < N; c++) pbs[c] = g->alpha[c] > 0.0 ? pb[c] : 0.0;
    /* corrector projection and solve */
    e = or_cc_project_adj(g, beta, x, pbs, o->rtol_proj, o->max_iter, o, &it);
    loc.it_proj[1] = it;
    if (e) err = e;
    e = visc_solve_adj(g, rho, dt, tp.ea, tp.eba, tp.us2, x, o->rtol_visc, o->max_iter, o, psib,
                       etab, etaebb, &it);
    loc.it_visc[1] = it;
    if (e) err = e;
    psi_adj(g, rho, dt, psib, ubm, Cb, Vb, pbs);
    /* averages: both stages receive half */
    for (long q = 0; q < N3; q++) {
        Ch[q] = 0.5 * Cb[q];
        Vh[q] = 0.5 * Vb[q];
    }
    for (long c = 0; c < N; c++) eh[c] = 0.5 * etab[c];
    for (int c = 0; c < g->ncut; c++) ebh[c] = 0.5 * etaebb[c];
    /* corrector derived quantities at u* */
    memset(x, 0, N3 * 8);
    e = or_derived_adj(g, rh, theta, tp.u1, (const double* const*)tp.uf1, o, Ch, eh, ebh, Vh, x,
                       tau0b, &it);
    loc.it_mac[1] = it;
    if (e) err = e;
    /* predictor projection and solve */
    e = or_cc_project_adj(g, beta, x, pbs, o->rtol_proj, o->max_iter, o, &it);
    loc.it_proj[0] = it;
    if (e) err = e;
    memset(psib, 0, N3 * 8);
    e = visc_solve_adj(g, rho, dt, tp.em, tp.ebm, tp.us1, x, o->rtol_visc, o->max_iter, o, psib,
                       eh, ebh, &it);
    loc.it_visc[0] = it;
    if (e) err = e;
    memcpy(Cb, Ch, N3 * 8);
    memcpy(Vb, Vh, N3 * 8);
    psi_adj(g, rho, dt, psib, ubm, Cb, Vb, pbs);
    e = or_derived_adj(g, rh, theta, u0, (const double* const*)tp.ufm, o, Cb, eh, ebh, Vb, ubm,
                       tau0b, &it);
    loc.it_mac[0] = it;
    if (e) err = e;
    for (long q = 0; q < N3; q++) ub[q] = g->alpha[q % N] > 0.0 ? ubm[q] : 0.0;
    for (long c = 0; c < N; c++) pb[c] = g->alpha[c] > 0.0 ? pbs[c] : 0.0;
    if (st) *st = loc;
    for (int d = 0; d < 3; d++) {
        free(tp.ufm[d]);
        free(tp.uf1[d]);
    }
    free(tp.em); free(tp.ea); free(tp.ebm); free(tp.eba); free(tp.us1); free(tp.u1);
    free(tp.us2); free(u); free(p); free(ubm); free(x); free(pbs); free(psib); free(Cb);
    free(Vb); free(etab); free(etaebb); free(Ch); free(Vh); free(eh); free(ebh);
    return err;
}

/* drag backward: Fb is d(loss)/dF; ub, pb, tau0b accumulate */
void or_drag_adj(const or_geom* g, const or_rheo* r, const double* theta, const double* u,
                 const double Fb[3], double* ub, double* pb, double* tau0b) {
    long N = g->N;
    double h = g->box.h;
    double* gw = calloc(3 * (g->ncut + 1), sizeof(double));
    double* gwb = calloc(3 * (g->ncut + 1), sizeof(double));
    double* gpb = calloc(3 * N, sizeof(double));
    or_wall_gradient(g, u, gw);
    for (int cid = 0; cid < g->ncut; cid++) {
        long c = g->cut[cid];
        const double* nv = &g->nrm[3 * cid];
        const double* gg = &gw[3 * cid];
        double Gm[3][3], Gmb[3][3], Sb[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Gm[a][b] = nv[a] * gg[b];
        double t0 = r->tau0 * (theta ? theta[c] : 1.0);
        double sr = strain_norm(Gm);
        double eeb = law_eta(r, t0, sr), dsr, dt0;
        law_deriv(r, t0, sr, &dsr, &dt0);
        double w[3], etab = 0.0, peb = 0.0;
        for (int a = 0; a < 3; a++) w[a] = Fb[a] * g->aeb[cid] * h * h;
        for (int a = 0; a < 3; a++) {
            for (int b = 0; b < 3; b++) etab += w[a] * (Gm[a][b] + Gm[b][a]) * nv[b];
            peb -= w[a] * nv[a];
        }
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Gmb[a][b] = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                Gmb[a][b] += eeb * w[a] * nv[b];
                Gmb[b][a] += eeb * w[a] * nv[b];
            }
        tau0b[c] += dt0 * etab;
        strain_norm_adj(Gm, sr, dsr * etab, Sb);
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) gwb[3 * cid + b] += nv[a] * (Gmb[a][b] + Sb[a][b]);
        pb[c] += peb;
        for (int d = 0; d < 3; d++) gpb[d * N + c] += h * g->bc[3 * cid + d] * peb;
    }
    or_wall_gradient_adj(g, gwb, ub);
    or_gcc_adj(g, gpb, pb);
    free(gw);
    free(gwb);
    free(gpb);
}
