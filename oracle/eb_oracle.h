/*
 * eb_oracle.h -- plain FP64 CPU oracle for the embedded-boundary (EB) viscoplastic RK2 step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline leg of the bench
 * may load this library.  It shares no code, header or constant with the HIP path.
 *
 * The method follows Sverdrup, Almgren & Nikiforakis, "An embedded boundary approach for efficient
 * simulations of viscoplastic fluids in three dimensions":
 *   Sec. II (Eq. governing, Eqs. bingham:viscosity, papabing:viscosity, Table rheology),
 *   Sec. III.A (Alg. advance, Alg. derived, Eqs. divtau, explicit-viscous, implicit-viscous,
 *               the cell-centred projection Eq. helmholtz, the end-of-stage projection),
 *   Sec. III.B (cut-cell geometry, Eqs. divergence_conservative ... divergence_final,
 *               Eqs. interpolation_distances and dudn, one-sided quadratic gradients),
 *   App. A (Lagrange interpolation).
 * Where the paper is silent, the comment at the function that decides states the reading taken.
 *
 * Layout: cell (i,j,k) -> i + nx*(j + ny*k); vectors are component-major [3][N];
 * faces normal to x: [nz][ny][nx+1], to y: [nz][ny+1][nx], to z: [nz+1][ny][nx].
 * All pointers are host pointers owned by the caller.
 */
#ifndef EB_ORACLE_H
#define EB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int n[3];            /* cells per direction, each even */
    double h;            /* uniform cell size */
    double lo[3];        /* lower domain corner */
    int periodic[3];
    double wall_u[6][3]; /* Dirichlet velocity of faces -x,+x,-y,+y,-z,+z */
} or_box;

/* CYLINDER: circular, radius radii[0], axis along y through the centre (Sec. V.C) */
enum { OR_BODY_NONE = 0, OR_BODY_SPHERE = 1, OR_BODY_ELLIPSOID = 2, OR_BODY_ZSLAB = 3,
       OR_BODY_PLANE = 4, OR_BODY_CYLINDER = 5,
       OR_BODY_CAVITY = 6 };

typedef struct {
    int kind;
    double center[3];
    double radii[3];      /* sphere uses radii[0] */
    double euler_zyx[3];  /* ellipsoid orientation R = Rz(a) Ry(b) Rx(c) */
    double zlo, zhi;      /* z-slab: fluid for zlo < z < zhi */
    double plane_n[3];    /* plane: fluid where n.x > plane_d */
    double plane_d;
    double u_eb[3];       /* velocity of the embedded wall */
} or_body;

/* Table rheology: Newtonian, regularised Bingham (two forms), power law, Herschel-Bulkley and
 * Souza Mendes-Dutra; kappa and n are the power-law consistency and flow index, eta0 the Souza
 * Mendes-Dutra viscosity at zero strain rate. */
enum { OR_LAW_NEWTONIAN = 0, OR_LAW_BINGHAM_REG = 1, OR_LAW_PAPANASTASIOU = 2, OR_LAW_POWER = 3,
       OR_LAW_HERSCHEL_BULKLEY = 4, OR_LAW_SOUZA_MENDES_DUTRA = 5 };

typedef struct {
    int law;
    double mu, tau0, eps, rho;
    double kappa, n, eta0;
} or_rheo;

typedef struct {
    double rtol_visc, rtol_mac, rtol_proj;
    int max_iter;
    int nu1, nu2, nbottom;   /* V(nu1,nu2) smoothing; bottom sweeps on the coarsest level */
    double force[3];         /* body force per unit volume */
    int projection;          /* end-of-stage projection: OR_PROJ_CELL (cell-centred pressure) or
                                OR_PROJ_NODAL (Sec. III.A.4: pressure on the nodes) */
} or_opts;

enum { OR_PROJ_CELL = 0, OR_PROJ_NODAL = 1 };

typedef struct {
    int it_mac[2], it_visc[2], it_proj[2];
    double div_proj[2];
} or_stats;

enum { OR_OK = 0, OR_EINVAL = -1, OR_EGEOM = -2, OR_ENOCONV = -3, OR_ENAN = -4 };

typedef struct or_geom or_geom;

or_geom* or_geom_build(const or_box* box, const or_body* body, int* err);
void or_geom_free(or_geom* g);
int or_geom_ncut(const or_geom* g);
int or_geom_nlevels(const or_geom* g);
int or_geom_nfallback(const or_geom* g);
/* flag: 0 covered, 1 cut, 2 regular */
void or_geom_export(const or_geom* g, uint8_t* flag, double* alpha, double* ax, double* ay,
                    double* az);
/* per cut cell: cell index and [nx ny nz A_EB bx by bz delta nfallback] */
void or_cut_export(const or_geom* g, int64_t* cell, double* data);

void or_wall_gradient(const or_geom* g, const double* u, double* gw /* [ncut][3] */);
void or_cell_gradient(const or_geom* g, const double* u, const double* gw,
                      double* G /* [3][3][N]: G[a][b] = du_b/dx_a */);
void or_viscosity(const or_geom* g, const or_rheo* r, const double* u, const double* theta,
                  double* eta, double* eta_eb, double* sr);
void or_visc_apply(const or_geom* g, double rho, double dt, const double* eta,
                   const double* eta_eb, const double* u, double* out, int homogeneous);
void or_transpose_term(const or_geom* g, const double* eta, const double* eta_eb,
                       const double* u, double* V);
void or_conv_term(const or_geom* g, const double* u, const double* uf_x, const double* uf_y,
                  const double* uf_z, double* C);
void or_redistribute(const or_geom* g, int ncomp, const double* DC, double* D);
void or_face_extrap(const or_geom* g, const double* u, double* fx, double* fy, double* fz);
void or_divergence(const or_geom* g, const double* fx, const double* fy, const double* fz,
                   double* div);
void or_gcc(const or_geom* g, const double* p, double* gp);
void or_poisson_apply(const or_geom* g, double beta, const double* p, double* out);
void or_vcycle(const or_geom* g, int system, double beta, double rho, double dt,
               const double* eta, const double* eta_eb, const double* r, double* e,
               const or_opts* o);
int or_visc_solve(const or_geom* g, double rho, double dt, const double* eta,
                  const double* eta_eb, const double* psi, double* x, double rtol, int maxit,
                  const or_opts* o, int* iters);
int or_mac_project(const or_geom* g, double beta, double* fx, double* fy, double* fz,
                   double* phi, double rtol, int maxit, const or_opts* o, double* div_inf,
                   int* iters);
int or_cc_project(const or_geom* g, double beta, double* u, double* p, double rtol, int maxit,
                  const or_opts* o, double* div_inf, int* iters);
int or_derived(const or_geom* g, const or_rheo* r, const double* theta, const double* u,
               const or_opts* o, double* C, double* eta, double* eta_eb, double* V,
               int* iters);
int or_rk2_step(const or_geom* g, const or_rheo* r, const double* theta, double dt,
                const or_opts* o, double* u, double* p, or_stats* st);
/* Time step of the stability rule (Sec. II.C.1, Eqs. cfl:dt ... cfl:viscous:new). */
double or_stable_dt(const or_geom* g, const or_rheo* r, const double* theta, const double* u,
                    const double force[3], double c_cfl);
void or_drag(const or_geom* g, const or_rheo* r, const double* theta, const double* u,
             const double* p, double F[3]);

/* ---- nodal projection (Sec. III.A.4).  Nodal arrays are [nz+1][ny+1][nx+1] (x fastest); in a
 * periodic direction the last node is a copy of the first. ---- */
/* weak nodal divergence of a cell field w [3][N] (boundary flux not included) */
void or_nodal_div(const or_geom* g, const double* w, double* dn);
/* the boundary flux B of the domain walls and the embedded wall */
void or_nodal_bflux(const or_geom* g, double* bn);
/* the volume-fraction-weighted trilinear stiffness matrix applied to a nodal field */
void or_nodal_apply(const or_geom* g, const double* x, double* y);
/* cell average of the gradient of the trilinear interpolant: gp [3][N] */
void or_nodal_grad(const or_geom* g, const double* q, double* gp);
/* end-of-stage projection with a nodal pressure pn (in: old, out: new) */
int or_nodal_project(const or_geom* g, double beta, double* u, double* pn, double rtol,
                     int maxit, double* div_inf, int* iters);
/* drag with a nodal pressure (trilinear interpolation of pn at the wall centroid) */
void or_drag_nodal(const or_geom* g, const or_rheo* r, const double* theta, const double* u,
                   const double* pn, double F[3]);

/* ---- adjoint (reverse mode): exact transposes of the linearised forward routines, solves taken
 * as exact, switches frozen at their forward values.  Arguments ending in b are adjoints
 * (d loss / d quantity) and accumulate unless stated otherwise. ---- */
void or_wall_gradient_adj(const or_geom* g, const double* gwb, double* ub);
void or_cell_gradient_adj(const or_geom* g, const double* Gb, double* ub, double* gwb);
void or_redistribute_adj(const or_geom* g, int ncomp, const double* Db, double* DCb);
void or_face_extrap_adj(const or_geom* g, const double* u, const double* fbx, const double* fby,
                        const double* fbz, double* ub);
void or_gcc_adj(const or_geom* g, const double* gpb, double* pb);
/* in place: face adjoints of the projected field in, of the input field out */
int or_mac_project_adj(const or_geom* g, double beta, double* fbx, double* fby, double* fbz,
                       double rtol, int maxit, const or_opts* o, int* iters);
/* in place: (ub, pb) of (u_new, p_new) in, of (u, p_old) out */
int or_cc_project_adj(const or_geom* g, double beta, double* ub, double* pb, double rtol,
                      int maxit, const or_opts* o, int* iters);
/* x: the forward solution; xb its adjoint; psib, etab, etaebb accumulate */
int or_visc_solve_adj(const or_geom* g, double rho, double dt, const double* eta,
                      const double* eta_eb, const double* x, const double* xb, double rtol,
                      int maxit, const or_opts* o, double* psib, double* etab, double* etaebb,
                      int* iters);
/* uf: projected face velocities of the forward (nullable: recomputed) */
int or_derived_adj(const or_geom* g, const or_rheo* r, const double* theta, const double* u,
                   const double* const uf[3], const or_opts* o, const double* Cb,
                   const double* etab, const double* etaebb, const double* Vb, double* ub,
                   double* tau0b, int* iters);
/* (u0, p0): the step's input.  ub, pb: adjoints of the step's output on entry, of its input on
 * exit.  tau0b[c] accumulates d loss / d tau0_c, with tau0_c = tau0 * theta[c]. */
int or_rk2_step_adjoint(const or_geom* g, const or_rheo* r, const double* theta, double dt,
                        const or_opts* o, const double* u0, const double* p0, double* ub,
                        double* pb, double* tau0b, or_stats* st);
void or_drag_adj(const or_geom* g, const or_rheo* r, const double* theta, const double* u,
                 const double Fb[3], double* ub, double* pb, double* tau0b);

#ifdef __cplusplus
}
#endif
#endif
