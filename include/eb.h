/*
 * eb.h -- C ABI of the MI355X (gfx950) library for one two-stage Runge-Kutta step of 3D
 * incompressible generalised-Newtonian flow on a single box with embedded-boundary (EB) cut
 * cells (Sverdrup, Almgren & Nikiforakis, "An embedded boundary approach for efficient
 * simulations of viscoplastic fluids in three dimensions").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers marked (device) are HIP device pointers; (host) are host pointers.
 *  - Cell fields are [nz][ny][nx] C-contiguous (x fastest), index c = i + nx*(j + ny*k).
 *    Vector fields are component-major [3][nz][ny][nx].  Face fields normal to x, y, z are
 *    [nz][ny][nx+1], [nz][ny+1][nx], [nz+1][ny][nx].  Per-cut-cell arrays follow the order of
 *    the cut list (ascending cell index).  All floating point data are IEEE binary64.
 *  - Ownership: the caller owns every buffer, including the device workspace handed to
 *    eb_geometry_build.  The library never allocates device memory.  The context (host
 *    memory, allocated by the library) refers into the workspace, so the workspace must stay
 *    alive until eb_ctx_destroy.  A context is not thread safe; calls on one context must be
 *    serialised by the caller.
 *  - Streams: `stream` is a hipStream_t passed as void*; NULL is the default stream.  Work is
 *    ordered on it: the library runs it on a stream of its own that waits for the caller's
 *    earlier work, and the caller's stream waits for the library's work before anything
 *    enqueued later.  Entry points that return host values (iteration counts, norms, forces)
 *    wait for the library's work before returning; the solvers poll one convergence word per
 *    iteration, one iteration behind the device.
 *  - Errors: every entry point returns 0 (EB_OK) or a negative code; eb_last_error() gives a
 *    thread-local message.  No exception crosses the ABI.  On EB_ENOCONV outputs hold the last
 *    iterate.
 *  - Covered cells (volume fraction 0) take u = u_EB, p = 0, eta = mu on output.
 */
#ifndef EB_H
#define EB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    EB_OK = 0,
    EB_EINVAL = -1,   /* null pointer, bad size, odd cell count, non-positive h */
    EB_EGEOM = -2,    /* ambiguous cut face, degenerate cut cell, wall stencil leaves the box */
    EB_ENOCONV = -3,  /* a linear solve hit max_iter */
    EB_ENAN = -4,     /* non-finite residual */
    EB_EHIP = -5,     /* HIP runtime error (message carries hipGetErrorString) */
    EB_ENOMEM = -6    /* workspace smaller than eb_workspace_bytes() */
};

/* Bodies (the fluid is where the level set is > 0).  CYLINDER: an infinitely long circular
 * cylinder of radius radii[0] whose axis runs along y through `center` (the body of Sec. V.C,
 * "Cylinder moving through Bingham fluid").  CAVITY: the fluid fills a sphere of radius
 * radii[0] about `center` and the body is everything outside it (a concave wall: its wall-flux
 * stencils reach across the cavity and take the covered-node fallback at coarse resolution). */
enum { EB_BODY_NONE = 0, EB_BODY_SPHERE = 1, EB_BODY_ELLIPSOID = 2, EB_BODY_ZSLAB = 3,
       EB_BODY_PLANE = 4, EB_BODY_CYLINDER = 5, EB_BODY_CAVITY = 6 };

/* Apparent-viscosity laws (Sec. II.B, Table rheology; Eq. papabing:viscosity), with
 * g = |gamma| the strain-rate norm and P(g) = kappa s^(n-1) the power-law term, where s = g, or
 * s = max(g, eps) when n < 1 (the term is unbounded at g = 0 there; for n >= 1, s = g):
 *   NEWTONIAN          eta = mu
 *   BINGHAM_REG        eta = mu + tau0/(g + eps)
 *   PAPANASTASIOU      eta = mu + tau0 (1 - exp(-g/eps))/g            (mu + tau0/eps at g = 0)
 *   POWER              eta = P(g)                                     (Ostwald-de Waele)
 *   HERSCHEL_BULKLEY   eta = P(g) + tau0 (1 - exp(-g/eps))/g          (P(0) + tau0/eps at 0)
 *   SOUZA_MENDES_DUTRA eta = P(g) + tau0 (1 - exp(-eta0 g/tau0))/g    (P(0) + eta0 at 0)
 * A zero yield stress leaves mu (the first three laws) or P(g) (the last two).  mu, eps, rho
 * > 0 where used; kappa > 0, n > 0 for the power-law laws; eta0 > 0 for Souza Mendes-Dutra.
 * Covered cells hold eta = mu under every law.  The time-step rule (eb_stable_dt) is stated
 * for the first three laws only. */
enum { EB_LAW_NEWTONIAN = 0, EB_LAW_BINGHAM_REG = 1, EB_LAW_PAPANASTASIOU = 2,
       EB_LAW_POWER = 3, EB_LAW_HERSCHEL_BULKLEY = 4, EB_LAW_SOUZA_MENDES_DUTRA = 5 };

/* Precision of the multigrid preconditioner.  EB_MIXED smooths, restricts and prolongates in
 * FP32 on the levels of at least 64^3 cells (those whose sweeps are bound by memory traffic;
 * smaller levels cost their launch latency whatever the precision and stay FP64); the Krylov
 * iteration, its residual with the full EB operator, the coarse levels with the coarsest solve,
 * the wall stencils and the divergence checks stay FP64, so the result meets the same FP64
 * residual target.  A mixed solve whose
 * residual has not fallen tenfold within 6 iterations, or that has not converged within
 * max(20, max_iter/10), has an operator too ill-conditioned for an FP32 V-cycle (e.g. a
 * viscosity contrast of 1e6 between a plug and a sheared layer); it is then solved again from
 * the same starting iterate with the FP64 V-cycle, giving the FP64 solve's result
 * (eb_step_stats.fp64_fallbacks counts these). */
enum { EB_FP64 = 0, EB_MIXED = 1 };
enum { EB_SYS_POISSON = 0, EB_SYS_VISC = 1 };  /* system for eb_mg_vcycle */

typedef struct {
    int n[3];             /* cells per direction; each a multiple of 2, fewer than 2^31 cells */
    double h;             /* cell size (> 0) */
    double lo[3];         /* lower domain corner */
    int periodic[3];      /* 1 = periodic in that direction */
    double wall_u[6][3];  /* Dirichlet velocity of the faces -x,+x,-y,+y,-z,+z */
} eb_box;

typedef struct {
    int kind;             /* EB_BODY_* */
    double center[3];
    double radii[3];      /* sphere: radii[0]; ellipsoid: semi-axes */
    double euler_zyx[3];  /* ellipsoid orientation R = Rz(a) Ry(b) Rx(c) */
    double zlo, zhi;      /* z-slab: fluid where zlo < z < zhi */
    double plane_n[3];    /* plane: fluid where plane_n . x > plane_d */
    double plane_d;
    double u_eb[3];       /* velocity of the embedded wall (no slip) */
} eb_body;

typedef struct {
    int law;              /* EB_LAW_* */
    double mu, tau0, eps, rho;
    double kappa, n;      /* consistency and flow index of the power-law term */
    double eta0;          /* Souza Mendes-Dutra: the viscosity at zero strain rate */
} eb_rheology;

typedef struct {
    int precision;        /* EB_FP64 or EB_MIXED */
    double rtol_visc, rtol_mac, rtol_proj;  /* max-norm relative residual targets */
    int max_iter;         /* per solve (<= 0: the default 400) */
    int nu1, nu2;         /* pre/post red-black Gauss-Seidel pairs per level (0: none on
                             that leg; negative: the default 2) */
    int nbottom;          /* sweep pairs on the coarsest level (<= 0: the default 16) */
    double force[3];      /* body force per unit volume (host values) */
    int projection;       /* end-of-stage projection: EB_PROJ_CELL (default; cell-centred
                             pressure [N]) or EB_PROJ_NODAL (Sec. III.A.4: the pressure on the
                             nodes [nz+1][ny+1][nx+1]; no adjoint) */
} eb_step_opts;

enum { EB_PROJ_CELL = 0, EB_PROJ_NODAL = 1 };

typedef struct {
    int it_mac[2], it_visc[2], it_proj[2];  /* Krylov iterations, predictor / corrector */
    double div_proj[2];                     /* max |div| of the projected face field */
    int vcycles;                            /* V-cycles executed in the step */
    int status;                             /* worst return code of the step's solves */
    int fp64_fallbacks;                     /* mixed precision: solves of the step that
                                               gave up the FP32 V-cycle and were solved again
                                               with the FP64 one (iteration counts include
                                               both attempts) */
    double dt_stable;                       /* eb_stable_dt of the step's input state with
                                               C_CFL = 0.5 and the step's force (forward
                                               steps; 0 in the adjoint and for the
                                               power-law laws): a dt above it is outside
                                               the paper's stability rule */
} eb_step_stats;

typedef struct eb_ctx eb_ctx;

/* Device workspace (bytes) that eb_geometry_build needs for this box and body.  Host only. */
size_t eb_workspace_bytes(const eb_box* box, const eb_body* body);

/* Builds the cut-cell geometry on the device (Sec. III.B: planar cut per cell, continuous at
 * faces; flags, volume fractions, face apertures, EB normal into the fluid, EB area and
 * centroid, the wall-flux stencils of Eqs. interpolation_distances and dudn) and the
 * multigrid level hierarchy.  ws: (device) workspace of ws_bytes >= eb_workspace_bytes().
 * On success *ctx receives a new context.  Errors: EB_EINVAL, EB_ENOMEM, EB_EGEOM, EB_EHIP. */
int eb_geometry_build(const eb_box* box, const eb_body* body, void* ws, size_t ws_bytes,
                      eb_ctx** ctx, void* stream);

/* Releases the host context (not the caller's workspace). */
void eb_ctx_destroy(eb_ctx* ctx);

/* Solver iterations are captured once per configuration as HIP graphs and replayed (on by
 * default; the environment variable EB_GRAPHS=0 turns it off for new contexts).  enable = 0
 * launches every kernel individually instead; results are identical either way.  Host only. */
int eb_ctx_set_graphs(eb_ctx* ctx, int enable);

/* Branch record and replay of the step's non-smooth switches, for checking the reverse mode
 * against finite differences (the adjoint differentiates the step with every switch frozen
 * at its forward value).  The switches are those of the derived quantities (Sec. III.A.3,
 * Sec. III.B.2): the branch of each monotonised-central slope (per component, direction and
 * cell), the normal upwind side of each face velocity, and the upwind side of each face's
 * convective flux.  Every derived-quantities evaluation (two per RK2 step, one per
 * eb_derived) takes the next eb_switch_bytes(ctx) bytes of `buf` (device, caller-owned):
 *   EB_SWITCH_RECORD  evaluates the switches as usual and writes them there;
 *   EB_SWITCH_REPLAY  reads them from there instead of evaluating them, so a perturbed run
 *                     stays on the recorded pieces of smoothness;
 *   EB_SWITCH_OFF     (default) neither.
 * Setting a mode rewinds to the start of `buf`; an evaluation beyond `bytes` fails with
 * EB_EINVAL.  Comparing two records byte by byte counts the switches two runs took
 * differently.  Host only. */
enum { EB_SWITCH_OFF = 0, EB_SWITCH_RECORD = 1, EB_SWITCH_REPLAY = 2 };
size_t eb_switch_bytes(const eb_ctx* ctx);
int eb_ctx_set_switches(eb_ctx* ctx, int mode, void* buf, size_t bytes);

/* Number of cut cells, multigrid levels, and wall stencils that needed the covered-node
 * fallback.  Host only. */
int eb_ctx_info(const eb_ctx* ctx, int* ncut, int* nlevels, int* nfallback);

/* Copies the geometry into caller buffers (device): flag u8[N] (0 covered, 1 cut, 2 regular),
 * alpha[N], apertures ax, ay, az (face layouts above); cut_cell int64[ncut]; cut_data
 * [ncut][9] = (n_x, n_y, n_z, A_EB, b_x, b_y, b_z, delta, fallback planes).  Any pointer may
 * be NULL to skip it. */
int eb_geometry_export(const eb_ctx* ctx, uint8_t* flag, double* alpha, double* ax, double* ay,
                       double* az, int64_t* cut_cell, double* cut_data, void* stream);

/* Strain rate and apparent viscosity (Sec. III.B.4, Sec. II Eq. governing:stress):
 * cell gradients by central differences, or one-sided quadratic differences where a face
 * neighbour is covered; |gamma| = sqrt(tr(gamma gamma^T)/2) with gamma = grad u + grad u^T;
 * eta from the law with tau0_i = tau0*theta_i.  At cut cells eta_eb comes from the wall
 * gradient n (x) du/dn of Eq. dudn.  u (device) [3][N]; theta (device, nullable = 1) [N];
 * eta (device) [N]; eta_eb (device) [ncut]; sr (device, nullable) [N]. */
int eb_apparent_viscosity(const eb_ctx* ctx, const eb_rheology* rheo, const double* u,
                          const double* theta, double* eta, double* eta_eb, double* sr,
                          void* stream);

/* Viscous operators, (device) arrays:
 *  EB_OP_HELMHOLTZ   out = alpha rho u - dt [div(eta grad u)] with the EB wall flux of
 *                    Eq. dudn, rows multiplied by the volume fraction (Eq. implicit-viscous);
 *                    Dirichlet domain walls and u_EB enter as given.
 *  EB_OP_HELMHOLTZ_H the same with homogeneous boundary values (the linear part).
 *  EB_OP_TRANSPOSE   out = div(eta (grad u)^T) (Eq. explicit-viscous without 1/rho), hybrid
 *                    divergence with flux redistribution (Eqs. divergence_conservative ...
 *                    divergence_final); rho and dt are ignored. */
enum { EB_OP_HELMHOLTZ = 0, EB_OP_HELMHOLTZ_H = 1, EB_OP_TRANSPOSE = 2 };
int eb_viscous_apply(const eb_ctx* ctx, int mode, double rho, double dt, const double* eta,
                     const double* eta_eb, const double* u, double* out, void* stream);

/* One multigrid V-cycle e = V(r) of the preconditioner for `system`, from a zero guess:
 * red-black Gauss-Seidel (nu1 pre, nu2 post pairs), volume-fraction-weighted restriction
 * (mean of the children of the already alpha-weighted rows), piecewise-constant prolongation
 * to uncovered children, nbottom sweep pairs on the coarsest level.  Poisson: beta*div(A grad)
 * with apertures A (the projection operator).  Viscous: the 7-point part of the Helmholtz
 * operator with the EB flux replaced by a diagonal term.  r, e (device): [N] for Poisson,
 * [3][N] for the viscous system.  eta/eta_eb used only for the viscous system. */
int eb_mg_vcycle(eb_ctx* ctx, int system, int precision, double beta, double rho, double dt,
                 const double* eta, const double* eta_eb, const double* r, double* e,
                 const eb_step_opts* opts, void* stream);

/* One red-black Gauss-Seidel half sweep (cells with (i+j+k) mod 2 == colour) on the finest
 * multigrid level, with the operator built by the most recent eb_mg_vcycle or solve for
 * `system` at `precision` (EB_FP64: b, x are (device) double [ncomp][N]; EB_MIXED: float).
 * ncomp = 1 (Poisson) or 3 (viscous).  b and x are in the finest level's colour-split order:
 * per component, the cells of colour 0 in natural order, then those of colour 1, so cell
 * c = (i,j,k) sits at ((i+j+k) mod 2) * N/2 + c/2.  Regular cells recompute their coefficients
 * from the viscosity array the operator was built from, which must still be valid.  The
 * multigrid smoother in isolation, for timing and tests; EB_EINVAL if no operator of that kind
 * has been built, or for EB_MIXED if the finest level runs in FP64 (fewer than 64^3 cells). */
int eb_mg_sweep(eb_ctx* ctx, int system, int precision, int colour, const void* b, void* x,
                void* stream);

/* Implicit viscous solve (Eq. implicit-viscous): (alpha rho - dt div(eta grad)) x = alpha psi
 * with the EB wall flux, BiCGSTAB right-preconditioned by eb_mg_vcycle, stopped when
 * max|r| <= rtol max|b|.  psi (device) [3][N]; x (device) [3][N] in: guess, out: solution.
 * *iters (host, nullable).  Returns EB_ENOCONV after max_iter. */
int eb_visc_solve(eb_ctx* ctx, double rho, double dt, const double* eta, const double* eta_eb,
                  const double* psi, double* x, double rtol, const eb_step_opts* opts,
                  int* iters, void* stream);

/* Cell-centred (MAC) projection of a face field (Eq. helmholtz and the Poisson problem that
 * follows it): beta div(A grad phi) = div(A w), w -= beta grad phi on open faces.  fx, fy, fz
 * (device) face fields, in/out; phi (device) [N], in: guess, out: zero-mean solution.
 * *div_inf (host, nullable) = max |div(A w)| after the correction; *iters (host, nullable). */
int eb_mac_project(eb_ctx* ctx, double beta, double* fx, double* fy, double* fz, double* phi,
                   double rtol, const eb_step_opts* opts, double* div_inf, int* iters,
                   void* stream);

/* End-of-stage projection with a cell-centred pressure (Sec. III.A.4 approximated by the exact
 * projection of face-averaged velocities): u += beta G p; w = face average of u; project w;
 * u -= beta G p_new with G the aperture-weighted average of the two face gradients.
 * u (device) [3][N] in/out; p (device) [N] in: old pressure, out: new pressure. */
int eb_cc_project(eb_ctx* ctx, double beta, double* u, double* p, double rtol,
                  const eb_step_opts* opts, double* div_inf, int* iters, void* stream);

/* The nodal end-of-stage projection (Sec. III.A.4, Alg. advance NodalProjection): velocities on
 * cell centres, the pressure on the nodes, an approximate projection.  Trilinear finite elements
 * on each cell weighted by its volume fraction: u += beta G(pn); solve L phi = D(u) - B, where
 * D is the weak nodal divergence, B the flux of the wall and embedded-wall velocities and L the
 * elements' stiffness matrix (singular: phi is normalised to zero mean over the nodes of open
 * cells), by CG with the diagonal as preconditioner (at most max(max_iter, 10 max n_d)
 * iterations) to max|r| <= rtol max(max|D - B|, the largest sum of |terms| of D at a node);
 * u -= G(phi) on open cells, with G(q) the cell average of the gradient of q's trilinear
 * interpolant; pn = phi / beta.  u (device) [3][N] in/out; pn (device) [nz+1][ny+1][nx+1]
 * in: old, out: new (in a periodic direction the last node is a copy of the first).
 * *div_inf (host, nullable) = max |D(u) - B| left (not zero: the projection is approximate). */
int eb_nodal_project(eb_ctx* ctx, double beta, double* u, double* pn, double rtol,
                     const eb_step_opts* opts, double* div_inf, int* iters, void* stream);

/* eb_drag with a nodal pressure pn (device) [nz+1][ny+1][nx+1] (a step with EB_PROJ_NODAL):
 * the wall pressure p_EB is the trilinear interpolation of pn at the EB centroid. */
int eb_drag_nodal(const eb_ctx* ctx, const eb_rheology* rheo, const double* theta,
                  const double* u, const double* pn, double F[3], void* stream);

/* DerivedQuantities (Alg. derived): limited slopes, face extrapolation and upwinding, the
 * MAC projection, convective term C = -div(u (x) u^F), eta and eta_eb, and the explicit term
 * V = div(eta (grad u)^T), both divergences hybridised and redistributed.  (device) arrays:
 * u [3][N] in; C [3][N], eta [N], eta_eb [ncut], V [3][N] out. */
int eb_derived(eb_ctx* ctx, const eb_rheology* rheo, const double* theta, const double* u,
               const eb_step_opts* opts, double* C, double* eta, double* eta_eb, double* V,
               int* iters, void* stream);

/* One RK2 step (Alg. advance): predictor and corrector, each DerivedQuantities, the
 * semi-implicit viscous solve and the end-of-stage projection; the corrector averages C, eta,
 * eta_eb and V.  u (device) [3][N] and p (device) [N] in/out.  stats (host, nullable). */
int eb_rk2_step(eb_ctx* ctx, const eb_rheology* rheo, const double* theta, double dt,
                const eb_step_opts* opts, double* u, double* p, eb_step_stats* stats,
                void* stream);

/* Force on the embedded body (Eq. drag-force): sum over cut cells of
 * A_EB h^2 [tau_EB n - p_EB n], tau_EB = eta_EB (n (x) g + g (x) n), g = du/dn from Eq. dudn,
 * p_EB = p + h b.G p.  n points from the body into the fluid.  F (host) [3]. */
int eb_drag(const eb_ctx* ctx, const eb_rheology* rheo, const double* theta, const double* u,
            const double* p, double F[3], void* stream);

/* eb_drag for callers that cannot allocate device memory or touch the context's workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation): the
 * same force, bit for bit, with its scratch (wall gradients and drag terms of the cut cells,
 * reduction partials) in a file-scope device array of 3.2 MB that each GPU the library runs on
 * holds until the process ends.  Calls no hipMalloc or hipFree and writes nothing into ctx's
 * workspace; enqueues on `stream` itself and waits for it to return F (host).  Limit: at most
 * 65536 cut cells (EB_EINVAL beyond).  Every call on one GPU shares that GPU's array, so calls
 * that overlap on one GPU (from several threads or streams) race; nothing in it needs to start
 * at zero (each call writes every entry it reads). */
int eb_drag_noalloc(const eb_ctx* ctx, const eb_rheology* rheo, const double* theta,
                    const double* u, const double* p, double F[3], void* stream);

/* Time step of the paper's stability rule (Sec. II.C.1) for the state u (device) [3][N]:
 * Eq. cfl:dt combining the convective coefficient max over open cells of (|u|+|v|+|w|)/h
 * (Eq. cfl:convective), the forcing coefficient sqrt(sum_d |force_d| / h) (Eq. cfl:forcing;
 * force on the host) and the viscous one 2 mu (Bi + 1) / rho * 3 / h^2 (Eq. cfl:viscous:new),
 * with Bi the largest tau0 * theta over open cells (theta nullable = 1; 0 for a Newtonian
 * law) and c_cfl in (0, 1] (the paper's default 0.5).  Writes *dt (host); synchronises
 * `stream`.  The step does not limit its dt by this; it reports it (eb_step_stats).  The rule
 * is stated for the Newtonian and Bingham laws: the power-law laws return EB_EINVAL. */
int eb_stable_dt(const eb_ctx* ctx, const eb_rheology* rheo, const double* theta,
                 const double* u, const double force[3], double c_cfl, double* dt,
                 void* stream);

/* Cell-centred pressure gradient G p (aperture-weighted mean of the two face gradients in
 * each direction; domain-wall faces carry a zero gradient).  p (device) [N], gp (device) [3][N]. */
int eb_pressure_gradient(const eb_ctx* ctx, const double* p, double* gp, void* stream);

/* ---------------------------------------------------------------------------------------
 * Reverse mode.  The adjoint of the step is the exact transpose of the step linearised about
 * its forward state: every solve is transposed rather than differentiated through its
 * iterations (the Poisson systems are symmetric, the viscous system is solved with A^T and the
 * same V-cycle), and every switch is frozen at its forward value (upwind side, slope-limiter
 * branch, one-sided gradient stencil, wall-stencil plane).  Adjoint arrays (suffix b) hold
 * d(loss)/d(quantity); unless stated otherwise they are (device) arrays in the layouts above
 * and the entry point adds into them.  Adjoints of covered cells are zero on output.  The
 * yield-stress adjoint tau0b[c] is d(loss)/d(tau0_c) with tau0_c = rheo->tau0 * theta[c]; the
 * Bingham-number derivative follows as sum_c theta[c] tau0b[c].
 * --------------------------------------------------------------------------------------- */

/* Bytes of the (device) tape one step records for its reverse sweep: the projected face
 * velocities and the viscosities of both stages and the velocities after each solve and
 * projection.  Host only. */
size_t eb_tape_bytes(const eb_ctx* ctx);

/* eb_rk2_step that also fills `tape` (device, eb_tape_bytes, caller-owned) for
 * eb_rk2_step_adjoint.  Same arguments, results and errors as eb_rk2_step. */
int eb_rk2_step_taped(eb_ctx* ctx, const eb_rheology* rheo, const double* theta, double dt,
                      const eb_step_opts* opts, double* u, double* p, void* tape,
                      eb_step_stats* stats, void* stream);

/* Adjoint of one RK2 step (Alg. advance).  u0 (device) [3][N]: the step's input velocity;
 * tape: recorded by eb_rk2_step_taped from u0 with the same rheo, theta, dt and opts.
 * ub [3][N], pb [N]: in, the adjoints of the step's output (u, p); out, those of its input
 * (overwritten).  The step's yield-stress adjoint, with tau0_c = rheo->tau0 * theta_c
 * (theta null = 1), is added into whichever of these is not null:
 *   tau0b   (device) [N]  d(loss)/d(tau0_c) per cell;
 *   thetab  (device) [N]  d(loss)/d(theta_c) = tau0 * tau0b_c;
 *   tau0bar (host) [1]    d(loss)/d(tau0) = sum_c theta_c tau0b_c, a fixed-order reduction
 *                         (the Bingham-number derivative when mu, U and L are 1); the call
 *                         then waits for its work.
 * stats (host, nullable): iterations of the six transposed solves (it_mac: adjoint MAC
 * projections, it_visc: transposed viscous solves, it_proj: adjoint end-of-stage projections).
 * Errors as eb_rk2_step. */
int eb_rk2_step_adjoint(eb_ctx* ctx, const eb_rheology* rheo, const double* theta, double dt,
                        const eb_step_opts* opts, const double* u0, const void* tape,
                        double* ub, double* pb, double* tau0b, double* thetab,
                        double* tau0bar, eb_step_stats* stats, void* stream);

/* Adjoint of eb_drag (Eq. drag-force) at (u, p): fbar (host) [3] = d(loss)/dF; ub [3][N] and
 * pb [N] accumulate (pb is set to zero on covered cells); the yield-stress adjoint goes to
 * tau0b, thetab and tau0bar (each nullable, accumulated) as in eb_rk2_step_adjoint. */
int eb_drag_adjoint(const eb_ctx* ctx, const eb_rheology* rheo, const double* theta,
                    const double* u, const double fbar[3], double* ub, double* pb,
                    double* tau0b, double* thetab, double* tau0bar, void* stream);

/* Adjoint of eb_mac_project on its face field: fbx, fby, fbz (device) in, the adjoint of the
 * projected field; out, that of the input field.  One Poisson solve to rtol. */
int eb_mac_project_adjoint(eb_ctx* ctx, double beta, double* fbx, double* fby, double* fbz,
                           double rtol, const eb_step_opts* opts, int* iters, void* stream);

/* Adjoint of eb_cc_project: ub [3][N], pb [N] in, the adjoints of (u, p) after the
 * projection; out, those of (u, p) before it (overwritten). */
int eb_cc_project_adjoint(eb_ctx* ctx, double beta, double* ub, double* pb, double rtol,
                          const eb_step_opts* opts, int* iters, void* stream);

/* Adjoint of eb_visc_solve at its solution x (device) [3][N] with adjoint xb [3][N]:
 * solves A^T lam = xb (BiCGSTAB, same V-cycle preconditioner); psib [3][N] is written
 * (= alpha lam); etab [N] and etaebb [ncut] accumulate the viscosity adjoints. */
int eb_visc_solve_adjoint(eb_ctx* ctx, double rho, double dt, const double* eta,
                          const double* eta_eb, const double* x, const double* xb, double rtol,
                          const eb_step_opts* opts, double* psib, double* etab, double* etaebb,
                          int* iters, void* stream);

/* Adjoint of eb_derived at u: Cb, Vb [3][N], etab [N], etaebb [ncut] are the adjoints of its
 * outputs; ub [3][N] and tau0b [N] accumulate.  The face velocities are recomputed (one
 * forward MAC projection) before the adjoint one. */
int eb_derived_adjoint(eb_ctx* ctx, const eb_rheology* rheo, const double* theta, const double* u,
                       const double* Cb, const double* etab, const double* etaebb,
                       const double* Vb, double* ub, double* tau0b, const eb_step_opts* opts,
                       int* iters, void* stream);

const char* eb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EB_H */
