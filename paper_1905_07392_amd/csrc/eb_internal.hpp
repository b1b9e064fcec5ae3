// eb_internal.hpp -- shared device structures and launcher declarations of the EB RK2 library.
//
// Layout: cell c = i + nx*(j + ny*k); faces normal to d have n_d + 1 entries along d.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/eb.h"

#define EB_MAXLEV 16
#define EB_BLOCK 256

// Records the first failing HIP runtime call (copy, event, stream or graph call) since the entry
// point's last error check; that check reports it as EB_EHIP with the call's text, and the
// solver loops stop polling once one has failed.
void hip_note(hipError_t e, const char* what);
bool hip_failed();
#define HIPN(call) hip_note((call), #call)

// ------------------------------------------------------------------------------------------
// views passed by value to kernels
// ------------------------------------------------------------------------------------------
struct GridV {
    int n[3];
    int per[3];
    double h;
};

struct BodyV {
    int kind;
    double lo[3];    // domain origin (node (0,0,0))
    double c[3];
    double r[3];
    double R[3][3];  // world <- body rotation (ellipsoid)
    double zlo, zhi;
    double pn[3];
    double pd;
};

// Fine-level geometry (read-only after the build)
struct GeomV {
    GridV grid;
    long N;
    int ncut;
    double wall[6][3];
    double ueb[3];
    const uint8_t* flag;
    const double* alpha;
    const double* ap[3];
    const int* cutid;   // per cell, -1 if not cut
    const int* cut;     // per cut: cell
    const double* nrm;  // [3][ncut] (component-major)
    const double* aeb;
    const double* bc;   // [3][ncut]
    const double* delta;
    const double* dd;   // [2][ncut]
    const int* sidx;    // [18][ncut]
    const double* sw;   // [18][ncut]
    const uint8_t* near;  // per cell: 1 if it or one of its 26 neighbours is a cut cell
};

template <typename T>
struct LevelV {
    GridV grid;
    long N;
    const T* K[3];
    const T* D;
    const uint8_t* mask;
    const int* gate;  // nullable: kernels return at once while *gate != 0
};

// ------------------------------------------------------------------------------------------
// small device helpers
// ------------------------------------------------------------------------------------------
__host__ __device__ inline long cell_index(const GridV& g, int i, int j, int k) {
    return (long)i + (long)g.n[0] * ((long)j + (long)g.n[1] * (long)k);
}
__host__ __device__ inline long face_index(const GridV& g, int d, int i, int j, int k) {
    long m0 = g.n[0] + (d == 0), m1 = g.n[1] + (d == 1);
    return (long)i + m0 * ((long)j + m1 * (long)k);
}
__host__ __device__ inline long face_count(const GridV& g, int d) {
    return (long)(g.n[0] + (d == 0)) * (g.n[1] + (d == 1)) * (g.n[2] + (d == 2));
}
// cell at integer coordinates (wrapping periodic directions); -1 outside a wall
__host__ __device__ inline long cell_at(const GridV& g, int i, int j, int k) {
    int q[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; d++) {
        if (q[d] < 0 || q[d] >= g.n[d]) {
            if (!g.per[d]) return -1;
            q[d] = q[d] < 0 ? q[d] + g.n[d] : q[d] - g.n[d];
        }
    }
    return cell_index(g, q[0], q[1], q[2]);
}
// natural index of the neighbour across face 2d + side of cell c = (i, j, k): cell_at of the
// neighbour's coordinates (-1 across a wall, wrapped in a periodic direction), with only the
// coordinate that moved tested and the index stepped from c by that direction's stride
__host__ __device__ inline long cell_step(const GridV& g, long c, int i, int j, int k, int d,
                                          int side) {
    int q = d == 0 ? i : (d == 1 ? j : k);
    long st = d == 0 ? 1L : (d == 1 ? (long)g.n[0] : (long)g.n[0] * g.n[1]);
    int e = q + (side ? 1 : -1);
    long in = side ? c + st : c - st;
    long wr = side ? in - (long)g.n[d] * st : in + (long)g.n[d] * st;
    bool inside = e >= 0 && e < g.n[d];
    return inside ? in : (g.per[d] ? wr : -1L);
}
// 32-bit unsigned division: boxes hold fewer than 2^32 cells, and 64-bit division is many
// times slower on the GPU
__host__ __device__ inline void cell_coords(const GridV& g, long c, int& i, int& j, int& k) {
    unsigned cu = (unsigned)c, nx = (unsigned)g.n[0], ny = (unsigned)g.n[1];
    unsigned t = cu / nx;
    i = (int)(cu - t * nx);
    unsigned k2 = t / ny;
    j = (int)(t - k2 * ny);
    k = (int)k2;
}

// coarse face f of direction d: scale x the sum of the four fine faces it covers (o = 0..3)
__device__ inline double coarsen_face_value(const GridV& gc, const GridV& gf, int d,
                                            const double* ff, long f, double scale) {
    int m0 = gc.n[0] + (d == 0), m1 = gc.n[1] + (d == 1);
    int q[3];
    q[0] = (int)(f % m0);
    long r = f / m0;
    q[1] = (int)(r % m1);
    q[2] = (int)(r / m1);
    int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    double s = 0.0;
    for (int o = 0; o < 4; o++) {
        int p[3];
        p[d] = 2 * q[d];
        p[t1] = 2 * q[t1] + (o & 1);
        p[t2] = 2 * q[t2] + (o >> 1);
        s += ff[face_index(gf, d, p[0], p[1], p[2])];
    }
    return s * scale;
}
// Viscous coarse face f of direction d: scale x the sum over the four fine faces f2 it covers of
// each one's line contribution.  The line of fine faces normal to the coarse face through the two
// coarse cells it separates (f1 inside the lower coarse cell, f2, f3 inside the upper) joins the
// two coarse centres, so its viscosity acts in series: the weighted harmonic mean
// H = W / sum(w_i / g_i) of g_i = K_i / A_i over the open faces of the line (weights 1/2, 1, 1/2;
// a domain-wall f2 has weight 1/2, no outer face, and g_2 = K_2 / (2 A_2), its ghost factor
// removed); the line contributes K_2 H / g_2.  A uniform viscosity gives the plain sum of K_2.
__device__ inline double coarsen_face_series(const GridV& gc, const GridV& gf, int d,
                                             const double* Kf, const double* apf, long f,
                                             double scale) {
    int m0 = gc.n[0] + (d == 0), m1 = gc.n[1] + (d == 1);
    int q[3];
    q[0] = (int)(f % m0);
    long r = f / m0;
    q[1] = (int)(r % m1);
    q[2] = (int)(r / m1);
    int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    bool per = gf.per[d] != 0;
    bool wall = !per && (q[d] == 0 || q[d] == gc.n[d]);
    double s = 0.0;
    for (int o = 0; o < 4; o++) {
        int p[3];
        p[d] = 2 * q[d];
        p[t1] = 2 * q[t1] + (o & 1);
        p[t2] = 2 * q[t2] + (o >> 1);
        long f2 = face_index(gf, d, p[0], p[1], p[2]);
        double K2 = Kf[f2], A2 = apf[f2];
        if (K2 == 0.0 || A2 == 0.0) {
            s += K2;
            continue;
        }
        double g2 = wall ? K2 / (2.0 * A2) : K2 / A2;
        double W = wall ? 0.5 : 1.0, R = W / g2;
        for (int side = -1; side <= 1; side += 2) {
            int e[3] = {p[0], p[1], p[2]};
            e[d] += side;
            if (e[d] < 0 || e[d] > gf.n[d]) {
                if (!per) continue;
                e[d] = e[d] < 0 ? e[d] + gf.n[d] : e[d] - gf.n[d];
            }
            long fi = face_index(gf, d, e[0], e[1], e[2]);
            double K = Kf[fi], A = apf[fi];
            if (K > 0.0 && A > 0.0) {
                W += 0.5;
                R += 0.5 / (K / A);
            }
        }
        s += K2 * (W / R) / g2;
    }
    return s * scale;
}
// coarse cell c: the mean of its eight children (q = 0..7)
__device__ inline double coarsen_cell_value(const GridV& gc, const GridV& gf, const double* af,
                                            long c) {
    int i, j, k;
    cell_coords(gc, c, i, j, k);
    double s = 0.0;
    for (int q = 0; q < 8; q++)
        s += af[cell_index(gf, 2 * i + (q & 1), 2 * j + ((q >> 1) & 1), 2 * k + (q >> 2))];
    return s / 8.0;
}

// max that keeps a NaN (fmax returns the other operand): the max-norms of the stop tests must
// see a non-finite residual so the solve can report it
__host__ __device__ __forceinline__ double nan_max(double a, double b) {
    return (a > b || a != a) ? a : b;
}

// Work-group index remapped so that each of the 8 XCDs, which receive work-groups round-robin,
// processes one contiguous range of tiles: vertically neighbouring rows and planes of a stencil
// then share that XCD's L2 instead of being fetched again by another XCD.
__device__ __forceinline__ unsigned xcd_block() {
    unsigned nb = gridDim.x, b = blockIdx.x;
    unsigned q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}
// the same mapping over the first nb blocks of a larger grid (block b < nb)
__device__ __forceinline__ unsigned xcd_block_in(unsigned nb) {
    unsigned b = blockIdx.x;
    unsigned q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

inline unsigned grid_for(long n, int block = EB_BLOCK) {
    long b = (n + block - 1) / block;
    return (unsigned)(b > 0 ? b : 1);
}

// ------------------------------------------------------------------------------------------
// host-side level storage
// ------------------------------------------------------------------------------------------
constexpr size_t MG_PACK_BYTES = 65536;  // the tail kernel's LDS budget

struct Level {
    GridV grid;
    long N;
    double* alpha;
    uint8_t* mask;
    double* ap[3];
    double* K[3];
    double* S;
    double* D;
    float* Kf[3];
    float* Df;
    double *x, *b;  // 3 components each
    float *xf, *bf;
    // the one-work-group tail's operator arrays in its LDS layout (MG_PACK_BYTES, shared by all
    // levels; filled when an operator is built)
    char* pack = nullptr;
    const int* gate = nullptr;
    // finest level only: what its operator was built from, so the smoother can recompute the
    // coefficients of regular cells instead of reading them (flag: 0 covered, 1 cut, 2 regular)
    const uint8_t* flag = nullptr;
    const int* cut = nullptr;  // the cut cells (flag 1) in ascending order, ncut of them
    int ncut = 0;
    const double* eta = nullptr;
    float* etaf = nullptr;  // FP32 copy of eta for the mixed-precision smoother
    // colour-split copies of eta and the flags, made when an operator is built (the FP64
    // two-cells-per-thread smoother reads them in pairs, like the iterate)
    double* etacs = nullptr;
    float* etafcs = nullptr;  // (mixed builds)
    uint8_t* flagcs = nullptr;
    int sys = 0;  // EB_SYS_POISSON or EB_SYS_VISC
    double rho = 0.0, dt = 0.0, beta = 0.0;
    LevelV<double> v64() const {
        LevelV<double> v;
        v.grid = grid;
        v.N = N;
        for (int d = 0; d < 3; d++) v.K[d] = K[d];
        v.D = D;
        v.mask = mask;
        v.gate = gate;
        return v;
    }
    LevelV<float> v32() const {
        LevelV<float> v;
        v.grid = grid;
        v.N = N;
        for (int d = 0; d < 3; d++) v.K[d] = Kf[d];
        v.D = Df;
        v.mask = mask;
        v.gate = gate;
        return v;
    }
};

// ------------------------------------------------------------------------------------------
// launchers (each .hip file owns its kernels)
// ------------------------------------------------------------------------------------------
// geometry
int geom_build_device(const GridV& grid, const BodyV& body, double* psi_nodes, uint8_t* flag,
                      double* alpha, double* ap[3], int* cutid, int* cut, int* blockcount,
                      int ncut_max, int* ncut_out, int* err_dev, hipStream_t s);
void geom_cut_fill(const GridV& grid, const BodyV& body, const double* psi, const double* ap[3],
                   const int* cut, int ncut, int* cutid, double* nrm, double* aeb, double* bc,
                   double* delta, hipStream_t s);
void geom_wall_stencil(const GeomV& g, double* dd, int* sidx, double* sw, int* nfb,
                       int* err_dev, hipStream_t s);
void level_coarsen_geometry(const Level& F, Level& C, hipStream_t s);
void level_mask(Level& L, hipStream_t s);
// near[c] = 1 for every cut cell and each of its 26 neighbours, 0 elsewhere
void geom_mark_near(const GridV& g, const int* cut, int ncut, uint8_t* near, hipStream_t s);

// pointwise and stencil operators
void op_wall_grad(const GeomV& g, const double* u, double* gw, hipStream_t s);
void op_grad_eta(const GeomV& g, const eb_rheology& r, const double* u, const double* gw,
                 const double* theta, double* G9, double* eta, double* sr, hipStream_t s);
void op_eta_eb(const GeomV& g, const eb_rheology& r, const double* gw, const double* theta,
               double* eta_eb, hipStream_t s);
void op_transpose_dc(const GeomV& g, const double* u, const double* G9, const double* eta,
                     const double* eta_eb, const double* gw, double* DC, hipStream_t s);
// Branch record of the derived quantities' switches (the limited slope's branch, the normal
// upwind side, the transverse upwind side): mode 0 computes them, 1 computes and records them,
// 2 evaluates the recorded ones (the step frozen on its pieces of smoothness).
struct SwitchV {
    int mode;
    uint8_t* slope;    // [component][direction][N]: 0 zero, 1 central, 2 twice left, 3 twice right
    uint8_t* norm[3];  // per face of each direction: 0 zero, 1 left state, 2 right state
    uint8_t* tr[3];    // per face: 1 left state, 2 right state, 3 their mean
};
void op_face_extrap(const GeomV& g, const double* u, double* f[3], const SwitchV& sw,
                    hipStream_t s);
void op_divergence(const GeomV& g, double* const f[3], double* div, hipStream_t s);
void op_conv_dc(const GeomV& g, const double* u, double* const f[3], double* DC,
                const SwitchV& sw, hipStream_t s);
void op_redistribute(const GeomV& g, const double* DC, double* DH, double* S, double* dD,
                     double* D, hipStream_t s);
void op_gcc(const GeomV& g, const double* p, double* gp, hipStream_t s);
void op_axpy_open(const GeomV& g, double a, const double* x, double* y, int ncomp,
                  hipStream_t s);
void op_cell_to_face(const GeomV& g, const double* u, double* f[3], hipStream_t s);
void op_face_correct(const GeomV& g, double beta, const double* p, double* f[3], hipStream_t s);
void op_psi(const GeomV& g, double rho, double dt, const double* u, const double* C,
            const double* V, const double* gp, const double f[3], double* psi, hipStream_t s);
void op_average(long n, const double* a, double* b, hipStream_t s);  // b = (a+b)/2
void op_finalize_state(const GeomV& g, double* u, double* p, hipStream_t s);
void op_drag_terms(const GeomV& g, const eb_rheology& r, const double* theta, const double* gw,
                   const double* p, const double* gp, double* terms, hipStream_t s,
                   const double* peb = nullptr);
void op_poisson_rhs(const GeomV& g, const double* div, const double* sumcnt, double* b,
                    hipStream_t s);
void op_shift_open(const GeomV& g, double* x, const double* sumcnt, hipStream_t s,
                   const int* gate = nullptr);

// device-resident Krylov scalars (slots of a double array) and scalar updates
// the stall test's window (iterations) for a solve preconditioned by the FP32 V-cycle
constexpr int KS_STALL_W = 6;
enum {
    KS_RTOL, KS_BN, KS_SCALE, KS_TOL, KS_RN, KS_SN, KS_RHO_OLD, KS_AL, KS_OM, KS_BE, KS_RZ,
    KS_RZN, KS_PQ, KS_RR, KS_RV, KS_TS, KS_TT, KS_SUM, KS_CNT, KS_RRN, KS_WATCH, KS_BEST_OLD,
    KS_RING, KS_COUNT = 32
};
static_assert(KS_RING + KS_STALL_W <= KS_COUNT, "Krylov scalar slots");
enum {
    KS_INIT, KS_CG_ALPHA, KS_CHECK_R, KS_CG_BETA, KS_BI_ALPHA, KS_BI_CHECK_S, KS_BI_OMEGA,
    KS_BI_CHECK_R, KS_INIT_WATCH
};
// The stall test of a watched solve (one preconditioned by the FP32 V-cycle), after the
// residual max-norm rn of iteration it is known and has not met the tolerance: rn enters a ring
// of the last KS_STALL_W values; from iteration KS_STALL_W + 1 on, the least of those must be
// at most a tenth of the least before them (KS_BEST_OLD), else the state becomes 4 (stalled).
// A working V-cycle gains a factor of ten in two or three iterations.
__device__ inline void ks_stall_test(double* __restrict__ ks, int* __restrict__ st, int it) {
    double* ring = ks + KS_RING;
    int j = it % KS_STALL_W;
    if (it > KS_STALL_W && ring[j] < ks[KS_BEST_OLD]) ks[KS_BEST_OLD] = ring[j];
    ring[j] = ks[KS_RN];
    if (it > KS_STALL_W) {
        double best_new = INFINITY;
        for (int q = 0; q < KS_STALL_W; q++) best_new = ring[q] < best_new ? ring[q] : best_new;
        if (!(best_new <= 0.1 * ks[KS_BEST_OLD])) *st = 4;
    }
}
// One Krylov scalar update, run by a single thread: op on the scalars ks of the solve whose
// state word and count are st[0], st[1] and whose device iteration counter is *itc.  The state
// is 0 while the solve runs, 1 when it converged at BiCGSTAB's half step (x update pending), 2
// converged, 3 non-finite residual, 4 stalled (a watched solve, KS_INIT_WATCH); once it leaves 0
// the ops do nothing more.
__device__ inline void ks_scalar_op(int op, double* __restrict__ ks, int* __restrict__ st,
                                    int* __restrict__ itc) {
    int s = *st;
    // the first scalar op of each iteration advances the count while the solve runs
    if (s == 0 && (op == KS_CG_ALPHA || op == KS_BI_ALPHA)) *itc += 1;
    int it = *itc;
    switch (op) {
    case KS_INIT:  // tol = rtol * max(bn, scale); converged already if rn <= tol
    case KS_INIT_WATCH: {
        double bn = ks[KS_BN] > ks[KS_SCALE] ? ks[KS_BN] : ks[KS_SCALE];
        ks[KS_TOL] = ks[KS_RTOL] * bn;
        st[1] = 0;
        *itc = 0;
        if (!isfinite(ks[KS_RN])) *st = 3;
        else if (bn == 0.0 || ks[KS_RN] <= ks[KS_TOL]) *st = 2;
        else *st = 0;
        ks[KS_RHO_OLD] = 1.0;
        ks[KS_AL] = 1.0;
        ks[KS_OM] = 1.0;
        ks[KS_WATCH] = op == KS_INIT_WATCH ? 1.0 : 0.0;
        ks[KS_BEST_OLD] = INFINITY;
        break;
    }
    case KS_CG_ALPHA:
        if (s == 0) ks[KS_AL] = ks[KS_RZ] / ks[KS_PQ];
        break;
    case KS_CHECK_R:  // after the x, r update (CG)
        if (s == 0) {
            if (!isfinite(ks[KS_RN])) *st = 3;
            else if (ks[KS_RN] <= ks[KS_TOL]) {
                *st = 2;
                st[1] = it;
            } else if (ks[KS_WATCH] != 0.0) {
                ks_stall_test(ks, st, it);
            }
        }
        break;
    case KS_CG_BETA:
        if (s == 0) {
            ks[KS_BE] = ks[KS_RZN] / ks[KS_RZ];
            ks[KS_RZ] = ks[KS_RZN];
        }
        break;
    case KS_BI_ALPHA:
        if (s == 0) ks[KS_AL] = ks[KS_RR] / ks[KS_RV];
        break;
    case KS_BI_CHECK_S:  // the count is in half iterations (= preconditioner applications)
        if (s == 0) {
            if (!isfinite(ks[KS_SN])) *st = 3;
            else if (ks[KS_SN] <= ks[KS_TOL]) {
                *st = 1;
                st[1] = 2 * it - 1;
            }
        }
        break;
    case KS_BI_CHECK_R:
        if (s == 0) {
            ks[KS_RHO_OLD] = ks[KS_RR];
            ks[KS_RR] = ks[KS_RRN];
            if (!isfinite(ks[KS_RN])) *st = 3;
            else if (ks[KS_RN] <= ks[KS_TOL]) {
                *st = 2;
                st[1] = 2 * it;
            } else if (ks[KS_WATCH] != 0.0) {
                ks_stall_test(ks, st, it);
            }
        }
        break;
    case KS_BI_OMEGA:  // also completes a convergence at the half step, whose x update is done
        if (s == 0) ks[KS_OM] = ks[KS_TS] / ks[KS_TT];
        else if (s == 1) *st = 2;
        break;
    default:
        break;
    }
}

// st: the solve's (state, count) pair; itc: its device iteration counter
void ks_op(int op, double* ks, int* st, int* itc, hipStream_t s);
void ks_set(double* ks, int idx, double v, hipStream_t s);
void ks_cg_p(long n, double* p, const double* z, const double* ks, const int* st, hipStream_t s);
void ks_bi_p(long n, double* p, const double* r, const double* v, const double* ks,
             const int* st, hipStream_t s);
void ks_bi_xs(long n, double* x, const double* ph, const double* ks, const int* st,
              hipStream_t s);
void ks_bi_xs(long n, double* x, const float* ph, const double* ks, const int* st,
              hipStream_t s);

// multigrid and Krylov
void mg_build_poisson(Level* lev, int nlev, const GeomV& g, double beta, bool mixed,
                      hipStream_t s);
void mg_build_visc(Level* lev, int nlev, const GeomV& g, double rho, double dt,
                   const double* eta, const double* eta_eb, bool mixed, hipStream_t s);
void mg_vcycle(Level* lev, int nlev, int ncomp, bool mixed, const double* b, double* x,
               int nu1, int nu2, int nbottom, hipStream_t s, const int* gate = nullptr);
// whether a V-cycle can hand its result over in FP32 without rounding (its finest level runs in
// FP32 in colour-split storage), and that V-cycle with an FP32 result
bool mg_vcycle_f32_out(Level* lev, int nlev, int ncomp, bool mixed, int nu1, int nu2);
void mg_vcycle(Level* lev, int nlev, int ncomp, bool mixed, const double* b, float* x, int nu1,
               int nu2, int nbottom, hipStream_t s, const int* gate = nullptr);
void mg_apply_level0(const Level& L, int ncomp, const double* x, double* y, hipStream_t s,
                     const int* gate = nullptr);
// whether a mixed-precision hierarchy runs its finest level in FP32 (levels of at least 64^3
// cells above the one-work-group tail do)
bool mg_level0_f32(const Level* lev, int nlev);
void mg_sweep_level0(const Level& L, int ncomp, bool f32, const void* b, void* x, int colour,
                     hipStream_t s);
void op_visc_apply(const GeomV& g, double rho, double dt, const double* eta,
                   const double* eta_eb, const double* u, double* out, int homogeneous,
                   hipStream_t s, const int* gate = nullptr);
void op_visc_apply(const GeomV& g, double rho, double dt, const double* eta,
                   const double* eta_eb, const float* u, double* out, int homogeneous,
                   hipStream_t s, const int* gate = nullptr);

// Krylov steps fused with their reductions and the scalar update that follows (results bit for
// bit those of the separate calls): red_dots_op reduces into ks[out_idx + p] then runs op;
// ks_bi_s_op is s = r - alpha v, max |s| -> KS_SN, KS_BI_CHECK_S; ks_bi_xr_op is the x and r
// update with rh . r -> KS_RRN, max |r| -> KS_RN, KS_BI_CHECK_R; ks_cg_xr_op is CG's x and r
// update with max |r| -> KS_RN, KS_CHECK_R
void red_dots_op(long n, int np, const double* const a[4], const double* const b[4],
                 double* part, int out_idx, int op, double* ks, int* st, int* itc,
                 hipStream_t s);
void ks_bi_s_op(long n, double* sv, const double* r, const double* v, double* part, double* ks,
                int* st, int* itc, hipStream_t s);
void ks_bi_xr_op(long n, double* x, double* r, const double* ph, const double* sh,
                 const double* sv, const double* t, const double* rh, double* part, double* ks,
                 int* st, int* itc, hipStream_t s);
void ks_bi_xr_op(long n, double* x, double* r, const float* ph, const float* sh,
                 const double* sv, const double* t, const double* rh, double* part, double* ks,
                 int* st, int* itc, hipStream_t s);
void ks_cg_xr_op(long n, double* x, double* r, const double* p, const double* q, double* part,
                 double* ks, int* st, int* itc, hipStream_t s);

// reductions: per-block partials (part, >= 4*1024 doubles) then one fixed-order final pass
// into out (device)
int red_blocks(long n);
void red_dots(long n, int npairs, const double* const a[4], const double* const b[4],
              double* part, double* out, hipStream_t s, const int* gate = nullptr);
void red_maxabs(long n, int ncomp, const double* x, double* part, double* out, hipStream_t s,
                const int* gate = nullptr);
void red_sum_open(const GeomV& g, const double* x, double* part, double* out, hipStream_t s,
                  const int* gate = nullptr);
// out[0] = max over open cells of |u|+|v|+|w|, out[1] = max of theta there (1 if null)
void red_cfl(const GeomV& g, const double* u, const double* theta, double* part, double* out,
             hipStream_t s);
void red_sum(long n, int nrow, const double* x, double* part, double* out, hipStream_t s);
void op_face_flux_max(const GeomV& g, double* const f[3], double* part, double* out,
                      hipStream_t s);

// fixed-order final pass of nrow rows of nb per-block partials (mode 0 sum, 1 max) into out
void red_final(const double* part, int nb, int nrow, int mode, double* out, hipStream_t s,
               const int* gate = nullptr);

// nodal projection (eb_nodal.hip): nodal arrays [nz+1][ny+1][nx+1]; mask marks the unknowns
long nd_count(const GridV& g);
// out = D(w) - bflux (bflux nullable) on masked nodes (mask nullable: all); tsum (nullable): the
// sum of the sizes of D's terms per node
void nd_div(const GeomV& g, const double* w, const double* bflux, const uint8_t* mask,
            double* out, double* tsum, hipStream_t s);
// once per geometry: the boundary flux, the diagonal of L and the mask of the unknowns
void nd_setup(const GeomV& g, double* bflux, double* dg, uint8_t* mask, hipStream_t s);
void nd_apply(const GeomV& g, const double* x, const uint8_t* mask, double* y, hipStream_t s,
              const int* gate = nullptr);
void nd_grad(const GeomV& g, const double* q, double* gp, hipStream_t s);
void nd_jacobi(long M, const double* r, const double* dg, const uint8_t* mask, double* z,
               hipStream_t s, const int* gate = nullptr);
// x minus its mean over the unknowns (0 elsewhere); sumcnt: two device doubles
void nd_mean_free(long M, double* x, const uint8_t* mask, double* part, double* sumcnt,
                  hipStream_t s, const int* gate = nullptr);
void nd_scale_masked(long M, double a, const double* x, const uint8_t* mask, double* y,
                     hipStream_t s);
void nd_sync(const GridV& g, double* x, hipStream_t s);
void nd_peb(const GeomV& g, const double* pn, double* peb, hipStream_t s);

// vector kernels
void vec_copy(long n, const double* x, double* y, hipStream_t s);
void vec_fill(long n, double v, double* y, hipStream_t s);
void vec_axpby(long n, double a, const double* x, double b, double* y, hipStream_t s);
// y = x + a*(y - b*z)
void vec_bicg_p(long n, const double* r, double beta, double omega, const double* v, double* p,
                hipStream_t s);
// z = x - a*y
void vec_sub_scaled(long n, const double* x, double a, const double* y, double* z,
                    hipStream_t s);
void vec_bicg_update(long n, double al, const double* ph, double om, const double* sh,
                     const double* sv, const double* t, double* x, double* r, hipStream_t s);
void vec_mask_rhs(const GeomV& g, const double* psi, const double* a0, double* b,
                  hipStream_t s);

// ------------------------------------------------------------------------------------------
// adjoint (eb_adjoint.hip)
// ------------------------------------------------------------------------------------------
// transposed wall stencil: for cell c with map[c] = r >= 0, entries ent[ptr[r] .. ptr[r+1])
// are the flat stencil positions (slot * ncut + cut) that read u at c, in increasing order
struct WallT {
    const int* map;
    const int* ptr;
    const int* ent;
};
// adjoints of the left/right face states, [component][face] per direction
struct LRV {
    double* L[3];
    double* R[3];
};
void adj_redistribute(const GeomV& g, const double* Db, double* X, double* Y, double* DCb,
                      hipStream_t s);
void adj_visc_terms(const GeomV& g, const eb_rheology& r, const double* theta, const double* u,
                    const double* G9, const double* eta, const double* eta_eb, const double* gw,
                    const double* DCb, const double* etab_in, const double* etaebb_in,
                    double* ub, double* Gb, double* gwb, double* tau0b, hipStream_t s);
void adj_grad_gather(const GeomV& g, const WallT& wt, const double* Gb, const double* gwb,
                     double* ub, hipStream_t s);
void adj_conv_face_w(const GeomV& g, const double* u, double* const w[3], const double* DCb,
                     double* wb[3], hipStream_t s);
void adj_conv_lr(const GeomV& g, const double* u, double* const w[3], const double* DCb,
                 double* const wbin[3], const LRV& lr, double* ub, hipStream_t s);
void adj_face_grad_T_neg(const GeomV& g, double* const fb[3], double* out, hipStream_t s);
void adj_div_T_add(const GeomV& g, double beta, const double* z, double* wb[3], hipStream_t s);
void adj_cc_cell(const GeomV& g, const double* z, double* ub, hipStream_t s);
void adj_gcc_T(const GeomV& g, double a, const double* v, const double* base, double* out,
               hipStream_t s);
void adj_visc_apply_T(const GeomV& g, double rho, double dt, const double* eta,
                      const double* eta_eb, const WallT& wt, const double* lam, double* out,
                      hipStream_t s, const int* gate = nullptr);
void adj_visc_coef(const GeomV& g, double dt, const double* x, const double* lam, double* etab,
                   double* etaebb, hipStream_t s);
void adj_psi(const GeomV& g, double rho, double dt, const double* lam, double* psib, double* ub,
             double* Cb, double* Vb, hipStream_t s);
void adj_drag(const GeomV& g, const eb_rheology& r, const double* theta, const double* gw,
              const double fb[3], double* gwb, double* tau0b, double* pb, double* gpb,
              hipStream_t s);
void adj_mask_open(const GeomV& g, int ncomp, const double* in, double* out, hipStream_t s);
void adj_scale(long n, double a, double* x, hipStream_t s);
