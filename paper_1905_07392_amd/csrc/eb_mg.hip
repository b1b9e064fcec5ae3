// eb_mg.hip -- geometric multigrid preconditioner, the exact EB viscous operator, reductions
// and Krylov vector kernels.
//
// Level operators are 7-point and symmetric: (M x)_c = D_c x_c - sum_f K_f x_nb(f), where a
// face on a Dirichlet domain wall only adds its K to D.  Level 0 takes its face coefficients
// from the apertures (Poisson) or apertures and face viscosities (viscous); coarse levels
// average four child faces (and rescale by 1/4 for the doubled spacing) and eight child
// cell shifts, the viscous faces with the viscosity along each child face's normal line taken
// in series (coarsen_face_series), which keeps the coarse operators faithful across the
// 1e7 viscosity contrast of a plug next to a sheared layer.  Smoothing is red-black
// Gauss-Seidel; within a colour every update depends only on the other colour, so the result
// does not depend on thread order (or on how many cells a thread updates).
#include "eb_internal.hpp"
#include <type_traits>

namespace {

// ------------------------------------------------------------------------------------------
// operator construction
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void face_ijk(const GridV& g, int d, long f, int& i, int& j, int& k) {
    unsigned m0 = g.n[0] + (d == 0), m1 = g.n[1] + (d == 1), fu = (unsigned)f;
    unsigned r = fu / m0;
    i = (int)(fu - r * m0);
    unsigned kk = r / m1;
    j = (int)(r - kk * m1);
    k = (int)kk;
}

__global__ void k_K_poisson(GeomV g, int d, double beta, double* __restrict__ K) {
    long nf = face_count(g.grid, d);
    long f = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int i, j, k;
    face_ijk(g.grid, d, f, i, j, k);
    int q[3] = {i, j, k};
    q[d] -= 1;
    long lo = cell_at(g.grid, q[0], q[1], q[2]);
    q[d] += 1;
    long hi = cell_at(g.grid, q[0], q[1], q[2]);
    double A = g.ap[d][f];
    double h = g.grid.h;
    K[f] = (A > 0.0 && lo >= 0 && hi >= 0) ? beta * A / (h * h) : 0.0;
}

__global__ void k_K_visc(GeomV g, int d, double dt, const double* __restrict__ eta,
                         double* __restrict__ K) {
    long nf = face_count(g.grid, d);
    long f = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int i, j, k;
    face_ijk(g.grid, d, f, i, j, k);
    int q[3] = {i, j, k};
    q[d] -= 1;
    long lo = cell_at(g.grid, q[0], q[1], q[2]);
    q[d] += 1;
    long hi = cell_at(g.grid, q[0], q[1], q[2]);
    double A = g.ap[d][f];
    double h2 = g.grid.h * g.grid.h;
    double v = 0.0;
    if (A > 0.0) {
        if (lo >= 0 && hi >= 0)
            v = dt * A * 0.5 * (eta[lo] + eta[hi]) / h2;
        else
            v = 2.0 * dt * A * eta[lo >= 0 ? lo : hi] / h2;
    }
    K[f] = v;
}

// The preconditioner's stand-in for the EB wall flux of a cut cell: the flux of a linear profile
// through u_EB and the cell value at this distance (in cells) from the wall, whatever the cell
// centre's own distance (under 0.87 for every cut cell).  The operator's wall flux reads two
// planes of other cells, so no diagonal term matches it mode by mode; a weaker term than the
// centre distance would give lets the Krylov solve converge in about a third fewer iterations.
constexpr double M_WALL_DIST = 2.0;

__global__ void k_S_visc(GeomV g, double rho, double dt, const double* __restrict__ eta_eb,
                         double* __restrict__ S) {
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= g.N) return;
    double al = g.alpha[c];
    double v = 0.0;
    if (al > 0.0) {
        v = al * rho;
        int q = g.cutid[c];
        if (q >= 0) {
            v += dt * g.aeb[q] * eta_eb[q] / (M_WALL_DIST * g.grid.h * g.grid.h);
        }
    }
    S[c] = v;
}

// diagonal of cell c: S plus the six face coefficients (0 on a closed cell)
__device__ __forceinline__ double diag_value(const GridV& g, const double* const K[3],
                                             const double* S, const uint8_t* mask, long c) {
    if (!mask[c]) return 0.0;
    int i, j, k;
    cell_coords(g, c, i, j, k);
    double s = S ? S[c] : 0.0;
    for (int d = 0; d < 3; d++) {
        int q[3] = {i, j, k};
        s += K[d][face_index(g, d, q[0], q[1], q[2])];
        q[d] += 1;
        s += K[d][face_index(g, d, q[0], q[1], q[2])];
    }
    return s;
}

__global__ void k_diag(GridV g, const double* __restrict__ Kx, const double* __restrict__ Ky,
                       const double* __restrict__ Kz, const double* __restrict__ S,
                       const uint8_t* __restrict__ mask, double* __restrict__ D) {
    long N = (long)g.n[0] * g.n[1] * g.n[2];
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    const double* K[3] = {Kx, Ky, Kz};
    D[c] = diag_value(g, K, S, mask, c);
}

// One operator-build launch per level: the coarse level's face coefficients (scale x the four
// fine faces) and cell terms (mean of the eight children) from the fine level, and the fine
// level's diagonal, which is complete by then.  Threads are dealt to the five parts in turn.
struct CoarsenArgs {
    GridV gc, gf;
    const double* Kf[3];
    const double* apf[3];  // fine apertures (the viscous system's series coarsening)
    int series;
    double* Kc[3];
    const double* Sf;
    double* Sc;
    double scale;
    const uint8_t* maskf;
    double* Df;
    long n[5];  // coarse faces per direction, coarse cells, fine cells
};
__global__ void k_coarsen_level(CoarsenArgs A) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    for (int d = 0; d < 3; d++) {
        if (t < A.n[d]) {
            A.Kc[d][t] = A.series
                             ? coarsen_face_series(A.gc, A.gf, d, A.Kf[d], A.apf[d], t, A.scale)
                             : coarsen_face_value(A.gc, A.gf, d, A.Kf[d], t, A.scale);
            return;
        }
        t -= A.n[d];
    }
    if (t < A.n[3]) {
        A.Sc[t] = coarsen_cell_value(A.gc, A.gf, A.Sf, t);
        return;
    }
    t -= A.n[3];
    if (t < A.n[4]) A.Df[t] = diag_value(A.gf, A.Kf, A.Sf, A.maskf, t);
}

__global__ void k_to_float(long n, const double* __restrict__ a, float* __restrict__ b) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) b[t] = (float)a[t];
}

template <typename A, typename B>
__global__ void k_cast(long n, const A* __restrict__ a, B* __restrict__ b, const int* gate) {
    if (gate && *gate) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) b[t] = (B)a[t];
}

// ------------------------------------------------------------------------------------------
// smoother, residual, transfers
// ------------------------------------------------------------------------------------------
// sum over the six faces of K_f x_nb (faces without a neighbour cell only feed the diagonal)
template <typename T, int NC>
__device__ __forceinline__ void offdiag(const LevelV<T>& L, const T* __restrict__ x, int i, int j,
                                        int k, T acc[NC]) {
    const GridV& g = L.grid;
    long N = L.N;
    long c = cell_index(g, i, j, k);
#pragma unroll
    for (int d = 0; d < 3; d++) {
#pragma unroll
        for (int side = 0; side < 2; side++) {
            int f[3] = {i, j, k};
            f[d] += side;
            T K = L.K[d][face_index(g, d, f[0], f[1], f[2])];
            if (K == (T)0) continue;
            long nb = cell_step(g, c, i, j, k, d, side);
            if (nb < 0) continue;
#pragma unroll
            for (int m = 0; m < NC; m++) acc[m] += K * x[m * N + nb];
        }
    }
}

// Prolongation carried by the first post-smoothing sweeps instead of a pass of its own: the
// coarse correction ec (on grid gc) is added on the fly where the separate pass would have
// stored it.  PRO_NBR: to every neighbour's value read by the update (the other colour, whose
// correction is still pending) and to the cell's own value where the cell is open but its row
// is degenerate (it is not updated); PRO_OWN: only the latter.  The Gauss-Seidel update itself
// does not read the cell's own value, so an updated cell needs no correction, and the sums are
// bit for bit those of the separate prolongation (the same addition, in the same precision).
// (PRO_ZERO, for the colour-split finest level only: no prolongation; a cell that is not updated
// is set to 0, so the pass before it need not zero this colour)
enum { PRO_NONE = 0, PRO_OWN = 1, PRO_NBR = 2, PRO_ZERO = 3 };
template <typename TC>
struct ProV {
    GridV gc;
    const TC* ec;
};

// coarse cell under the neighbour across face f = 2d + side of fine cell (i, j, k), which
// exists: its coordinates wrapped as cell_at wraps them, then halved
__device__ __forceinline__ long nb_parent(const GridV& gf, const GridV& gc, int i, int j, int k,
                                          int f) {
    int q[3] = {i, j, k};
    int d = f >> 1;
    q[d] += (f & 1) ? 1 : -1;
    if (q[d] < 0) q[d] += gf.n[d];
    else if (q[d] >= gf.n[d]) q[d] -= gf.n[d];
    return cell_index(gc, q[0] >> 1, q[1] >> 1, q[2] >> 1);
}

// The corrections a fused prolongation adds to the six neighbour values of fine cell (i, j, k)
// (0 where there is no neighbour).  The separate pass adds e only to open cells, but a closed
// neighbour's value is never used: every face of a covered cell has aperture 0 (that is how
// cells are classified), so its coupling K is 0, and on a coarse level a nonzero K is a sum of
// open fine faces, whose cells make both coarse cells open.  In each direction one neighbour
// shares the cell's coarse parent and the other lies in the adjacent parent, so four coarse
// values are read.  nbr_load issues the loads (before anything waits on memory),
// nbr_corrections forms the corrections once they are needed.
template <int NC, typename TC>
struct NbrE {
    TC e0[NC], eo[3][NC];
};
template <int NC, typename TC>
__device__ __forceinline__ void nbr_load(const GridV& gf, const ProV<TC>& P, int i, int j, int k,
                                         const long nb[6], NbrE<NC, TC>& E) {
    long Nc = (long)P.gc.n[0] * P.gc.n[1] * P.gc.n[2];
    const TC* __restrict__ ec = P.ec;
    int q[3] = {i, j, k};
    long p0 = cell_index(P.gc, i >> 1, j >> 1, k >> 1);
#pragma unroll
    for (int m = 0; m < NC; m++) E.e0[m] = ec[m * Nc + p0];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        int f = 2 * d + (q[d] & 1);
        long po = nb[f] >= 0 ? nb_parent(gf, P.gc, i, j, k, f) : p0;
#pragma unroll
        for (int m = 0; m < NC; m++) E.eo[d][m] = ec[m * Nc + po];
    }
}
template <typename T, int NC, typename TC>
__device__ __forceinline__ void nbr_corrections(const NbrE<NC, TC>& E, int i, int j, int k,
                                                const long nb[6], T pe[6][NC]) {
    int q[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            int f = 2 * d + side;
            bool on = nb[f] >= 0;
            bool outer = side == (q[d] & 1);
#pragma unroll
            for (int m = 0; m < NC; m++)
                pe[f][m] = on ? (T)(outer ? E.eo[d][m] : E.e0[m]) : (T)0;
        }
}

// one Gauss-Seidel update of the t-th cell of colour col (cells of a colour are numbered row by
// row, nx/2 per row), with the prolongation PRO fused in
template <typename T, int NC, int PRO = PRO_NONE, typename TC = T>
__device__ __forceinline__ void smooth_cell(const LevelV<T>& L, const T* __restrict__ b,
                                            T* __restrict__ x, long t, int col,
                                            const ProV<TC>* P = nullptr) {
    const GridV& g = L.grid;
    unsigned nxh = (unsigned)g.n[0] >> 1, ny = (unsigned)g.n[1];
    unsigned row = (unsigned)t / nxh;
    int ih = (int)((unsigned)t - row * nxh);
    unsigned kk = row / ny;
    int j = (int)(row - kk * ny);
    int k = (int)kk;
    int i = 2 * ih + ((j + k + col) & 1);
    long c = cell_index(g, i, j, k);
    // every load before the first use (offdiag's terms, in its order)
    long nb[6];
    T K[6], xn[6][NC], acc[NC];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            int f[3] = {i, j, k};
            f[d] += side;
            K[2 * d + side] = L.K[d][face_index(g, d, f[0], f[1], f[2])];
            nb[2 * d + side] = cell_step(g, c, i, j, k, d, side);
        }
    uint8_t msk = L.mask[c];
    T dg = L.D[c];
#pragma unroll
    for (int m = 0; m < NC; m++) acc[m] = b[m * L.N + c];
#pragma unroll
    for (int f = 0; f < 6; f++)
#pragma unroll
        for (int m = 0; m < NC; m++) xn[f][m] = nb[f] >= 0 ? x[m * L.N + nb[f]] : (T)0;
    long Nc = 0;
    if (PRO != PRO_NONE) Nc = (long)P->gc.n[0] * P->gc.n[1] * P->gc.n[2];
    T pe[6][NC];
    NbrE<NC, TC> E;
    if (PRO == PRO_NBR) {
        nbr_load<NC, TC>(g, *P, i, j, k, nb, E);
        nbr_corrections<T, NC, TC>(E, i, j, k, nb, pe);
    }
    if (!msk) return;
    if (!(dg > (T)0)) {
        if (PRO != PRO_NONE) {
            long pc = cell_index(P->gc, i >> 1, j >> 1, k >> 1);
#pragma unroll
            for (int m = 0; m < NC; m++) x[m * L.N + c] += (T)P->ec[m * Nc + pc];
        }
        return;
    }
    if (PRO == PRO_NBR) {
#pragma unroll
        for (int f = 0; f < 6; f++)
#pragma unroll
            for (int m = 0; m < NC; m++) xn[f][m] = xn[f][m] + pe[f][m];
    }
#pragma unroll
    for (int f = 0; f < 6; f++) {
        if (K[f] == (T)0 || nb[f] < 0) continue;
#pragma unroll
        for (int m = 0; m < NC; m++) acc[m] += K[f] * xn[f][m];
    }
#pragma unroll
    for (int m = 0; m < NC; m++) x[m * L.N + c] = acc[m] / dg;
}

// piecewise-constant prolongation of the coarse correction to open children
template <typename TC, typename TF, int NC>
__device__ __forceinline__ void prolong_cell(const GridV& gf, const GridV& gc,
                                             const uint8_t* __restrict__ mf,
                                             const TC* __restrict__ ec, TF* __restrict__ xf,
                                             long f) {
    long Nc = (long)gc.n[0] * gc.n[1] * gc.n[2];
    long Nf = (long)gf.n[0] * gf.n[1] * gf.n[2];
    if (!mf[f]) return;
    int i, j, k;
    cell_coords(gf, f, i, j, k);
    long c = cell_index(gc, i >> 1, j >> 1, k >> 1);
#pragma unroll
    for (int m = 0; m < NC; m++) xf[m * Nf + f] += (TF)ec[m * Nc + c];
}

// first red half sweep from a zero iterate, over the whole grid: red cells get b/D (all their
// neighbours are zero), every other cell 0 -- the zero fill and the first sweep in one pass
template <typename T, int NC>
__global__ void k_smooth_first(LevelV<T> L, const T* __restrict__ b, T* __restrict__ x) {
    if (L.gate && *L.gate) return;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= L.N) return;
    int i, j, k;
    cell_coords(L.grid, c, i, j, k);
    bool upd = ((i + j + k) & 1) == 0 && L.mask[c] && L.D[c] > (T)0;
    T dg = upd ? L.D[c] : (T)1;
#pragma unroll
    for (int m = 0; m < NC; m++) x[m * L.N + c] = upd ? (b[m * L.N + c] + (T)0) / dg : (T)0;
}

// Residual of the fine level restricted to the coarse right-hand side in one pass.  A block
// handles RR_COARSE consecutive coarse cells: each thread forms the residual of one of their
// eight children, then one thread per coarse cell sums the children in the fixed order
// q = 0..7 (child (2i + (q&1), 2j + (q>>1&1), 2k + (q>>2))).
constexpr int RR_COARSE = 32;
constexpr int RR_THREADS = 8 * RR_COARSE;

// thread t of a block: child bits and coarse slot, x fastest so rows of fine cells are read
// contiguously
__device__ __forceinline__ void rr_child(int t, int& a, int& cl, int& bq, int& cq) {
    a = t & 1;
    cl = (t >> 1) & (RR_COARSE - 1);
    bq = (t >> 6) & 1;
    cq = t >> 7;
}
__device__ __forceinline__ int rr_thread(int cl, int q) {
    return ((q >> 2) * 2 + ((q >> 1) & 1)) * (2 * RR_COARSE) + cl * 2 + (q & 1);
}

// The coarse level's first pre-smoothing pass carried by the restriction into it: with x set,
// the thread that stores a coarse right-hand side also stores k_smooth_first's iterate for that
// cell (b / D on open colour-0 cells with a positive diagonal, 0 elsewhere), computed from the
// stored right-hand side exactly as k_smooth_first computes it.
template <typename TC>
struct FirstV {
    TC* x;          // null: no fused first pass
    const TC* D;    // the coarse level's diagonal, in its precision
};

template <typename TF, typename TC, int NC>
__device__ __forceinline__ void rr_store(const GridV& gc, long Nc, long cc,
                                         const uint8_t* __restrict__ mc, const TF sum[NC],
                                         TC* __restrict__ bc, const FirstV<TC>& F1) {
    bool open = mc[cc] != 0;
    TC bcv[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) {
        bcv[m] = open ? (TC)(sum[m] / (TF)8) : (TC)0;
        bc[m * Nc + cc] = bcv[m];
    }
    if (F1.x) {
        int i, j, k;
        cell_coords(gc, cc, i, j, k);
        bool upd = ((i + j + k) & 1) == 0 && open && F1.D[cc] > (TC)0;
        TC dg = upd ? F1.D[cc] : (TC)1;
#pragma unroll
        for (int m = 0; m < NC; m++) F1.x[m * Nc + cc] = upd ? (bcv[m] + (TC)0) / dg : (TC)0;
    }
}


template <typename TF, typename TC, int NC>
__global__ void __launch_bounds__(RR_THREADS)
    k_resid_restrict(LevelV<TF> L, const TF* __restrict__ b, const TF* __restrict__ x, GridV gc,
                     const uint8_t* __restrict__ mc, TC* __restrict__ bc, FirstV<TC> F1) {
    if (L.gate && *L.gate) return;
    __shared__ TF rs[RR_THREADS * NC];
    long Nc = (long)gc.n[0] * gc.n[1] * gc.n[2];
    int a, cl, bq, cq;
    rr_child(threadIdx.x, a, cl, bq, cq);
    long c = (long)blockIdx.x * RR_COARSE + cl;
    TF r[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) r[m] = (TF)0;
    if (c < Nc) {
        int i, j, k;
        cell_coords(gc, c, i, j, k);
        int fi = 2 * i + a, fj = 2 * j + bq, fk = 2 * k + cq;
        long f = cell_index(L.grid, fi, fj, fk);
        // every load before the first use (offdiag's terms, in its order)
        const GridV& g = L.grid;
        long nb[6];
        TF K[6], xn[6][NC], bv[NC], xv[NC];
#pragma unroll
        for (int d = 0; d < 3; d++)
#pragma unroll
            for (int side = 0; side < 2; side++) {
                int e[3] = {fi, fj, fk};
                e[d] += side;
                K[2 * d + side] = L.K[d][face_index(g, d, e[0], e[1], e[2])];
                nb[2 * d + side] = cell_step(g, f, fi, fj, fk, d, side);
            }
        uint8_t msk = L.mask[f];
        TF dg = L.D[f];
#pragma unroll
        for (int m = 0; m < NC; m++) {
            bv[m] = b[m * L.N + f];
            xv[m] = x[m * L.N + f];
        }
#pragma unroll
        for (int e = 0; e < 6; e++)
#pragma unroll
            for (int m = 0; m < NC; m++) xn[e][m] = nb[e] >= 0 ? x[m * L.N + nb[e]] : (TF)0;
        if (msk) {
            TF acc[NC];
#pragma unroll
            for (int m = 0; m < NC; m++) acc[m] = (TF)0;
#pragma unroll
            for (int e = 0; e < 6; e++) {
                if (K[e] == (TF)0 || nb[e] < 0) continue;
#pragma unroll
                for (int m = 0; m < NC; m++) acc[m] += K[e] * xn[e][m];
            }
#pragma unroll
            for (int m = 0; m < NC; m++) r[m] = bv[m] - (dg * xv[m] - acc[m]);
        }
    }
#pragma unroll
    for (int m = 0; m < NC; m++) rs[threadIdx.x * NC + m] = r[m];
    __syncthreads();
    if (threadIdx.x < RR_COARSE) {
        long cc = (long)blockIdx.x * RR_COARSE + threadIdx.x;
        if (cc >= Nc) return;
        TF sum[NC];
#pragma unroll
        for (int m = 0; m < NC; m++) sum[m] = (TF)0;
        for (int q = 0; q < 8; q++) {
            int t = rr_thread(threadIdx.x, q);
#pragma unroll
            for (int m = 0; m < NC; m++) sum[m] += rs[t * NC + m];
        }
        rr_store<TF, TC, NC>(gc, Nc, cc, mc, sum, bc, F1);
    }
}

template <typename T, int NC>
__global__ void k_smooth(LevelV<T> L, const T* __restrict__ b, T* __restrict__ x, int col) {
    if (L.gate && *L.gate) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < L.N / 2) smooth_cell<T, NC>(L, b, x, t, col);
}

// a half sweep with the prolongation of ec fused in (PRO_NBR or PRO_OWN)
template <typename T, typename TC, int NC, int PRO>
__global__ void k_smooth_pro(LevelV<T> L, const T* __restrict__ b, T* __restrict__ x, int col,
                             ProV<TC> P) {
    if (L.gate && *L.gate) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < L.N / 2) smooth_cell<T, NC, PRO, TC>(L, b, x, t, col, &P);
}

template <typename TC, typename TF, int NC>
__global__ void k_prolong(GridV gf, GridV gc, const uint8_t* __restrict__ mf,
                          const TC* __restrict__ ec, TF* __restrict__ xf, const int* gate) {
    if (gate && *gate) return;
    long Nf = (long)gf.n[0] * gf.n[1] * gf.n[2];
    long f = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (f < Nf) prolong_cell<TC, TF, NC>(gf, gc, mf, ec, xf, f);
}

// ------------------------------------------------------------------------------------------
// finest level in colour-split storage.  Vectors of level 0 are kept as [component][colour]
// [cell of that colour in natural order]: cell c = (i, j, k) of colour (i+j+k) mod 2 sits at
// colour * N/2 + c/2 (nx is even).  A half sweep then reads the other colour of the iterate and
// its own colour of the right-hand side contiguously and writes its own colour contiguously;
// the FP64 and FP32 half sweeps take two and four cells of one colour per thread, with 16-byte
// loads (k_smooth_rb_pair, k_smooth_rb_quad).  Coefficients of regular cells (all six
// apertures 1) are recomputed from eta with the same expressions, in the same order, as the
// stored operator, so results are bitwise those of the stored coefficients; cut cells read the
// stored faces and diagonal.
// ------------------------------------------------------------------------------------------
// unsigned division by a fixed divisor d, for dividends below 2^31, as a multiply-high, an add
// and a shift (m and s from fast_div); the index arithmetic of the finest level's one-thread-
// per-cell kernels would otherwise spend two integer division sequences per thread
struct FastDiv {
    unsigned d, m, s;
};
inline FastDiv fast_div(unsigned d) {
    FastDiv f;
    f.d = d;
    f.s = 0;
    while ((1u << f.s) < d) f.s++;
    f.m = (unsigned)(((1ull << 32) * ((1ull << f.s) - d)) / d + 1);
    return f;
}
__device__ __forceinline__ unsigned fdiv(unsigned n, const FastDiv& f) {
    return (__umulhi(n, f.m) + n) >> f.s;
}

struct Rb0V {
    GridV grid;
    FastDiv dnx, dny, dnxh;  // n_x, n_y, n_x / 2
    long N;
    const uint8_t* flag;
    const int* cut;  // the cut cells (flag 1), ncut of them
    int ncut;
    const double* etacs;     // colour-split copies of eta, its FP32 copy, and the flags
    const float* etafcs;     // (may be null)
    const uint8_t* flagcs;
    const double* eta;
    const float* etaf;
    const double* K[3];
    const double* D;
    int sys;
    double rho;
    double kin, kwall, kpois;  // dt/(2h^2), 2dt/h^2, beta/h^2
    const int* gate;
};

__device__ __forceinline__ long rb_slot(long N, int i, int j, int k, long c) {
    return (long)((i + j + k) & 1) * (N >> 1) + (c >> 1);
}

// the operator row of cell c: K and neighbours (natural index, -1 = none) of the six faces in
// the order (d, lower), (d, upper); returns false when the cell is not smoothed.  In FP64 a
// regular cell's coefficients are bitwise the stored ones; the FP32 smoother forms them in
// FP32 from an FP32 copy of eta (cut cells round the stored FP64 values).
template <typename T>
__device__ __forceinline__ const T* eta_of(const Rb0V& L);
template <>
__device__ __forceinline__ const double* eta_of<double>(const Rb0V& L) { return L.eta; }
template <>
__device__ __forceinline__ const float* eta_of<float>(const Rb0V& L) { return L.etaf; }

template <typename T>
__device__ __forceinline__ bool rb0_row(const Rb0V& L, long c, int i, int j, int k, T K[6],
                                        long nb[6], T& D) {
    uint8_t fl = L.flag[c];
    if (fl == 0) return false;
    const GridV& g = L.grid;
    if (fl == 2) {
        // all six apertures are 1: K = dt (eta_c + eta_n)/(2 h^2) inside, 2 dt eta_c/h^2 on a
        // domain wall (viscous); beta/h^2 inside, 0 on a wall (Poisson)
        const T* eta = eta_of<T>(L);
        T kin = (T)L.kin, kwall = (T)L.kwall, kp = (T)L.kpois;
        T s = L.sys == EB_SYS_VISC ? (T)L.rho : (T)0;
        T ec = L.sys == EB_SYS_VISC ? eta[c] : (T)0;
#pragma unroll
        for (int d = 0; d < 3; d++)
#pragma unroll
            for (int side = 0; side < 2; side++) {
                long n = cell_step(g, c, i, j, k, d, side);
                T kf;
                if (L.sys == EB_SYS_VISC) kf = n >= 0 ? kin * (ec + eta[n]) : kwall * ec;
                else kf = n >= 0 ? kp : (T)0;
                s += kf;
                K[2 * d + side] = kf;
                nb[2 * d + side] = n;
            }
        D = s;
        return D > (T)0;
    }
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            int f[3] = {i, j, k};
            f[d] += side;
            K[2 * d + side] = (T)L.K[d][face_index(g, d, f[0], f[1], f[2])];
            nb[2 * d + side] = cell_step(g, c, i, j, k, d, side);
        }
    D = (T)L.D[c];
    return D > (T)0;
}

// cell coordinates of the t-th cell of colour col (the same as rb_cell below, with the
// divisions of L's extents)
__device__ __forceinline__ void rb_cell(const Rb0V& L, unsigned t, int col, int& i, int& j,
                                        int& k) {
    unsigned row = fdiv(t, L.dnxh);
    unsigned ih = t - row * L.dnxh.d;
    unsigned kk = fdiv(row, L.dny);
    j = (int)(row - kk * L.dny.d);
    k = (int)kk;
    i = 2 * (int)ih + ((j + k + col) & 1);
}
// natural cell c's coordinates with L's divisions (cell_coords)
__device__ __forceinline__ void rb_coords(const Rb0V& L, long c, int& i, int& j, int& k) {
    unsigned cu = (unsigned)c;
    unsigned t = fdiv(cu, L.dnx);
    i = (int)(cu - t * L.dnx.d);
    unsigned k2 = fdiv(t, L.dny);
    j = (int)(t - k2 * L.dny.d);
    k = (int)k2;
}

// cell coordinates of the t-th cell of colour col
__device__ __forceinline__ void rb_cell(const GridV& g, unsigned t, int col, int& i, int& j,
                                        int& k) {
    unsigned nxh = (unsigned)g.n[0] >> 1;
    unsigned row = t / nxh;
    unsigned ih = t - row * nxh;
    j = (int)(row % (unsigned)g.n[1]);
    k = (int)(row / (unsigned)g.n[1]);
    i = 2 * (int)ih + ((j + k + col) & 1);
}

// Every load of a cell (flag, right-hand side, the other colour's six neighbours, the seven
// viscosities of a regular cell) is issued before the first one is needed, so a thread waits for
// memory once; the row and the update are then rb0_row's and the order of the sums is unchanged.
// rb0_row with every load issued before the first is needed: the flag, the seven viscosities of
// a regular cell and, with NBR, the NC values of the six neighbours from the other colour's half
// xo (xn[f] = 0 where there is none).  The row is rb0_row's bit for bit.
template <typename T, int NC, bool NBR>
__device__ __forceinline__ bool rb0_row_ld(const Rb0V& L, long c, int i, int j, int k,
                                           const T* __restrict__ xo, T K[6], long nb[6], T& D,
                                           T xn[6][NC]) {
    const GridV& g = L.grid;
    long N = L.N;
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            nb[2 * d + side] = cell_step(g, c, i, j, k, d, side);
        }
    uint8_t fl = L.flag[c];
    if (NBR)
#pragma unroll
        for (int f = 0; f < 6; f++)
#pragma unroll
            for (int m = 0; m < NC; m++) xn[f][m] = nb[f] >= 0 ? xo[m * N + (nb[f] >> 1)] : (T)0;
    const T* eta = eta_of<T>(L);
    bool visc = L.sys == EB_SYS_VISC;
    T ec = visc ? eta[c] : (T)0, en[6];
#pragma unroll
    for (int f = 0; f < 6; f++) en[f] = (visc && nb[f] >= 0) ? eta[nb[f]] : (T)0;
    if (fl == 0) return false;
    if (fl == 2) {
        T kin = (T)L.kin, kwall = (T)L.kwall, kp = (T)L.kpois;
        T sd = visc ? (T)L.rho : (T)0;
#pragma unroll
        for (int f = 0; f < 6; f++) {
            T kf;
            if (visc) kf = nb[f] >= 0 ? kin * (ec + en[f]) : kwall * ec;
            else kf = nb[f] >= 0 ? kp : (T)0;
            sd += kf;
            K[f] = kf;
        }
        D = sd;
        return D > (T)0;
    }
    long nb2[6];
    return rb0_row<T>(L, c, i, j, k, K, nb2, D);
}

// one colour-split Gauss-Seidel update of the t-th cell of colour col, with the prolongation PRO
// fused in (the open cells of level 0 are those with a nonzero flag)
template <typename T, int NC, int PRO, typename TC>
__device__ __forceinline__ void smooth_rb_cell(const Rb0V& L, const T* __restrict__ b,
                                               T* __restrict__ x, int col, long t,
                                               const ProV<TC>* P) {
    long N = L.N, Nh = N >> 1;
    int i, j, k;
    rb_cell(L, (unsigned)t, col, i, j, k);
    long c = cell_index(L.grid, i, j, k);
    long own = (long)col * Nh + t, oth = (long)(1 - col) * Nh;
    T acc[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) acc[m] = b[m * N + own];
    T K[6], dg, xn[6][NC];
    long nb[6];
    long Nc = 0;
    constexpr bool PROL = PRO == PRO_OWN || PRO == PRO_NBR;
    if (PROL) Nc = (long)P->gc.n[0] * P->gc.n[1] * P->gc.n[2];
    T pe[6][NC];
    NbrE<NC, TC> E;
    if (PRO == PRO_NBR) {
        // the neighbours' indices (rb0_row_ld forms the same ones) and the coarse loads first
#pragma unroll
        for (int d = 0; d < 3; d++)
#pragma unroll
            for (int side = 0; side < 2; side++) {
                nb[2 * d + side] = cell_step(L.grid, c, i, j, k, d, side);
            }
        nbr_load<NC, TC>(L.grid, *P, i, j, k, nb, E);
    }
    bool upd = rb0_row_ld<T, NC, true>(L, c, i, j, k, x + oth, K, nb, dg, xn);
    if (PRO == PRO_NBR) nbr_corrections<T, NC, TC>(E, i, j, k, nb, pe);
    if (!upd) {
        if (PRO == PRO_ZERO) {
#pragma unroll
            for (int m = 0; m < NC; m++) x[m * N + own] = (T)0;
        } else if (PROL && L.flag[c] != 0) {
            long pc = cell_index(P->gc, i >> 1, j >> 1, k >> 1);
#pragma unroll
            for (int m = 0; m < NC; m++) x[m * N + own] += (T)P->ec[m * Nc + pc];
        }
        return;
    }
    if (PRO == PRO_NBR) {
#pragma unroll
        for (int f = 0; f < 6; f++)
#pragma unroll
            for (int m = 0; m < NC; m++) xn[f][m] = xn[f][m] + pe[f][m];
    }
#pragma unroll
    for (int f = 0; f < 6; f++) {
        T kf = K[f];
        if (kf == (T)0 || nb[f] < 0) continue;
#pragma unroll
        for (int m = 0; m < NC; m++) acc[m] += kf * xn[f][m];
    }
    T inv = (T)1 / dg;
#pragma unroll
    for (int m = 0; m < NC; m++) x[m * N + own] = acc[m] * inv;
}

// y = M x on level 0 in natural order, the regular cells' coefficients formed on the fly as the
// colour-split smoother forms them (bit for bit the stored ones), so only x, the flags and y
// move: every load is issued first, and y is resid_cell's (without b) bit for bit
template <int NC>
__global__ void __launch_bounds__(EB_BLOCK)
    k_apply0(Rb0V L, const double* __restrict__ x, double* __restrict__ y) {
    if (L.gate && *L.gate) return;
    long N = L.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    int i, j, k;
    rb_coords(L, c, i, j, k);
    long nb[6];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            nb[2 * d + side] = cell_step(L.grid, c, i, j, k, d, side);
        }
    double xv[NC], xn[6][NC];
#pragma unroll
    for (int m = 0; m < NC; m++) xv[m] = x[m * N + c];
#pragma unroll
    for (int f = 0; f < 6; f++)
#pragma unroll
        for (int m = 0; m < NC; m++) xn[f][m] = nb[f] >= 0 ? x[m * N + nb[f]] : 0.0;
    double K[6], dg, unused[6][NC];
    rb0_row_ld<double, NC, false>(L, c, i, j, k, x, K, nb, dg, unused);
    if (L.flag[c] == 0) {
#pragma unroll
        for (int m = 0; m < NC; m++) y[m * N + c] = 0.0;
        return;
    }
    double acc[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) acc[m] = 0.0;
#pragma unroll
    for (int f = 0; f < 6; f++) {
        if (K[f] == 0.0 || nb[f] < 0) continue;
#pragma unroll
        for (int m = 0; m < NC; m++) acc[m] += K[f] * xn[f][m];
    }
#pragma unroll
    for (int m = 0; m < NC; m++) y[m * N + c] = dg * xv[m] - acc[m];
}

template <typename T, int NC>
__global__ void __launch_bounds__(EB_BLOCK)
    k_smooth_rb(Rb0V L, const T* __restrict__ b, T* __restrict__ x, int col) {
    if (L.gate && *L.gate) return;
    long t = xcd_block() * (long)blockDim.x + threadIdx.x;
    if (t >= (L.N >> 1)) return;
    smooth_rb_cell<T, NC, PRO_NONE, T>(L, b, x, col, t, nullptr);
}

// the row of a regular cell (flag 2: every aperture 1, no wall flux) from its loaded
// viscosities, as rb0_row_ld forms it: K[f] per face and the diagonal, returned.  nb[f] >= 0
// where the cell has a neighbour across face f; VISC: the viscous system (else Poisson).
template <typename T, bool VISC>
__device__ __forceinline__ T rb0_regular_row(const Rb0V& L, const long nb[6], T ec,
                                             const T en[6], T K[6]) {
    T kin = (T)L.kin, kwall = (T)L.kwall, kp = (T)L.kpois;
    T sd = VISC ? (T)L.rho : (T)0;
#pragma unroll
    for (int f = 0; f < 6; f++) {
        T kf;
        if (VISC) kf = nb[f] >= 0 ? kin * (ec + en[f]) : kwall * ec;
        else kf = nb[f] >= 0 ? kp : (T)0;
        sd += kf;
        K[f] = kf;
    }
    return sd;
}
// smooth_rb_cell's update of acc (b on entry) from that row and the loaded neighbours
template <typename T, int NC>
__device__ __forceinline__ void rb0_apply_row(const long nb[6], const T K[6], T dg,
                                              const T xn[6][NC], T acc[NC]) {
#pragma unroll
    for (int f = 0; f < 6; f++) {
        T kf = K[f];
        if (kf == (T)0 || nb[f] < 0) continue;
#pragma unroll
        for (int m = 0; m < NC; m++) acc[m] += kf * xn[f][m];
    }
    T inv = (T)1 / dg;
#pragma unroll
    for (int m = 0; m < NC; m++) acc[m] = acc[m] * inv;
}

// k_smooth_rb with two cells per thread: half indices ih0 and ih0 + 1 (ih0 even) of one half
// row, natural cells a = (i_a, j, k) and b = (i_a + 2, j, k), which needs n_x a multiple of 4.
// The other colour's values come in 16-byte pairs: its pair (ih0, ih0 + 1) in the same row holds
// three of the four x neighbours (the fourth is a lone load, wrapped in the row when periodic),
// and the pair at ih0 in the neighbour row of each y and z face holds that face's neighbour of
// both cells.  The viscosities and flags come from colour-split copies (Level::etacs, flagcs)
// at the same slots, so they are pairs too.  Every load is unconditional (a missing
// neighbour loads the cell's own row or value, never used), so a thread waits once.  The first
// ncb blocks (a multiple of 8) take one cut cell per thread (those of colour col) through the
// one-cell path (smooth_rb_cell), which loads a cut cell's stored row; the blocks after them
// update the regular cells of their pairs from the loaded values and leave covered and cut cells
// alone.  Within a colour every update reads only the other colour, so the split changes
// nothing: the rows and updates are the one-cell kernel's, bit for bit.  The cut-cell blocks are
// dispatched first and spread over the XCDs by the hardware's round-robin, so their longer
// dependent loads neither trail the launch nor load the few XCDs whose slabs hold the body.
// Three components are the viscous system and one the Poisson system (the launch checks this
// against L.sys).  Four waves per SIMD (at most 128 VGPRs) keep enough loads in flight; blocks
// of one wave (PAIR_BLOCK) measured fastest on the 128^3 sphere (17.5 us against 17.7 and
// 17.9 us for 128 and 256 threads, alternated on one GPU).  PRO as in smooth_rb_cell: PRO_NONE,
// or PRO_ZERO (a cell that is not updated is set to 0; this half sweep writes every cell of its
// colour).  PRO_OWN stays with k_smooth_rb_pro: its rare non-updated regular cell needs the
// cell's own value and the coarse correction, which push this kernel past 128 VGPRs.
constexpr int PAIR_BLOCK = 64;
template <typename T, int NC, int PRO = PRO_NONE>
__global__ void __launch_bounds__(PAIR_BLOCK, 4)
    k_smooth_rb_pair(Rb0V L, const T* __restrict__ b, T* __restrict__ x, int col, unsigned ncb) {
    static_assert(PRO == PRO_NONE || PRO == PRO_ZERO, "no prolongation in the pair kernel");
    static_assert(sizeof(T) == 8, "pairs of FP64 values");
    constexpr bool VISC = NC == 3;
    if (L.gate && *L.gate) return;
    long N = L.N, Nh = N >> 1;
    if (blockIdx.x < ncb) {
        long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
        if (q >= L.ncut) return;
        long c = L.cut[q];
        int i, j, k;
        rb_coords(L, c, i, j, k);
        if (((i + j + k) & 1) != col) return;
        smooth_rb_cell<T, NC, PRO, T>(L, b, x, col, c >> 1, nullptr);
        return;
    }
    // the pair blocks, mapped to tiles per XCD as xcd_block does (ncb is a multiple of 8, so
    // block ncb + u runs on the XCD of u)
    unsigned npb = gridDim.x - ncb, u = blockIdx.x - ncb;
    unsigned tile = (u & 7) * (npb >> 3) + ((u & 7) < (npb & 7) ? (u & 7) : (npb & 7)) + (u >> 3);
    long p = tile * (long)blockDim.x + threadIdx.x;
    if (p >= (Nh >> 1)) return;
    const GridV& g = L.grid;
    unsigned t = 2u * (unsigned)p;
    unsigned row = fdiv(t, L.dnxh);
    int nxh = (int)L.dnxh.d;
    int ih0 = (int)(t - row * (unsigned)nxh);
    unsigned kq = fdiv(row, L.dny);
    int j = (int)(row - kq * L.dny.d), k = (int)kq;
    int s = (j + k + col) & 1;
    int ia = 2 * ih0 + s;
    long ca = cell_index(g, ia, j, k), cb = ca + 2;
    long nba[6], nbb[6];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            nba[2 * d + side] = cell_step(g, ca, ia, j, k, d, side);
            nbb[2 * d + side] = cell_step(g, cb, ia + 2, j, k, d, side);
        }
    const T* xo = x + (long)(1 - col) * Nh;
    long own = (long)col * Nh + t;
    // the first slots of the half rows holding the y and z neighbours (the natural row of a's
    // neighbour: the same row index in the other colour)
    long ry[2], rz[2];
#pragma unroll
    for (int side = 0; side < 2; side++) {
        long q = nba[2 + side] >= 0 ? nba[2 + side] : ca;
        ry[side] = (long)fdiv((unsigned)q, L.dnx) * nxh;
        q = nba[4 + side] >= 0 ? nba[4 + side] : ca;
        rz[side] = (long)fdiv((unsigned)q, L.dnx) * nxh;
    }
    long rx = (long)row * nxh;
    // the lone x neighbour: a's lower one (s = 0) or b's upper one (s = 1)
    long xe = s == 0 ? (ih0 > 0 ? ih0 - 1 : nxh - 1) : (ih0 + 2 < nxh ? ih0 + 2 : 0);
    T acca[NC], accb[NC], xa[6][NC], xb[6][NC];
#pragma unroll
    for (int m = 0; m < NC; m++) {
        double2 bv = *reinterpret_cast<const double2*>(b + m * N + own);
        acca[m] = bv.x;
        accb[m] = bv.y;
        double2 xc = *reinterpret_cast<const double2*>(xo + m * N + rx + ih0);
        T e = xo[m * N + rx + xe];
        xa[0][m] = s == 0 ? e : xc.x;
        xa[1][m] = s == 0 ? xc.x : xc.y;
        xb[0][m] = s == 0 ? xc.x : xc.y;
        xb[1][m] = s == 0 ? xc.y : e;
#pragma unroll
        for (int side = 0; side < 2; side++) {
            double2 yv = *reinterpret_cast<const double2*>(xo + m * N + ry[side] + ih0);
            double2 zv = *reinterpret_cast<const double2*>(xo + m * N + rz[side] + ih0);
            xa[2 + side][m] = yv.x;
            xb[2 + side][m] = yv.y;
            xa[4 + side][m] = zv.x;
            xb[4 + side][m] = zv.y;
        }
    }
    // the viscosities from the colour-split copy, at the same slots as the values: the two
    // cells' own pair, and the other colour's pairs and lone x neighbour
    T eca = (T)0, ecb = (T)0, ena[6], enb[6];
    if (VISC) {
        const T* eo = L.etacs + (long)(1 - col) * Nh;
        double2 ec2 = *reinterpret_cast<const double2*>(L.etacs + own);
        double2 ex2 = *reinterpret_cast<const double2*>(eo + rx + ih0);
        T ex = eo[rx + xe];
        eca = ec2.x;
        ecb = ec2.y;
        ena[0] = s == 0 ? ex : ex2.x;
        ena[1] = s == 0 ? ex2.x : ex2.y;
        enb[0] = s == 0 ? ex2.x : ex2.y;
        enb[1] = s == 0 ? ex2.y : ex;
#pragma unroll
        for (int side = 0; side < 2; side++) {
            double2 ey = *reinterpret_cast<const double2*>(eo + ry[side] + ih0);
            double2 ez = *reinterpret_cast<const double2*>(eo + rz[side] + ih0);
            ena[2 + side] = ey.x;
            enb[2 + side] = ey.y;
            ena[4 + side] = ez.x;
            enb[4 + side] = ez.y;
        }
    } else {
#pragma unroll
        for (int f = 0; f < 6; f++) ena[f] = enb[f] = (T)0;
    }
    uchar2 fl2 = *reinterpret_cast<const uchar2*>(L.flagcs + own);
    uint8_t fla = fl2.x, flb = fl2.y;
    // the rows of regular cells from the loaded viscosities (those of covered and cut cells are
    // formed but never stored)
    T Ka[6], Kb[6];
    T da = rb0_regular_row<T, VISC>(L, nba, eca, ena, Ka);
    T db = rb0_regular_row<T, VISC>(L, nbb, ecb, enb, Kb);
    rb0_apply_row<T, NC>(nba, Ka, da, xa, acca);
    rb0_apply_row<T, NC>(nbb, Kb, db, xb, accb);
    bool ua = fla == 2 && da > (T)0, ub = flb == 2 && db > (T)0;
    if (PRO == PRO_ZERO) {
        // every cell that is not cut is written: its update, or 0
        bool wa = fla != 1, wb = flb != 1;
#pragma unroll
        for (int m = 0; m < NC; m++) {
            acca[m] = ua ? acca[m] : (T)0;
            accb[m] = ub ? accb[m] : (T)0;
        }
        if (wa && wb) {
#pragma unroll
            for (int m = 0; m < NC; m++) {
                double2 o;
                o.x = acca[m];
                o.y = accb[m];
                *reinterpret_cast<double2*>(x + m * N + own) = o;
            }
        } else {
#pragma unroll
            for (int m = 0; m < NC; m++) {
                if (wa) x[m * N + own] = acca[m];
                if (wb) x[m * N + own + 1] = accb[m];
            }
        }
        return;
    }
    if (ua && ub) {
#pragma unroll
        for (int m = 0; m < NC; m++) {
            double2 o;
            o.x = acca[m];
            o.y = accb[m];
            *reinterpret_cast<double2*>(x + m * N + own) = o;
        }
    } else {
        // a regular cell whose diagonal is not positive is not updated (as in smooth_rb_cell)
#pragma unroll
        for (int m = 0; m < NC; m++) {
            if (ua) x[m * N + own] = acca[m];
            if (ub) x[m * N + own + 1] = accb[m];
        }
    }
}

// rb0_regular_row and rb0_apply_row with the neighbour test given as in[f] (bit for bit the
// same arithmetic)
template <typename T, bool VISC>
__device__ __forceinline__ T rb0_regular_row_in(const Rb0V& L, const bool in[6], T ec,
                                                const T en[6], T K[6]) {
    T kin = (T)L.kin, kwall = (T)L.kwall, kp = (T)L.kpois;
    T sd = VISC ? (T)L.rho : (T)0;
#pragma unroll
    for (int f = 0; f < 6; f++) {
        T kf;
        if (VISC) kf = in[f] ? kin * (ec + en[f]) : kwall * ec;
        else kf = in[f] ? kp : (T)0;
        sd += kf;
        K[f] = kf;
    }
    return sd;
}
template <typename T, int NC>
__device__ __forceinline__ void rb0_apply_row_in(const bool in[6], const T K[6], T dg,
                                                 const T xn[6][NC], T acc[NC]) {
#pragma unroll
    for (int f = 0; f < 6; f++) {
        T kf = K[f];
        if (kf == (T)0 || !in[f]) continue;
#pragma unroll
        for (int m = 0; m < NC; m++) acc[m] += kf * xn[f][m];
    }
    T inv = (T)1 / dg;
#pragma unroll
    for (int m = 0; m < NC; m++) acc[m] = acc[m] * inv;
}

// The FP32 counterpart of k_smooth_rb_pair: four cells of colour col per thread, half indices
// ih0 .. ih0 + 3 (ih0 a multiple of 4) of one half row, natural cells i_a + 2q (q = 0..3), which
// needs n_x a multiple of 8.  The other colour's values come in 16-byte quads: its quad
// (ih0 .. ih0 + 3) in the same row holds seven of the eight x neighbours (the eighth is a lone
// load, wrapped in the row when periodic), and the quad at ih0 in the neighbour row of each y and
// z face holds that face's neighbour of the four cells; the viscosities (FP32, the values of
// Level::etaf) and flags come from the colour-split copies at the same slots.  The four cells
// share their y and z neighbours' existence; only cell 0's lower and cell 3's upper x face can
// meet a wall.  Cut cells, covered cells, PRO and the launch as in k_smooth_rb_pair; the rows and
// updates are the one-cell FP32 kernel's, bit for bit.
template <int NC, int PRO = PRO_NONE>
__global__ void __launch_bounds__(PAIR_BLOCK, 4)
    k_smooth_rb_quad(Rb0V L, const float* __restrict__ b, float* __restrict__ x, int col,
                     unsigned ncb) {
    static_assert(PRO == PRO_NONE || PRO == PRO_ZERO, "no prolongation in the quad kernel");
    using T = float;
    constexpr bool VISC = NC == 3;
    if (L.gate && *L.gate) return;
    long N = L.N, Nh = N >> 1;
    if (blockIdx.x < ncb) {
        long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
        if (q >= L.ncut) return;
        long c = L.cut[q];
        int i, j, k;
        rb_coords(L, c, i, j, k);
        if (((i + j + k) & 1) != col) return;
        smooth_rb_cell<T, NC, PRO, T>(L, b, x, col, c >> 1, nullptr);
        return;
    }
    unsigned npb = gridDim.x - ncb, u = blockIdx.x - ncb;
    unsigned tile = (u & 7) * (npb >> 3) + ((u & 7) < (npb & 7) ? (u & 7) : (npb & 7)) + (u >> 3);
    long p = tile * (long)blockDim.x + threadIdx.x;
    if (p >= (Nh >> 2)) return;
    const GridV& g = L.grid;
    unsigned t = 4u * (unsigned)p;
    unsigned row = fdiv(t, L.dnxh);
    int nxh = (int)L.dnxh.d;
    int ih0 = (int)(t - row * (unsigned)nxh);
    unsigned kq = fdiv(row, L.dny);
    int j = (int)(row - kq * L.dny.d), k = (int)kq;
    int s = (j + k + col) & 1;
    int ia = 2 * ih0 + s;
    long c0 = cell_index(g, ia, j, k);
    // which faces have a neighbour: y and z from cell 0 (the same for all four), x at the ends
    long nyz[4];
#pragma unroll
    for (int side = 0; side < 2; side++) {
        nyz[side] = cell_step(g, c0, ia, j, k, 1, side);
        nyz[2 + side] = cell_step(g, c0, ia, j, k, 2, side);
    }
    bool in[4][6];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        in[q][0] = (q > 0 || ia > 0) || g.per[0];
        in[q][1] = (q < 3 || ia + 6 < g.n[0] - 1) || g.per[0];
#pragma unroll
        for (int f = 2; f < 6; f++) in[q][f] = nyz[f - 2] >= 0;
    }
    const T* xo = x + (long)(1 - col) * Nh;
    long own = (long)col * Nh + t;
    long ry[2], rz[2];
#pragma unroll
    for (int side = 0; side < 2; side++) {
        long q = nyz[side] >= 0 ? nyz[side] : c0;
        ry[side] = (long)fdiv((unsigned)q, L.dnx) * nxh;
        q = nyz[2 + side] >= 0 ? nyz[2 + side] : c0;
        rz[side] = (long)fdiv((unsigned)q, L.dnx) * nxh;
    }
    long rx = (long)row * nxh;
    // the lone x neighbour: cell 0's lower one (s = 0) or cell 3's upper one (s = 1)
    long xe = s == 0 ? (ih0 > 0 ? ih0 - 1 : nxh - 1) : (ih0 + 4 < nxh ? ih0 + 4 : 0);
    T acc[4][NC], xn[4][6][NC];
#pragma unroll
    for (int m = 0; m < NC; m++) {
        float4 bv = *reinterpret_cast<const float4*>(b + m * N + own);
        acc[0][m] = bv.x;
        acc[1][m] = bv.y;
        acc[2][m] = bv.z;
        acc[3][m] = bv.w;
        float4 xc = *reinterpret_cast<const float4*>(xo + m * N + rx + ih0);
        T e = xo[m * N + rx + xe];
        T v[4] = {xc.x, xc.y, xc.z, xc.w};
#pragma unroll
        for (int q = 0; q < 4; q++) {
            xn[q][0][m] = s == 0 ? (q == 0 ? e : v[q > 0 ? q - 1 : 0]) : v[q];
            xn[q][1][m] = s == 0 ? v[q] : (q == 3 ? e : v[q < 3 ? q + 1 : 3]);
        }
#pragma unroll
        for (int side = 0; side < 2; side++) {
            float4 yv = *reinterpret_cast<const float4*>(xo + m * N + ry[side] + ih0);
            float4 zv = *reinterpret_cast<const float4*>(xo + m * N + rz[side] + ih0);
            xn[0][2 + side][m] = yv.x;
            xn[1][2 + side][m] = yv.y;
            xn[2][2 + side][m] = yv.z;
            xn[3][2 + side][m] = yv.w;
            xn[0][4 + side][m] = zv.x;
            xn[1][4 + side][m] = zv.y;
            xn[2][4 + side][m] = zv.z;
            xn[3][4 + side][m] = zv.w;
        }
    }
    T ec[4], en[4][6];
    if (VISC) {
        const T* eo = L.etafcs + (long)(1 - col) * Nh;
        float4 e4 = *reinterpret_cast<const float4*>(L.etafcs + own);
        float4 ex4 = *reinterpret_cast<const float4*>(eo + rx + ih0);
        T ex = eo[rx + xe];
        ec[0] = e4.x;
        ec[1] = e4.y;
        ec[2] = e4.z;
        ec[3] = e4.w;
        T v[4] = {ex4.x, ex4.y, ex4.z, ex4.w};
#pragma unroll
        for (int q = 0; q < 4; q++) {
            en[q][0] = s == 0 ? (q == 0 ? ex : v[q > 0 ? q - 1 : 0]) : v[q];
            en[q][1] = s == 0 ? v[q] : (q == 3 ? ex : v[q < 3 ? q + 1 : 3]);
        }
#pragma unroll
        for (int side = 0; side < 2; side++) {
            float4 ey = *reinterpret_cast<const float4*>(eo + ry[side] + ih0);
            float4 ez = *reinterpret_cast<const float4*>(eo + rz[side] + ih0);
            en[0][2 + side] = ey.x;
            en[1][2 + side] = ey.y;
            en[2][2 + side] = ey.z;
            en[3][2 + side] = ey.w;
            en[0][4 + side] = ez.x;
            en[1][4 + side] = ez.y;
            en[2][4 + side] = ez.z;
            en[3][4 + side] = ez.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            ec[q] = (T)0;
#pragma unroll
            for (int f = 0; f < 6; f++) en[q][f] = (T)0;
        }
    }
    unsigned fl4 = *reinterpret_cast<const unsigned*>(L.flagcs + own);
    bool upd[4], wr[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        unsigned fl = (fl4 >> (8 * q)) & 0xffu;
        T K[6];
        T dg = rb0_regular_row_in<T, VISC>(L, in[q], ec[q], en[q], K);
        rb0_apply_row_in<T, NC>(in[q], K, dg, xn[q], acc[q]);
        upd[q] = fl == 2 && dg > (T)0;
        // PRO_ZERO: every cell that is not cut is written (its update, or 0)
        wr[q] = PRO == PRO_ZERO ? fl != 1 : upd[q];
        if (PRO == PRO_ZERO && !upd[q]) {
#pragma unroll
            for (int m = 0; m < NC; m++) acc[q][m] = (T)0;
        }
    }
    if (wr[0] && wr[1] && wr[2] && wr[3]) {
#pragma unroll
        for (int m = 0; m < NC; m++)
            *reinterpret_cast<float4*>(x + m * N + own) =
                make_float4(acc[0][m], acc[1][m], acc[2][m], acc[3][m]);
    } else {
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int m = 0; m < NC; m++)
                if (wr[q]) x[m * N + own + q] = acc[q][m];
    }
}

// y = M x of the Poisson system (one component) on level 0, two neighbouring natural cells
// a = (i, j, k), b = (i + 1, j, k), i even, per thread: a's upper and b's lower x neighbour are
// each other, the outer x neighbours are lone loads, and each y and z face's neighbours of both
// cells are one aligned pair, as are the two cells' own values and flags.  The first ncb blocks
// (a multiple of 8) take one cut cell per thread through k_apply0's row (the stored one);
// covered cells get 0.  Each y is k_apply0's bit for bit.
__global__ void __launch_bounds__(PAIR_BLOCK)
    k_apply0_pair(Rb0V L, const double* __restrict__ x, double* __restrict__ y, unsigned ncb) {
    if (L.gate && *L.gate) return;
    long N = L.N;
    const GridV& g = L.grid;
    if (blockIdx.x < ncb) {
        long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
        if (q >= L.ncut) return;
        long c = L.cut[q];
        int i, j, k;
        rb_coords(L, c, i, j, k);
        long nb[6];
#pragma unroll
        for (int d = 0; d < 3; d++)
#pragma unroll
            for (int side = 0; side < 2; side++) nb[2 * d + side] = cell_step(g, c, i, j, k, d, side);
        double xv = x[c], xn[6][1];
#pragma unroll
        for (int f = 0; f < 6; f++) xn[f][0] = nb[f] >= 0 ? x[nb[f]] : 0.0;
        double K[6], dg, unused[6][1];
        rb0_row_ld<double, 1, false>(L, c, i, j, k, x, K, nb, dg, unused);
        double acc = 0.0;
#pragma unroll
        for (int f = 0; f < 6; f++) {
            if (K[f] == 0.0 || nb[f] < 0) continue;
            acc += K[f] * xn[f][0];
        }
        y[c] = dg * xv - acc;
        return;
    }
    unsigned npb = gridDim.x - ncb, u = blockIdx.x - ncb;
    unsigned tile = (u & 7) * (npb >> 3) + ((u & 7) < (npb & 7) ? (u & 7) : (npb & 7)) + (u >> 3);
    long p = tile * (long)blockDim.x + threadIdx.x;
    if (p >= (N >> 1)) return;
    long ca = 2 * p;
    int i, j, k;
    rb_coords(L, ca, i, j, k);
    long nba[6], nbb[6];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            nba[2 * d + side] = cell_step(g, ca, i, j, k, d, side);
            nbb[2 * d + side] = cell_step(g, ca + 1, i + 1, j, k, d, side);
        }
    uchar2 fl2 = *reinterpret_cast<const uchar2*>(L.flag + ca);
    double2 xo = *reinterpret_cast<const double2*>(x + ca);
    double xla = x[nba[0] >= 0 ? nba[0] : ca], xlb = x[nbb[1] >= 0 ? nbb[1] : ca + 1];
    double xa[6][1], xb[6][1];
    xa[0][0] = xla;
    xa[1][0] = xo.y;
    xb[0][0] = xo.x;
    xb[1][0] = xlb;
#pragma unroll
    for (int side = 0; side < 2; side++) {
        long qy = nba[2 + side] >= 0 ? nba[2 + side] : ca;
        long qz = nba[4 + side] >= 0 ? nba[4 + side] : ca;
        double2 y2 = *reinterpret_cast<const double2*>(x + qy);
        double2 z2 = *reinterpret_cast<const double2*>(x + qz);
        xa[2 + side][0] = y2.x;
        xb[2 + side][0] = y2.y;
        xa[4 + side][0] = z2.x;
        xb[4 + side][0] = z2.y;
    }
    double en[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, Ka[6], Kb[6];
    double da = rb0_regular_row<double, false>(L, nba, 0.0, en, Ka);
    double db = rb0_regular_row<double, false>(L, nbb, 0.0, en, Kb);
    double acca = 0.0, accb = 0.0;
#pragma unroll
    for (int f = 0; f < 6; f++) {
        if (!(Ka[f] == 0.0 || nba[f] < 0)) acca += Ka[f] * xa[f][0];
        if (!(Kb[f] == 0.0 || nbb[f] < 0)) accb += Kb[f] * xb[f][0];
    }
    double ya = fl2.x == 0 ? 0.0 : da * xo.x - acca;
    double yb = fl2.y == 0 ? 0.0 : db * xo.y - accb;
    if (fl2.x != 1 && fl2.y != 1) {
        double2 o;
        o.x = ya;
        o.y = yb;
        *reinterpret_cast<double2*>(y + ca) = o;
    } else {
        if (fl2.x != 1) y[ca] = ya;
        if (fl2.y != 1) y[ca + 1] = yb;
    }
}

template <typename T, typename TC, int NC, int PRO>
__global__ void __launch_bounds__(EB_BLOCK)
    k_smooth_rb_pro(Rb0V L, const T* __restrict__ b, T* __restrict__ x, int col, ProV<TC> P) {
    if (L.gate && *L.gate) return;
    long t = xcd_block() * (long)blockDim.x + threadIdx.x;
    if (t >= (L.N >> 1)) return;
    smooth_rb_cell<T, NC, PRO, TC>(L, b, x, col, t, &P);
}

// k_smooth_first_rb fused with the conversion of the right-hand side: reads b in natural
// order (FP64), stores its colour-split copy (precision T) and the first iterate's colour 0;
// colour 1 is left to the colour-1 half sweep that follows (PRO_ZERO: it writes every cell).
// Thread t takes slot t of both colours: the natural cells 2t and 2t + 1 (one of each colour,
// n_x being even), read as one 16-byte pair, so a wave reads whole natural lines once.
template <typename T, int NC>
__global__ void k_smooth_first_rb_from(Rb0V L, const double* __restrict__ bnat,
                                       T* __restrict__ b, T* __restrict__ x) {
    if (L.gate && *L.gate) return;
    long N = L.N, Nh = N >> 1;
    long t = xcd_block() * (long)blockDim.x + threadIdx.x;
    if (t >= Nh) return;
    int i, j, k;
    rb_cell(L, (unsigned)t, 0, i, j, k);
    long c = cell_index(L.grid, i, j, k);  // the colour-0 cell: 2t or 2t + 1
    bool odd = (c & 1) != 0;
    T b0[NC], b1[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) {
        double2 q = *reinterpret_cast<const double2*>(bnat + m * N + 2 * t);
        b0[m] = (T)(odd ? q.y : q.x);
        b1[m] = (T)(odd ? q.x : q.y);
    }
    T K[6], xn[6][NC], Dd = (T)1;
    long nb[6];
    bool upd = rb0_row_ld<T, NC, false>(L, c, i, j, k, x, K, nb, Dd, xn);
    T inv = upd ? (T)1 / Dd : (T)0;
#pragma unroll
    for (int m = 0; m < NC; m++) {
        b[m * N + t] = b0[m];
        b[m * N + Nh + t] = b1[m];
        x[m * N + t] = upd ? b0[m] * inv : (T)0;
    }
}

// the last half sweep (colour 0) fused with the conversion of the iterate back to natural
// order (FP64, or FP32 from an FP32 level, which loses nothing): a thread updates its colour-0
// cell and also copies the colour-1 cell next to it in x, so every cell of the natural output is
// written once
template <typename T, int NC, int PRO = PRO_NONE, typename TC = T, typename TD = double>
__global__ void k_smooth_last_rb_to(Rb0V L, const T* __restrict__ b, const T* __restrict__ x,
                                    TD* __restrict__ xnat, ProV<TC> P) {
    if (L.gate && *L.gate) return;
    long N = L.N, Nh = N >> 1;
    long t = xcd_block() * (long)blockDim.x + threadIdx.x;
    if (t >= Nh) return;
    int i, j, k;
    rb_cell(L, (unsigned)t, 0, i, j, k);
    long c = cell_index(L.grid, i, j, k);
    long c1 = cell_index(L.grid, i ^ 1, j, k);
    T val[NC], bv[NC], x1[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) {
        val[m] = x[m * N + t];
        bv[m] = b[m * N + t];
        x1[m] = x[m * N + Nh + (c1 >> 1)];
    }
    T K[6], dg, xn[6][NC];
    long nb[6];
    bool upd = rb0_row_ld<T, NC, true>(L, c, i, j, k, x + Nh, K, nb, dg, xn);
    if (upd) {
#pragma unroll
        for (int m = 0; m < NC; m++) val[m] = bv[m];
#pragma unroll
        for (int f = 0; f < 6; f++) {
            T kf = K[f];
            if (kf == (T)0 || nb[f] < 0) continue;
#pragma unroll
            for (int m = 0; m < NC; m++) val[m] += kf * xn[f][m];
        }
        T inv = (T)1 / dg;
#pragma unroll
        for (int m = 0; m < NC; m++) val[m] = val[m] * inv;
    } else if (PRO != PRO_NONE && L.flag[c] != 0) {
        long Nc = (long)P.gc.n[0] * P.gc.n[1] * P.gc.n[2];
        long pc = cell_index(P.gc, i >> 1, j >> 1, k >> 1);
#pragma unroll
        for (int m = 0; m < NC; m++) val[m] += (T)P.ec[m * Nc + pc];
    }
#pragma unroll
    for (int m = 0; m < NC; m++) {
        xnat[m * N + c] = (TD)val[m];
        xnat[m * N + c1] = (TD)x1[m];
    }
}

// residual of level 0 restricted to the coarse right-hand side (natural storage there), with
// the thread layout and summation order of k_resid_restrict
template <typename TF, typename TC, int NC>
__global__ void __launch_bounds__(RR_THREADS)
    k_resid_restrict_rb(Rb0V L, const TF* __restrict__ b, const TF* __restrict__ x, GridV gc,
                        const uint8_t* __restrict__ mc, TC* __restrict__ bc, FirstV<TC> F1) {
    if (L.gate && *L.gate) return;
    __shared__ TF rs[RR_THREADS * NC];
    long N = L.N;
    long Nc = (long)gc.n[0] * gc.n[1] * gc.n[2];
    int a, cl, bq, cq;
    rr_child(threadIdx.x, a, cl, bq, cq);
    unsigned blk = xcd_block();
    long c = (long)blk * RR_COARSE + cl;
    TF r[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) r[m] = (TF)0;
    if (c < Nc) {
        int ci, cj, ck;
        cell_coords(gc, c, ci, cj, ck);
        int fi = 2 * ci + a, fj = 2 * cj + bq, fk = 2 * ck + cq;
        long f = cell_index(L.grid, fi, fj, fk);
        long oth = (long)(1 - ((fi + fj + fk) & 1)) * (N >> 1);
        long qf = rb_slot(N, fi, fj, fk, f);
        TF bv[NC], xv[NC];
#pragma unroll
        for (int m = 0; m < NC; m++) {
            bv[m] = b[m * N + qf];
            xv[m] = x[m * N + qf];
        }
        TF K[6], dg, xn[6][NC];
        long nb[6];
        bool open = L.flag[f] != 0;
        rb0_row_ld<TF, NC, true>(L, f, fi, fj, fk, x + oth, K, nb, dg, xn);
        if (open) {
            TF acc[NC];
#pragma unroll
            for (int m = 0; m < NC; m++) acc[m] = (TF)0;
#pragma unroll
            for (int e = 0; e < 6; e++) {
                TF kf = K[e];
                if (kf == (TF)0 || nb[e] < 0) continue;
#pragma unroll
                for (int m = 0; m < NC; m++) acc[m] += kf * xn[e][m];
            }
#pragma unroll
            for (int m = 0; m < NC; m++) r[m] = bv[m] - (dg * xv[m] - acc[m]);
        }
    }
#pragma unroll
    for (int m = 0; m < NC; m++) rs[threadIdx.x * NC + m] = r[m];
    __syncthreads();
    if (threadIdx.x < RR_COARSE) {
        long cc = (long)blk * RR_COARSE + threadIdx.x;
        if (cc >= Nc) return;
        TF sum[NC];
#pragma unroll
        for (int m = 0; m < NC; m++) sum[m] = (TF)0;
        for (int q = 0; q < 8; q++) {
            int t = rr_thread(threadIdx.x, q);
#pragma unroll
            for (int m = 0; m < NC; m++) sum[m] += rs[t * NC + m];
        }
        rr_store<TF, TC, NC>(gc, Nc, cc, mc, sum, bc, F1);
    }
}

// residual b - M x of level-0 cell (fi, fj, fk) (0 on a covered cell), every load first
template <typename TF, int NC>
__device__ __forceinline__ void rb_resid(const Rb0V& L, const TF* __restrict__ b,
                                         const TF* __restrict__ x, int fi, int fj, int fk,
                                         TF r[NC]) {
    long N = L.N;
    long f = cell_index(L.grid, fi, fj, fk);
    long oth = (long)(1 - ((fi + fj + fk) & 1)) * (N >> 1);
    long qf = rb_slot(N, fi, fj, fk, f);
    TF bv[NC], xv[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) {
        bv[m] = b[m * N + qf];
        xv[m] = x[m * N + qf];
    }
    TF K[6], dg, xn[6][NC];
    long nb[6];
    bool open = L.flag[f] != 0;
    rb0_row_ld<TF, NC, true>(L, f, fi, fj, fk, x + oth, K, nb, dg, xn);
#pragma unroll
    for (int m = 0; m < NC; m++) r[m] = (TF)0;
    if (!open) return;
    TF acc[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) acc[m] = (TF)0;
#pragma unroll
    for (int e = 0; e < 6; e++) {
        TF kf = K[e];
        if (kf == (TF)0 || nb[e] < 0) continue;
#pragma unroll
        for (int m = 0; m < NC; m++) acc[m] += kf * xn[e][m];
    }
#pragma unroll
    for (int m = 0; m < NC; m++) r[m] = bv[m] - (dg * xv[m] - acc[m]);
}

// k_resid_restrict_rb after a pre-smoothing that ended with a colour-1 half sweep: the residual
// of every colour-1 cell that sweep updated is zero in exact arithmetic (its row was just
// solved with the current colour-0 neighbours), so it is taken as 0 and only colour-0 cells,
// and colour-1 cells the sweep skipped, are evaluated.  A block handles RR_COARSE coarse cells
// with one thread per colour-0 child (x fastest: the colour-0 children of consecutive coarse
// cells are consecutive in the colour-split order); the thread also owns the colour-1 child
// next to it in x.  The eight children are summed in the order q = 0..7 as before.
constexpr int RR0_THREADS = 4 * RR_COARSE;
template <typename TF, typename TC, int NC>
__global__ void __launch_bounds__(RR0_THREADS)
    k_resid_restrict_rb0(Rb0V L, const TF* __restrict__ b, const TF* __restrict__ x, GridV gc,
                         const uint8_t* __restrict__ mc, TC* __restrict__ bc, FirstV<TC> F1) {
    if (L.gate && *L.gate) return;
    __shared__ TF rs[RR_COARSE * 8 * NC];
    long Nc = (long)gc.n[0] * gc.n[1] * gc.n[2];
    int cl = threadIdx.x & (RR_COARSE - 1);
    int bq = (threadIdx.x / RR_COARSE) & 1, cq = threadIdx.x / (2 * RR_COARSE);
    int a0 = (bq + cq) & 1;  // x bit of the colour-0 child in row (bq, cq)
    unsigned blk = xcd_block();
    long c = (long)blk * RR_COARSE + cl;
    TF r0[NC], r1[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) {
        r0[m] = (TF)0;
        r1[m] = (TF)0;
    }
    if (c < Nc) {
        int ci, cj, ck;
        cell_coords(gc, c, ci, cj, ck);
        int fj = 2 * cj + bq, fk = 2 * ck + cq;
        int f0i = 2 * ci + a0, f1i = 2 * ci + (1 - a0);
        uint8_t fl1 = L.flag[cell_index(L.grid, f1i, fj, fk)];
        rb_resid<TF, NC>(L, b, x, f0i, fj, fk, r0);
        // a cut colour-1 child: the sweep may have skipped it, so evaluate it
        if (fl1 == 1) rb_resid<TF, NC>(L, b, x, f1i, fj, fk, r1);
    }
    int q0 = a0 + 2 * bq + 4 * cq, q1 = (1 - a0) + 2 * bq + 4 * cq;
#pragma unroll
    for (int m = 0; m < NC; m++) {
        rs[(cl * 8 + q0) * NC + m] = r0[m];
        rs[(cl * 8 + q1) * NC + m] = r1[m];
    }
    __syncthreads();
    if (threadIdx.x < RR_COARSE) {
        long cc = (long)blk * RR_COARSE + threadIdx.x;
        if (cc >= Nc) return;
        TF sum[NC];
#pragma unroll
        for (int m = 0; m < NC; m++) sum[m] = (TF)0;
        for (int q = 0; q < 8; q++)
#pragma unroll
            for (int m = 0; m < NC; m++) sum[m] += rs[(threadIdx.x * 8 + q) * NC + m];
        rr_store<TF, TC, NC>(gc, Nc, cc, mc, sum, bc, F1);
    }
}

// piecewise-constant prolongation onto the open cells of level 0 (colour-split storage)
template <typename TC, typename TF, int NC>
__global__ void k_prolong_rb(Rb0V L, GridV gc, const TC* __restrict__ ec, TF* __restrict__ x) {
    if (L.gate && *L.gate) return;
    long N = L.N, Nh = N >> 1;
    long Nc = (long)gc.n[0] * gc.n[1] * gc.n[2];
    long v = xcd_block() * (long)blockDim.x + threadIdx.x;
    if (v >= N) return;
    int col = (int)(v & 1);  // threads 2t, 2t + 1: slot t of colours 0 and 1
    long u = (long)col * Nh + (v >> 1);
    int i, j, k;
    rb_cell(L, (unsigned)(v >> 1), col, i, j, k);
    long f = cell_index(L.grid, i, j, k);
    if (L.flag[f] == 0) return;
    long c = cell_index(gc, i >> 1, j >> 1, k >> 1);
#pragma unroll
    for (int m = 0; m < NC; m++) x[m * N + u] += (TF)ec[m * Nc + c];
}

// natural -> colour-split (with a precision change)
template <typename TS, typename TD, int NC>
__global__ void k_to_rb(GridV g, long N, const TS* __restrict__ a, TD* __restrict__ r,
                        const int* gate) {
    if (gate && *gate) return;
    long Nh = N >> 1;
    long v = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (v >= N) return;
    int col = (int)(v & 1);  // threads 2t, 2t + 1: slot t of colours 0 and 1 (whole natural lines)
    long u = (long)col * Nh + (v >> 1);
    int i, j, k;
    rb_cell(g, (unsigned)(v >> 1), col, i, j, k);
    long c = cell_index(g, i, j, k);
#pragma unroll
    for (int m = 0; m < NC; m++) r[m * N + u] = (TD)a[m * N + c];
}

// colour-split -> natural (with a precision change)
template <typename TS, typename TD, int NC>
__global__ void k_from_rb(GridV g, long N, const TS* __restrict__ r, TD* __restrict__ a,
                          const int* gate) {
    if (gate && *gate) return;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    int i, j, k;
    cell_coords(g, c, i, j, k);
    long u = rb_slot(N, i, j, k, c);
#pragma unroll
    for (int m = 0; m < NC; m++) a[m * N + c] = (TD)r[m * N + u];
}

// ------------------------------------------------------------------------------------------
// the small coarse levels of a V-cycle, all in one work-group (one launch instead of ~100):
// the same operations in the same order as the per-level kernels, separated by barriers.  The
// operators, right-hand sides and iterates of these levels are staged in LDS, so each of the
// ~100 barrier-separated phases costs LDS latency instead of a global-memory round trip.
// ------------------------------------------------------------------------------------------
constexpr int TAIL_MAXL = 8;
constexpr int TAIL_THREADS = 256;
static_assert(TAIL_THREADS >= 3 * 64, "the in-wave levels need one wavefront per component");
constexpr size_t TAIL_LDS_BYTES = MG_PACK_BYTES;

struct TailArgs {
    int nl, nu1, nu2, nbottom;
    LevelV<double> L[TAIL_MAXL];
    double* x0;        // iterate of the first tail level (global, written back)
    const int* gate;
    const double* b0;  // right-hand side of the first tail level (global)
    // LDS byte offsets per level: x, b, K[3], D, mask; and the first level's residual.  The
    // operator arrays (K, D, mask of every tail level) come first, in [0, nstatic), and are
    // staged from pack, a copy with exactly that layout made when the operator is built
    unsigned ox[TAIL_MAXL], ob[TAIL_MAXL], oK[TAIL_MAXL][3], oD[TAIL_MAXL], om[TAIL_MAXL];
    unsigned orr;
    unsigned nstatic;
    const char* pack;
};

// residual b - M x at fine cell f (0 outside the open cells)
template <int NC>
__device__ __forceinline__ void resid_value(const LevelV<double>& L, const double* b,
                                            const double* x, long f, double r[NC]) {
    if (!L.mask[f]) {
#pragma unroll
        for (int m = 0; m < NC; m++) r[m] = 0.0;
        return;
    }
    int i, j, k;
    cell_coords(L.grid, f, i, j, k);
    double acc[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) acc[m] = 0.0;
    offdiag<double, NC>(L, x, i, j, k, acc);
#pragma unroll
    for (int m = 0; m < NC; m++) r[m] = b[m * L.N + f] - (L.D[f] * x[m * L.N + f] - acc[m]);
}

template <int NC>
__device__ void tail_sweep(const LevelV<double>& L, const double* b, double* x, int col) {
    for (long t = threadIdx.x; t < L.N / 2; t += blockDim.x) smooth_cell<double, NC>(L, b, x, t, col);
    __syncthreads();
}

// ---- levels of at most one wavefront of cells, run by wave 0 alone: lane = cell, the other
// ---- colour's values come through cross-lane shuffles, so no barrier is needed
constexpr int WAVE_MAXL = 3;

struct WaveRow {
    double K[6];
    int nb[6];     // neighbour lane (cell index), -1 where there is none
    double D;
    bool open;
    int colour;
};

__device__ __forceinline__ void wave_row(const LevelV<double>& L, int lane, WaveRow& r) {
#pragma unroll
    for (int f = 0; f < 6; f++) {
        r.K[f] = 0.0;
        r.nb[f] = -1;
    }
    r.D = 0.0;
    r.open = false;
    r.colour = 0;
    if (lane >= L.N) return;
    int i, j, k;
    cell_coords(L.grid, lane, i, j, k);
    r.colour = (i + j + k) & 1;
    r.open = L.mask[lane] != 0;
    r.D = L.D[lane];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            int f[3] = {i, j, k};
            f[d] += side;
            r.K[2 * d + side] = L.K[d][face_index(L.grid, d, f[0], f[1], f[2])];
            int q[3] = {i, j, k};
            q[d] += side ? 1 : -1;
            r.nb[2 * d + side] = (int)cell_at(L.grid, q[0], q[1], q[2]);
        }
}

// acc = sum_f K_f x_nb(f) in face order (faces with K = 0 or no neighbour skipped)
template <int NC>
__device__ __forceinline__ void wave_offdiag(const WaveRow& r, int lane, const double x[NC],
                                             double acc[NC]) {
#pragma unroll
    for (int f = 0; f < 6; f++) {
        int src = r.nb[f] >= 0 ? r.nb[f] : lane;
        bool use = r.K[f] != 0.0 && r.nb[f] >= 0;
#pragma unroll
        for (int m = 0; m < NC; m++) {
            double v = __shfl(x[m], src, 64);
            if (use) acc[m] += r.K[f] * v;
        }
    }
}

template <int NC>
__device__ __forceinline__ void wave_sweep(const WaveRow& r, int lane, const double b[NC],
                                           double x[NC], int col) {
    double acc[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) acc[m] = b[m];
    wave_offdiag<NC>(r, lane, x, acc);
    bool upd = r.open && r.colour == col && r.D > 0.0;
#pragma unroll
    for (int m = 0; m < NC; m++)
        if (upd) x[m] = acc[m] / r.D;
}

// The coarsest solve (nbottom red-black pairs, then nbottom black-red pairs) on a 2 x 2 x 2
// level.  There both faces of a direction d couple cell c to the same cell, c ^ (1 << d) (or
// one face is a wall), so with lane L = c + 8 m holding component m of cell c (the
// preconditioner's components are uncoupled) a half sweep needs three cross-lane exchanges,
// L ^ 1, L ^ 2 and L ^ 4, instead of one per face and component.  Every update is wave_sweep's
// (b plus the K x terms in face order, then / D), so the result is bit for bit the same.  On
// entry lane c < 8 holds b[m] and x[m] of cell c (its row in r), and on return x[m] again.
template <int NC>
__device__ __forceinline__ void bottom_cube2(const WaveRow& r, int lane, const double b[NC],
                                             double x[NC], int nbottom) {
    int c = lane & 7, m = lane >> 3;
    double K[6];
    bool use[6];
#pragma unroll
    for (int f = 0; f < 6; f++) {
        K[f] = __shfl(r.K[f], c, 64);
        int nbf = __shfl(r.nb[f], c, 64);
        use[f] = K[f] != 0.0 && nbf >= 0;
    }
    double D = __shfl(r.D, c, 64);
    bool open = __shfl(r.open ? 1 : 0, c, 64) != 0;
    int colour = __shfl(r.colour, c, 64);
    double bb = 0.0, xx = 0.0;
#pragma unroll
    for (int q = 0; q < NC; q++) {
        double tb = __shfl(b[q], c, 64), tx = __shfl(x[q], c, 64);
        if (m == q) {
            bb = tb;
            xx = tx;
        }
    }
    bool upd0 = open && colour == 0 && D > 0.0, upd1 = open && colour == 1 && D > 0.0;
    auto half = [&](bool upd) {
        double v[3];
        v[0] = __shfl_xor(xx, 1, 64);
        v[1] = __shfl_xor(xx, 2, 64);
        v[2] = __shfl_xor(xx, 4, 64);
        double acc = bb;
#pragma unroll
        for (int f = 0; f < 6; f++)
            if (use[f]) acc += K[f] * v[f >> 1];
        if (upd) xx = acc / D;
    };
    for (int s = 0; s < nbottom; s++) {
        half(upd0);
        half(upd1);
    }
    for (int s = 0; s < nbottom; s++) {
        half(upd1);
        half(upd0);
    }
#pragma unroll
    for (int q = 0; q < NC; q++) {
        double t = __shfl(xx, c + 8 * q, 64);
        if (lane < 8) x[q] = t;
    }
}

// levels [w0, w0 + nw) of the tail (each at most 64 cells) by one wavefront (lane = cell; the
// tail runs one wavefront per component): b of level w0 is read from LDS, its correction x
// written back to LDS; same operations and order as the barrier-separated version
template <int NC>
__device__ __forceinline__ void wave_levels(const LevelV<double>* Lw, int nw, int nu1, int nu2, int nbottom,
                            const double* b0, double* x0) {
    int lane = threadIdx.x & 63;
    WaveRow R[WAVE_MAXL];
    double xs[WAVE_MAXL][NC], bs[WAVE_MAXL][NC];
#pragma unroll
    for (int v = 0; v < WAVE_MAXL; v++) {
        if (v < nw) wave_row(Lw[v], lane, R[v]);
#pragma unroll
        for (int m = 0; m < NC; m++) {
            xs[v][m] = 0.0;
            bs[v][m] = 0.0;
        }
    }
    if (lane < Lw[0].N)
#pragma unroll
        for (int m = 0; m < NC; m++) bs[0][m] = b0[m * Lw[0].N + lane];
#pragma unroll
    for (int v = 0; v < WAVE_MAXL; v++) {
        if (v == nw - 1) {
            const GridV& gb = Lw[v].grid;
            if (gb.n[0] == 2 && gb.n[1] == 2 && gb.n[2] == 2) {
                bottom_cube2<NC>(R[v], lane, bs[v], xs[v], nbottom);
            } else {
                for (int s = 0; s < nbottom; s++) {
                    wave_sweep<NC>(R[v], lane, bs[v], xs[v], 0);
                    wave_sweep<NC>(R[v], lane, bs[v], xs[v], 1);
                }
                for (int s = 0; s < nbottom; s++) {
                    wave_sweep<NC>(R[v], lane, bs[v], xs[v], 1);
                    wave_sweep<NC>(R[v], lane, bs[v], xs[v], 0);
                }
            }
        }
        if (v >= nw - 1) continue;
        for (int s = 0; s < nu1; s++) {
            wave_sweep<NC>(R[v], lane, bs[v], xs[v], 0);
            wave_sweep<NC>(R[v], lane, bs[v], xs[v], 1);
        }
        if (v + 1 < WAVE_MAXL) {
            // residual of this level, then the mean of the eight children on the next
            double r[NC];
            {
                double acc[NC];
#pragma unroll
                for (int m = 0; m < NC; m++) acc[m] = 0.0;
                wave_offdiag<NC>(R[v], lane, xs[v], acc);
#pragma unroll
                for (int m = 0; m < NC; m++)
                    r[m] = R[v].open ? bs[v][m] - (R[v].D * xs[v][m] - acc[m]) : 0.0;
            }
            const LevelV<double>& F = Lw[v];
            const LevelV<double>& C = Lw[v + 1];
            int ci = 0, cj = 0, ck = 0;
            if (lane < C.N) cell_coords(C.grid, lane, ci, cj, ck);
            double sum[NC];
#pragma unroll
            for (int m = 0; m < NC; m++) sum[m] = 0.0;
            for (int q = 0; q < 8; q++) {
                int src = lane < C.N ? (int)cell_index(F.grid, 2 * ci + (q & 1),
                                                       2 * cj + ((q >> 1) & 1), 2 * ck + (q >> 2))
                                     : lane;
#pragma unroll
                for (int m = 0; m < NC; m++) sum[m] += __shfl(r[m], src, 64);
            }
            bool copen = lane < C.N && C.mask[lane];
#pragma unroll
            for (int m = 0; m < NC; m++) bs[v + 1][m] = copen ? sum[m] / 8.0 : 0.0;
        }
    }
#pragma unroll
    for (int v = WAVE_MAXL - 2; v >= 0; v--) {
        if (v >= nw - 1) continue;
        const LevelV<double>& F = Lw[v];
        const LevelV<double>& C = Lw[v + 1];
        int src = lane;
        if (lane < F.N) {
            int i, j, k;
            cell_coords(F.grid, lane, i, j, k);
            src = (int)cell_index(C.grid, i >> 1, j >> 1, k >> 1);
        }
#pragma unroll
        for (int m = 0; m < NC; m++) {
            double e = __shfl(xs[v + 1][m], src, 64);
            if (lane < F.N && R[v].open) xs[v][m] += e;
        }
        for (int s = 0; s < nu2; s++) {
            wave_sweep<NC>(R[v], lane, bs[v], xs[v], 1);
            wave_sweep<NC>(R[v], lane, bs[v], xs[v], 0);
        }
    }
    if (lane < Lw[0].N)
#pragma unroll
        for (int m = 0; m < NC; m++) x0[m * Lw[0].N + lane] = xs[0][m];
}

// ---- a block level of at most two cells per thread (thread t owns cells 2t and 2t + 1, one of
// ---- each colour since nx is even): the rows (face coefficients with their neighbours, the
// ---- diagonal) are built once per V-cycle into registers, so a half sweep costs its LDS reads
struct BlockRow {
    double K[6];
    int nb[6];  // neighbour cell, or the cell itself where the face has no coupling (K = 0)
    double D;
    int c;      // the cell, -1 if the thread has none
    bool upd;   // open with a positive diagonal (updated by the smoother)
    bool open;
};

__device__ __forceinline__ void block_row(const LevelV<double>& L, long c, BlockRow& r) {
    r.c = c < L.N ? (int)c : -1;
    r.open = r.c >= 0 && L.mask[c] != 0;
    r.D = r.c >= 0 ? L.D[c] : 0.0;
    r.upd = r.open && r.D > 0.0;
    int i = 0, j = 0, k = 0;
    if (r.c >= 0) cell_coords(L.grid, c, i, j, k);
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            double K = 0.0;
            long nb = -1;
            if (r.c >= 0) {
                int f[3] = {i, j, k};
                f[d] += side;
                K = L.K[d][face_index(L.grid, d, f[0], f[1], f[2])];
                nb = cell_step(L.grid, c, i, j, k, d, side);
            }
            bool use = K != 0.0 && nb >= 0;
            r.K[2 * d + side] = use ? K : 0.0;
            r.nb[2 * d + side] = use ? (int)nb : (r.c >= 0 ? r.c : 0);
        }
}

// sum_f K_f x_nb(f) in the face order of offdiag (absent couplings add exactly zero)
template <int NC>
__device__ __forceinline__ void block_offdiag(const BlockRow& r, const double* x, long N,
                                              double acc[NC]) {
#pragma unroll
    for (int f = 0; f < 6; f++)
#pragma unroll
        for (int m = 0; m < NC; m++) acc[m] += r.K[f] * x[m * N + r.nb[f]];
}

template <int NC>
__device__ __forceinline__ void block_update(const BlockRow& r, const double* b, double* x,
                                             long N) {
    if (!r.upd) return;
    double acc[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) acc[m] = b[m * N + r.c];
    block_offdiag<NC>(r, x, N, acc);
#pragma unroll
    for (int m = 0; m < NC; m++) x[m * N + r.c] = acc[m] / r.D;
}

// one half sweep of colour col: the thread's cell of that colour
template <int NC>
__device__ __forceinline__ void block_sweep(const BlockRow& r0, const BlockRow& r1, int col0,
                                            const double* b, double* x, long N, int col) {
    block_update<NC>(col0 == col ? r0 : r1, b, x, N);
    __syncthreads();
}

template <int NC>
__device__ __forceinline__ void block_resid(const BlockRow& r, const double* b, const double* x,
                                            long N, double* res) {
    if (r.c < 0) return;
    if (!r.open) {
#pragma unroll
        for (int m = 0; m < NC; m++) res[m * N + r.c] = 0.0;
        return;
    }
    double acc[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) acc[m] = 0.0;
    block_offdiag<NC>(r, x, N, acc);
#pragma unroll
    for (int m = 0; m < NC; m++) res[m * N + r.c] = b[m * N + r.c] - (r.D * x[m * N + r.c] - acc[m]);
}

template <int NC>
__global__ void __launch_bounds__(TAIL_THREADS) k_vcycle_tail(TailArgs A) {
    if (A.gate && *A.gate) return;
    extern __shared__ double lds_d[];
    char* lds = reinterpret_cast<char*>(lds_d);
    int nl = A.nl;
    // stage the operators (one contiguous copy of the pack) and the first right-hand side in
    // LDS: every thread issues all of its loads, then stores them
    {
        const uint4* __restrict__ ps = reinterpret_cast<const uint4*>(A.pack);
        uint4* pd = reinterpret_cast<uint4*>(lds);
        const double* __restrict__ bs = A.b0;
        double* bd = reinterpret_cast<double*>(lds + A.ob[0]);
        unsigned n16 = A.nstatic / 16, nb = NC * (unsigned)A.L[0].N;
        constexpr int PS = 8, BS = 8;
        uint4 pv[PS];
        double bv[BS];
#pragma unroll
        for (int u = 0; u < PS; u++) {
            unsigned t = u * blockDim.x + threadIdx.x;
            if (t < n16) pv[u] = ps[t];
        }
#pragma unroll
        for (int u = 0; u < BS; u++) {
            unsigned t = u * blockDim.x + threadIdx.x;
            if (t < nb) bv[u] = bs[t];
        }
#pragma unroll
        for (int u = 0; u < PS; u++) {
            unsigned t = u * blockDim.x + threadIdx.x;
            if (t < n16) pd[t] = pv[u];
        }
#pragma unroll
        for (int u = 0; u < BS; u++) {
            unsigned t = u * blockDim.x + threadIdx.x;
            if (t < nb) bd[t] = bv[u];
        }
        for (unsigned t = PS * blockDim.x + threadIdx.x; t < n16; t += blockDim.x) pd[t] = ps[t];
        for (unsigned t = BS * blockDim.x + threadIdx.x; t < nb; t += blockDim.x) bd[t] = bs[t];
    }
    __syncthreads();
    auto lv = [&](int l) {
        LevelV<double> v = A.L[l];
#pragma unroll
        for (int d = 0; d < 3; d++) v.K[d] = reinterpret_cast<const double*>(lds + A.oK[l][d]);
        v.D = reinterpret_cast<const double*>(lds + A.oD[l]);
        v.mask = reinterpret_cast<const uint8_t*>(lds + A.om[l]);
        return v;
    };
    auto X = [&](int l) { return reinterpret_cast<double*>(lds + A.ox[l]); };
    auto B = [&](int l) { return reinterpret_cast<double*>(lds + A.ob[l]); };
    // first level small enough for one wavefront (all coarser ones are smaller)
    int w0 = nl;
    while (w0 > 0 && A.L[w0 - 1].N <= 64 && nl - (w0 - 1) <= WAVE_MAXL) w0--;
    if (w0 == 1 && nl > 1 && A.L[0].N <= 2 * (long)blockDim.x && (A.L[0].grid.n[0] & 1) == 0) {
        // one block level above the in-wave levels, its rows in registers
        LevelV<double> L = lv(0);
        LevelV<double> C = lv(1);
        long N = L.N;
        double* x = X(0);
        double* b = B(0);
        BlockRow r0, r1;
        block_row(L, 2 * (long)threadIdx.x, r0);
        block_row(L, 2 * (long)threadIdx.x + 1, r1);
        int col0 = 0;
        if (r0.c >= 0) {
            int i, j, k;
            cell_coords(L.grid, r0.c, i, j, k);
            col0 = (i + j + k) & 1;
        }
        for (long t = threadIdx.x; t < NC * N; t += blockDim.x) x[t] = 0.0;
        __syncthreads();
        for (int s = 0; s < A.nu1; s++) {
            block_sweep<NC>(r0, r1, col0, b, x, N, 0);
            block_sweep<NC>(r0, r1, col0, b, x, N, 1);
        }
        // residuals of both cells, then the coarse right-hand side as the mean of the eight
        // children in the order q = 0..7
        double* res = reinterpret_cast<double*>(lds + A.orr);
        block_resid<NC>(r0, b, x, N, res);
        block_resid<NC>(r1, b, x, N, res);
        __syncthreads();
        double* bc = B(1);
        for (long c = threadIdx.x; c < C.N; c += blockDim.x) {
            int i, j, k;
            cell_coords(C.grid, c, i, j, k);
            double sm[NC];
#pragma unroll
            for (int m = 0; m < NC; m++) sm[m] = 0.0;
            for (int q = 0; q < 8; q++) {
                long f = cell_index(L.grid, 2 * i + (q & 1), 2 * j + ((q >> 1) & 1),
                                    2 * k + (q >> 2));
#pragma unroll
                for (int m = 0; m < NC; m++) sm[m] += res[m * N + f];
            }
#pragma unroll
            for (int m = 0; m < NC; m++) bc[m * C.N + c] = C.mask[c] ? sm[m] / 8.0 : 0.0;
        }
        __syncthreads();
        // the in-wave levels: wave m runs component m (the components are uncoupled)
        int wv = threadIdx.x >> 6;
        if (wv < NC) {
            LevelV<double> Lw[WAVE_MAXL];
            for (int v = 0; v < WAVE_MAXL; v++) Lw[v] = lv(1 + (1 + v < nl ? v : 0));
            long off = wv * A.L[1].N;
            wave_levels<1>(Lw, nl - 1, A.nu1, A.nu2, A.nbottom, B(1) + off, X(1) + off);
        }
        __syncthreads();
        // prolongation of the coarse correction to the thread's open cells
        const double* xc = X(1);
        for (int h = 0; h < 2; h++) {
            const BlockRow& r = h ? r1 : r0;
            if (r.c < 0 || !r.open) continue;
            int i, j, k;
            cell_coords(L.grid, r.c, i, j, k);
            long pc = cell_index(C.grid, i >> 1, j >> 1, k >> 1);
#pragma unroll
            for (int m = 0; m < NC; m++) x[m * N + r.c] += xc[m * C.N + pc];
        }
        __syncthreads();
        for (int s = 0; s < A.nu2; s++) {
            block_sweep<NC>(r0, r1, col0, b, x, N, 1);
            block_sweep<NC>(r0, r1, col0, b, x, N, 0);
        }
        for (long t = threadIdx.x; t < NC * N; t += blockDim.x) A.x0[t] = x[t];
        return;
    }
    for (int l = 0; l < w0; l++) {
        LevelV<double> L = lv(l);
        double* x = X(l);
        double* b = B(l);
        for (long t = threadIdx.x; t < NC * L.N; t += blockDim.x) x[t] = 0.0;
        __syncthreads();
        if (l == nl - 1) {
            for (int s = 0; s < A.nbottom; s++) {
                tail_sweep<NC>(L, b, x, 0);
                tail_sweep<NC>(L, b, x, 1);
            }
            for (int s = 0; s < A.nbottom; s++) {
                tail_sweep<NC>(L, b, x, 1);
                tail_sweep<NC>(L, b, x, 0);
            }
            break;
        }
        for (int s = 0; s < A.nu1; s++) {
            tail_sweep<NC>(L, b, x, 0);
            tail_sweep<NC>(L, b, x, 1);
        }
        // residual and restriction fused: the coarse right-hand side is the mean of the eight
        // children's residuals
        LevelV<double> C = lv(l + 1);
        double* bc = B(l + 1);
        for (long c = threadIdx.x; c < C.N; c += blockDim.x) {
            int i, j, k;
            cell_coords(C.grid, c, i, j, k);
            double s[NC];
#pragma unroll
            for (int m = 0; m < NC; m++) s[m] = 0.0;
            for (int q = 0; q < 8; q++) {
                long f = cell_index(L.grid, 2 * i + (q & 1), 2 * j + ((q >> 1) & 1), 2 * k + (q >> 2));
                double r[NC];
                resid_value<NC>(L, b, x, f, r);
#pragma unroll
                for (int m = 0; m < NC; m++) s[m] += r[m];
            }
#pragma unroll
            for (int m = 0; m < NC; m++) bc[m * C.N + c] = C.mask[c] ? s[m] / 8.0 : 0.0;
        }
        __syncthreads();
    }
    if (w0 < nl) {
        int wv = threadIdx.x >> 6;
        if (wv < NC) {
            LevelV<double> Lw[WAVE_MAXL];
            for (int v = 0; v < WAVE_MAXL; v++) Lw[v] = lv(w0 + (w0 + v < nl ? v : 0));
            long off = wv * A.L[w0].N;
            wave_levels<1>(Lw, nl - w0, A.nu1, A.nu2, A.nbottom, B(w0) + off, X(w0) + off);
        }
        __syncthreads();
    }
    for (int l = (w0 < nl ? w0 : nl - 1) - 1; l >= 0; l--) {
        LevelV<double> L = lv(l);
        LevelV<double> C = lv(l + 1);
        double* x = X(l);
        for (long f = threadIdx.x; f < L.N; f += blockDim.x)
            prolong_cell<double, double, NC>(L.grid, C.grid, L.mask, X(l + 1), x, f);
        __syncthreads();
        for (int s = 0; s < A.nu2; s++) {
            tail_sweep<NC>(L, B(l), x, 1);
            tail_sweep<NC>(L, B(l), x, 0);
        }
    }
    double* x0 = X(0);
    for (long t = threadIdx.x; t < NC * A.L[0].N; t += blockDim.x) A.x0[t] = x0[t];
}

// LDS bytes for levels [t, nlev) with nc components; fills the offsets when A is given
size_t tail_layout(const Level* lev, int nlev, int t, int nc, TailArgs* A) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = (off + bytes + 15) & ~size_t(15);
        return (unsigned)o;
    };
    // the operator arrays of every level first (the pack's layout), then the vectors
    for (int l = t; l < nlev; l++) {
        const Level& L = lev[l];
        int q = l - t;
        unsigned oK[3];
        for (int d = 0; d < 3; d++) oK[d] = take(face_count(L.grid, d) * 8);
        unsigned oD = take(L.N * 8), om = take(L.N);
        if (A) {
            for (int d = 0; d < 3; d++) A->oK[q][d] = oK[d];
            A->oD[q] = oD;
            A->om[q] = om;
        }
    }
    if (A) A->nstatic = (unsigned)off;
    for (int l = t; l < nlev; l++) {
        const Level& L = lev[l];
        int q = l - t;
        unsigned ox = take(nc * L.N * 8), ob = take(nc * L.N * 8);
        unsigned orr = q == 0 ? take(nc * L.N * 8) : 0;
        if (A) {
            A->ox[q] = ox;
            A->ob[q] = ob;
            if (q == 0) A->orr = orr;
        }
    }
    return off;
}

// the pack: the tail levels' K, D and mask copied into the LDS layout of tail_layout, once per
// operator build (one work-group per array)
constexpr int PACK_SEGS = 5 * TAIL_MAXL;
struct PackArgs {
    int nseg;
    const char* src[PACK_SEGS];
    unsigned dst[PACK_SEGS], bytes[PACK_SEGS];
    char* pack;
};
__global__ void k_tail_pack(PackArgs P) {
    int sg = blockIdx.x;
    if (sg >= P.nseg) return;
    const char* __restrict__ src = P.src[sg];
    char* dst = P.pack + P.dst[sg];
    unsigned n = P.bytes[sg];
    if ((n & 7) == 0) {
        for (unsigned t = threadIdx.x; t < n / 8; t += blockDim.x)
            reinterpret_cast<double*>(dst)[t] = reinterpret_cast<const double*>(src)[t];
    } else {
        for (unsigned t = threadIdx.x; t < n; t += blockDim.x) dst[t] = src[t];
    }
}

// ------------------------------------------------------------------------------------------
// exact EB viscous Helmholtz operator (Eq. implicit-viscous with the wall flux of Eq. dudn)
// ------------------------------------------------------------------------------------------
// the operator row of a regular cell (volume fraction and all six apertures 1, no wall flux)
// from its loaded velocity, neighbours and viscosities; in[f]: a neighbour across face f
__device__ __forceinline__ void visc_regular_row(const GeomV& g, double rho, double kin,
                                                 double kwall, int homog, double ec,
                                                 const double en[6], const double uc[3],
                                                 const double un[6][3], const bool in[6],
                                                 double acc[3]) {
    for (int m = 0; m < 3; m++) acc[m] = 1.0 * rho * uc[m];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            int f = 2 * d + side;
            if (in[f]) {
                double K = kin * (ec + en[f]);
                for (int m = 0; m < 3; m++) acc[m] -= K * (un[f][m] - uc[m]);
            } else {
                double K = kwall * ec;
                for (int m = 0; m < 3; m++) {
                    double uw = homog ? 0.0 : g.wall[2 * d + side][m];
                    acc[m] -= K * (uw - uc[m]);
                }
            }
        }
}

// One cell c = (i, j, k) of the operator, every load (flag, its velocity, the six neighbours'
// velocities and viscosities) issued before the first is needed.  kin = dt/(2 h^2) and kwall =
// 2 dt/h^2 as the level-0 smoother forms them (regular cells take K = kin (eta_c + eta_n) inside
// and kwall eta_c on a domain wall, with no division per face).  TU: the input's type; FP32
// input is widened exactly.
template <typename TU>
__device__ __forceinline__ void visc_apply_cell(const GeomV& g, double rho, double dt,
                                                double kin, double kwall,
                                                const double* __restrict__ eta,
                                                const TU* __restrict__ u,
                                                double* __restrict__ out, int homog, long c,
                                                int i, int j, int k) {
    long N = g.N;
    long nb[6];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            nb[2 * d + side] = cell_step(g.grid, c, i, j, k, d, side);
        }
    uint8_t fl = g.flag[c];
    // a missing neighbour (across a wall) loads the cell itself, a value never used: the loads
    // are unconditional, so none waits behind a branch (an FP32 input widened inside a branch
    // would make each load wait before the next is issued)
    double uc[3], un[6][3], en[6];
#pragma unroll
    for (int m = 0; m < 3; m++) uc[m] = (double)u[m * N + c];
#pragma unroll
    for (int f = 0; f < 6; f++) {
        long q = nb[f] >= 0 ? nb[f] : c;
        en[f] = eta[q];
#pragma unroll
        for (int m = 0; m < 3; m++) un[f][m] = (double)u[m * N + q];
    }
    double ec = eta[c];
    if (fl == 0) {
        for (int m = 0; m < 3; m++) out[m * N + c] = 0.0;
        return;
    }
    double h2 = g.grid.h * g.grid.h;
    double acc[3];
    if (fl == 2) {
        bool in[6];
#pragma unroll
        for (int f = 0; f < 6; f++) in[f] = nb[f] >= 0;
        visc_regular_row(g, rho, kin, kwall, homog, ec, en, uc, un, in, acc);
        for (int m = 0; m < 3; m++) out[m * N + c] = acc[m];
        return;
    }
    double al = g.alpha[c];
    for (int m = 0; m < 3; m++) acc[m] = al * rho * uc[m];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            int fi[3] = {i, j, k};
            fi[d] += side;
            double A = g.ap[d][face_index(g.grid, d, fi[0], fi[1], fi[2])];
            if (A == 0.0) continue;
            int f = 2 * d + side;
            if (nb[f] >= 0) {
                double K = dt * A * 0.5 * (ec + en[f]) / h2;
                for (int m = 0; m < 3; m++) acc[m] -= K * (un[f][m] - uc[m]);
            } else {
                double K = 2.0 * dt * A * ec / h2;
                for (int m = 0; m < 3; m++) {
                    double uw = homog ? 0.0 : g.wall[2 * d + side][m];
                    acc[m] -= K * (uw - uc[m]);
                }
            }
        }
    for (int m = 0; m < 3; m++) out[m * N + c] = acc[m];
}

// one cell per thread (any alignment of eta, u and out)
template <typename TU>
__global__ void __launch_bounds__(EB_BLOCK)
    k_visc_apply_one(GeomV g, double rho, double dt, double kin, double kwall, FastDiv dnx,
                     FastDiv dny, const double* __restrict__ eta, const TU* __restrict__ u,
                     double* __restrict__ out, int homog, const int* gate) {
    if (gate && *gate) return;
    long c = xcd_block() * (long)blockDim.x + threadIdx.x;
    if (c >= g.N) return;
    unsigned cu = (unsigned)c;
    unsigned t = fdiv(cu, dnx);
    unsigned k2 = fdiv(t, dny);
    visc_apply_cell<TU>(g, rho, dt, kin, kwall, eta, u, out, homog, c, (int)(cu - t * dnx.d),
                        (int)(t - k2 * dny.d), (int)k2);
}

template <typename TU> struct Two;
template <> struct Two<double> { using t = double2; };
template <> struct Two<float> { using t = float2; };

// The operator on two neighbouring cells a = (i0, j, k) and b = (i0 + 1, j, k), i0 even, per
// thread: a's upper and b's lower x neighbour are each other, the two outer x neighbours are
// lone loads, and each y and z face's neighbours of both cells are one aligned pair (16 bytes in
// FP64), as are the two cells' own values and viscosities, so a regular cell needs about half
// the load instructions of the one-cell form.  The first ncb blocks (a multiple of 8) take one
// cut cell per thread through visc_apply_cell; the pair blocks write regular (and covered) cells
// only.  Results are visc_apply_cell's, bit for bit.  dnx, dny divide by the extents.  FP32
// input needs 124 VGPRs (four waves per SIMD); FP64 input 134 (three waves: at four it spills),
// which still measured 0.35 ms per step faster at 128^3 than the one-cell kernel (35.1-35.2
// against 35.5 ms, alternated on one GPU).
template <typename TU>
__global__ void __launch_bounds__(PAIR_BLOCK, 3)
    k_visc_apply(GeomV g, double rho, double dt, double kin, double kwall, FastDiv dnx,
                 FastDiv dny, const double* __restrict__ eta, const TU* __restrict__ u,
                 double* __restrict__ out, int homog, const int* gate, unsigned ncb) {
    using P2 = typename Two<TU>::t;
    if (gate && *gate) return;
    long N = g.N;
    if (blockIdx.x < ncb) {
        long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
        if (q >= g.ncut) return;
        long c = g.cut[q];
        unsigned cu = (unsigned)c;
        unsigned t = fdiv(cu, dnx);
        unsigned k2 = fdiv(t, dny);
        visc_apply_cell<TU>(g, rho, dt, kin, kwall, eta, u, out, homog, c,
                            (int)(cu - t * dnx.d), (int)(t - k2 * dny.d), (int)k2);
        return;
    }
    unsigned npb = gridDim.x - ncb, v = blockIdx.x - ncb;
    unsigned tile = (v & 7) * (npb >> 3) + ((v & 7) < (npb & 7) ? (v & 7) : (npb & 7)) + (v >> 3);
    long p = tile * (long)blockDim.x + threadIdx.x;
    if (p >= (N >> 1)) return;
    long ca = 2 * p;
    int i, j, k;
    {
        unsigned cu = (unsigned)ca;
        unsigned t = fdiv(cu, dnx);
        i = (int)(cu - t * dnx.d);
        unsigned k2 = fdiv(t, dny);
        j = (int)(t - k2 * dny.d);
        k = (int)k2;
    }
    long nba[6], nbb[6];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int side = 0; side < 2; side++) {
            nba[2 * d + side] = cell_step(g.grid, ca, i, j, k, d, side);
            nbb[2 * d + side] = cell_step(g.grid, ca + 1, i + 1, j, k, d, side);
        }
    uint8_t fla = g.flag[ca], flb = g.flag[ca + 1];
    long qxa = nba[0] >= 0 ? nba[0] : ca, qxb = nbb[1] >= 0 ? nbb[1] : ca + 1;
    long qy[2], qz[2];  // the even cell of each y and z neighbour pair (a's neighbour)
#pragma unroll
    for (int side = 0; side < 2; side++) {
        qy[side] = nba[2 + side] >= 0 ? nba[2 + side] : ca;
        qz[side] = nba[4 + side] >= 0 ? nba[4 + side] : ca;
    }
    double uca[3], ucb[3], una[6][3], unb[6][3];
#pragma unroll
    for (int m = 0; m < 3; m++) {
        P2 o = *reinterpret_cast<const P2*>(u + m * N + ca);
        uca[m] = (double)o.x;
        ucb[m] = (double)o.y;
        una[0][m] = (double)u[m * N + qxa];
        unb[1][m] = (double)u[m * N + qxb];
#pragma unroll
        for (int side = 0; side < 2; side++) {
            P2 y2 = *reinterpret_cast<const P2*>(u + m * N + qy[side]);
            P2 z2 = *reinterpret_cast<const P2*>(u + m * N + qz[side]);
            una[2 + side][m] = (double)y2.x;
            unb[2 + side][m] = (double)y2.y;
            una[4 + side][m] = (double)z2.x;
            unb[4 + side][m] = (double)z2.y;
        }
        una[1][m] = ucb[m];
        unb[0][m] = uca[m];
    }
    double ena[6], enb[6];
    double2 e2 = *reinterpret_cast<const double2*>(eta + ca);
    double eca = e2.x, ecb = e2.y;
    ena[0] = eta[qxa];
    enb[1] = eta[qxb];
    ena[1] = ecb;
    enb[0] = eca;
#pragma unroll
    for (int side = 0; side < 2; side++) {
        double2 y2 = *reinterpret_cast<const double2*>(eta + qy[side]);
        double2 z2 = *reinterpret_cast<const double2*>(eta + qz[side]);
        ena[2 + side] = y2.x;
        enb[2 + side] = y2.y;
        ena[4 + side] = z2.x;
        enb[4 + side] = z2.y;
    }
    bool ina[6], inb[6];
#pragma unroll
    for (int f = 0; f < 6; f++) {
        ina[f] = nba[f] >= 0;
        inb[f] = nbb[f] >= 0;
    }
    // one cell after the other (their values die sooner); covered cells are 0, cut cells the
    // first blocks'
    double acc[3];
    visc_regular_row(g, rho, kin, kwall, homog, eca, ena, uca, una, ina, acc);
    if (fla != 1) {
#pragma unroll
        for (int m = 0; m < 3; m++) out[m * N + ca] = fla == 0 ? 0.0 : acc[m];
    }
    visc_regular_row(g, rho, kin, kwall, homog, ecb, enb, ucb, unb, inb, acc);
    if (flb != 1) {
#pragma unroll
        for (int m = 0; m < 3; m++) out[m * N + ca + 1] = flb == 0 ? 0.0 : acc[m];
    }
}

// the wall-flux term of the cut-cell rows, added after k_visc_apply (one thread per cut cell,
// each writing only its own row): dt A_EB eta_EB (du/dn of Eq. dudn) / h
template <typename TU>
__global__ void __launch_bounds__(EB_BLOCK) k_visc_apply_eb(GeomV g, double dt,
                                                            const double* __restrict__ eta_eb,
                                                            const TU* __restrict__ u,
                                                            double* __restrict__ out, int homog,
                                                            const int* gate) {
    if (gate && *gate) return;
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = g.ncut;
    if (q >= nc) return;
    long N = g.N;
    const int* __restrict__ sidx = g.sidx;
    const double* __restrict__ sw = g.sw;
    // every load first: the stencil's 18 indices and weights, then the 54 velocity values and
    // the three rows being added to
    long c = g.cut[q];
    int ci[18];
    double wi[18];
#pragma unroll
    for (int t = 0; t < 18; t++) {
        ci[t] = sidx[(long)t * nc + q];
        wi[t] = sw[(long)t * nc + q];
    }
    double d1 = g.dd[q], d2 = g.dd[nc + q];
    double coef = dt * g.aeb[q] * eta_eb[q] / g.grid.h;
    double uv[3][18], o[3];
#pragma unroll
    for (int m = 0; m < 3; m++) {
        double ue = homog ? 0.0 : g.ueb[m];
#pragma unroll
        for (int t = 0; t < 18; t++) {
            TU v = u[m * N + (ci[t] >= 0 ? (long)ci[t] : c)];  // unconditional, as above
            uv[m][t] = ci[t] >= 0 ? (double)v : ue;
        }
        o[m] = out[m * N + c];
    }
    double den = d1 * d2 * (d2 - d1) * g.grid.h;
#pragma unroll
    for (int m = 0; m < 3; m++) {
        double ue = homog ? 0.0 : g.ueb[m];
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int t = 0; t < 9; t++) {
            s1 += wi[t] * uv[m][t];
            s2 += wi[t + 9] * uv[m][t + 9];
        }
        double gn = (d2 * d2 * (s1 - ue) - d1 * d1 * (s2 - ue)) / den;
        out[m * N + c] = o[m] + coef * gn;
    }
}

// ------------------------------------------------------------------------------------------
// reductions (fixed grid, fixed order: deterministic for a given size)
// ------------------------------------------------------------------------------------------
constexpr int RED_MAXB = 1024;

__device__ __forceinline__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}
__device__ __forceinline__ double block_max(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) sh[threadIdx.x] = nan_max(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// row p of nb per-block partials reduced in a fixed order (a sum, or a maximum if mx): thread i
// takes partials i, i + B, i + 2B, ... in turn (B threads), then the block combines the
// threads; the loads of four turns are issued before the first is used
__device__ __forceinline__ double red_row(const double* __restrict__ part, int nb, int p, bool mx,
                                          double* sh) {
    double v = 0.0;
    const int B = blockDim.x;
    for (int t0 = 0; t0 < nb; t0 += 4 * B) {
        double w[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            int t = t0 + k * B + threadIdx.x;
            w[k] = t < nb ? part[p * nb + t] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (t0 + k * B + (int)threadIdx.x < nb) v = mx ? nan_max(v, w[k]) : v + w[k];
    }
    return mx ? block_max(v, sh) : block_sum(v, sh);
}

struct DotArgs {
    const double* a[4];
    const double* b[4];
};

template <int NP>
__global__ void k_dots(long n, DotArgs args, double* __restrict__ part, const int* gate) {
    if (gate && *gate) return;
    __shared__ double sh[EB_BLOCK];
    double s[NP];
#pragma unroll
    for (int p = 0; p < NP; p++) s[p] = 0.0;
#pragma unroll 4
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
         t += (long)gridDim.x * blockDim.x)
#pragma unroll
        for (int p = 0; p < NP; p++) s[p] += args.a[p][t] * args.b[p][t];
#pragma unroll
    for (int p = 0; p < NP; p++) {
        double v = block_sum(s[p], sh);
        if (threadIdx.x == 0) part[p * gridDim.x + blockIdx.x] = v;
    }
}

// per-component max |x| of a [ncomp][n] array
__global__ void k_maxabs(long n, int ncomp, const double* __restrict__ x,
                         double* __restrict__ part, const int* gate) {
    if (gate && *gate) return;
    __shared__ double sh[EB_BLOCK];
    for (int m = 0; m < ncomp; m++) {
        double v = 0.0;
#pragma unroll 4
        for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
             t += (long)gridDim.x * blockDim.x)
            v = nan_max(v, fabs(x[m * n + t]));
        v = block_max(v, sh);
        if (threadIdx.x == 0) part[m * gridDim.x + blockIdx.x] = v;
    }
}

// ---- Krylov steps fused with the reductions that follow them (same grid, same per-thread
// ---- order and the same final pass as k_dots / k_maxabs, so the scalars are bit for bit those
// ---- of the separate kernels), and final passes that go on to the scalar update
struct OpOut {
    int idx[4];   // ks slot receiving each reduced row
    int maxmask;  // bit p set: row p is a maximum (else a sum)
};

// rows of per-block partials reduced into ks[idx[p]], then the scalar update op; the rows are
// skipped once the solve has stopped (the op itself then does nothing)
__global__ void k_final_op(const double* __restrict__ part, int nb, int nrow, OpOut o, int op,
                           double* __restrict__ ks, int* __restrict__ st, int* __restrict__ itc) {
    __shared__ double sh[EB_BLOCK];
    if (*st == 0) {
        for (int p = 0; p < nrow; p++) {
            double v = red_row(part, nb, p, (o.maxmask >> p) & 1, sh);
            if (threadIdx.x == 0) ks[o.idx[p]] = v;
        }
    }
    if (threadIdx.x == 0) ks_scalar_op(op, ks, st, itc);
}

// BiCGSTAB: s = r - alpha v, with the per-block max |s|
__global__ void k_bi_s_max(long n, double* __restrict__ sv, const double* __restrict__ r,
                           const double* __restrict__ v, const double* __restrict__ ks,
                           const int* __restrict__ st, double* __restrict__ part) {
    if (*st != 0) return;
    __shared__ double sh[EB_BLOCK];
    double al = ks[KS_AL], m = 0.0;
#pragma unroll 4
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
         t += (long)gridDim.x * blockDim.x) {
        double s = r[t] - al * v[t];
        sv[t] = s;
        m = nan_max(m, fabs(s));
    }
    m = block_max(m, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// BiCGSTAB: x += alpha ph + omega sh, r = s - omega t, with the per-block partials of rh . r
// (row 0) and max |r| (row 1)
template <typename TP>
__global__ void k_bi_xr_red(long n, double* __restrict__ x, double* __restrict__ r,
                            const TP* __restrict__ ph, const TP* __restrict__ sh_,
                            const double* __restrict__ sv, const double* __restrict__ tv,
                            const double* __restrict__ rh, const double* __restrict__ ks,
                            const int* __restrict__ st, double* __restrict__ part) {
    if (*st != 0) return;
    __shared__ double sh[EB_BLOCK];
    double al = ks[KS_AL], om = ks[KS_OM];
    double dot = 0.0, m = 0.0;
#pragma unroll 4
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
         t += (long)gridDim.x * blockDim.x) {
        x[t] += al * (double)ph[t] + om * (double)sh_[t];
        double rn = sv[t] - om * tv[t];
        r[t] = rn;
        dot += rh[t] * rn;
        m = nan_max(m, fabs(rn));
    }
    dot = block_sum(dot, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = dot;
    m = block_max(m, sh);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = m;
}

// CG: x += alpha p, r -= alpha q, with the per-block max |r|
__global__ void k_cg_xr_max(long n, double* __restrict__ x, double* __restrict__ r,
                            const double* __restrict__ p, const double* __restrict__ q,
                            const double* __restrict__ ks, const int* __restrict__ st,
                            double* __restrict__ part) {
    if (*st != 0) return;
    __shared__ double sh[EB_BLOCK];
    double a = ks[KS_AL], m = 0.0;
#pragma unroll 4
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
         t += (long)gridDim.x * blockDim.x) {
        x[t] += a * p[t];
        double rn = r[t] - a * q[t];
        r[t] = rn;
        m = nan_max(m, fabs(rn));
    }
    m = block_max(m, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// over open cells: the largest |u| + |v| + |w| (row 0) and the largest yield-stress multiplier
// (row 1; 1 without a field), per block
__global__ void k_cfl_max(GeomV g, const double* __restrict__ u, const double* __restrict__ theta,
                          double* __restrict__ part) {
    __shared__ double sh[EB_BLOCK];
    long N = g.N;
    double a = 0.0, t = 0.0;
    for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < N;
         c += (long)gridDim.x * blockDim.x)
        if (g.alpha[c] > 0.0) {
            a = nan_max(a, fabs(u[c]) + fabs(u[N + c]) + fabs(u[2 * N + c]));
            t = nan_max(t, theta ? theta[c] : 1.0);
        }
    a = block_max(a, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
    t = block_max(t, sh);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = t;
}

__global__ void k_sum_open(GeomV g, const double* __restrict__ x, double* __restrict__ part,
                           const int* gate) {
    if (gate && *gate) return;
    __shared__ double sh[EB_BLOCK];
    double s = 0.0, cnt = 0.0;
#pragma unroll 4
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < g.N;
         t += (long)gridDim.x * blockDim.x)
        if (g.alpha[t] > 0.0) {
            s += x[t];
            cnt += 1.0;
        }
    double v = block_sum(s, sh);
    double w = block_sum(cnt, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v;
        part[gridDim.x + blockIdx.x] = w;
    }
}

// per-row sums of a [nrow][n] array
__global__ void k_rowsum(long n, int nrow, const double* __restrict__ x,
                         double* __restrict__ part) {
    __shared__ double sh[EB_BLOCK];
    for (int p = 0; p < nrow; p++) {
        double v = 0.0;
        for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
             t += (long)gridDim.x * blockDim.x)
            v += x[p * n + t];
        v = block_sum(v, sh);
        if (threadIdx.x == 0) part[p * gridDim.x + blockIdx.x] = v;
    }
}

__global__ void k_face_flux_max(GeomV g, const double* __restrict__ fx,
                                const double* __restrict__ fy, const double* __restrict__ fz,
                                double* __restrict__ part) {
    __shared__ double sh[EB_BLOCK];
    const double* fo[3] = {fx, fy, fz};
    double v = 0.0;
    for (int d = 0; d < 3; d++) {
        long nf = face_count(g.grid, d);
        for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < nf;
             t += (long)gridDim.x * blockDim.x)
            v = nan_max(v, fabs(g.ap[d][t] * fo[d][t]));
    }
    v = block_max(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v / g.grid.h;
}

// out[p] = reduction over nb partials of row p (mode 0 sum, 1 max), fixed order
__global__ void k_final(const double* __restrict__ part, int nb, int nrow, int mode,
                        double* __restrict__ out, const int* gate) {
    if (gate && *gate) return;
    __shared__ double sh[EB_BLOCK];
    for (int p = 0; p < nrow; p++) {
        double v = red_row(part, nb, p, mode != 0, sh);
        if (threadIdx.x == 0) out[p] = v;
    }
}

// ------------------------------------------------------------------------------------------
// vector kernels
// ------------------------------------------------------------------------------------------
__global__ void k_copy(long n, const double* __restrict__ x, double* __restrict__ y) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = x[t];
}
__global__ void k_fill(long n, double v, double* __restrict__ y) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = v;
}
template <typename T>
__global__ void k_zero(long n, T* __restrict__ y, const int* gate = nullptr) {
    if (gate && *gate) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = (T)0;
}
__global__ void k_axpby(long n, double a, const double* __restrict__ x, double b,
                        double* __restrict__ y) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = a * x[t] + b * y[t];
}
__global__ void k_bicg_p(long n, const double* __restrict__ r, double beta, double omega,
                         const double* __restrict__ v, double* __restrict__ p) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) p[t] = r[t] + beta * (p[t] - omega * v[t]);
}
__global__ void k_sub_scaled(long n, const double* __restrict__ x, double a,
                             const double* __restrict__ y, double* __restrict__ z) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) z[t] = x[t] - a * y[t];
}
__global__ void k_bicg_update(long n, double al, const double* __restrict__ ph, double om,
                              const double* __restrict__ sh, const double* __restrict__ sv,
                              const double* __restrict__ tv, double* __restrict__ x,
                              double* __restrict__ r) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) {
        x[t] += al * ph[t] + om * sh[t];
        r[t] = sv[t] - om * tv[t];
    }
}
// b = alpha psi - a0 on open cells (a0 = A(0), the boundary part of the affine operator)
__global__ void k_mask_rhs(GeomV g, const double* __restrict__ psi, const double* __restrict__ a0,
                           double* __restrict__ b) {
    long N = g.N;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 3 * N) return;
    long c = (long)((unsigned)t % (unsigned)N);  // 3N < 2^32
    double al = g.alpha[c];
    b[t] = al > 0.0 ? al * psi[t] - a0[t] : 0.0;
}

// ------------------------------------------------------------------------------------------
// V-cycle driver helpers
// ------------------------------------------------------------------------------------------
template <typename T>
void smooth_pass(const Level& L, int nc, const T* b, T* x, int col, hipStream_t s);
template <>
void smooth_pass<double>(const Level& L, int nc, const double* b, double* x, int col,
                         hipStream_t s) {
    unsigned gb = grid_for(L.N / 2);
    if (nc == 3) k_smooth<double, 3><<<gb, EB_BLOCK, 0, s>>>(L.v64(), b, x, col);
    else k_smooth<double, 1><<<gb, EB_BLOCK, 0, s>>>(L.v64(), b, x, col);
}
template <>
void smooth_pass<float>(const Level& L, int nc, const float* b, float* x, int col,
                        hipStream_t s) {
    unsigned gb = grid_for(L.N / 2);
    if (nc == 3) k_smooth<float, 3><<<gb, EB_BLOCK, 0, s>>>(L.v32(), b, x, col);
    else k_smooth<float, 1><<<gb, EB_BLOCK, 0, s>>>(L.v32(), b, x, col);
}
template <typename T>
LevelV<T> level_view(const Level& L);
template <>
LevelV<double> level_view<double>(const Level& L) { return L.v64(); }
template <>
LevelV<float> level_view<float>(const Level& L) { return L.v32(); }



template <typename T>
void first_pass(const Level& L, int nc, const T* b, T* x, hipStream_t s) {
    if (nc == 3) k_smooth_first<T, 3><<<grid_for(L.N), EB_BLOCK, 0, s>>>(level_view<T>(L), b, x);
    else k_smooth_first<T, 1><<<grid_for(L.N), EB_BLOCK, 0, s>>>(level_view<T>(L), b, x);
}
template <typename TF, typename TC>
void resid_restrict_pass(const Level& F, const Level& C, int nc, const TF* b, const TF* x,
                         TC* bc, FirstV<TC> F1, hipStream_t s) {
    unsigned gr = grid_for(C.N, RR_COARSE);
    if (nc == 3)
        k_resid_restrict<TF, TC, 3><<<gr, RR_THREADS, 0, s>>>(level_view<TF>(F), b, x, C.grid,
                                                              C.mask, bc, F1);
    else
        k_resid_restrict<TF, TC, 1><<<gr, RR_THREADS, 0, s>>>(level_view<TF>(F), b, x, C.grid,
                                                              C.mask, bc, F1);
}
// the first post-smoothing pair (colour 1, then colour 0) with the prolongation of ec fused in
template <typename T, typename TC>
void smooth_pro_pair(const Level& L, const Level& C, int nc, const T* b, T* x, const TC* ec,
                     hipStream_t s) {
    unsigned gb = grid_for(L.N / 2);
    ProV<TC> P{C.grid, ec};
    LevelV<T> v = level_view<T>(L);
    if (nc == 3) {
        k_smooth_pro<T, TC, 3, PRO_NBR><<<gb, EB_BLOCK, 0, s>>>(v, b, x, 1, P);
        k_smooth_pro<T, TC, 3, PRO_OWN><<<gb, EB_BLOCK, 0, s>>>(v, b, x, 0, P);
    } else {
        k_smooth_pro<T, TC, 1, PRO_NBR><<<gb, EB_BLOCK, 0, s>>>(v, b, x, 1, P);
        k_smooth_pro<T, TC, 1, PRO_OWN><<<gb, EB_BLOCK, 0, s>>>(v, b, x, 0, P);
    }
}

template <typename TC, typename TF>
void prolong_pass(const Level& F, const Level& C, int nc, const TC* ec, TF* xf, hipStream_t s) {
    if (nc == 3)
        k_prolong<TC, TF, 3><<<grid_for(F.N), EB_BLOCK, 0, s>>>(F.grid, C.grid, F.mask, ec, xf, F.gate);
    else
        k_prolong<TC, TF, 1><<<grid_for(F.N), EB_BLOCK, 0, s>>>(F.grid, C.grid, F.mask, ec, xf, F.gate);
}

Rb0V rb0_view(const Level& L) {
    Rb0V v;
    v.grid = L.grid;
    v.dnx = fast_div((unsigned)L.grid.n[0]);
    v.dny = fast_div((unsigned)L.grid.n[1]);
    v.dnxh = fast_div((unsigned)L.grid.n[0] / 2);
    v.N = L.N;
    v.flag = L.flag;
    v.cut = L.cut;
    v.ncut = L.ncut;
    v.etacs = L.etacs;
    v.etafcs = L.etafcs;
    v.flagcs = L.flagcs;
    v.eta = L.eta;
    v.etaf = L.etaf;
    for (int d = 0; d < 3; d++) v.K[d] = L.K[d];
    v.D = L.D;
    v.sys = L.sys;
    v.rho = L.rho;
    double h2 = L.grid.h * L.grid.h;
    v.kin = L.dt * 0.5 / h2;
    v.kwall = 2.0 * L.dt / h2;
    v.kpois = L.beta / h2;
    v.gate = L.gate;
    return v;
}

// whether the two-cells-per-thread kernel can take a level-0 half sweep: n_x a multiple of 4,
// the component count matching the system, and the colour-split copies made
bool pair_ok(const Rb0V& v, int nc) {
    return (v.grid.n[0] & 3) == 0 && (nc == 3) == (v.sys == EB_SYS_VISC) && v.flagcs &&
           (v.sys != EB_SYS_VISC || v.etacs);
}
// the same for the four-cells-per-thread FP32 kernel: n_x a multiple of 8
bool quad_ok(const Rb0V& v, int nc) {
    return (v.grid.n[0] & 7) == 0 && (nc == 3) == (v.sys == EB_SYS_VISC) && v.flagcs &&
           (v.sys != EB_SYS_VISC || v.etafcs);
}
template <int PRO>
void launch_quad(const Rb0V& v, int nc, const float* b, float* x, int col, hipStream_t s) {
    unsigned gp = grid_for(v.N / 8, PAIR_BLOCK);
    unsigned gc = v.ncut > 0 ? (grid_for(v.ncut, PAIR_BLOCK) + 7) & ~7u : 0;
    if (nc == 3) k_smooth_rb_quad<3, PRO><<<gc + gp, PAIR_BLOCK, 0, s>>>(v, b, x, col, gc);
    else k_smooth_rb_quad<1, PRO><<<gc + gp, PAIR_BLOCK, 0, s>>>(v, b, x, col, gc);
}

// one colour's half sweep of level 0: the two-cells-per-thread kernel in FP64 (n_x a multiple
// of 4), the four-cells-per-thread kernel in FP32 (n_x a multiple of 8), else the one-cell
// kernel; the same result either way
template <typename T>
void rb_half_sweep(const Rb0V& v, int nc, const T* b, T* x, int col, hipStream_t s) {
    if constexpr (std::is_same<T, double>::value) {
        if (pair_ok(v, nc)) {
            unsigned gp = grid_for(v.N / 4, PAIR_BLOCK);
            unsigned gc = v.ncut > 0 ? (grid_for(v.ncut, PAIR_BLOCK) + 7) & ~7u : 0;
            if (nc == 3)
                k_smooth_rb_pair<T, 3><<<gc + gp, PAIR_BLOCK, 0, s>>>(v, b, x, col, gc);
            else
                k_smooth_rb_pair<T, 1><<<gc + gp, PAIR_BLOCK, 0, s>>>(v, b, x, col, gc);
            return;
        }
    } else {
        if (quad_ok(v, nc)) {
            launch_quad<PRO_NONE>(v, nc, b, x, col, s);
            return;
        }
    }
    unsigned gb = grid_for(v.N / 2);
    if (nc == 3) k_smooth_rb<T, 3><<<gb, EB_BLOCK, 0, s>>>(v, b, x, col);
    else k_smooth_rb<T, 1><<<gb, EB_BLOCK, 0, s>>>(v, b, x, col);
}

// a half sweep of level 0 with a PRO variant: for PRO_ZERO the two- or four-cells-per-thread
// kernel where rb_half_sweep takes it, else k_smooth_rb_pro
template <typename T, typename TC, int PRO>
void rb_half_sweep_pro(const Rb0V& v, int nc, const T* b, T* x, int col, ProV<TC> P,
                       hipStream_t s) {
    if constexpr (std::is_same<T, double>::value && PRO == PRO_ZERO) {
        if (pair_ok(v, nc)) {
            unsigned gp = grid_for(v.N / 4, PAIR_BLOCK);
            unsigned gc = v.ncut > 0 ? (grid_for(v.ncut, PAIR_BLOCK) + 7) & ~7u : 0;
            if (nc == 3)
                k_smooth_rb_pair<T, 3, PRO><<<gc + gp, PAIR_BLOCK, 0, s>>>(v, b, x, col, gc);
            else
                k_smooth_rb_pair<T, 1, PRO><<<gc + gp, PAIR_BLOCK, 0, s>>>(v, b, x, col, gc);
            return;
        }
    }
    if constexpr (std::is_same<T, float>::value && PRO == PRO_ZERO) {
        if (quad_ok(v, nc)) {
            launch_quad<PRO>(v, nc, b, x, col, s);
            return;
        }
    }
    unsigned gh = grid_for(v.N / 2);
    if (nc == 3) k_smooth_rb_pro<T, TC, 3, PRO><<<gh, EB_BLOCK, 0, s>>>(v, b, x, col, P);
    else k_smooth_rb_pro<T, TC, 1, PRO><<<gh, EB_BLOCK, 0, s>>>(v, b, x, col, P);
}

template <typename T>
void smooth_rb_pass(const Level& L, int nc, const T* b, T* x, int col, hipStream_t s) {
    rb_half_sweep<T>(rb0_view(L), nc, b, x, col, s);
}

// first level handled by the one-work-group tail: the largest set of coarsest levels whose
// viscous (three-component) data fit in the LDS budget
int tail_level(const Level* lev, int nlev) {
    int t = nlev - 1;
    while (t > 0 && nlev - (t - 1) <= TAIL_MAXL &&
           tail_layout(lev, nlev, t - 1, 3, nullptr) <= TAIL_LDS_BYTES)
        t--;
    return t;
}

struct VArgs {
    Level* lev;
    int nlev, nc, nu1, nu2, nbottom;
    bool mixed;
    hipStream_t s;
    int tail;
    bool tail_fits;  // the tail levels fit the LDS budget (else per-level kernels)
};

// In mixed mode the levels whose sweeps move enough bytes to be bandwidth-bound run in FP32;
// below that size a sweep costs its launch and latency whatever the precision, and FP64 keeps the
// preconditioner closer to the FP64 one (fewer Krylov iterations).  The tail (and so the
// coarsest solve) is always FP64.
constexpr long F32_MIN_CELLS = 1L << 18;  // 64^3
bool level_f32(const VArgs& a, int l) {
    return a.mixed && l < a.tail && a.lev[l].N >= F32_MIN_CELLS;
}

void launch_tail(const VArgs& a) {
    TailArgs T;
    T.nl = a.nlev - a.tail;
    T.nu1 = a.nu1;
    T.nu2 = a.nu2;
    T.nbottom = a.nbottom;
    for (int q = 0; q < T.nl; q++) T.L[q] = a.lev[a.tail + q].v64();
    T.x0 = a.lev[a.tail].x;
    T.gate = a.lev[a.tail].gate;
    T.b0 = a.lev[a.tail].b;
    T.pack = a.lev[a.tail].pack;
    size_t bytes = tail_layout(a.lev, a.nlev, a.tail, a.nc, &T);
    if (a.nc == 3) k_vcycle_tail<3><<<1, TAIL_THREADS, bytes, a.s>>>(T);
    else k_vcycle_tail<1><<<1, TAIL_THREADS, bytes, a.s>>>(T);
}

template <typename T>
T* xl(Level& L);
template <>
double* xl<double>(Level& L) { return L.x; }
template <>
float* xl<float>(Level& L) { return L.xf; }
template <typename T>
T* bl(Level& L);
template <>
double* bl<double>(Level& L) { return L.b; }
template <>
float* bl<float>(Level& L) { return L.bf; }

void vcycle_rec(const VArgs& a, int l);

// whether level l's first pre-smoothing pass is carried by the restriction into it (a level
// with pre-smoothing below level 0 that is neither the coarsest nor run by the tail kernel)
bool first_fused(const VArgs& a, int l) {
    return l >= 1 && l < a.nlev - 1 && a.nu1 >= 1 && !(l >= a.tail && a.tail_fits);
}
// the fused first pass into level l (in level l's precision), or none
template <typename TC>
FirstV<TC> first_into(const VArgs& a, int l);
template <>
FirstV<double> first_into<double>(const VArgs& a, int l) {
    if (!first_fused(a, l)) return FirstV<double>{nullptr, nullptr};
    return FirstV<double>{a.lev[l].x, a.lev[l].D};
}
template <>
FirstV<float> first_into<float>(const VArgs& a, int l) {
    if (!first_fused(a, l)) return FirstV<float>{nullptr, nullptr};
    return FirstV<float>{a.lev[l].xf, a.lev[l].Df};
}

template <typename T>
void vcycle_level(const VArgs& a, int l) {
    Level& L = a.lev[l];
    T* x = xl<T>(L);
    T* b = bl<T>(L);
    if (l == a.nlev - 1 || a.nu1 < 1)
        k_zero<T><<<grid_for(a.nc * L.N), EB_BLOCK, 0, a.s>>>(a.nc * L.N, x, L.gate);
    if (l == a.nlev - 1) {
        for (int t = 0; t < a.nbottom; t++) {
            smooth_pass<T>(L, a.nc, b, x, 0, a.s);
            smooth_pass<T>(L, a.nc, b, x, 1, a.s);
        }
        for (int t = 0; t < a.nbottom; t++) {
            smooth_pass<T>(L, a.nc, b, x, 1, a.s);
            smooth_pass<T>(L, a.nc, b, x, 0, a.s);
        }
        return;
    }
    for (int t = 0; t < a.nu1; t++) {
        if (t == 0) {
            if (!first_fused(a, l)) first_pass<T>(L, a.nc, b, x, a.s);
        } else {
            smooth_pass<T>(L, a.nc, b, x, 0, a.s);
        }
        smooth_pass<T>(L, a.nc, b, x, 1, a.s);
    }
    Level& C = a.lev[l + 1];
    if (level_f32(a, l + 1))
        resid_restrict_pass<T, float>(L, C, a.nc, b, x, C.bf, first_into<float>(a, l + 1), a.s);
    else
        resid_restrict_pass<T, double>(L, C, a.nc, b, x, C.b, first_into<double>(a, l + 1), a.s);
    vcycle_rec(a, l + 1);
    bool cf32 = level_f32(a, l + 1);
    if (a.nu2 < 1) {
        if (cf32) prolong_pass<float, T>(L, C, a.nc, C.xf, x, a.s);
        else prolong_pass<double, T>(L, C, a.nc, C.x, x, a.s);
    }
    for (int t = 0; t < a.nu2; t++) {
        if (t == 0) {
            if (cf32) smooth_pro_pair<T, float>(L, C, a.nc, b, x, C.xf, a.s);
            else smooth_pro_pair<T, double>(L, C, a.nc, b, x, C.x, a.s);
            continue;
        }
        smooth_pass<T>(L, a.nc, b, x, 1, a.s);
        smooth_pass<T>(L, a.nc, b, x, 0, a.s);
    }
}

void vcycle_rec(const VArgs& a, int l) {
    if (l == a.tail && a.tail_fits) launch_tail(a);
    else if (level_f32(a, l)) vcycle_level<float>(a, l);
    else vcycle_level<double>(a, l);
}

// level 0's residual restricted to level 1 (with level 1's fused first pass): after
// pre-smoothing, which ends with a colour-1 half sweep, only colour-0 cells are evaluated
template <typename T, typename TC>
void resid_restrict_rb(const VArgs& a, const Rb0V& v, const Level& C, const T* b, const T* x,
                       TC* bc, FirstV<TC> F1) {
    unsigned gc = grid_for(C.N, RR_COARSE);
    int nc = a.nc;
    if (a.nu1 >= 1) {
        if (nc == 3) k_resid_restrict_rb0<T, TC, 3><<<gc, RR0_THREADS, 0, a.s>>>(v, b, x, C.grid, C.mask, bc, F1);
        else k_resid_restrict_rb0<T, TC, 1><<<gc, RR0_THREADS, 0, a.s>>>(v, b, x, C.grid, C.mask, bc, F1);
    } else {
        if (nc == 3) k_resid_restrict_rb<T, TC, 3><<<gc, RR_THREADS, 0, a.s>>>(v, b, x, C.grid, C.mask, bc, F1);
        else k_resid_restrict_rb<T, TC, 1><<<gc, RR_THREADS, 0, a.s>>>(v, b, x, C.grid, C.mask, bc, F1);
    }
}

// level 0's prolongation and post-smoothing: the prolongation of ec rides on the first pair of
// half sweeps (a pass of its own only without post-smoothing); the last half sweep writes the
// natural-order FP64 result x0
template <typename T, typename TC, typename TD>
void up_leg_rb(const VArgs& a, const Rb0V& v, const GridV& gc, const TC* ec, const T* b, T* x,
               TD* x0) {
    int nc = a.nc;
    long N = v.N;
    unsigned gh = grid_for(N / 2);
    ProV<TC> P{gc, ec}, none{gc, nullptr};
    if (a.nu2 < 1) {
        unsigned gf = grid_for(N);
        if (nc == 3) k_prolong_rb<TC, T, 3><<<gf, EB_BLOCK, 0, a.s>>>(v, gc, ec, x);
        else k_prolong_rb<TC, T, 1><<<gf, EB_BLOCK, 0, a.s>>>(v, gc, ec, x);
        return;
    }
    for (int t = 0; t < a.nu2; t++) {
        bool first = t == 0, last = t == a.nu2 - 1;
        if (first) {
            if (nc == 3) k_smooth_rb_pro<T, TC, 3, PRO_NBR><<<gh, EB_BLOCK, 0, a.s>>>(v, b, x, 1, P);
            else k_smooth_rb_pro<T, TC, 1, PRO_NBR><<<gh, EB_BLOCK, 0, a.s>>>(v, b, x, 1, P);
        } else {
            rb_half_sweep<T>(v, nc, b, x, 1, a.s);
        }
        if (last && first) {
            if (nc == 3) k_smooth_last_rb_to<T, 3, PRO_OWN, TC, TD><<<gh, EB_BLOCK, 0, a.s>>>(v, b, x, x0, P);
            else k_smooth_last_rb_to<T, 1, PRO_OWN, TC, TD><<<gh, EB_BLOCK, 0, a.s>>>(v, b, x, x0, P);
        } else if (last) {
            if (nc == 3) k_smooth_last_rb_to<T, 3, PRO_NONE, TC, TD><<<gh, EB_BLOCK, 0, a.s>>>(v, b, x, x0, none);
            else k_smooth_last_rb_to<T, 1, PRO_NONE, TC, TD><<<gh, EB_BLOCK, 0, a.s>>>(v, b, x, x0, none);
        } else if (first) {
            rb_half_sweep_pro<T, TC, PRO_OWN>(v, nc, b, x, 0, P, a.s);
        } else {
            rb_half_sweep<T>(v, nc, b, x, 0, a.s);
        }
    }
}

// level 0 of a V-cycle in colour-split storage (it is neither the coarsest nor a tail level):
// b and x are the level's own colour-split arrays
// b0, x0: the caller's natural-order FP64 right-hand side and output; b, x: the level's
// colour-split arrays (precision T).  The conversions ride on the first and last passes.
template <typename T, typename TD>
void vcycle_level0_rb(const VArgs& a, const double* b0, TD* x0, T* b, T* x) {
    Level& L = a.lev[0];
    Level& C = a.lev[1];
    Rb0V v = rb0_view(L);
    int nc = a.nc;
    unsigned g = grid_for(L.N);
    if (a.nu1 < 1) {
        if (nc == 3) k_to_rb<double, T, 3><<<g, EB_BLOCK, 0, a.s>>>(L.grid, L.N, b0, b, L.gate);
        else k_to_rb<double, T, 1><<<g, EB_BLOCK, 0, a.s>>>(L.grid, L.N, b0, b, L.gate);
        k_zero<T><<<grid_for(nc * L.N), EB_BLOCK, 0, a.s>>>(nc * L.N, x, L.gate);
    }
    for (int t = 0; t < a.nu1; t++) {
        if (t == 0) {
            // one thread per slot of both colours
            unsigned gh = grid_for(L.N / 2);
            if (nc == 3) k_smooth_first_rb_from<T, 3><<<gh, EB_BLOCK, 0, a.s>>>(v, b0, b, x);
            else k_smooth_first_rb_from<T, 1><<<gh, EB_BLOCK, 0, a.s>>>(v, b0, b, x);
            // colour 1 of the first iterate is still unset: this sweep writes all of it
            ProV<T> Z{L.grid, nullptr};
            rb_half_sweep_pro<T, T, PRO_ZERO>(v, nc, b, x, 1, Z, a.s);
            continue;
        }
        smooth_rb_pass<T>(L, nc, b, x, 0, a.s);
        smooth_rb_pass<T>(L, nc, b, x, 1, a.s);
    }
    bool cf32 = level_f32(a, 1);
    if (cf32) resid_restrict_rb<T, float>(a, v, C, b, x, C.bf, first_into<float>(a, 1));
    else resid_restrict_rb<T, double>(a, v, C, b, x, C.b, first_into<double>(a, 1));
    vcycle_rec(a, 1);
    if (cf32) up_leg_rb<T, float, TD>(a, v, C.grid, C.xf, b, x, x0);
    else up_leg_rb<T, double, TD>(a, v, C.grid, C.x, b, x, x0);
    if (a.nu2 < 1) {
        if (nc == 3) k_from_rb<T, TD, 3><<<g, EB_BLOCK, 0, a.s>>>(L.grid, L.N, x, x0, L.gate);
        else k_from_rb<T, TD, 1><<<g, EB_BLOCK, 0, a.s>>>(L.grid, L.N, x, x0, L.gate);
    }
}

template <typename T, typename TD>
void vcycle_rb(const VArgs& a, const double* b, TD* x, T* brb, T* xrb) {
    vcycle_level0_rb<T, TD>(a, b, x, brb, xrb);
}

void tail_pack(const Level* lev, int nlev, hipStream_t s) {
    int t = tail_level(lev, nlev);
    TailArgs A;
    tail_layout(lev, nlev, t, 1, &A);
    // a tail kernel runs only when its whole layout fits, so its operator part always does
    if (A.nstatic > MG_PACK_BYTES || !lev[t].pack) return;
    PackArgs P;
    P.nseg = 0;
    P.pack = lev[t].pack;
    for (int l = t; l < nlev; l++) {
        const Level& L = lev[l];
        int q = l - t;
        for (int d = 0; d < 3; d++) {
            P.src[P.nseg] = reinterpret_cast<const char*>(L.K[d]);
            P.dst[P.nseg] = A.oK[q][d];
            P.bytes[P.nseg++] = (unsigned)(face_count(L.grid, d) * 8);
        }
        P.src[P.nseg] = reinterpret_cast<const char*>(L.D);
        P.dst[P.nseg] = A.oD[q];
        P.bytes[P.nseg++] = (unsigned)(L.N * 8);
        P.src[P.nseg] = reinterpret_cast<const char*>(L.mask);
        P.dst[P.nseg] = A.om[q];
        P.bytes[P.nseg++] = (unsigned)L.N;
    }
    k_tail_pack<<<P.nseg, EB_BLOCK, 0, s>>>(P);
}

void finish_operator(Level* lev, int nlev, bool mixed, hipStream_t s) {
    int tail = tail_level(lev, nlev);
    for (int l = 1; l < nlev; l++) {
        const Level& F = lev[l - 1];
        Level& C = lev[l];
        CoarsenArgs A;
        A.gc = C.grid;
        A.gf = F.grid;
        for (int d = 0; d < 3; d++) {
            A.Kf[d] = F.K[d];
            A.apf[d] = F.ap[d];
            A.Kc[d] = C.K[d];
            A.n[d] = face_count(C.grid, d);
        }
        A.series = lev[0].sys == EB_SYS_VISC;
        A.Sf = F.S;
        A.Sc = C.S;
        A.scale = 1.0 / 16.0;
        A.maskf = F.mask;
        A.Df = F.D;
        A.n[3] = C.N;
        A.n[4] = F.N;
        k_coarsen_level<<<grid_for(A.n[0] + A.n[1] + A.n[2] + A.n[3] + A.n[4]), EB_BLOCK, 0, s>>>(A);
    }
    {
        Level& L = lev[nlev - 1];
        k_diag<<<grid_for(L.N), EB_BLOCK, 0, s>>>(L.grid, L.K[0], L.K[1], L.K[2], L.S, L.mask,
                                                  L.D);
    }
    for (int l = 0; l < nlev; l++) {
        Level& L = lev[l];
        if (mixed && l < tail && L.N >= F32_MIN_CELLS) {
            for (int d = 0; d < 3; d++) {
                long nf = face_count(L.grid, d);
                k_to_float<<<grid_for(nf), EB_BLOCK, 0, s>>>(nf, L.K[d], L.Kf[d]);
            }
            k_to_float<<<grid_for(L.N), EB_BLOCK, 0, s>>>(L.N, L.D, L.Df);
        }
    }
    tail_pack(lev, nlev, s);
}

}  // namespace

void mg_build_poisson(Level* lev, int nlev, const GeomV& g, double beta, bool mixed,
                      hipStream_t s) {
    lev[0].flag = g.flag;
    lev[0].cut = g.cut;
    lev[0].ncut = g.ncut;
    lev[0].eta = nullptr;
    if (lev[0].flagcs && (g.grid.n[0] & 1) == 0)
        k_to_rb<uint8_t, uint8_t, 1><<<grid_for(g.N), EB_BLOCK, 0, s>>>(g.grid, g.N, g.flag,
                                                                        lev[0].flagcs, nullptr);
    lev[0].sys = EB_SYS_POISSON;
    lev[0].beta = beta;
    for (int d = 0; d < 3; d++)
        k_K_poisson<<<grid_for(face_count(g.grid, d)), EB_BLOCK, 0, s>>>(g, d, beta, lev[0].K[d]);
    k_zero<double><<<grid_for(g.N), EB_BLOCK, 0, s>>>(g.N, lev[0].S);
    finish_operator(lev, nlev, mixed, s);
}

void mg_build_visc(Level* lev, int nlev, const GeomV& g, double rho, double dt,
                   const double* eta, const double* eta_eb, bool mixed, hipStream_t s) {
    lev[0].flag = g.flag;
    lev[0].cut = g.cut;
    lev[0].ncut = g.ncut;
    lev[0].eta = eta;
    if (lev[0].flagcs && lev[0].etacs && (g.grid.n[0] & 1) == 0) {
        k_to_rb<uint8_t, uint8_t, 1><<<grid_for(g.N), EB_BLOCK, 0, s>>>(g.grid, g.N, g.flag,
                                                                        lev[0].flagcs, nullptr);
        k_to_rb<double, double, 1><<<grid_for(g.N), EB_BLOCK, 0, s>>>(g.grid, g.N, eta,
                                                                      lev[0].etacs, nullptr);
    }
    lev[0].sys = EB_SYS_VISC;
    lev[0].rho = rho;
    lev[0].dt = dt;
    if (mixed && lev[0].etaf)
        k_to_float<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g.N, eta, lev[0].etaf);
    if (mixed && lev[0].etafcs && (g.grid.n[0] & 1) == 0)
        k_to_rb<double, float, 1><<<grid_for(g.N), EB_BLOCK, 0, s>>>(g.grid, g.N, eta,
                                                                     lev[0].etafcs, nullptr);
    for (int d = 0; d < 3; d++)
        k_K_visc<<<grid_for(face_count(g.grid, d)), EB_BLOCK, 0, s>>>(g, d, dt, eta, lev[0].K[d]);
    k_S_visc<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, rho, dt, eta_eb, lev[0].S);
    finish_operator(lev, nlev, mixed, s);
}

void mg_vcycle(Level* lev, int nlev, int ncomp, bool mixed, const double* b, double* x, int nu1,
               int nu2, int nbottom, hipStream_t s, const int* gate) {
    for (int l = 0; l < nlev; l++) lev[l].gate = gate;
    int tl = tail_level(lev, nlev);
    VArgs a{lev, nlev, ncomp, nu1, nu2, nbottom, mixed, s, tl,
            tail_layout(lev, nlev, tl, ncomp, nullptr) <= TAIL_LDS_BYTES};
    Level& L0 = lev[0];
    long n = (long)ncomp * L0.N;
    if (nlev > 1 && !(a.tail == 0 && a.tail_fits) && L0.flag) {
        // the finest level in colour-split storage (its own arrays)
        if (level_f32(a, 0)) vcycle_rb<float, double>(a, b, x, L0.bf, L0.xf);
        else vcycle_rb<double, double>(a, b, x, L0.b, L0.x);
        for (int l = 0; l < nlev; l++) lev[l].gate = nullptr;
        return;
    }
    // level 0 works on the caller's arrays in FP64 mode; in mixed mode on FP32 copies
    double* keep_b = L0.b;
    double* keep_x = L0.x;
    if (level_f32(a, 0)) {
        k_cast<double, float><<<grid_for(n), EB_BLOCK, 0, s>>>(n, b, L0.bf, gate);
        vcycle_rec(a, 0);
        k_cast<float, double><<<grid_for(n), EB_BLOCK, 0, s>>>(n, L0.xf, x, gate);
    } else {
        L0.b = const_cast<double*>(b);
        L0.x = x;
        vcycle_rec(a, 0);
        L0.b = keep_b;
        L0.x = keep_x;
    }
    for (int l = 0; l < nlev; l++) lev[l].gate = nullptr;
}

// the V-cycle's VArgs as mg_vcycle forms them
VArgs vargs(Level* lev, int nlev, int ncomp, bool mixed, int nu1, int nu2, int nbottom,
            hipStream_t s) {
    int tl = tail_level(lev, nlev);
    return VArgs{lev, nlev, ncomp, nu1, nu2, nbottom, mixed, s, tl,
                 tail_layout(lev, nlev, tl, ncomp, nullptr) <= TAIL_LDS_BYTES};
}

bool mg_vcycle_f32_out(Level* lev, int nlev, int ncomp, bool mixed, int nu1, int nu2) {
    VArgs a = vargs(lev, nlev, ncomp, mixed, nu1, nu2, 0, nullptr);
    return nlev > 1 && !(a.tail == 0 && a.tail_fits) && lev[0].flag && level_f32(a, 0);
}

void mg_vcycle(Level* lev, int nlev, int ncomp, bool mixed, const double* b, float* x, int nu1,
               int nu2, int nbottom, hipStream_t s, const int* gate) {
    for (int l = 0; l < nlev; l++) lev[l].gate = gate;
    VArgs a = vargs(lev, nlev, ncomp, mixed, nu1, nu2, nbottom, s);
    vcycle_rb<float, float>(a, b, x, lev[0].bf, lev[0].xf);
    for (int l = 0; l < nlev; l++) lev[l].gate = nullptr;
}

void mg_sweep_level0(const Level& L, int ncomp, bool f32, const void* b, void* x, int colour,
                     hipStream_t s) {
    if (f32)
        smooth_rb_pass<float>(L, ncomp, (const float*)b, (float*)x, colour, s);
    else
        smooth_rb_pass<double>(L, ncomp, (const double*)b, (double*)x, colour, s);
}

void mg_apply_level0(const Level& L, int ncomp, const double* x, double* y, hipStream_t s,
                     const int* gate) {
    Rb0V v = rb0_view(L);
    v.gate = gate;
    auto al = [](const void* q) { return reinterpret_cast<uintptr_t>(q) % 16 == 0; };
    if (ncomp == 1 && v.sys == EB_SYS_POISSON && al(x) && al(y)) {
        unsigned gp = grid_for(L.N / 2, PAIR_BLOCK);
        unsigned gc = v.ncut > 0 ? (grid_for(v.ncut, PAIR_BLOCK) + 7) & ~7u : 0;
        k_apply0_pair<<<gc + gp, PAIR_BLOCK, 0, s>>>(v, x, y, gc);
    } else if (ncomp == 3) {
        k_apply0<3><<<grid_for(L.N), EB_BLOCK, 0, s>>>(v, x, y);
    } else {
        k_apply0<1><<<grid_for(L.N), EB_BLOCK, 0, s>>>(v, x, y);
    }
}

template <typename TU>
void op_visc_apply_t(const GeomV& g, double rho, double dt, const double* eta,
                     const double* eta_eb, const TU* u, double* out, int homogeneous,
                     hipStream_t s, const int* gate) {
    double h2 = g.grid.h * g.grid.h;
    double kin = dt * 0.5 / h2, kwall = 2.0 * dt / h2;
    FastDiv dnx = fast_div((unsigned)g.grid.n[0]), dny = fast_div((unsigned)g.grid.n[1]);
    bool pair = false;
    {
        // the pair kernel reads eta and u in aligned pairs (one-cell kernel otherwise)
        auto al = [](const void* q, size_t a) { return reinterpret_cast<uintptr_t>(q) % a == 0; };
        if (al(eta, 16) && al(u, 2 * sizeof(TU))) {
            unsigned gp = grid_for(g.N / 2, PAIR_BLOCK);
            unsigned gc = g.ncut > 0 ? (grid_for(g.ncut, PAIR_BLOCK) + 7) & ~7u : 0;
            k_visc_apply<TU><<<gc + gp, PAIR_BLOCK, 0, s>>>(g, rho, dt, kin, kwall, dnx, dny,
                                                            eta, u, out, homogeneous, gate, gc);
            pair = true;
        }
    }
    if (!pair)
        k_visc_apply_one<TU><<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, rho, dt, kin, kwall, dnx, dny,
                                                               eta, u, out, homogeneous, gate);
    if (g.ncut > 0)
        k_visc_apply_eb<TU><<<grid_for(g.ncut), EB_BLOCK, 0, s>>>(g, dt, eta_eb, u, out,
                                                                homogeneous, gate);
}
void op_visc_apply(const GeomV& g, double rho, double dt, const double* eta,
                   const double* eta_eb, const double* u, double* out, int homogeneous,
                   hipStream_t s, const int* gate) {
    op_visc_apply_t<double>(g, rho, dt, eta, eta_eb, u, out, homogeneous, s, gate);
}
void op_visc_apply(const GeomV& g, double rho, double dt, const double* eta,
                   const double* eta_eb, const float* u, double* out, int homogeneous,
                   hipStream_t s, const int* gate) {
    op_visc_apply_t<float>(g, rho, dt, eta, eta_eb, u, out, homogeneous, s, gate);
}

// ------------------------------------------------------------------------------------------
// reductions: results land in out (device); the caller copies what it needs to the host
// ------------------------------------------------------------------------------------------
int red_blocks(long n) {
    long b = (n + EB_BLOCK - 1) / EB_BLOCK;
    if (b > RED_MAXB) b = RED_MAXB;
    return (int)(b < 1 ? 1 : b);
}

void dots_launch(long n, int np, const DotArgs& args, double* part, const int* gate, int nb,
                 hipStream_t s) {
    switch (np) {
        case 1: k_dots<1><<<nb, EB_BLOCK, 0, s>>>(n, args, part, gate); break;
        case 2: k_dots<2><<<nb, EB_BLOCK, 0, s>>>(n, args, part, gate); break;
        case 3: k_dots<3><<<nb, EB_BLOCK, 0, s>>>(n, args, part, gate); break;
        default: k_dots<4><<<nb, EB_BLOCK, 0, s>>>(n, args, part, gate); break;
    }
}

void red_dots(long n, int np, const double* const a[4], const double* const b[4], double* part,
              double* out, hipStream_t s, const int* gate) {
    DotArgs args;
    for (int p = 0; p < 4; p++) {
        args.a[p] = p < np ? a[p] : nullptr;
        args.b[p] = p < np ? b[p] : nullptr;
    }
    int nb = red_blocks(n);
    dots_launch(n, np, args, part, gate, nb, s);
    k_final<<<1, EB_BLOCK, 0, s>>>(part, nb, np, 0, out, gate);
}

void red_dots_op(long n, int np, const double* const a[4], const double* const b[4],
                 double* part, int out_idx, int op, double* ks, int* st, int* itc,
                 hipStream_t s) {
    DotArgs args;
    OpOut o;
    for (int p = 0; p < 4; p++) {
        args.a[p] = p < np ? a[p] : nullptr;
        args.b[p] = p < np ? b[p] : nullptr;
        o.idx[p] = out_idx + p;
    }
    o.maxmask = 0;
    int nb = red_blocks(n);
    dots_launch(n, np, args, part, st, nb, s);
    k_final_op<<<1, EB_BLOCK, 0, s>>>(part, nb, np, o, op, ks, st, itc);
}

void ks_bi_s_op(long n, double* sv, const double* r, const double* v, double* part, double* ks,
                int* st, int* itc, hipStream_t s) {
    OpOut o = {{KS_SN, 0, 0, 0}, 1};
    int nb = red_blocks(n);
    k_bi_s_max<<<nb, EB_BLOCK, 0, s>>>(n, sv, r, v, ks, st, part);
    k_final_op<<<1, EB_BLOCK, 0, s>>>(part, nb, 1, o, KS_BI_CHECK_S, ks, st, itc);
}

template <typename TP>
void ks_bi_xr_op_t(long n, double* x, double* r, const TP* ph, const TP* sh, const double* sv,
                   const double* t, const double* rh, double* part, double* ks, int* st,
                   int* itc, hipStream_t s) {
    OpOut o = {{KS_RRN, KS_RN, 0, 0}, 2};
    int nb = red_blocks(n);
    k_bi_xr_red<TP><<<nb, EB_BLOCK, 0, s>>>(n, x, r, ph, sh, sv, t, rh, ks, st, part);
    k_final_op<<<1, EB_BLOCK, 0, s>>>(part, nb, 2, o, KS_BI_CHECK_R, ks, st, itc);
}
void ks_bi_xr_op(long n, double* x, double* r, const double* ph, const double* sh,
                 const double* sv, const double* t, const double* rh, double* part, double* ks,
                 int* st, int* itc, hipStream_t s) {
    ks_bi_xr_op_t<double>(n, x, r, ph, sh, sv, t, rh, part, ks, st, itc, s);
}
void ks_bi_xr_op(long n, double* x, double* r, const float* ph, const float* sh,
                 const double* sv, const double* t, const double* rh, double* part, double* ks,
                 int* st, int* itc, hipStream_t s) {
    ks_bi_xr_op_t<float>(n, x, r, ph, sh, sv, t, rh, part, ks, st, itc, s);
}

void ks_cg_xr_op(long n, double* x, double* r, const double* p, const double* q, double* part,
                 double* ks, int* st, int* itc, hipStream_t s) {
    OpOut o = {{KS_RN, 0, 0, 0}, 1};
    int nb = red_blocks(n);
    k_cg_xr_max<<<nb, EB_BLOCK, 0, s>>>(n, x, r, p, q, ks, st, part);
    k_final_op<<<1, EB_BLOCK, 0, s>>>(part, nb, 1, o, KS_CHECK_R, ks, st, itc);
}

void red_maxabs(long n, int ncomp, const double* x, double* part, double* out, hipStream_t s,
                const int* gate) {
    int nb = red_blocks(n);
    k_maxabs<<<nb, EB_BLOCK, 0, s>>>(n, ncomp, x, part, gate);
    k_final<<<1, EB_BLOCK, 0, s>>>(part, nb, ncomp, 1, out, gate);
}

void red_cfl(const GeomV& g, const double* u, const double* theta, double* part, double* out,
             hipStream_t s) {
    int nb = red_blocks(g.N);
    k_cfl_max<<<nb, EB_BLOCK, 0, s>>>(g, u, theta, part);
    k_final<<<1, EB_BLOCK, 0, s>>>(part, nb, 2, 1, out, nullptr);
}

void red_sum_open(const GeomV& g, const double* x, double* part, double* out, hipStream_t s,
                  const int* gate) {
    int nb = red_blocks(g.N);
    k_sum_open<<<nb, EB_BLOCK, 0, s>>>(g, x, part, gate);
    k_final<<<1, EB_BLOCK, 0, s>>>(part, nb, 2, 0, out, gate);
}

void red_final(const double* part, int nb, int nrow, int mode, double* out, hipStream_t s,
               const int* gate) {
    k_final<<<1, EB_BLOCK, 0, s>>>(part, nb, nrow, mode, out, gate);
}

void red_sum(long n, int nrow, const double* x, double* part, double* out, hipStream_t s) {
    int nb = red_blocks(n);
    k_rowsum<<<nb, EB_BLOCK, 0, s>>>(n, nrow, x, part);
    k_final<<<1, EB_BLOCK, 0, s>>>(part, nb, nrow, 0, out, nullptr);
}

void op_face_flux_max(const GeomV& g, double* const f[3], double* part, double* out,
                      hipStream_t s) {
    long n = face_count(g.grid, 0);
    int nb = red_blocks(n);
    k_face_flux_max<<<nb, EB_BLOCK, 0, s>>>(g, f[0], f[1], f[2], part);
    k_final<<<1, EB_BLOCK, 0, s>>>(part, nb, 1, 1, out, nullptr);
}

void vec_copy(long n, const double* x, double* y, hipStream_t s) {
    if (n > 0) k_copy<<<grid_for(n), EB_BLOCK, 0, s>>>(n, x, y);
}
void vec_fill(long n, double v, double* y, hipStream_t s) {
    if (n > 0) k_fill<<<grid_for(n), EB_BLOCK, 0, s>>>(n, v, y);
}
void vec_axpby(long n, double a, const double* x, double b, double* y, hipStream_t s) {
    k_axpby<<<grid_for(n), EB_BLOCK, 0, s>>>(n, a, x, b, y);
}
void vec_bicg_p(long n, const double* r, double beta, double omega, const double* v, double* p,
                hipStream_t s) {
    k_bicg_p<<<grid_for(n), EB_BLOCK, 0, s>>>(n, r, beta, omega, v, p);
}
void vec_sub_scaled(long n, const double* x, double a, const double* y, double* z,
                    hipStream_t s) {
    k_sub_scaled<<<grid_for(n), EB_BLOCK, 0, s>>>(n, x, a, y, z);
}
void vec_bicg_update(long n, double al, const double* ph, double om, const double* sh,
                     const double* sv, const double* t, double* x, double* r, hipStream_t s) {
    k_bicg_update<<<grid_for(n), EB_BLOCK, 0, s>>>(n, al, ph, om, sh, sv, t, x, r);
}
void vec_mask_rhs(const GeomV& g, const double* psi, const double* a0, double* b,
                  hipStream_t s) {
    k_mask_rhs<<<grid_for(3 * g.N), EB_BLOCK, 0, s>>>(g, psi, a0, b);
}

bool mg_level0_f32(const Level* lev, int nlev) {
    return tail_level(lev, nlev) > 0 && lev[0].N >= F32_MIN_CELLS;
}
