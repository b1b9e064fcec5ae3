// eb_mg.hip -- geometric multigrid preconditioner, the exact EB viscous operator, reductions
// and Krylov vector kernels.
//
// Level operators are 7-point and symmetric: (M x)_c = D_c x_c - sum_f K_f x_nb(f), where a
// face on a Dirichlet domain wall only adds its K to D.  Level 0 takes its face coefficients
// from the apertures (Poisson) or apertures and face viscosities (viscous); coarse levels
// average four child faces (and rescale by 1/4 for the doubled spacing) and eight child
// cell shifts.  Smoothing is red-black Gauss-Seidel; within a colour every update depends only
// on the other colour, so the result does not depend on thread order.
#include "eb_internal.hpp"

namespace {

// ------------------------------------------------------------------------------------------
// operator construction
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void face_ijk(const GridV& g, int d, long f, int& i, int& j, int& k) {
    int m0 = g.n[0] + (d == 0), m1 = g.n[1] + (d == 1);
    i = (int)(f % m0);
    long r = f / m0;
    j = (int)(r % m1);
    k = (int)(r / m1);
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
            double del = g.delta[q] > 0.5 ? g.delta[q] : 0.5;
            v += dt * g.aeb[q] * eta_eb[q] / (del * g.grid.h * g.grid.h);
        }
    }
    S[c] = v;
}

__global__ void k_diag(GridV g, const double* __restrict__ Kx, const double* __restrict__ Ky,
                       const double* __restrict__ Kz, const double* __restrict__ S,
                       const uint8_t* __restrict__ mask, double* __restrict__ D) {
    long N = (long)g.n[0] * g.n[1] * g.n[2];
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    if (!mask[c]) {
        D[c] = 0.0;
        return;
    }
    int i, j, k;
    cell_coords(g, c, i, j, k);
    const double* K[3] = {Kx, Ky, Kz};
    double s = S ? S[c] : 0.0;
    for (int d = 0; d < 3; d++) {
        int q[3] = {i, j, k};
        s += K[d][face_index(g, d, q[0], q[1], q[2])];
        q[d] += 1;
        s += K[d][face_index(g, d, q[0], q[1], q[2])];
    }
    D[c] = s;
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
#pragma unroll
    for (int d = 0; d < 3; d++) {
#pragma unroll
        for (int side = 0; side < 2; side++) {
            int f[3] = {i, j, k};
            f[d] += side;
            T K = L.K[d][face_index(g, d, f[0], f[1], f[2])];
            if (K == (T)0) continue;
            int q[3] = {i, j, k};
            q[d] += side ? 1 : -1;
            long nb = cell_at(g, q[0], q[1], q[2]);
            if (nb < 0) continue;
#pragma unroll
            for (int m = 0; m < NC; m++) acc[m] += K * x[m * N + nb];
        }
    }
}

// one Gauss-Seidel update of the t-th cell of colour col (cells of a colour are numbered row by
// row, nx/2 per row)
template <typename T, int NC>
__device__ __forceinline__ void smooth_cell(const LevelV<T>& L, const T* __restrict__ b,
                                            T* __restrict__ x, long t, int col) {
    const GridV& g = L.grid;
    int nxh = g.n[0] / 2;
    long row = t / nxh;
    int ih = (int)(t - row * nxh);
    int j = (int)(row % g.n[1]);
    int k = (int)(row / g.n[1]);
    int i = 2 * ih + ((j + k + col) & 1);
    long c = cell_index(g, i, j, k);
    if (!L.mask[c]) return;
    T dg = L.D[c];
    if (!(dg > (T)0)) return;
    T acc[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) acc[m] = b[m * L.N + c];
    offdiag<T, NC>(L, x, i, j, k, acc);
#pragma unroll
    for (int m = 0; m < NC; m++) x[m * L.N + c] = acc[m] / dg;
}

// r = b - M x at cell c (b null: r = M x)
template <typename T, int NC>
__device__ __forceinline__ void resid_cell(const LevelV<T>& L, const T* __restrict__ b,
                                           const T* __restrict__ x, T* __restrict__ r, long c) {
    if (!L.mask[c]) {
#pragma unroll
        for (int m = 0; m < NC; m++) r[m * L.N + c] = (T)0;
        return;
    }
    int i, j, k;
    cell_coords(L.grid, c, i, j, k);
    T acc[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) acc[m] = (T)0;
    offdiag<T, NC>(L, x, i, j, k, acc);
    T dg = L.D[c];
#pragma unroll
    for (int m = 0; m < NC; m++) {
        T mx = dg * x[m * L.N + c] - acc[m];
        r[m * L.N + c] = b ? b[m * L.N + c] - mx : mx;
    }
}

// coarse right-hand side: mean of the eight children (rows are already alpha-weighted)
template <typename TF, typename TC, int NC>
__device__ __forceinline__ void restrict_cell(const GridV& gf, const GridV& gc,
                                              const uint8_t* __restrict__ mf,
                                              const uint8_t* __restrict__ mc,
                                              const TF* __restrict__ rf, TC* __restrict__ bc,
                                              long c) {
    long Nc = (long)gc.n[0] * gc.n[1] * gc.n[2];
    long Nf = (long)gf.n[0] * gf.n[1] * gf.n[2];
    int i, j, k;
    cell_coords(gc, c, i, j, k);
    TF s[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) s[m] = (TF)0;
    for (int q = 0; q < 8; q++) {
        long f = cell_index(gf, 2 * i + (q & 1), 2 * j + ((q >> 1) & 1), 2 * k + (q >> 2));
        if (!mf[f]) continue;
#pragma unroll
        for (int m = 0; m < NC; m++) s[m] += rf[m * Nf + f];
    }
#pragma unroll
    for (int m = 0; m < NC; m++) bc[m * Nc + c] = mc[c] ? (TC)(s[m] / (TF)8) : (TC)0;
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

// residual of the fine level restricted to the coarse right-hand side in one pass
template <typename TF, typename TC, int NC>
__global__ void k_resid_restrict(LevelV<TF> L, const TF* __restrict__ b, const TF* __restrict__ x,
                                 GridV gc, const uint8_t* __restrict__ mc, TC* __restrict__ bc) {
    if (L.gate && *L.gate) return;
    long Nc = (long)gc.n[0] * gc.n[1] * gc.n[2];
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= Nc) return;
    int i, j, k;
    cell_coords(gc, c, i, j, k);
    TF s[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) s[m] = (TF)0;
    for (int q = 0; q < 8; q++) {
        int fi = 2 * i + (q & 1), fj = 2 * j + ((q >> 1) & 1), fk = 2 * k + (q >> 2);
        long f = cell_index(L.grid, fi, fj, fk);
        if (!L.mask[f]) continue;
        TF acc[NC];
#pragma unroll
        for (int m = 0; m < NC; m++) acc[m] = (TF)0;
        offdiag<TF, NC>(L, x, fi, fj, fk, acc);
        TF dg = L.D[f];
#pragma unroll
        for (int m = 0; m < NC; m++) s[m] += b[m * L.N + f] - (dg * x[m * L.N + f] - acc[m]);
    }
#pragma unroll
    for (int m = 0; m < NC; m++) bc[m * Nc + c] = mc[c] ? (TC)(s[m] / (TF)8) : (TC)0;
}

template <typename T, int NC>
__global__ void k_smooth(LevelV<T> L, const T* __restrict__ b, T* __restrict__ x, int col) {
    if (L.gate && *L.gate) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < L.N / 2) smooth_cell<T, NC>(L, b, x, t, col);
}

template <typename T, int NC>
__global__ void k_resid(LevelV<T> L, const T* __restrict__ b, const T* __restrict__ x,
                        T* __restrict__ r) {
    if (L.gate && *L.gate) return;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c < L.N) resid_cell<T, NC>(L, b, x, r, c);
}

template <typename TF, typename TC, int NC>
__global__ void k_restrict(GridV gf, GridV gc, const uint8_t* __restrict__ mf,
                           const uint8_t* __restrict__ mc, const TF* __restrict__ rf,
                           TC* __restrict__ bc, const int* gate) {
    if (gate && *gate) return;
    long Nc = (long)gc.n[0] * gc.n[1] * gc.n[2];
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c < Nc) restrict_cell<TF, TC, NC>(gf, gc, mf, mc, rf, bc, c);
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
// the small coarse levels of a V-cycle, all in one work-group (one launch instead of ~100):
// the same operations in the same order as the per-level kernels, separated by barriers.  The
// operators, right-hand sides and iterates of these levels are staged in LDS, so each of the
// ~100 barrier-separated phases costs LDS latency instead of a global-memory round trip.
// ------------------------------------------------------------------------------------------
constexpr int TAIL_MAXL = 8;
constexpr int TAIL_THREADS = 1024;
constexpr size_t TAIL_LDS_BYTES = 65536;

struct TailArgs {
    int nl, nu1, nu2, nbottom;
    LevelV<double> L[TAIL_MAXL];
    double* x0;        // iterate of the first tail level (global, written back)
    const int* gate;
    const double* b0;  // right-hand side of the first tail level (global)
    // LDS byte offsets per level: x, b, K[3], D, mask
    unsigned ox[TAIL_MAXL], ob[TAIL_MAXL], oK[TAIL_MAXL][3], oD[TAIL_MAXL], om[TAIL_MAXL];
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

template <int NC>
__global__ void __launch_bounds__(TAIL_THREADS) k_vcycle_tail(TailArgs A) {
    if (A.gate && *A.gate) return;
    extern __shared__ double lds_d[];
    char* lds = reinterpret_cast<char*>(lds_d);
    int nl = A.nl;
    // stage the operators and the first right-hand side in LDS
    for (int l = 0; l < nl; l++) {
        const LevelV<double>& G = A.L[l];
        for (int d = 0; d < 3; d++) {
            long nf = face_count(G.grid, d);
            double* dst = reinterpret_cast<double*>(lds + A.oK[l][d]);
            for (long t = threadIdx.x; t < nf; t += blockDim.x) dst[t] = G.K[d][t];
        }
        double* Dd = reinterpret_cast<double*>(lds + A.oD[l]);
        uint8_t* md = reinterpret_cast<uint8_t*>(lds + A.om[l]);
        for (long t = threadIdx.x; t < G.N; t += blockDim.x) {
            Dd[t] = G.D[t];
            md[t] = G.mask[t];
        }
    }
    {
        double* bd = reinterpret_cast<double*>(lds + A.ob[0]);
        for (long t = threadIdx.x; t < NC * A.L[0].N; t += blockDim.x) bd[t] = A.b0[t];
    }
    __syncthreads();
    auto lv = [&](int l) {
        LevelV<double> v = A.L[l];
        for (int d = 0; d < 3; d++) v.K[d] = reinterpret_cast<const double*>(lds + A.oK[l][d]);
        v.D = reinterpret_cast<const double*>(lds + A.oD[l]);
        v.mask = reinterpret_cast<const uint8_t*>(lds + A.om[l]);
        return v;
    };
    auto X = [&](int l) { return reinterpret_cast<double*>(lds + A.ox[l]); };
    auto B = [&](int l) { return reinterpret_cast<double*>(lds + A.ob[l]); };
    for (int l = 0; l < nl; l++) {
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
    for (int l = nl - 2; l >= 0; l--) {
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
    for (int l = t; l < nlev; l++) {
        const Level& L = lev[l];
        int q = l - t;
        unsigned ox = take(nc * L.N * 8), ob = take(nc * L.N * 8);
        unsigned oK[3];
        for (int d = 0; d < 3; d++) oK[d] = take(face_count(L.grid, d) * 8);
        unsigned oD = take(L.N * 8), om = take(L.N);
        if (A) {
            A->ox[q] = ox;
            A->ob[q] = ob;
            for (int d = 0; d < 3; d++) A->oK[q][d] = oK[d];
            A->oD[q] = oD;
            A->om[q] = om;
        }
    }
    return off;
}

// ------------------------------------------------------------------------------------------
// exact EB viscous Helmholtz operator (Eq. implicit-viscous with the wall flux of Eq. dudn)
// ------------------------------------------------------------------------------------------
__global__ void k_visc_apply(GeomV g, double rho, double dt, const double* __restrict__ eta,
                             const double* __restrict__ eta_eb, const double* __restrict__ u,
                             double* __restrict__ out, int homog, const int* gate) {
    if (gate && *gate) return;
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    double al = g.alpha[c];
    if (!(al > 0.0)) {
        for (int m = 0; m < 3; m++) out[m * N + c] = 0.0;
        return;
    }
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    double h2 = g.grid.h * g.grid.h;
    double acc[3];
    for (int m = 0; m < 3; m++) acc[m] = al * rho * u[m * N + c];
    double ec = eta[c];
    for (int d = 0; d < 3; d++)
        for (int side = 0; side < 2; side++) {
            int f[3] = {i, j, k};
            f[d] += side;
            double A = g.ap[d][face_index(g.grid, d, f[0], f[1], f[2])];
            if (A == 0.0) continue;
            int q[3] = {i, j, k};
            q[d] += side ? 1 : -1;
            long nb = cell_at(g.grid, q[0], q[1], q[2]);
            if (nb >= 0) {
                double K = dt * A * 0.5 * (ec + eta[nb]) / h2;
                for (int m = 0; m < 3; m++) acc[m] -= K * (u[m * N + nb] - u[m * N + c]);
            } else {
                double K = 2.0 * dt * A * ec / h2;
                for (int m = 0; m < 3; m++) {
                    double uw = homog ? 0.0 : g.wall[2 * d + side][m];
                    acc[m] -= K * (uw - u[m * N + c]);
                }
            }
        }
    int q = g.cutid[c];
    if (q >= 0) {
        int nc = g.ncut;
        double d1 = g.dd[q], d2 = g.dd[nc + q];
        double den = d1 * d2 * (d2 - d1) * g.grid.h;
        double coef = dt * g.aeb[q] * eta_eb[q] / g.grid.h;
        for (int m = 0; m < 3; m++) {
            double ue = homog ? 0.0 : g.ueb[m];
            double s1 = 0.0, s2 = 0.0;
            for (int t = 0; t < 9; t++) {
                int c1 = g.sidx[(long)t * nc + q];
                s1 += g.sw[(long)t * nc + q] * (c1 >= 0 ? u[m * N + c1] : ue);
                int c2 = g.sidx[(long)(t + 9) * nc + q];
                s2 += g.sw[(long)(t + 9) * nc + q] * (c2 >= 0 ? u[m * N + c2] : ue);
            }
            double gn = (d2 * d2 * (s1 - ue) - d1 * d1 * (s2 - ue)) / den;
            acc[m] += coef * gn;
        }
    }
    for (int m = 0; m < 3; m++) out[m * N + c] = acc[m];
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
        if (threadIdx.x < (unsigned)o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

struct DotArgs {
    const double* a[4];
    const double* b[4];
};

__global__ void k_dots(long n, int np, DotArgs args, double* __restrict__ part, const int* gate) {
    if (gate && *gate) return;
    __shared__ double sh[EB_BLOCK];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
         t += (long)gridDim.x * blockDim.x)
        for (int p = 0; p < np; p++) s[p] += args.a[p][t] * args.b[p][t];
    for (int p = 0; p < np; p++) {
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
        for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
             t += (long)gridDim.x * blockDim.x)
            v = fmax(v, fabs(x[m * n + t]));
        v = block_max(v, sh);
        if (threadIdx.x == 0) part[m * gridDim.x + blockIdx.x] = v;
    }
}

__global__ void k_sum_open(GeomV g, const double* __restrict__ x, double* __restrict__ part) {
    __shared__ double sh[EB_BLOCK];
    double s = 0.0, cnt = 0.0;
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
            v = fmax(v, fabs(g.ap[d][t] * fo[d][t]));
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
        double v = 0.0;
        for (int t = threadIdx.x; t < nb; t += blockDim.x)
            v = mode ? fmax(v, part[p * nb + t]) : v + part[p * nb + t];
        v = mode ? block_max(v, sh) : block_sum(v, sh);
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
    long c = t % N;
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
void resid_pass(const Level& L, int nc, const T* b, const T* x, T* r, hipStream_t s);
template <>
void resid_pass<double>(const Level& L, int nc, const double* b, const double* x, double* r,
                        hipStream_t s) {
    if (nc == 3) k_resid<double, 3><<<grid_for(L.N), EB_BLOCK, 0, s>>>(L.v64(), b, x, r);
    else k_resid<double, 1><<<grid_for(L.N), EB_BLOCK, 0, s>>>(L.v64(), b, x, r);
}
template <>
void resid_pass<float>(const Level& L, int nc, const float* b, const float* x, float* r,
                       hipStream_t s) {
    if (nc == 3) k_resid<float, 3><<<grid_for(L.N), EB_BLOCK, 0, s>>>(L.v32(), b, x, r);
    else k_resid<float, 1><<<grid_for(L.N), EB_BLOCK, 0, s>>>(L.v32(), b, x, r);
}
template <typename TF, typename TC>
void restrict_pass(const Level& F, const Level& C, int nc, const TF* rf, TC* bc, hipStream_t s) {
    if (nc == 3)
        k_restrict<TF, TC, 3><<<grid_for(C.N), EB_BLOCK, 0, s>>>(F.grid, C.grid, F.mask, C.mask,
                                                                rf, bc, F.gate);
    else
        k_restrict<TF, TC, 1><<<grid_for(C.N), EB_BLOCK, 0, s>>>(F.grid, C.grid, F.mask, C.mask,
                                                                rf, bc, F.gate);
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
                         TC* bc, hipStream_t s) {
    if (nc == 3)
        k_resid_restrict<TF, TC, 3><<<grid_for(C.N), EB_BLOCK, 0, s>>>(level_view<TF>(F), b, x,
                                                                      C.grid, C.mask, bc);
    else
        k_resid_restrict<TF, TC, 1><<<grid_for(C.N), EB_BLOCK, 0, s>>>(level_view<TF>(F), b, x,
                                                                      C.grid, C.mask, bc);
}
template <typename TC, typename TF>
void prolong_pass(const Level& F, const Level& C, int nc, const TC* ec, TF* xf, hipStream_t s) {
    if (nc == 3)
        k_prolong<TC, TF, 3><<<grid_for(F.N), EB_BLOCK, 0, s>>>(F.grid, C.grid, F.mask, ec, xf, F.gate);
    else
        k_prolong<TC, TF, 1><<<grid_for(F.N), EB_BLOCK, 0, s>>>(F.grid, C.grid, F.mask, ec, xf, F.gate);
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

// levels above the tail run in FP32 in mixed mode; the tail (and so the coarsest solve) is FP64
bool level_f32(const VArgs& a, int l) { return a.mixed && l < a.tail; }

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
template <typename T>
T* rl(Level& L);
template <>
double* rl<double>(Level& L) { return L.r; }
template <>
float* rl<float>(Level& L) { return L.rf; }

void vcycle_rec(const VArgs& a, int l);

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
        if (t == 0) first_pass<T>(L, a.nc, b, x, a.s);
        else smooth_pass<T>(L, a.nc, b, x, 0, a.s);
        smooth_pass<T>(L, a.nc, b, x, 1, a.s);
    }
    Level& C = a.lev[l + 1];
    if (level_f32(a, l + 1)) resid_restrict_pass<T, float>(L, C, a.nc, b, x, C.bf, a.s);
    else resid_restrict_pass<T, double>(L, C, a.nc, b, x, C.b, a.s);
    vcycle_rec(a, l + 1);
    if (level_f32(a, l + 1)) prolong_pass<float, T>(L, C, a.nc, C.xf, x, a.s);
    else prolong_pass<double, T>(L, C, a.nc, C.x, x, a.s);
    for (int t = 0; t < a.nu2; t++) {
        smooth_pass<T>(L, a.nc, b, x, 1, a.s);
        smooth_pass<T>(L, a.nc, b, x, 0, a.s);
    }
}

void vcycle_rec(const VArgs& a, int l) {
    if (l == a.tail && a.tail_fits) launch_tail(a);
    else if (level_f32(a, l)) vcycle_level<float>(a, l);
    else vcycle_level<double>(a, l);
}

void finish_operator(Level* lev, int nlev, bool mixed, hipStream_t s) {
    int tail = tail_level(lev, nlev);
    for (int l = 1; l < nlev; l++) {
        for (int d = 0; d < 3; d++)
            level_coarsen_faces(lev[l].grid, lev[l - 1].grid, d, lev[l - 1].K[d], lev[l].K[d],
                                1.0 / 16.0, s);
        level_coarsen_cells(lev[l].grid, lev[l - 1].grid, lev[l - 1].S, lev[l].S, s);
    }
    for (int l = 0; l < nlev; l++) {
        Level& L = lev[l];
        k_diag<<<grid_for(L.N), EB_BLOCK, 0, s>>>(L.grid, L.K[0], L.K[1], L.K[2], L.S, L.mask,
                                                  L.D);
        if (mixed && l < tail) {
            for (int d = 0; d < 3; d++) {
                long nf = face_count(L.grid, d);
                k_to_float<<<grid_for(nf), EB_BLOCK, 0, s>>>(nf, L.K[d], L.Kf[d]);
            }
            k_to_float<<<grid_for(L.N), EB_BLOCK, 0, s>>>(L.N, L.D, L.Df);
        }
    }
}

}  // namespace

void mg_build_poisson(Level* lev, int nlev, const GeomV& g, double beta, bool mixed,
                      hipStream_t s) {
    for (int d = 0; d < 3; d++)
        k_K_poisson<<<grid_for(face_count(g.grid, d)), EB_BLOCK, 0, s>>>(g, d, beta, lev[0].K[d]);
    k_zero<double><<<grid_for(g.N), EB_BLOCK, 0, s>>>(g.N, lev[0].S);
    finish_operator(lev, nlev, mixed, s);
}

void mg_build_visc(Level* lev, int nlev, const GeomV& g, double rho, double dt,
                   const double* eta, const double* eta_eb, bool mixed, hipStream_t s) {
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

void mg_sweep_level0(const Level& L, int ncomp, bool f32, const void* b, void* x, int colour,
                     hipStream_t s) {
    if (f32)
        smooth_pass<float>(L, ncomp, (const float*)b, (float*)x, colour, s);
    else
        smooth_pass<double>(L, ncomp, (const double*)b, (double*)x, colour, s);
}

void mg_apply_level0(const Level& L, int ncomp, const double* x, double* y, hipStream_t s,
                     const int* gate) {
    Level G = L;
    G.gate = gate;
    resid_pass<double>(G, ncomp, nullptr, x, y, s);
}

void op_visc_apply(const GeomV& g, double rho, double dt, const double* eta,
                   const double* eta_eb, const double* u, double* out, int homogeneous,
                   hipStream_t s, const int* gate) {
    k_visc_apply<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, rho, dt, eta, eta_eb, u, out, homogeneous,
                                                    gate);
}

// ------------------------------------------------------------------------------------------
// reductions: results land in out (device); the caller copies what it needs to the host
// ------------------------------------------------------------------------------------------
int red_blocks(long n) {
    long b = (n + EB_BLOCK - 1) / EB_BLOCK;
    if (b > RED_MAXB) b = RED_MAXB;
    return (int)(b < 1 ? 1 : b);
}

void red_dots(long n, int np, const double* const a[4], const double* const b[4], double* part,
              double* out, hipStream_t s, const int* gate) {
    DotArgs args;
    for (int p = 0; p < 4; p++) {
        args.a[p] = p < np ? a[p] : nullptr;
        args.b[p] = p < np ? b[p] : nullptr;
    }
    int nb = red_blocks(n);
    k_dots<<<nb, EB_BLOCK, 0, s>>>(n, np, args, part, gate);
    k_final<<<1, EB_BLOCK, 0, s>>>(part, nb, np, 0, out, gate);
}

void red_maxabs(long n, int ncomp, const double* x, double* part, double* out, hipStream_t s,
                const int* gate) {
    int nb = red_blocks(n);
    k_maxabs<<<nb, EB_BLOCK, 0, s>>>(n, ncomp, x, part, gate);
    k_final<<<1, EB_BLOCK, 0, s>>>(part, nb, ncomp, 1, out, gate);
}

void red_sum_open(const GeomV& g, const double* x, double* part, double* out, hipStream_t s) {
    int nb = red_blocks(g.N);
    k_sum_open<<<nb, EB_BLOCK, 0, s>>>(g, x, part);
    k_final<<<1, EB_BLOCK, 0, s>>>(part, nb, 2, 0, out, nullptr);
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

int mg_tail_level(const Level* lev, int nlev) { return tail_level(lev, nlev); }
