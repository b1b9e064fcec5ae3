// eb_device.hpp -- device helpers shared by the forward and the adjoint kernels.
#pragma once
#include "eb_internal.hpp"

// strain rate at which the power-law term kappa s^(n-1) is evaluated: for n < 1 the term is
// unbounded at zero strain rate, and rates below eps are raised to eps
__device__ __forceinline__ double power_rate(const eb_rheology& r, double sr) {
    return (r.n < 1.0 && sr < r.eps) ? r.eps : sr;
}

// apparent viscosity (Table rheology, Eq. papabing:viscosity): a base term (mu, or the power-law
// term of the last three laws) plus the yield term tau0 * (1 - exp(-x))/sr, with x = sr/eps
// (Papanastasiou, Herschel-Bulkley) or x = eta0 sr/tau0 (Souza Mendes-Dutra), and its sr -> 0
// limit; a zero tau0 leaves the base term
__device__ __forceinline__ double eta_law(const eb_rheology& r, double tau0, double sr) {
    const int law = r.law;
    if (law == EB_LAW_NEWTONIAN) return r.mu;
    bool pl = law >= EB_LAW_POWER;
    double base = pl ? r.kappa * pow(power_rate(r, sr), r.n - 1.0) : r.mu;
    if (law == EB_LAW_POWER || tau0 == 0.0) return base;
    if (law == EB_LAW_BINGHAM_REG) return base + tau0 / (sr + r.eps);
    bool smd = law == EB_LAW_SOUZA_MENDES_DUTRA;
    if (sr == 0.0) return base + (smd ? r.eta0 : tau0 / r.eps);
    double x = smd ? r.eta0 * sr / tau0 : sr / r.eps;
    return base + tau0 * (-expm1(-x)) / sr;
}

// sqrt(tr(gamma gamma^T)/2), gamma = G + G^T
__device__ __forceinline__ double strain_rate(const double G[3][3]) {
    double s = 0.0;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double y = G[a][b] + G[b][a];
            s += y * y;
        }
    return sqrt(0.5 * s);
}

__device__ __forceinline__ long nbr(const GridV& g, int i, int j, int k, int d, int side) {
    int q[3] = {i, j, k};
    q[d] += side;
    return cell_at(g, q[0], q[1], q[2]);
}

// monotonised-central limited slope of component uj along d at cell c
// branch of the monotonised-central slope of uj at c in direction d: 0 zero (a wall or covered
// neighbour, or an extremum), else which of |dc|, 2|dl|, 2|dr| is least (1, 2, 3)
__device__ inline int mc_branch(const GeomV& g, const double* __restrict__ uj, long c, int d) {
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    long lo = nbr(g.grid, i, j, k, d, -1), hi = nbr(g.grid, i, j, k, d, 1);
    if (lo < 0 || hi < 0) return 0;
    if (!(g.alpha[lo] > 0.0) || !(g.alpha[hi] > 0.0)) return 0;
    double uc = uj[c];
    double dl = uc - uj[lo], dr = uj[hi] - uc, dc = 0.5 * (uj[hi] - uj[lo]);
    if (dl * dr <= 0.0) return 0;
    double a = fabs(dc), b = 2.0 * fabs(dl), e = 2.0 * fabs(dr);
    if (a <= b && a <= e) return 1;
    return b <= e ? 2 : 3;
}

// the slope on a given branch; on the branch mc_branch picks it equals mc_slope bit for bit
// (the three differences share their sign there)
__device__ inline double mc_eval(const GeomV& g, const double* __restrict__ uj, long c, int d,
                                 int code) {
    if (code == 0) return 0.0;
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    long lo = nbr(g.grid, i, j, k, d, -1), hi = nbr(g.grid, i, j, k, d, 1);
    if (lo < 0 || hi < 0) return 0.0;
    if (code == 1) return 0.5 * (uj[hi] - uj[lo]);
    return code == 2 ? 2.0 * (uj[c] - uj[lo]) : 2.0 * (uj[hi] - uj[c]);
}

__device__ inline double mc_slope(const GeomV& g, const double* __restrict__ uj, long c, int d) {
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    long lo = nbr(g.grid, i, j, k, d, -1), hi = nbr(g.grid, i, j, k, d, 1);
    if (lo < 0 || hi < 0) return 0.0;
    if (!(g.alpha[lo] > 0.0) || !(g.alpha[hi] > 0.0)) return 0.0;
    double uc = uj[c];
    double dl = uc - uj[lo], dr = uj[hi] - uc, dc = 0.5 * (uj[hi] - uj[lo]);
    if (dl * dr <= 0.0) return 0.0;
    double m = fmin(fabs(dc), fmin(2.0 * fabs(dl), 2.0 * fabs(dr)));
    return dc > 0.0 ? m : -m;
}

// cells on either side of face (d; fi, fj, fk); -1 at a wall
__device__ __forceinline__ void face_cells(const GridV& g, int d, int fi, int fj, int fk,
                                           long& lo, long& hi) {
    int q[3] = {fi, fj, fk};
    q[d] -= 1;
    lo = cell_at(g, q[0], q[1], q[2]);
    q[d] += 1;
    hi = cell_at(g, q[0], q[1], q[2]);
}

__device__ __forceinline__ void face_coords(const GridV& g, int d, long f, int& i, int& j,
                                            int& k) {
    unsigned m0 = g.n[0] + (d == 0), m1 = g.n[1] + (d == 1), fu = (unsigned)f;
    unsigned r = fu / m0;
    i = (int)(fu - r * m0);
    unsigned kk = r / m1;
    j = (int)(r - kk * m1);
    k = (int)kk;
}
