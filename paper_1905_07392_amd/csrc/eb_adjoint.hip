// eb_adjoint.hip -- reverse-mode kernels of the RK2 step and of the drag.
//
// Each kernel is the transpose of a linearised forward kernel, written as a gather: one thread
// per output entry sums every term that reads it, so no atomics are needed and the result is
// bitwise reproducible.  Switches (upwind side, limiter branch, one-sided stencil choice, the
// wall-stencil planes) are re-evaluated from the forward state and frozen.  Adjoint arrays are
// named *b; "acc" in a comment means the kernel adds to the array.
//
// Periodic seams: along a periodic direction the faces with index 0 and n are the same
// physical face stored twice.  Forward kernels that loop over cells use a cell's own face
// indices (cell 0 reads face 0, cell n-1 reads face n); kernels that loop over faces write
// both copies.  The gathers below follow the same convention, face by face.
#include "eb_device.hpp"

namespace {

// g'(x) of g(x) = (1 - e^-x)/x, i.e. (x e^-x + expm1(-x))/x^2; below x = 1e-2 the Taylor
// polynomial of g' replaces the cancelling quotient
__device__ __forceinline__ double dg_exp(double x) {
    if (x < 1e-2)
        return -0.5 + x * (1.0 / 3.0 + x * (-1.0 / 8.0 + x * (1.0 / 30.0 - x / 144.0)));
    return (x * exp(-x) + expm1(-x)) / (x * x);
}

// d eta / d(strain-rate norm) and d eta / d tau0 of eta_law.  The power-law term contributes
// kappa (n-1) sr^(n-2) where it follows the rate (not at sr = 0, where |.| has no derivative,
// nor below the cap of n < 1).  The yield term tau0 (1 - e^-x)/sr equals tau0 g(x)/sr:
// Papanastasiou and Herschel-Bulkley (x = sr/eps) give tau0 g'(x)/eps^2 and (1 - e^-x)/sr
// (1/eps at sr = 0); Souza Mendes-Dutra writes it eta0 g(x) with x = eta0 sr/tau0, giving
// eta0^2 g'(x)/tau0 and -eta0 x g'(x)/tau0, and at tau0 = 0 the tau0-limit 1/sr (0 at sr = 0).
__device__ __forceinline__ void law_deriv(const eb_rheology& r, double tau0, double sr,
                                          double& d_sr, double& d_tau0) {
    const int law = r.law;
    d_sr = 0.0;
    d_tau0 = 0.0;
    if (law == EB_LAW_NEWTONIAN) return;
    if (law == EB_LAW_BINGHAM_REG) {
        double q = 1.0 / (sr + r.eps);
        d_tau0 = q;
        d_sr = -tau0 * q * q;
        return;
    }
    if (law >= EB_LAW_POWER && r.n != 1.0 && sr > 0.0 && power_rate(r, sr) == sr)
        d_sr = r.kappa * (r.n - 1.0) * pow(sr, r.n - 2.0);
    if (law == EB_LAW_POWER) return;
    if (law == EB_LAW_SOUZA_MENDES_DUTRA) {
        if (tau0 == 0.0) {
            d_tau0 = sr > 0.0 ? 1.0 / sr : 0.0;
            return;
        }
        double x = r.eta0 * sr / tau0, gp = dg_exp(x);
        d_sr += r.eta0 * r.eta0 * gp / tau0;
        d_tau0 = -r.eta0 * x * gp / tau0;
        return;
    }
    double x = sr / r.eps;
    d_tau0 = sr == 0.0 ? 1.0 / r.eps : -expm1(-x) / sr;
    d_sr += tau0 * dg_exp(x) / (r.eps * r.eps);
}

// coefficient of wall-stencil entry e (flat index slot * ncut + cut) in the wall gradient
__device__ __forceinline__ double wall_coef(const GeomV& g, int e) {
    int nc = g.ncut;
    int q = e % nc, m = e / nc;
    double d1 = g.dd[q], d2 = g.dd[nc + q];
    double den = d1 * d2 * (d2 - d1) * g.grid.h;
    return g.sw[e] * (m < 9 ? d2 * d2 : -d1 * d1) / den;
}

__device__ __forceinline__ bool open_cell(const GeomV& g, long c) {
    return c >= 0 && g.alpha[c] > 0.0;
}

// face index of cell (i,j,k)'s face on `side` (0 low, 1 high) along d
__device__ __forceinline__ long own_face(const GridV& g, int d, int i, int j, int k, int side) {
    int f[3] = {i, j, k};
    f[d] += side;
    return face_index(g, d, f[0], f[1], f[2]);
}

// the other stored copy of a seam face (-1 if face coordinate fd is not on a periodic seam)
__device__ __forceinline__ int seam_twin(const GridV& g, int d, int fd) {
    if (!g.per[d]) return -1;
    if (fd == 0) return g.n[d];
    if (fd == g.n[d]) return 0;
    return -1;
}

// Coefficients of u at offsets -2..2 along d in the one-sided/central gradient of cell c
// (ghost values 2 u_wall - u_c fold into offset 0).  Returns false where both neighbours are
// covered and the gradient comes from the wall gradient instead.
__device__ bool grad_coefs(const GeomV& g, long c, int d, double cf[5]) {
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    long lo = nbr(g.grid, i, j, k, d, -1), hi = nbr(g.grid, i, j, k, d, 1);
    long lo2 = nbr(g.grid, i, j, k, d, -2), hi2 = nbr(g.grid, i, j, k, d, 2);
    bool lo_wall = lo < 0, hi_wall = hi < 0;
    bool lo_open = !lo_wall && g.alpha[lo] > 0.0;
    bool hi_open = !hi_wall && g.alpha[hi] > 0.0;
    bool lo2_open = lo2 >= 0 && g.alpha[lo2] > 0.0;
    bool hi2_open = hi2 >= 0 && g.alpha[hi2] > 0.0;
    bool lo_ok = lo_open || lo_wall, hi_ok = hi_open || hi_wall;
    double ih = 1.0 / g.grid.h;
    for (int o = 0; o < 5; o++) cf[o] = 0.0;
    if (lo_ok && hi_ok) {
        double w = 0.5 * ih;
        if (hi_open) cf[3] += w;
        else cf[2] -= w;
        if (lo_open) cf[1] -= w;
        else cf[2] += w;
    } else if (hi_ok) {
        if (hi_open && hi2_open) {
            cf[2] += -1.5 * ih;
            cf[3] += 2.0 * ih;
            cf[4] += -0.5 * ih;
        } else {
            if (hi_open) cf[3] += ih;
            else cf[2] -= ih;
            cf[2] -= ih;
        }
    } else if (lo_ok) {
        if (lo_open && lo2_open) {
            cf[2] += 1.5 * ih;
            cf[1] += -2.0 * ih;
            cf[0] += 0.5 * ih;
        } else {
            cf[2] += ih;
            if (lo_open) cf[1] -= ih;
            else cf[2] += ih;
        }
    } else {
        return false;
    }
    return true;
}

// coefficient of u at offset off (-1, 0, 1) in the limited slope of component uj at cell c
__device__ double slope_coef(const GeomV& g, const double* __restrict__ uj, long c, int d,
                             int off) {
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    long lo = nbr(g.grid, i, j, k, d, -1), hi = nbr(g.grid, i, j, k, d, 1);
    if (lo < 0 || hi < 0) return 0.0;
    if (!(g.alpha[lo] > 0.0) || !(g.alpha[hi] > 0.0)) return 0.0;
    double uc = uj[c];
    double dl = uc - uj[lo], dr = uj[hi] - uc, dc = 0.5 * (uj[hi] - uj[lo]);
    if (dl * dr <= 0.0) return 0.0;
    double adc = fabs(dc), al = 2.0 * fabs(dl), ar = 2.0 * fabs(dr);
    if (adc <= fmin(al, ar)) return off == 0 ? 0.0 : 0.5 * off;  // central difference
    if (al <= ar) return off == -1 ? -2.0 : (off == 0 ? 2.0 : 0.0);  // twice the left one
    return off == 1 ? 2.0 : (off == 0 ? -2.0 : 0.0);                // twice the right one
}

// ------------------------------------------------------------------------------------------
// redistribution backward: per cut cell, then a gather over the 26-neighbourhood
// ------------------------------------------------------------------------------------------
__global__ void k_redist_adj_cut(GeomV g, const double* __restrict__ Db, double* __restrict__ X,
                                 double* __restrict__ Y) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = g.ncut;
    if (q >= nc) return;
    long N = g.N;
    long c = g.cut[q];
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    double s = 0.0, sum[3] = {0.0, 0.0, 0.0};
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                if (!dx && !dy && !dz) continue;
                long cc = cell_at(g.grid, i + dx, j + dy, k + dz);
                if (cc < 0) continue;
                double a = g.alpha[cc];
                if (!(a > 0.0)) continue;
                s += a;
                for (int m = 0; m < 3; m++) sum[m] += Db[m * N + cc];
            }
    double al = g.alpha[c];
    for (int m = 0; m < 3; m++) {
        double dhb = Db[m * N + c];
        double ddb = s > 0.0 ? sum[m] / s : 0.0;  // adjoint of dD (spread only when S > 0)
        double self = al * dhb + al * (1.0 - al) * ddb;
        double dncb = (1.0 - al) * dhb - al * (1.0 - al) * ddb;
        if (s > 0.0) {
            X[(long)m * nc + q] = dncb / s;
        } else {
            X[(long)m * nc + q] = 0.0;
            self += dncb;
        }
        Y[(long)m * nc + q] = self;
    }
}

__global__ void k_redist_adj_gather(GeomV g, const double* __restrict__ Db,
                                    const double* __restrict__ X, const double* __restrict__ Y,
                                    double* __restrict__ DCb) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    double a = g.alpha[c];
    if (!(a > 0.0)) {
        for (int m = 0; m < 3; m++) DCb[m * N + c] = 0.0;
        return;
    }
    int nc = g.ncut;
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    int qc = g.flag[c] == 1 ? g.cutid[c] : -1;
    double acc[3];
    for (int m = 0; m < 3; m++) acc[m] = qc >= 0 ? Y[(long)m * nc + qc] : Db[m * N + c];
    if (!g.near[c]) {  // no cut cell in the 3x3x3 block: nothing to gather
        for (int m = 0; m < 3; m++) DCb[m * N + c] = acc[m];
        return;
    }
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                if (!dx && !dy && !dz) continue;
                long cc = cell_at(g.grid, i + dx, j + dy, k + dz);
                if (cc < 0 || g.flag[cc] != 1) continue;
                int q = g.cutid[cc];
                for (int m = 0; m < 3; m++) acc[m] += a * X[(long)m * nc + q];
            }
    for (int m = 0; m < 3; m++) DCb[m * N + c] = acc[m];
}

// ------------------------------------------------------------------------------------------
// backward of V's flux divergence (transpose stress), of the viscosity law at cells and at
// the wall, and of the wall-gradient branch of the cell gradients.  Per cell: ub (acc),
// Gb (written), tau0b (acc); per cut cell: gwb (written).
// ------------------------------------------------------------------------------------------
__global__ void k_visc_terms_adj(GeomV g, eb_rheology rh, const double* __restrict__ theta,
                                 const double* __restrict__ u, const double* __restrict__ G9,
                                 const double* __restrict__ eta,
                                 const double* __restrict__ eta_eb,
                                 const double* __restrict__ gw, const double* __restrict__ DCb,
                                 const double* __restrict__ etab_in,
                                 const double* __restrict__ etaebb_in, double* __restrict__ ub,
                                 double* __restrict__ Gb, double* __restrict__ gwb,
                                 double* __restrict__ tau0b) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    double al = g.alpha[c];
    if (!(al > 0.0)) {
        for (int a = 0; a < 9; a++) Gb[a * N + c] = 0.0;
        return;
    }
    int i, j0, k;
    cell_coords(g.grid, c, i, j0, k);
    double h = g.grid.h;
    double etab = etab_in ? etab_in[c] : 0.0;
    double Gbl[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double ubl[3] = {0.0, 0.0, 0.0};
    double wc[3];
    for (int j = 0; j < 3; j++) wc[j] = DCb[j * N + c] / (al * h);
    double ec = eta[c];
    for (int d = 0; d < 3; d++) {
        const double* ud = u + (long)d * N;
        for (int side = -1; side <= 1; side += 2) {
            double Ac = g.ap[d][own_face(g.grid, d, i, j0, k, side > 0)];
            long nb = nbr(g.grid, i, j0, k, d, side);
            if (nb >= 0) {
                double An = 0.0, wn[3] = {0.0, 0.0, 0.0};
                double an = g.alpha[nb];
                if (an > 0.0) {
                    int ni, nj, nk;
                    cell_coords(g.grid, nb, ni, nj, nk);
                    An = g.ap[d][own_face(g.grid, d, ni, nj, nk, side < 0)];
                    for (int j = 0; j < 3; j++) wn[j] = DCb[j * N + nb] / (an * h);
                }
                if (Ac == 0.0 && An == 0.0) continue;
                double ef = 0.5 * (ec + eta[nb]);
                for (int j = 0; j < 3; j++) {
                    double Fb = (Ac != 0.0 ? side * Ac * wc[j] : 0.0) +
                                (An != 0.0 ? -side * An * wn[j] : 0.0);
                    double der;
                    if (j == d)
                        der = side > 0 ? (ud[nb] - ud[c]) / h : (ud[c] - ud[nb]) / h;
                    else
                        der = 0.5 * (G9[(j * 3 + d) * N + c] + G9[(j * 3 + d) * N + nb]);
                    etab += 0.5 * Fb * der;
                    if (j == d) ubl[d] += Fb * ef * (side > 0 ? -1.0 : 1.0) / h;
                    else Gbl[j][d] += 0.5 * Fb * ef;
                }
            } else if (Ac != 0.0) {
                double Fb = side * Ac * wc[d];
                double uw = g.wall[2 * d + (side > 0)][d];
                double der = side > 0 ? (uw - ud[c]) / (0.5 * h) : (ud[c] - uw) / (0.5 * h);
                etab += Fb * der;
                ubl[d] += Fb * ec * (side > 0 ? -1.0 : 1.0) / (0.5 * h);
            }
        }
    }
    // law backward at the cell centre
    double G[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) G[a][b] = G9[(a * 3 + b) * N + c];
    double t0 = rh.tau0 * (theta ? theta[c] : 1.0);
    double s = strain_rate(G), dsr, dt0;
    law_deriv(rh, t0, s, dsr, dt0);
    double tb = dt0 * etab;
    if (s > 0.0) {
        double sb = dsr * etab / s;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Gbl[a][b] += sb * (G[a][b] + G[b][a]);
    }
    int q = g.cutid[c];
    if (q >= 0) {
        int nc = g.ncut;
        double nv[3], gv[3], gwbl[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 3; a++) {
            nv[a] = g.nrm[(long)a * nc + q];
            gv[a] = gw[(long)a * nc + q];
        }
        double ng = nv[0] * gv[0] + nv[1] * gv[1] + nv[2] * gv[2];
        double eebb = etaebb_in ? etaebb_in[q] : 0.0;
        double eeb = eta_eb[q];
        // wall-flux term of V: -A_EB eta_EB n_j (n . gw)
        for (int j = 0; j < 3; j++) {
            double t = -g.aeb[q] * nv[j] * wc[j];
            eebb += t * ng;
            for (int b = 0; b < 3; b++) gwbl[b] += t * eeb * nv[b];
        }
        // law backward at the wall: (grad u)_ab = n_a gw_b
        double Ge[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Ge[a][b] = nv[a] * gv[b];
        double se = strain_rate(Ge), dsre, dt0e;
        law_deriv(rh, t0, se, dsre, dt0e);
        tb += dt0e * eebb;
        if (se > 0.0) {
            double sb = dsre * eebb / se;
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) gwbl[b] += nv[a] * sb * (Ge[a][b] + Ge[b][a]);
        }
        // cell gradients taken from the wall gradient where both neighbours are covered
        for (int d = 0; d < 3; d++) {
            double cf[5];
            if (!grad_coefs(g, c, d, cf))
                for (int j = 0; j < 3; j++) gwbl[j] += nv[d] * Gbl[d][j];
        }
        for (int b = 0; b < 3; b++) gwb[(long)b * nc + q] = gwbl[b];
    }
    tau0b[c] += tb;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) Gb[(a * 3 + b) * N + c] = Gbl[a][b];
    for (int d = 0; d < 3; d++) ub[d * N + c] += ubl[d];
}

// ub (acc) += (cell gradient)^T Gb + (wall gradient)^T gwb; either input may be null
__global__ void k_grad_adj_gather(GeomV g, WallT wt, const double* __restrict__ Gb,
                                  const double* __restrict__ gwb, double* __restrict__ ub) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    double acc[3] = {0.0, 0.0, 0.0};
    if (Gb && g.alpha[c] > 0.0) {
        int i, j, k;
        cell_coords(g.grid, c, i, j, k);
        for (int d = 0; d < 3; d++)
            for (int o = -2; o <= 2; o++) {
                long cp = nbr(g.grid, i, j, k, d, o);
                if (!open_cell(g, cp)) continue;
                double cf[5];
                if (!grad_coefs(g, cp, d, cf)) continue;
                double w = cf[2 - o];  // c sits at offset -o from cp
                if (w == 0.0) continue;
                for (int m = 0; m < 3; m++) acc[m] += w * Gb[(d * 3 + m) * N + cp];
            }
    }
    if (gwb) {
        int r = wt.map[c];
        if (r >= 0) {
            int nc = g.ncut;
            for (int e = wt.ptr[r]; e < wt.ptr[r + 1]; e++) {
                int idx = wt.ent[e];
                double w = wall_coef(g, idx);
                int q = idx % nc;
                for (int m = 0; m < 3; m++) acc[m] += w * gwb[(long)m * nc + q];
            }
        }
    }
    for (int m = 0; m < 3; m++)
        if (acc[m] != 0.0) ub[m * N + c] += acc[m];
}

// ------------------------------------------------------------------------------------------
// convective term backward
// ------------------------------------------------------------------------------------------
// adjoint of the face flux w_f up_f,j: each cell that reads this face index contributes
__device__ void conv_flux_bar(const GeomV& g, int d, int fd, long lo, long hi, double A,
                              const double* __restrict__ DCb, double Fb[3]) {
    Fb[0] = Fb[1] = Fb[2] = 0.0;
    if (A == 0.0) return;
    long N = g.N;
    double h = g.grid.h;
    if (fd >= 1 && open_cell(g, lo)) {
        double w = -A / (g.alpha[lo] * h);
        for (int j = 0; j < 3; j++) Fb[j] += w * DCb[j * N + lo];
    }
    if (fd <= g.grid.n[d] - 1 && open_cell(g, hi)) {
        double w = A / (g.alpha[hi] * h);
        for (int j = 0; j < 3; j++) Fb[j] += w * DCb[j * N + hi];
    }
}

// wb_f = sum_j Fb_j up_f,j (adjoint of the projected face velocity)
__global__ void k_conv_face_w(GeomV g, int d, const double* __restrict__ u,
                              const double* __restrict__ w, const double* __restrict__ DCb,
                              double* __restrict__ wb) {
    long nf = face_count(g.grid, d);
    long f = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int fi[3];
    face_coords(g.grid, d, f, fi[0], fi[1], fi[2]);
    long lo, hi;
    face_cells(g.grid, d, fi[0], fi[1], fi[2], lo, hi);
    double Fb[3];
    conv_flux_bar(g, d, fi[d], lo, hi, g.ap[d][f], DCb, Fb);
    double s = 0.0;
    if (Fb[0] != 0.0 || Fb[1] != 0.0 || Fb[2] != 0.0) {
        for (int j = 0; j < 3; j++) {
            double up;
            if (lo < 0 || hi < 0) {
                up = g.wall[2 * d + (lo >= 0)][j];
            } else {
                const double* uj = u + (long)j * g.N;
                double uL = uj[lo] + 0.5 * mc_slope(g, uj, lo, d);
                double uR = uj[hi] - 0.5 * mc_slope(g, uj, hi, d);
                double wf = w[f];
                up = wf > 0.0 ? uL : (wf < 0.0 ? uR : 0.5 * (uL + uR));
            }
            s += Fb[j] * up;
        }
    }
    wb[f] = s;
}

// adjoints of the left/right face states of face f (conv term for every component; face
// extrapolation for component d, from the adjoint wbin of the unprojected face field)
__device__ void face_state_bar(const GeomV& g, int d, long f, const double* __restrict__ u,
                               const double* __restrict__ w, const double* __restrict__ DCb,
                               const double* __restrict__ wbin, double L[3], double R[3]) {
    for (int j = 0; j < 3; j++) L[j] = R[j] = 0.0;
    int fi[3];
    face_coords(g.grid, d, f, fi[0], fi[1], fi[2]);
    long lo, hi;
    face_cells(g.grid, d, fi[0], fi[1], fi[2], lo, hi);
    if (lo < 0 || hi < 0) return;
    double A = g.ap[d][f];
    double Fb[3];
    conv_flux_bar(g, d, fi[d], lo, hi, A, DCb, Fb);
    double wf = w[f];
    for (int j = 0; j < 3; j++) {
        double upb = Fb[j] * wf;
        if (wf > 0.0) L[j] = upb;
        else if (wf < 0.0) R[j] = upb;
        else L[j] = R[j] = 0.5 * upb;
    }
    if (A > 0.0 && wbin[f] != 0.0) {
        const double* ud = u + (long)d * g.N;
        double uL = ud[lo] + 0.5 * mc_slope(g, ud, lo, d);
        double uR = ud[hi] - 0.5 * mc_slope(g, ud, hi, d);
        if (uL > 0.0 && uL + uR > 0.0) L[d] += wbin[f];
        else if (uR < 0.0 && uL + uR < 0.0) R[d] += wbin[f];
    }
}

// per face: L (adjoint of u_L, owned by the low cell) and R (of u_R, owned by the high cell),
// the two seam copies folded onto the copy the owning cell reads
__global__ void k_conv_face_lr(GeomV g, int d, const double* __restrict__ u,
                               const double* __restrict__ w, const double* __restrict__ DCb,
                               const double* __restrict__ wbin, double* __restrict__ Lo,
                               double* __restrict__ Ro) {
    long nf = face_count(g.grid, d);
    long f = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int f0, f1, f2;
    face_coords(g.grid, d, f, f0, f1, f2);
    int fd = d == 0 ? f0 : (d == 1 ? f1 : f2);
    double L[3], R[3];
    face_state_bar(g, d, f, u, w, DCb, wbin, L, R);
    int tw = seam_twin(g.grid, d, fd);
    if (tw >= 0) {
        long ft = face_index(g.grid, d, d == 0 ? tw : f0, d == 1 ? tw : f1, d == 2 ? tw : f2);
        double L2[3], R2[3];
        face_state_bar(g, d, ft, u, w, DCb, wbin, L2, R2);
        bool top = fd == g.grid.n[d];  // cell n-1 reads face n, cell 0 reads face 0
#pragma unroll
        for (int j = 0; j < 3; j++) {
            if (top) L[j] += L2[j];
            else R[j] += R2[j];
        }
    }
    for (int j = 0; j < 3; j++) {
        Lo[(long)j * nf + f] = L[j];
        Ro[(long)j * nf + f] = R[j];
    }
}

// ub (acc): states u_L = u_lo + s_lo/2, u_R = u_hi - s_hi/2 and their limited slopes
__global__ void k_conv_cell_gather(GeomV g, const double* __restrict__ u, LRV lr,
                                   double* __restrict__ ub) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N || !(g.alpha[c] > 0.0)) return;
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    for (int m = 0; m < 3; m++) {
        const double* um = u + (long)m * N;
        double acc = 0.0;
        for (int d = 0; d < 3; d++) {
            long nf = face_count(g.grid, d);
            const double* L = lr.L[d] + (long)m * nf;
            const double* R = lr.R[d] + (long)m * nf;
            acc += L[own_face(g.grid, d, i, j, k, 1)] + R[own_face(g.grid, d, i, j, k, 0)];
            for (int o = -1; o <= 1; o++) {
                long cp = nbr(g.grid, i, j, k, d, o);
                if (!open_cell(g, cp)) continue;
                double w = slope_coef(g, um, cp, d, -o);
                if (w == 0.0) continue;
                int pi, pj, pk;
                cell_coords(g.grid, cp, pi, pj, pk);
                double sb = 0.5 * L[own_face(g.grid, d, pi, pj, pk, 1)] -
                            0.5 * R[own_face(g.grid, d, pi, pj, pk, 0)];
                acc += w * sb;
            }
        }
        ub[m * N + c] += acc;
    }
}

// ------------------------------------------------------------------------------------------
// projections backward
// ------------------------------------------------------------------------------------------
// visit the faces whose low (side 1) or high (side 0) cell is c, seam copies included
template <typename F>
__device__ __forceinline__ void faces_touching(const GridV& g, int d, int i, int j, int k,
                                               F&& fn) {
    int q[3] = {i, j, k};
    for (int side = 0; side < 2; side++) {
        int f[3] = {i, j, k};
        f[d] += side;
        fn(face_index(g, d, f[0], f[1], f[2]), side);
        int tw = seam_twin(g, d, f[d]);
        if (tw >= 0) {
            f[d] = tw;
            fn(face_index(g, d, f[0], f[1], f[2]), side);
        }
    }
    (void)q;
}

// rhs = G_f^T wb (open interior faces, seam copies included), stored negated so that the
// Poisson solve of a "divergence" -y returns L^+ y
__global__ void k_face_grad_T_neg(GeomV g, const double* __restrict__ fx,
                                  const double* __restrict__ fy, const double* __restrict__ fz,
                                  double* __restrict__ out) {
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= g.N) return;
    if (!(g.alpha[c] > 0.0)) {
        out[c] = 0.0;
        return;
    }
    const double* fb[3] = {fx, fy, fz};
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    double h = g.grid.h, acc = 0.0;
    for (int d = 0; d < 3; d++)
        faces_touching(g.grid, d, i, j, k, [&](long f, int side) {
            int fi[3];
            face_coords(g.grid, d, f, fi[0], fi[1], fi[2]);
            long lo, hi;
            face_cells(g.grid, d, fi[0], fi[1], fi[2], lo, hi);
            if (lo < 0 || hi < 0 || g.ap[d][f] == 0.0) return;
            acc += side ? -fb[d][f] / h : fb[d][f] / h;  // c is lo on side 1, hi on side 0
        });
    out[c] = -acc;
}

// wb += beta D^T z (transpose of the divergence; a cell reads only its own face indices)
__global__ void k_div_T_add(GeomV g, int d, double beta, const double* __restrict__ z,
                            double* __restrict__ wb) {
    long nf = face_count(g.grid, d);
    long f = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int fi[3];
    face_coords(g.grid, d, f, fi[0], fi[1], fi[2]);
    long lo, hi;
    face_cells(g.grid, d, fi[0], fi[1], fi[2], lo, hi);
    double t = 0.0;
    if (fi[d] >= 1 && open_cell(g, lo)) t += z[lo];
    if (fi[d] <= g.grid.n[d] - 1 && open_cell(g, hi)) t -= z[hi];
    wb[f] += beta * g.ap[d][f] * t / g.grid.h;
}

// end-of-stage projection: ub -= F^T D^T z (F: face average), covered entries zeroed
__global__ void k_cc_adj_cell(GeomV g, const double* __restrict__ z, double* __restrict__ ub) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    if (!(g.alpha[c] > 0.0)) {
        for (int d = 0; d < 3; d++) ub[d * N + c] = 0.0;
        return;
    }
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    double h = g.grid.h;
    for (int d = 0; d < 3; d++) {
        double acc = 0.0;
        faces_touching(g.grid, d, i, j, k, [&](long f, int) {
            int fi[3];
            face_coords(g.grid, d, f, fi[0], fi[1], fi[2]);
            long lo, hi;
            face_cells(g.grid, d, fi[0], fi[1], fi[2], lo, hi);
            double A = g.ap[d][f];
            if (lo < 0 || hi < 0 || !(A > 0.0)) return;
            double t = 0.0;
            if (fi[d] >= 1 && open_cell(g, lo)) t += z[lo];
            if (fi[d] <= g.grid.n[d] - 1 && open_cell(g, hi)) t -= z[hi];
            acc += 0.5 * A * t / h;
        });
        ub[d * N + c] -= acc;
    }
}

// out = base (open cells; 0 if base is null) + a Gcc^T v
__global__ void k_gcc_T(GeomV g, double a, const double* __restrict__ v,
                        const double* base, double* out) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    if (!(g.alpha[c] > 0.0)) {
        out[c] = 0.0;
        return;
    }
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    double h = g.grid.h;
    double acc = base ? base[c] : 0.0;
    for (int d = 0; d < 3; d++) {
        double A2[2] = {g.ap[d][own_face(g.grid, d, i, j, k, 0)],
                        g.ap[d][own_face(g.grid, d, i, j, k, 1)]};
        double den = (A2[0] != 0.0 ? A2[0] : 0.0) + (A2[1] != 0.0 ? A2[1] : 0.0);
        for (int side = -1; side <= 1; side += 2) {
            long nb = nbr(g.grid, i, j, k, d, side);
            if (nb < 0) continue;
            double Ac = A2[side > 0];
            if (Ac != 0.0 && den > 0.0) acc += a * v[d * N + c] / den * Ac * (-side) / h;
            if (!(g.alpha[nb] > 0.0)) continue;
            int ni, nj, nk;
            cell_coords(g.grid, nb, ni, nj, nk);
            double B0 = g.ap[d][own_face(g.grid, d, ni, nj, nk, 0)];
            double B1 = g.ap[d][own_face(g.grid, d, ni, nj, nk, 1)];
            double dn = (B0 != 0.0 ? B0 : 0.0) + (B1 != 0.0 ? B1 : 0.0);
            double An = side > 0 ? B0 : B1;  // the neighbour's face towards c
            if (An != 0.0 && dn > 0.0) acc += a * v[d * N + nb] / dn * An * (-side) / h;
        }
    }
    out[c] = acc;
}

// ------------------------------------------------------------------------------------------
// viscous solve backward
// ------------------------------------------------------------------------------------------
// out = A^T lam for the homogeneous viscous operator (rows of open cells)
__global__ void k_visc_apply_T(GeomV g, double rho, double dt, const double* __restrict__ eta,
                               const double* __restrict__ eta_eb, WallT wt,
                               const double* __restrict__ lam, double* __restrict__ out,
                               const int* gate) {
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
    for (int m = 0; m < 3; m++) acc[m] = al * rho * lam[m * N + c];
    double ec = eta[c];
    for (int d = 0; d < 3; d++)
        for (int side = 0; side < 2; side++) {
            double A = g.ap[d][own_face(g.grid, d, i, j, k, side)];
            long nb = nbr(g.grid, i, j, k, d, side ? 1 : -1);
            if (nb >= 0) {
                double K = dt * A * 0.5 * (ec + eta[nb]) / h2;
                for (int m = 0; m < 3; m++) acc[m] += K * lam[m * N + c];
                if (g.alpha[nb] > 0.0) {
                    int ni, nj, nk;
                    cell_coords(g.grid, nb, ni, nj, nk);
                    double An = g.ap[d][own_face(g.grid, d, ni, nj, nk, 1 - side)];
                    double Kn = dt * An * 0.5 * (eta[nb] + ec) / h2;
                    for (int m = 0; m < 3; m++) acc[m] -= Kn * lam[m * N + nb];
                }
            } else if (A != 0.0) {
                double K = 2.0 * dt * A * ec / h2;
                for (int m = 0; m < 3; m++) acc[m] += K * lam[m * N + c];
            }
        }
    int r = wt.map[c];
    if (r >= 0) {
        int nc = g.ncut;
        for (int e = wt.ptr[r]; e < wt.ptr[r + 1]; e++) {
            int idx = wt.ent[e];
            int q = idx % nc;
            double w = wall_coef(g, idx) * dt * g.aeb[q] * eta_eb[q] / g.grid.h;
            long cq = g.cut[q];
            for (int m = 0; m < 3; m++) acc[m] += w * lam[m * N + cq];
        }
    }
    for (int m = 0; m < 3; m++) out[m * N + c] = acc[m];
}

// etab (acc) -= (d R / d eta)^T lam, R the viscous residual at the solution x
__global__ void k_visc_coef_adj(GeomV g, double dt, const double* __restrict__ x,
                                const double* __restrict__ lam, double* __restrict__ etab) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N || !(g.alpha[c] > 0.0)) return;
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    double h2 = g.grid.h * g.grid.h;
    double acc = 0.0;
    for (int d = 0; d < 3; d++)
        for (int side = 0; side < 2; side++) {
            double A = g.ap[d][own_face(g.grid, d, i, j, k, side)];
            long nb = nbr(g.grid, i, j, k, d, side ? 1 : -1);
            if (nb >= 0) {
                if (A != 0.0) {
                    double s = 0.0;
                    for (int m = 0; m < 3; m++)
                        s += (x[m * N + nb] - x[m * N + c]) * lam[m * N + c];
                    acc += dt * A / (2.0 * h2) * s;
                }
                if (g.alpha[nb] > 0.0) {
                    int ni, nj, nk;
                    cell_coords(g.grid, nb, ni, nj, nk);
                    double An = g.ap[d][own_face(g.grid, d, ni, nj, nk, 1 - side)];
                    if (An != 0.0) {
                        double s = 0.0;
                        for (int m = 0; m < 3; m++)
                            s += (x[m * N + c] - x[m * N + nb]) * lam[m * N + nb];
                        acc += dt * An / (2.0 * h2) * s;
                    }
                }
            } else if (A != 0.0) {
                double s = 0.0;
                for (int m = 0; m < 3; m++)
                    s += (g.wall[2 * d + side][m] - x[m * N + c]) * lam[m * N + c];
                acc += 2.0 * dt * A / h2 * s;
            }
        }
    etab[c] += acc;
}

__global__ void k_visc_coef_adj_eb(GeomV g, double dt, const double* __restrict__ x,
                                   const double* __restrict__ lam, double* __restrict__ etaebb) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = g.ncut;
    if (q >= nc) return;
    long N = g.N;
    long c = g.cut[q];
    double d1 = g.dd[q], d2 = g.dd[nc + q];
    double den = d1 * d2 * (d2 - d1) * g.grid.h;
    double s = 0.0;
    for (int m = 0; m < 3; m++) {
        double ue = g.ueb[m], s1 = 0.0, s2 = 0.0;
        for (int t = 0; t < 9; t++) {
            int c1 = g.sidx[(long)t * nc + q];
            s1 += g.sw[(long)t * nc + q] * (c1 >= 0 ? x[m * N + c1] : ue);
            int c2 = g.sidx[(long)(t + 9) * nc + q];
            s2 += g.sw[(long)(t + 9) * nc + q] * (c2 >= 0 ? x[m * N + c2] : ue);
        }
        double gn = (d2 * d2 * (s1 - ue) - d1 * d1 * (s2 - ue)) / den;
        s += gn * lam[m * N + c];
    }
    etaebb[q] -= dt * g.aeb[q] / g.grid.h * s;
}

// psi = rho u + dt (rho C + V - Gcc p + f), psib = alpha lam
__global__ void k_psi_adj(GeomV g, double rho, double dt, const double* __restrict__ lam,
                          double* __restrict__ psib, double* __restrict__ ub,
                          double* __restrict__ Cb, double* __restrict__ Vb) {
    long N = g.N;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 3 * N) return;
    long c = (long)((unsigned)t % (unsigned)N);  // 3N < 2^32
    double a = g.alpha[c];
    double ps = a > 0.0 ? a * lam[t] : 0.0;
    psib[t] = ps;
    ub[t] += rho * ps;
    Cb[t] += dt * rho * ps;
    Vb[t] += dt * ps;
}

// ------------------------------------------------------------------------------------------
// drag backward (per cut cell): gwb (written), tau0b, pb (acc), gpb at the cut cell (written)
// ------------------------------------------------------------------------------------------
__global__ void k_drag_adj(GeomV g, eb_rheology rh, const double* __restrict__ theta,
                           const double* __restrict__ gw, double fb0, double fb1, double fb2,
                           double* __restrict__ gwb, double* __restrict__ tau0b,
                           double* __restrict__ pb, double* __restrict__ gpb) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = g.ncut;
    if (q >= nc) return;
    long N = g.N;
    long c = g.cut[q];
    double h = g.grid.h;
    double nv[3], gv[3];
    for (int a = 0; a < 3; a++) {
        nv[a] = g.nrm[(long)a * nc + q];
        gv[a] = gw[(long)a * nc + q];
    }
    double G[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) G[a][b] = nv[a] * gv[b];
    double t0 = rh.tau0 * (theta ? theta[c] : 1.0);
    double sr = strain_rate(G);
    double e = eta_law(rh, t0, sr), dsr, dt0;
    law_deriv(rh, t0, sr, dsr, dt0);
    double area = g.aeb[q] * h * h;
    double w[3] = {fb0 * area, fb1 * area, fb2 * area};
    double eb = 0.0, peb = 0.0;
    for (int a = 0; a < 3; a++) {
        for (int b = 0; b < 3; b++) eb += w[a] * (G[a][b] + G[b][a]) * nv[b];
        peb -= w[a] * nv[a];
    }
    double Gmb[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) Gmb[a][b] = e * (w[a] * nv[b] + w[b] * nv[a]);
    if (sr > 0.0) {
        double sb = dsr * eb / sr;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Gmb[a][b] += sb * (G[a][b] + G[b][a]);
    }
    for (int b = 0; b < 3; b++) {
        double s = 0.0;
        for (int a = 0; a < 3; a++) s += nv[a] * Gmb[a][b];
        gwb[(long)b * nc + q] = s;
    }
    tau0b[c] += dt0 * eb;
    pb[c] += peb;
    for (int d = 0; d < 3; d++) gpb[d * N + c] = h * g.bc[(long)d * nc + q] * peb;
}

__global__ void k_mask_open(GeomV g, int ncomp, const double* __restrict__ in,
                            double* __restrict__ out) {
    long N = g.N;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= N * ncomp) return;
    out[t] = g.alpha[(unsigned)t % (unsigned)N] > 0.0 ? in[t] : 0.0;
}

__global__ void k_scale(long n, double a, double* __restrict__ x) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) x[t] *= a;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
void adj_redistribute(const GeomV& g, const double* Db, double* X, double* Y, double* DCb,
                      hipStream_t s) {
    if (g.ncut > 0) k_redist_adj_cut<<<grid_for(g.ncut), EB_BLOCK, 0, s>>>(g, Db, X, Y);
    k_redist_adj_gather<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, Db, X, Y, DCb);
}
void adj_visc_terms(const GeomV& g, const eb_rheology& r, const double* theta, const double* u,
                    const double* G9, const double* eta, const double* eta_eb, const double* gw,
                    const double* DCb, const double* etab_in, const double* etaebb_in,
                    double* ub, double* Gb, double* gwb, double* tau0b, hipStream_t s) {
    k_visc_terms_adj<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, r, theta, u, G9, eta, eta_eb, gw, DCb,
                                                        etab_in, etaebb_in, ub, Gb, gwb, tau0b);
}
void adj_grad_gather(const GeomV& g, const WallT& wt, const double* Gb, const double* gwb,
                     double* ub, hipStream_t s) {
    k_grad_adj_gather<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, wt, Gb, g.ncut > 0 ? gwb : nullptr,
                                                         ub);
}
void adj_conv_face_w(const GeomV& g, const double* u, double* const w[3], const double* DCb,
                     double* wb[3], hipStream_t s) {
    for (int d = 0; d < 3; d++)
        k_conv_face_w<<<grid_for(face_count(g.grid, d)), EB_BLOCK, 0, s>>>(g, d, u, w[d], DCb,
                                                                            wb[d]);
}
void adj_conv_lr(const GeomV& g, const double* u, double* const w[3], const double* DCb,
                 double* const wbin[3], const LRV& lr, double* ub, hipStream_t s) {
    for (int d = 0; d < 3; d++)
        k_conv_face_lr<<<grid_for(face_count(g.grid, d)), EB_BLOCK, 0, s>>>(
            g, d, u, w[d], DCb, wbin[d], lr.L[d], lr.R[d]);
    k_conv_cell_gather<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, u, lr, ub);
}
void adj_face_grad_T_neg(const GeomV& g, double* const fb[3], double* out, hipStream_t s) {
    k_face_grad_T_neg<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, fb[0], fb[1], fb[2], out);
}
void adj_div_T_add(const GeomV& g, double beta, const double* z, double* wb[3], hipStream_t s) {
    for (int d = 0; d < 3; d++)
        k_div_T_add<<<grid_for(face_count(g.grid, d)), EB_BLOCK, 0, s>>>(g, d, beta, z, wb[d]);
}
void adj_cc_cell(const GeomV& g, const double* z, double* ub, hipStream_t s) {
    k_cc_adj_cell<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, z, ub);
}
void adj_gcc_T(const GeomV& g, double a, const double* v, const double* base, double* out,
               hipStream_t s) {
    k_gcc_T<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, a, v, base, out);
}
void adj_visc_apply_T(const GeomV& g, double rho, double dt, const double* eta,
                      const double* eta_eb, const WallT& wt, const double* lam, double* out,
                      hipStream_t s, const int* gate) {
    k_visc_apply_T<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, rho, dt, eta, eta_eb, wt, lam, out,
                                                      gate);
}
void adj_visc_coef(const GeomV& g, double dt, const double* x, const double* lam, double* etab,
                   double* etaebb, hipStream_t s) {
    k_visc_coef_adj<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, dt, x, lam, etab);
    if (g.ncut > 0) k_visc_coef_adj_eb<<<grid_for(g.ncut), EB_BLOCK, 0, s>>>(g, dt, x, lam, etaebb);
}
void adj_psi(const GeomV& g, double rho, double dt, const double* lam, double* psib, double* ub,
             double* Cb, double* Vb, hipStream_t s) {
    k_psi_adj<<<grid_for(3 * g.N), EB_BLOCK, 0, s>>>(g, rho, dt, lam, psib, ub, Cb, Vb);
}
void adj_drag(const GeomV& g, const eb_rheology& r, const double* theta, const double* gw,
              const double fb[3], double* gwb, double* tau0b, double* pb, double* gpb,
              hipStream_t s) {
    if (g.ncut > 0)
        k_drag_adj<<<grid_for(g.ncut), EB_BLOCK, 0, s>>>(g, r, theta, gw, fb[0], fb[1], fb[2],
                                                         gwb, tau0b, pb, gpb);
}
void adj_mask_open(const GeomV& g, int ncomp, const double* in, double* out, hipStream_t s) {
    k_mask_open<<<grid_for(g.N * ncomp), EB_BLOCK, 0, s>>>(g, ncomp, in, out);
}
void adj_scale(long n, double a, double* x, hipStream_t s) {
    if (n > 0) k_scale<<<grid_for(n), EB_BLOCK, 0, s>>>(n, a, x);
}
