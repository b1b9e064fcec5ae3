// eb_ops.hip -- pointwise and stencil operators of the RK2 step (Sec. III.A.3, III.B).
//
// One thread per cell (or face, or cut cell); x is the fastest index so a wavefront reads
// contiguous rows.  All arithmetic is binary64.
#include "eb_device.hpp"

namespace {

// ------------------------------------------------------------------------------------------
// wall gradient (Eq. dudn) per cut cell, gw [3][ncut]
// ------------------------------------------------------------------------------------------
__global__ void k_wall_grad(GeomV g, const double* __restrict__ u, double* __restrict__ gw) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = g.ncut;
    if (q >= nc) return;
    double d1 = g.dd[q], d2 = g.dd[nc + q];
    double den = d1 * d2 * (d2 - d1) * g.grid.h;
    for (int j = 0; j < 3; j++) {
        const double* uj = u + (long)j * g.N;
        double ue = g.ueb[j];
        double s1 = 0.0, s2 = 0.0;
        for (int m = 0; m < 9; m++) {
            int c1 = g.sidx[(long)m * nc + q];
            s1 += g.sw[(long)m * nc + q] * (c1 >= 0 ? uj[c1] : ue);
        }
        for (int m = 9; m < 18; m++) {
            int c2 = g.sidx[(long)m * nc + q];
            s2 += g.sw[(long)m * nc + q] * (c2 >= 0 ? uj[c2] : ue);
        }
        gw[(long)j * nc + q] = (d2 * d2 * (s1 - ue) - d1 * d1 * (s2 - ue)) / den;
    }
}

// ------------------------------------------------------------------------------------------
// cell gradients (central / one-sided quadratic, Sec. III.B.4), strain rate and eta
// ------------------------------------------------------------------------------------------
__global__ void k_grad_eta(GeomV g, eb_rheology rh, const double* __restrict__ u,
                           const double* __restrict__ gw, const double* __restrict__ theta,
                           double* __restrict__ G9, double* __restrict__ eta,
                           double* __restrict__ sr) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    if (!(g.alpha[c] > 0.0)) {
        for (int a = 0; a < 9; a++) G9[a * N + c] = 0.0;
        eta[c] = rh.mu;
        if (sr) sr[c] = 0.0;
        return;
    }
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    double h = g.grid.h;
    double G[3][3];
    for (int d = 0; d < 3; d++) {
        long lo = nbr(g.grid, i, j, k, d, -1), hi = nbr(g.grid, i, j, k, d, 1);
        long lo2 = nbr(g.grid, i, j, k, d, -2), hi2 = nbr(g.grid, i, j, k, d, 2);
        bool lo_wall = lo < 0, hi_wall = hi < 0;
        bool lo_open = !lo_wall && g.alpha[lo] > 0.0;
        bool hi_open = !hi_wall && g.alpha[hi] > 0.0;
        bool lo2_open = lo2 >= 0 && g.alpha[lo2] > 0.0;
        bool hi2_open = hi2 >= 0 && g.alpha[hi2] > 0.0;
        bool lo_ok = lo_open || lo_wall, hi_ok = hi_open || hi_wall;
        for (int m = 0; m < 3; m++) {
            const double* um = u + (long)m * N;
            double uc = um[c];
            double vlo = lo_open ? um[lo] : 2.0 * g.wall[2 * d][m] - uc;
            double vhi = hi_open ? um[hi] : 2.0 * g.wall[2 * d + 1][m] - uc;
            double gr;
            if (lo_ok && hi_ok) {
                gr = (vhi - vlo) / (2.0 * h);
            } else if (hi_ok) {
                gr = (hi_open && hi2_open) ? (-1.5 * uc + 2.0 * vhi - 0.5 * um[hi2]) / h
                                           : (vhi - uc) / h;
            } else if (lo_ok) {
                gr = (lo_open && lo2_open) ? (1.5 * uc - 2.0 * vlo + 0.5 * um[lo2]) / h
                                           : (uc - vlo) / h;
            } else {
                int q = g.cutid[c];
                gr = q >= 0 ? g.nrm[(long)d * g.ncut + q] * gw[(long)m * g.ncut + q] : 0.0;
            }
            G[d][m] = gr;
        }
    }
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) G9[(a * 3 + b) * N + c] = G[a][b];
    double s = strain_rate(G);
    double t0 = rh.tau0 * (theta ? theta[c] : 1.0);
    eta[c] = eta_law(rh, t0, s);
    if (sr) sr[c] = s;
}

__global__ void k_eta_eb(GeomV g, eb_rheology rh, const double* __restrict__ gw,
                         const double* __restrict__ theta, double* __restrict__ eta_eb) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = g.ncut;
    if (q >= nc) return;
    double G[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) G[a][b] = g.nrm[(long)a * nc + q] * gw[(long)b * nc + q];
    double t0 = rh.tau0 * (theta ? theta[g.cut[q]] : 1.0);
    eta_eb[q] = eta_law(rh, t0, strain_rate(G));
}

// ------------------------------------------------------------------------------------------
// conservative divergence of the transpose stress eta (grad u)^T, per cell and component
// ------------------------------------------------------------------------------------------
__global__ void k_transpose_dc(GeomV g, const double* __restrict__ u,
                               const double* __restrict__ G9, const double* __restrict__ eta,
                               const double* __restrict__ eta_eb, const double* __restrict__ gw,
                               double* __restrict__ DC) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    double al = g.alpha[c];
    if (!(al > 0.0)) {
        for (int j = 0; j < 3; j++) DC[j * N + c] = 0.0;
        return;
    }
    int i, j0, k;
    cell_coords(g.grid, c, i, j0, k);
    double h = g.grid.h;
    int q = g.cutid[c];
    // every value the six faces need, loaded once: apertures, neighbours' viscosity and normal
    // velocity, and the two tangential gradient entries of the cell and of each neighbour
    long nb[6];
    double A[6], en[6], un[6], uc[3], gc[3][3], gn[6][3];
    double ec = eta[c];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        uc[d] = u[(long)d * N + c];
#pragma unroll
        for (int jj = 0; jj < 3; jj++) gc[jj][d] = jj == d ? 0.0 : G9[(jj * 3 + d) * N + c];
#pragma unroll
        for (int side = 0; side < 2; side++) {
            int f[3] = {i, j0, k};
            if (side) f[d] += 1;
            int fs = 2 * d + side;
            A[fs] = g.ap[d][face_index(g.grid, d, f[0], f[1], f[2])];
            nb[fs] = nbr(g.grid, i, j0, k, d, side ? 1 : -1);
            long n = nb[fs] >= 0 ? nb[fs] : c;
            en[fs] = eta[n];
            un[fs] = u[(long)d * N + n];
#pragma unroll
            for (int jj = 0; jj < 3; jj++) gn[fs][jj] = jj == d ? 0.0 : G9[(jj * 3 + d) * N + n];
        }
    }
    double ng = 0.0;
    if (q >= 0) {
        int nc = g.ncut;
        for (int a = 0; a < 3; a++) ng += g.nrm[(long)a * nc + q] * gw[(long)a * nc + q];
    }
    for (int j = 0; j < 3; j++) {
        double acc = 0.0;
        for (int d = 0; d < 3; d++) {
            for (int side = -1; side <= 1; side += 2) {
                int fs = 2 * d + (side > 0);
                if (A[fs] == 0.0) continue;
                double F;
                if (nb[fs] >= 0) {
                    double ef = 0.5 * (ec + en[fs]);
                    double der;
                    if (j == d)
                        der = side > 0 ? (un[fs] - uc[d]) / h : (uc[d] - un[fs]) / h;
                    else
                        der = 0.5 * (gc[j][d] + gn[fs][j]);
                    F = ef * der;
                } else {
                    double der = 0.0;
                    if (j == d) {
                        double uw = g.wall[2 * d + (side > 0)][d];
                        der = side > 0 ? (uw - uc[d]) / (0.5 * h) : (uc[d] - uw) / (0.5 * h);
                    }
                    F = ec * der;
                }
                acc += side * A[fs] * F;
            }
        }
        if (q >= 0) acc -= g.aeb[q] * eta_eb[q] * g.nrm[(long)j * g.ncut + q] * ng;
        DC[j * N + c] = acc / (al * h);
    }
}

// ------------------------------------------------------------------------------------------
// limited slopes and face states (Sec. III.A.3)
// ------------------------------------------------------------------------------------------
// limited slope of component j at c in direction d, computed, recorded or taken from the
// record (duplicate records of one slope by several threads carry the same value)
__device__ inline double slope_sw(const GeomV& g, const double* __restrict__ uj, long c, int d,
                                  int j, const SwitchV& sw) {
    if (sw.mode == 0) return mc_slope(g, uj, c, d);
    long at = (long)(3 * j + d) * g.N + c;
    int code = sw.mode == 2 ? (int)sw.slope[at] : mc_branch(g, uj, c, d);
    if (sw.mode == 1) sw.slope[at] = (uint8_t)code;
    return mc_eval(g, uj, c, d, code);
}

__global__ void k_face_extrap(GeomV g, int d, const double* __restrict__ u,
                              double* __restrict__ w, SwitchV sw) {
    long nf = face_count(g.grid, d);
    long f = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int i, j, k;
    face_coords(g.grid, d, f, i, j, k);
    long lo, hi;
    face_cells(g.grid, d, i, j, k, lo, hi);
    double val = 0.0;
    if (lo < 0 || hi < 0) {
        val = g.wall[2 * d + (lo >= 0)][d];
    } else if (g.ap[d][f] > 0.0) {
        const double* ud = u + (long)d * g.N;
        double uL = ud[lo] + 0.5 * slope_sw(g, ud, lo, d, d, sw);
        double uR = ud[hi] - 0.5 * slope_sw(g, ud, hi, d, d, sw);
        int side;  // normal upwinding: 1 left, 2 right, 0 neither
        if (sw.mode == 2) side = sw.norm[d][f];
        else side = (uL > 0.0 && uL + uR > 0.0) ? 1 : ((uR < 0.0 && uL + uR < 0.0) ? 2 : 0);
        if (sw.mode == 1) sw.norm[d][f] = (uint8_t)side;
        val = side == 1 ? uL : (side == 2 ? uR : 0.0);
    }
    w[f] = val;
}

__global__ void k_divergence(GeomV g, const double* __restrict__ fx,
                             const double* __restrict__ fy, const double* __restrict__ fz,
                             double* __restrict__ div) {
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= g.N) return;
    if (!(g.alpha[c] > 0.0)) {
        div[c] = 0.0;
        return;
    }
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    const double* fo[3] = {fx, fy, fz};
    double acc = 0.0;
    for (int d = 0; d < 3; d++) {
        int q[3] = {i, j, k};
        long f0 = face_index(g.grid, d, q[0], q[1], q[2]);
        q[d] += 1;
        long f1 = face_index(g.grid, d, q[0], q[1], q[2]);
        acc += g.ap[d][f1] * fo[d][f1] - g.ap[d][f0] * fo[d][f0];
    }
    int cq = g.cutid[c];
    if (cq >= 0) {
        int nc = g.ncut;
        double un = g.ueb[0] * g.nrm[cq] + g.ueb[1] * g.nrm[nc + cq] + g.ueb[2] * g.nrm[2 * nc + cq];
        acc -= g.aeb[cq] * un;
    }
    div[c] = acc / g.grid.h;
}

// convective flux divergence -(1/(alpha h)) sum_f A_f w_f u_up (upwinded by w_f)
// branch (0 zero, 1 central, 2 twice left, 3 twice right) and value of the
// monotonised-central slope from the three values along a line; ok: both neighbours exist and
// are open.  Together they are mc_branch / mc_eval (and mc_slope) on values already loaded.
__device__ __forceinline__ int mc_code(bool ok, double ul, double uc, double ur) {
    if (!ok) return 0;
    double dl = uc - ul, dr = ur - uc, dc = 0.5 * (ur - ul);
    if (dl * dr <= 0.0) return 0;
    double a = fabs(dc), b = 2.0 * fabs(dl), e = 2.0 * fabs(dr);
    if (a <= b && a <= e) return 1;
    return b <= e ? 2 : 3;
}
__device__ __forceinline__ double mc_val(int code, bool both, double ul, double uc, double ur) {
    if (code == 0 || !both) return 0.0;
    if (code == 1) return 0.5 * (ur - ul);
    return code == 2 ? 2.0 * (uc - ul) : 2.0 * (ur - uc);
}

// The convective term D^C of Eq. divergence_conservative for one cell: the six faces' upwind
// states from the extrapolations u +- slope/2 of the cells on either side.  Each thread loads
// its cell's five-cell line in every direction once (the cell, its neighbours and theirs) and
// forms the three slopes its two faces in that direction need, instead of every slope
// reloading its own stencil.  The slope branches are recorded (own cell) or replayed through
// sw like slope_sw, and every sum is in the order of the face loop, so D^C is unchanged.
__global__ void k_conv_dc(GeomV g, const double* __restrict__ u, const double* __restrict__ fx,
                          const double* __restrict__ fy, const double* __restrict__ fz,
                          double* __restrict__ DC, SwitchV sw) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    double al = g.alpha[c];
    if (!(al > 0.0)) {
        for (int j = 0; j < 3; j++) DC[j * N + c] = 0.0;
        return;
    }
    int i, j0, k;
    cell_coords(g.grid, c, i, j0, k);
    const double* fo[3] = {fx, fy, fz};
    double acc[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < 3; d++) {
        // the line c-2 .. c+2 along d (index -1 past a wall), its open flags and values
        long id[5];
        bool ex[5], op[5];
        double uv[3][5];
#pragma unroll
        for (int p = 0; p < 5; p++) {
            int q[3] = {i, j0, k};
            q[d] += p - 2;
            id[p] = p == 2 ? c : cell_at(g.grid, q[0], q[1], q[2]);
        }
#pragma unroll
        for (int p = 0; p < 5; p++) {
            ex[p] = id[p] >= 0;
            op[p] = p == 2 ? true : (ex[p] && g.alpha[ex[p] ? id[p] : c] > 0.0);
#pragma unroll
            for (int m = 0; m < 3; m++) uv[m][p] = ex[p] ? u[(long)m * N + id[p]] : 0.0;
        }
        // slopes at positions 1, 2, 3 (cells c-1, c, c+1) of each component
        double sl[3][3];
#pragma unroll
        for (int s3 = 0; s3 < 3; s3++) {
            int p = s3 + 1;
            bool both = ex[p - 1] && ex[p + 1];
            bool ok = both && op[p - 1] && op[p + 1];
#pragma unroll
            for (int m = 0; m < 3; m++) {
                double ul = uv[m][p - 1], uc = uv[m][p], ur = uv[m][p + 1];
                if (sw.mode == 0 || !ex[p]) {
                    sl[m][s3] = mc_val(mc_code(ok, ul, uc, ur), both, ul, uc, ur);
                    continue;
                }
                long at = (long)(3 * m + d) * N + id[p];
                int code = sw.mode == 2 ? (int)sw.slope[at] : mc_code(ok, ul, uc, ur);
                if (sw.mode == 1 && p == 2) sw.slope[at] = (uint8_t)code;
                sl[m][s3] = mc_val(code, both, ul, uc, ur);
            }
        }
        for (int side = -1; side <= 1; side += 2) {
            int f[3] = {i, j0, k};
            if (side > 0) f[d] += 1;
            long fi = face_index(g.grid, d, f[0], f[1], f[2]);
            double A = g.ap[d][fi];
            if (A == 0.0) continue;
            // lo and hi: positions 1 and 2 (side -1) or 2 and 3 (side +1)
            int pl = side < 0 ? 1 : 2, ph = pl + 1;
            bool lo_ok = ex[pl], hi_ok = ex[ph];
            double w = fo[d][fi];
            int ups = 0;  // upwind side by the face velocity: 1 left, 2 right, 3 the mean
            if (lo_ok && hi_ok) {
                if (sw.mode == 2) ups = sw.tr[d][fi];
                else ups = w > 0.0 ? 1 : (w < 0.0 ? 2 : 3);
                if (sw.mode == 1) sw.tr[d][fi] = (uint8_t)ups;
            }
            for (int m = 0; m < 3; m++) {
                double up;
                if (!lo_ok || !hi_ok) {
                    up = g.wall[2 * d + (lo_ok ? 1 : 0)][m];
                } else {
                    double uL = uv[m][pl] + 0.5 * sl[m][pl - 1];
                    double uR = uv[m][ph] - 0.5 * sl[m][ph - 1];
                    up = ups == 1 ? uL : (ups == 2 ? uR : 0.5 * (uL + uR));
                }
                acc[m] += side * A * w * up;
            }
        }
    }
    int cq = g.cutid[c];
    if (cq >= 0) {
        int nc = g.ncut;
        double un = -(g.ueb[0] * g.nrm[cq] + g.ueb[1] * g.nrm[nc + cq] +
                      g.ueb[2] * g.nrm[2 * nc + cq]);
        for (int j = 0; j < 3; j++) acc[j] += g.aeb[cq] * un * g.ueb[j];
    }
    for (int j = 0; j < 3; j++) DC[j * N + c] = -acc[j] / (al * g.grid.h);
}

// ------------------------------------------------------------------------------------------
// redistribution (Eqs. divergence_nonconservative ... divergence_final)
// ------------------------------------------------------------------------------------------
__global__ void k_redist_cut(GeomV g, const double* __restrict__ DC, double* __restrict__ DH,
                             double* __restrict__ S, double* __restrict__ dD) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = g.ncut;
    if (q >= nc) return;
    long N = g.N;
    long c = g.cut[q];
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    double s = 0.0, acc[3] = {0.0, 0.0, 0.0};
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                if (!dx && !dy && !dz) continue;
                long cc = cell_at(g.grid, i + dx, j + dy, k + dz);
                if (cc < 0) continue;
                double a = g.alpha[cc];
                if (!(a > 0.0)) continue;
                s += a;
                for (int m = 0; m < 3; m++) acc[m] += a * DC[m * N + cc];
            }
    double al = g.alpha[c];
    S[q] = s;
    for (int m = 0; m < 3; m++) {
        double dcv = DC[m * N + c];
        double dnc = s > 0.0 ? acc[m] / s : dcv;
        DH[(long)m * nc + q] = al * dcv + (1.0 - al) * dnc;
        dD[(long)m * nc + q] = al * (1.0 - al) * (dcv - dnc);
    }
}

__global__ void k_redist_gather(GeomV g, const double* __restrict__ DC,
                                const double* __restrict__ DH, const double* __restrict__ S,
                                const double* __restrict__ dD, double* __restrict__ D) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    if (!(g.alpha[c] > 0.0)) {
        for (int m = 0; m < 3; m++) D[m * N + c] = 0.0;
        return;
    }
    int nc = g.ncut;
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    int qc = g.flag[c] == 1 ? g.cutid[c] : -1;
    double acc[3];
    for (int m = 0; m < 3; m++) acc[m] = qc >= 0 ? DH[(long)m * nc + qc] : DC[m * N + c];
    double extra[3] = {0.0, 0.0, 0.0};
    // a cell with no cut cell in its 3x3x3 block receives nothing: skip the neighbour scan
    if (!g.near[c]) {
        for (int m = 0; m < 3; m++) D[m * N + c] = acc[m] + extra[m];
        return;
    }
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                if (!dx && !dy && !dz) continue;
                long cc = cell_at(g.grid, i + dx, j + dy, k + dz);
                if (cc < 0 || g.flag[cc] != 1) continue;
                int q = g.cutid[cc];
                double sq = S[q];
                if (!(sq > 0.0)) continue;
                for (int m = 0; m < 3; m++) extra[m] += dD[(long)m * nc + q] / sq;
            }
    for (int m = 0; m < 3; m++) D[m * N + c] = acc[m] + extra[m];
}

// ------------------------------------------------------------------------------------------
// projections, pressure gradient, RHS assembly
// ------------------------------------------------------------------------------------------
// component d of the cell-centred pressure gradient of open cell c = (i, j, k): the
// aperture-weighted mean of its two face gradients (a domain-wall face carries 0)
__device__ inline double gcc_cell(const GeomV& g, const double* __restrict__ p, long c, int i,
                                  int j, int k, int d) {
    double h = g.grid.h;
    double num = 0.0, den = 0.0;
    for (int side = -1; side <= 1; side += 2) {
        int f[3] = {i, j, k};
        if (side > 0) f[d] += 1;
        double A = g.ap[d][face_index(g.grid, d, f[0], f[1], f[2])];
        if (A == 0.0) continue;
        long nb = nbr(g.grid, i, j, k, d, side);
        double gf = 0.0;
        if (nb >= 0) gf = side > 0 ? (p[nb] - p[c]) / h : (p[c] - p[nb]) / h;
        num += A * gf;
        den += A;
    }
    return den > 0.0 ? num / den : 0.0;
}

__global__ void k_gcc(GeomV g, const double* __restrict__ p, double* __restrict__ gp) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    if (!(g.alpha[c] > 0.0)) {
        for (int d = 0; d < 3; d++) gp[d * N + c] = 0.0;
        return;
    }
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    for (int d = 0; d < 3; d++) gp[d * N + c] = gcc_cell(g, p, c, i, j, k, d);
}

__global__ void k_axpy_open(GeomV g, double a, const double* __restrict__ x,
                            double* __restrict__ y, int ncomp) {
    long N = g.N;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= N * ncomp) return;
    long c = (long)((unsigned)t % (unsigned)N);  // 3N < 2^32
    if (g.alpha[c] > 0.0) y[t] += a * x[t];
}

__global__ void k_cell_to_face(GeomV g, int d, const double* __restrict__ u,
                               double* __restrict__ w) {
    long nf = face_count(g.grid, d);
    long f = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int i, j, k;
    face_coords(g.grid, d, f, i, j, k);
    long lo, hi;
    face_cells(g.grid, d, i, j, k, lo, hi);
    double v = 0.0;
    if (lo < 0 || hi < 0)
        v = g.wall[2 * d + (lo >= 0)][d];
    else if (g.ap[d][f] > 0.0)
        v = 0.5 * (u[(long)d * g.N + lo] + u[(long)d * g.N + hi]);
    w[f] = v;
}

__global__ void k_face_correct(GeomV g, int d, double beta, const double* __restrict__ p,
                               double* __restrict__ w) {
    long nf = face_count(g.grid, d);
    long f = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int i, j, k;
    face_coords(g.grid, d, f, i, j, k);
    long lo, hi;
    face_cells(g.grid, d, i, j, k, lo, hi);
    if (lo < 0 || hi < 0 || g.ap[d][f] == 0.0) return;
    w[f] -= beta * (p[hi] - p[lo]) / g.grid.h;
}

__global__ void k_psi(GeomV g, double rho, double dt, const double* __restrict__ u,
                      const double* __restrict__ C, const double* __restrict__ V,
                      const double* __restrict__ gp, double f0, double f1, double f2,
                      double* __restrict__ psi) {
    long N = g.N;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 3 * N) return;
    int d = (int)(t / N);
    double fd = d == 0 ? f0 : (d == 1 ? f1 : f2);
    psi[t] = rho * u[t] + dt * (rho * C[t] + V[t] - gp[t] + fd);
}

__global__ void k_average(long n, const double* __restrict__ a, double* __restrict__ b) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) b[t] = 0.5 * (a[t] + b[t]);
}

__global__ void k_finalize_state(GeomV g, double* __restrict__ u, double* __restrict__ p) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    if (!(g.alpha[c] > 0.0)) {
        for (int d = 0; d < 3; d++) u[d * N + c] = g.ueb[d];
        if (p) p[c] = 0.0;  // null for a nodal pressure
    }
}

// gp null: the pressure gradient of each cut cell is formed here (gcc_cell, the same
// arithmetic as k_gcc) instead of being read from a full [3][N] array
// peb non-null: the wall pressure of each cut cell is given (the nodal projection's pressure
// interpolated at the wall centroid) and p, gp are not read
__global__ void k_drag_terms(GeomV g, eb_rheology rh, const double* __restrict__ theta,
                             const double* __restrict__ gw, const double* __restrict__ p,
                             const double* __restrict__ gp, double* __restrict__ terms,
                             const double* __restrict__ peb) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = g.ncut;
    if (q >= nc) return;
    long N = g.N;
    long c = g.cut[q];
    int ci, cj, ck;
    cell_coords(g.grid, c, ci, cj, ck);
    double nv[3], gv[3];
    for (int a = 0; a < 3; a++) {
        nv[a] = g.nrm[(long)a * nc + q];
        gv[a] = gw[(long)a * nc + q];
    }
    double G[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) G[a][b] = nv[a] * gv[b];
    double t0 = rh.tau0 * (theta ? theta[c] : 1.0);
    double e = eta_law(rh, t0, strain_rate(G));
    double h = g.grid.h;
    double pe;
    if (peb) {
        pe = peb[q];
    } else {
        pe = p[c];
        for (int d = 0; d < 3; d++)
            pe += h * g.bc[(long)d * nc + q] *
                  (gp ? gp[d * N + c] : gcc_cell(g, p, c, ci, cj, ck, d));
    }
    double area = g.aeb[q] * h * h;
    for (int a = 0; a < 3; a++) {
        double tn = 0.0;
        for (int b = 0; b < 3; b++) tn += e * (G[a][b] + G[b][a]) * nv[b];
        terms[(long)a * nc + q] = area * (tn - pe * nv[a]);
    }
}

// b = -(div - mean) on open cells; mean = sumcnt[0]/sumcnt[1] computed on the device
__global__ void k_poisson_rhs(GeomV g, const double* __restrict__ div,
                              const double* __restrict__ sumcnt, double* __restrict__ b) {
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= g.N) return;
    double mean = sumcnt[1] > 0.0 ? sumcnt[0] / sumcnt[1] : 0.0;
    b[c] = g.alpha[c] > 0.0 ? -(div[c] - mean) : 0.0;
}

// x -= mean on open cells (0 elsewhere)
__global__ void k_shift_open(GeomV g, double* __restrict__ x, const double* __restrict__ sumcnt,
                             const int* gate) {
    if (gate && *gate) return;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= g.N) return;
    double mean = sumcnt[1] > 0.0 ? sumcnt[0] / sumcnt[1] : 0.0;
    x[c] = g.alpha[c] > 0.0 ? x[c] - mean : 0.0;
}

}  // namespace

void op_wall_grad(const GeomV& g, const double* u, double* gw, hipStream_t s) {
    if (g.ncut > 0) k_wall_grad<<<grid_for(g.ncut), EB_BLOCK, 0, s>>>(g, u, gw);
}
void op_grad_eta(const GeomV& g, const eb_rheology& r, const double* u, const double* gw,
                 const double* theta, double* G9, double* eta, double* sr, hipStream_t s) {
    k_grad_eta<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, r, u, gw, theta, G9, eta, sr);
}
void op_eta_eb(const GeomV& g, const eb_rheology& r, const double* gw, const double* theta,
               double* eta_eb, hipStream_t s) {
    if (g.ncut > 0) k_eta_eb<<<grid_for(g.ncut), EB_BLOCK, 0, s>>>(g, r, gw, theta, eta_eb);
}
void op_transpose_dc(const GeomV& g, const double* u, const double* G9, const double* eta,
                     const double* eta_eb, const double* gw, double* DC, hipStream_t s) {
    k_transpose_dc<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, u, G9, eta, eta_eb, gw, DC);
}
void op_face_extrap(const GeomV& g, const double* u, double* f[3], const SwitchV& sw,
                    hipStream_t s) {
    for (int d = 0; d < 3; d++)
        k_face_extrap<<<grid_for(face_count(g.grid, d)), EB_BLOCK, 0, s>>>(g, d, u, f[d], sw);
}
void op_divergence(const GeomV& g, double* const f[3], double* div, hipStream_t s) {
    k_divergence<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, f[0], f[1], f[2], div);
}
void op_conv_dc(const GeomV& g, const double* u, double* const f[3], double* DC,
                const SwitchV& sw, hipStream_t s) {
    k_conv_dc<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, u, f[0], f[1], f[2], DC, sw);
}
void op_redistribute(const GeomV& g, const double* DC, double* DH, double* S, double* dD,
                     double* D, hipStream_t s) {
    if (g.ncut > 0) k_redist_cut<<<grid_for(g.ncut), EB_BLOCK, 0, s>>>(g, DC, DH, S, dD);
    k_redist_gather<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, DC, DH, S, dD, D);
}
void op_gcc(const GeomV& g, const double* p, double* gp, hipStream_t s) {
    k_gcc<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, p, gp);
}
void op_axpy_open(const GeomV& g, double a, const double* x, double* y, int ncomp,
                  hipStream_t s) {
    k_axpy_open<<<grid_for(g.N * ncomp), EB_BLOCK, 0, s>>>(g, a, x, y, ncomp);
}
void op_cell_to_face(const GeomV& g, const double* u, double* f[3], hipStream_t s) {
    for (int d = 0; d < 3; d++)
        k_cell_to_face<<<grid_for(face_count(g.grid, d)), EB_BLOCK, 0, s>>>(g, d, u, f[d]);
}
void op_face_correct(const GeomV& g, double beta, const double* p, double* f[3],
                     hipStream_t s) {
    for (int d = 0; d < 3; d++)
        k_face_correct<<<grid_for(face_count(g.grid, d)), EB_BLOCK, 0, s>>>(g, d, beta, p, f[d]);
}
void op_psi(const GeomV& g, double rho, double dt, const double* u, const double* C,
            const double* V, const double* gp, const double f[3], double* psi, hipStream_t s) {
    k_psi<<<grid_for(3 * g.N), EB_BLOCK, 0, s>>>(g, rho, dt, u, C, V, gp, f[0], f[1], f[2], psi);
}
void op_average(long n, const double* a, double* b, hipStream_t s) {
    if (n > 0) k_average<<<grid_for(n), EB_BLOCK, 0, s>>>(n, a, b);
}
void op_finalize_state(const GeomV& g, double* u, double* p, hipStream_t s) {
    k_finalize_state<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, u, p);
}
void op_drag_terms(const GeomV& g, const eb_rheology& r, const double* theta, const double* gw,
                   const double* p, const double* gp, double* terms, hipStream_t s,
                   const double* peb) {
    if (g.ncut > 0)
        k_drag_terms<<<grid_for(g.ncut), EB_BLOCK, 0, s>>>(g, r, theta, gw, p, gp, terms, peb);
}
void op_poisson_rhs(const GeomV& g, const double* div, const double* sumcnt, double* b,
                    hipStream_t s) {
    k_poisson_rhs<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, div, sumcnt, b);
}
void op_shift_open(const GeomV& g, double* x, const double* sumcnt, hipStream_t s,
                   const int* gate) {
    k_shift_open<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, x, sumcnt, gate);
}
