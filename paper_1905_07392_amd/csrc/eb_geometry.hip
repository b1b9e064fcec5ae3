// eb_geometry.hip -- cut-cell geometry on the device (Sec. III.B).
//
// The body is an implicit function psi (> 0 in the fluid) sampled at grid nodes.  Each cell edge
// with a change of sign carries one exact root of psi along the edge (psi is a quadric, so the
// root is the root of a quadratic).  A face's fluid part is the polygon bounded by its fluid
// corners and the cut points on its edges, so neighbouring cells see the same aperture.  Per cut
// cell: the EB normal comes from the apertures (the divergence theorem), the EB plane offset is
// the mean of n.p over the cut points, the volume fraction follows from the divergence theorem
// with the position field, and the EB centroid is the centroid of the plane's section of the
// cell.  The wall-flux stencil of Eqs. interpolation_distances and dudn is precomputed per cut
// cell.
#include "eb_internal.hpp"

namespace {

__device__ __forceinline__ long node_at(const GridV& g, int i, int j, int k) {
    return (long)i + (long)(g.n[0] + 1) * ((long)j + (long)(g.n[1] + 1) * (long)k);
}

__device__ double body_psi(const BodyV& b, double x, double y, double z) {
    switch (b.kind) {
    case EB_BODY_SPHERE: {
        double dx = x - b.c[0], dy = y - b.c[1], dz = z - b.c[2];
        return dx * dx + dy * dy + dz * dz - b.r[0] * b.r[0];
    }
    case EB_BODY_ELLIPSOID: {
        double v[3] = {x - b.c[0], y - b.c[1], z - b.c[2]};
        double acc = 0.0;
        for (int a = 0; a < 3; a++) {
            double ya = b.R[0][a] * v[0] + b.R[1][a] * v[1] + b.R[2][a] * v[2];
            double q = ya / b.r[a];
            acc += q * q;
        }
        return acc - 1.0;
    }
    case EB_BODY_ZSLAB:
        return (z - b.zlo) * (b.zhi - z);
    case EB_BODY_PLANE:
        return b.pn[0] * x + b.pn[1] * y + b.pn[2] * z - b.pd;
    case EB_BODY_CYLINDER: {
        double dx = x - b.c[0], dz = z - b.c[2];
        return dx * dx + dz * dz - b.r[0] * b.r[0];
    }
    case EB_BODY_CAVITY: {
        double dx = x - b.c[0], dy = y - b.c[1], dz = z - b.c[2];
        return b.r[0] * b.r[0] - (dx * dx + dy * dy + dz * dz);
    }
    default:
        return 1.0;
    }
}

// psi(x0 + t h e_d) = qa t^2 + qb t + psi(x0)
__device__ void body_edge_poly(const BodyV& b, const double x0[3], int d, double h, double& qa,
                               double& qb) {
    qa = 0.0;
    qb = 0.0;
    if (b.kind == EB_BODY_SPHERE) {
        qa = h * h;
        qb = 2.0 * h * (x0[d] - b.c[d]);
    } else if (b.kind == EB_BODY_ELLIPSOID) {
        double v[3] = {x0[0] - b.c[0], x0[1] - b.c[1], x0[2] - b.c[2]};
        for (int a = 0; a < 3; a++) {
            double ya = b.R[0][a] * v[0] + b.R[1][a] * v[1] + b.R[2][a] * v[2];
            double ra2 = b.r[a] * b.r[a];
            qa += h * h * b.R[d][a] * b.R[d][a] / ra2;
            qb += 2.0 * h * ya * b.R[d][a] / ra2;
        }
    } else if (b.kind == EB_BODY_ZSLAB) {
        if (d == 2) {
            qa = -h * h;
            qb = h * (b.zhi + b.zlo - 2.0 * x0[2]);
        }
    } else if (b.kind == EB_BODY_PLANE) {
        qb = h * b.pn[d];
    } else if (b.kind == EB_BODY_CYLINDER && d != 1) {
        qa = h * h;
        qb = 2.0 * h * (x0[d] - b.c[d]);
    } else if (b.kind == EB_BODY_CAVITY) {
        qa = -h * h;
        qb = -2.0 * h * (x0[d] - b.c[d]);
    }
}

// the root in [0,1] of qa t^2 + qb t + p0, knowing p(0) = p0 and p(1) = p1 differ in sign class
__device__ double quad_root01(double qa, double qb, double p0, double p1) {
    if (p0 == 0.0) return 0.0;
    if (p1 == 0.0) return 1.0;
    double t;
    if (qa == 0.0) {
        t = -p0 / qb;
    } else {
        double disc = qb * qb - 4.0 * qa * p0;
        disc = disc > 0.0 ? disc : 0.0;
        double sq = sqrt(disc);
        double q = qb >= 0.0 ? -0.5 * (qb + sq) : -0.5 * (qb - sq);
        double ra = q / qa;
        double rb = q != 0.0 ? p0 / q : ra;
        bool ina = ra >= 0.0 && ra <= 1.0;
        bool inb = rb >= 0.0 && rb <= 1.0;
        if (ina && !inb) t = ra;
        else if (inb && !ina) t = rb;
        else if (ina && inb) t = fabs(ra - 0.5) <= fabs(rb - 0.5) ? ra : rb;
        else {
            double ea = ra < 0.0 ? -ra : ra - 1.0;
            double eb = rb < 0.0 ? -rb : rb - 1.0;
            t = ea <= eb ? ra : rb;
        }
    }
    return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
}

// edge from node (i,j,k) along d: true and the cut fraction t when the fluid state changes
__device__ bool edge_cut(const GridV& g, const BodyV& b, const double* psi, int i, int j, int k,
                         int d, double& t) {
    int q1[3] = {i, j, k};
    q1[d] += 1;
    double p0 = psi[node_at(g, i, j, k)];
    double p1 = psi[node_at(g, q1[0], q1[1], q1[2])];
    if ((p0 > 0.0) == (p1 > 0.0)) return false;
    double x0[3] = {b.lo[0] + i * g.h, b.lo[1] + j * g.h, b.lo[2] + k * g.h};
    double qa, qb;
    body_edge_poly(b, x0, d, g.h, qa, qb);
    t = quad_root01(qa, qb, p0, p1);
    return true;
}

__global__ void k_node_psi(GridV g, BodyV b, double* psi) {
    long nn = (long)(g.n[0] + 1) * (g.n[1] + 1) * (g.n[2] + 1);
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= nn) return;
    int i = (int)(t % (g.n[0] + 1));
    long r = t / (g.n[0] + 1);
    int j = (int)(r % (g.n[1] + 1));
    int k = (int)(r / (g.n[1] + 1));
    psi[t] = body_psi(b, b.lo[0] + i * g.h, b.lo[1] + j * g.h, b.lo[2] + k * g.h);
}

__global__ void k_face_aperture(GridV g, BodyV b, const double* psi, int d, double* ap,
                                int* err) {
    long nf = face_count(g, d);
    long f = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int m0 = g.n[0] + (d == 0), m1 = g.n[1] + (d == 1);
    int q[3];
    q[0] = (int)(f % m0);
    long r = f / m0;
    q[1] = (int)(r % m1);
    q[2] = (int)(r / m1);
    int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    // corners in counter-clockwise order in the (t1, t2) plane
    int oc1[4] = {0, 1, 1, 0}, oc2[4] = {0, 0, 1, 1};
    bool fl[4];
    int nfl = 0;
    for (int m = 0; m < 4; m++) {
        int c[3] = {q[0], q[1], q[2]};
        c[t1] += oc1[m];
        c[t2] += oc2[m];
        fl[m] = psi[node_at(g, c[0], c[1], c[2])] > 0.0;
        nfl += fl[m];
    }
    if (nfl == 4) {
        ap[f] = 1.0;
        return;
    }
    if (nfl == 0) {
        ap[f] = 0.0;
        return;
    }
    double vx[8], vy[8];
    int nv = 0, ncuts = 0;
    for (int m = 0; m < 4; m++) {
        if (fl[m]) {
            vx[nv] = oc1[m];
            vy[nv] = oc2[m];
            nv++;
        }
        int m2 = (m + 1) & 3;
        if (fl[m] != fl[m2]) {
            // the edge between corners m and m2, evaluated from its low node
            int lo1 = oc1[m] < oc1[m2] ? oc1[m] : oc1[m2];
            int lo2 = oc2[m] < oc2[m2] ? oc2[m] : oc2[m2];
            int dir = (oc1[m] != oc1[m2]) ? t1 : t2;
            int c[3] = {q[0], q[1], q[2]};
            c[t1] += lo1;
            c[t2] += lo2;
            double t = 0.0;
            edge_cut(g, b, psi, c[0], c[1], c[2], dir, t);
            if (dir == t1) {
                vx[nv] = t;
                vy[nv] = lo2;
            } else {
                vx[nv] = lo1;
                vy[nv] = t;
            }
            nv++;
            ncuts++;
        }
    }
    if (ncuts > 2) atomicOr(err, 1);
    double a2 = 0.0;
    for (int m = 0; m < nv; m++) {
        int m2 = m + 1 == nv ? 0 : m + 1;
        a2 += vx[m] * vy[m2] - vx[m2] * vy[m];
    }
    ap[f] = 0.5 * fabs(a2);
}

__global__ void k_face_periodic_copy(GridV g, int d, double* ap) {
    // the face at index n_d along d duplicates face 0
    int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    long nt = (long)g.n[t1] * g.n[t2];
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= nt) return;
    int a = (int)(t % g.n[t1]);
    int bq = (int)(t / g.n[t1]);
    int q[3];
    q[t1] = a;
    q[t2] = bq;
    q[d] = 0;
    long f0 = face_index(g, d, q[0], q[1], q[2]);
    q[d] = g.n[d];
    ap[face_index(g, d, q[0], q[1], q[2])] = ap[f0];
}

struct CutGeo {
    double nv[3];
    double aeb;
    double s;      // plane n.x = s in cell-centred units
    double alpha;
};

// apertures of cell (i,j,k) -> class: 2 regular, 0 covered, 1 cut (geo filled), -1 degenerate
__device__ int classify(const GridV& g, const BodyV& b, const double* psi, const double* ax,
                        const double* ay, const double* az, int i, int j, int k, CutGeo& cg) {
    const double* aps[3] = {ax, ay, az};
    double a[3][2];
    bool all1 = true, all0 = true;
    double sum = 0.0;
    for (int d = 0; d < 3; d++)
        for (int s = 0; s < 2; s++) {
            int q[3] = {i, j, k};
            q[d] += s;
            double v = aps[d][face_index(g, d, q[0], q[1], q[2])];
            a[d][s] = v;
            all1 = all1 && v == 1.0;
            all0 = all0 && v == 0.0;
            sum += v;
        }
    if (all1) return 2;
    if (all0) return 0;
    double m[3], mm = 0.0;
    for (int d = 0; d < 3; d++) {
        m[d] = a[d][1] - a[d][0];
        mm += m[d] * m[d];
    }
    double aeb = sqrt(mm);
    if (aeb == 0.0) return -1;
    for (int d = 0; d < 3; d++) cg.nv[d] = m[d] / aeb;
    cg.aeb = aeb;
    double acc = 0.0;
    int npts = 0;
    for (int d = 0; d < 3; d++) {
        int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        for (int o = 0; o < 4; o++) {
            int o1 = o & 1, o2 = o >> 1;
            int q[3] = {i, j, k};
            q[t1] += o1;
            q[t2] += o2;
            double t;
            if (edge_cut(g, b, psi, q[0], q[1], q[2], d, t)) {
                double p[3];
                p[d] = t - 0.5;
                p[t1] = o1 - 0.5;
                p[t2] = o2 - 0.5;
                acc += cg.nv[0] * p[0] + cg.nv[1] * p[1] + cg.nv[2] * p[2];
                npts++;
            }
        }
    }
    cg.s = npts ? acc / npts : 0.0;
    double al = (0.5 * sum - cg.s * aeb) / 3.0;
    cg.alpha = al > 1.0 ? 1.0 : (al < 1e-12 ? 1e-12 : al);
    return 1;
}

__global__ void k_cells(GridV g, BodyV b, const double* psi, const double* ax, const double* ay,
                        const double* az, uint8_t* flag, double* alpha, int* cutid,
                        int* blockcount, int* err) {
    long N = (long)g.n[0] * g.n[1] * g.n[2];
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    int is_cut = 0;
    if (c < N) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        CutGeo cg;
        int cls = classify(g, b, psi, ax, ay, az, i, j, k, cg);
        if (cls < 0) {
            atomicOr(err, 2);
            cls = 0;
        }
        flag[c] = (uint8_t)cls;
        alpha[c] = cls == 2 ? 1.0 : (cls == 0 ? 0.0 : cg.alpha);
        cutid[c] = -1;
        is_cut = cls == 1;
    }
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    if (is_cut) atomicAdd(&cnt, 1);
    __syncthreads();
    if (threadIdx.x == 0) blockcount[blockIdx.x] = cnt;
}

// exclusive scan of the per-block counts by one block (each thread scans a contiguous chunk)
__global__ void k_scan_counts(int* blockcount, int nb, int* total) {
    __shared__ int part[1024];
    int tid = threadIdx.x;
    int chunk = (nb + blockDim.x - 1) / blockDim.x;
    int lo = tid * chunk, hi = min(nb, lo + chunk);
    int s = 0;
    for (int t = lo; t < hi; t++) s += blockcount[t];
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int t = 0; t < (int)blockDim.x; t++) {
            int v = part[t];
            part[t] = run;
            run += v;
        }
        *total = run;
    }
    __syncthreads();
    int run = part[tid];
    for (int t = lo; t < hi; t++) {
        int v = blockcount[t];
        blockcount[t] = run;
        run += v;
    }
}

// ordered compaction: cut cells in ascending cell order
__global__ void k_scatter_cut(long N, const uint8_t* flag, const int* blockoff, int* cut,
                              int ncut_max) {
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    int is_cut = c < N && flag[c] == 1;
    __shared__ int pref[EB_BLOCK];
    pref[threadIdx.x] = is_cut;
    __syncthreads();
    // inclusive scan in shared memory (Hillis-Steele)
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        int v = threadIdx.x >= (unsigned)off ? pref[threadIdx.x - off] : 0;
        __syncthreads();
        pref[threadIdx.x] += v;
        __syncthreads();
    }
    if (is_cut) {
        int pos = blockoff[blockIdx.x] + pref[threadIdx.x] - 1;
        if (pos < ncut_max) cut[pos] = (int)c;
    }
}

// centroid of the polygon where the plane n.x = s cuts the cell [-1/2,1/2]^3
__device__ void section_centroid(const double nv[3], double s, double out[3]) {
    double P[12][3];
    int np = 0;
    for (int d = 0; d < 3; d++) {
        if (nv[d] == 0.0) continue;
        int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        for (int o = 0; o < 4; o++) {
            double x1 = (o & 1) - 0.5, x2 = (o >> 1) - 0.5;
            double xd = (s - nv[t1] * x1 - nv[t2] * x2) / nv[d];
            if (xd >= -0.5 && xd <= 0.5) {
                P[np][d] = xd;
                P[np][t1] = x1;
                P[np][t2] = x2;
                np++;
            }
        }
    }
    if (np == 0) {
        for (int e = 0; e < 3; e++) out[e] = s * nv[e];
        return;
    }
    double m0[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < np; q++)
        for (int e = 0; e < 3; e++) m0[e] += P[q][e] / np;
    // orthonormal in-plane frame from the axis least aligned with n
    int dm = 0;
    for (int e = 1; e < 3; e++)
        if (fabs(nv[e]) < fabs(nv[dm])) dm = e;
    double e1[3] = {-nv[dm] * nv[0], -nv[dm] * nv[1], -nv[dm] * nv[2]};
    e1[dm] += 1.0;
    double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int e = 0; e < 3; e++) e1[e] /= l1;
    double e2[3] = {nv[1] * e1[2] - nv[2] * e1[1], nv[2] * e1[0] - nv[0] * e1[2],
                    nv[0] * e1[1] - nv[1] * e1[0]};
    double ang[12];
    for (int q = 0; q < np; q++) {
        double ax = 0.0, ay = 0.0;
        for (int e = 0; e < 3; e++) {
            ax += (P[q][e] - m0[e]) * e1[e];
            ay += (P[q][e] - m0[e]) * e2[e];
        }
        ang[q] = atan2(ay, ax);
    }
    for (int q = 1; q < np; q++) {  // insertion sort by angle
        double a = ang[q], v0 = P[q][0], v1 = P[q][1], v2 = P[q][2];
        int m = q - 1;
        while (m >= 0 && ang[m] > a) {
            ang[m + 1] = ang[m];
            P[m + 1][0] = P[m][0];
            P[m + 1][1] = P[m][1];
            P[m + 1][2] = P[m][2];
            m--;
        }
        ang[m + 1] = a;
        P[m + 1][0] = v0;
        P[m + 1][1] = v1;
        P[m + 1][2] = v2;
    }
    double area = 0.0, cs[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < np; q++) {
        int q2 = q + 1 == np ? 0 : q + 1;
        double a[3], bb[3];
        for (int e = 0; e < 3; e++) {
            a[e] = P[q][e] - m0[e];
            bb[e] = P[q2][e] - m0[e];
        }
        double cr0 = a[1] * bb[2] - a[2] * bb[1];
        double cr1 = a[2] * bb[0] - a[0] * bb[2];
        double cr2 = a[0] * bb[1] - a[1] * bb[0];
        double tri = 0.5 * (cr0 * nv[0] + cr1 * nv[1] + cr2 * nv[2]);
        area += tri;
        for (int e = 0; e < 3; e++) cs[e] += tri * (m0[e] + P[q][e] + P[q2][e]) / 3.0;
    }
    if (fabs(area) < 1e-300) {
        for (int e = 0; e < 3; e++) out[e] = m0[e];
    } else {
        for (int e = 0; e < 3; e++) out[e] = cs[e] / area;
    }
}

__global__ void k_cut_fill(GridV g, BodyV b, const double* psi, const double* ax,
                           const double* ay, const double* az, const int* cut, int ncut,
                           int* cutid, double* nrm, double* aeb, double* bc, double* delta) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ncut) return;
    long c = cut[q];
    int i, j, k;
    cell_coords(g, c, i, j, k);
    CutGeo cg;
    classify(g, b, psi, ax, ay, az, i, j, k, cg);
    cutid[c] = q;
    for (int e = 0; e < 3; e++) nrm[e * ncut + q] = cg.nv[e];
    aeb[q] = cg.aeb;
    double cen[3];
    section_centroid(cg.nv, cg.s, cen);
    for (int e = 0; e < 3; e++) bc[e * ncut + q] = cen[e];
    delta[q] = -cg.s;
}

__device__ __forceinline__ void lagrange_w(double x, double w[3]) {
    // nodes -1, 0, +1 (App. A)
    w[0] = 0.5 * x * (x - 1.0);
    w[1] = (1.0 - x) * (1.0 + x);
    w[2] = 0.5 * x * (x + 1.0);
}

__global__ void k_wall_stencil(GeomV g, double* dd, int* sidx, double* sw, int* nfb, int* err) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = g.ncut;
    if (q >= nc) return;
    long c = g.cut[q];
    int ijk[3];
    cell_coords(g.grid, c, ijk[0], ijk[1], ijk[2]);
    double nv[3] = {g.nrm[q], g.nrm[nc + q], g.nrm[2 * nc + q]};
    double bb[3] = {g.bc[q], g.bc[nc + q], g.bc[2 * nc + q]};
    int ds = 0;
    if (fabs(nv[1]) > fabs(nv[ds])) ds = 1;
    if (fabs(nv[2]) > fabs(nv[ds])) ds = 2;
    int sg = nv[ds] > 0.0 ? 1 : -1;
    int t1 = ds == 0 ? 1 : 0, t2 = ds == 2 ? 1 : 2;
    int fb = 0;
    for (int kk = 1; kk <= 2; kk++) {
        double dk = (kk * sg - bb[ds]) / nv[ds];
        dd[(kk - 1) * nc + q] = dk;
        double p1 = bb[t1] + dk * nv[t1], p2 = bb[t2] + dk * nv[t2];
        int c1 = (int)floor(p1 + 0.5), c2 = (int)floor(p2 + 0.5);
        bool ok = false;
        for (int attempt = 0; attempt < 2 && !ok; attempt++) {
            if (attempt == 1) {
                c1 += (nv[t1] > 0.0) - (nv[t1] < 0.0);
                c2 += (nv[t2] > 0.0) - (nv[t2] < 0.0);
            }
            ok = true;
            for (int m = 0; m < 9; m++) {
                int r[3];
                r[ds] = ijk[ds] + kk * sg;
                r[t1] = ijk[t1] + c1 + m / 3 - 1;
                r[t2] = ijk[t2] + c2 + m % 3 - 1;
                long cc = cell_at(g.grid, r[0], r[1], r[2]);
                if (cc < 0) {
                    atomicOr(err, 4);
                    return;
                }
                if (!(g.alpha[cc] > 0.0)) ok = false;
            }
        }
        if (!ok) fb++;
        double w1[3], w2[3];
        lagrange_w(p1 - c1, w1);
        lagrange_w(p2 - c2, w2);
        for (int m = 0; m < 9; m++) {
            int r[3];
            r[ds] = ijk[ds] + kk * sg;
            r[t1] = ijk[t1] + c1 + m / 3 - 1;
            r[t2] = ijk[t2] + c2 + m % 3 - 1;
            long cc = cell_at(g.grid, r[0], r[1], r[2]);
            int slot = (kk - 1) * 9 + m;
            sw[(long)slot * nc + q] = w1[m / 3] * w2[m % 3];
            sidx[(long)slot * nc + q] = g.alpha[cc] > 0.0 ? (int)cc : -1;
        }
    }
    nfb[q] = fb;
}

__global__ void k_coarsen_alpha(GridV gc, GridV gf, const double* af, double* ac) {
    long Nc = (long)gc.n[0] * gc.n[1] * gc.n[2];
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= Nc) return;
    ac[c] = coarsen_cell_value(gc, gf, af, c);
}

__global__ void k_coarsen_face(GridV gc, GridV gf, int d, const double* ff, double* fc,
                               double scale) {
    long nf = face_count(gc, d);
    long f = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (f >= nf) return;
    fc[f] = coarsen_face_value(gc, gf, d, ff, f, scale);
}

__global__ void k_mark_near(GridV g, const int* __restrict__ cut, int ncut,
                            uint8_t* __restrict__ near) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ncut) return;
    int i, j, k;
    cell_coords(g, cut[q], i, j, k);
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                long cc = cell_at(g, i + dx, j + dy, k + dz);
                if (cc >= 0) near[cc] = 1;  // every writer stores the same value
            }
}

__global__ void k_mask(long N, const double* alpha, uint8_t* mask) {
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c < N) mask[c] = alpha[c] > 0.0 ? 1 : 0;
}

}  // namespace

int geom_build_device(const GridV& grid, const BodyV& body, double* psi, uint8_t* flag,
                      double* alpha, double* ap[3], int* cutid, int* cut, int* blockcount,
                      int ncut_max, int* ncut_out, int* err_dev, hipStream_t s) {
    long nn = (long)(grid.n[0] + 1) * (grid.n[1] + 1) * (grid.n[2] + 1);
    long N = (long)grid.n[0] * grid.n[1] * grid.n[2];
    HIPN(hipMemsetAsync(err_dev, 0, sizeof(int), s));
    k_node_psi<<<grid_for(nn), EB_BLOCK, 0, s>>>(grid, body, psi);
    for (int d = 0; d < 3; d++) {
        k_face_aperture<<<grid_for(face_count(grid, d)), EB_BLOCK, 0, s>>>(grid, body, psi, d,
                                                                          ap[d], err_dev);
        if (grid.per[d]) {
            int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            k_face_periodic_copy<<<grid_for((long)grid.n[t1] * grid.n[t2]), EB_BLOCK, 0, s>>>(
                grid, d, ap[d]);
        }
    }
    int nb = (int)grid_for(N);
    k_cells<<<nb, EB_BLOCK, 0, s>>>(grid, body, psi, ap[0], ap[1], ap[2], flag, alpha, cutid,
                                    blockcount, err_dev);
    k_scan_counts<<<1, 1024, 0, s>>>(blockcount, nb, blockcount + nb);
    k_scatter_cut<<<nb, EB_BLOCK, 0, s>>>(N, flag, blockcount, cut, ncut_max);
    int tot = 0;
    HIPN(hipMemcpyAsync(&tot, blockcount + nb, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPN(hipStreamSynchronize(s));
    *ncut_out = tot;
    return 0;
}

void geom_cut_fill(const GridV& grid, const BodyV& body, const double* psi, const double* ap[3],
                   const int* cut, int ncut, int* cutid, double* nrm, double* aeb, double* bc,
                   double* delta, hipStream_t s) {
    if (ncut <= 0) return;
    k_cut_fill<<<grid_for(ncut), EB_BLOCK, 0, s>>>(grid, body, psi, ap[0], ap[1], ap[2], cut,
                                                   ncut, cutid, nrm, aeb, bc, delta);
}

void geom_wall_stencil(const GeomV& g, double* dd, int* sidx, double* sw, int* nfb, int* err,
                       hipStream_t s) {
    if (g.ncut <= 0) return;
    k_wall_stencil<<<grid_for(g.ncut), EB_BLOCK, 0, s>>>(g, dd, sidx, sw, nfb, err);
}

void level_coarsen_geometry(const Level& F, Level& C, hipStream_t s) {
    k_coarsen_alpha<<<grid_for(C.N), EB_BLOCK, 0, s>>>(C.grid, F.grid, F.alpha, C.alpha);
    for (int d = 0; d < 3; d++)
        k_coarsen_face<<<grid_for(face_count(C.grid, d)), EB_BLOCK, 0, s>>>(
            C.grid, F.grid, d, F.ap[d], C.ap[d], 0.25);
}

void geom_mark_near(const GridV& g, const int* cut, int ncut, uint8_t* near, hipStream_t s) {
    long N = (long)g.n[0] * g.n[1] * g.n[2];
    HIPN(hipMemsetAsync(near, 0, N, s));
    if (ncut > 0) k_mark_near<<<grid_for(ncut), EB_BLOCK, 0, s>>>(g, cut, ncut, near);
}

void level_mask(Level& L, hipStream_t s) {
    k_mask<<<grid_for(L.N), EB_BLOCK, 0, s>>>(L.N, L.alpha, L.mask);
}

