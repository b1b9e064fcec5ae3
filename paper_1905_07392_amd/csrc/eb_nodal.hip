// eb_nodal.hip -- the nodal end-of-stage projection (Sec. III.A.4 "Incompressibility constraint",
// Alg. advance NodalProjection): velocities on cell centres, the pressure on the nodes (cell
// corners), an approximate projection.  Discretisation: trilinear finite elements on each cell,
// weighted by the cell's volume fraction alpha.
//   D(w)_n  weak divergence of the cell field w against node n's hat function, minus the flux B_n
//           of the given boundary velocity (domain walls and the embedded wall);
//   L       the elements' stiffness matrix, L_nm = sum_c alpha_c h Khat(a, b), where the unit-cube
//           trilinear stiffness Khat is 1/3 on the diagonal, 0 between corners that differ in one
//           direction and -1/12 between corners that differ in two or three;
//   G(q)_c  the cell average of the gradient of q's trilinear interpolant.
// Nodal arrays are [nz+1][ny+1][nx+1], x fastest.  Every kernel is a gather over the (up to)
// eight cells around a node or the eight corners of a cell (no atomics, fixed order).  In a
// periodic direction the last node is a copy of the first: it sees the same cells, but it is not
// an unknown of the solve (its mask is 0) and is filled from the first after the solve.
#include "eb_internal.hpp"

namespace {

__device__ __forceinline__ long nd_index(const GridV& g, int i, int j, int k) {
    return (long)i + (long)(g.n[0] + 1) * ((long)j + (long)(g.n[1] + 1) * (long)k);
}
__device__ __forceinline__ void nd_coords(const GridV& g, long m, int& i, int& j, int& k) {
    unsigned mu = (unsigned)m, m0 = (unsigned)g.n[0] + 1, m1 = (unsigned)g.n[1] + 1;
    unsigned t = mu / m0;
    i = (int)(mu - t * m0);
    unsigned k2 = t / m1;
    j = (int)(t - k2 * m1);
    k = (int)k2;
}
// node of corner a (bit d: upper side in d) of cell (i, j, k), the last node of a periodic
// direction mapped to the first
__device__ __forceinline__ long nd_corner(const GridV& g, int i, int j, int k, int a) {
    int r[3] = {i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1)};
#pragma unroll
    for (int d = 0; d < 3; d++)
        if (g.per[d] && r[d] == g.n[d]) r[d] = 0;
    return nd_index(g, r[0], r[1], r[2]);
}
// cell o (bit d: 1 = the cell above node (i,j,k) in d) around node (i, j, k), or -1
__device__ __forceinline__ long nd_cell(const GridV& g, int i, int j, int k, int o, int q[3]) {
    q[0] = i - 1 + (o & 1);
    q[1] = j - 1 + ((o >> 1) & 1);
    q[2] = k - 1 + ((o >> 2) & 1);
#pragma unroll
    for (int d = 0; d < 3; d++) {
        if (q[d] < 0 || q[d] >= g.n[d]) {
            if (!g.per[d]) return -1;
            q[d] = q[d] < 0 ? q[d] + g.n[d] : q[d] - g.n[d];
        }
    }
    return cell_index(g, q[0], q[1], q[2]);
}
__device__ __forceinline__ bool nd_is_copy(const GridV& g, int i, int j, int k) {
    return (g.per[0] && i == g.n[0]) || (g.per[1] && j == g.n[1]) || (g.per[2] && k == g.n[2]);
}

// weak divergence minus the boundary flux (bflux nullable), and optionally the sum of the sizes
// of its terms (the solve's second scale); 0 on masked-out nodes when mask is given
__global__ void k_nd_div(GeomV g, const double* __restrict__ w, const double* __restrict__ bflux,
                         const uint8_t* __restrict__ mask, double* __restrict__ out,
                         double* __restrict__ tsum, long M) {
    long m = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (m >= M) return;
    int i, j, k;
    nd_coords(g.grid, m, i, j, k);
    long N = g.N;
    double h = g.grid.h;
    double s = 0.0, t = 0.0;
    for (int o = 0; o < 8; o++) {
        int q[3];
        long c = nd_cell(g.grid, i, j, k, o, q);
        if (c < 0) continue;
        double al = g.alpha[c];
        if (!(al > 0.0)) continue;
        int a = ~o & 7;
        double e = 0.0, ea = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            double wd = w[d * N + c];
            e += (((a >> d) & 1) ? 1.0 : -1.0) * wd;
            ea += fabs(wd);
        }
        s += al * h * h / 4.0 * e;
        t += al * h * h / 4.0 * ea;
    }
    if (bflux) s -= bflux[m];
    bool on = !mask || mask[m];
    out[m] = on ? s : 0.0;
    if (tsum) tsum[m] = on ? t : 0.0;
}

// boundary flux of the given normal velocity at each node: A_f h^2/4 (u_wall . n_out) per
// domain-wall face at the node, A_EB h^2/8 (u_EB . -n_EB) per cut cell at the node
__global__ void k_nd_bflux(GeomV g, double* __restrict__ out, long M) {
    long m = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (m >= M) return;
    int ijk[3];
    nd_coords(g.grid, m, ijk[0], ijk[1], ijk[2]);
    double h = g.grid.h;
    double s = 0.0;
    for (int d = 0; d < 3; d++) {
        if (g.grid.per[d]) continue;
        for (int side = 0; side < 2; side++) {
            if (ijk[d] != (side ? g.grid.n[d] : 0)) continue;
            double un = g.wall[2 * d + side][d] * (side ? 1.0 : -1.0);
            int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            for (int o = 0; o < 4; o++) {
                int q[3];
                q[d] = side ? g.grid.n[d] - 1 : 0;
                q[t1] = ijk[t1] - 1 + (o & 1);
                q[t2] = ijk[t2] - 1 + (o >> 1);
                bool ok = true;
                for (int te = 0; te < 2; te++) {
                    int e = te ? t2 : t1;
                    if (q[e] < 0 || q[e] >= g.grid.n[e]) {
                        if (!g.grid.per[e]) ok = false;
                        else q[e] = q[e] < 0 ? q[e] + g.grid.n[e] : q[e] - g.grid.n[e];
                    }
                }
                if (!ok) continue;
                int f[3] = {q[0], q[1], q[2]};
                f[d] += side;
                double A = g.ap[d][face_index(g.grid, d, f[0], f[1], f[2])];
                if (A == 0.0) continue;
                s += A * h * h / 4.0 * un;
            }
        }
    }
    for (int o = 0; o < 8; o++) {
        int q[3];
        long c = nd_cell(g.grid, ijk[0], ijk[1], ijk[2], o, q);
        if (c < 0) continue;
        int cid = g.cutid[c];
        if (cid < 0) continue;
        double un = 0.0;
        for (int d = 0; d < 3; d++) un -= g.ueb[d] * g.nrm[(long)d * g.ncut + cid];
        s += g.aeb[cid] * h * h / 8.0 * un;
    }
    out[m] = s;
}

// the diagonal of L and the mask of the solve's unknowns (a node of an open cell that is not a
// periodic copy)
__global__ void k_nd_diag(GeomV g, double* __restrict__ dg, uint8_t* __restrict__ mask, long M) {
    long m = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (m >= M) return;
    int i, j, k;
    nd_coords(g.grid, m, i, j, k);
    double h = g.grid.h, s = 0.0;
    for (int o = 0; o < 8; o++) {
        int q[3];
        long c = nd_cell(g.grid, i, j, k, o, q);
        if (c < 0) continue;
        double al = g.alpha[c];
        if (al > 0.0) s += al * h / 3.0;
    }
    bool on = s > 0.0 && !nd_is_copy(g.grid, i, j, k);
    dg[m] = on ? s : 0.0;
    mask[m] = on ? 1 : 0;
}

// y = L x on the unknowns (0 elsewhere): per open cell around the node, alpha h (x_n/3 - the sum
// over the four corners that differ from the node's in two or three directions / 12)
__global__ void __launch_bounds__(EB_BLOCK)
    k_nd_apply(GeomV g, const double* __restrict__ x, const uint8_t* __restrict__ mask,
               double* __restrict__ y, long M, const int* gate) {
    if (gate && *gate) return;
    long m = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (m >= M) return;
    if (!mask[m]) {
        y[m] = 0.0;
        return;
    }
    int i, j, k;
    nd_coords(g.grid, m, i, j, k);
    double h = g.grid.h, xn = x[m], acc = 0.0;
    for (int o = 0; o < 8; o++) {
        int q[3];
        long c = nd_cell(g.grid, i, j, k, o, q);
        if (c < 0) continue;
        double al = g.alpha[c];
        if (!(al > 0.0)) continue;
        int a = ~o & 7;
        double far = 0.0;
        for (int b = 0; b < 8; b++) {
            int df = a ^ b;
            if ((df & (df - 1)) == 0) continue;  // same corner or one direction apart
            far += x[nd_corner(g.grid, q[0], q[1], q[2], b)];
        }
        acc += al * h * (xn / 3.0 - far / 12.0);
    }
    y[m] = acc;
}

// cell average of the gradient of q's trilinear interpolant on open cells (0 elsewhere)
__global__ void k_nd_grad(GeomV g, const double* __restrict__ qn, double* __restrict__ gp) {
    long N = g.N;
    long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (c >= N) return;
    if (!(g.alpha[c] > 0.0)) {
        for (int d = 0; d < 3; d++) gp[d * N + c] = 0.0;
        return;
    }
    int i, j, k;
    cell_coords(g.grid, c, i, j, k);
    double v[8];
#pragma unroll
    for (int a = 0; a < 8; a++) v[a] = qn[nd_corner(g.grid, i, j, k, a)];
    double h = g.grid.h;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < 8; a++) s += (((a >> d) & 1) ? 1.0 : -1.0) * v[a];
        gp[d * N + c] = s / (4.0 * h);
    }
}

// z = r / diag on the unknowns
__global__ void k_nd_jacobi(long M, const double* __restrict__ r, const double* __restrict__ dg,
                            const uint8_t* __restrict__ mask, double* __restrict__ z,
                            const int* gate) {
    if (gate && *gate) return;
    long m = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (m < M) z[m] = mask[m] ? r[m] / dg[m] : 0.0;
}

// per-block sums of x and of the count over the unknowns
__global__ void k_nd_sum(long M, const double* __restrict__ x, const uint8_t* __restrict__ mask,
                         double* __restrict__ part, const int* gate) {
    if (gate && *gate) return;
    __shared__ double sh[EB_BLOCK];
    double s = 0.0, cnt = 0.0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < M;
         t += (long)gridDim.x * blockDim.x)
        if (mask[t]) {
            s += x[t];
            cnt += 1.0;
        }
    // block sums in a fixed tree
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = EB_BLOCK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    double v = sh[0];
    __syncthreads();
    sh[threadIdx.x] = cnt;
    __syncthreads();
    for (int o = EB_BLOCK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v;
        part[gridDim.x + blockIdx.x] = sh[0];
    }
}

// x -= sum/count on the unknowns, 0 elsewhere
__global__ void k_nd_shift(long M, double* __restrict__ x, const uint8_t* __restrict__ mask,
                           const double* __restrict__ sumcnt, const int* gate) {
    if (gate && *gate) return;
    long m = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (m >= M) return;
    double mean = sumcnt[1] > 0.0 ? sumcnt[0] / sumcnt[1] : 0.0;
    x[m] = mask[m] ? x[m] - mean : 0.0;
}

// y = a x on the unknowns (0 elsewhere)
__global__ void k_nd_scale_masked(long M, double a, const double* __restrict__ x,
                                  const uint8_t* __restrict__ mask, double* __restrict__ y) {
    long m = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (m < M) y[m] = mask[m] ? a * x[m] : 0.0;
}

// the last node of a periodic direction takes the first node's value
__global__ void k_nd_sync(GridV g, double* __restrict__ x, long M) {
    long m = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (m >= M) return;
    int r[3];
    nd_coords(g, m, r[0], r[1], r[2]);
    bool copy = false;
    for (int d = 0; d < 3; d++)
        if (g.per[d] && r[d] == g.n[d]) {
            r[d] = 0;
            copy = true;
        }
    if (copy) x[m] = x[nd_index(g, r[0], r[1], r[2])];
}

// the nodal pressure at each cut cell's wall centroid: trilinear interpolation over its corners
__global__ void k_nd_peb(GeomV g, const double* __restrict__ pn, double* __restrict__ peb) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = g.ncut;
    if (q >= nc) return;
    int i, j, k;
    cell_coords(g.grid, g.cut[q], i, j, k);
    double xi[3];
    for (int d = 0; d < 3; d++) xi[d] = g.bc[(long)d * nc + q] + 0.5;
    double s = 0.0;
    for (int a = 0; a < 8; a++) {
        double wgt = 1.0;
        for (int d = 0; d < 3; d++) wgt *= ((a >> d) & 1) ? xi[d] : 1.0 - xi[d];
        s += wgt * pn[nd_corner(g.grid, i, j, k, a)];
    }
    peb[q] = s;
}

}  // namespace

long nd_count(const GridV& g) { return (long)(g.n[0] + 1) * (g.n[1] + 1) * (g.n[2] + 1); }

void nd_div(const GeomV& g, const double* w, const double* bflux, const uint8_t* mask,
            double* out, double* tsum, hipStream_t s) {
    long M = nd_count(g.grid);
    k_nd_div<<<grid_for(M), EB_BLOCK, 0, s>>>(g, w, bflux, mask, out, tsum, M);
}
void nd_setup(const GeomV& g, double* bflux, double* dg, uint8_t* mask, hipStream_t s) {
    long M = nd_count(g.grid);
    k_nd_bflux<<<grid_for(M), EB_BLOCK, 0, s>>>(g, bflux, M);
    k_nd_diag<<<grid_for(M), EB_BLOCK, 0, s>>>(g, dg, mask, M);
}
void nd_apply(const GeomV& g, const double* x, const uint8_t* mask, double* y, hipStream_t s,
              const int* gate) {
    long M = nd_count(g.grid);
    k_nd_apply<<<grid_for(M), EB_BLOCK, 0, s>>>(g, x, mask, y, M, gate);
}
void nd_grad(const GeomV& g, const double* q, double* gp, hipStream_t s) {
    k_nd_grad<<<grid_for(g.N), EB_BLOCK, 0, s>>>(g, q, gp);
}
void nd_jacobi(long M, const double* r, const double* dg, const uint8_t* mask, double* z,
               hipStream_t s, const int* gate) {
    k_nd_jacobi<<<grid_for(M), EB_BLOCK, 0, s>>>(M, r, dg, mask, z, gate);
}
void nd_mean_free(long M, double* x, const uint8_t* mask, double* part, double* sumcnt,
                  hipStream_t s, const int* gate) {
    int nb = red_blocks(M);
    k_nd_sum<<<nb, EB_BLOCK, 0, s>>>(M, x, mask, part, gate);
    red_final(part, nb, 2, 0, sumcnt, s, gate);
    k_nd_shift<<<grid_for(M), EB_BLOCK, 0, s>>>(M, x, mask, sumcnt, gate);
}
void nd_scale_masked(long M, double a, const double* x, const uint8_t* mask, double* y,
                     hipStream_t s) {
    k_nd_scale_masked<<<grid_for(M), EB_BLOCK, 0, s>>>(M, a, x, mask, y);
}
void nd_sync(const GridV& g, double* x, hipStream_t s) {
    long M = nd_count(g);
    k_nd_sync<<<grid_for(M), EB_BLOCK, 0, s>>>(g, x, M);
}
void nd_peb(const GeomV& g, const double* pn, double* peb, hipStream_t s) {
    if (g.ncut > 0) k_nd_peb<<<grid_for(g.ncut), EB_BLOCK, 0, s>>>(g, pn, peb);
}
