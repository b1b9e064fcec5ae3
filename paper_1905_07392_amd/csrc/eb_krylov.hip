// eb_krylov.hip -- Krylov coefficients and convergence state kept on the device.
//
// The host enqueues whole iterations without waiting; every scalar (alpha, beta, omega, rho,
// norms) lives in a small device array and every kernel of an iteration reads a device state
// word: 0 running, 1 converged at the half step (BiCGSTAB, x update pending), 2 converged,
// 3 non-finite residual.  Once the state leaves 0 the remaining kernels of the solve return at
// once, so iterations the host enqueued ahead of the convergence test do no work.  The
// iteration number is counted on the device as well, so every iteration launches identical
// kernels with identical arguments (and can be replayed as one captured graph).
#include "eb_internal.hpp"

namespace {

__global__ void k_scal(int op, double* __restrict__ ks, int* __restrict__ st,
                       int* __restrict__ itc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    ks_scalar_op(op, ks, st, itc);
}

// p = z + beta p   (CG)
__global__ void k_cg_p(long n, double* __restrict__ p, const double* __restrict__ z,
                       const double* __restrict__ ks, const int* __restrict__ st) {
    if (*st != 0) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) p[t] = z[t] + ks[KS_BE] * p[t];
}
// p = r + beta (p - omega v) with beta = (rho / rho_old) (alpha / omega), formed by every
// thread from the scalars of the previous iteration   (BiCGSTAB)
__global__ void k_bi_p(long n, double* __restrict__ p, const double* __restrict__ r,
                       const double* __restrict__ v, const double* __restrict__ ks,
                       const int* __restrict__ st) {
    if (*st != 0) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    double be = (ks[KS_RR] / ks[KS_RHO_OLD]) * (ks[KS_AL] / ks[KS_OM]);
    if (t < n) p[t] = r[t] + be * (p[t] - ks[KS_OM] * v[t]);
}
// converged at the half step: x += alpha ph (grid-stride over a small grid: almost every launch
// returns at once, and a small grid returns sooner)
template <typename TP>
__global__ void k_bi_xs(long n, double* __restrict__ x, const TP* __restrict__ ph,
                        const double* __restrict__ ks, const int* __restrict__ st) {
    if (*st != 1) return;
    double al = ks[KS_AL];
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
         t += (long)gridDim.x * blockDim.x)
        x[t] += al * (double)ph[t];
}

__global__ void k_set(double* __restrict__ ks, int idx, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ks[idx] = v;
}

}  // namespace

void ks_op(int op, double* ks, int* st, int* itc, hipStream_t s) {
    k_scal<<<1, 64, 0, s>>>(op, ks, st, itc);
}
void ks_set(double* ks, int idx, double v, hipStream_t s) { k_set<<<1, 64, 0, s>>>(ks, idx, v); }
void ks_cg_p(long n, double* p, const double* z, const double* ks, const int* st, hipStream_t s) {
    k_cg_p<<<grid_for(n), EB_BLOCK, 0, s>>>(n, p, z, ks, st);
}
void ks_bi_p(long n, double* p, const double* r, const double* v, const double* ks,
             const int* st, hipStream_t s) {
    k_bi_p<<<grid_for(n), EB_BLOCK, 0, s>>>(n, p, r, v, ks, st);
}
void ks_bi_xs(long n, double* x, const double* ph, const double* ks, const int* st,
              hipStream_t s) {
    k_bi_xs<double><<<red_blocks(n), EB_BLOCK, 0, s>>>(n, x, ph, ks, st);
}
void ks_bi_xs(long n, double* x, const float* ph, const double* ks, const int* st,
              hipStream_t s) {
    k_bi_xs<float><<<red_blocks(n), EB_BLOCK, 0, s>>>(n, x, ph, ks, st);
}
