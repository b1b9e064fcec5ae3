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

__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

__global__ void k_scal(int op, double* __restrict__ ks, int* __restrict__ st,
                       int* __restrict__ itc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int s = *st;
    // the first scalar op of each iteration advances the count while the solve runs
    if (s == 0 && (op == KS_CG_ALPHA || op == KS_BI_BETA)) *itc += 1;
    int it = *itc;
    switch (op) {
    case KS_INIT: {  // tol = rtol * max(bn, scale); converged already if rn <= tol
        double bn = ks[KS_BN] > ks[KS_SCALE] ? ks[KS_BN] : ks[KS_SCALE];
        ks[KS_TOL] = ks[KS_RTOL] * bn;
        st[1] = 0;
        *itc = 0;
        if (!finite_d(ks[KS_RN])) *st = 3;
        else if (bn == 0.0 || ks[KS_RN] <= ks[KS_TOL]) *st = 2;
        else *st = 0;
        ks[KS_RHO_OLD] = 1.0;
        ks[KS_AL] = 1.0;
        ks[KS_OM] = 1.0;
        break;
    }
    case KS_CG_ALPHA:
        if (s == 0) ks[KS_AL] = ks[KS_RZ] / ks[KS_PQ];
        break;
    case KS_CHECK_R:  // after the x, r update (CG)
        if (s == 0) {
            if (!finite_d(ks[KS_RN])) *st = 3;
            else if (ks[KS_RN] <= ks[KS_TOL]) {
                *st = 2;
                st[1] = it;
            }
        }
        break;
    case KS_CG_BETA:
        if (s == 0) {
            ks[KS_BE] = ks[KS_RZN] / ks[KS_RZ];
            ks[KS_RZ] = ks[KS_RZN];
        }
        break;
    case KS_BI_BETA:
        if (s == 0) ks[KS_BE] = (ks[KS_RR] / ks[KS_RHO_OLD]) * (ks[KS_AL] / ks[KS_OM]);
        break;
    case KS_BI_ALPHA:
        if (s == 0) ks[KS_AL] = ks[KS_RR] / ks[KS_RV];
        break;
    case KS_BI_CHECK_S:  // the count is in half iterations (= preconditioner applications)
        if (s == 0) {
            if (!finite_d(ks[KS_SN])) *st = 3;
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
            if (!finite_d(ks[KS_RN])) *st = 3;
            else if (ks[KS_RN] <= ks[KS_TOL]) {
                *st = 2;
                st[1] = 2 * it;
            }
        }
        break;
    case KS_BI_FINISH_S:
        if (s == 1) *st = 2;
        break;
    case KS_BI_OMEGA:
        if (s == 0) ks[KS_OM] = ks[KS_TS] / ks[KS_TT];
        break;
    default:
        break;
    }
}

// x += a p ; r -= a q   (CG)
__global__ void k_cg_xr(long n, double* __restrict__ x, double* __restrict__ r,
                        const double* __restrict__ p, const double* __restrict__ q,
                        const double* __restrict__ ks, const int* __restrict__ st) {
    if (*st != 0) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    double a = ks[KS_AL];
    x[t] += a * p[t];
    r[t] -= a * q[t];
}
// p = z + beta p   (CG)
__global__ void k_cg_p(long n, double* __restrict__ p, const double* __restrict__ z,
                       const double* __restrict__ ks, const int* __restrict__ st) {
    if (*st != 0) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) p[t] = z[t] + ks[KS_BE] * p[t];
}
// p = r + beta (p - omega v)   (BiCGSTAB)
__global__ void k_bi_p(long n, double* __restrict__ p, const double* __restrict__ r,
                       const double* __restrict__ v, const double* __restrict__ ks,
                       const int* __restrict__ st) {
    if (*st != 0) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) p[t] = r[t] + ks[KS_BE] * (p[t] - ks[KS_OM] * v[t]);
}
// s = r - alpha v
__global__ void k_bi_s(long n, double* __restrict__ sv, const double* __restrict__ r,
                       const double* __restrict__ v, const double* __restrict__ ks,
                       const int* __restrict__ st) {
    if (*st != 0) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) sv[t] = r[t] - ks[KS_AL] * v[t];
}
// converged at the half step: x += alpha ph
__global__ void k_bi_xs(long n, double* __restrict__ x, const double* __restrict__ ph,
                        const double* __restrict__ ks, const int* __restrict__ st) {
    if (*st != 1) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) x[t] += ks[KS_AL] * ph[t];
}
// x += alpha ph + omega sh ; r = s - omega t
__global__ void k_bi_xr(long n, double* __restrict__ x, double* __restrict__ r,
                        const double* __restrict__ ph, const double* __restrict__ sh,
                        const double* __restrict__ sv, const double* __restrict__ tv,
                        const double* __restrict__ ks, const int* __restrict__ st) {
    if (*st != 0) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    double al = ks[KS_AL], om = ks[KS_OM];
    x[t] += al * ph[t] + om * sh[t];
    r[t] = sv[t] - om * tv[t];
}

__global__ void k_set(double* __restrict__ ks, int idx, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ks[idx] = v;
}

}  // namespace

void ks_op(int op, double* ks, int* st, int* itc, hipStream_t s) {
    k_scal<<<1, 64, 0, s>>>(op, ks, st, itc);
}
void ks_set(double* ks, int idx, double v, hipStream_t s) { k_set<<<1, 64, 0, s>>>(ks, idx, v); }
void ks_cg_xr(long n, double* x, double* r, const double* p, const double* q, const double* ks,
              const int* st, hipStream_t s) {
    k_cg_xr<<<grid_for(n), EB_BLOCK, 0, s>>>(n, x, r, p, q, ks, st);
}
void ks_cg_p(long n, double* p, const double* z, const double* ks, const int* st, hipStream_t s) {
    k_cg_p<<<grid_for(n), EB_BLOCK, 0, s>>>(n, p, z, ks, st);
}
void ks_bi_p(long n, double* p, const double* r, const double* v, const double* ks,
             const int* st, hipStream_t s) {
    k_bi_p<<<grid_for(n), EB_BLOCK, 0, s>>>(n, p, r, v, ks, st);
}
void ks_bi_s(long n, double* sv, const double* r, const double* v, const double* ks,
             const int* st, hipStream_t s) {
    k_bi_s<<<grid_for(n), EB_BLOCK, 0, s>>>(n, sv, r, v, ks, st);
}
void ks_bi_xs(long n, double* x, const double* ph, const double* ks, const int* st,
              hipStream_t s) {
    k_bi_xs<<<grid_for(n), EB_BLOCK, 0, s>>>(n, x, ph, ks, st);
}
void ks_bi_xr(long n, double* x, double* r, const double* ph, const double* sh, const double* sv,
              const double* t, const double* ks, const int* st, hipStream_t s) {
    k_bi_xr<<<grid_for(n), EB_BLOCK, 0, s>>>(n, x, r, ph, sh, sv, t, ks, st);
}
