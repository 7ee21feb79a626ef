// Krylov vector algebra (see blas.hip).
#pragma once
#include "internal.h"

namespace dfl {

constexpr int BLAS_BS = 256;    // threads per workgroup of the reduction kernels
constexpr int BLAS_NBLK = 512;  // maximum workgroups per right-hand side (partials per value)
constexpr int NKV_MAX = 32;     // Krylov vectors per cycle
// little-solve iterations of the low-mode correction in solves without
// host synchronisation (one cycle of the little GCR)
constexpr int LOW_MODE_FIXED_ITERS = 12;

// Reduced sums land in `out` ([n][nv] doubles); `part` needs n * nv * BLAS_NBLK doubles.
int blas_reduce(const double *part, int nv, int nblk, int n, double *out, hipStream_t s);
// (W_j, W_k) for j < k; returns the value stride nv of out (2 per j)
template <class E> int blas_multidot(const E *W, long ne, int n, int k, double *part, double *out, hipStream_t s);
// W_k -= sum_j beta_j W_j ; out[rhs][0..2] = ||W_k||^2, (W_k, rho)
template <class E> int blas_gs_sub(E *W, const E *rho, long ne, int n, int k, const double *beta, int bstride,
                                   double *part, double *out, hipStream_t s);
// w *= coef0 ; rho -= (coef1 + i coef2) w ; out[rhs] = ||rho||^2
template <class E> int blas_scal_update(E *wk, E *rho, long ne, int n, const double *coef, double *part,
                                        double *out, hipStream_t s);
template <class E> int blas_norm2(const E *v, long ne, int n, double *part, double *out, hipStream_t s);
// y += sgn * a_rhs * x
template <class E> int blas_caxpy(E *y, const E *x, long ne, int n, const double *a, double sgn, hipStream_t s);
template <class E> int blas_zero(E *y, long ne, int n, hipStream_t s);
int blas_resid(const double2 *b, const double2 *t, double2 *r, long ne, int n, double *part, double *out,
               hipStream_t s);
int blas_d2f(const double2 *x, float4 *y, long V, int n, hipStream_t s);
int blas_accum_f(double2 *x, const float4 *Z, long V, int n, int k, const double *alpha, int astride, hipStream_t s);
int blas_accum_d(double2 *x, const double2 *Z, long ne, int n, int k, const double *alpha, int astride,
                 hipStream_t s);

// GCR step bookkeeping on the device (one thread per rhs), see blas.hip
int gcr_scalars(const double *beta, int bstride, const double *gs, int n, int k, double *R, double *cvec,
                double *coef, hipStream_t s);
int gcr_trisolve(const double *R, const double *cvec, int n, int k, double *alpha, hipStream_t s);

// per-solve scalar work space: partial sums, reductions, R, c, alpha
struct Scal {
    double *part, *red, *red2, *R, *cvec, *coef, *alpha;
    double *bn2;   // ||b||^2 per rhs, kept on the device by solves that do not synchronise
};
size_t scalar_bytes(int n);
int scalar_buffers_at(void *p, int n, Scal &sc);

}  // namespace dfl
