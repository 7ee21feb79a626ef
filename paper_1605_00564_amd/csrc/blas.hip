// Vector algebra of the Krylov solvers: multi-dot products and Gram-Schmidt
// updates with FP64 accumulation, norms, precision conversions.
//
// A vector set holds n right-hand sides of ne elements each; an element is
// a float4 (two complex, FP32 storage) or a double2 (one complex, FP64).
// Sums are reduced deterministically: each workgroup writes one partial per
// (rhs, value) and a second kernel adds the partials in a fixed order.
#include "blas.h"

namespace dfl {

// conj(a) * b accumulated into (re, im), in double
__device__ inline void edot(const float4 &a, const float4 &b, double &re, double &im) {
    re += (double)a.x * b.x + (double)a.y * b.y + (double)a.z * b.z + (double)a.w * b.w;
    im += (double)a.x * b.y - (double)a.y * b.x + (double)a.z * b.w - (double)a.w * b.z;
}
__device__ inline void edot(const double2 &a, const double2 &b, double &re, double &im) {
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
}
__device__ inline double enorm2(const float4 &a) {
    return (double)a.x * a.x + (double)a.y * a.y + (double)a.z * a.z + (double)a.w * a.w;
}
__device__ inline double enorm2(const double2 &a) { return a.x * a.x + a.y * a.y; }
// a - c b for complex c
__device__ inline float4 esub(const float4 &a, double cr, double ci, const float4 &b) {
    const float r = (float)cr, i = (float)ci;
    return make_float4(a.x - (r * b.x - i * b.y), a.y - (r * b.y + i * b.x), a.z - (r * b.z - i * b.w),
                       a.w - (r * b.w + i * b.z));
}
__device__ inline double2 esub(const double2 &a, double cr, double ci, const double2 &b) {
    return make_double2(a.x - (cr * b.x - ci * b.y), a.y - (cr * b.y + ci * b.x));
}
__device__ inline float4 escale(const float4 &a, double s) {
    const float f = (float)s;
    return make_float4(a.x * f, a.y * f, a.z * f, a.w * f);
}
__device__ inline double2 escale(const double2 &a, double s) { return make_double2(a.x * s, a.y * s); }

template <int NV>
__device__ inline void block_partials(double v[NV], double *part, int nblk) {
    __shared__ double sh[NV][BLAS_BS / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        if (lane == 0) sh[q][w] = t;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0;
#pragma unroll
        for (int k = 0; k < BLAS_BS / 64; ++k) t += sh[threadIdx.x][k];
        part[((size_t)blockIdx.y * NV + threadIdx.x) * nblk + blockIdx.x] = t;
    }
}

// part[rhs][2j + (0 re | 1 im)][blk] = partial of (W_j, W_k), j < k
template <class E, int KMAX>
__global__ void __launch_bounds__(BLAS_BS) k_multidot(const E *__restrict__ W, long ne, int n, int k,
                                                      double *__restrict__ part) {
    const int r = blockIdx.y;
    const E *wk = W + ((size_t)k * n + r) * ne;
    double acc[2 * KMAX];
#pragma unroll
    for (int q = 0; q < 2 * KMAX; ++q) acc[q] = 0;
    for (long i = (long)blockIdx.x * BLAS_BS + threadIdx.x; i < ne; i += (long)gridDim.x * BLAS_BS) {
        const E b = wk[i];
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < k) edot(W[((size_t)j * n + r) * ne + i], b, acc[2 * j], acc[2 * j + 1]);
    }
    block_partials<2 * KMAX>(acc, part, gridDim.x);
}

// W_k -= sum_j beta_j W_j ; partials of ||W_k||^2 and (W_k, rho)
template <class E, int KMAX>
__global__ void __launch_bounds__(BLAS_BS) k_gs_sub(E *__restrict__ W, const E *__restrict__ rho, long ne, int n,
                                                    int k, const double *__restrict__ beta, int bstride,
                                                    double *__restrict__ part) {
    const int r = blockIdx.y;
    E *wk = W + ((size_t)k * n + r) * ne;
    const E *rr = rho + (size_t)r * ne;
    double bre[KMAX], bim[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        bre[j] = j < k ? beta[(size_t)r * bstride + 2 * j] : 0.0;
        bim[j] = j < k ? beta[(size_t)r * bstride + 2 * j + 1] : 0.0;
    }
    double acc[3] = {0, 0, 0};
    for (long i = (long)blockIdx.x * BLAS_BS + threadIdx.x; i < ne; i += (long)gridDim.x * BLAS_BS) {
        E w = wk[i];
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < k) w = esub(w, bre[j], bim[j], W[((size_t)j * n + r) * ne + i]);
        wk[i] = w;
        acc[0] += enorm2(w);
        edot(w, rr[i], acc[1], acc[2]);
    }
    block_partials<3>(acc, part, gridDim.x);
}

// W_k *= inv_gamma ; rho -= c W_k ; partial ||rho||^2.  coef[rhs] = (inv_gamma, c_re, c_im)
template <class E>
__global__ void __launch_bounds__(BLAS_BS) k_scal_update(E *__restrict__ wk_all, E *__restrict__ rho, long ne,
                                                         const double *__restrict__ coef, double *__restrict__ part) {
    const int r = blockIdx.y;
    E *wk = wk_all + (size_t)r * ne;
    E *rr = rho + (size_t)r * ne;
    const double ig = coef[3 * r], cr = coef[3 * r + 1], ci = coef[3 * r + 2];
    double acc[1] = {0};
    for (long i = (long)blockIdx.x * BLAS_BS + threadIdx.x; i < ne; i += (long)gridDim.x * BLAS_BS) {
        const E w = escale(wk[i], ig);
        wk[i] = w;
        const E q = esub(rr[i], cr, ci, w);
        rr[i] = q;
        acc[0] += enorm2(q);
    }
    block_partials<1>(acc, part, gridDim.x);
}

// partial ||v||^2
template <class E>
__global__ void __launch_bounds__(BLAS_BS) k_norm2(const E *__restrict__ v, long ne, double *__restrict__ part) {
    const E *vr = v + (size_t)blockIdx.y * ne;
    double acc[1] = {0};
    for (long i = (long)blockIdx.x * BLAS_BS + threadIdx.x; i < ne; i += (long)gridDim.x * BLAS_BS)
        acc[0] += enorm2(vr[i]);
    block_partials<1>(acc, part, gridDim.x);
}

// r = b - t (FP64), partial ||r||^2
__global__ void __launch_bounds__(BLAS_BS) k_resid(const double2 *__restrict__ b, const double2 *__restrict__ t,
                                                   double2 *__restrict__ r, long ne, double *__restrict__ part) {
    const size_t off = (size_t)blockIdx.y * ne;
    double acc[1] = {0};
    for (long i = (long)blockIdx.x * BLAS_BS + threadIdx.x; i < ne; i += (long)gridDim.x * BLAS_BS) {
        const double2 bb = b[off + i], tt = t[off + i];
        const double2 q = make_double2(bb.x - tt.x, bb.y - tt.y);
        r[off + i] = q;
        acc[0] += q.x * q.x + q.y * q.y;
    }
    block_partials<1>(acc, part, gridDim.x);
}

// out[rhs][v] = sum over blocks of part[rhs][v][blk]: one wave per value,
// lane j sums partials j, j+64, ... and a fixed butterfly combines the
// lanes, so the order of additions (and the result) never changes
__global__ void __launch_bounds__(256) k_reduce(const double *__restrict__ part, int nv, int nblk, int n,
                                                double *__restrict__ out) {
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= n * nv) return;
    const double *p = part + (size_t)t * nblk;
    double s = 0;
    for (int b = lane; b < nblk; b += 64) s += p[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) out[t] = s;
}

// FP64 internal spinor (12 chunks of one complex) <-> FP32 internal spinor
// (6 chunks of two complex): chunk c of FP32 = complex 2c, 2c+1 of FP64.
__global__ void k_d2f(const double2 *__restrict__ x, float4 *__restrict__ y, long V) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * V) return;
    const size_t r = blockIdx.y;
    const long c = t / V, s = t - c * V;
    const double2 a = x[r * 12 * V + (2 * c) * V + s], b = x[r * 12 * V + (2 * c + 1) * V + s];
    y[r * 6 * V + t] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
}

// x (FP64) += sum_j alpha_j z_j (FP32 or FP64 Krylov vectors)
template <int KMAX>
__global__ void k_accum_f(double2 *__restrict__ x, const float4 *__restrict__ Z, long V, int n, int k,
                          const double *__restrict__ alpha, int astride) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * V) return;
    const int r = blockIdx.y;
    const long c = t / V, s = t - c * V;
    double2 *xa = x + (size_t)r * 12 * V + (2 * c) * V + s;
    double2 *xb = x + (size_t)r * 12 * V + (2 * c + 1) * V + s;
    double2 a = *xa, b = *xb;
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
        if (j < k) {
            const float4 z = Z[((size_t)j * n + r) * 6 * V + t];
            const double ar = alpha[(size_t)r * astride + 2 * j], ai = alpha[(size_t)r * astride + 2 * j + 1];
            a.x += ar * z.x - ai * z.y;
            a.y += ar * z.y + ai * z.x;
            b.x += ar * z.z - ai * z.w;
            b.y += ar * z.w + ai * z.z;
        }
    *xa = a;
    *xb = b;
}

template <int KMAX>
__global__ void k_accum_d(double2 *__restrict__ x, const double2 *__restrict__ Z, long ne, int n, int k,
                          const double *__restrict__ alpha, int astride) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne) return;
    const int r = blockIdx.y;
    double2 a = x[(size_t)r * ne + t];
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
        if (j < k) {
            const double2 z = Z[((size_t)j * n + r) * ne + t];
            const double ar = alpha[(size_t)r * astride + 2 * j], ai = alpha[(size_t)r * astride + 2 * j + 1];
            a.x += ar * z.x - ai * z.y;
            a.y += ar * z.y + ai * z.x;
        }
    x[(size_t)r * ne + t] = a;
}

// y = a * x + y (complex a per rhs, given as (re, im) pairs), FP64 or FP32 elements
template <class E>
__global__ void k_caxpy(E *__restrict__ y, const E *__restrict__ x, long ne, const double *__restrict__ a, double sgn) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne) return;
    const int r = blockIdx.y;
    const double ar = -sgn * a[2 * r], ai = -sgn * a[2 * r + 1];
    y[(size_t)r * ne + t] = esub(y[(size_t)r * ne + t], ar, ai, x[(size_t)r * ne + t]);
}

template <class E>
__global__ void k_zero(E *__restrict__ y, long ne) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne) return;
    E z{};
    y[(size_t)blockIdx.y * ne + t] = z;
}

// per-rhs scalar bookkeeping of one GCR step (one thread per rhs):
// beta_jk from the multi-dot, gamma_k = ||w_k||, c_k = (w_k, rho)/gamma_k
__global__ void k_gcr_scalars(const double *__restrict__ beta, int bstride, const double *__restrict__ gs, int n,
                              int k, double *__restrict__ R, double *__restrict__ cvec, double *__restrict__ coef) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double *Rr = R + (size_t)r * NKV_MAX * NKV_MAX * 2;
    for (int j = 0; j < k; ++j) {
        Rr[(j * NKV_MAX + k) * 2] = beta[(size_t)r * bstride + 2 * j];
        Rr[(j * NKV_MAX + k) * 2 + 1] = beta[(size_t)r * bstride + 2 * j + 1];
    }
    const double nn = gs[3 * r], dr = gs[3 * r + 1], di = gs[3 * r + 2];
    const double g = sqrt(nn);
    double ig = 0, cr = 0, ci = 0, gg = 1;
    if (g > 0 && isfinite(g)) {
        ig = 1.0 / g;
        cr = dr * ig;
        ci = di * ig;
        gg = g;
    }
    Rr[(k * NKV_MAX + k) * 2] = gg;
    Rr[(k * NKV_MAX + k) * 2 + 1] = 0;
    cvec[((size_t)r * NKV_MAX + k) * 2] = cr;
    cvec[((size_t)r * NKV_MAX + k) * 2 + 1] = ci;
    coef[3 * r] = ig;
    coef[3 * r + 1] = cr;
    coef[3 * r + 2] = ci;
}

// back substitution R alpha = c (upper triangular, complex), one thread per rhs
__global__ void k_trisolve(const double *__restrict__ R, const double *__restrict__ cvec, int n, int k,
                           double *__restrict__ alpha) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double *Rr = R + (size_t)r * NKV_MAX * NKV_MAX * 2;
    double *a = alpha + (size_t)r * NKV_MAX * 2;
    for (int i = k - 1; i >= 0; --i) {
        double sr = cvec[((size_t)r * NKV_MAX + i) * 2], si = cvec[((size_t)r * NKV_MAX + i) * 2 + 1];
        for (int j = i + 1; j < k; ++j) {
            const double rr = Rr[(i * NKV_MAX + j) * 2], ri = Rr[(i * NKV_MAX + j) * 2 + 1];
            sr -= rr * a[2 * j] - ri * a[2 * j + 1];
            si -= rr * a[2 * j + 1] + ri * a[2 * j];
        }
        const double dr = Rr[(i * NKV_MAX + i) * 2], di = Rr[(i * NKV_MAX + i) * 2 + 1];
        const double den = dr * dr + di * di;
        a[2 * i] = (sr * dr + si * di) / den;
        a[2 * i + 1] = (si * dr - sr * di) / den;
    }
}

// ---------------------------------------------------------------------------
// host wrappers
// ---------------------------------------------------------------------------
static int grid_blocks(long ne) {
    long b = (ne + BLAS_BS - 1) / BLAS_BS;
    return (int)(b < BLAS_NBLK ? (b < 1 ? 1 : b) : BLAS_NBLK);
}

int blas_reduce(const double *part, int nv, int nblk, int n, double *out, hipStream_t s) {
    const int tot = n * nv;
    k_reduce<<<(tot + 3) / 4, 256, 0, s>>>(part, nv, nblk, n, out);
    DFL_HIP(hipGetLastError());
    return 0;
}

template <class E>
int blas_multidot(const E *W, long ne, int n, int k, double *part, double *out, hipStream_t s) {
    if (k <= 0) return 0;
    const int nb = grid_blocks(ne);
    dim3 g(nb, n);
    ProfScope ps(PROF_BLAS, s);
    if (k <= 4) k_multidot<E, 4><<<g, BLAS_BS, 0, s>>>(W, ne, n, k, part);
    else if (k <= 8) k_multidot<E, 8><<<g, BLAS_BS, 0, s>>>(W, ne, n, k, part);
    else if (k <= 16) k_multidot<E, 16><<<g, BLAS_BS, 0, s>>>(W, ne, n, k, part);
    else if (k <= 32) k_multidot<E, 32><<<g, BLAS_BS, 0, s>>>(W, ne, n, k, part);
    else return set_error(QCD_EINVAL, "at most 32 Krylov vectors per cycle");
    const int nv = 2 * (k <= 4 ? 4 : k <= 8 ? 8 : k <= 16 ? 16 : 32);
    DFL_TRY(blas_reduce(part, nv, nb, n, out, s));
    return nv;
}

template <class E>
int blas_gs_sub(E *W, const E *rho, long ne, int n, int k, const double *beta, int bstride, double *part,
                double *out, hipStream_t s) {
    const int nb = grid_blocks(ne);
    dim3 g(nb, n);
    ProfScope ps(PROF_BLAS, s);
    if (k <= 4) k_gs_sub<E, 4><<<g, BLAS_BS, 0, s>>>(W, rho, ne, n, k, beta, bstride, part);
    else if (k <= 8) k_gs_sub<E, 8><<<g, BLAS_BS, 0, s>>>(W, rho, ne, n, k, beta, bstride, part);
    else if (k <= 16) k_gs_sub<E, 16><<<g, BLAS_BS, 0, s>>>(W, rho, ne, n, k, beta, bstride, part);
    else if (k <= 32) k_gs_sub<E, 32><<<g, BLAS_BS, 0, s>>>(W, rho, ne, n, k, beta, bstride, part);
    else return set_error(QCD_EINVAL, "at most 32 Krylov vectors per cycle");
    return blas_reduce(part, 3, nb, n, out, s);
}

template <class E>
int blas_scal_update(E *wk, E *rho, long ne, int n, const double *coef, double *part, double *out, hipStream_t s) {
    const int nb = grid_blocks(ne);
    ProfScope ps(PROF_BLAS, s);
    k_scal_update<E><<<dim3(nb, n), BLAS_BS, 0, s>>>(wk, rho, ne, coef, part);
    return blas_reduce(part, 1, nb, n, out, s);
}

template <class E>
int blas_norm2(const E *v, long ne, int n, double *part, double *out, hipStream_t s) {
    const int nb = grid_blocks(ne);
    ProfScope ps(PROF_BLAS, s);
    k_norm2<E><<<dim3(nb, n), BLAS_BS, 0, s>>>(v, ne, part);
    return blas_reduce(part, 1, nb, n, out, s);
}

int blas_resid(const double2 *b, const double2 *t, double2 *r, long ne, int n, double *part, double *out,
               hipStream_t s) {
    const int nb = grid_blocks(ne);
    ProfScope ps(PROF_BLAS, s);
    k_resid<<<dim3(nb, n), BLAS_BS, 0, s>>>(b, t, r, ne, part);
    return blas_reduce(part, 1, nb, n, out, s);
}

int blas_d2f(const double2 *x, float4 *y, long V, int n, hipStream_t s) {
    ProfScope ps(PROF_BLAS, s);
    k_d2f<<<dim3(nblocks(6 * V, 256), n), 256, 0, s>>>(x, y, V);
    DFL_HIP(hipGetLastError());
    return 0;
}

int blas_accum_f(double2 *x, const float4 *Z, long V, int n, int k, const double *alpha, int astride,
                 hipStream_t s) {
    if (k <= 0) return 0;
    ProfScope ps(PROF_BLAS, s);
    dim3 g(nblocks(6 * V, 256), n);
    if (k <= 4) k_accum_f<4><<<g, 256, 0, s>>>(x, Z, V, n, k, alpha, astride);
    else if (k <= 8) k_accum_f<8><<<g, 256, 0, s>>>(x, Z, V, n, k, alpha, astride);
    else if (k <= 16) k_accum_f<16><<<g, 256, 0, s>>>(x, Z, V, n, k, alpha, astride);
    else k_accum_f<32><<<g, 256, 0, s>>>(x, Z, V, n, k, alpha, astride);
    DFL_HIP(hipGetLastError());
    return 0;
}

int blas_accum_d(double2 *x, const double2 *Z, long ne, int n, int k, const double *alpha, int astride,
                 hipStream_t s) {
    if (k <= 0) return 0;
    ProfScope ps(PROF_BLAS, s);
    dim3 g(nblocks(ne, 256), n);
    if (k <= 4) k_accum_d<4><<<g, 256, 0, s>>>(x, Z, ne, n, k, alpha, astride);
    else if (k <= 8) k_accum_d<8><<<g, 256, 0, s>>>(x, Z, ne, n, k, alpha, astride);
    else if (k <= 16) k_accum_d<16><<<g, 256, 0, s>>>(x, Z, ne, n, k, alpha, astride);
    else k_accum_d<32><<<g, 256, 0, s>>>(x, Z, ne, n, k, alpha, astride);
    DFL_HIP(hipGetLastError());
    return 0;
}

template <class E>
int blas_caxpy(E *y, const E *x, long ne, int n, const double *a, double sgn, hipStream_t s) {
    ProfScope ps(PROF_BLAS, s);
    k_caxpy<E><<<dim3(nblocks(ne, 256), n), 256, 0, s>>>(y, x, ne, a, sgn);
    DFL_HIP(hipGetLastError());
    return 0;
}

template <class E>
int blas_zero(E *y, long ne, int n, hipStream_t s) {
    k_zero<E><<<dim3(nblocks(ne, 256), n), 256, 0, s>>>(y, ne);
    DFL_HIP(hipGetLastError());
    return 0;
}

int gcr_scalars(const double *beta, int bstride, const double *gs, int n, int k, double *R, double *cvec,
                double *coef, hipStream_t s) {
    k_gcr_scalars<<<(n + 63) / 64, 64, 0, s>>>(beta, bstride, gs, n, k, R, cvec, coef);
    DFL_HIP(hipGetLastError());
    return 0;
}

int gcr_trisolve(const double *R, const double *cvec, int n, int k, double *alpha, hipStream_t s) {
    k_trisolve<<<(n + 63) / 64, 64, 0, s>>>(R, cvec, n, k, alpha);
    DFL_HIP(hipGetLastError());
    return 0;
}

int scalar_buffers_at(void *p, int n, Scal &sc) {
    const size_t npart = (size_t)n * 2 * NKV_MAX * BLAS_NBLK;
    const size_t nred = (size_t)n * 2 * NKV_MAX;
    const size_t nR = (size_t)n * NKV_MAX * NKV_MAX * 2;
    const size_t nc = (size_t)n * NKV_MAX * 2;
    double *d = static_cast<double *>(p);
    sc.part = d;
    d += npart;
    sc.red = d;
    d += nred;
    sc.red2 = d;
    d += nred;
    sc.R = d;
    d += nR;
    sc.cvec = d;
    d += nc;
    sc.coef = d;
    d += 3 * (size_t)n;
    sc.alpha = d;
    d += nc;
    sc.bn2 = d;
    return 0;
}


size_t scalar_bytes(int n) {
    const size_t npart = (size_t)n * 2 * NKV_MAX * BLAS_NBLK;
    const size_t nred = (size_t)n * 2 * NKV_MAX;
    const size_t nR = (size_t)n * NKV_MAX * NKV_MAX * 2;
    const size_t nc = (size_t)n * NKV_MAX * 2;
    return (npart + 2 * nred + nR + nc + 3 * (size_t)n + nc + (size_t)n) * sizeof(double);
}

#define DFL_INST(E)                                                                                      \
    template int blas_multidot<E>(const E *, long, int, int, double *, double *, hipStream_t);          \
    template int blas_gs_sub<E>(E *, const E *, long, int, int, const double *, int, double *, double *, \
                                hipStream_t);                                                            \
    template int blas_scal_update<E>(E *, E *, long, int, const double *, double *, double *, hipStream_t); \
    template int blas_norm2<E>(const E *, long, int, double *, double *, hipStream_t);                 \
    template int blas_caxpy<E>(E *, const E *, long, int, const double *, double, hipStream_t);        \
    template int blas_zero<E>(E *, long, int, hipStream_t);
DFL_INST(float4)
DFL_INST(double2)
#undef DFL_INST

}  // namespace dfl
