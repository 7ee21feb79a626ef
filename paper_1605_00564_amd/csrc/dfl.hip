// Block-local deflation (section 2.2): subspace from Ns global fields
// restricted to the Schwarz blocks and orthonormalised per block, the little
// Dirac operator A_kl = (phi_k, M phi_l) (eq. little), restriction Phi^+ v,
// prolongation Phi c, and the little solve A^{-1} by GCR on the block
// even-odd Schur complement.
#include <cmath>

#include "blas.h"
#include "dflint.h"

namespace dfl {

qcd_field dfl_field(qcd_dfl d) { return d->f; }

// ---------------------------------------------------------------------------
// random fields: SplitMix64 counter-based generator with Box-Muller
// (Steele, Lea, Flood 2014).  Field l, lexicographic site i, component sc is
// complex number j = (l V + i) 12 + sc; its real and imaginary parts are the
// cosine and sine branches of Box-Muller on outputs 2j and 2j+1.
// ---------------------------------------------------------------------------

__global__ void k_random_fields(float4 *__restrict__ v, unsigned long long key, const int *__restrict__ lex_of,
                                long V) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= V) return;
    const int l = blockIdx.y;
    const long i = lex_of[idx];
    float c[24];
    for (int sc = 0; sc < 12; ++sc) {
        const unsigned long long j = ((unsigned long long)l * V + i) * 12 + sc;
        const double u1 = 1.0 - (double)(sm64(key, 2 * j) >> 11) * 0x1.0p-53;
        const double u2 = (double)(sm64(key, 2 * j + 1) >> 11) * 0x1.0p-53;
        const double r = sqrt(-2.0 * log(u1));
        const double a = 2.0 * M_PI * u2;
        c[2 * sc] = (float)(r * cos(a));
        c[2 * sc + 1] = (float)(r * sin(a));
    }
    for (int ch = 0; ch < 6; ++ch)
        v[((size_t)l * 6 + ch) * V + idx] = make_float4(c[4 * ch], c[4 * ch + 1], c[4 * ch + 2], c[4 * ch + 3]);
}

// v_r *= 1/sqrt(nrm2_r)
__global__ void k_normalise(float4 *__restrict__ v, long ne, const double *__restrict__ nrm2) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne) return;
    const double n2 = nrm2[blockIdx.y];
    const float s = n2 > 0 ? (float)(1.0 / sqrt(n2)) : 0.f;
    float4 a = v[(size_t)blockIdx.y * ne + t];
    v[(size_t)blockIdx.y * ne + t] = make_float4(a.x * s, a.y * s, a.z * s, a.w * s);
}

// A deflation block is the union of r Schwarz blocks (r = 1 when the two
// sizes are tied).  Element q of one of its vectors (12 r Vbh float4, the
// member Schwarz blocks one after the other, each in the (chunk, parity, j)
// order) -> FP32 chunk c and internal site index; boff[B r + m] is the
// internal offset (memory rank x Vbh) of member m of deflation block B.
__device__ inline long dfl_site(const int *__restrict__ boff, int B, int r, int Vbh, long Vh, long q, int &c) {
    const long per_b = 12L * Vbh;
    const int m = (int)(q / per_b);
    const long qq = q - (long)m * per_b;
    c = (int)(qq / (2 * Vbh));
    const int p = (int)((qq / Vbh) % 2), j = (int)(qq % Vbh);
    return p * Vh + boff[(long)B * r + m] + j;
}

// global fields [Ns][6][V] -> block storage phi[B][l][12 r Vbh]
__global__ void k_to_blocks(const float4 *__restrict__ v, float4 *__restrict__ phi, const int *__restrict__ boff,
                            long V, long Vh, int Vbh, int r, int Ns, int Nb) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long per = 12L * Vbh * r;
    if (t >= (long)Nb * Ns * per) return;
    const long q = t % per;
    const long bl = t / per;
    const int l = (int)(bl % Ns), B = (int)(bl / Ns);
    int c;
    const long site = dfl_site(boff, B, r, Vbh, Vh, q, c);
    phi[t] = v[((size_t)l * 6 + c) * V + site];
}

// phi_l of every block as one global FP32 field [6][V]
__global__ void k_phi_field(const float4 *__restrict__ phi, int l, float4 *__restrict__ out, const int *__restrict__ boff,
                            long V, long Vh, int Vbh, int r, int Ns, int Nb) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long per = 12L * Vbh * r;
    if (t >= (long)Nb * per) return;
    const int B = (int)(t / per);
    const long q = t % per;
    int c;
    const long site = dfl_site(boff, B, r, Vbh, Vh, q, c);
    out[(size_t)c * V + site] = phi[((size_t)B * Ns + l) * per + q];
}

// FP32 internal vectors [n][6][V] <-> FP64 internal vectors [n][12][V]
__global__ void k_widen(const float4 *__restrict__ in, double2 *__restrict__ out, long V) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * V) return;
    const long c = t / V, x = t - c * V;
    const float4 a = in[(size_t)blockIdx.y * 6 * V + t];
    double2 *o = out + (size_t)blockIdx.y * 12 * V;
    o[(size_t)(2 * c) * V + x] = make_double2(a.x, a.y);
    o[(size_t)(2 * c + 1) * V + x] = make_double2(a.z, a.w);
}

__global__ void k_narrow(const double2 *__restrict__ in, float4 *__restrict__ out, long V) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * V) return;
    const long c = t / V, x = t - c * V;
    const double2 *i = in + (size_t)blockIdx.y * 12 * V;
    const double2 a = i[(size_t)(2 * c) * V + x], b = i[(size_t)(2 * c + 1) * V + x];
    out[(size_t)blockIdx.y * 6 * V + t] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
}

template <int NV>
__device__ inline void wg_sum(double v[NV], double out[NV]) {
    __shared__ double sh[NV][16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        if (lane == 0) sh[q][w] = t;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = 0;
        for (int k = 0; k < nw; ++k) t += sh[q][k];
        out[q] = t;
    }
    __syncthreads();
}

// two passes of modified Gram-Schmidt over l inside each deflation block
// (one workgroup per block; per = float4 elements of one block vector)
__global__ void __launch_bounds__(256) k_block_mgs(float4 *__restrict__ phi, int Ns, long per, int *flag) {
    float4 *base = phi + (size_t)blockIdx.x * Ns * per;
    for (int l = 0; l < Ns; ++l) {
        float4 *pl = base + (size_t)l * per;
        double v[1], o[1];
        v[0] = 0;
        for (long i = threadIdx.x; i < per; i += blockDim.x) {
            const float4 a = pl[i];
            v[0] += (double)a.x * a.x + (double)a.y * a.y + (double)a.z * a.z + (double)a.w * a.w;
        }
        wg_sum<1>(v, o);
        const double n0 = sqrt(o[0]);
        for (int pass = 0; pass < 2; ++pass)
            for (int k = 0; k < l; ++k) {
                const float4 *pk = base + (size_t)k * per;
                double d[2] = {0, 0}, od[2];
                for (long i = threadIdx.x; i < per; i += blockDim.x) {
                    const float4 a = pk[i], b = pl[i];
                    d[0] += (double)a.x * b.x + (double)a.y * b.y + (double)a.z * b.z + (double)a.w * b.w;
                    d[1] += (double)a.x * b.y - (double)a.y * b.x + (double)a.z * b.w - (double)a.w * b.z;
                }
                wg_sum<2>(d, od);
                const float cr = (float)od[0], ci = (float)od[1];
                for (long i = threadIdx.x; i < per; i += blockDim.x) {
                    const float4 a = pk[i];
                    float4 b = pl[i];
                    b.x -= cr * a.x - ci * a.y;
                    b.y -= cr * a.y + ci * a.x;
                    b.z -= cr * a.z - ci * a.w;
                    b.w -= cr * a.w + ci * a.z;
                    pl[i] = b;
                }
                __syncthreads();
            }
        v[0] = 0;
        for (long i = threadIdx.x; i < per; i += blockDim.x) {
            const float4 a = pl[i];
            v[0] += (double)a.x * a.x + (double)a.y * a.y + (double)a.z * a.z + (double)a.w * a.w;
        }
        wg_sum<1>(v, o);
        const double nl = sqrt(o[0]);
        if (!(nl > 1e-10 * n0) || !(nl > 0)) {
            if (threadIdx.x == 0) atomicOr(flag, 2);
            return;
        }
        const float s = (float)(1.0 / nl);
        for (long i = threadIdx.x; i < per; i += blockDim.x) {
            float4 a = pl[i];
            pl[i] = make_float4(a.x * s, a.y * s, a.z * s, a.w * s);
        }
        __syncthreads();
    }
}

// Direction-resolved operator on a FP32 field (FP64 arithmetic):
// out[0] = clover + hops inside the deflation block, out[1 + 2 mu + dir] =
// -kappa times the single hop (mu, dir) when it leaves the deflation block
// (zero otherwise).  dbof: deflation block of each Schwarz block (by memory
// rank, the site's internal index within its parity / Vbh).
__global__ void __launch_bounds__(128) k_dirac_split(const float4 *__restrict__ in, double2 *__restrict__ out,
                                                     const void *__restrict__ U, const void *__restrict__ clo,
                                                     const int *__restrict__ nbr, const int *__restrict__ dbof,
                                                     long V, long Vh, int Vbh, double kappa) {
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= V) return;
    const long bx = dbof[(x >= Vh ? x - Vh : x) / Vbh];
    cx<double> acc[12], w[9], p[12], h[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {0, 0};
#define DFL_SPLIT(MU, FWD)                                                                   \
    {                                                                                        \
        const int e = nbr_at(nbr, 2 * MU + (FWD ? 0 : 1), V, x);                                 \
        const long y = nb_index(e);                                                          \
        const long by = dbof[(y >= Vh ? y - Vh : y) / Vbh];                                  \
        Link<LNK_F64>::load(U, V, MU, FWD ? x : y, w);                                       \
        Spin<float>::load(in, V, y, p);                                                      \
        const int d = 1 + 2 * MU + (FWD ? 0 : 1);                                            \
        if (by == bx) {                                                                      \
            hop<double, MU, FWD>(w, p, nb_sign<double>(e), acc);                             \
            _Pragma("unroll") for (int k = 0; k < 12; ++k) h[k] = {0, 0};                    \
        } else {                                                                             \
            _Pragma("unroll") for (int k = 0; k < 12; ++k) h[k] = {0, 0};                    \
            hop<double, MU, FWD>(w, p, nb_sign<double>(e), h);                               \
            _Pragma("unroll") for (int k = 0; k < 12; ++k) h[k] = (-kappa) * h[k];           \
        }                                                                                    \
        Spin<double>::store(out + (size_t)d * 12 * V, V, x, h);                              \
    }
    DFL_SPLIT(0, true) DFL_SPLIT(0, false) DFL_SPLIT(1, true) DFL_SPLIT(1, false)
    DFL_SPLIT(2, true) DFL_SPLIT(2, false) DFL_SPLIT(3, true) DFL_SPLIT(3, false)
#undef DFL_SPLIT
    Spin<float>::load(in, V, x, p);
    clover_apply<CLO_F64>(clo, V, x, p, h);
#pragma unroll
    for (int k = 0; k < 12; ++k) h[k] = rmac(h[k], -kappa, acc[k]);
    Spin<double>::store(out, V, x, h);
}

// FP32 restriction u = Phi^+ v as a real GEMM on the matrix cores
// (v_mfma_f32_16x16x4f32, FP32 accumulation).  Rows: 16 deflation fields;
// columns: 8 right-hand sides x (re, im); K: the real components of the
// block's sites.  With phi = a + ib and v = c + id, conj(phi) v =
// (ac + bd) + i(ad - bc): column 2r carries (c, d) and column 2r+1 (d, -c)
// against the row (a, b).  Lane L supplies A[L % 16][L / 16] and B[L / 16][L % 16]
// and receives D[4 (L / 16) + i][L % 16], i = 0..3.  Each lane loads one
// float4 (two complex) of phi and of v per four MFMAs; the K order is
// (element q + L / 16, component i), identical for both operands.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_restrict_mfma(const float4 *__restrict__ v, const float4 *__restrict__ phi,
                                                       const int *__restrict__ boff, double2 *__restrict__ u, long V,
                                                       long Vh, int Vbh, int rb, int Ns, int Nb, int n) {
    __shared__ float red[4][16][17];
    const int B = blockIdx.x, r0 = blockIdx.y * 8;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kk = lane >> 4;
    const int col = lane & 15, rr = col >> 1, which = col & 1;
    const long per = 12L * Vbh * rb;
    const bool rv = r0 + rr < n;
    const float4 *vr = v + (size_t)(rv ? r0 + rr : 0) * 6 * V;
    for (int l0 = 0; l0 < Ns; l0 += 16) {
        const bool lv = l0 + row < Ns;
        const float4 *pl = phi + ((size_t)B * Ns + (lv ? l0 + row : 0)) * per;
        f4v acc = {0.f, 0.f, 0.f, 0.f};
        // each wave takes every fourth group of four float4 elements
        for (long q0 = (long)wave * 4; q0 < per; q0 += 16) {
            const long q = q0 + kk;
            float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = make_float4(0.f, 0.f, 0.f, 0.f);
            if (q < per) {
                if (lv) a = pl[q];
                if (rv) {
                    int c;
                    const long site = dfl_site(boff, B, rb, Vbh, Vh, q, c);
                    b = vr[(long)c * V + site];
                }
            }
            // B operand per component: column (c, d) for which = 0, (d, -c) for which = 1
            const float b0 = which ? b.y : b.x, b1 = which ? -b.x : b.y;
            const float b2 = which ? b.w : b.z, b3 = which ? -b.z : b.w;
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b0, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b1, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b2, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b3, acc, 0, 0, 0);
        }
        for (int i = 0; i < 4; ++i) red[wave][4 * kk + i][col] = acc[i];
        __syncthreads();
        if (threadIdx.x < 128) {
            const int orow = threadIdx.x >> 3, orr = threadIdx.x & 7;
            if (l0 + orow < Ns && r0 + orr < n) {
                double re = 0, im = 0;
                for (int w = 0; w < 4; ++w) {
                    re += red[w][orow][2 * orr];
                    im += red[w][orow][2 * orr + 1];
                }
                u[((size_t)(r0 + orr) * Nb + B) * Ns + l0 + orow] = make_double2(re, im);
            }
        }
        __syncthreads();
    }
}

// FP64 restriction u = Phi^+ v for FP64 vectors on the FP64 matrix cores
// (little-operator assembly and the outer loop's low-mode corrections).
// Per block a complex GEMM (Ns x 24 Vb) (24 Vb x n): with phi = a + ib and
// v = c + id, conj(phi) v = (ac + bd) + i(ad - bc), accumulated as four real
// 16x16x4 products.  Rows: 16 fields; columns: 16 right-hand sides; lane L
// supplies phi[row L % 16][k L / 16] and v[k L / 16][rhs L % 16] (k: one
// float4 element = two complex, one MFMA quadruple each) and receives
// u[field L / 16 + 4 i][rhs L % 16], i = 0..3.  The four waves
// take every fourth group of four elements; their partial sums are added in
// a fixed order.
__global__ void __launch_bounds__(256) k_restrict_mfma64(const double2 *__restrict__ v, const float4 *__restrict__ phi,
                                                         const int *__restrict__ boff, double2 *__restrict__ u, long V,
                                                         long Vh, int Vbh, int rb, int Ns, int Nb, int n) {
    __shared__ double red[4][2][16][17];
    const int B = blockIdx.x, r0 = blockIdx.y * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kk = lane >> 4;
    const long per = 12L * Vbh * rb;
    const bool rv = r0 + row < n;
    const double2 *vr = v + (size_t)(rv ? r0 + row : 0) * 12 * V;
    for (int l0 = 0; l0 < Ns; l0 += 16) {
        const bool lv = l0 + row < Ns;
        const float4 *pl = phi + ((size_t)B * Ns + (lv ? l0 + row : 0)) * per;
        d4v ac = {0, 0, 0, 0}, bd = {0, 0, 0, 0}, ad = {0, 0, 0, 0}, bc = {0, 0, 0, 0};
        for (long q0 = (long)wave * 4; q0 < per; q0 += 16) {
            const long q = q0 + kk;
            float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
            double2 b0 = make_double2(0.0, 0.0), b1 = make_double2(0.0, 0.0);
            if (q < per) {
                if (lv) a = pl[q];
                if (rv) {
                    int c;
                    const long site = dfl_site(boff, B, rb, Vbh, Vh, q, c);
                    b0 = vr[(long)(2 * c) * V + site];
                    b1 = vr[(long)(2 * c + 1) * V + site];
                }
            }
            ac = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a.x, b0.x, ac, 0, 0, 0);
            bd = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a.y, b0.y, bd, 0, 0, 0);
            ad = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a.x, b0.y, ad, 0, 0, 0);
            bc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a.y, b0.x, bc, 0, 0, 0);
            ac = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a.z, b1.x, ac, 0, 0, 0);
            bd = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a.w, b1.y, bd, 0, 0, 0);
            ad = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a.z, b1.y, ad, 0, 0, 0);
            bc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a.w, b1.x, bc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            red[wave][0][kk + 4 * i][row] = ac[i] + bd[i];
            red[wave][1][kk + 4 * i][row] = ad[i] - bc[i];
        }
        __syncthreads();
        {
            const int orow = threadIdx.x >> 4, orr = threadIdx.x & 15;
            if (l0 + orow < Ns && r0 + orr < n) {
                double re = 0, im = 0;
                for (int w = 0; w < 4; ++w) {
                    re += red[w][0][orow][orr];
                    im += red[w][1][orow][orr];
                }
                u[((size_t)(r0 + orr) * Nb + B) * Ns + l0 + orow] = make_double2(re, im);
            }
        }
        __syncthreads();
    }
}

// v_r (op)= sum_l phi_{B,l} c[r][B][l]; MODE 0: v = .., 1: v -= .., 2: v += ..
// Each thread owns one float4 element (two complex) of a block and PR
// right-hand sides, so phi is read once per PR vectors.  A workgroup covers
// one chunk of 256 elements of one block (grid.x = blocks x chunks), so the
// block's coefficients are the same for all its threads: they are staged in
// LDS when they fit (Ns x PR complex), which takes the chain of dependent
// coefficient loads out of the inner loop.  Sums are FP64 either way.
constexpr int PR = 12;
template <class E, int MODE, bool STG>
__global__ void __launch_bounds__(256) k_prolong(E *__restrict__ v, const float4 *__restrict__ phi,
                                                 const int *__restrict__ boff, const double2 *__restrict__ cf,
                                                 long V, long Vh, int Vbh, int rb, int Ns, int Nb, int n,
                                                 int nchunk) {
    const int B = blockIdx.x / nchunk;
    const long per = 12L * Vbh * rb;
    const long q = (long)(blockIdx.x - B * nchunk) * 256 + threadIdx.x;
    const int r0 = blockIdx.y * PR;
    const int nr = min(PR, n - r0);
    // STG: the workgroup's coefficients c[r0 + k][B][l] staged in LDS once
    // (cs[l][k], zero for k >= nr), read back as broadcasts; otherwise each
    // is read from global memory where it is used
    extern __shared__ double2 cs[];
    if constexpr (STG) {
        for (int i = threadIdx.x; i < Ns * PR; i += 256) {
            const int l = i / PR, k = i - l * PR;
            cs[i] = k < nr ? cf[((size_t)(r0 + k) * Nb + B) * Ns + l] : make_double2(0, 0);
        }
        __syncthreads();
    }
    if (q >= per) return;
    int c;
    const long site = dfl_site(boff, B, rb, Vbh, Vh, q, c);
    double ar[PR], ai[PR], br[PR], bi[PR];
#pragma unroll
    for (int k = 0; k < PR; ++k) ar[k] = ai[k] = br[k] = bi[k] = 0;
    for (int l = 0; l < Ns; ++l) {
        const float4 f = phi[((size_t)B * Ns + l) * per + q];
#pragma unroll
        for (int k = 0; k < PR; ++k)
            if (STG || k < nr) {
                const double2 w = STG ? cs[l * PR + k] : cf[((size_t)(r0 + k) * Nb + B) * Ns + l];
                ar[k] += f.x * w.x - f.y * w.y;
                ai[k] += f.x * w.y + f.y * w.x;
                br[k] += f.z * w.x - f.w * w.y;
                bi[k] += f.z * w.y + f.w * w.x;
            }
    }
    constexpr bool F32V = sizeof(E) == 16 && sizeof(((E *)0)->x) == 4;
#pragma unroll
    for (int k = 0; k < PR; ++k) {
        if (k >= nr) break;
        const int r = r0 + k;
        if constexpr (F32V) {
            float4 *dst = reinterpret_cast<float4 *>(v) + (size_t)r * 6 * V + (size_t)c * V + site;
            float4 o = MODE == 0 ? make_float4(0, 0, 0, 0) : *dst;
            const float sg = MODE == 1 ? -1.f : 1.f;
            *dst = make_float4(o.x + sg * (float)ar[k], o.y + sg * (float)ai[k], o.z + sg * (float)br[k],
                               o.w + sg * (float)bi[k]);
        } else {
            double2 *d0 = reinterpret_cast<double2 *>(v) + (size_t)r * 12 * V + (size_t)(2 * c) * V + site;
            double2 *d1 = reinterpret_cast<double2 *>(v) + (size_t)r * 12 * V + (size_t)(2 * c + 1) * V + site;
            double2 o0 = MODE == 0 ? make_double2(0, 0) : *d0, o1 = MODE == 0 ? make_double2(0, 0) : *d1;
            const double sg = MODE == 1 ? -1.0 : 1.0;
            *d0 = make_double2(o0.x + sg * ar[k], o0.y + sg * ai[k]);
            *d1 = make_double2(o1.x + sg * br[k], o1.y + sg * bi[k]);
        }
    }
}

// w[r][B] = sgn sum_{d0 <= d < ND} M[B][d] v_d[r][nb(B, d)] with Ns x Ns
// complex blocks M[B][d] (ND = 9: the little operator, neighbour d of block B
// from the table; ND = 1: the block-Jacobi inverse acting on block B
// itself).  The self block (d = 0) reads vs, the neighbours vn (the same
// array for a plain product); d0 = 1 leaves the self block out.  Rows: the
// blocks listed in rows[0..nrows) (all Nb blocks when rows is null); other
// blocks of w are not written.  Per block this is a complex GEMM
// (Ns x ND Ns) (ND Ns x n) on the FP64 matrix cores: a wave owns one block,
// 16 rows and 16 right-hand sides, and with M = a + ib, v = c + id
// accumulates Re w = a c - b d and Im w = a d + b c as real 16x16x4 products
// over four complex elements of K at a time.  Lane L supplies
// M[row L % 16][k L / 16] and v[k L / 16][rhs L % 16] and receives
// w[row L / 16 + 4 i][rhs L % 16], i = 0..3 (the FP64 product's result
// layout; the FP32 16x16x4 product returns row 4 (L / 16) + i).
template <int ND>
__global__ void __launch_bounds__(256) k_little_mfma(const double2 *__restrict__ M, const int *__restrict__ bnbr,
                                                     const double2 *__restrict__ vs, const double2 *__restrict__ vn,
                                                     double2 *__restrict__ w, const int *__restrict__ rows,
                                                     int nrows, int d0, double sgn, int Nb, int Ns, int n, int nmt,
                                                     int nrt) {
    const int lane = threadIdx.x & 63;
    const long wid = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const long per_block = (long)nmt * nrt;
    if (wid >= (long)nrows * per_block) return;
    const int ri = (int)(wid / per_block);
    const int B = rows ? rows[ri] : ri;
    const int rem = (int)(wid - (long)ri * per_block);
    const int m0 = (rem / nrt) * 16, r0 = (rem % nrt) * 16;
    const int row = lane & 15, kk = lane >> 4;
    const int m = m0 + row, r = r0 + row;
    const bool mv = m < Ns, rv = r < n;
    const size_t N = (size_t)Nb * Ns;
    d4v ac = {0, 0, 0, 0}, bd = {0, 0, 0, 0}, ad = {0, 0, 0, 0}, bc = {0, 0, 0, 0};
    for (int d = d0; d < ND; ++d) {
        const double2 *Md = M + ((size_t)B * ND + d) * Ns * Ns + (size_t)(mv ? m : 0) * Ns;
        const int nb = (ND == 1 || d == 0) ? B : bnbr[B * 9 + d];
        const double2 *vd = (d == 0 ? vs : vn) + (size_t)(rv ? r : 0) * N + (size_t)nb * Ns;
        for (int l0 = 0; l0 < Ns; l0 += 4) {
            const int l = l0 + kk;
            double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
            if (l < Ns) {
                if (mv) a = Md[l];
                if (rv) b = vd[l];
            }
            ac = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, ac, 0, 0, 0);
            bd = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, bd, 0, 0, 0);
            ad = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, ad, 0, 0, 0);
            bc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, bc, 0, 0, 0);
        }
    }
    if (!rv) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int mo = m0 + kk + 4 * i;
        if (mo < Ns)
            w[(size_t)r * N + (size_t)B * Ns + mo] = make_double2(sgn * (ac[i] - bd[i]), sgn * (ad[i] + bc[i]));
    }
}

// v[r][B] = 0 for the blocks B listed in rows[0..nrows)
__global__ void k_zero_rows(double2 *__restrict__ v, const int *__restrict__ rows, int nrows, int Nb, int Ns, int n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)n * nrows * Ns) return;
    const int k = (int)(i % Ns);
    const long rb = i / Ns;
    const int ri = (int)(rb % nrows), r = (int)(rb / nrows);
    v[((size_t)r * Nb + rows[ri]) * Ns + k] = make_double2(0.0, 0.0);
}

// Dinv[B] = A[B][0]^{-1}: Gauss-Jordan with partial pivoting, one thread per
// block, working copy in `work` ([Nb][Ns][Ns])
__global__ void k_block_inverse(const double2 *__restrict__ A, double2 *__restrict__ Dinv,
                                double2 *__restrict__ work, int Nb, int Ns, int *flag) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= Nb) return;
    double2 *a = work + (size_t)B * Ns * Ns;
    double2 *b = Dinv + (size_t)B * Ns * Ns;
    const double2 *src = A + (size_t)B * 9 * Ns * Ns;
    for (int i = 0; i < Ns * Ns; ++i) {
        a[i] = src[i];
        b[i] = make_double2((i / Ns) == (i % Ns) ? 1.0 : 0.0, 0.0);
    }
    double scale = 0;
    for (int i = 0; i < Ns * Ns; ++i) scale = fmax(scale, a[i].x * a[i].x + a[i].y * a[i].y);
    for (int c = 0; c < Ns; ++c) {
        int p = c;
        double best = a[c * Ns + c].x * a[c * Ns + c].x + a[c * Ns + c].y * a[c * Ns + c].y;
        for (int r = c + 1; r < Ns; ++r) {
            const double v = a[r * Ns + c].x * a[r * Ns + c].x + a[r * Ns + c].y * a[r * Ns + c].y;
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (!(best > 1e-28 * scale)) {
            atomicOr(flag, 4);
            return;
        }
        if (p != c)
            for (int k = 0; k < Ns; ++k) {
                double2 t = a[c * Ns + k];
                a[c * Ns + k] = a[p * Ns + k];
                a[p * Ns + k] = t;
                t = b[c * Ns + k];
                b[c * Ns + k] = b[p * Ns + k];
                b[p * Ns + k] = t;
            }
        const double2 pv = a[c * Ns + c];
        const double den = pv.x * pv.x + pv.y * pv.y;
        const double2 iv = make_double2(pv.x / den, -pv.y / den);
        for (int k = 0; k < Ns; ++k) {
            double2 t = a[c * Ns + k];
            a[c * Ns + k] = make_double2(t.x * iv.x - t.y * iv.y, t.x * iv.y + t.y * iv.x);
            t = b[c * Ns + k];
            b[c * Ns + k] = make_double2(t.x * iv.x - t.y * iv.y, t.x * iv.y + t.y * iv.x);
        }
        for (int r = 0; r < Ns; ++r) {
            if (r == c) continue;
            const double2 f = a[r * Ns + c];
            if (f.x == 0 && f.y == 0) continue;
            for (int k = 0; k < Ns; ++k) {
                const double2 u = a[c * Ns + k], q = b[c * Ns + k];
                a[r * Ns + k].x -= f.x * u.x - f.y * u.y;
                a[r * Ns + k].y -= f.x * u.y + f.y * u.x;
                b[r * Ns + k].x -= f.x * q.x - f.y * q.y;
                b[r * Ns + k].y -= f.x * q.y + f.y * q.x;
            }
        }
    }
}

// loc[idx] = lexicographic site index inside its block, blex[idx] = lexicographic block
__global__ void k_block_site_tables(Geom g, const int *__restrict__ lex_of, int *__restrict__ loc,
                                    int *__restrict__ blex) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.V) return;
    long r = lex_of[idx];
    int c[4];
    for (int m = 3; m >= 0; --m) {
        c[m] = (int)(r % g.L[m]);
        r /= g.L[m];
    }
    int Bl = 0, l = 0;
    for (int m = 0; m < 4; ++m) {
        Bl = Bl * g.nb[m] + c[m] / g.b[m];
        l = l * g.b[m] + c[m] % g.b[m];
    }
    loc[idx] = l;
    blex[idx] = Bl;
}

// canonical phi [Nb][Ns][Vb][12] complex128 (Vb = 2 r Vbh sites of a
// deflation block in local lexicographic order) <-> internal block storage
__global__ void k_phi_export(const float4 *__restrict__ phi, double2 *__restrict__ out, const int *__restrict__ boff,
                             const int *__restrict__ loc, long Vh, int Vbh, int r, int Ns, int Nb) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;  // over (B, l, m, p, j)
    if (t >= (long)Nb * Ns * r * 2 * Vbh) return;
    const int j = (int)(t % Vbh), p = (int)((t / Vbh) % 2);
    const long q2 = t / (2 * Vbh);
    const int m = (int)(q2 % r);
    const long bl = q2 / r;
    const int l = (int)(bl % Ns), B = (int)(bl / Ns);
    const long site = p * Vh + boff[(long)B * r + m] + j;
    const int jl = loc[site];
    const long Vb = 2L * Vbh * r;
    const float4 *src = phi + (((size_t)B * Ns + l) * r + m) * 12 * Vbh;
    double2 *dst = out + (((size_t)B * Ns + l) * Vb + jl) * 12;
    for (int c = 0; c < 6; ++c) {
        const float4 f = src[(size_t)c * 2 * Vbh + p * Vbh + j];
        dst[2 * c] = make_double2(f.x, f.y);
        dst[2 * c + 1] = make_double2(f.z, f.w);
    }
}

__global__ void k_phi_import(const double2 *__restrict__ in, float4 *__restrict__ phi, const int *__restrict__ boff,
                             const int *__restrict__ loc, long Vh, int Vbh, int r, int Ns, int Nb) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)Nb * Ns * r * 2 * Vbh) return;
    const int j = (int)(t % Vbh), p = (int)((t / Vbh) % 2);
    const long q2 = t / (2 * Vbh);
    const int m = (int)(q2 % r);
    const long bl = q2 / r;
    const int l = (int)(bl % Ns), B = (int)(bl / Ns);
    const long site = p * Vh + boff[(long)B * r + m] + j;
    const int jl = loc[site];
    const long Vb = 2L * Vbh * r;
    float4 *dst = phi + (((size_t)B * Ns + l) * r + m) * 12 * Vbh;
    const double2 *src = in + (((size_t)B * Ns + l) * Vb + jl) * 12;
    for (int c = 0; c < 6; ++c) {
        const double2 a = src[2 * c], b = src[2 * c + 1];
        dst[(size_t)c * 2 * Vbh + p * Vbh + j] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

int dfl_work(qcd_dfl d, size_t bytes, void **p) {
    if (bytes > d->lw_bytes) {
        if (capturing()) return set_error(QCD_EINVAL, "workspace growth during stream capture");
        ++d->f->graph_gen;
        if (d->lw) {
            DFL_HIP(hipDeviceSynchronize());
            ws_release(d->device, d->lw, d->lw_bytes);
        }
        d->lw = nullptr;
        d->lw_bytes = 0;
        size_t got = 0;
        DFL_TRY(ws_acquire(d->device, bytes, &d->lw, &got));
        d->lw_bytes = got;
    }
    *p = d->lw;
    return 0;
}

// algorithmic work of Phi^+ v or Phi c: 8 flop per complex multiply-add,
// Ns x 12 V of them per rhs; bytes: phi once per call plus the vectors
inline void dfl_work_counts(qcd_dfl d, int n, size_t vbytes_site, double &fl, double &by) {
    const double V = (double)d->f->g.V;
    fl = 8.0 * d->Ns * 12.0 * V * n;
    by = 8.0 * d->Ns * 12.0 * V + (double)vbytes_site * V * n;
}

template <class E>
int restrict_v(qcd_dfl d, const E *v, double2 *u, int n, hipStream_t s) {
    const Geom &g = d->f->g;
    constexpr bool F32V = sizeof(E) == 16 && sizeof(((E *)0)->x) == 4;
    double fl, by;
    dfl_work_counts(d, n, F32V ? 96 : 192, fl, by);
    ProfScope ps(PROF_DFL, s, fl, by, (double)g.V * n);
    if constexpr (F32V)
        k_restrict_mfma<<<dim3(d->Nb, (n + 7) / 8), 256, 0, s>>>(reinterpret_cast<const float4 *>(v), d->phi, d->boff,
                                                                  u, g.V, g.Vh, g.Vbh, d->r, d->Ns, d->Nb, n);
    else
        k_restrict_mfma64<<<dim3(d->Nb, (n + 15) / 16), 256, 0, s>>>(v, d->phi, d->boff, u, g.V, g.Vh, g.Vbh, d->r,
                                                                    d->Ns, d->Nb, n);
    DFL_HIP(hipGetLastError());
    return 0;
}

template <class E, int MODE>
int prolong_v(qcd_dfl d, E *v, const double2 *c, int n, hipStream_t s) {
    const Geom &g = d->f->g;
    constexpr bool F32V = sizeof(E) == 16 && sizeof(((E *)0)->x) == 4;
    double fl, by;
    dfl_work_counts(d, n, (F32V ? 96 : 192) * (MODE == 0 ? 1 : 2), fl, by);
    ProfScope ps(PROF_DFL, s, fl, by, (double)g.V * n);
    const int nchunk = (int)nblocks(12L * g.Vbh * d->r, 256);
    const dim3 grid((unsigned)(d->Nb * nchunk), (n + PR - 1) / PR);
    const size_t stg = sizeof(double2) * (size_t)d->Ns * PR;
    if (stg <= 48 * 1024)
        k_prolong<E, MODE, true><<<grid, 256, stg, s>>>(v, d->phi, d->boff, c, g.V, g.Vh, g.Vbh, d->r, d->Ns, d->Nb,
                                                        n, nchunk);
    else
        k_prolong<E, MODE, false><<<grid, 256, 0, s>>>(v, d->phi, d->boff, c, g.V, g.Vh, g.Vbh, d->r, d->Ns, d->Nb,
                                                       n, nchunk);
    DFL_HIP(hipGetLastError());
    return 0;
}

template <int ND>
static int launch_little(qcd_dfl d, const double2 *M, const double2 *vs, const double2 *vn, double2 *w, int n,
                         hipStream_t s, const int *rows = nullptr, int nrows = -1, int d0 = 0, double sgn = 1.0) {
    if (nrows < 0) nrows = d->Nb;
    const int nmt = (d->Ns + 15) / 16, nrt = (n + 15) / 16;
    const long waves = (long)nrows * nmt * nrt;
    k_little_mfma<ND><<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(M, d->bnbr, vs, vn, w, rows, nrows, d0, sgn, d->Nb,
                                                                  d->Ns, n, nmt, nrt);
    DFL_HIP(hipGetLastError());
    return 0;
}

int little_apply_dev(qcd_dfl d, const double2 *v, double2 *w, int n, hipStream_t s) {
    const long N = (long)d->Nb * d->Ns;
    // 9 Ns^2 complex multiply-adds per block row and rhs; A read once per 16
    // right-hand sides, v and w once per rhs
    ProfScope ps(PROF_LITTLE, s, 8.0 * 9 * d->Ns * N * n,
                 16.0 * (9.0 * d->Ns * N * ((n + 15) / 16) + 2.0 * N * n), (double)N * n);
    return launch_little<9>(d, d->A, v, v, w, n, s);
}

// one colour's block rows of A (d0 = 1: without the self block) or of the
// block-Jacobi inverse, times sgn; the work accounting per row as for the
// full product
static int little_rows(qcd_dfl d, bool inverse, const double2 *vs, const double2 *vn, double2 *w, int n, int colour,
                       int d0, double sgn, hipStream_t s) {
    const int nh = d->Nb / 2;
    const double rows = (double)nh * d->Ns;
    const double nd = inverse ? 1.0 : 9.0 - d0;
    ProfScope ps(PROF_LITTLE, s, 8.0 * nd * d->Ns * rows * n,
                 16.0 * (nd * d->Ns * rows * ((n + 15) / 16) + 2.0 * rows * n), rows * n);
    const int *rl = d->brow + (size_t)colour * nh;
    if (inverse) return launch_little<1>(d, d->Dinv, vs, vn, w, n, s, rl, nh, 0, sgn);
    return launch_little<9>(d, d->A, vs, vn, w, n, s, rl, nh, d0, sgn);
}

static int zero_rows(qcd_dfl d, double2 *v, int n, int colour, hipStream_t s) {
    const int nh = d->Nb / 2;
    k_zero_rows<<<nblocks((long)n * nh * d->Ns, 256), 256, 0, s>>>(v, d->brow + (size_t)colour * nh, nh, d->Nb,
                                                                   d->Ns, n);
    DFL_HIP(hipGetLastError());
    return 0;
}

// w = S v_E on the even blocks, S = A_EE - A_EO A_OO^{-1} A_OE (only v's
// even blocks are read; w's odd blocks are zero); t, q: work vectors
static int schur_apply(qcd_dfl d, const double2 *v, double2 *w, double2 *t, double2 *q, int n, hipStream_t s) {
    const long N = (long)d->Nb * d->Ns;
    DFL_TRY(little_rows(d, false, v, v, t, n, 1, 1, 1.0, s));      // t_O = A_OE v_E
    DFL_TRY(little_rows(d, true, t, t, q, n, 1, 0, -1.0, s));      // q_O = -A_OO^{-1} t_O
    DFL_TRY(blas_zero<double2>(w, N, n, s));
    return little_rows(d, false, v, q, w, n, 0, 0, 1.0, s);        // w_E = A_EE v_E + A_EO q_O
}

// x = A^{-1} u (FP64) by the block even-odd Schur complement.  Blocks are
// coloured by the parity of their coordinates on the deflation-block grid
// (an even number of blocks along every axis), so every coupling of A joins
// blocks of opposite colour and A_EE, A_OO are block diagonal:
//   u'_E = u_E - A_EO A_OO^{-1} u_O,
//   S x_E = u'_E, S = A_EE - A_EO A_OO^{-1} A_OE, by GCR preconditioned
//   with A_EE^{-1} (the block-Jacobi factors of the even blocks),
//   x_O = A_OO^{-1} (u_O - A_OE x_E).
// Vectors are full length [n][Nb][Ns]; the Krylov space lives on the even
// blocks.  The residual of the full system equals that of the Schur system
// (x_O is exact given x_E), and it is reported relative to ||u||.  poll:
// check it on the host after every iteration and stop at tol; otherwise run
// one cycle of min(maxit, nkv) iterations without host synchronisation.
int little_solve(qcd_dfl d, const double2 *u, double2 *x, int n, double tol, int maxit, bool poll, int *iters_out,
                 double *relres_out, hipStream_t s) {
    // polled norms pass through the handle's pinned buffer of 4096 doubles
    if (n > 4096) return set_error(QCD_EINVAL, "too many right-hand sides in one little solve (max 4096)");
    const long N = (long)d->Nb * d->Ns;
    const int nkv = std::max(1, std::min(maxit, 24));
    const size_t vb = sizeof(double2) * N * n;
    const size_t need = vb * (2 * (size_t)nkv + 4) + scalar_bytes(n);
    void *p;
    DFL_TRY(dfl_work(d, need, &p));
    double2 *Z = static_cast<double2 *>(p);
    double2 *W = Z + (size_t)nkv * n * N;
    double2 *r = W + (size_t)nkv * n * N;
    double2 *t = r + (size_t)n * N;
    double2 *q = t + (size_t)n * N;
    double2 *us = q + (size_t)n * N;      // the Schur right-hand side u'
    Scal sc;
    DFL_TRY(scalar_buffers_at(us + (size_t)n * N, n, sc));
    std::vector<double> bn(n, 0.0), h(n);
    auto fetch = [&](const double *dev) -> int {
        DFL_HIP(hipMemcpyAsync(d->hp, dev, n * sizeof(double), hipMemcpyDeviceToHost, s));
        DFL_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < n; ++i) h[i] = d->hp[i];
        return 0;
    };
    if (poll) {
        DFL_TRY(blas_norm2<double2>(u, N, n, sc.part, sc.red, s));
        DFL_TRY(fetch(sc.red));
        for (int i = 0; i < n; ++i) bn[i] = std::sqrt(h[i]);
    }
    // u'_E = u_E - A_EO A_OO^{-1} u_O (odd blocks zero); r = u', x = 0
    DFL_TRY(little_rows(d, true, u, u, q, n, 1, 0, 1.0, s));       // q_O = A_OO^{-1} u_O
    DFL_TRY(blas_zero<double2>(t, N, n, s));
    DFL_TRY(little_rows(d, false, q, q, t, n, 0, 1, 1.0, s));      // t_E = A_EO q_O
    DFL_TRY(blas_resid(u, t, us, N, n, sc.part, sc.red, s));       // us = u - t
    DFL_TRY(zero_rows(d, us, n, 1, s));
    DFL_HIP(hipMemcpyAsync(r, us, vb, hipMemcpyDeviceToDevice, s));
    DFL_TRY(blas_zero<double2>(x, N, n, s));
    int iters = 0;
    double worst = 0;
    bool done = false;
    while (!done && iters < maxit) {
        int k = 0;
        while (k < nkv && iters < maxit) {
            double2 *zk = Z + (size_t)k * n * N, *wk = W + (size_t)k * n * N;
            // z = A_EE^{-1} r on the even blocks (the odd blocks of z are never read)
            DFL_TRY(little_rows(d, true, r, r, zk, n, 0, 0, 1.0, s));
            DFL_TRY(schur_apply(d, zk, wk, t, q, n, s));
            int bstride = 2;
            if (k > 0) bstride = blas_multidot<double2>(W, N, n, k, sc.part, sc.red2, s);
            if (bstride < 0) return bstride;
            DFL_TRY(blas_gs_sub<double2>(W, r, N, n, k, sc.red2, bstride, sc.part, sc.red, s));
            DFL_TRY(gcr_scalars(sc.red2, bstride, sc.red, n, k, sc.R, sc.cvec, sc.coef, s));
            DFL_TRY(blas_scal_update<double2>(wk, r, N, n, sc.coef, sc.part, sc.red, s));
            ++k;
            ++iters;
            if (poll) {
                DFL_TRY(fetch(sc.red));
                bool ok = true;
                worst = 0;
                for (int i = 0; i < n; ++i) {
                    const double rel = bn[i] > 0 ? std::sqrt(h[i]) / bn[i] : 0.0;
                    worst = std::max(worst, rel);
                    if (!(rel <= tol)) ok = false;
                }
                if (ok) {
                    done = true;
                    break;
                }
            }
        }
        DFL_TRY(gcr_trisolve(sc.R, sc.cvec, n, k, sc.alpha, s));
        DFL_TRY(blas_accum_d(x, Z, N, n, k, sc.alpha, 2 * NKV_MAX, s));
        if (!poll) break;
        if (!done && iters < maxit) {  // restart from the true Schur residual
            DFL_TRY(schur_apply(d, x, t, q, W, n, s));   // the Krylov vectors are free at a restart
            DFL_TRY(blas_resid(us, t, r, N, n, sc.part, sc.red, s));
        }
    }
    // x_O = A_OO^{-1} (u_O - A_OE x_E)
    DFL_TRY(little_rows(d, false, x, x, t, n, 1, 1, 1.0, s));      // t_O = A_OE x_E
    DFL_TRY(blas_resid(u, t, q, N, n, sc.part, sc.red, s));        // q = u - t (odd blocks used)
    DFL_TRY(little_rows(d, true, q, q, x, n, 1, 0, 1.0, s));       // x_O = A_OO^{-1} q_O
    if (iters_out) *iters_out = iters;
    if (relres_out) *relres_out = worst;
    return (poll && !done) ? QCD_NOCONV : 0;
}

// A[B][dd][k][l] = u9[dd][B][k] for one column l
__global__ void k_little_column(const double2 *__restrict__ u9, double2 *__restrict__ A, int Nb, int Ns, int l) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 9L * Nb * Ns) return;
    const int k = (int)(i % Ns);
    const long dB = i / Ns;
    const int B = (int)(dB % Nb), dd = (int)(dB / Nb);
    A[(((size_t)B * 9 + dd) * Ns + k) * Ns + l] = u9[i];
}

// A[:, d, :, l] for every l from the direction-resolved operator
int build_little(qcd_dfl d, hipStream_t s) {
    qcd_field f = d->f;
    const Geom &g = f->g;
    const long V = g.V;
    const int Ns = d->Ns, Nb = d->Nb;
    void *p;
    const size_t fbytes = sizeof(float4) * 6 * V;
    const size_t obytes = sizeof(double2) * 12 * V * 9;
    const size_t ubytes = sizeof(double2) * (size_t)9 * Nb * Ns;
    DFL_TRY(dfl_work(d, fbytes + obytes + ubytes + sizeof(double2) * (size_t)Nb * Ns * Ns, &p));
    float4 *fl = static_cast<float4 *>(p);
    double2 *out9 = reinterpret_cast<double2 *>(static_cast<char *>(p) + fbytes);
    double2 *u9 = out9 + (size_t)12 * V * 9;
    double2 *work = u9 + (size_t)9 * Nb * Ns;
    for (int l = 0; l < Ns; ++l) {
        {
            ProfScope ps(PROF_DFL, s);
            k_phi_field<<<nblocks((long)Nb * 12 * g.Vbh * d->r, 256), 256, 0, s>>>(d->phi, l, fl, d->boff, V, g.Vh,
                                                                                   g.Vbh, d->r, Ns, Nb);
            k_dirac_split<<<nblocks(V, 128), 128, 0, s>>>(fl, out9, f->U[LNK_F64], f->clo[CLO_F64], f->nbr, d->dbof,
                                                          V, g.Vh, g.Vbh, f->lat.kappa);
        }
        DFL_HIP(hipGetLastError());
        // u9[dd][B][k] = (phi_{B,k}, out_dd) ; treat the 9 outputs as 9 right-hand sides
        DFL_TRY(restrict_v<double2>(d, out9, u9, 9, s));
        k_little_column<<<nblocks(9L * Nb * Ns, 256), 256, 0, s>>>(u9, d->A, Nb, Ns, l);
        DFL_HIP(hipGetLastError());
    }
    DFL_HIP(hipMemsetAsync(f->flag, 0, sizeof(int), s));
    k_block_inverse<<<nblocks(Nb, 64), 64, 0, s>>>(d->A, d->Dinv, work, Nb, Ns, f->flag);
    DFL_HIP(hipGetLastError());
    int flag = 0;
    DFL_HIP(hipMemcpyAsync(&flag, f->flag, sizeof(int), hipMemcpyDeviceToHost, s));
    DFL_HIP(hipStreamSynchronize(s));
    if (flag) return set_error(QCD_ESINGULAR, "a diagonal block of the little operator is singular");
    return 0;
}

void dfl_free(qcd_dfl d) {
    if (!d) return;
    (void)hipFree(d->phi);
    (void)hipFree(d->A);
    (void)hipFree(d->Dinv);
    (void)hipFree(d->bnbr);
    (void)hipFree(d->brow);
    (void)hipFree(d->boff);
    (void)hipFree(d->dbof);
    (void)hipFree(d->loc);
    (void)hipFree(d->blex);
    (void)hipDeviceSynchronize();
    ws_release(d->device, d->lw, d->lw_bytes);
    if (d->hp) (void)hipHostFree(d->hp);
    delete d;
}

// v_l <- v_l / ||v_l|| for Ns FP32 internal fields
int normalise_fields(qcd_field f, float4 *v, int Ns, hipStream_t s) {
    const long V = f->g.V;
    void *sp;
    DFL_TRY(field_buffer(f, BUF_RED, scalar_bytes(Ns), &sp));
    Scal sc;
    DFL_TRY(scalar_buffers_at(sp, Ns, sc));
    DFL_TRY(blas_norm2<float4>(v, 6 * V, Ns, sc.part, sc.red, s));
    k_normalise<<<dim3(nblocks(6 * V, 256), Ns), 256, 0, s>>>(v, 6 * V, sc.red);
    DFL_HIP(hipGetLastError());
    return 0;
}

// the global fields restricted to the deflation blocks, orthonormalised per
// block, and the little operator of that subspace
int fields_to_subspace(qcd_dfl d, const float4 *v, hipStream_t s) {
    qcd_field f = d->f;
    const Geom &g = f->g;
    const long per = 12L * g.Vbh * d->r;
    const long tot = (long)d->Nb * d->Ns * per;
    k_to_blocks<<<nblocks(tot, 256), 256, 0, s>>>(v, d->phi, d->boff, g.V, g.Vh, g.Vbh, d->r, d->Ns, d->Nb);
    DFL_HIP(hipGetLastError());
    DFL_HIP(hipMemsetAsync(f->flag, 0, sizeof(int), s));
    k_block_mgs<<<d->Nb, 256, 0, s>>>(d->phi, d->Ns, per, f->flag);
    DFL_HIP(hipGetLastError());
    int flag = 0;
    DFL_HIP(hipMemcpyAsync(&flag, f->flag, sizeof(int), hipMemcpyDeviceToHost, s));
    DFL_HIP(hipStreamSynchronize(s));
    if (flag) return set_error(QCD_ESINGULAR, "deflation fields are linearly dependent on a block");
    return build_little(d, s);
}

// one round v_l <- M^{-1} v_l / ||M^{-1} v_l|| for the Ns FP32 global
// fields, each solve by the deflated SAP-GCR solver on the handle's current
// subspace to relative residual params.ref_res (at most 256 iterations; a
// solve stopped there still gives a valid inverse-iteration step), in
// batches that fit the free device memory
int inverse_iteration(qcd_dfl d, float4 *v, hipStream_t s) {
    qcd_field f = d->f;
    const long V = f->g.V;
    const int Ns = d->Ns;
    qcd_gcr q{};
    q.nkv = 8;
    q.nmx = 256;
    q.fixed_iters = 0;
    q.res = d->params.ref_res;
    q.sap = d->params.sap;
    q.dfl = d;
    q.little_tol = 1e-8;
    q.little_maxit = 16;
    // the global fields stay in the handle's source buffer during the solves
    const int nb = std::max(1, std::min(Ns, pick_batch(f, q, 0, BUF_AMA)));
    void *p;
    DFL_TRY(field_buffer(f, BUF_APPLY, 2 * spinor_bytes(QCD_F64, V) * nb, &p));
    double2 *b64 = static_cast<double2 *>(p), *x64 = b64 + (size_t)12 * V * nb;
    for (int l0 = 0; l0 < Ns; l0 += nb) {
        const int n = std::min(nb, Ns - l0);
        float4 *vl = v + (size_t)6 * V * l0;
        k_widen<<<dim3(nblocks(6 * V, 256), n), 256, 0, s>>>(vl, b64, V);
        DFL_HIP(hipGetLastError());
        const int rc = gcr_internal(f, &q, b64, x64, n, nullptr, s);
        if (rc < 0) return rc;
        k_narrow<<<dim3(nblocks(6 * V, 256), n), 256, 0, s>>>(x64, vl, V);
        DFL_HIP(hipGetLastError());
    }
    return normalise_fields(f, v, Ns, s);
}

}  // namespace

int dfl_low_mode(qcd_dfl d, const double2 *b, double2 *x, int n, double tol, int maxit, bool set, hipStream_t s) {
    const size_t nv = (size_t)d->Nb * d->Ns * n;
    void *p;
    DFL_TRY(field_buffer(d->f, BUF_DFL, 2 * nv * sizeof(double2), &p));
    double2 *u = static_cast<double2 *>(p), *c = u + nv;
    DFL_TRY(restrict_v<double2>(d, b, u, n, s));
    // polled to tol, except without host synchronisation (fixed budget)
    int rc = little_solve(d, u, c, n, tol, maxit, !nosync(), nullptr, nullptr, s);
    if (rc < 0) return rc;
    return set ? prolong_v<double2, 0>(d, x, c, n, s) : prolong_v<double2, 2>(d, x, c, n, s);
}

int dfl_project_R(qcd_dfl d, void *z, void *tmp, int n, qcd_prec vec, qcd_prec storage, int maxit, hipStream_t s) {
    const size_t nv = (size_t)d->Nb * d->Ns * n;
    void *p;
    DFL_TRY(field_buffer(d->f, BUF_DFL, 2 * nv * sizeof(double2), &p));
    double2 *u = static_cast<double2 *>(p), *c = u + nv;
    DFL_TRY(dirac_internal(d->f, z, tmp, n, vec, storage, s));
    if (vec == QCD_F32) {
        DFL_TRY(restrict_v<float4>(d, static_cast<const float4 *>(tmp), u, n, s));
    } else {
        DFL_TRY(restrict_v<double2>(d, static_cast<const double2 *>(tmp), u, n, s));
    }
    int rc = little_solve(d, u, c, n, 0.0, maxit, false, nullptr, nullptr, s);
    if (rc < 0) return rc;
    if (vec == QCD_F32) return prolong_v<float4, 1>(d, static_cast<float4 *>(z), c, n, s);
    return prolong_v<double2, 1>(d, static_cast<double2 *>(z), c, n, s);
}

}  // namespace dfl

using namespace dfl;

extern "C" {

int deflation_setup(qcd_field f, const qcd_dfl_params *prm, hipStream_t s, qcd_dfl *out) {
    if (!f || !prm || !out) return set_error(QCD_EINVAL, "null argument to deflation_setup");
    *out = nullptr;
    const Geom &g = f->g;
    // deflation blocks: the Schwarz block, or a multiple of it in every
    // direction with an even number of blocks along each axis
    Geom dg = g;
    int rr[4];
    for (int m = 0; m < 4; ++m) {
        const int bd = prm->block[m] ? prm->block[m] : g.b[m];
        if (bd < g.b[m] || bd % g.b[m] || g.L[m] % bd || (g.L[m] / bd) % 2)
            return set_error(QCD_EGEOM, "the deflation block must be a multiple of the Schwarz block with an even "
                                        "number of deflation blocks along every axis");
        dg.b[m] = bd;
        dg.nb[m] = g.L[m] / bd;
        rr[m] = bd / g.b[m];
    }
    dg.Vb = dg.b[0] * dg.b[1] * dg.b[2] * dg.b[3];
    dg.Vbh = dg.Vb / 2;
    dg.Nb = (int)(g.V / dg.Vb);
    if (prm->Ns < 1 || prm->Ns > 12 * dg.Vb)
        return set_error(QCD_ESINGULAR, "Ns must be between 1 and 12 times the deflation block volume");
    if (prm->ninv < 0 || prm->nref < 0) return set_error(QCD_EINVAL, "ninv and nref must be >= 0");
    if (prm->nref > 0 && !(prm->ref_res > 0 && prm->ref_res < 1))
        return set_error(QCD_EINVAL, "ref_res must be in (0, 1) when nref > 0");
    qcd_dfl d = new qcd_dfl_s();
    d->f = f;
    d->device = f->device;
    d->params = *prm;
    d->Ns = prm->Ns;
    d->Nb = dg.Nb;
    d->dg = dg;
    d->r = rr[0] * rr[1] * rr[2] * rr[3];
    auto fail = [&](int rc) {
        dfl_free(d);
        return rc;
    };
    const int Ns = d->Ns, Nb = d->Nb, r = d->r;
    const long V = g.V;
    // Schwarz blocks: memory rank (colour-major) of each lexicographic block
    std::vector<int> srank(g.Nb);
    {
        int cnt[2] = {0, 0};
        for (int B = 0; B < g.Nb; ++B) {
            int q = B, sum = 0;
            for (int m = 3; m >= 0; --m) {
                sum += q % g.nb[m];
                q /= g.nb[m];
            }
            srank[B] = (sum & 1) * (g.Nb / 2) + cnt[sum & 1]++;
        }
    }
    // deflation-block tables (lexicographic order of the deflation-block grid)
    std::vector<int> boff((size_t)Nb * r), dbof(g.Nb), bnbr((size_t)Nb * 9), brow;
    brow.reserve(Nb);
    for (int colour = 0; colour < 2; ++colour)
        for (int B = 0; B < Nb; ++B) {
            int q = B, sum = 0;
            for (int m = 3; m >= 0; --m) {
                sum += q % dg.nb[m];
                q /= dg.nb[m];
            }
            if ((sum & 1) == colour) brow.push_back(B);
        }
    for (int B = 0; B < Nb; ++B) {
        int c[4], q = B;
        for (int m = 3; m >= 0; --m) {
            c[m] = q % dg.nb[m];
            q /= dg.nb[m];
        }
        for (int k = 0; k < r; ++k) {   // member k: lexicographic inside the deflation block
            int sc[4], t = k;
            for (int m = 3; m >= 0; --m) {
                sc[m] = c[m] * rr[m] + t % rr[m];
                t /= rr[m];
            }
            int Bs = 0;
            for (int m = 0; m < 4; ++m) Bs = Bs * g.nb[m] + sc[m];
            boff[(size_t)B * r + k] = srank[Bs] * g.Vbh;
            dbof[srank[Bs]] = B;
        }
        bnbr[(size_t)B * 9] = B;
        for (int mu = 0; mu < 4; ++mu)
            for (int dir = 0; dir < 2; ++dir) {
                int cc[4] = {c[0], c[1], c[2], c[3]};
                cc[mu] = (cc[mu] + (dir == 0 ? 1 : -1) + dg.nb[mu]) % dg.nb[mu];
                int k = 0;
                for (int m = 0; m < 4; ++m) k = k * dg.nb[m] + cc[m];
                bnbr[(size_t)B * 9 + 1 + 2 * mu + dir] = k;
            }
    }
#define DALLOC(ptr, bytes)                                                                 \
    if (!dev_alloc(d->device, (void **)&(ptr), (bytes))) {                                \
        return fail(set_error(QCD_ENOMEM, "device allocation failed in deflation_setup")); \
    }
    DALLOC(d->phi, sizeof(float4) * (size_t)Nb * Ns * 12 * r * g.Vbh);
    DALLOC(d->A, sizeof(double2) * (size_t)Nb * 9 * Ns * Ns);
    DALLOC(d->Dinv, sizeof(double2) * (size_t)Nb * Ns * Ns);
    DALLOC(d->bnbr, sizeof(int) * (size_t)Nb * 9);
    DALLOC(d->brow, sizeof(int) * (size_t)Nb);
    DALLOC(d->boff, sizeof(int) * (size_t)Nb * r);
    DALLOC(d->dbof, sizeof(int) * (size_t)g.Nb);
    DALLOC(d->loc, sizeof(int) * V);
    DALLOC(d->blex, sizeof(int) * V);
#undef DALLOC
    if (hipHostMalloc((void **)&d->hp, sizeof(double) * 4096) != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_error(QCD_ENOMEM, "pinned host allocation failed"));
    }
    hipError_t e = hipMemcpyAsync(d->bnbr, bnbr.data(), sizeof(int) * bnbr.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d->boff, boff.data(), sizeof(int) * boff.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d->dbof, dbof.data(), sizeof(int) * dbof.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d->brow, brow.data(), sizeof(int) * brow.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        k_block_site_tables<<<nblocks(V, 256), 256, 0, s>>>(dg, f->lex_of, d->loc, d->blex);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(set_error(QCD_EHIP, std::string("deflation upload: ") + hipGetErrorString(e)));

    // Ns random global fields, ninv rounds of v <- M_SAP v / ||.||
    void *vp;
    int rc = field_buffer(f, BUF_AMA, sizeof(float4) * 6 * V * (size_t)Ns * 2, &vp);
    if (rc < 0) return fail(rc);
    float4 *v = static_cast<float4 *>(vp), *w = v + (size_t)6 * V * Ns;
    const unsigned long long key = sm64(prm->seed, 5ULL);   // stream 5: deflation fields
    k_random_fields<<<dim3(nblocks(V, 256), Ns), 256, 0, s>>>(v, key, f->lex_of, V);
    if ((e = hipGetLastError()) != hipSuccess) return fail(set_error(QCD_EHIP, hipGetErrorString(e)));
    qcd_sap sap = prm->sap;
    if (sap.storage == QCD_F64) sap.storage = QCD_F32;   // the fields are refined in FP32
    for (int it = 0; it < prm->ninv; ++it) {
        rc = sap_internal(f, &sap, v, w, Ns, s);
        if (rc < 0) return fail(rc);
        std::swap(v, w);
        rc = normalise_fields(f, v, Ns, s);
        if (rc < 0) return fail(rc);
    }
    rc = fields_to_subspace(d, v, s);
    if (rc < 0) return fail(rc);
    // refinement: inverse iteration v <- M^{-1} v / ||.|| with the deflated
    // solver on the current subspace, a new subspace after every round
    for (int it = 0; it < prm->nref; ++it) {
        rc = inverse_iteration(d, v, s);
        if (rc < 0) return fail(rc);
        rc = fields_to_subspace(d, v, s);
        if (rc < 0) return fail(rc);
    }
    *out = d;
    return 0;
}

int deflation_destroy(qcd_dfl d) {
    dfl_free(d);
    return 0;
}

int deflation_dims(qcd_dfl d, int *Nb, int *Ns) {
    if (!d || !Nb || !Ns) return set_error(QCD_EINVAL, "null argument to deflation_dims");
    *Nb = d->Nb;
    *Ns = d->Ns;
    return 0;
}

int deflation_get_phi(qcd_dfl d, void *phi, hipStream_t s) {
    if (!d || !phi) return set_error(QCD_EINVAL, "null argument to deflation_get_phi");
    const Geom &g = d->f->g;
    const long tot = (long)d->Nb * d->Ns * d->r * 2 * g.Vbh;
    k_phi_export<<<nblocks(tot, 256), 256, 0, s>>>(d->phi, static_cast<double2 *>(phi), d->boff, d->loc, g.Vh, g.Vbh,
                                                   d->r, d->Ns, d->Nb);
    DFL_HIP(hipGetLastError());
    return 0;
}

int deflation_set_phi(qcd_dfl d, const void *phi, hipStream_t s) {
    if (!d || !phi) return set_error(QCD_EINVAL, "null argument to deflation_set_phi");
    const Geom &g = d->f->g;
    const long tot = (long)d->Nb * d->Ns * d->r * 2 * g.Vbh;
    k_phi_import<<<nblocks(tot, 256), 256, 0, s>>>(static_cast<const double2 *>(phi), d->phi, d->boff, d->loc, g.Vh,
                                                   g.Vbh, d->r, d->Ns, d->Nb);
    DFL_HIP(hipGetLastError());
    return build_little(d, s);
}

int little_dirac_apply(qcd_dfl d, const void *v, void *w, int nrhs, hipStream_t s) {
    if (!d || !v || !w || nrhs <= 0) return set_error(QCD_EINVAL, "bad arguments to little_dirac_apply");
    return little_apply_dev(d, static_cast<const double2 *>(v), static_cast<double2 *>(w), nrhs, s);
}

int little_dirac_solve(qcd_dfl d, const void *v, void *w, int nrhs, double tol, int maxit, int *iters,
                       hipStream_t s) {
    if (!d || !v || !w || nrhs <= 0 || maxit < 1) return set_error(QCD_EINVAL, "bad arguments to little_dirac_solve");
    if (nrhs > 4096) return set_error(QCD_EINVAL, "little_dirac_solve: at most 4096 right-hand sides per call");
    double rel = 0;
    int rc = little_solve(d, static_cast<const double2 *>(v), static_cast<double2 *>(w), nrhs, tol, maxit, true, iters,
                          &rel, s);
    if (rc < 0) return rc;
    DFL_HIP(hipStreamSynchronize(s));
    return rc;
}

int deflation_restrict(qcd_dfl d, const void *v, void *u, int nrhs, qcd_prec io, hipStream_t s) {
    if (!d || !v || !u || nrhs <= 0) return set_error(QCD_EINVAL, "bad arguments to deflation_restrict");
    // FP32 io takes the FP32 path of the solver (matrix-core GEMM, FP32
    // accumulation); FP64 io the FP64-accumulated one
    const qcd_prec vec = io == QCD_F32 ? QCD_F32 : QCD_F64;
    const size_t nb = spinor_bytes(vec, d->f->g.V) * nrhs;
    void *ws;
    DFL_TRY(field_buffer(d->f, BUF_APPLY, nb, &ws));
    DFL_TRY(pack_spinor(d->f, v, io, ws, vec, nrhs, s));
    if (vec == QCD_F32)
        return restrict_v<float4>(d, static_cast<const float4 *>(ws), static_cast<double2 *>(u), nrhs, s);
    return restrict_v<double2>(d, static_cast<const double2 *>(ws), static_cast<double2 *>(u), nrhs, s);
}

int deflation_prolong(qcd_dfl d, const void *u, void *v, int nrhs, qcd_prec io, hipStream_t s) {
    if (!d || !v || !u || nrhs <= 0) return set_error(QCD_EINVAL, "bad arguments to deflation_prolong");
    const qcd_prec vec = io == QCD_F32 ? QCD_F32 : QCD_F64;
    const size_t nb = spinor_bytes(vec, d->f->g.V) * nrhs;
    void *ws;
    DFL_TRY(field_buffer(d->f, BUF_APPLY, nb, &ws));
    if (vec == QCD_F32)
        DFL_TRY((prolong_v<float4, 0>(d, static_cast<float4 *>(ws), static_cast<const double2 *>(u), nrhs, s)));
    else
        DFL_TRY((prolong_v<double2, 0>(d, static_cast<double2 *>(ws), static_cast<const double2 *>(u), nrhs, s)));
    return unpack_spinor(d->f, ws, vec, v, io, nrhs, s);
}

}  // extern "C"
