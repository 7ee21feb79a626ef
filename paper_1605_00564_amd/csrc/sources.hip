// Source vectors built on the device: Z2 noise (all-mode averaging with
// stochastic sources) and sequential sources for three-point functions
// (the simplified gamma insertion used by the multi-right-hand-side
// workload: the forward solution times gamma_5 gamma_mu gamma_5 on one
// timeslice).  Both write canonical [n][V][4][3] vectors.
#include <complex>

#include "internal.h"

namespace dfl {

// noise vector r (of index index0 + r): component j = 12 lex + sc takes the
// sign of the top bit of SplitMix64 output (index0 + r) 12 V + j of the
// stream key
template <class CT>
__global__ void k_z2(CT *__restrict__ out, unsigned long long key, long V, long index0) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    const long r = blockIdx.y;
    CT *o = out + ((size_t)r * V + i) * 12;
    const unsigned long long base = ((unsigned long long)(index0 + r) * V + i) * 12;
#pragma unroll
    for (int sc = 0; sc < 12; ++sc) {
        const unsigned long long b = sm64(key, base + sc) >> 63;
        o[sc].x = b ? -1 : 1;
        o[sc].y = 0;
    }
}

// out(x) = G in(x) on timeslice t_sink (spin matrix G, colour untouched),
// 0 elsewhere; G given as 16 complex, row-major
struct Spin4 {
    double re[16], im[16];
};
template <class CT>
__global__ void k_seq(const CT *__restrict__ in, CT *__restrict__ out, long V, long spatial, int t_sink, Spin4 G) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    const size_t off = ((size_t)blockIdx.y * V + i) * 12;
    const bool on = i / spatial == t_sink;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double ar = 0, ai = 0;
            if (on)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const CT v = in[off + 3 * t + c];
                    ar += G.re[4 * s + t] * v.x - G.im[4 * s + t] * v.y;
                    ai += G.re[4 * s + t] * v.y + G.im[4 * s + t] * v.x;
                }
            out[off + 3 * s + c].x = ar;
            out[off + 3 * s + c].y = ai;
        }
}

// Euclidean chiral basis: gamma_0 = [[0,-1],[-1,0]], gamma_k = [[0,-i s_k],
// [i s_k, 0]], gamma_5 = diag(1,1,-1,-1); returns gamma_5 gamma_mu gamma_5
static Spin4 g5_gmu_g5(int mu) {
    using C = std::complex<double>;
    C g[4][4] = {};
    const C I(0, 1);
    if (mu == 0) {
        for (int a = 0; a < 2; ++a) g[a][a + 2] = g[a + 2][a] = -1.0;
    } else {
        C p[2][2];
        if (mu == 1) { p[0][0] = 0; p[0][1] = 1; p[1][0] = 1; p[1][1] = 0; }
        if (mu == 2) { p[0][0] = 0; p[0][1] = -I; p[1][0] = I; p[1][1] = 0; }
        if (mu == 3) { p[0][0] = 1; p[0][1] = 0; p[1][0] = 0; p[1][1] = -1.0; }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                g[a][b + 2] = -I * p[a][b];
                g[a + 2][b] = I * p[a][b];
            }
    }
    const double g5[4] = {1, 1, -1, -1};
    Spin4 G{};
    for (int s = 0; s < 4; ++s)
        for (int t = 0; t < 4; ++t) {
            const C v = g5[s] * g[s][t] * g5[t];
            G.re[4 * s + t] = v.real();
            G.im[4 * s + t] = v.imag();
        }
    return G;
}

// The same sources written straight into one internal FP64 right-hand side
// (the solver's layout), for the AMA driver.
__global__ void k_z2_internal(double2 *__restrict__ b, unsigned long long key, const int *__restrict__ lex_of,
                              long V, long index) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= V) return;
    const unsigned long long base = ((unsigned long long)index * V + lex_of[idx]) * 12;
#pragma unroll
    for (int sc = 0; sc < 12; ++sc)
        b[(size_t)sc * V + idx] = make_double2((sm64(key, base + sc) >> 63) ? -1.0 : 1.0, 0.0);
}

template <class CT>
__global__ void k_seq_internal(const CT *__restrict__ in, double2 *__restrict__ b, const int *__restrict__ lex_of,
                               long V, long spatial, int t_sink, Spin4 G) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= V) return;
    const long lex = lex_of[idx];
    const bool on = lex / spatial == t_sink;
    const CT *v = in + (size_t)lex * 12;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double ar = 0, ai = 0;
            if (on)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double vr = v[3 * t + c].x, vi = v[3 * t + c].y;
                    ar += G.re[4 * s + t] * vr - G.im[4 * s + t] * vi;
                    ai += G.re[4 * s + t] * vi + G.im[4 * s + t] * vr;
                }
            b[(size_t)(3 * s + c) * V + idx] = make_double2(ar, ai);
        }
}

int z2_source_internal(qcd_field f, unsigned long long seed, long long index, double2 *b, hipStream_t s) {
    const long V = f->g.V;
    k_z2_internal<<<nblocks(V, 256), 256, 0, s>>>(b, sm64(seed, 6ULL), f->lex_of, V, (long)index);
    DFL_HIP(hipGetLastError());
    return 0;
}

int seq_source_internal(qcd_field f, const void *fwd, qcd_prec io, int t_sink, int mu, double2 *b, hipStream_t s) {
    const long V = f->g.V, spatial = V / f->g.L[0];
    const Spin4 G = g5_gmu_g5(mu);
    if (io == QCD_F64)
        k_seq_internal<double2><<<nblocks(V, 256), 256, 0, s>>>(static_cast<const double2 *>(fwd), b, f->lex_of, V,
                                                                spatial, t_sink, G);
    else
        k_seq_internal<float2><<<nblocks(V, 256), 256, 0, s>>>(static_cast<const float2 *>(fwd), b, f->lex_of, V,
                                                               spatial, t_sink, G);
    DFL_HIP(hipGetLastError());
    return 0;
}

}  // namespace dfl

using namespace dfl;

extern "C" int make_z2_sources(qcd_field f, unsigned long long seed, long long index0, int n, void *out, qcd_prec io,
                               hipStream_t s) {
    if (!f || !out || n <= 0 || index0 < 0) return set_error(QCD_EINVAL, "bad arguments to make_z2_sources");
    const long V = f->g.V;
    const unsigned long long key = sm64(seed, 6ULL);   // stream 6: Z2 noise
    const dim3 grid(nblocks(V, 256), n);
    ProfScope ps(PROF_OTHER, s);
    if (io == QCD_F64)
        k_z2<double2><<<grid, 256, 0, s>>>(static_cast<double2 *>(out), key, V, (long)index0);
    else if (io == QCD_F32)
        k_z2<float2><<<grid, 256, 0, s>>>(static_cast<float2 *>(out), key, V, (long)index0);
    else
        return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    DFL_HIP(hipGetLastError());
    return 0;
}

extern "C" int make_sequential_sources(qcd_field f, const void *psi, void *eta, int n, qcd_prec io, int t_sink,
                                       int mu, hipStream_t s) {
    if (!f || !psi || !eta || n <= 0 || psi == eta) return set_error(QCD_EINVAL, "bad arguments to make_sequential_sources");
    if (mu < 0 || mu > 3) return set_error(QCD_EINVAL, "mu must be 0..3");
    if (t_sink < 0 || t_sink >= f->g.L[0]) return set_error(QCD_EINVAL, "sink timeslice outside the lattice");
    const long V = f->g.V, spatial = V / f->g.L[0];
    const Spin4 G = g5_gmu_g5(mu);
    const dim3 grid(nblocks(V, 256), n);
    ProfScope ps(PROF_OTHER, s);
    if (io == QCD_F64)
        k_seq<double2><<<grid, 256, 0, s>>>(static_cast<const double2 *>(psi), static_cast<double2 *>(eta), V, spatial,
                                            t_sink, G);
    else if (io == QCD_F32)
        k_seq<float2><<<grid, 256, 0, s>>>(static_cast<const float2 *>(psi), static_cast<float2 *>(eta), V, spatial,
                                           t_sink, G);
    else
        return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    DFL_HIP(hipGetLastError());
    return 0;
}
