// Nucleon correlators from the solver's propagators, and the all-mode-
// averaging combination of observables (the steps after the solve:
// section 2.3, eq. Nop; section 2.1, eqs. caa1-caa2).
//
// A point-source propagator is the 12 canonical solutions x_j = M^{-1}
// delta_{x0} e_j (j = 3 spin + colour): S(x)[s c][s' c'] = x_{3s'+c'}(x)[s c].
// With Gamma = C gamma_5 (C = gamma_0 gamma_2) and the conjugate field
// Nbar = eps (ubar (dbar Gamma ubar^T)), Wick's theorem gives per sink site
//   C_{al al'}(x) = eps_abc eps_a'b'c' [ U^{cc'}_{al al'} tr(Q^{bb'} U^{aa' T})
//                                        - (U^{ca'} Q^{bb' T} U^{ac'})_{al al'} ],
// Q^{bb'} = Gamma D^{bb'} Gamma, with U = D = S for degenerate flavours.
// Gamma has one nonzero entry per row: Gamma_{b, pi(b)} = g_b, so
// Q_{bb'} = g_b g_{pi^-1(b')} S_{pi(b), pi^-1(b')}.
//
// All arithmetic is FP64 (the correlator falls off exponentially in time and
// the covariance test compares it at the 1e-12 level); timeslice sums are
// reduced in a fixed order (per-workgroup partials, then one pass per
// timeslice), so results do not depend on the launch order.
#include <complex>

#include "blas.h"
#include "internal.h"

namespace dfl {

namespace {

using cd = cx<double>;

// spin matrix with one nonzero entry per row: M_{b, pi[b]} = g[b]
struct Mono4 {
    int pi[4], pinv[4];
    double gre[4], gim[4];
};
// general 4x4 complex spin matrix, row-major
struct Mat4 {
    double re[16], im[16];
};

__device__ inline cd mono_g(const Mono4 &G, int b) { return {G.gre[b], G.gim[b]}; }

template <class CT>
struct Prop {
    const CT *p;
    long V;
    unsigned long long x;
    // S[s c][s' c'] at this thread's site
    __device__ inline cd operator()(int s, int c, int sp, int cp) const {
        const CT v = p[((unsigned long long)(3 * sp + cp) * V + x) * 12 + 3 * s + c];
        return {(double)v.x, (double)v.y};
    }
};

// the two colours other than b with the sign of eps(first, b, second)
__device__ inline void others(int b, int &a, int &c) {
    a = (b + 1) % 3;
    c = (b + 2) % 3;   // eps(a, b, c) = eps(b+1, b, b+2) = -1
}

// sum of 2 * NV doubles over the workgroup (256 threads), into out (thread 0)
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double (*sh)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = sh[0][k] + sh[1][k] + sh[2][k] + sh[3][k];
}

// Two-point contraction: a workgroup takes SPW2 = 8 consecutive sites of
// timeslice blockIdx.y (chunk blockIdx.x), 16 threads per site.  The sites'
// propagators are staged in LDS (one 12 x 12 complex matrix per site,
// S[s c][s' c']), and the colour sums are factored:
//   T^{cc'}        = eps_abc eps_a'b'c' tr(Q^{bb'} S^{aa' T})         (9 per site)
//   Y^{ca'}_{r al'} = eps_abc eps_a'b'c' sum_s Q^{bb'}_{s r} S^{ac'}_{s al'}   (9 x 16)
//   C_{al al'}     = sum_cc' T^{cc'} S^{cc'}_{al al'} - sum_{c a' r} S^{ca'}_{al r} Y^{ca'}_{r al'}
// with Q^{bb'}_{s r} = g_s g_{q} S_{pi(s) b, q b'}, q = pi^-1(r).  Thread
// l = 0..15 of a site computes T^{cc'} (l < 9), then Y for (r, al') =
// (l / 4, l % 4), then C for (al, al') = (l / 4, l % 4).  The 16 sites'
// values are summed in a fixed order into part[t][chunk][16].  LDS: 40 KB
// per workgroup of 128 threads.
constexpr int SPW2 = 8;
// Q^{bb'}_{s r} = coef[4 s + r] S_{row[4 s + r] b, col[4 s + r] b'} (built on
// the host from Gamma; the unrolled loops read it from kernel arguments)
struct QMap {
    double re[16], im[16];
    int row[16], col[16];
};
template <class CT>
__global__ void __launch_bounds__(16 * SPW2) k_nucleon_2pt(const CT *__restrict__ prop, long V, long spatial,
                                                           QMap M, double2 *__restrict__ part) {
    __shared__ cd Sh[SPW2][144];
    __shared__ cd Th[SPW2][9];
    __shared__ cd Yh[SPW2][9][16];
    __shared__ cd Ch[SPW2][16];
    const long base = (long)blockIdx.x * SPW2;          // first spatial site of the workgroup
    const long x0 = (long)blockIdx.y * spatial + base;  // its lexicographic index
    const int nsite = (int)min((long)SPW2, spatial - base);
    // stage: for vector j the workgroup's sites are 12 nsite consecutive complex numbers
    for (int e = threadIdx.x; e < 12 * 12 * SPW2; e += 16 * SPW2) {
        const int j = e / (12 * SPW2), rem = e - j * 12 * SPW2;
        const int site = rem / 12, k = rem - site * 12;
        cd v = {0.0, 0.0};
        if (site < nsite) {
            const CT t = prop[((size_t)j * V + x0 + site) * 12 + k];
            v = {(double)t.x, (double)t.y};
        }
        Sh[site][k * 12 + j] = v;
    }
    __syncthreads();
    const int site = threadIdx.x >> 4, l = threadIdx.x & 15;
    const cd *S = Sh[site];
    // eps_abc for the two (a, b) of a given c: (c+1, c+2) -> +1, (c+2, c+1) -> -1
    if (l < 9) {
        const int c = l / 3, cp = l % 3;
        cd T = {0.0, 0.0};
#pragma unroll 1
        for (int o = 0; o < 4; ++o) {
            const int a = (o & 2) ? (c + 2) % 3 : (c + 1) % 3, b = (o & 2) ? (c + 1) % 3 : (c + 2) % 3;
            const int ap = (o & 1) ? (cp + 2) % 3 : (cp + 1) % 3, bp = (o & 1) ? (cp + 1) % 3 : (cp + 2) % 3;
            const cd *Sb = S + b * 12 + bp, *Sa = S + a * 12 + ap;
            cd tr = {0.0, 0.0};
#pragma unroll
            for (int sr = 0; sr < 16; ++sr) {
                const cd Q = cd{M.re[sr], M.im[sr]} * Sb[36 * M.row[sr] + 3 * M.col[sr]];
                tr = cmac(tr, Q, Sa[36 * (sr >> 2) + 3 * (sr & 3)]);
            }
            T = (o == 0 || o == 3) ? T + tr : T - tr;
        }
        Th[site][l] = T;
    }
    {
        const int r = l >> 2, alp = l & 3;
#pragma unroll 1
        for (int cap = 0; cap < 9; ++cap) {
            const int c = cap / 3, ap = cap - 3 * c;
            cd Y = {0.0, 0.0};
#pragma unroll 1
            for (int o = 0; o < 4; ++o) {
                const int a = (o & 2) ? (c + 2) % 3 : (c + 1) % 3, b = (o & 2) ? (c + 1) % 3 : (c + 2) % 3;
                // (b', c') with eps_a'b'c': (a'+1, a'+2) -> +1, (a'+2, a'+1) -> -1
                const int bp = (o & 1) ? (ap + 2) % 3 : (ap + 1) % 3, cp = (o & 1) ? (ap + 1) % 3 : (ap + 2) % 3;
                const cd *Sb = S + b * 12 + bp, *Sa = S + a * 12 + 3 * alp + cp;
                cd y = {0.0, 0.0};
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                    // Q_{s r} for this thread's r: one of the 16 map entries per s
                    const int sr = 4 * s4;
                    cd Q = {0.0, 0.0};
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr)
                        if (rr == r) Q = cd{M.re[sr + rr], M.im[sr + rr]} * Sb[36 * M.row[sr + rr] + 3 * M.col[sr + rr]];
                    y = cmac(y, Q, Sa[36 * s4]);
                }
                Y = (o == 0 || o == 3) ? Y + y : Y - y;
            }
            Yh[site][cap][l] = Y;
        }
    }
    __syncthreads();
    {
        const int al = l >> 2, alp = l & 3;
        const cd *Sl = S + 36 * al;
        cd C = {0.0, 0.0};
#pragma unroll 1
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int cp = 0; cp < 3; ++cp) C = cmac(C, Th[site][3 * c + cp], Sl[c * 12 + 3 * alp + cp]);
#pragma unroll 1
        for (int cap = 0; cap < 9; ++cap) {
            const int c = cap / 3, ap = cap - 3 * c;
#pragma unroll
            for (int r = 0; r < 4; ++r) C = C - Sl[c * 12 + 3 * r + ap] * Yh[site][cap][4 * r + alp];
        }
        Ch[site][l] = site < nsite ? C : cd{0.0, 0.0};
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        cd sum = {0.0, 0.0};
        for (int k = 0; k < SPW2; ++k) sum = sum + Ch[k][threadIdx.x];
        part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 16 + threadIdx.x] = make_double2(sum.re, sum.im);
    }
}

// corr[(t - t0) mod T][k] = sum over chunks of part[t][chunk][k], in order
__global__ void k_timeslice_reduce(const double2 *__restrict__ part, int nchunk, int T, int nk, int t0,
                                   double2 *__restrict__ corr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T * nk) return;
    const int t = i / nk, k = i - t * nk;
    double re = 0, im = 0;
    for (int c = 0; c < nchunk; ++c) {
        const double2 v = part[((size_t)t * nchunk + c) * nk + k];
        re += v.x;
        im += v.y;
    }
    corr[(size_t)(((t - t0) % T + T) % T) * nk + k] = make_double2(re, im);
}

// eps(i, j, k) for colours 0..2
__device__ inline double eps3(int i, int j, int k) {
    if (i == j || j == k || i == k) return 0.0;
    return j == (i + 1) % 3 ? 1.0 : -1.0;
}

// Sequential sources: eta_j(x)_i = g5_i conj(K(x)_{i j}) on timeslice t_sink,
// zero elsewhere, with K = d tr(P C(x)) / d S_f(x) (flavour d: one line; u:
// the two lines, four occurrences).  i = (spin g, colour e) at the sink,
// j = 3 h + e' at the source.  The 3 x 3 colour blocks K^{ee'} are computed
// each by its own thread, from the Wick terms in which the differentiated
// line carries the colours (e, e').  Threads cover the sink timeslice only,
// nine per site (the other timeslices are zeroed by a fill beforehand).
template <class CT>
__global__ void __launch_bounds__(128) k_nucleon_seq(const CT *__restrict__ prop, CT *__restrict__ eta, long V,
                                                     long spatial, int t_sink, Mono4 G, Mat4 P, int flavour) {
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= 9 * spatial) return;
    const long x = (long)t_sink * spatial + tid / 9;
    const int e = (int)(tid % 9) / 3, ep = (int)(tid % 3);
    const Prop<CT> S{prop, V, (unsigned long long)x};
    auto pm = [&](int i, int j) { return cd{P.re[4 * i + j], P.im[4 * i + j]}; };
    // tr(P S^{aa'}) = sum_{ij} P_{ji} S^{aa'}_{ij}
    auto trPU = [&](int a, int ap) {
        cd t = {0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) t = cmac(t, pm(j, i), S(i, a, j, ap));
        return t;
    };
    // Q^{bb'}_{gh} = (Gamma S^{bb'} Gamma)_{gh}
    auto make_q = [&](int b, int bp, cd Q[4][4]) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                const int q = G.pinv[sp];
                Q[s][sp] = (mono_g(G, s) * mono_g(G, q)) * S(G.pi[s], b, q, bp);
            }
    };
    {
            cd K[4][4];
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int h = 0; h < 4; ++h) K[g][h] = {0.0, 0.0};
            if (flavour == 1) {
                // d line with colours (b, b') = (e, e'):
                //   eps eps [ tr(P U^{cc'}) (G^T U^{aa'} G^T) - G^T U^{ac'} P U^{ca'} G^T ]
                for (int a = 0; a < 3; ++a)
                    for (int ap = 0; ap < 3; ++ap) {
                        const int c = 3 - e - a, cp = 3 - ep - ap;
                        const double sg = eps3(a, e, c) * eps3(ap, ep, cp);
                        if (sg == 0.0) continue;
                        const cd tp = trPU(c, cp);
#pragma unroll
                        for (int h = 0; h < 4; ++h) {
                            // column l = pi(h) of P U^{ca'}
                            const int l = G.pi[h];
                            cd pu[4];
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                cd t = {0.0, 0.0};
#pragma unroll
                                for (int k = 0; k < 4; ++k) t = cmac(t, pm(j, k), S(k, c, l, ap));
                                pu[j] = t;
                            }
#pragma unroll
                            for (int g = 0; g < 4; ++g) {
                                // (G^T M G^T)_{gh} = g_{pinv(g)} M_{pinv(g), pi(h)} g_h, with
                                // M = tr(P U^{cc'}) U^{aa'} - U^{ac'} P U^{ca'}
                                const int k = G.pinv[g];
                                cd y = {0.0, 0.0};
#pragma unroll
                                for (int j = 0; j < 4; ++j) y = cmac(y, S(k, a, j, cp), pu[j]);
                                const cd f = mono_g(G, k) * mono_g(G, h);
                                const cd v = tp * S(k, a, l, ap) - y;
                                K[g][h] = rmac(K[g][h], sg, f * v);
                            }
                        }
                    }
            } else {
                // u line with colours (e, e'), in each of its four places
                for (int b = 0; b < 3; ++b)
                    for (int bp = 0; bp < 3; ++bp) {
                        if (b == e || bp == ep) continue;
                        const int o = 3 - e - b, op = 3 - ep - bp;   // the remaining colours
                        cd Q[4][4];
                        make_q(b, bp, Q);
                        // term 1, U^{cc'} with (c, c') = (e, e'), (a, a') = (o, o'): P_{hg} tr(Q U^{oo' T})
                        const double s1 = eps3(o, b, e) * eps3(op, bp, ep);
                        cd tr = {0.0, 0.0};
#pragma unroll
                        for (int s = 0; s < 4; ++s)
#pragma unroll
                            for (int sp = 0; sp < 4; ++sp) tr = cmac(tr, Q[s][sp], S(s, o, sp, op));
                        // term 1, U^{aa'} with (a, a') = (e, e'), (c, c') = (o, o'): Q_{gh} tr(P U^{oo'})
                        const double s2 = eps3(e, b, o) * eps3(ep, bp, op);
                        // term 2, U^{ca'} with c = e, a' = e' (a = o, c' = o'):
                        //   -sum_{km} P_{kg} U^{oo'}_{mk} Q_{mh}
                        const double s3 = eps3(o, b, e) * eps3(ep, bp, op);
                        // term 2, U^{ac'} with a = e, c' = e' (c = o, a' = o'):
                        //   -sum_{km} P_{hk} U^{oo'}_{km} Q_{gm}
                        const double s4 = eps3(e, b, o) * eps3(op, bp, ep);
                        const cd tpo = trPU(o, op);
#pragma unroll
                        for (int g = 0; g < 4; ++g)
#pragma unroll
                            for (int h = 0; h < 4; ++h)
                                K[g][h] = K[g][h] + rmac(s1 * (pm(h, g) * tr), s2, Q[g][h] * tpo);
                        // term 2 terms as products: sum_{km} P_{kg} U_{mk} Q_{mh} = ((U P)^T Q)_{gh},
                        // sum_{km} P_{hk} U_{km} Q_{gm} = (Q (P U)^T)_{gh}, U = U^{oo'}
                        {
                            cd W[4][4];   // U P
#pragma unroll
                            for (int m = 0; m < 4; ++m)
#pragma unroll
                                for (int g = 0; g < 4; ++g) {
                                    cd t = {0.0, 0.0};
#pragma unroll
                                    for (int k = 0; k < 4; ++k) t = cmac(t, S(m, o, k, op), pm(k, g));
                                    W[m][g] = t;
                                }
#pragma unroll
                            for (int g = 0; g < 4; ++g)
#pragma unroll
                                for (int h = 0; h < 4; ++h) {
                                    cd t = {0.0, 0.0};
#pragma unroll
                                    for (int m = 0; m < 4; ++m) t = cmac(t, W[m][g], Q[m][h]);
                                    K[g][h] = rmac(K[g][h], -s3, t);
                                }
                        }
                        {
                            cd W[4][4];   // P U
#pragma unroll
                            for (int h = 0; h < 4; ++h)
#pragma unroll
                                for (int m = 0; m < 4; ++m) {
                                    cd t = {0.0, 0.0};
#pragma unroll
                                    for (int k = 0; k < 4; ++k) t = cmac(t, pm(h, k), S(k, o, m, op));
                                    W[h][m] = t;
                                }
#pragma unroll
                            for (int g = 0; g < 4; ++g)
#pragma unroll
                                for (int h = 0; h < 4; ++h) {
                                    cd t = {0.0, 0.0};
#pragma unroll
                                    for (int m = 0; m < 4; ++m) t = cmac(t, Q[g][m], W[h][m]);
                                    K[g][h] = rmac(K[g][h], -s4, t);
                                }
                        }
                    }
            }
            // eta_{3h+e'}(x)[g][e] = g5_g conj(K[g][h]); g5 = diag(1, 1, -1, -1)
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                CT *o = eta + ((size_t)(3 * h + ep) * V + x) * 12;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const double s5 = g < 2 ? 1.0 : -1.0;
                    o[3 * g + e].x = s5 * K[g][h].re;
                    o[3 * g + e].y = -s5 * K[g][h].im;
                }
            }
        }
}

// Three-point contraction: sum_j (g5 Sigma_j(y))^+ (Gamma_op x_j(y)) summed
// over the sites of timeslice blockIdx.y, chunk blockIdx.x; partials part[t][chunk]
template <class CT>
__global__ void __launch_bounds__(256) k_nucleon_3pt(const CT *__restrict__ seq, const CT *__restrict__ prop,
                                                     long V, long spatial, Mat4 Gop, double2 *__restrict__ part) {
    __shared__ double sh[4][2];
    const long loc = (long)blockIdx.x * 256 + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (loc < spatial) {
        const unsigned long long x = (unsigned long long)((long)blockIdx.y * spatial + loc);
        cd sum = {0.0, 0.0};
        for (int j = 0; j < 12; ++j) {
            const CT *sj = seq + ((size_t)j * V + x) * 12;
            const CT *pj = prop + ((size_t)j * V + x) * 12;
            cd p[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) p[k] = {(double)pj[k].x, (double)pj[k].y};
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    cd gp = {0.0, 0.0};
#pragma unroll
                    for (int t = 0; t < 4; ++t) gp = cmac(gp, cd{Gop.re[4 * s + t], Gop.im[4 * s + t]}, p[3 * t + c]);
                    const double s5 = s < 2 ? 1.0 : -1.0;
                    const cd sv = {s5 * (double)sj[3 * s + c].x, s5 * (double)sj[3 * s + c].y};
                    sum = cmacc(sum, sv, gp);
                }
        }
        acc[0] = sum.re;
        acc[1] = sum.im;
    }
    block_sum<2>(acc, sh);
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = make_double2(acc[0], acc[1]);
}

// O_AMA[k] = (1/n_org) sum_f (exact_f[f][k] - appx_f[f][k]) + (1/n_g) sum_g appx_g[g][k]
__global__ void k_ama_combine(const double2 *__restrict__ appx_g, int n_g, const double2 *__restrict__ exact_f,
                              const double2 *__restrict__ appx_f, int n_org, long len, double2 *__restrict__ out) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    double rr = 0, ri = 0, gr = 0, gi = 0;
    for (int f = 0; f < n_org; ++f) {
        const double2 e = exact_f[(size_t)f * len + k], a = appx_f[(size_t)f * len + k];
        rr += e.x - a.x;
        ri += e.y - a.y;
    }
    for (int g = 0; g < n_g; ++g) {
        const double2 a = appx_g[(size_t)g * len + k];
        gr += a.x;
        gi += a.y;
    }
    out[k] = make_double2((n_org ? rr / n_org : 0.0) + gr / n_g, (n_org ? ri / n_org : 0.0) + gi / n_g);
}

// Gamma = C gamma_5 with C = gamma_0 gamma_2 in the operator's chiral basis,
// as a spin matrix with one nonzero entry per row
Mono4 cg5_mono() {
    using C = std::complex<double>;
    const C I(0, 1);
    C g0[4][4] = {}, g2[4][4] = {};
    for (int a = 0; a < 2; ++a) g0[a][a + 2] = g0[a + 2][a] = -1.0;
    // gamma_2 = [[0, -i s2], [i s2, 0]], s2 = [[0, -i], [i, 0]]
    const C s2[2][2] = {{0.0, -I}, {I, 0.0}};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            g2[a][b + 2] = -I * s2[a][b];
            g2[a + 2][b] = I * s2[a][b];
        }
    const double g5[4] = {1, 1, -1, -1};
    Mono4 m{};
    for (int r = 0; r < 4; ++r)
        for (int k = 0; k < 4; ++k) {
            C v = 0;
            for (int j = 0; j < 4; ++j) v += g0[r][j] * g2[j][k];
            v *= g5[k];
            if (std::abs(v) > 0.5) {
                m.pi[r] = k;
                m.pinv[k] = r;
                m.gre[r] = v.real();
                m.gim[r] = v.imag();
            }
        }
    return m;
}

Mat4 mat4(const double *h) {
    Mat4 m{};
    for (int k = 0; k < 16; ++k) {
        m.re[k] = h[2 * k];
        m.im[k] = h[2 * k + 1];
    }
    return m;
}

int check_prop_args(qcd_field f, const void *a, const void *b, qcd_prec io) {
    if (!f || !a || !b) return set_error(QCD_EINVAL, "null argument to a nucleon contraction");
    if (io != QCD_F64 && io != QCD_F32) return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    return 0;
}

// per-chunk partial sums of a timeslice reduction, nk complex values each,
// chunks of `per` spatial sites
int partials(qcd_field f, int nk, unsigned &nchunk, double2 **part, long per = 256) {
    const long spatial = f->g.V / f->g.L[0];
    nchunk = nblocks(spatial, per);
    void *p;
    DFL_TRY(field_buffer(f, BUF_CONTRACT, sizeof(double2) * (size_t)f->g.L[0] * nchunk * nk, &p));
    *part = static_cast<double2 *>(p);
    return 0;
}

}  // namespace
}  // namespace dfl

using namespace dfl;

extern "C" int nucleon_2pt(qcd_field f, const void *prop, qcd_prec io, int t0, void *corr, hipStream_t s) {
    DFL_TRY(check_prop_args(f, prop, corr, io));
    const int T = f->g.L[0];
    if (t0 < 0 || t0 >= T) return set_error(QCD_EINVAL, "source timeslice outside the lattice");
    const long V = f->g.V, spatial = V / T;
    unsigned nchunk;
    double2 *part;
    DFL_TRY(partials(f, 16, nchunk, &part, SPW2));
    const Mono4 G = cg5_mono();
    QMap QM;
    for (int s4 = 0; s4 < 4; ++s4)
        for (int r = 0; r < 4; ++r) {
            const int q = G.pinv[r];
            const std::complex<double> g = std::complex<double>(G.gre[s4], G.gim[s4]) *
                                           std::complex<double>(G.gre[q], G.gim[q]);
            QM.re[4 * s4 + r] = g.real();
            QM.im[4 * s4 + r] = g.imag();
            QM.row[4 * s4 + r] = G.pi[s4];
            QM.col[4 * s4 + r] = q;
        }
    {
        ProfScope ps(PROF_OTHER, s);
        const dim3 grid(nchunk, T);
        if (io == QCD_F64)
            k_nucleon_2pt<double2><<<grid, 16 * SPW2, 0, s>>>(static_cast<const double2 *>(prop), V, spatial, QM,
                                                               part);
        else
            k_nucleon_2pt<float2><<<grid, 16 * SPW2, 0, s>>>(static_cast<const float2 *>(prop), V, spatial, QM,
                                                              part);
        DFL_HIP(hipGetLastError());
        k_timeslice_reduce<<<nblocks(16L * T, 64), 64, 0, s>>>(part, nchunk, T, 16, t0, static_cast<double2 *>(corr));
        DFL_HIP(hipGetLastError());
    }
    return 0;
}

extern "C" int nucleon_seq_sources(qcd_field f, const void *prop, qcd_prec io, int t_sink, const double *proj,
                                   int flavour, void *eta, hipStream_t s) {
    DFL_TRY(check_prop_args(f, prop, eta, io));
    if (!proj) return set_error(QCD_EINVAL, "null projector");
    if (prop == eta) return set_error(QCD_EINVAL, "propagator and sequential sources must not overlap");
    if (flavour != 0 && flavour != 1) return set_error(QCD_EINVAL, "flavour must be 0 (u) or 1 (d)");
    if (t_sink < 0 || t_sink >= f->g.L[0]) return set_error(QCD_EINVAL, "sink timeslice outside the lattice");
    const long V = f->g.V, spatial = V / f->g.L[0];
    const Mono4 G = cg5_mono();
    const Mat4 P = mat4(proj);
    ProfScope ps(PROF_OTHER, s);
    // zero everywhere (a coalesced fill: 12 vectors x V sites x 12 complex),
    // then the sink timeslice
    const size_t bytes = (size_t)12 * V * 12 * (io == QCD_F64 ? 16 : 8);
    DFL_TRY(blas_zero<double2>(static_cast<double2 *>(eta), (long)(bytes / 16), 1, s));
    if (io == QCD_F64)
        k_nucleon_seq<double2><<<nblocks(9 * spatial, 128), 128, 0, s>>>(static_cast<const double2 *>(prop),
                                                                         static_cast<double2 *>(eta), V, spatial,
                                                                         t_sink, G, P, flavour);
    else
        k_nucleon_seq<float2><<<nblocks(9 * spatial, 128), 128, 0, s>>>(static_cast<const float2 *>(prop),
                                                                        static_cast<float2 *>(eta), V, spatial,
                                                                        t_sink, G, P, flavour);
    DFL_HIP(hipGetLastError());
    return 0;
}

extern "C" int nucleon_3pt(qcd_field f, const void *seqprop, const void *prop, qcd_prec io, int t0,
                           const double *gamma_op, void *corr, hipStream_t s) {
    DFL_TRY(check_prop_args(f, seqprop, prop, io));
    if (!gamma_op || !corr) return set_error(QCD_EINVAL, "null argument to nucleon_3pt");
    const int T = f->g.L[0];
    if (t0 < 0 || t0 >= T) return set_error(QCD_EINVAL, "source timeslice outside the lattice");
    const long V = f->g.V, spatial = V / T;
    unsigned nchunk;
    double2 *part;
    DFL_TRY(partials(f, 1, nchunk, &part));
    const Mat4 Gop = mat4(gamma_op);
    ProfScope ps(PROF_OTHER, s);
    const dim3 grid(nchunk, T);
    if (io == QCD_F64)
        k_nucleon_3pt<double2><<<grid, 256, 0, s>>>(static_cast<const double2 *>(seqprop),
                                                    static_cast<const double2 *>(prop), V, spatial, Gop, part);
    else
        k_nucleon_3pt<float2><<<grid, 256, 0, s>>>(static_cast<const float2 *>(seqprop),
                                                   static_cast<const float2 *>(prop), V, spatial, Gop, part);
    DFL_HIP(hipGetLastError());
    k_timeslice_reduce<<<nblocks(T, 64), 64, 0, s>>>(part, nchunk, T, 1, t0, static_cast<double2 *>(corr));
    DFL_HIP(hipGetLastError());
    return 0;
}

extern "C" int ama_combine(long long len, int n_g, const void *appx_g, int n_org, const void *exact_f,
                           const void *appx_f, void *out, hipStream_t s) {
    if (len < 1 || n_g < 1 || n_org < 0 || !appx_g || !out || (n_org > 0 && (!exact_f || !appx_f)))
        return set_error(QCD_EINVAL, "bad arguments to ama_combine");
    k_ama_combine<<<nblocks((long)len, 256), 256, 0, s>>>(static_cast<const double2 *>(appx_g), n_g,
                                                          static_cast<const double2 *>(exact_f),
                                                          static_cast<const double2 *>(appx_f), n_org, (long)len,
                                                          static_cast<double2 *>(out));
    DFL_HIP(hipGetLastError());
    return 0;
}
