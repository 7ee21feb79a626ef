// Schwarz alternating procedure (SAP) on the block checkerboard.
//
// One launch = one colour sweep: every workgroup owns one Schwarz block of
// that colour and one right-hand side.  It forms the block residual
// rho = eta - M psi, solves the Dirichlet block equation approximately with
// nmr minimal-residual steps on the even-odd reduced block operator
//     Dhat = A_ee - kappa^2 H_eo A_oo^{-1} H_oe
// and adds the correction to psi.  Thread t owns the even site j = t and the
// odd site j = t of the block (and j = t + NT when KS = 2).  The two
// exchange vectors of the MinRes iteration (r on even sites, t = A_oo^{-1}
// H_oe r on odd sites) live in LDS when they fit, else in a per-workgroup
// global buffer; everything else stays in registers.
//
// The block residual is kept up to date instead of recomputed.  After a
// block's update its residual equals the final minimal-residual vector on
// the block's even sites, and rho_o + kappa H_oe x_e - A_oo delta_o on its
// odd sites (zero when the stored inverse clover is the exact inverse of the
// stored clover; at FP16 storage it is not); both are stored (`res`).  Within
// a sweep the block's rho_o waits in its own odd sites of `res` while the
// MinRes steps use the LDS; the back substitution then forms
// u_o = rho_o + kappa H_oe x_e, delta_o = A_oo^{-1} u_o and the odd residual
// from it, so s_o = A_oo^{-1} rho_o (needed for rhat_e) is never stored.
// Until the block is visited again only the blocks of the other colour
// change, by their corrections delta, and they enter the block's residual
// only through the hops that cross its faces:
//     rho_block = res_block + kappa H_{block <- neighbours} delta.
// Each sweep but the last hands those hops over ready-made: a block ends by
// writing, for every face site of its neighbours, the link times the spin
// projection of its delta (a half-spinor), in the order of the neighbour's
// face table, so the neighbour's next sweep reads them contiguously.
// The stored residuals and the half-spinors take the sweep's own storage
// type SI (the arithmetic type, or FP16 with a power-of-two scale per site);
// eta and psi keep the arithmetic type.
// The first cycle starts from rho = eta (psi = 0).  The face hops of a block
// are listed per direction mu (block-face table, the same for every block):
// all threads of the workgroup take one direction per round, so no two of
// them touch the same site in a round and no lane waits on another's branch.
#include "internal.h"

namespace dfl {

// sum over aligned groups of G lanes (G = 64: the whole wave)
template <int G = 64, class R>
__device__ inline R wave_sum(R v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// acc = sum over hops that stay inside the block (Dirichlet boundary) of the
// hopping term applied to the exchange buffer buf (opposite-parity sites of
// the block, local index).  Site: local index j of parity ODD in the block at
// offset boff.  The in-block neighbours come from the block-shape table
// lnbr (identical for every block); hops inside a block never cross the
// lattice boundary, so no boundary sign enters.
template <class R, int LF, bool ODD>
__device__ inline void block_hop(const void *U, const short *lnbr, long V, long Vh, long boff, int j, int Vbh,
                                 const cx<R> *buf, cx<R> acc[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
    cx<R> w[9], p[12];
    const uint4 nb4 = ld<uint4>(lnbr, 0, 0, (unsigned)((ODD ? Vbh : 0) + j));
    const unsigned nbw[4] = {nb4.x, nb4.y, nb4.z, nb4.w};
    const unsigned x = (unsigned)((ODD ? Vh : 0) + boff + j);
    const unsigned yoff = (unsigned)((ODD ? 0 : Vh) + boff);
#define DFL_BHOP(MU)                                                                    \
    {                                                                                   \
        const int lf = (short)(nbw[MU] & 0xffffu);                                      \
        const int lb = (short)(nbw[MU] >> 16);                                          \
        if (lf >= 0) {                                                                  \
            Link<LF>::load(U, V, MU, x, w);                                             \
            _Pragma("unroll") for (int k = 0; k < 12; ++k) p[k] = buf[k * Vbh + lf];    \
            hop<R, MU, true>(w, p, R(1), acc);                                          \
        }                                                                               \
        if (lb >= 0) {                                                                  \
            Link<LF>::load(U, V, MU, yoff + (unsigned)lb, w);                           \
            _Pragma("unroll") for (int k = 0; k < 12; ++k) p[k] = buf[k * Vbh + lb];    \
            hop<R, MU, false>(w, p, R(1), acc);                                         \
        }                                                                               \
    }
    DFL_BHOP(0)
    DFL_BHOP(1)
    DFL_BHOP(2)
    DFL_BHOP(3)
#undef DFL_BHOP
}

// Storage of the sweep's own vectors: the block residuals (with the parked
// rho_o) as full spinors, and the face exchange as half-spinors (the spin
// projection times the link: two colour vectors, 6 complex).  Each type is a
// structure-of-arrays per right-hand side, and q is the right-hand side's
// place in the workgroup's pair (its data follow those of the first), so the
// base stays the same in every lane.  FP16 keeps a power-of-two scale per
// site (per face entry), after the 16-byte (8-byte) chunks.
template <class SI>
struct VecI;
template <>
struct VecI<double> {
    static constexpr size_t BYTES = 192;
    template <class R>
    __device__ static inline void load(const void *b, long V, unsigned i, int q, cx<R> v[12]) {
        Spin<double>::load(b, V, i + (unsigned)(q * 12 * V), v);
    }
    template <class R>
    __device__ static inline void store(void *b, long V, unsigned i, int q, const cx<R> v[12]) {
        Spin<double>::store(b, V, i + (unsigned)(q * 12 * V), v);
    }
};
template <>
struct VecI<float> {
    static constexpr size_t BYTES = 96;
    template <class R>
    __device__ static inline void load(const void *b, long V, unsigned i, int q, cx<R> v[12]) {
        Spin<float>::load(b, V, i + (unsigned)(q * 6 * V), v);
    }
    template <class R>
    __device__ static inline void store(void *b, long V, unsigned i, int q, const cx<R> v[12]) {
        Spin<float>::store(b, V, i + (unsigned)(q * 6 * V), v);
    }
};
// 52 V bytes per right-hand side: V is a multiple of 16, so the second one
// starts at a whole number of 16-byte (13 V / 4) and 4-byte (13 V) units
template <>
struct VecI<__half> {
    static constexpr size_t BYTES = 52;
    template <class R>
    __device__ static inline void load(const void *b, long V, unsigned i, int q, cx<R> v[12]) {
        h8 t[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) t[c] = ld<h8>(b, c, V, i + (unsigned)(q * 13 * V / 4));
        Spin<__half>::decode(t, ld<float>(b, 12, V, i + (unsigned)(q * 13 * V)), v);
    }
    template <class R>
    __device__ static inline void store(void *b, long V, unsigned i, int q, const cx<R> v[12]) {
        h8 t[3];
        float sc;
        Spin<__half>::encode(v, t, sc);
#pragma unroll
        for (int c = 0; c < 3; ++c) st<h8>(b, c, V, i + (unsigned)(q * 13 * V / 4), t[c]);
        st<float>(b, 12, V, i + (unsigned)(q * 13 * V), sc);
    }
};

template <class SI>
struct HalfI;
template <>
struct HalfI<double> {
    static constexpr size_t BYTES = 96;
    template <class R>
    __device__ static inline void load(const void *base, long n, unsigned idx, int q, cx<R> v[6]) {
        idx += (unsigned)(q * 6 * n);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double2 t = ld<double2>(base, k, n, idx);
            v[k] = {R(t.x), R(t.y)};
        }
    }
    template <class R>
    __device__ static inline void store(void *base, long n, unsigned idx, int q, const cx<R> v[6]) {
        idx += (unsigned)(q * 6 * n);
#pragma unroll
        for (int k = 0; k < 6; ++k) st<double2>(base, k, n, idx, make_double2(double(v[k].re), double(v[k].im)));
    }
};
template <>
struct HalfI<float> {
    static constexpr size_t BYTES = 48;
    template <class R>
    __device__ static inline void load(const void *base, long n, unsigned idx, int q, cx<R> v[6]) {
        idx += (unsigned)(q * 3 * n);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float4 t = ld<float4>(base, c, n, idx);
            v[2 * c] = {R(t.x), R(t.y)};
            v[2 * c + 1] = {R(t.z), R(t.w)};
        }
    }
    template <class R>
    __device__ static inline void store(void *base, long n, unsigned idx, int q, const cx<R> v[6]) {
        idx += (unsigned)(q * 3 * n);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            st<float4>(base, c, n, idx,
                       make_float4(float(v[2 * c].re), float(v[2 * c].im), float(v[2 * c + 1].re),
                                   float(v[2 * c + 1].im)));
    }
};
// 28 n bytes per right-hand side (3 chunks of 8 bytes, then the scales); n is
// even, so the second one starts at 7 n / 2 eight-byte and 7 n four-byte units
template <>
struct HalfI<__half> {
    static constexpr size_t BYTES = 28;
    template <class R>
    __device__ static inline void load(const void *base, long n, unsigned idx, int q, cx<R> v[6]) {
        const float sc = ld<float>(base, 6, n, idx + (unsigned)(q * 7 * n));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const h4 t = ld<h4>(base, c, n, idx + (unsigned)(q * 7 * n / 2));
            v[2 * c] = {R(__half2float(t.v[0]) * sc), R(__half2float(t.v[1]) * sc)};
            v[2 * c + 1] = {R(__half2float(t.v[2]) * sc), R(__half2float(t.v[3]) * sc)};
        }
    }
    template <class R>
    __device__ static inline void store(void *base, long n, unsigned idx, int q, const cx<R> v[6]) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) m = fmaxf(m, fmaxf(fabsf(float(v[k].re)), fabsf(float(v[k].im))));
        float sc, inv;
        r16_scale(m, sc, inv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            h4 t;
            t.v[0] = __float2half_rn(float(v[2 * c].re) * inv);
            t.v[1] = __float2half_rn(float(v[2 * c].im) * inv);
            t.v[2] = __float2half_rn(float(v[2 * c + 1].re) * inv);
            t.v[3] = __float2half_rn(float(v[2 * c + 1].im) * inv);
            st<h4>(base, c, n, idx + (unsigned)(q * 7 * n / 2), t);
        }
        st<float>(base, 6, n, idx + (unsigned)(q * 7 * n), sc);
    }
};

// Face exchange.  Entry k of direction MU of block B's face table (site x of
// B, forward (d = 0) or backward (d = 1) face) receives the hop from the site
// y = x +- mu of the neighbouring block N that swept last:
//     d = 0: sign U_mu(x) (1 - gamma_mu) delta(y),
//     d = 1: sign U_mu(y)^+ (1 + gamma_mu) delta(y),
// as a half-spinor (the spin projection times the link).  N writes it at
// the end of its sweep into slot (B, MU, k) of the exchange buffer (face_emit),
// so that B's next sweep reads its face entries in table order, contiguous,
// and only rebuilds the four spin components and scales by kappa
// (face_absorb).  Slots: [rhs][chunk][block][sum of the face table lengths],
// direction MU at offset fo (the lengths before it).
template <class SI, class R, int MU>
__device__ inline void face_absorb(const int *bface, int fcap, int nf, int fo, int nft, int tid, int NT,
                                   const void *fx, int qr, long nfx, long B, int Vbh, R kappa, cx<R> *Rb,
                                   cx<R> *Tb) {
    for (int k = tid; k < nf; k += NT) {
        const int ent = bface[MU * fcap + k];
        const int par = ent >> 30, bwd = (ent >> 29) & 1, j = ent & 0x1fffffff;
        cx<R> g[6], a[12];
        HalfI<SI>::load(fx, nfx, (unsigned)(B * nft + fo + k), qr, g);
        cx<R> *buf = par ? Tb : Rb;
#pragma unroll
        for (int c = 0; c < 12; ++c) a[c] = buf[c * Vbh + j];
        if (!bwd)
            reconstruct_add<R, MU, -1>(g, kappa, a);
        else
            reconstruct_add<R, MU, +1>(g, kappa, a);
#pragma unroll
        for (int c = 0; c < 12; ++c) buf[c * Vbh + j] = a[c];
    }
}

// The hops of this block's correction (delta_e in De, delta_o in Do, local
// index) into the face entries of its neighbours, for direction MU.
template <class SI, class R, int LF, int MU>
__device__ inline void face_emit(const int *bface, const int *bfsrc, const int *bfnb, int fcap, int nf, int fo,
                                 int nft, int tid, int NT, const void *U, void *fx, int qr, long nfx, long V,
                                 long Vh, long B, int Vbh, const cx<R> *De, const cx<R> *Do) {
    for (int k = tid; k < nf; k += NT) {
        const int ent = bface[MU * fcap + k], src = bfsrc[MU * fcap + k];
        const int par = ent >> 30, bwd = (ent >> 29) & 1, j = ent & 0x1fffffff;
        const int py = src >> 30, jy = src & 0x3fffffff;
        const int nb = bfnb[B * 8 + 2 * MU + bwd];
        const long Rblk = nb & 0x7fffffff;
        const cx<R> *buf = py ? Do : De;
        cx<R> d[12], h[6], g[6], w[9];
#pragma unroll
        for (int c = 0; c < 12; ++c) d[c] = buf[c * Vbh + jy];
        if (!bwd) {
            Link<LF>::load(U, V, MU, (unsigned)(par * Vh + Rblk * Vbh + j), w);
            project<R, MU, -1>(d, h);
            su3_mul2<R, false>(w, h, g);
        } else {
            Link<LF>::load(U, V, MU, (unsigned)(py * Vh + B * Vbh + jy), w);
            project<R, MU, +1>(d, h);
            su3_mul2<R, true>(w, h, g);
        }
        if (nb < 0) {
#pragma unroll
            for (int c = 0; c < 6; ++c) g[c] = {-g[c].re, -g[c].im};
        }
        HalfI<SI>::store(fx, nfx, (unsigned)(Rblk * nft + fo + k), qr, g);
    }
}

enum SweepFlags { SW_FIRST = 1, SW_FACES = 2, SW_STORE_RES = 4, SW_EMIT = 8 };

// VBHC > 0: the block's sites per parity as a compile-time constant (the
// component planes of the exchange buffers then sit at immediate LDS
// offsets); 0: taken from the argument.
// NR = 2 (FP32 vectors in LDS, KS = 1): a workgroup takes two right-hand
// sides of its block, each wave 64 / NR sites for both, so the two lanes of
// a site read the same links and clover entries in one instruction.  Every
// thread still does one site pair of one right-hand side; the vector bases
// stay wave-uniform and a lane's right-hand side enters through its element
// index (qr x NCH x V chunks further).
template <class S, class R, int LF, int CF, bool LDS, int KS, int MAXT, int VBHC = 0, int NR = 1, class SI = S>
__global__ void __launch_bounds__(MAXT, (sizeof(R) == 4 && LF >= LNK_F16 && LDS && MAXT == 256 && VBHC > 0) ? 3 : 1)
    k_sap_sweep(const void *__restrict__ eta_all, void *__restrict__ psi_all, void *__restrict__ res_all,
                void *__restrict__ fx_all, const void *__restrict__ U, const void *__restrict__ clo,
                const void *__restrict__ cinv, const short *__restrict__ lnbr, const int *__restrict__ bface,
                const int *__restrict__ bfsrc, const int *__restrict__ bfnb, int fcap, int4 nface, long V, long Vh,
                int Vbh_arg, int nbc, int colour, R kappa, int nmr, int flags, cx<R> *gbuf) {
    // flags: SW_FIRST: first cycle (rho starts from eta, psi is zero on this
    // colour); SW_FACES: add the neighbours' hops across the faces;
    // SW_STORE_RES: keep the block residual; SW_EMIT: write this block's hops
    // into the neighbours' face entries
    static_assert(NR == 1 || (LDS && KS == 1 && Spin<S>::NCH * 16 == Spin<S>::BYTES), "NR = 2 layout");
    constexpr int SPW = 64 / NR;   // sites per wave
    const int Vbh = VBHC > 0 ? VBHC : Vbh_arg;
    extern __shared__ unsigned char dsm[];
    __shared__ R red[16][NR][3];
    const int lane = threadIdx.x & 63, qr = NR > 1 ? lane / SPW : 0;   // this lane's right-hand side
    const int NT = blockDim.x / NR;                                       // sites per sweep of the workgroup
    const int tid = NR > 1 ? (int)(threadIdx.x >> 6) * SPW + (lane - qr * SPW) : (int)threadIdx.x;
    unsigned bx, rg;
    xcd_order(bx, rg);
    const unsigned rhs = rg * NR + qr;
    const size_t fs = (size_t)Spin<S>::BYTES * V;
    const void *eta = wave_uniform(static_cast<const char *>(eta_all) + (size_t)rg * NR * fs);
    void *psi = wave_uniform(static_cast<char *>(psi_all) + (size_t)rg * NR * fs);
    void *res = wave_uniform(static_cast<char *>(res_all) + (size_t)rg * NR * VecI<SI>::BYTES * V);
    const unsigned qoff = (unsigned)(qr * Spin<S>::NCH * V);    // its offset, in chunks
    // face exchange: nft entries per block, nfx per chunk plane
    const int fo1 = nface.x, fo2 = fo1 + nface.y, fo3 = fo2 + nface.z, nft = fo3 + nface.w;
    const long nfx = (long)nbc * 2 * nft;
    void *fx = wave_uniform(static_cast<char *>(fx_all) + (size_t)rg * NR * HalfI<SI>::BYTES * nfx);
    const bool first = flags & SW_FIRST;
    const long B = (long)colour * nbc + bx;
    const long boff = B * Vbh;
    cx<R> *Rb, *Tb;
    if (LDS) {
        Rb = reinterpret_cast<cx<R> *>(dsm) + (size_t)qr * 24 * Vbh;
    } else {
        Rb = gbuf + ((size_t)rhs * gridDim.x + bx) * (size_t)24 * Vbh;
    }
    Tb = Rb + 12 * Vbh;

    cx<R> xe[KS][12];
    // ---- block residual: eta (first cycle) or the stored residual, then the
    //      neighbours' corrections across the faces ----
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int j = tid + k * NT;
        if (j < Vbh) {
            const long xe_i = boff + j, xo_i = Vh + boff + j;
            cx<R> e[12];
            if (first)
                Spin<S>::load(eta, V, xe_i + qoff, e);
            else
                VecI<SI>::load(res, V, xe_i, qr, e);
#pragma unroll
            for (int c = 0; c < 12; ++c) Rb[c * Vbh + j] = e[c];
            if (first)
                Spin<S>::load(eta, V, xo_i + qoff, e);
            else
                VecI<SI>::load(res, V, xo_i, qr, e);
#pragma unroll
            for (int c = 0; c < 12; ++c) Tb[c * Vbh + j] = e[c];
        }
    }
    if (flags & SW_FACES) {
        __syncthreads();
        face_absorb<SI, R, 0>(bface, fcap, nface.x, 0, nft, tid, NT, fx, qr, nfx, B, Vbh, kappa, Rb, Tb);
        __syncthreads();
        face_absorb<SI, R, 1>(bface, fcap, nface.y, fo1, nft, tid, NT, fx, qr, nfx, B, Vbh, kappa, Rb, Tb);
        __syncthreads();
        face_absorb<SI, R, 2>(bface, fcap, nface.z, fo2, nft, tid, NT, fx, qr, nfx, B, Vbh, kappa, Rb, Tb);
        __syncthreads();
        face_absorb<SI, R, 3>(bface, fcap, nface.w, fo3, nft, tid, NT, fx, qr, nfx, B, Vbh, kappa, Rb, Tb);
        __syncthreads();
    }
    // ---- s_o = A_oo^{-1} rho_o into T; rho_o is parked in the residual
    //      buffer for the back substitution (this block's odd sites only) ----
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int j = tid + k * NT;
        if (j < Vbh) {
            cx<R> e[12], m[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) e[c] = Tb[c * Vbh + j];
            VecI<SI>::store(res, V, Vh + boff + j, qr, e);
            clover_apply<CF>(cinv, Vh, boff + j, e, m);
#pragma unroll
            for (int c = 0; c < 12; ++c) Tb[c * Vbh + j] = m[c];
        }
    }
    __syncthreads();
    // ---- r = rhat_e = rho_e + kappa H_eo s_o ; x_e = 0 ----
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int j = tid + k * NT;
        if (j < Vbh) {
            cx<R> acc[12];
            block_hop<R, LF, false>(U, lnbr, V, Vh, boff, j, Vbh, Tb, acc);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                Rb[c * Vbh + j] = rmac(Rb[c * Vbh + j], kappa, acc[c]);
                xe[k][c] = {R(0), R(0)};
            }
        }
    }
    __syncthreads();
    const R k2 = kappa * kappa;
    for (int it = 0; it < nmr; ++it) {
        // t_o = A_oo^{-1} H_oe r
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int j = tid + k * NT;
            if (j < Vbh) {
                cx<R> acc[12], t[12];
                block_hop<R, LF, true>(U, lnbr, V, Vh, boff, j, Vbh, Rb, acc);
                clover_apply<CF>(cinv, Vh, boff + j, acc, t);
#pragma unroll
                for (int c = 0; c < 12; ++c) Tb[c * Vbh + j] = t[c];
            }
        }
        __syncthreads();
        // p = A_ee r - kappa^2 H_eo t ; alpha = (p, r) / (p, p)
        cx<R> p[KS][12];
        R pr_re = 0, pr_im = 0, pp = 0;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int j = tid + k * NT;
            if (j < Vbh) {
                cx<R> acc[12], r[12];
#pragma unroll
                for (int c = 0; c < 12; ++c) r[c] = Rb[c * Vbh + j];
                clover_apply<CF>(clo, V, boff + j, r, p[k]);
                block_hop<R, LF, false>(U, lnbr, V, Vh, boff, j, Vbh, Tb, acc);
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    p[k][c] = rmac(p[k][c], -k2, acc[c]);
                    const cx<R> rc = r[c];
                    // (p, r) = sum conj(p) r and (p, p)
                    pr_re = ffma(p[k][c].im, rc.im, ffma(p[k][c].re, rc.re, pr_re));
                    pr_im = ffma(-p[k][c].im, rc.re, ffma(p[k][c].re, rc.im, pr_im));
                    pp = ffma(p[k][c].im, p[k][c].im, ffma(p[k][c].re, p[k][c].re, pp));
                }
            }
        }
        pr_re = wave_sum<SPW>(pr_re);
        pr_im = wave_sum<SPW>(pr_im);
        pp = wave_sum<SPW>(pp);
        if (lane == qr * SPW) {
            red[threadIdx.x >> 6][qr][0] = pr_re;
            red[threadIdx.x >> 6][qr][1] = pr_im;
            red[threadIdx.x >> 6][qr][2] = pp;
        }
        __syncthreads();
        R s0 = 0, s1 = 0, s2 = 0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) {
            s0 += red[w][qr][0];
            s1 += red[w][qr][1];
            s2 += red[w][qr][2];
        }
        const cx<R> alpha = s2 > R(0) ? cx<R>{s0 / s2, s1 / s2} : cx<R>{R(0), R(0)};
        const bool last = it + 1 == nmr;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int j = tid + k * NT;
            if (j < Vbh) {
                if (last && (flags & SW_STORE_RES)) {
                    // the block's residual after the update: the new r on even sites
                    cx<R> rn[12];
#pragma unroll
                    for (int c = 0; c < 12; ++c) rn[c] = cmac(Rb[c * Vbh + j], -alpha, p[k][c]);
                    VecI<SI>::store(res, V, boff + j, qr, rn);
                }
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const cx<R> rc = Rb[c * Vbh + j];
                    xe[k][c] = cmac(xe[k][c], alpha, rc);
                    Rb[c * Vbh + j] = last ? xe[k][c] : cmac(rc, -alpha, p[k][c]);
                }
            }
        }
        __syncthreads();
    }
    if (nmr == 0) {
        // x_e = 0: the residual is rhat_e; publish x_e for the back substitution
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int j = tid + k * NT;
            if (j < Vbh) {
                cx<R> rn[12];
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    rn[c] = Rb[c * Vbh + j];
                    Rb[c * Vbh + j] = {R(0), R(0)};
                }
                if (flags & SW_STORE_RES) VecI<SI>::store(res, V, boff + j, qr, rn);
            }
        }
        __syncthreads();
    }
    // ---- u_o = rho_o + kappa H_oe x_e, delta_o = A_oo^{-1} u_o, delta_e = x_e;
    //      psi += delta ----
    // (the neighbour blocks' corrections were read before the barriers above,
    //  and no other workgroup of this colour touches this block)
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int j = tid + k * NT;
        if (j < Vbh) {
            const long xe_i = boff + j, xo_i = Vh + boff + j;
            cx<R> acc[12], t[12], q[12];
            block_hop<R, LF, true>(U, lnbr, V, Vh, boff, j, Vbh, Rb, acc);
            VecI<SI>::load(res, V, xo_i, qr, t);
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[c] = rmac(t[c], kappa, acc[c]);   // u_o
            clover_apply<CF>(cinv, Vh, boff + j, acc, q);                       // delta_o
            if (flags & SW_EMIT) {
                // delta_o for the face exchange (T is free: only R = x_e is read here)
#pragma unroll
                for (int c = 0; c < 12; ++c) Tb[c * Vbh + j] = q[c];
            }
            if (flags & SW_STORE_RES) {
                // odd residual u_o - A_oo delta_o: zero up to rounding when the
                // stored inverse is exact, the stored inverse's defect otherwise
                clover_apply<CF>(clo, V, xo_i, q, t);
#pragma unroll
                for (int c = 0; c < 12; ++c) t[c] = acc[c] - t[c];
                VecI<SI>::store(res, V, xo_i, qr, t);
            }
            // both halves of psi are loaded before either is stored, so that
            // their latencies overlap
            cx<R> po[12], pe[12];
            if (!first) {
                Spin<S>::load(psi, V, xo_i + qoff, po);
                Spin<S>::load(psi, V, xe_i + qoff, pe);
            }
            if (first) {
                Spin<S>::store(psi, V, xo_i + qoff, q);
                Spin<S>::store(psi, V, xe_i + qoff, xe[k]);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    po[c] = q[c] + po[c];
                    pe[c] = pe[c] + xe[k][c];
                }
                Spin<S>::store(psi, V, xo_i + qoff, po);
                Spin<S>::store(psi, V, xe_i + qoff, pe);
            }
        }
    }
    if (flags & SW_EMIT) {
        __syncthreads();
        face_emit<SI, R, LF, 0>(bface, bfsrc, bfnb, fcap, nface.x, 0, nft, tid, NT, U, fx, qr, nfx, V, Vh, B, Vbh, Rb,
                               Tb);
        face_emit<SI, R, LF, 1>(bface, bfsrc, bfnb, fcap, nface.y, fo1, nft, tid, NT, U, fx, qr, nfx, V, Vh, B, Vbh,
                               Rb, Tb);
        face_emit<SI, R, LF, 2>(bface, bfsrc, bfnb, fcap, nface.z, fo2, nft, tid, NT, U, fx, qr, nfx, V, Vh, B, Vbh,
                               Rb, Tb);
        face_emit<SI, R, LF, 3>(bface, bfsrc, bfnb, fcap, nface.w, fo3, nft, tid, NT, U, fx, qr, nfx, V, Vh, B, Vbh,
                               Rb, Tb);
    }
}

template <class S, class R, int LF, int CF, class SI = S>
static int run_sap(qcd_field f, int ncy, int nmr, const void *eta, void *psi, int nrhs, hipStream_t s) {
    const Geom &g = f->g;
    const int Vbh = g.Vbh;
    const int nbc = g.Nb / 2;
    const size_t lds = (size_t)24 * Vbh * sizeof(cx<R>);
    const bool use_lds = lds <= 150 * 1024;
    int NT = ((Vbh + 63) / 64) * 64;
    int KS = 1;
    if (NT > 1024) {
        NT = 1024;
        KS = (Vbh + NT - 1) / NT;
    }
    if (KS > 2) return set_error(QCD_EINVAL, "Schwarz block too large (more than 4096 sites)");
    cx<R> *gbuf = nullptr;
    if (!use_lds) {
        void *p;
        DFL_TRY(field_buffer(f, BUF_SAP, (size_t)nbc * nrhs * lds, &p));
        gbuf = static_cast<cx<R> *>(p);
    }
    // the blocks' stored residuals and the face exchange (half-spinors)
    void *rp;
    const size_t rbytes = VecI<SI>::BYTES * g.V * nrhs;
    const size_t xbytes = HalfI<SI>::BYTES * g.Nb * f->nface_tot * nrhs;
    DFL_TRY(field_buffer(f, BUF_SAP_RES, rbytes + xbytes, &rp));
    void *res = rp, *fx = static_cast<char *>(rp) + rbytes;
    // the FP16 layouts start a workgroup's second right-hand side at whole
    // units (V is a product of four even extents; so is every face length)
    if (sizeof(SI) == 2 && (g.V % 16 || ((long)g.Nb * f->nface_tot) % 2))
        return set_error(QCD_EINVAL, "FP16 Schwarz vectors need V a multiple of 16");
    const R kappa = (R)f->lat.kappa;
    const int4 nface = make_int4(f->nface[0], f->nface[1], f->nface[2], f->nface[3]);
    const bool pair = sizeof(S) == 4 && f->st_sap_pair && use_lds && Vbh == 128 && NT == 128 && nrhs % 2 == 0;
    // Algorithmic work of one sweep per (even, odd) site pair of the swept
    // colour, with h = 165 flop per hop times the hops that stay inside the
    // block (sum over mu of 2 (b_mu - 1) / b_mu per site) and nf the hops
    // that cross the block's faces per pair (sum over mu of 4 / b_mu):
    //   the neighbours' hops across the faces nf 48 (not in the first sweep),
    //   s_o = A^-1 rho_o 504, rhat_e h + 72, each MinRes step 2h + 1392,
    //   back substitution and correction h + 576, odd residual 552 (when kept),
    //   this block's hops into the neighbours' faces nf 144 (but the last sweep).
    // Compulsory bytes per pair: eta (first cycle) or the stored residual,
    // the face half-spinors in (nf of them), psi in (after the first cycle)
    // and out, the stored residual out, the face half-spinors out; 4 links
    // and the clover term per site, the inverse clover per odd site.  The
    // stored residual and the half-spinors take the internal storage type.
    double hops = 0, nf = 0;
    for (int m = 0; m < 4; ++m) {
        hops += 2.0 * (g.b[m] - 1) / g.b[m];
        nf += 4.0 / g.b[m];
    }
    const double h = 165.0 * hops, B = Spin<S>::BYTES, BI = VecI<SI>::BYTES, BH = HalfI<SI>::BYTES;
    const double lbytes = LF == LNK_F64 ? 144 : (LF == LNK_F16 || LF == LNK_BF16) ? 24 : 48;
    const double cbytes = CF == CLO_F64 ? 576 : CF == CLO_F32 ? 288 : 144;
    const double pairs = (double)nbc * Vbh * nrhs;
    for (int cy = 0; cy < ncy; ++cy)
        for (int col = 0; col < 2; ++col) {
            int flags = 0;
            if (cy == 0) flags |= SW_FIRST;
            if (cy > 0 || col == 1) flags |= SW_FACES;
            if (cy + 1 < ncy) flags |= SW_STORE_RES;
            if (!(cy + 1 == ncy && col == 1)) flags |= SW_EMIT;
            dim3 grid(nbc, nrhs);
            const double fl = pairs * (((flags & SW_FACES) ? nf * 48.0 : 0.0) + 504 + (h + 72) +
                                       nmr * (2 * h + 1392) + (h + 576) + ((flags & SW_STORE_RES) ? 552 : 0) +
                                       ((flags & SW_EMIT) ? nf * 144.0 : 0.0));
            const double by = pairs * ((cy == 0 ? 2 * B : 2 * BI) + ((flags & SW_FACES) ? nf * BH : 0) +
                                       B * (cy == 0 ? 2 : 4) + ((flags & SW_STORE_RES) ? 2 * BI : 0) +
                                       ((flags & SW_EMIT) ? nf * BH : 0)) +
                              (double)nbc * Vbh * 2 * (4 * lbytes + cbytes) + (double)nbc * Vbh * cbytes;
            ProfScope ps(PROF_SAP, s, fl, by, 2 * pairs);
#define DFL_SAP_ARGS                                                                                             \
    eta, psi, res, fx, f->U[LF], f->clo[CF], f->cloinv[CF], f->lnbr, f->bface, f->bfsrc, f->bfnb, f->face_cap, \
        nface, g.V, g.Vh, Vbh, nbc, col, kappa, nmr, flags, gbuf
#define DFL_SAP_LAUNCH(LDSV, KSV, MAXT, VBHC)                                                                  \
    {                                                                                                          \
        auto kern = k_sap_sweep<S, R, LF, CF, LDSV, KSV, MAXT, VBHC, 1, SI>;                                   \
        size_t sh = LDSV ? lds : 0;                                                                            \
        if (LDSV && sh > 64 * 1024) (void)hipFuncSetAttribute((const void *)kern,                              \
                                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh); \
        kern<<<grid, NT, sh, s>>>(DFL_SAP_ARGS);                                                               \
    }
            if constexpr (sizeof(S) == 4) {
                // two right-hand sides per workgroup (4^4 blocks, even count)
                if (pair) {
                    k_sap_sweep<S, R, LF, CF, true, 1, 256, 128, 2, SI><<<dim3(nbc, nrhs / 2), 2 * NT, 2 * lds, s>>>(
                        DFL_SAP_ARGS);
                    continue;
                }
            }
            if (use_lds) {
                if (Vbh == 128) DFL_SAP_LAUNCH(true, 1, 256, 128)
                else if (Vbh == 256) DFL_SAP_LAUNCH(true, 1, 256, 256)
                else if (NT <= 256) DFL_SAP_LAUNCH(true, 1, 256, 0)
                // a bound of 768 threads (e.g. 6^4 blocks, 704) leaves 168
                // registers per lane where 1024 would cap them at 128
                else if (NT <= 768) DFL_SAP_LAUNCH(true, 1, 768, 0)
                else DFL_SAP_LAUNCH(true, 1, 1024, 0)
            } else {
                if (KS == 1) DFL_SAP_LAUNCH(false, 1, 1024, 0)
                else DFL_SAP_LAUNCH(false, 2, 1024, 0)
            }
#undef DFL_SAP_LAUNCH
#undef DFL_SAP_ARGS
        }
    DFL_HIP(hipGetLastError());
    return 0;
}

int sap_internal(qcd_field f, const qcd_sap *sap, const void *eta, void *psi, int nrhs, hipStream_t s) {
    if (sap->ncy < 1 || sap->nmr < 0) return set_error(QCD_EINVAL, "SAP needs ncy >= 1 and nmr >= 0");
    const bool v16 = sap->vecs == QCD_F16;
    if (v16 && sap->storage != QCD_F16 && sap->storage != QCD_BF16)
        return set_error(QCD_EINVAL, "FP16 Schwarz vectors go with FP16 or BF16 link storage");
    const int c = sap->ncy, m = sap->nmr;
    switch (sap->storage) {
        case QCD_F64: return run_sap<double, double, LNK_F64, CLO_F64>(f, c, m, eta, psi, nrhs, s);
        case QCD_F32: return run_sap<float, float, LNK_F32, CLO_F32>(f, c, m, eta, psi, nrhs, s);
        // FP16 / BF16 link storage enters the Schwarz kernel with row 2
        // precomputed (the same matrices as the reconstruct-12 copies)
        case QCD_F16:
            return v16 ? run_sap<float, float, LNK_F16R, CLO_F16, __half>(f, c, m, eta, psi, nrhs, s)
                       : run_sap<float, float, LNK_F16R, CLO_F16>(f, c, m, eta, psi, nrhs, s);
        case QCD_BF16:
            return v16 ? run_sap<float, float, LNK_BF16R, CLO_F16, __half>(f, c, m, eta, psi, nrhs, s)
                       : run_sap<float, float, LNK_BF16R, CLO_F16>(f, c, m, eta, psi, nrhs, s);
        default: return set_error(QCD_EINVAL, "bad SAP storage precision");
    }
}

}  // namespace dfl

using namespace dfl;

extern "C" int sap_precond(qcd_field f, const qcd_sap *sap, const void *eta, void *psi, int nrhs, qcd_prec io,
                           hipStream_t s) {
    if (!f || !sap || !eta || !psi || nrhs <= 0) return set_error(QCD_EINVAL, "bad arguments to sap_precond");
    if (io != QCD_F64 && io != QCD_F32) return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    const qcd_prec vec = sap->storage == QCD_F64 ? QCD_F64 : QCD_F32;
    const size_t nb = spinor_bytes(vec, f->g.V) * nrhs;
    void *ws;
    DFL_TRY(field_buffer(f, BUF_SAP_IO, 2 * nb, &ws));
    char *a = static_cast<char *>(ws), *b = a + nb;
    DFL_TRY(pack_spinor(f, eta, io, a, vec, nrhs, s));
    DFL_TRY(sap_internal(f, sap, a, b, nrhs, s));
    DFL_TRY(unpack_spinor(f, b, vec, psi, io, nrhs, s));
    return 0;
}
