// Even-odd ordered Wilson-clover stencil  out = A in - kappa H in  on the
// full lattice (both parities in one launch), multi right-hand side, and the
// canonical <-> internal vector conversions.
#include <type_traits>
#include "internal.h"
#include "blas.h"

namespace dfl {

// Site mapping: a workgroup owns a tile of `tile` consecutive sites of the
// even half and the same tile of the odd half (the same Schwarz-block
// positions), so the opposite-parity neighbours and the backward links a
// site needs were fetched by the other half of the same workgroup.  The
// workgroup covers RG right-hand sides over the same tile, one per group of
// waves: the right-hand side (and with it the spinor buffer descriptor) is
// uniform in a wave, and the other waves of the workgroup find the tile's
// links and clover term in the CU's cache.  The clover term is read once
// per site and workgroup, so its loads are non-temporal and do not evict the
// reused spinors and links from L2.  With `border` the tiles walk the
// Schwarz blocks in lexicographic block order (border maps it to the
// colour-major memory order), so that the blocks next to a tile, which hold
// its off-block neighbours, are processed close by in time and on the same
// XCD; without it they walk memory order.
template <class S, class SO, class R, int LF, int CF, int RG>
__global__ void __launch_bounds__(256) k_dirac_rg(const void *__restrict__ in, void *__restrict__ out,
                                                  const void *__restrict__ U, const void *__restrict__ clo,
                                                  const int *__restrict__ nbr, const int *__restrict__ border,
                                                  long V, int Vbh, R kappa, int nrhs) {
    unsigned bx, by;
    xcd_order(bx, by);
    const int tile = blockDim.x / (2 * RG);
    // 2 tile is a multiple of the wave size (RG <= 4 at 256 threads), so the
    // right-hand side is wave-uniform; say so, or the compiler wraps every
    // buffer load in a loop over the distinct descriptors
    const int sub = __builtin_amdgcn_readfirstlane(threadIdx.x / (2 * tile));
    const int sl = threadIdx.x - sub * 2 * tile;
    const int par = sl >= tile ? 1 : 0;
    long pos = (long)bx * tile + (sl - par * tile);
    if (border) {
        const long k = pos / Vbh;
        pos = (long)border[k] * Vbh + (pos - k * Vbh);
    }
    const long x = (long)par * (V / 2) + pos;
    const int r = by * RG + sub;
    if (r >= nrhs) return;
    const char *inb = static_cast<const char *>(in) + (size_t)r * Spin<S>::BYTES * V;
    char *outb = static_cast<char *>(out) + (size_t)r * Spin<SO>::BYTES * V;
    cx<R> acc[12], w[9], p[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
#define DFL_HOP_RG(MU)                                     \
    {                                                      \
        const int ef = nbr_at(nbr, 2 * MU, V, x);          \
        Link<LF>::load(U, V, MU, x, w);                    \
        Spin<S>::load(inb, V, nb_index(ef), p);            \
        hop<R, MU, true>(w, p, nb_sign<R>(ef), acc);       \
        const int eb = nbr_at(nbr, 2 * MU + 1, V, x);      \
        Link<LF>::load(U, V, MU, nb_index(eb), w);         \
        Spin<S>::load(inb, V, nb_index(eb), p);            \
        hop<R, MU, false>(w, p, nb_sign<R>(eb), acc);      \
        __builtin_amdgcn_sched_barrier(0);                 \
    }
    DFL_HOP_RG(0)
    DFL_HOP_RG(1)
    DFL_HOP_RG(2)
    DFL_HOP_RG(3)
#undef DFL_HOP_RG
    cx<R> o[12];
    Spin<S>::load(inb, V, x, p);
    clover_apply<CF, R, true>(clo, V, x, p, o);
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = rmac(o[k], -kappa, acc[k]);
    Spin<SO>::store(outb, V, x, o);
}

// Block-staged stencil: one workgroup per (Schwarz block, right-hand side),
// one thread per site (thread t: parity t / Vbh, local index t % Vbh).  The
// block's input spinors are staged in LDS once, with coalesced loads; the
// hops that stay inside the block (the in-block neighbour table is the same
// for every block, and such hops never cross the lattice boundary) read them
// there, and only the hops leaving the block read global memory.  For 4^4
// blocks three quarters of the neighbour reads stay on the CU, however many
// right-hand sides compete for the L2.  Blocks are taken in lexicographic
// order (border), right-hand sides of one block on one XCD back to back, so
// links, clover and the off-block neighbours are shared through L2.
template <class S>
struct Chunk;
template <>
struct Chunk<float> {
    using T = float4;
};
template <>
struct Chunk<double> {
    using T = double2;
};
template <>
struct Chunk<__half> {
    using T = h8;
};

// one site's spinor from 16-byte chunks `stride` apart, through a generic
// pointer (LDS or global memory); `sc` is the site's scale (FP16 storage)
template <class S, class R>
__device__ inline void gen_spin(const typename Chunk<S>::T *src, long stride, const float *sc, cx<R> v[12]) {
    if constexpr (Spin<S>::NCH == 6) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const float4 t = src[c * stride];
            v[2 * c] = {R(t.x), R(t.y)};
            v[2 * c + 1] = {R(t.z), R(t.w)};
        }
    } else if constexpr (Spin<S>::NCH == 12) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double2 t = src[c * stride];
            v[c] = {R(t.x), R(t.y)};
        }
    } else {
        h8 t[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) t[c] = src[c * stride];
        Spin<__half>::decode(t, *sc, v);
    }
}

// NR right-hand sides per workgroup (NR divides nrhs), Vb x NR threads: a
// wave holds 64 / NR sites of the block for each of the NR right-hand
// sides, lane l taking site l % (64 / NR) of the wave's run and right-hand
// side l / (64 / NR).  Every thread does the one-site, one-right-hand-side
// work, but the NR lanes of a site read the same link, clover and table
// entries in the same instruction, so each of those loads fetches the data
// of 64 / NR sites instead of 64 (NR = 1 is the plain layout).
// RES: out = b - M in, and the workgroup's share of ||out||^2 into
// part[rhs][block in memory] (a fixed order of additions, so the norm is
// reproducible and independent of the launch order).
// S: input spinor storage (staged in LDS), SO: output storage.
template <class S, class SO, class R, int LF, int CF, int MAXT, int NR = 1, bool RES = false>
__global__ void __launch_bounds__(MAXT) k_dirac_blk(const void *__restrict__ in, void *__restrict__ out,
                                                    const void *__restrict__ U, const void *__restrict__ clo,
                                                    const int *__restrict__ nbr, const short *__restrict__ lnbr,
                                                    const int *__restrict__ border, long V, long Vh, int Vbh,
                                                    R kappa, const void *__restrict__ b = nullptr,
                                                    double *__restrict__ part = nullptr,
                                                    float4 *__restrict__ rho32 = nullptr) {
    using T = typename Chunk<S>::T;
    constexpr int NCH = Spin<S>::NCH;
    constexpr bool HALF = NCH == 3;
    extern __shared__ unsigned char dsm_raw[];
    unsigned bx, rg;
    xcd_order(bx, rg);
    const long B = border[bx];
    const int Vb = 2 * Vbh;
    constexpr int SPW = 64 / NR;                       // sites per wave
    const int lane = threadIdx.x & 63, q = lane / SPW;
    const int t = (threadIdx.x >> 6) * SPW + (lane - q * SPW);   // site in the block
    // LDS: one block of NCH chunks per site for each right-hand side, then
    // the per-site scales (FP16 storage)
    T *sm = reinterpret_cast<T *>(dsm_raw) + q * NCH * Vb;
    float *smsc = reinterpret_cast<float *>(reinterpret_cast<T *>(dsm_raw) + NR * NCH * Vb) + q * Vb;
    const int par = t >= Vbh ? 1 : 0;
    const int j = t - par * Vbh;
    const unsigned x = (unsigned)(par * Vh + B * Vbh + j);
    const unsigned xi = x + (unsigned)(q * Spin<S>::NCH * V);     // this lane's input spinor
    const unsigned xo = x + (unsigned)(q * Spin<SO>::NCH * V);    // and output spinor
    // buffer bases stay wave-uniform (the first right-hand side of the
    // workgroup); a lane's own right-hand side enters through its element
    // index: q x NCH x V 16-byte chunks further (FP32 and FP64 storage only)
    static_assert(NR == 1 || (Spin<S>::NCH * 16 == Spin<S>::BYTES && Spin<SO>::NCH * 16 == Spin<SO>::BYTES),
                  "several right-hand sides per workgroup need chunk-only spinor storage");
    const char *inb = wave_uniform(static_cast<const char *>(in) + (size_t)rg * NR * Spin<S>::BYTES * V);
    char *outb = wave_uniform(static_cast<char *>(out) + (size_t)rg * NR * Spin<SO>::BYTES * V);
#pragma unroll
    for (int c = 0; c < NCH; ++c) sm[c * Vb + t] = ld<T>(inb, c, V, xi);
    if constexpr (HALF) smsc[t] = ld<float>(inb, 12, V, x);
    __syncthreads();
    const uint4 nb4 = ld<uint4>(lnbr, 0, 0, (unsigned)t);
    const unsigned nbw[4] = {nb4.x, nb4.y, nb4.z, nb4.w};
    const int obase = (1 - par) * Vbh;  // LDS offset of the other parity
    cx<R> acc[12], w[9], p[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
    // Each hop ends in a scheduling fence: without it the compiler hoists
    // all 48 neighbour loads to the top and keeps them live (up to 250
    // registers).  Neighbour spinor through a generic pointer: LDS inside the block,
    // global memory outside, one flat load per chunk and no divergent branch.
    // The neighbour table is read for every hop (in-block entries carry the
    // right index and no boundary sign): a load guarded by the in-block test
    // becomes a branch that costs far more registers than the table read.
    const T *sm_g = sm;
    const T *in_g = reinterpret_cast<const T *>(inb) + (size_t)q * NCH * V;
    const float *smsc_g = smsc;
    const float *insc_g = reinterpret_cast<const float *>(inb) + 12 * V;
#define DFL_BLK_HOP(MU)                                                                                 \
    {                                                                                                   \
        const int lf = (short)(nbw[MU] & 0xffffu);                                                      \
        const int lb = (short)(nbw[MU] >> 16);                                                          \
        const int ef = nbr_at(nbr, 2 * MU, V, x);                                                       \
        const int eb = nbr_at(nbr, 2 * MU + 1, V, x);                                                   \
        Link<LF>::load(U, V, MU, x, w);                                                                 \
        const unsigned yf = nb_index(ef);                                                               \
        gen_spin<S, R>(lf >= 0 ? sm_g + obase + lf : in_g + yf, lf >= 0 ? Vb : V,                       \
                       lf >= 0 ? smsc_g + obase + lf : insc_g + yf, p);                                 \
        hop<R, MU, true>(w, p, nb_sign<R>(ef), acc);                                                    \
        const unsigned y = nb_index(eb);                                                                \
        gen_spin<S, R>(lb >= 0 ? sm_g + obase + lb : in_g + y, lb >= 0 ? Vb : V,                        \
                       lb >= 0 ? smsc_g + obase + lb : insc_g + y, p);                                  \
        Link<LF>::load(U, V, MU, y, w);                                                                 \
        hop<R, MU, false>(w, p, nb_sign<R>(eb), acc);                                                   \
        __builtin_amdgcn_sched_barrier(0);                                                              \
    }
    DFL_BLK_HOP(0)
    DFL_BLK_HOP(1)
    DFL_BLK_HOP(2)
    DFL_BLK_HOP(3)
#undef DFL_BLK_HOP
    cx<R> o[12];
    gen_spin<S, R>(sm_g + t, Vb, smsc_g + t, p);
    clover_apply<CF, R, false>(clo, V, x, p, o);
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = rmac(o[k], -kappa, acc[k]);
    if constexpr (RES) {
        __shared__ double red[NR][MAXT / 64];
        Spin<S>::load(wave_uniform(static_cast<const char *>(b) + (size_t)rg * NR * Spin<S>::BYTES * V), V, xi, p);
        double nn = 0;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            o[k] = p[k] - o[k];
            nn = ffma((double)o[k].re, (double)o[k].re, ffma((double)o[k].im, (double)o[k].im, nn));
        }
#pragma unroll
        for (int off = SPW / 2; off > 0; off >>= 1) nn += __shfl_xor(nn, off, 64);
        if (lane == q * SPW) red[q][threadIdx.x >> 6] = nn;
        __syncthreads();
        if (threadIdx.x < NR) {
            double sum = 0;
            for (int w = 0; w < Vb / SPW; ++w) sum += red[threadIdx.x][w];
            // memory order of the blocks: the same sum for any launch order
            part[(size_t)(rg * NR + threadIdx.x) * gridDim.x + B] = sum;
        }
    }
    Spin<SO>::store(outb, V, xo, o);
    if constexpr (RES) {
        // the residual rounded to FP32 as well, for the next Krylov cycle
        if (rho32 != nullptr)
            Spin<float>::store(wave_uniform(reinterpret_cast<char *>(rho32) + (size_t)rg * NR * 96 * V), V,
                               x + (unsigned)(q * 6 * V), o);
    }
}

// Link rows 0-1 of a half-precision reconstruct-12 link from three 8-byte
// chunks `stride` apart, through a generic pointer (LDS or global memory),
// and its third row rebuilt
template <class H4, class R>
__device__ inline void gen_link(const H4 *src, long stride, cx<R> w[9]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const H4 t = src[c * stride];
        w[2 * c] = {R(to_f(t.v[0])), R(to_f(t.v[1]))};
        w[2 * c + 1] = {R(to_f(t.v[2])), R(to_f(t.v[3]))};
    }
    rebuild_row2(w);
}

// Block-staged stencil that keeps the block's links in LDS and loops over
// all right-hand sides of the call, NR at a time (FP32 vectors, FP16 or BF16
// reconstruct-12 links, blocks of at most 256 sites).  One workgroup per
// block: the block's 4 forward links per site are loaded once (24 KB for a
// 4^4 block) and read from LDS by every group of right-hand sides; the
// backward hop into the block reads its neighbour's forward link there too,
// and only backward hops from outside the block read global memory, through
// the same generic pointer.  Lanes and right-hand sides as in k_dirac_blk.
template <class H4, int LF, int CF, int NR>
__global__ void __launch_bounds__(256 * NR) __attribute__((amdgpu_waves_per_eu(4))) k_dirac_blkL(const void *__restrict__ in, void *__restrict__ out,
                                                         const void *__restrict__ U, const void *__restrict__ clo,
                                                         const int *__restrict__ nbr, const short *__restrict__ lnbr,
                                                         const int *__restrict__ border, long V, long Vh, int Vbh,
                                                         float kappa, int ngroups) {
    using T = float4;
    constexpr int NCH = 6;
    extern __shared__ unsigned char dsm_raw[];
    unsigned bx, unused;
    xcd_order(bx, unused);
    const long B = border[bx];
    const int Vb = 2 * Vbh;
    constexpr int SPW = 64 / NR;
    const int lane = threadIdx.x & 63, q = lane / SPW;
    const int t0 = (threadIdx.x >> 6) * SPW + (lane - q * SPW);   // site in the block
    // LDS: links [mu][3 chunks][Vb] (8 B each), then NR blocks of spinors
    H4 *lk = reinterpret_cast<H4 *>(dsm_raw);
    T *sm = reinterpret_cast<T *>(dsm_raw + sizeof(H4) * 12 * Vb) + q * NCH * Vb;
    const int par = t0 >= Vbh ? 1 : 0;
    const unsigned x0 = (unsigned)(par * Vh + B * Vbh + (t0 - par * Vbh));
    const int t = t0;
    const unsigned x = x0;
    const H4 *Ug = static_cast<const H4 *>(U);
    for (int k = q; k < 12; k += NR) lk[k * Vb + t] = ld<H4>(Ug, k, V, x);
    const H4 *lk_g = lk;
    const T *sm_g = sm;
    const float *nosc = nullptr;
    for (int g = 0; g < ngroups; ++g) {
        // the site indices are made opaque here, so that nothing derived
        // from them (table entries, addresses) is kept live across groups:
        // the compiler would otherwise hold all of it in registers
        unsigned x = x0;
        int t = t0;
        asm volatile("" : "+v"(x), "+v"(t));
        const int obase = t >= Vbh ? 0 : Vbh;   // LDS offset of the other parity
        const uint4 nb4 = ld<uint4>(lnbr, 0, 0, (unsigned)t);
        const unsigned nbw[4] = {nb4.x, nb4.y, nb4.z, nb4.w};
        const unsigned xi = x + (unsigned)(q * NCH * V);
        const char *inb = wave_uniform(static_cast<const char *>(in) + (size_t)g * NR * 96 * V);
        char *outb = wave_uniform(static_cast<char *>(out) + (size_t)g * NR * 96 * V);
        if (g > 0) __syncthreads();   // the previous group's spinors are no longer read
#pragma unroll
        for (int c = 0; c < NCH; ++c) sm[c * Vb + t] = ld<T>(inb, c, V, xi);
        __syncthreads();
        const T *in_g = reinterpret_cast<const T *>(inb) + (size_t)q * NCH * V;
        cx<float> acc[12], w[9], p[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {0.f, 0.f};
#define DFL_BLKL_HOP(MU)                                                                                \
    {                                                                                                   \
        const int lf = (short)(nbw[MU] & 0xffffu);                                                      \
        const int lb = (short)(nbw[MU] >> 16);                                                          \
        const int ef = nbr_at(nbr, 2 * MU, V, x);                                                       \
        const int eb = nbr_at(nbr, 2 * MU + 1, V, x);                                                   \
        gen_link<H4, float>(lk_g + MU * 3 * Vb + t, Vb, w);                                             \
        const unsigned yf = nb_index(ef);                                                               \
        gen_spin<float, float>(lf >= 0 ? sm_g + obase + lf : in_g + yf, lf >= 0 ? Vb : V, nosc, p);     \
        hop<float, MU, true>(w, p, nb_sign<float>(ef), acc);                                            \
        const unsigned y = nb_index(eb);                                                                \
        gen_spin<float, float>(lb >= 0 ? sm_g + obase + lb : in_g + y, lb >= 0 ? Vb : V, nosc, p);      \
        gen_link<H4, float>(lb >= 0 ? lk_g + MU * 3 * Vb + obase + lb : Ug + (size_t)MU * 3 * V + y,    \
                            lb >= 0 ? Vb : V, w);                                                       \
        hop<float, MU, false>(w, p, nb_sign<float>(eb), acc);                                           \
        __builtin_amdgcn_sched_barrier(0);                                                              \
    }
        DFL_BLKL_HOP(0)
        DFL_BLKL_HOP(1)
        DFL_BLKL_HOP(2)
        DFL_BLKL_HOP(3)
#undef DFL_BLKL_HOP
        cx<float> o[12];
        gen_spin<float, float>(sm_g + t, Vb, nosc, p);
        clover_apply<CF, float, false>(clo, V, x, p, o);
#pragma unroll
        for (int k = 0; k < 12; ++k) o[k] = rmac(o[k], -kappa, acc[k]);
        Spin<float>::store(outb, V, x + (unsigned)(q * NCH * V), o);
    }
}

// right-hand sides per block-staged workgroup: the handle's choice (0:
// automatic, 2), reduced until it divides nrhs, the workgroup has at most
// 1024 threads and 256 per right-hand side, and the staged blocks fit the
// device's LDS per workgroup
template <class S, class SO>
static int blk_nr(qcd_field f, int nrhs, int Vb, size_t lds) {
    if (Spin<S>::NCH * 16 != Spin<S>::BYTES || Spin<SO>::NCH * 16 != Spin<SO>::BYTES) return 1;   // FP16 storage
    int nr = f->st_nr > 0 ? f->st_nr : 2;
    while (nr > 1 && (nrhs % nr || Vb > 256 || (size_t)nr * lds > f->lds_max)) nr /= 2;
    return nr;
}

template <class S, class SO, class R, int LF, int CF>
static int launch_dirac(qcd_field f, const void *in, void *out, int nrhs, hipStream_t s) {
    const long V = f->g.V;
    const R kappa = (R)f->lat.kappa;
    const void *U = f->U[LF];
    const void *C = f->clo[CF];
    constexpr int BS = 256;
    // algorithmic work: 1872 flop per site and right-hand side; compulsory
    // bytes = 4 links + clover per site once, spinor in + out per rhs
    const double lbytes = LF == LNK_F64 ? 144 : LF == LNK_F32 ? 48 : 24;
    const double cbytes = CF == CLO_F64 ? 576 : CF == CLO_F32 ? 288 : 144;
    const double sbytes = (double)Spin<S>::BYTES + Spin<SO>::BYTES;
    auto work = [&](int n) { return std::make_tuple(1872.0 * V * n, V * (4 * lbytes + cbytes + n * sbytes), 1.0 * V * n); };
    // tuning knobs of the handle: right-hand sides per site tile (0 =
    // automatic), tile order (lexicographic blocks or memory order), and
    // the block-staged kernel when the block fits one workgroup and its
    // spinors fit 64 KB of LDS
    const int rg = f->st_rg > 0 ? f->st_rg : (nrhs >= 2 ? 2 : 1);
    const int *border = f->st_order ? f->border : nullptr;
    auto [fl, by, un] = work(nrhs);
    ProfScope ps(PROF_DIRAC, s, fl, by, un);
    const int Vb = 2 * f->g.Vbh;
    const size_t lds = (size_t)Spin<S>::BYTES * Vb;
    if constexpr (sizeof(S) == 4 && sizeof(SO) == 4 && (LF == LNK_F16 || LF == LNK_BF16)) {
        // links in LDS, right-hand sides looped within the workgroup
        using H4 = std::conditional_t<LF == LNK_F16, h4, b4>;
        const size_t ldsL = sizeof(H4) * 12 * Vb + 2 * lds;
        // from 16 right-hand sides on (fewer do not amortise the link staging)
        if (f->st_block && f->st_linklds && nrhs >= 16 && Vb % 64 == 0 && Vb <= 256 && nrhs % 2 == 0 &&
            ldsL <= f->lds_max) {
            k_dirac_blkL<H4, LF, CF, 2><<<dim3((unsigned)f->g.Nb), Vb * 2, ldsL, s>>>(
                in, out, U, C, f->nbr, f->lnbr, f->border, V, f->g.Vh, f->g.Vbh, (float)kappa, nrhs / 2);
            DFL_HIP(hipGetLastError());
            return 0;
        }
    }
    if (f->st_block && Vb % 64 == 0 && Vb <= 1024 && lds <= 64 * 1024 && (Vb <= 512 || sizeof(R) == 4)) {
        const int nr = blk_nr<S, SO>(f, nrhs, Vb, lds);
        const dim3 grid((unsigned)f->g.Nb, (unsigned)(nrhs / nr));
#define DFL_BLK_LAUNCH(MAXT, NR)                                                                              \
    k_dirac_blk<S, SO, R, LF, CF, MAXT, NR><<<grid, Vb * NR, NR * lds, s>>>(in, out, U, C, f->nbr, f->lnbr,      \
                                                                        f->border, V, f->g.Vh, f->g.Vbh, kappa)
        constexpr bool chunked = Spin<S>::NCH * 16 == Spin<S>::BYTES && Spin<SO>::NCH * 16 == Spin<SO>::BYTES;
        bool launched = false;
        if constexpr (chunked) {
            if (nr == 4) DFL_BLK_LAUNCH(1024, 4);
            if (nr == 2) DFL_BLK_LAUNCH(512, 2);
            launched = nr > 1;
        }
        if (!launched) {
            if (Vb <= 256) DFL_BLK_LAUNCH(256, 1);
            else if (Vb <= 512) DFL_BLK_LAUNCH(512, 1);
            else DFL_BLK_LAUNCH(1024, 1);
        }
#undef DFL_BLK_LAUNCH
        DFL_HIP(hipGetLastError());
        return 0;
    }
    // grid: (V / 2) / tile site tiles x ceil(nrhs / RG) groups; V/2 is a multiple of 128
#define DFL_RG_LAUNCH(RGV)                                                                            \
    k_dirac_rg<S, SO, R, LF, CF, RGV><<<dim3((unsigned)(V / 2 / (BS / (2 * RGV))), (nrhs + RGV - 1) / RGV), BS, 0, s>>>( \
        in, out, U, C, f->nbr, border, V, f->g.Vbh, kappa, nrhs)
    switch (rg) {
        case 2: DFL_RG_LAUNCH(2); break;
        case 4: DFL_RG_LAUNCH(4); break;
        default: DFL_RG_LAUNCH(1);
    }
#undef DFL_RG_LAUNCH
    DFL_HIP(hipGetLastError());
    return 0;
}

int dirac_resid(qcd_field f, const double2 *x, const double2 *b, double2 *r, int nrhs, double *norm2,
                hipStream_t s, float4 *rho32) {
    const Geom &g = f->g;
    const int Vb = 2 * g.Vbh;
    const size_t lds = (size_t)12 * Vb * 16;
    if (!(Vb % 64 == 0 && Vb <= 512 && lds <= 64 * 1024)) {
        // blocks that do not fit one workgroup: stencil, then a separate pass
        const size_t tb = sizeof(double2) * 12 * g.V * nrhs;
        void *tp;
        DFL_TRY(field_buffer(f, BUF_RES, tb + sizeof(double) * (size_t)nrhs * BLAS_NBLK, &tp));
        double2 *t = static_cast<double2 *>(tp);
        DFL_TRY(dirac_internal(f, x, t, nrhs, QCD_F64, QCD_F64, s));
        DFL_TRY(blas_resid(b, t, r, 12 * g.V, nrhs, reinterpret_cast<double *>(static_cast<char *>(tp) + tb), norm2,
                           s));
        return rho32 ? blas_d2f(r, rho32, g.V, nrhs, s) : 0;
    }
    void *pp;
    DFL_TRY(field_buffer(f, BUF_RES, sizeof(double) * (size_t)nrhs * g.Nb, &pp));
    double *part = static_cast<double *>(pp);
    {
        // 1872 flop per site (+ 2 x 24 for the difference and the norm);
        // bytes: FP64 links and clover once, x, b in and r out per rhs
        ProfScope ps(PROF_DIRAC, s, 1920.0 * g.V * nrhs, g.V * (4 * 144.0 + 576.0 + nrhs * 3 * 192.0),
                     1.0 * g.V * nrhs);
        const int nr = blk_nr<double, double>(f, nrhs, Vb, lds);
        const dim3 grid((unsigned)g.Nb, (unsigned)(nrhs / nr));
#define DFL_RES_LAUNCH(MAXT, NR)                                                                        \
    k_dirac_blk<double, double, double, LNK_F64, CLO_F64, MAXT, NR, true><<<grid, Vb * NR, NR * lds, s>>>( \
        x, r, f->U[LNK_F64], f->clo[CLO_F64], f->nbr, f->lnbr, f->border, g.V, g.Vh, g.Vbh, f->lat.kappa, b, part, \
        rho32)
        if (nr == 4) DFL_RES_LAUNCH(1024, 4);
        else if (nr == 2) DFL_RES_LAUNCH(512, 2);
        else if (Vb <= 256) DFL_RES_LAUNCH(256, 1);
        else DFL_RES_LAUNCH(512, 1);
#undef DFL_RES_LAUNCH
        DFL_HIP(hipGetLastError());
    }
    return blas_reduce(part, 1, g.Nb, nrhs, norm2, s);
}

// vin / vout: internal vector storage of input and output (F64, F32, or
// F16 = FP16 with per-site scale); FP16 vectors need FP16/BF16 operator
// storage, FP64 vectors FP64 storage
int dirac_internal2(qcd_field f, const void *in, qcd_prec vin, void *out, qcd_prec vout, int nrhs,
                    qcd_prec storage, hipStream_t s) {
    if (vin == QCD_F64 || vout == QCD_F64) {
        if (vin != vout || storage != QCD_F64)
            return set_error(QCD_EINVAL, "FP64 vectors need FP64 operator storage on both sides");
        return launch_dirac<double, double, double, LNK_F64, CLO_F64>(f, in, out, nrhs, s);
    }
    if (vin == QCD_F16 && storage != QCD_F16 && storage != QCD_BF16)
        return set_error(QCD_EINVAL, "FP16 spinors need FP16 or BF16 operator storage");
#define DFL_DIRAC_IO(LF, CF)                                                                        \
    if (vin == QCD_F32 && vout == QCD_F32) return launch_dirac<float, float, float, LF, CF>(f, in, out, nrhs, s);    \
    if (vin == QCD_F16 && vout == QCD_F32) return launch_dirac<__half, float, float, LF, CF>(f, in, out, nrhs, s);  \
    if (vin == QCD_F16 && vout == QCD_F16) return launch_dirac<__half, __half, float, LF, CF>(f, in, out, nrhs, s); \
    if (vin == QCD_F32 && vout == QCD_F16) return launch_dirac<float, __half, float, LF, CF>(f, in, out, nrhs, s);  \
    return set_error(QCD_EINVAL, "vector precision must be F64, F32 or F16");
    switch (storage) {
        case QCD_F32: {
            if (vin == QCD_F16 || vout == QCD_F16) return set_error(QCD_EINVAL, "FP16 spinors need FP16/BF16 storage");
            return launch_dirac<float, float, float, LNK_F32, CLO_F32>(f, in, out, nrhs, s);
        }
        case QCD_F16: { DFL_DIRAC_IO(LNK_F16, CLO_F16) }
        case QCD_BF16: { DFL_DIRAC_IO(LNK_BF16, CLO_F16) }
        default: return set_error(QCD_EINVAL, "FP32 and FP16 vectors take F32, F16 or BF16 operator storage");
    }
#undef DFL_DIRAC_IO
}

int dirac_internal(qcd_field f, const void *in, void *out, int nrhs, qcd_prec vec, qcd_prec storage,
                   hipStream_t s) {
    return dirac_internal2(f, in, vec, out, vec, nrhs, storage, s);
}

// ---------------------------------------------------------------------------
// canonical [n][V][4][3] complex (lexicographic) <-> internal [n][chunk][V]
// ---------------------------------------------------------------------------
template <class CT, class S>
__global__ void k_pack(const CT *__restrict__ canon, void *__restrict__ out, const int *__restrict__ lex_of,
                       long V) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= V) return;
    const int r = blockIdx.y;
    const CT *src = canon + ((size_t)r * V + lex_of[idx]) * 12;
    using R = decltype(CT::x);
    cx<R> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = {src[k].x, src[k].y};
    Spin<S>::store(static_cast<char *>(out) + (size_t)r * Spin<S>::BYTES * V, V, idx, v);
}

template <class CT, class S>
__global__ void k_unpack(const void *__restrict__ in, CT *__restrict__ canon, const int *__restrict__ lex_of,
                         long V) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= V) return;
    const int r = blockIdx.y;
    using R = decltype(CT::x);
    cx<R> v[12];
    Spin<S>::load(static_cast<const char *>(in) + (size_t)r * Spin<S>::BYTES * V, V, idx, v);
    CT *dst = canon + ((size_t)r * V + lex_of[idx]) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        dst[k].x = v[k].re;
        dst[k].y = v[k].im;
    }
}

int pack_spinor(qcd_field f, const void *canon, qcd_prec io, void *internal, qcd_prec vec, int nrhs,
                hipStream_t s) {
    const long V = f->g.V;
    dim3 grid(nblocks(V, 256), nrhs);
    ProfScope ps(PROF_OTHER, s);
    if (io == QCD_F64 && vec == QCD_F64)
        k_pack<double2, double><<<grid, 256, 0, s>>>((const double2 *)canon, internal, f->lex_of, V);
    else if (io == QCD_F64 && vec == QCD_F32)
        k_pack<double2, float><<<grid, 256, 0, s>>>((const double2 *)canon, internal, f->lex_of, V);
    else if (io == QCD_F32 && vec == QCD_F32)
        k_pack<float2, float><<<grid, 256, 0, s>>>((const float2 *)canon, internal, f->lex_of, V);
    else if (io == QCD_F32 && vec == QCD_F64)
        k_pack<float2, double><<<grid, 256, 0, s>>>((const float2 *)canon, internal, f->lex_of, V);
    else if (io == QCD_F32 && vec == QCD_F16)
        k_pack<float2, __half><<<grid, 256, 0, s>>>((const float2 *)canon, internal, f->lex_of, V);
    else if (io == QCD_F64 && vec == QCD_F16)
        k_pack<double2, __half><<<grid, 256, 0, s>>>((const double2 *)canon, internal, f->lex_of, V);
    else
        return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    DFL_HIP(hipGetLastError());
    return 0;
}

int unpack_spinor(qcd_field f, const void *internal, qcd_prec vec, void *canon, qcd_prec io, int nrhs,
                  hipStream_t s) {
    const long V = f->g.V;
    dim3 grid(nblocks(V, 256), nrhs);
    ProfScope ps(PROF_OTHER, s);
    if (io == QCD_F64 && vec == QCD_F64)
        k_unpack<double2, double><<<grid, 256, 0, s>>>(internal, (double2 *)canon, f->lex_of, V);
    else if (io == QCD_F64 && vec == QCD_F32)
        k_unpack<double2, float><<<grid, 256, 0, s>>>(internal, (double2 *)canon, f->lex_of, V);
    else if (io == QCD_F32 && vec == QCD_F32)
        k_unpack<float2, float><<<grid, 256, 0, s>>>(internal, (float2 *)canon, f->lex_of, V);
    else if (io == QCD_F32 && vec == QCD_F64)
        k_unpack<float2, double><<<grid, 256, 0, s>>>(internal, (float2 *)canon, f->lex_of, V);
    else if (io == QCD_F32 && vec == QCD_F16)
        k_unpack<float2, __half><<<grid, 256, 0, s>>>(internal, (float2 *)canon, f->lex_of, V);
    else if (io == QCD_F64 && vec == QCD_F16)
        k_unpack<double2, __half><<<grid, 256, 0, s>>>(internal, (double2 *)canon, f->lex_of, V);
    else
        return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    DFL_HIP(hipGetLastError());
    return 0;
}

}  // namespace dfl

using namespace dfl;

extern "C" int dirac_apply_ex(qcd_field f, const void *in, void *out, int nrhs, qcd_prec io, qcd_prec storage,
                              qcd_prec spinor_in, qcd_prec spinor_out, hipStream_t s) {
    if (!f || !in || !out || nrhs <= 0) return set_error(QCD_EINVAL, "bad arguments to dirac_apply");
    if (io != QCD_F64 && io != QCD_F32) return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    if (in == out) return set_error(QCD_EINVAL, "dirac_apply: in and out must differ");
    for (qcd_prec v : {spinor_in, spinor_out})
        if (v != QCD_F64 && v != QCD_F32 && v != QCD_F16)
            return set_error(QCD_EINVAL, "spinor storage must be F64, F32 or F16");
    const size_t na = spinor_bytes(spinor_in, f->g.V) * nrhs, nb = spinor_bytes(spinor_out, f->g.V) * nrhs;
    void *ws;
    DFL_TRY(field_buffer(f, BUF_APPLY, na + nb, &ws));
    char *a = static_cast<char *>(ws), *b = a + na;
    DFL_TRY(pack_spinor(f, in, io, a, spinor_in, nrhs, s));
    DFL_TRY(dirac_internal2(f, a, spinor_in, b, spinor_out, nrhs, storage, s));
    DFL_TRY(unpack_spinor(f, b, spinor_out, out, io, nrhs, s));
    return 0;
}

extern "C" int dirac_apply(qcd_field f, const void *in, void *out, int nrhs, qcd_prec io, qcd_prec storage,
                           hipStream_t s) {
    const qcd_prec vec = storage == QCD_F64 ? QCD_F64 : QCD_F32;
    return dirac_apply_ex(f, in, out, nrhs, io, storage, vec, vec, s);
}
