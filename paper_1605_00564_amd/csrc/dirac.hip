// Even-odd ordered Wilson-clover stencil  out = A in - kappa H in  on the
// full lattice (both parities in one launch), multi right-hand side, and the
// canonical <-> internal vector conversions.
#include "internal.h"

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
template <class S, class R, int LF, int CF, int RG>
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
    const size_t fs = (size_t)Spin<S>::NCH * V * 16;
    const char *inb = static_cast<const char *>(in) + (size_t)r * fs;
    char *outb = static_cast<char *>(out) + (size_t)r * fs;
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
    Spin<S>::store(outb, V, x, o);
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

template <class S, class R>
__device__ inline void lds_spin(const typename Chunk<S>::T *sm, int stride, int at, cx<R> v[12]) {
    if constexpr (Spin<S>::NCH == 6) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const float4 t = sm[c * stride + at];
            v[2 * c] = {R(t.x), R(t.y)};
            v[2 * c + 1] = {R(t.z), R(t.w)};
        }
    } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double2 t = sm[c * stride + at];
            v[c] = {R(t.x), R(t.y)};
        }
    }
}

template <class S, class R, int LF, int CF, int MAXT>
__global__ void __launch_bounds__(MAXT) k_dirac_blk(const void *__restrict__ in, void *__restrict__ out,
                                                    const void *__restrict__ U, const void *__restrict__ clo,
                                                    const int *__restrict__ nbr, const short *__restrict__ lnbr,
                                                    const int *__restrict__ border, long V, long Vh, int Vbh,
                                                    R kappa) {
    using T = typename Chunk<S>::T;
    constexpr int NCH = Spin<S>::NCH;
    extern __shared__ unsigned char dsm_raw[];
    T *sm = reinterpret_cast<T *>(dsm_raw);
    unsigned bx, r;
    xcd_order(bx, r);
    const long B = border[bx];
    const int Vb = 2 * Vbh;
    const int t = threadIdx.x;
    const int par = t >= Vbh ? 1 : 0;
    const int j = t - par * Vbh;
    const unsigned x = (unsigned)(par * Vh + B * Vbh + j);
    const size_t fs = (size_t)NCH * V * 16;
    const char *inb = wave_uniform(static_cast<const char *>(in) + (size_t)r * fs);
    char *outb = wave_uniform(static_cast<char *>(out) + (size_t)r * fs);
#pragma unroll
    for (int c = 0; c < NCH; ++c) sm[c * Vb + t] = ld<T>(inb, c, V, x);
    __syncthreads();
    const uint4 nb4 = ld<uint4>(lnbr, 0, 0, (unsigned)t);
    const unsigned nbw[4] = {nb4.x, nb4.y, nb4.z, nb4.w};
    const int obase = (1 - par) * Vbh;  // LDS offset of the other parity
    cx<R> acc[12], w[9], p[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
    // Neighbour spinor through a generic pointer: LDS inside the block,
    // global memory outside, one flat load per chunk and no divergent branch.
    // The neighbour table is read for every hop (in-block entries carry the
    // right index and no boundary sign): a load guarded by the in-block test
    // becomes a branch that costs far more registers than the table read.
    const T *sm_g = sm;
    const T *in_g = reinterpret_cast<const T *>(inb);
    auto flat_spin = [&](const T *src, long stride, cx<R> v[12]) {
        if constexpr (NCH == 6) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const float4 q = src[c * stride];
                v[2 * c] = {R(q.x), R(q.y)};
                v[2 * c + 1] = {R(q.z), R(q.w)};
            }
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const double2 q = src[c * stride];
                v[c] = {R(q.x), R(q.y)};
            }
        }
    };
#define DFL_BLK_HOP(MU)                                                                  \
    {                                                                                    \
        const int lf = (short)(nbw[MU] & 0xffffu);                                       \
        const int lb = (short)(nbw[MU] >> 16);                                           \
        const int ef = nbr_at(nbr, 2 * MU, V, x);                                        \
        const int eb = nbr_at(nbr, 2 * MU + 1, V, x);                                    \
        Link<LF>::load(U, V, MU, x, w);                                                  \
        flat_spin(lf >= 0 ? sm_g + obase + lf : in_g + nb_index(ef), lf >= 0 ? Vb : V, p); \
        hop<R, MU, true>(w, p, nb_sign<R>(ef), acc);                                     \
        const unsigned y = nb_index(eb);                                                 \
        flat_spin(lb >= 0 ? sm_g + obase + lb : in_g + y, lb >= 0 ? Vb : V, p);          \
        Link<LF>::load(U, V, MU, y, w);                                                  \
        hop<R, MU, false>(w, p, nb_sign<R>(eb), acc);                                    \
    }
    DFL_BLK_HOP(0)
    DFL_BLK_HOP(1)
    DFL_BLK_HOP(2)
    DFL_BLK_HOP(3)
#undef DFL_BLK_HOP
    cx<R> o[12];
    lds_spin<S, R>(sm, Vb, t, p);
    clover_apply<CF, R, true>(clo, V, x, p, o);
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = rmac(o[k], -kappa, acc[k]);
    Spin<S>::store(outb, V, x, o);
}

template <class S, class R, int LF, int CF>
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
    const double sbytes = 2.0 * 24 * sizeof(S);
    auto work = [&](int n) { return std::make_tuple(1872.0 * V * n, V * (4 * lbytes + cbytes + n * sbytes), 1.0 * V * n); };
    // right-hand sides per site group (tuning knob; 0 = automatic)
    static const int rg_env = [] {
        const char *e = getenv("DFL_STENCIL_RG");
        return e ? atoi(e) : 0;
    }();
    int rg = rg_env > 0 ? rg_env : (nrhs >= 2 ? 2 : 1);
    // tile order (tuning knob): 1 = lexicographic blocks, 0 = memory order
    static const int ord_env = [] {
        const char *e = getenv("DFL_STENCIL_ORDER");
        return e ? atoi(e) : 1;
    }();
    const int *border = ord_env ? f->border : nullptr;
    auto [fl, by, un] = work(nrhs);
    ProfScope ps(PROF_DIRAC, s, fl, by, un);
    // kernel choice (tuning knob): block-staged when the block fits one
    // workgroup and its spinors fit 64 KB of LDS, else site tiles
    static const int blk_env = [] {
        const char *e = getenv("DFL_STENCIL_BLOCK");
        return e ? atoi(e) : 1;
    }();
    const int Vb = 2 * f->g.Vbh;
    const size_t lds = (size_t)Spin<S>::NCH * Vb * 16;
    if (blk_env && Vb % 64 == 0 && Vb <= 1024 && lds <= 64 * 1024 && (Vb <= 512 || sizeof(S) == 4)) {
        const dim3 grid((unsigned)f->g.Nb, (unsigned)nrhs);
#define DFL_BLK_LAUNCH(MAXT)                                                                                  \
    k_dirac_blk<S, R, LF, CF, MAXT><<<grid, Vb, lds, s>>>(in, out, U, C, f->nbr, f->lnbr, f->border, V, f->g.Vh, \
                                                          f->g.Vbh, kappa)
        if (Vb <= 256) DFL_BLK_LAUNCH(256);
        else if (Vb <= 512) DFL_BLK_LAUNCH(512);
        else DFL_BLK_LAUNCH(1024);
#undef DFL_BLK_LAUNCH
        DFL_HIP(hipGetLastError());
        return 0;
    }
    // grid: (V / 2) / tile site tiles x ceil(nrhs / RG) groups; V/2 is a multiple of 128
#define DFL_RG_LAUNCH(RGV)                                                                            \
    k_dirac_rg<S, R, LF, CF, RGV><<<dim3((unsigned)(V / 2 / (BS / (2 * RGV))), (nrhs + RGV - 1) / RGV), BS, 0, s>>>( \
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

int dirac_internal(qcd_field f, const void *in, void *out, int nrhs, qcd_prec vec, qcd_prec storage,
                   hipStream_t s) {
    if (vec == QCD_F64) {
        if (storage != QCD_F64) return set_error(QCD_EINVAL, "FP64 vectors need FP64 operator storage");
        return launch_dirac<double, double, LNK_F64, CLO_F64>(f, in, out, nrhs, s);
    }
    if (vec != QCD_F32) return set_error(QCD_EINVAL, "vector precision must be F64 or F32");
    switch (storage) {
        case QCD_F32: return launch_dirac<float, float, LNK_F32, CLO_F32>(f, in, out, nrhs, s);
        case QCD_F16: return launch_dirac<float, float, LNK_F16, CLO_F16>(f, in, out, nrhs, s);
        case QCD_BF16: return launch_dirac<float, float, LNK_BF16, CLO_F16>(f, in, out, nrhs, s);
        default: return set_error(QCD_EINVAL, "FP32 vectors take F32, F16 or BF16 operator storage");
    }
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
    Spin<S>::store(static_cast<char *>(out) + (size_t)r * Spin<S>::NCH * V * 16, V, idx, v);
}

template <class CT, class S>
__global__ void k_unpack(const void *__restrict__ in, CT *__restrict__ canon, const int *__restrict__ lex_of,
                         long V) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= V) return;
    const int r = blockIdx.y;
    using R = decltype(CT::x);
    cx<R> v[12];
    Spin<S>::load(static_cast<const char *>(in) + (size_t)r * Spin<S>::NCH * V * 16, V, idx, v);
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
    else
        return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    DFL_HIP(hipGetLastError());
    return 0;
}

}  // namespace dfl

using namespace dfl;

extern "C" int dirac_apply(qcd_field f, const void *in, void *out, int nrhs, qcd_prec io, qcd_prec storage,
                           hipStream_t s) {
    if (!f || !in || !out || nrhs <= 0) return set_error(QCD_EINVAL, "bad arguments to dirac_apply");
    if (io != QCD_F64 && io != QCD_F32) return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    if (in == out) return set_error(QCD_EINVAL, "dirac_apply: in and out must differ");
    const qcd_prec vec = storage == QCD_F64 ? QCD_F64 : QCD_F32;
    const size_t nb = spinor_bytes(vec, f->g.V) * nrhs;
    void *ws;
    DFL_TRY(field_buffer(f, BUF_APPLY, 2 * nb, &ws));
    char *a = static_cast<char *>(ws), *b = a + nb;
    DFL_TRY(pack_spinor(f, in, io, a, vec, nrhs, s));
    DFL_TRY(dirac_internal(f, a, b, nrhs, vec, storage, s));
    DFL_TRY(unpack_spinor(f, b, vec, out, io, nrhs, s));
    return 0;
}
