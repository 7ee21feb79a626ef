// Even-odd ordered Wilson-clover stencil  out = A in - kappa H in  on the
// full lattice (both parities in one launch), multi right-hand side, and the
// canonical <-> internal vector conversions.
#include "internal.h"

namespace dfl {

// Site mapping: a workgroup owns a tile of `tile` consecutive sites of the
// even half and the same tile of the odd half (the same Schwarz-block
// positions), so the opposite-parity neighbours and the backward links a
// site needs were fetched by the other half of the same workgroup.  RG
// adjacent lanes share one site, one right-hand side each: their link and
// clover loads hit the same address inside one wave instruction (fetched
// once per group) while spinor loads stay coalesced per right-hand side.
// The clover term is read exactly once per site and group, so its loads are
// non-temporal and do not evict the reused spinors and links from L2.
template <class S, class R, int LF, int CF, int RG>
__global__ void __launch_bounds__(256) k_dirac_rg(const void *__restrict__ in, void *__restrict__ out,
                                                  const void *__restrict__ U, const void *__restrict__ clo,
                                                  const int *__restrict__ nbr, long V, R kappa, int nrhs) {
    unsigned bx, by;
    xcd_order(bx, by);
    const int tile = blockDim.x / (2 * RG);
    const int sub = threadIdx.x % RG;
    const int sl = threadIdx.x / RG;
    const int par = sl >= tile ? 1 : 0;
    const long x = (long)par * (V / 2) + (long)bx * tile + (sl - par * tile);
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
    for (int k = 0; k < 12; ++k) o[k] = o[k] - kappa * acc[k];
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
    auto [fl, by, un] = work(nrhs);
    ProfScope ps(PROF_DIRAC, s, fl, by, un);
    // grid: (V / 2) / tile site tiles x ceil(nrhs / RG) groups; V/2 is a multiple of 128
#define DFL_RG_LAUNCH(RGV)                                                                            \
    k_dirac_rg<S, R, LF, CF, RGV><<<dim3((unsigned)(V / 2 / (BS / (2 * RGV))), (nrhs + RGV - 1) / RGV), BS, 0, s>>>( \
        in, out, U, C, f->nbr, V, kappa, nrhs)
    switch (rg) {
        case 2: DFL_RG_LAUNCH(2); break;
        case 4: DFL_RG_LAUNCH(4); break;
        case 8: DFL_RG_LAUNCH(8); break;
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
