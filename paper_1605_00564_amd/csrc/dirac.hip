// Even-odd ordered Wilson-clover stencil  out = A in - kappa H in  on the
// full lattice (both parities in one launch), multi right-hand side, and the
// canonical <-> internal vector conversions.
#include "internal.h"

namespace dfl {

// One thread per site; NR right-hand sides per thread share every link load.
template <class S, class R, int LF, int CF, int NR>
__global__ void __launch_bounds__(256) k_dirac(const void *__restrict__ in, void *__restrict__ out,
                                               const void *__restrict__ U, const void *__restrict__ clo,
                                               const int *__restrict__ nbr, long V, R kappa, int rhs0) {
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= V) return;
    const size_t fs = (size_t)Spin<S>::NCH * V * 16;  // bytes per right-hand side
    const char *inb = static_cast<const char *>(in) + (size_t)(rhs0 + blockIdx.y * NR) * fs;
    char *outb = static_cast<char *>(out) + (size_t)(rhs0 + blockIdx.y * NR) * fs;
    cx<R> acc[NR][12];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[r][k] = {R(0), R(0)};
    cx<R> w[9], p[12];
#define DFL_HOP_MU(MU)                                                        \
    {                                                                         \
        const int ef = nbr_at(nbr, 2 * MU, V, x);                                 \
        const long yf = nb_index(ef);                                         \
        Link<LF>::load(U, V, MU, x, w);                                       \
        _Pragma("unroll") for (int r = 0; r < NR; ++r) {                      \
            Spin<S>::load(inb + r * fs, V, yf, p);                            \
            hop<R, MU, true>(w, p, nb_sign<R>(ef), acc[r]);                   \
        }                                                                     \
        const int eb = nbr_at(nbr, 2 * MU + 1, V, x);                             \
        const long yb = nb_index(eb);                                         \
        Link<LF>::load(U, V, MU, yb, w);                                      \
        _Pragma("unroll") for (int r = 0; r < NR; ++r) {                      \
            Spin<S>::load(inb + r * fs, V, yb, p);                            \
            hop<R, MU, false>(w, p, nb_sign<R>(eb), acc[r]);                  \
        }                                                                     \
    }
    DFL_HOP_MU(0)
    DFL_HOP_MU(1)
    DFL_HOP_MU(2)
    DFL_HOP_MU(3)
#undef DFL_HOP_MU
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        cx<R> o[12];
        Spin<S>::load(inb + r * fs, V, x, p);
        clover_apply<CF>(clo, V, x, p, o);
#pragma unroll
        for (int k = 0; k < 12; ++k) o[k] = o[k] - kappa * acc[r][k];
        Spin<S>::store(outb + r * fs, V, x, o);
    }
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
    int done = 0;
    constexpr int NR = sizeof(R) == 8 ? 2 : 4;
    if (nrhs >= NR) {
        int ng = nrhs / NR;
        auto [fl, by, un] = work(ng * NR);
        ProfScope ps(PROF_DIRAC, s, fl, by, un);
        k_dirac<S, R, LF, CF, NR><<<dim3(nblocks(V, BS), ng), BS, 0, s>>>(in, out, U, C, f->nbr, V, kappa, 0);
        done = ng * NR;
    }
    if (done < nrhs) {
        auto [fl, by, un] = work(nrhs - done);
        ProfScope ps(PROF_DIRAC, s, fl, by, un);
        k_dirac<S, R, LF, CF, 1><<<dim3(nblocks(V, BS), nrhs - done), BS, 0, s>>>(in, out, U, C, f->nbr, V, kappa,
                                                                                  done);
    }
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
