// Source and sink smearing (section 2.3): Gaussian smearing of quark fields
// with APE-smeared spatial links in the Laplacian.  The paper takes the
// parameters from earlier work; here they are arguments.
//
// APE step, for each spatial direction i and site x:
//   V = (1 - alpha) U_i(x) + (alpha / 4) sum_{j != i spatial}
//         [ U_j(x) U_i(x + j) U_j(x + i)^+ + U_j(x - j)^+ U_i(x - j) U_j(x - j + i) ],
//   U'_i(x) = W / det(W)^(1/3),  W = V (V^+ V)^(-1/2)  (polar factor; the cube
//   root is exp(i arg(det W) / 3), arg in (-pi, pi]).
// W is found by the Newton iteration W <- (W + W^{-+}) / 2, which converges
// quadratically to the polar factor of a nonsingular matrix; for 3 x 3
// matrices W^{-+} = conj(cof(W) / det(W)) with cof(W) the cofactor matrix,
// whose rows are cross products of the other two rows.
//
// Gaussian step: psi'(x) = [psi(x) + kappa sum_{i spatial} (U'_i(x) psi(x + i)
//   + U'_i(x - i)^+ psi(x - i))] / (1 + 6 kappa), colour only, each timeslice
// on its own.  Links and vectors are FP64 in the internal site order; the
// neighbour table supplies x +- i (spatial hops carry no boundary sign).
#include <cmath>

#include "internal.h"

namespace dfl {

namespace {

using cd = cx<double>;

__device__ inline void m_load(const double2 *U, long V, int i, unsigned x, cd m[9]) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 t = U[((size_t)i * 9 + k) * V + x];
        m[k] = {t.x, t.y};
    }
}
// c = a b, a b^+, a^+ b
__device__ inline void m_mul(const cd a[9], const cd b[9], cd c[9]) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) c[3 * r + q] = cmac(cmac(a[3 * r] * b[q], a[3 * r + 1], b[3 + q]), a[3 * r + 2], b[6 + q]);
}
__device__ inline void m_mul_dag(const cd a[9], const cd b[9], cd c[9]) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q)
            c[3 * r + q] = cmac(cmac(a[3 * r] * conj(b[3 * q]), a[3 * r + 1], conj(b[3 * q + 1])), a[3 * r + 2],
                                conj(b[3 * q + 2]));
}
__device__ inline void m_dag_mul(const cd a[9], const cd b[9], cd c[9]) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) c[3 * r + q] = cmacc(cmacc(cmulc(a[r], b[q]), a[3 + r], b[3 + q]), a[6 + r], b[6 + q]);
}

// projection onto SU(3): polar factor (Newton) divided by a cube root of its determinant
__device__ inline void project_su3(cd w[9]) {
    for (int it = 0; it < 40; ++it) {
        cd cof[9];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const cd *u = w + 3 * ((r + 1) % 3), *v = w + 3 * ((r + 2) % 3);
            cof[3 * r] = cmac(u[1] * v[2], -u[2], v[1]);
            cof[3 * r + 1] = cmac(u[2] * v[0], -u[0], v[2]);
            cof[3 * r + 2] = cmac(u[0] * v[1], -u[1], v[0]);
        }
        const cd det = cmac(cmac(w[0] * cof[0], w[1], cof[1]), w[2], cof[2]);
        const double dn = 1.0 / norm2(det);
        // conj(cof / det) = conj(cof) det / |det|^2
        double change = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const cd inv = dn * (conj(cof[k]) * det);
            const cd nw = 0.5 * (w[k] + inv);
            change += norm2(nw - w[k]);
            w[k] = nw;
        }
        if (change < 1e-30) break;
    }
    cd c0[3];
    const cd *u = w + 3, *v = w + 6;
    c0[0] = cmac(u[1] * v[2], -u[2], v[1]);
    c0[1] = cmac(u[2] * v[0], -u[0], v[2]);
    c0[2] = cmac(u[0] * v[1], -u[1], v[0]);
    const cd det = cmac(cmac(w[0] * c0[0], w[1], c0[1]), w[2], c0[2]);
    const double th = atan2(det.im, det.re) / 3.0;
    const cd ph = {cos(th), -sin(th)};
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = w[k] * ph;
}

// one APE step on the spatial links Uin [3][9][V] -> Uout (internal order);
// each XCD takes a contiguous range of site tiles, so that the staples'
// neighbour links come through its L2
__global__ void __launch_bounds__(128) k_ape_step(const double2 *__restrict__ Uin, double2 *__restrict__ Uout,
                                                  const int *__restrict__ nbr, long V, double alpha) {
    unsigned bx, by;
    xcd_order(bx, by);
    const long xl = (long)bx * blockDim.x + threadIdx.x;
    if (xl >= V) return;
    const unsigned x = (unsigned)xl;
    for (int i = 0; i < 3; ++i) {
        const int mi = i + 1;
        cd acc[9], a[9], b[9], c[9], t[9];
        m_load(Uin, V, i, x, a);
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] = (1.0 - alpha) * a[k];
        const unsigned xpi = nb_index(nbr_at(nbr, 2 * mi, V, x));
        for (int j = 0; j < 3; ++j) {
            if (j == i) continue;
            const int mj = j + 1;
            const unsigned xpj = nb_index(nbr_at(nbr, 2 * mj, V, x));
            const unsigned xmj = nb_index(nbr_at(nbr, 2 * mj + 1, V, x));
            const unsigned xmjpi = nb_index(nbr_at(nbr, 2 * mi, V, xmj));
            // U_j(x) U_i(x + j) U_j(x + i)^+
            m_load(Uin, V, j, x, a);
            m_load(Uin, V, i, xpj, b);
            m_mul(a, b, t);
            m_load(Uin, V, j, xpi, c);
            m_mul_dag(t, c, a);
#pragma unroll
            for (int k = 0; k < 9; ++k) acc[k] = rmac(acc[k], 0.25 * alpha, a[k]);
            // U_j(x - j)^+ U_i(x - j) U_j(x - j + i)
            m_load(Uin, V, j, xmj, a);
            m_load(Uin, V, i, xmj, b);
            m_dag_mul(a, b, t);
            m_load(Uin, V, j, xmjpi, c);
            m_mul(t, c, a);
#pragma unroll
            for (int k = 0; k < 9; ++k) acc[k] = rmac(acc[k], 0.25 * alpha, a[k]);
        }
        project_su3(acc);
#pragma unroll
        for (int k = 0; k < 9; ++k) Uout[((size_t)i * 9 + k) * V + x] = make_double2(acc[k].re, acc[k].im);
    }
}

// one Gaussian step on n internal FP64 vectors ([n][12][V]): one thread per
// site and vector; the workgroups of one site tile (all vectors) run back to
// back on one XCD, so that they share the tile's links through its L2
// (threads that take two vectors to load the links once need 256 registers)
__global__ void __launch_bounds__(128) k_gauss_step(const double2 *__restrict__ in, double2 *__restrict__ out,
                                                    const double2 *__restrict__ U, const int *__restrict__ nbr, long V,
                                                    double kappa, double norm) {
    unsigned bx, by;
    xcd_order(bx, by);
    const long xl = (long)bx * blockDim.x + threadIdx.x;
    if (xl >= V) return;
    const unsigned x = (unsigned)xl;
    const double2 *src = in + (size_t)by * 12 * V;
    cd acc[12], p[12], w[9];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const double2 t = src[(size_t)k * V + x];
        acc[k] = {t.x, t.y};
    }
    for (int i = 0; i < 3; ++i) {
        const int mi = i + 1;
        const unsigned yf = nb_index(nbr_at(nbr, 2 * mi, V, x));
        const unsigned yb = nb_index(nbr_at(nbr, 2 * mi + 1, V, x));
        m_load(U, V, i, x, w);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double2 t = src[(size_t)k * V + yf];
            p[k] = {t.x, t.y};
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                cd v = cmac(cmac(w[3 * a] * p[3 * s], w[3 * a + 1], p[3 * s + 1]), w[3 * a + 2], p[3 * s + 2]);
                acc[3 * s + a] = rmac(acc[3 * s + a], kappa, v);
            }
        m_load(U, V, i, yb, w);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double2 t = src[(size_t)k * V + yb];
            p[k] = {t.x, t.y};
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                cd v = cmacc(cmacc(cmulc(w[a], p[3 * s]), w[3 + a], p[3 * s + 1]), w[6 + a], p[3 * s + 2]);
                acc[3 * s + a] = rmac(acc[3 * s + a], kappa, v);
            }
    }
    double2 *dst = out + (size_t)by * 12 * V;
#pragma unroll
    for (int k = 0; k < 12; ++k) dst[(size_t)k * V + x] = make_double2(norm * acc[k].re, norm * acc[k].im);
}

// canonical [V][3][3][3] (lexicographic site, spatial direction i = mu - 1)
__global__ void k_ape_export(const double2 *__restrict__ U, double2 *__restrict__ out, const int *__restrict__ lex_of,
                             long V) {
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= V) return;
    const long lex = lex_of[x];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 9; ++k) out[((size_t)lex * 3 + i) * 9 + k] = U[((size_t)i * 9 + k) * V + x];
}

}  // namespace
}  // namespace dfl

using namespace dfl;

extern "C" int qcd_field_ape_smear(qcd_field f, double alpha, int n_iter, hipStream_t s) {
    if (!f || n_iter < 0 || !std::isfinite(alpha)) return set_error(QCD_EINVAL, "bad arguments to qcd_field_ape_smear");
    const long V = f->g.V;
    const size_t bytes = sizeof(double2) * 27 * (size_t)V;
    if (!f->Uape && !dev_alloc(f->device, (void **)&f->Uape, bytes))
        return set_error(QCD_ENOMEM, "device allocation of the smeared links failed");
    // spatial links of the FP64 copy, then n_iter steps ping-ponging through
    // the handle's scratch
    const double2 *U64 = static_cast<const double2 *>(f->U[LNK_F64]);
    DFL_HIP(hipMemcpyAsync(f->Uape, U64 + (size_t)9 * V, bytes, hipMemcpyDeviceToDevice, s));
    if (n_iter > 0) {
        void *w;
        DFL_TRY(field_buffer(f, BUF_APPLY, bytes, &w));
        double2 *a = static_cast<double2 *>(f->Uape), *b = static_cast<double2 *>(w);
        ProfScope ps(PROF_OTHER, s);
        for (int it = 0; it < n_iter; ++it) {
            k_ape_step<<<nblocks(V, 128), 128, 0, s>>>(a, b, f->nbr, V, alpha);
            std::swap(a, b);
        }
        DFL_HIP(hipGetLastError());
        if (a != f->Uape) DFL_HIP(hipMemcpyAsync(f->Uape, a, bytes, hipMemcpyDeviceToDevice, s));
    }
    return 0;
}

extern "C" int qcd_field_get_ape_links(qcd_field f, void *links, hipStream_t s) {
    if (!f || !links) return set_error(QCD_EINVAL, "bad arguments to qcd_field_get_ape_links");
    if (!f->Uape) return set_error(QCD_ENOTSET, "no smeared links: call qcd_field_ape_smear first");
    k_ape_export<<<nblocks(f->g.V, 256), 256, 0, s>>>(static_cast<const double2 *>(f->Uape),
                                                      static_cast<double2 *>(links), f->lex_of, f->g.V);
    DFL_HIP(hipGetLastError());
    return 0;
}

extern "C" int gauss_smear(qcd_field f, const void *in, void *out, int nrhs, qcd_prec io, double kappa_g, int n_iter,
                           hipStream_t s) {
    if (!f || !in || !out || nrhs <= 0 || n_iter < 0 || !std::isfinite(kappa_g))
        return set_error(QCD_EINVAL, "bad arguments to gauss_smear");
    if (io != QCD_F64 && io != QCD_F32) return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    if (!f->Uape) return set_error(QCD_ENOTSET, "no smeared links: call qcd_field_ape_smear first");
    if (1 + 6 * kappa_g == 0) return set_error(QCD_EINVAL, "kappa_g = -1/6 is singular");
    const long V = f->g.V;
    const size_t nb = spinor_bytes(QCD_F64, V) * nrhs;
    void *ws;
    DFL_TRY(field_buffer(f, BUF_SAP_IO, 2 * nb, &ws));
    double2 *a = static_cast<double2 *>(ws), *b = a + (size_t)12 * V * nrhs;
    DFL_TRY(pack_spinor(f, in, io, a, QCD_F64, nrhs, s));
    {
        ProfScope ps(PROF_OTHER, s);
        for (int it = 0; it < n_iter; ++it) {
            k_gauss_step<<<dim3(nblocks(V, 128), nrhs), 128, 0, s>>>(a, b, static_cast<const double2 *>(f->Uape),
                                                                      f->nbr, V, kappa_g, 1.0 / (1 + 6 * kappa_g));
            std::swap(a, b);
        }
        DFL_HIP(hipGetLastError());
    }
    return unpack_spinor(f, a, QCD_F64, out, io, nrhs, s);
}
