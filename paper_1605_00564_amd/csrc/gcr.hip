// Flexible, restarted GCR for M x = b with the Schwarz preconditioner and
// optional block-local deflation (section 2.2 of the paper: right
// preconditioned GCR on D M_SAP phi = eta with psi = M_SAP phi; deflated
// solution psi = chi + Phi A^{-1} Phi^+ eta).
//
// Mixed precision: the outer loop keeps x and r = b - M x in FP64 and
// recomputes r with the FP64 operator at every restart; inside a cycle the
// residual rho and the Krylov pairs (z_k, w_k) are stored in FP32 (or FP64
// when the preconditioner runs in FP64), and every Gram-Schmidt coefficient
// is accumulated in FP64.
#include <type_traits>
#include <cmath>

#include "blas.h"
#include "dflint.h"

namespace dfl {

namespace {

int fetch(qcd_field f, const double *dev, size_t count, hipStream_t s, std::vector<double> &host) {
    host.resize(count);
    if (count > 4096) return set_error(QCD_EINVAL, "too many right-hand sides in one batch (max 4096)");
    DFL_HIP(hipMemcpyAsync(f->hp, dev, count * sizeof(double), hipMemcpyDeviceToHost, s));
    DFL_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < count; ++i) host[i] = f->hp[i];
    return 0;
}

template <class E>
struct Inner;
template <>
struct Inner<float4> {
    static constexpr qcd_prec vec = QCD_F32;
    static long ne(long V) { return 6 * V; }
};
template <>
struct Inner<double2> {
    static constexpr qcd_prec vec = QCD_F64;
    static long ne(long V) { return 12 * V; }
};

// rho (inner precision) = r (FP64)
inline int to_inner(const double2 *r, float4 *rho, long V, int n, hipStream_t s) {
    return blas_d2f(r, rho, V, n, s);
}
inline int to_inner(const double2 *r, double2 *rho, long V, int n, hipStream_t s) {
    DFL_HIP(hipMemcpyAsync(rho, r, sizeof(double2) * 12 * V * n, hipMemcpyDeviceToDevice, s));
    return 0;
}
inline int accum(double2 *x, const float4 *Z, long V, int n, int k, const double *alpha, hipStream_t s) {
    return blas_accum_f(x, Z, V, n, k, alpha, 2 * NKV_MAX, s);
}
inline int accum(double2 *x, const double2 *Z, long V, int n, int k, const double *alpha, hipStream_t s) {
    return blas_accum_d(x, Z, 12 * V, n, k, alpha, 2 * NKV_MAX, s);
}

template <class E>
int gcr_run(qcd_field f, const qcd_gcr *p, const double2 *b, double2 *x, int n, qcd_info *info, hipStream_t s) {
    const long V = f->g.V;
    const long ne = Inner<E>::ne(V);
    const long ne64 = 12 * V;
    const int nkv = p->nkv;
    const qcd_prec vin = Inner<E>::vec;
    const qcd_prec opst = vin == QCD_F64 ? QCD_F64 : (p->sap.storage == QCD_F64 ? QCD_F32 : p->sap.storage);
    const size_t vbytes = sizeof(E) * ne;  // one rhs

    // work space: Z[nkv][n], W[nkv][n], rho[n], tmp[n] (inner); r (FP64)
    void *wp, *wio;
    DFL_TRY(field_buffer(f, BUF_GCR, vbytes * n * (2 * (size_t)nkv + 2), &wp));
    DFL_TRY(field_buffer(f, BUF_GCR_IO, sizeof(double2) * ne64 * n, &wio));
    E *Z = static_cast<E *>(wp);
    E *W = Z + (size_t)nkv * n * ne;
    E *rho = W + (size_t)nkv * n * ne;
    E *tmp = rho + (size_t)n * ne;
    double2 *r = static_cast<double2 *>(wio);
    Scal sc;
    void *sp;
    DFL_TRY(field_buffer(f, BUF_RED, scalar_bytes(n), &sp));
    DFL_TRY(scalar_buffers_at(sp, n, sc));

    // Without host synchronisation (stream capture) the norms stay on the
    // device: ||b||^2 in sc.bn2, the final ||r||^2 in sc.red, read by the
    // caller after the captured work ran; iteration counts are fixed.
    const bool ns = nosync();
    if (ns && p->fixed_iters <= 0) return set_error(QCD_EINVAL, "solves without synchronisation need fixed_iters");
    std::vector<double> h(n, 1.0);
    DFL_TRY(blas_norm2(b, ne64, n, sc.part, ns ? sc.bn2 : sc.red, s));
    if (!ns) DFL_TRY(fetch(f, sc.red, n, s, h));
    std::vector<double> bn(n);
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(h[i])) return set_error(QCD_ENAN, "NaN or Inf in the right-hand side");
        bn[i] = std::sqrt(h[i]);
    }

    auto converged = [&](const std::vector<double> &res) {
        for (int i = 0; i < n; ++i)
            if (res[i] > p->res * bn[i]) return false;
        return true;
    };
    // initial guess x = 0, r = b
    std::vector<double> rn(n);
    rn = bn;
    bool done = p->fixed_iters <= 0 && converged(rn);
    // with deflation the first low-mode correction reads b and writes x
    // itself, so x = 0 and r = b need not be stored
    bool x_zero = p->dfl && !done;
    if (!x_zero) {
        DFL_TRY(blas_zero(x, ne64, n, s));
        DFL_HIP(hipMemcpyAsync(r, b, sizeof(double2) * ne64 * n, hipMemcpyDeviceToDevice, s));
    }
    // With deflation every cycle starts with the low-mode correction
    // x += Phi A^{-1} Phi^+ r (eq. deflsoln applied to the current residual):
    // the search directions M P_R z = P_L M z only span range(P_L), so the
    // part of r outside it, left by inexact little solves and FP32 rounding,
    // is removed here, in FP64, before the next cycle.
    // FP32 Krylov vectors: the FP64 residual kernel also writes rho, the
    // residual rounded to FP32, which the next cycle starts from
    float4 *rho32 = nullptr;
    if constexpr (std::is_same_v<E, float4>) rho32 = rho;
    bool rho_ready = false;
    auto low_mode_correction = [&]() -> int {
        // without host polls the correction's little solve runs one
        // Krylov cycle of 12 iterations (or little_maxit if larger): the
        // Schur-complement little GCR reaches about 1e-8 there on 4^4
        // blocks, where the P_R budget of a few iterations leaves ~1e-3
        DFL_TRY(dfl_low_mode(p->dfl, x_zero ? b : r, x, n, p->little_tol,
                             ns ? std::max(p->little_maxit, LOW_MODE_FIXED_ITERS) : std::max(p->little_maxit, 200),
                             x_zero, s));
        x_zero = false;
        DFL_TRY(dirac_resid(f, x, b, r, n, sc.red, s, rho32));
        rho_ready = rho32 != nullptr;
        if (ns) return 0;
        DFL_TRY(fetch(f, sc.red, n, s, h));
        for (int i = 0; i < n; ++i) rn[i] = std::sqrt(h[i]);
        return 0;
    };

    const int limit = p->fixed_iters > 0 ? p->fixed_iters : p->nmx;
    // A cycle ends once its residual has dropped by inner_rel: with FP32
    // Krylov vectors that is their precision limit; with deflation (in
    // either precision) the next cycle's low-mode correction removes what
    // the inexact little solves leave outside range(P_L), which the
    // search directions cannot reach.
    const double inner_rel = (vin == QCD_F64 && !p->dfl) ? 0.0 : 1e-6;
    int iters = 0;
    while (!done && iters < limit) {
        if (p->dfl) {
            DFL_TRY(low_mode_correction());
            if (p->fixed_iters <= 0 && converged(rn)) break;
        }
        if (!rho_ready) DFL_TRY(to_inner(r, rho, V, n, s));
        rho_ready = false;
        const std::vector<double> rstart = rn;
        int k = 0;
        while (k < nkv && iters < limit) {
            E *zk = Z + (size_t)k * n * ne;
            E *wk = W + (size_t)k * n * ne;
            DFL_TRY(sap_internal(f, &p->sap, rho, zk, n, s));
            if (p->dfl) DFL_TRY(dfl_project_R(p->dfl, zk, tmp, n, vin, opst, p->little_maxit, s));
            DFL_TRY(dirac_internal(f, zk, wk, n, vin, opst, s));
            int bstride = 2;
            if (k > 0) bstride = blas_multidot<E>(W, ne, n, k, sc.part, sc.red2, s);
            if (bstride < 0) return bstride;
            DFL_TRY(blas_gs_sub<E>(W, rho, ne, n, k, sc.red2, bstride, sc.part, sc.red, s));
            DFL_TRY(gcr_scalars(sc.red2, bstride, sc.red, n, k, sc.R, sc.cvec, sc.coef, s));
            DFL_TRY(blas_scal_update<E>(wk, rho, ne, n, sc.coef, sc.part, sc.red, s));
            ++k;
            ++iters;
            if (p->fixed_iters <= 0) {
                DFL_TRY(fetch(f, sc.red, n, s, h));
                bool inner_done = true;
                for (int i = 0; i < n; ++i) {
                    if (!std::isfinite(h[i])) return set_error(QCD_ENAN, "NaN in the GCR residual");
                    const double tgt = std::max(p->res * bn[i], inner_rel * rstart[i]);
                    if (std::sqrt(h[i]) > tgt) inner_done = false;
                }
                if (inner_done) break;
            }
        }
        DFL_TRY(gcr_trisolve(sc.R, sc.cvec, n, k, sc.alpha, s));
        DFL_TRY(accum(x, Z, V, n, k, sc.alpha, s));
        // without deflation the next cycle starts from this residual
        DFL_TRY(dirac_resid(f, x, b, r, n, sc.red, s, p->dfl ? nullptr : rho32));
        rho_ready = !p->dfl && rho32 != nullptr;
        if (!ns) {
            DFL_TRY(fetch(f, sc.red, n, s, h));
            for (int i = 0; i < n; ++i) {
                if (!std::isfinite(h[i])) return set_error(QCD_ENAN, "NaN in the recomputed residual");
                rn[i] = std::sqrt(h[i]);
            }
        }
        if (p->fixed_iters > 0 ? iters >= p->fixed_iters : converged(rn)) done = true;
    }
    if (ns) return 0;
    bool all = true;
    for (int i = 0; i < n; ++i) {
        const double rel = bn[i] > 0 ? rn[i] / bn[i] : 0.0;
        const bool ok = rel <= p->res;
        all = all && ok;
        if (info) info[i] = qcd_info{ok ? 0 : QCD_NOCONV, iters, rel};
    }
    return all ? 0 : QCD_NOCONV;
}

}  // namespace

int gcr_internal(qcd_field f, const qcd_gcr *p, const double2 *b, double2 *x, int n, qcd_info *info,
                 hipStream_t s) {
    if (p->nkv < 1 || p->nkv > NKV_MAX) return set_error(QCD_EINVAL, "nkv must be in 1..32");
    if (p->fixed_iters <= 0 && (p->nmx < 1 || !(p->res > 0)))
        return set_error(QCD_EINVAL, "need nmx >= 1 and res > 0 (or fixed_iters > 0)");
    if (p->dfl && dfl_field(p->dfl) != f) return set_error(QCD_EINVAL, "deflation handle belongs to another field");
    if (p->sap.storage == QCD_F64) return gcr_run<double2>(f, p, b, x, n, info, s);
    return gcr_run<float4>(f, p, b, x, n, info, s);
}

}  // namespace dfl

using namespace dfl;

extern "C" int gcr_solve(qcd_field f, const qcd_gcr *p, const void *b, void *x, int nrhs, qcd_prec io,
                         qcd_info *info, hipStream_t s) {
    if (!f || !p || !b || !x || nrhs <= 0) return set_error(QCD_EINVAL, "bad arguments to gcr_solve");
    if (io != QCD_F64 && io != QCD_F32) return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    const size_t nb = spinor_bytes(QCD_F64, f->g.V) * nrhs;
    void *ws;
    DFL_TRY(field_buffer(f, BUF_APPLY, 2 * nb, &ws));
    double2 *b64 = static_cast<double2 *>(ws);
    double2 *x64 = b64 + (size_t)12 * f->g.V * nrhs;
    DFL_TRY(pack_spinor(f, b, io, b64, QCD_F64, nrhs, s));
    int rc = gcr_internal(f, p, b64, x64, nrhs, info, s);
    if (rc < 0) return rc;
    DFL_TRY(unpack_spinor(f, x64, QCD_F64, x, io, nrhs, s));
    DFL_HIP(hipStreamSynchronize(s));
    return rc;
}
