// All-mode averaging driver (section 2.1): truncated ("sloppy") solves for
// the 12 spin-colour point sources of every source position in G, exact
// solves for the flagged subset, many right-hand sides per GCR batch.
#include <algorithm>
#include <cmath>

#include "blas.h"

namespace dfl {

// b[r] = point source at lexicographic site lex[r], spin-colour sc[r] (FP64 internal)
__global__ void k_point_sources(double2 *__restrict__ b, const int *__restrict__ src, const int *__restrict__ int_of,
                                long V, int n) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int lex = src[2 * r], sc = src[2 * r + 1];
    b[((size_t)r * 12 + sc) * V + int_of[lex]] = make_double2(1.0, 0.0);
}

namespace {

// Positions must differ by translations that map the block checkerboard onto
// itself: whole blocks in every direction with an even number of block steps.
int check_positions(const Geom &g, const int *pos, int npos) {
    for (int i = 0; i < npos; ++i) {
        int steps = 0;
        for (int m = 0; m < 4; ++m) {
            const int v = pos[4 * i + m];
            if (v < 0 || v >= g.L[m]) return set_error(QCD_EINVAL, "source position outside the lattice");
            const int dlt = ((v - pos[m]) % g.L[m] + g.L[m]) % g.L[m];
            if (dlt % g.b[m])
                return set_error(QCD_EGEOM, "source positions are not related by whole Schwarz blocks");
            steps += dlt / g.b[m];
        }
        if (steps % 2)
            return set_error(QCD_EGEOM, "source positions change the colour of the block checkerboard");
    }
    return 0;
}

// default right-hand sides per batch: as many as fit a modest share of HBM
int pick_batch(qcd_field f, const qcd_gcr &p, int want) {
    if (want > 0) return want;
    size_t freeb = 0, total = 0;
    if (hipMemGetInfo(&freeb, &total) != hipSuccess) {
        (void)hipGetLastError();
        return 12;
    }
    freeb += ws_cached_bytes(f->device);   // cached workspace is reusable
    const size_t V = f->g.V;
    const size_t inner = p.sap.storage == QCD_F64 ? 192 : 96;
    const size_t per = V * (inner * (2 * (size_t)p.nkv + 3) + 192 * 5);
    size_t n = (size_t)(0.6 * (double)freeb) / std::max<size_t>(per, 1);
    n = std::min<size_t>(std::max<size_t>(n, 1), 48);
    if (n >= 12) n -= n % 12;
    return (int)n;
}

int solve_set(qcd_field f, const qcd_gcr &p, const std::vector<int> &lex_sc, void *const *outs, qcd_prec io,
              qcd_info *info, int batch, hipStream_t s, int &status) {
    const long V = f->g.V;
    const int total = (int)lex_sc.size() / 2;
    const int nb = std::max(1, std::min(batch, total));
    void *ws;
    DFL_TRY(field_buffer(f, BUF_AMA, (sizeof(double2) * 12 * V) * 2 * nb + sizeof(int) * 2 * nb, &ws));
    double2 *b64 = static_cast<double2 *>(ws);
    double2 *x64 = b64 + (size_t)12 * V * nb;
    int *dsrc = reinterpret_cast<int *>(x64 + (size_t)12 * V * nb);
    const size_t cbytes = (io == QCD_F64 ? 16 : 8) * (size_t)12 * V;  // one canonical vector
    for (int r0 = 0; r0 < total; r0 += nb) {
        const int n = std::min(nb, total - r0);
        DFL_TRY(blas_zero<double2>(b64, 12 * V, n, s));
        DFL_HIP(hipMemcpyAsync(dsrc, lex_sc.data() + 2 * r0, sizeof(int) * 2 * n, hipMemcpyHostToDevice, s));
        k_point_sources<<<(n + 63) / 64, 64, 0, s>>>(b64, dsrc, f->int_of, V, n);
        DFL_HIP(hipGetLastError());
        const int rc = gcr_internal(f, &p, b64, x64, n, info ? info + r0 : nullptr, s);
        if (rc < 0) return rc;
        if (rc == QCD_NOCONV) status = QCD_NOCONV;
        // a position's spin-colour solutions are contiguous in its output:
        // one unpack per run of them
        for (int r = 0; r < n;) {
            const int g = (r0 + r) / 12, sc = (r0 + r) % 12;
            const int run = std::min(12 - sc, n - r);
            char *dst = static_cast<char *>(outs[g]) + sc * cbytes;
            DFL_TRY(unpack_spinor(f, x64 + (size_t)r * 12 * V, QCD_F64, dst, io, run, s));
            r += run;
        }
    }
    return 0;
}

}  // namespace
}  // namespace dfl

using namespace dfl;

extern "C" int ama_solve(qcd_field f, const qcd_ama *a, void *const *x_sloppy, void *const *x_exact, qcd_prec io,
                         qcd_info *info_sloppy, qcd_info *info_exact, hipStream_t s) {
    if (!f || !a || a->npos < 1 || !a->pos || !x_sloppy) return set_error(QCD_EINVAL, "bad arguments to ama_solve");
    if (io != QCD_F64 && io != QCD_F32) return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    DFL_TRY(check_positions(f->g, a->pos, a->npos));
    const Geom &g = f->g;
    std::vector<int> sl, ex;
    int nex = 0;
    for (int i = 0; i < a->npos; ++i) {
        const int *c = a->pos + 4 * i;
        const int lex = c[3] + g.L[3] * (c[2] + g.L[2] * (c[1] + g.L[1] * c[0]));
        for (int sc = 0; sc < 12; ++sc) {
            sl.push_back(lex);
            sl.push_back(sc);
        }
        if (a->exact && a->exact[i]) {
            ++nex;
            for (int sc = 0; sc < 12; ++sc) {
                ex.push_back(lex);
                ex.push_back(sc);
            }
        }
    }
    if (nex && !x_exact) return set_error(QCD_EINVAL, "exact positions flagged but no output buffers");
    int status = 0;
    DFL_TRY(solve_set(f, a->sloppy, sl, x_sloppy, io, info_sloppy, pick_batch(f, a->sloppy, a->batch), s, status));
    if (nex)
        DFL_TRY(solve_set(f, a->exact_params, ex, x_exact, io, info_exact, pick_batch(f, a->exact_params, a->batch), s,
                          status));
    DFL_HIP(hipStreamSynchronize(s));
    return status;
}
