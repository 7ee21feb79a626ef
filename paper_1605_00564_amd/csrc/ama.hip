// All-mode averaging driver (section 2.1): truncated ("sloppy") solves for
// every source of the set G, exact solves for the flagged subset F of G,
// many right-hand sides per GCR batch.  A source is 12 point sources at a
// position (one per spin-colour), Z2-noise vectors, 12 sequential sources
// built from forward solutions (section 2.3), or caller vectors.  Sloppy
// solves with a fixed iteration count (section 3.5, Table 3) replay one
// captured HIP graph per batch size; a solution that the fixed count left
// above the target residual is solved again with the residual-stopping
// solver.
#include <algorithm>
#include <cmath>

#include "batch_rule.h"
#include "blas.h"

namespace dfl {

// b[slot] = point source at lexicographic site lex, spin-colour sc (FP64
// internal, b zeroed before); src holds (slot, lex, sc) triplets
__global__ void k_point_sources(double2 *__restrict__ b, const int *__restrict__ src, const int *__restrict__ int_of,
                                long V, int n) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int slot = src[3 * r], lex = src[3 * r + 1], sc = src[3 * r + 2];
    b[((size_t)slot * 12 + sc) * V + int_of[lex]] = make_double2(1.0, 0.0);
}

// right-hand sides per launch.  Without a request (want = 0): as many as
// 60% of the available device memory holds for these parameters, at most 48
// and a multiple of 12 when possible.  A request is lowered only when 90% of
// the available memory cannot hold it, and then to an even count (the
// Schwarz and stencil kernels take right-hand sides in pairs).  Available:
// free device memory, the library's cached workspace and the handle's own
// buffers except slot `busy` (one the caller keeps using).  Memory only: per
// right-hand side the results do not depend on the batch.
int pick_batch(qcd_field f, const qcd_gcr &p, int want, int busy) {
    size_t freeb = 0, total = 0;
    if (hipMemGetInfo(&freeb, &total) != hipSuccess) {
        (void)hipGetLastError();
        return want > 0 ? want : 12;
    }
    freeb += ws_cached_bytes(f->device);
    for (int k = 0; k < (int)(sizeof(f->buf_bytes) / sizeof(f->buf_bytes[0])); ++k)
        if (k != busy) freeb += f->buf_bytes[k];
    const size_t V = f->g.V;
    const size_t inner = p.sap.storage == QCD_F64 ? 192 : 96;
    return batch_rule(freeb, V * (inner * (2 * (size_t)p.nkv + 3) + 192 * 5), want);
}

namespace {

// one right-hand side of a set: vector k of source src
struct Rhs {
    int src, k;
};

int nvec_of(const qcd_source &q) { return (q.kind == QCD_SRC_POINT || q.kind == QCD_SRC_SEQ) ? 12 : q.nvec; }

int lex_of_pos(const Geom &g, const int *c) { return c[3] + g.L[3] * (c[2] + g.L[2] * (c[1] + g.L[1] * c[0])); }

// Every source is well formed, and point-source positions differ by
// translations that map the block checkerboard onto itself (whole blocks in
// every direction, an even number of block steps), so that M_SAP is
// covariant under the translations relating them (section 2.2).
int check_set(const Geom &g, const qcd_ama *a) {
    if (!a || a->nsrc < 1 || !a->src) return set_error(QCD_EINVAL, "an AMA set needs nsrc >= 1 sources");
    if (a->sloppy_out != QCD_F64 && a->sloppy_out != QCD_F32)
        return set_error(QCD_EINVAL, "sloppy_out must be F64 or F32");
    const int *ref = nullptr;
    for (int i = 0; i < a->nsrc; ++i) {
        const qcd_source &q = a->src[i];
        switch (q.kind) {
            case QCD_SRC_POINT: {
                for (int m = 0; m < 4; ++m)
                    if (q.pos[m] < 0 || q.pos[m] >= g.L[m])
                        return set_error(QCD_EINVAL, "source position outside the lattice");
                if (!ref) {
                    ref = q.pos;
                    break;
                }
                int steps = 0;
                for (int m = 0; m < 4; ++m) {
                    const int dlt = ((q.pos[m] - ref[m]) % g.L[m] + g.L[m]) % g.L[m];
                    if (dlt % g.b[m])
                        return set_error(QCD_EGEOM, "source positions are not related by whole Schwarz blocks");
                    steps += dlt / g.b[m];
                }
                if (steps % 2)
                    return set_error(QCD_EGEOM, "source positions change the colour of the block checkerboard");
                break;
            }
            case QCD_SRC_Z2:
                if (q.nvec < 1 || q.index < 0) return set_error(QCD_EINVAL, "Z2 source needs nvec >= 1, index >= 0");
                break;
            case QCD_SRC_SEQ:
                if (!q.vec) return set_error(QCD_EINVAL, "sequential source without forward solutions");
                if (q.mu < 0 || q.mu > 3) return set_error(QCD_EINVAL, "sequential source: mu must be 0..3");
                if (q.t_sink < 0 || q.t_sink >= g.L[0])
                    return set_error(QCD_EINVAL, "sequential source: sink timeslice outside the lattice");
                break;
            case QCD_SRC_VEC:
                if (!q.vec || q.nvec < 1) return set_error(QCD_EINVAL, "vector source needs vec and nvec >= 1");
                break;
            default: return set_error(QCD_EINVAL, "unknown source kind");
        }
    }
    return 0;
}

// bytes of one canonical vector at precision p
size_t canon_bytes(qcd_prec p, long V) { return (p == QCD_F64 ? 16 : 8) * (size_t)12 * V; }

// b64[0..n) = sources of list[r0 .. r0+n)
int build_sources(qcd_field f, const qcd_ama &a, const std::vector<Rhs> &list, int r0, int n, double2 *b64,
                  int *dsrc, qcd_prec io, hipStream_t s) {
    const Geom &g = f->g;
    const long V = g.V;
    std::vector<int> pts;
    for (int r = 0; r < n; ++r) {
        const Rhs &e = list[r0 + r];
        const qcd_source &q = a.src[e.src];
        double2 *b = b64 + (size_t)r * 12 * V;
        switch (q.kind) {
            case QCD_SRC_POINT:
                DFL_TRY(blas_zero<double2>(b, 12 * V, 1, s));
                pts.insert(pts.end(), {r, lex_of_pos(g, q.pos), e.k});
                break;
            case QCD_SRC_Z2: DFL_TRY(z2_source_internal(f, q.seed, q.index + e.k, b, s)); break;
            case QCD_SRC_SEQ:
                DFL_TRY(seq_source_internal(f, static_cast<const char *>(q.vec) + e.k * canon_bytes(io, V), io,
                                            q.t_sink, q.mu, b, s));
                break;
            default:
                DFL_TRY(pack_spinor(f, static_cast<const char *>(q.vec) + e.k * canon_bytes(io, V), io, b, QCD_F64,
                                    1, s));
        }
    }
    if (!pts.empty()) {
        const int np = (int)pts.size() / 3;
        DFL_HIP(hipMemcpyAsync(dsrc, pts.data(), sizeof(int) * pts.size(), hipMemcpyHostToDevice, s));
        k_point_sources<<<(np + 63) / 64, 64, 0, s>>>(b64, dsrc, f->int_of, V, np);
        DFL_HIP(hipGetLastError());
        // the host vector must outlive the copy
        DFL_HIP(hipStreamSynchronize(s));
    }
    return 0;
}

// unpack x64[0..n) into the outputs of list[r0 .. r0+n), one call per run of
// consecutive vectors of one source
int store_solutions(qcd_field f, const std::vector<Rhs> &list, const std::vector<int> &slots, const double2 *x64,
                    void *const *outs, const std::vector<int> &out_of_src, qcd_prec out, hipStream_t s) {
    const long V = f->g.V;
    const int n = (int)slots.size();
    for (int i = 0; i < n;) {
        const Rhs &e = list[slots[i]];
        int run = 1;
        while (i + run < n && slots[i + run] == slots[i] + run && list[slots[i + run]].src == e.src) ++run;
        char *dst = static_cast<char *>(outs[out_of_src[e.src]]) + e.k * canon_bytes(out, V);
        DFL_TRY(unpack_spinor(f, x64 + (size_t)i * 12 * V, QCD_F64, dst, out, run, s));
        i += run;
    }
    return 0;
}

// Solve every right-hand side of `list` with parameters p in batches of nb;
// fixed-iteration parameters replay graphs, and their misses are solved
// again with the residual-stopping solver (rescue) when p.res > 0.
int solve_set(qcd_field f, const qcd_ama &a, const qcd_gcr &p, const std::vector<Rhs> &list,
              const std::vector<int> &out_of_src, void *const *outs, qcd_prec out, qcd_prec io, qcd_info *info,
              int batch, hipStream_t s, int &status) {
    const long V = f->g.V;
    const int total = (int)list.size();
    if (total == 0) return 0;
    const int nb = std::max(1, std::min(batch, total));
    void *ws;
    DFL_TRY(field_buffer(f, BUF_AMA, (sizeof(double2) * 12 * V) * 2 * nb + sizeof(int) * 3 * nb, &ws));
    double2 *b64 = static_cast<double2 *>(ws);
    double2 *x64 = b64 + (size_t)12 * V * nb;
    int *dsrc = reinterpret_cast<int *>(x64 + (size_t)12 * V * nb);
    const bool graph = p.fixed_iters > 0;
    std::vector<qcd_info> inf(nb);
    for (int r0 = 0; r0 < total; r0 += nb) {
        const int n = std::min(nb, total - r0);
        DFL_TRY(build_sources(f, a, list, r0, n, b64, dsrc, io, s));
        int st = 0;
        DFL_TRY(solve_batch(f, p, b64, x64, n, graph, inf.data(), s, st));
        std::vector<int> slots(n);
        for (int r = 0; r < n; ++r) slots[r] = r0 + r;
        DFL_TRY(store_solutions(f, list, slots, x64, outs, out_of_src, out, s));
        if (graph && st == QCD_NOCONV && p.res > 0) {
            // rescue: the sources of the misses, compacted to the front of
            // the batch, solved to p.res without the fixed count
            std::vector<int> miss;
            for (int r = 0; r < n; ++r)
                if (inf[r].status != 0) miss.push_back(r);
            for (size_t j = 0; j < miss.size(); ++j)
                if ((int)j != miss[j])
                    DFL_HIP(hipMemcpyAsync(b64 + j * 12 * V, b64 + (size_t)miss[j] * 12 * V, sizeof(double2) * 12 * V,
                                           hipMemcpyDeviceToDevice, s));
            qcd_gcr q = p;
            q.fixed_iters = 0;
            std::vector<qcd_info> ri(miss.size());
            int rst = 0;
            DFL_TRY(solve_batch(f, q, b64, x64, (int)miss.size(), false, ri.data(), s, rst));
            std::vector<int> mslots(miss.size());
            for (size_t j = 0; j < miss.size(); ++j) {
                mslots[j] = r0 + miss[j];
                inf[miss[j]] = ri[j];
                inf[miss[j]].iters += p.fixed_iters;
            }
            // each miss is its own run (its slots need not be consecutive)
            for (size_t j = 0; j < miss.size(); ++j)
                DFL_TRY(store_solutions(f, list, {mslots[j]}, x64 + j * 12 * V, outs, out_of_src, out, s));
            st = rst;
        }
        if (st == QCD_NOCONV) status = QCD_NOCONV;
        if (info)
            for (int r = 0; r < n; ++r) info[r0 + r] = inf[r];
    }
    return 0;
}

int run_set(qcd_field f, const qcd_ama &a, void *const *x_sloppy, void *const *x_exact, qcd_prec io,
            qcd_info *info_sloppy, qcd_info *info_exact, hipStream_t s, int &status) {
    std::vector<Rhs> sl, ex;
    std::vector<int> out_s(a.nsrc), out_e(a.nsrc, -1);
    int nex = 0;
    for (int i = 0; i < a.nsrc; ++i) {
        const int nv = nvec_of(a.src[i]);
        out_s[i] = i;
        for (int k = 0; k < nv; ++k) sl.push_back({i, k});
        if (a.exact && a.exact[i]) {
            out_e[i] = nex++;
            for (int k = 0; k < nv; ++k) ex.push_back({i, k});
        }
    }
    DFL_TRY(solve_set(f, a, a.sloppy, sl, out_s, x_sloppy, a.sloppy_out, io, info_sloppy,
                      pick_batch(f, a.sloppy, a.batch), s, status));
    DFL_TRY(solve_set(f, a, a.exact_params, ex, out_e, x_exact, io, io, info_exact,
                      pick_batch(f, a.exact_params, a.batch), s, status));
    return 0;
}

int check_call(qcd_field f, const qcd_ama *a, void *const *x_sloppy, void *const *x_exact) {
    if (!f || !a || !x_sloppy) return set_error(QCD_EINVAL, "bad arguments to ama_solve");
    DFL_TRY(check_set(f->g, a));
    bool any_exact = false;
    for (int i = 0; i < a->nsrc; ++i) any_exact = any_exact || (a->exact && a->exact[i]);
    if (any_exact && !x_exact) return set_error(QCD_EINVAL, "exact sources flagged but no output buffers");
    return 0;
}

}  // namespace
}  // namespace dfl

using namespace dfl;

extern "C" int ama_solve(qcd_field f, const qcd_ama *a, void *const *x_sloppy, void *const *x_exact, qcd_prec io,
                         qcd_info *info_sloppy, qcd_info *info_exact, hipStream_t s) {
    if (io != QCD_F64 && io != QCD_F32) return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    DFL_TRY(check_call(f, a, x_sloppy, x_exact));
    int status = 0;
    DFL_TRY(run_set(f, *a, x_sloppy, x_exact, io, info_sloppy, info_exact, s, status));
    DFL_HIP(hipStreamSynchronize(s));
    return status;
}

extern "C" int ama_solve_multi(int nfield, const qcd_field *fields, const qcd_ama *sets, void *const *const *x_sloppy,
                               void *const *const *x_exact, qcd_prec io, qcd_info *const *info_sloppy,
                               qcd_info *const *info_exact, hipStream_t s) {
    if (nfield < 1 || !fields || !sets || !x_sloppy || !x_exact)
        return set_error(QCD_EINVAL, "bad arguments to ama_solve_multi");
    if (io != QCD_F64 && io != QCD_F32) return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    for (int k = 0; k < nfield; ++k) {
        const int rc = check_call(fields[k], &sets[k], x_sloppy[k], x_exact[k]);
        if (rc < 0) return set_error(rc, "gauge field " + std::to_string(k) + ": " + qcd_last_error());
        if (fields[k]->device != fields[0]->device)
            return set_error(QCD_EINVAL, "all gauge fields of one call must live on one device");
    }
    int status = 0;
    for (int k = 0; k < nfield; ++k) {
        DFL_TRY(run_set(fields[k], sets[k], x_sloppy[k], x_exact[k], io, info_sloppy ? info_sloppy[k] : nullptr,
                        info_exact ? info_exact[k] : nullptr, s, status));
        // a finished field's solver buffers go back to the workspace cache,
        // so that the next field (of another size) can take their room
        if (k + 1 < nfield) DFL_TRY(qcd_field_trim(fields[k]));
    }
    DFL_HIP(hipStreamSynchronize(s));
    return status;
}
