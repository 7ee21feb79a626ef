// Batched solves of arbitrary source vectors (Z2 noise, point, sequential),
// optionally replayed from HIP graphs.
//
// With a fixed iteration count (the truncated sloppy solves of all-mode
// averaging, section 3.5, Table 3) the solver needs no host decisions, so
// its whole sequence of launches for one batch can be captured once into a
// HIP graph and replayed for every later batch of the same size: the graph
// reads the batch's sources from, and writes its solutions to, the same
// workspace vectors, which are filled and emptied around each replay.
// Norms stay on the device and are read after the replay.  A graph refers to
// the handle's workspace buffers, so every graph of a handle is dropped when
// one of them moves (grows).
#include <cmath>
#include <cstring>

#include "blas.h"
#include "dflint.h"

namespace dfl {

// A graph is valid for the batch size, the solver parameters, the workspace
// generation and the two workspace vectors it reads and writes: the
// solution vectors follow the batch's sources, so their address depends on
// the batch size of the call that laid out the workspace.
struct GraphEntry {
    int n;
    qcd_gcr p;
    unsigned gen;
    const double2 *b64;
    const double2 *x64;
    hipGraphExec_t exec;
};
struct GraphCache {
    std::vector<GraphEntry> e;
};

void graph_cache_free(qcd_field f) {
    auto *c = static_cast<GraphCache *>(f->graphs);
    if (!c) return;
    for (auto &g : c->e) (void)hipGraphExecDestroy(g.exec);
    delete c;
    f->graphs = nullptr;
}

namespace {

GraphEntry *find_graph(qcd_field f, int n, const qcd_gcr &p, const double2 *b64, const double2 *x64) {
    auto *c = static_cast<GraphCache *>(f->graphs);
    if (!c) return nullptr;
    // graphs captured before a workspace buffer moved are stale
    for (size_t i = 0; i < c->e.size();)
        if (c->e[i].gen != f->graph_gen) {
            (void)hipGraphExecDestroy(c->e[i].exec);
            c->e.erase(c->e.begin() + i);
        } else {
            ++i;
        }
    for (auto &g : c->e)
        if (g.n == n && g.b64 == b64 && g.x64 == x64 && std::memcmp(&g.p, &p, sizeof(qcd_gcr)) == 0) return &g;
    return nullptr;
}

// capture the fixed-iteration solve of n right-hand sides (workspace b64 ->
// x64) on the handle's own stream (capture needs a non-default stream)
int capture(qcd_field f, const qcd_gcr &p, const double2 *b64, double2 *x64, int n) {
    if (!f->cap) DFL_HIP(hipStreamCreateWithFlags(&f->cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    DFL_HIP(hipStreamBeginCapture(f->cap, hipStreamCaptureModeThreadLocal));
    set_nosync(true);
    set_capturing(true);
    const int rc = gcr_internal(f, &p, b64, x64, n, nullptr, f->cap);
    set_capturing(false);
    set_nosync(false);
    const hipError_t e = hipStreamEndCapture(f->cap, &g);
    if (rc < 0) {
        if (e == hipSuccess && g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return set_error(QCD_EHIP, std::string("stream capture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return set_error(QCD_EHIP, std::string("graph instantiation: ") + hipGetErrorString(ei));
    auto *c = static_cast<GraphCache *>(f->graphs);
    if (!c) f->graphs = c = new GraphCache();
    c->e.push_back({n, p, f->graph_gen, b64, x64, exec});
    return 0;
}

// relative residuals of a solve that kept its norms on the device
int read_info(qcd_field f, const qcd_gcr &p, int n, qcd_info *info, hipStream_t s, int &status) {
    void *sp;
    DFL_TRY(field_buffer(f, BUF_RED, scalar_bytes(n), &sp));
    Scal sc;
    DFL_TRY(scalar_buffers_at(sp, n, sc));
    std::vector<double> bn2(n), rn2(n);
    DFL_HIP(hipMemcpyAsync(bn2.data(), sc.bn2, n * sizeof(double), hipMemcpyDeviceToHost, s));
    DFL_HIP(hipMemcpyAsync(rn2.data(), sc.red, n * sizeof(double), hipMemcpyDeviceToHost, s));
    DFL_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(bn2[i]) || !std::isfinite(rn2[i])) return set_error(QCD_ENAN, "NaN in a batched solve");
        const double rel = bn2[i] > 0 ? std::sqrt(rn2[i] / bn2[i]) : 0.0;
        const bool ok = !(p.res > 0) || rel <= p.res;
        if (!ok) status = QCD_NOCONV;
        if (info) info[i] = qcd_info{ok ? 0 : QCD_NOCONV, p.fixed_iters, rel};
    }
    return 0;
}

}  // namespace

int solve_batch(qcd_field f, const qcd_gcr &p, const double2 *b64, double2 *x64, int n, bool graph, qcd_info *info,
                hipStream_t s, int &status) {
    if (!graph) {
        const int rc = gcr_internal(f, &p, b64, x64, n, info, s);
        if (rc < 0) return rc;
        if (rc == QCD_NOCONV) status = QCD_NOCONV;
        return 0;
    }
    if (p.fixed_iters <= 0) return set_error(QCD_EINVAL, "graph replay needs fixed_iters > 0");
    if (GraphEntry *g = find_graph(f, n, p, b64, x64)) {
        DFL_HIP(hipGraphLaunch(g->exec, s));
    } else {
        // eager run without synchronisation (this batch's result, and every
        // workspace allocated), then capture the same sequence
        set_nosync(true);
        const int rc = gcr_internal(f, &p, b64, x64, n, nullptr, s);
        set_nosync(false);
        if (rc < 0) return rc;
        DFL_TRY(capture(f, p, b64, x64, n));
    }
    return read_info(f, p, n, info, s, status);
}

}  // namespace dfl

using namespace dfl;

extern "C" int gcr_solve_batched(qcd_field f, const qcd_gcr *p, const void *const *b, void *const *x, int nrhs,
                                 qcd_prec io, int batch, int graph, qcd_info *info, hipStream_t s) {
    if (!f || !p || !b || !x || nrhs <= 0) return set_error(QCD_EINVAL, "bad arguments to gcr_solve_batched");
    if (io != QCD_F64 && io != QCD_F32) return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    if (graph && p->fixed_iters <= 0) return set_error(QCD_EINVAL, "graph replay needs fixed_iters > 0");
    const long V = f->g.V;
    const int nb = std::max(1, std::min(batch > 0 ? batch : 12, nrhs));
    void *ws;
    DFL_TRY(field_buffer(f, BUF_AMA, sizeof(double2) * 12 * V * 2 * nb, &ws));
    double2 *b64 = static_cast<double2 *>(ws);
    double2 *x64 = b64 + (size_t)12 * V * nb;
    int status = 0;
    for (int r0 = 0; r0 < nrhs; r0 += nb) {
        const int n = std::min(nb, nrhs - r0);
        for (int r = 0; r < n; ++r)
            DFL_TRY(pack_spinor(f, b[r0 + r], io, b64 + (size_t)r * 12 * V, QCD_F64, 1, s));
        DFL_TRY(solve_batch(f, *p, b64, x64, n, graph != 0, info ? info + r0 : nullptr, s, status));
        for (int r = 0; r < n; ++r)
            DFL_TRY(unpack_spinor(f, x64 + (size_t)r * 12 * V, QCD_F64, x[r0 + r], io, 1, s));
    }
    DFL_HIP(hipStreamSynchronize(s));
    return status;
}
