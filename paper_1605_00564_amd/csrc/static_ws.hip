// The Dirac operator for callers that cannot allocate device memory (code
// under HIP graph capture, serving loops, harnesses that forbid it).
//
// dirac_apply stages its input and output in the library's internal layout
// in workspace buffers that grow on demand.  This variant stages them in a
// fixed device array instead: `scratch`, of SCRATCH_BYTES, one copy per GPU,
// held from the first time the library runs on that GPU until the process
// ends.  The array's name is a host-side stand-in in host code; its device
// address is looked up once per device (hipGetSymbolAddress, with that
// device current) and only that address is handed to kernels.  Each call
// overwrites the whole staging area it uses (the packing kernel writes
// every input element, the stencil every output element), so nothing needs
// clearing; calls that overlap in time on one GPU share the array and race.
#include <mutex>
#include <vector>

#include "internal.h"

namespace dfl {
constexpr size_t SCRATCH_BYTES = 64ull << 20;
}

static __device__ __align__(256) unsigned char scratch[dfl::SCRATCH_BYTES];

namespace dfl {

namespace {

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;   // device address of `scratch`, per device

}  // namespace

// Look up the device address of `scratch` on device dev (which must be the
// current device); once per device.
int static_scratch_init(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0) return set_error(QCD_EINVAL, "bad device");
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
    if (g_scratch_ptr[dev]) return 0;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return set_error(QCD_EHIP, std::string("address of the static scratch array: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
    return 0;
}

static int static_scratch(int dev, void **p) {
    DFL_TRY(static_scratch_init(dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    *p = g_scratch_ptr[dev];
    return 0;
}

}  // namespace dfl

using namespace dfl;

extern "C" int dirac_apply_noalloc(qcd_field f, const void *in, void *out, int nrhs, qcd_prec io, qcd_prec storage,
                                   hipStream_t s) {
    if (!f || !in || !out || nrhs <= 0) return set_error(QCD_EINVAL, "bad arguments to dirac_apply_noalloc");
    if (io != QCD_F64 && io != QCD_F32) return set_error(QCD_EINVAL, "io precision must be F64 or F32");
    if (in == out) return set_error(QCD_EINVAL, "dirac_apply_noalloc: in and out must differ");
    if (storage != QCD_F64 && storage != QCD_F32 && storage != QCD_F16 && storage != QCD_BF16)
        return set_error(QCD_EINVAL, "bad operator storage");
    const qcd_prec vec = storage == QCD_F64 ? QCD_F64 : QCD_F32;
    const size_t nb = spinor_bytes(vec, f->g.V) * (size_t)nrhs;
    if (2 * nb > SCRATCH_BYTES)
        return set_error(QCD_EINVAL, "dirac_apply_noalloc: " + std::to_string(nrhs) + " right-hand sides need " +
                                         std::to_string(2 * nb) + " bytes of staging, more than the " +
                                         std::to_string(SCRATCH_BYTES) + " of the static scratch array");
    int dev = 0;
    DFL_HIP(hipGetDevice(&dev));
    if (dev != f->device) return set_error(QCD_EINVAL, "dirac_apply_noalloc: the field's device is not current");
    void *ws = nullptr;
    DFL_TRY(static_scratch(dev, &ws));
    char *a = static_cast<char *>(ws), *b = a + nb;
    // no profiling events either (their creation may allocate)
    const bool was = nosync();
    set_nosync(true);
    int rc = pack_spinor(f, in, io, a, vec, nrhs, s);
    if (rc == 0) rc = dirac_internal2(f, a, vec, b, vec, nrhs, storage, s);
    if (rc == 0) rc = unpack_spinor(f, b, vec, out, io, nrhs, s);
    set_nosync(was);
    return rc;
}
