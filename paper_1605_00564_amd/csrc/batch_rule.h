// The AMA driver's batch size: right-hand sides per solver launch, from the
// memory available to the solver.  Plain C++, shared by the driver and a CPU
// test.
#pragma once

#include <algorithm>
#include <cstddef>

namespace dfl {

// avail: bytes available (free device memory, the workspace cache and the
// handle's own buffers); per: bytes one right-hand side needs; want: the
// caller's request (0: none).  A request that 90% of avail holds is kept;
// otherwise the batch is what 60% holds (at least 1, at most 48 and at most
// the request, a multiple of 12 when possible, else even: the Schwarz and
// stencil kernels pair right-hand sides), so that the caller keeps room for
// its own allocations.
inline int batch_rule(size_t avail, size_t per, int want) {
    per = std::max<size_t>(per, 1);
    if (want > 0 && (size_t)want <= (size_t)(0.9 * (double)avail) / per) return want;
    size_t n = std::min<size_t>(std::max<size_t>((size_t)(0.6 * (double)avail) / per, 1), 48);
    if (want > 0) n = std::min<size_t>(n, (size_t)want);
    if (n >= 12)
        n -= n % 12;
    else if (n > 1)
        n -= n % 2;
    return (int)n;
}

}  // namespace dfl
