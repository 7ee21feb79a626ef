"""MI355X (gfx950) deflated SAP-GCR Wilson-clover solver for all-mode averaging.

Thin Python binding over the C ABI in ``include/dfl.h`` (libdfl.so, built
in-tree from ``csrc/`` by ``build.py``).  The binding only marshals
arguments: device buffers are torch tensors on the GPU, streams are torch's
current HIP stream, and every step of the computation runs in the HIP
library.  There is no CPU fallback: without the built library, or without a
GPU, every call raises.
"""

from ._lib import (  # noqa: F401
    F64, F32, F16, BF16, NOCONV, SRC_POINT, SRC_Z2, SRC_SEQ, SRC_VEC,
    DflError, Field, Deflation, SapParams, GcrParams, SolveInfo, Source, point, z2, sequential, vectors,
    lib_path, load, dirac_apply, dirac_apply_noalloc, sap_precond, gcr_solve, gcr_solve_batched, ama_solve, ama_solve_multi, z2_sources,
    sequential_sources, nucleon_2pt, nucleon_seq_sources, nucleon_3pt, ama_combine, gauss_smear,
    workspace_cached, workspace_trim, prof_enable, prof_reset, prof_get, PROF_CLASSES,
)
