"""ctypes binding of libdfl.so (argument marshalling only).

Vectors are torch tensors on the GPU in the canonical layout
``[nrhs, V, 4, 3]`` (complex128 for F64 io, complex64 for F32 io).  Every
function enqueues on torch's current stream.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

F64, F32, F16, BF16 = 0, 1, 2, 3
SRC_POINT, SRC_Z2, SRC_SEQ, SRC_VEC = 0, 1, 2, 3
# return codes (include/dfl.h)
QCD_NOCONV, QCD_EINVAL, QCD_EGEOM, QCD_ENOMEM, QCD_EHIP, QCD_ESINGULAR, QCD_ENAN, QCD_ENOTSET = 1, -1, -2, -3, -4, -5, -6, -7
NOCONV = 1
PROF_CLASSES = ("dirac", "sap", "deflation", "little", "blas", "other")

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libdfl.so")


class DflError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# C structures (mirror include/dfl.h)
# ---------------------------------------------------------------------------

class _Lattice(C.Structure):
    _fields_ = [("dims", C.c_int * 4), ("block", C.c_int * 4), ("kappa", C.c_double), ("csw", C.c_double),
                ("bc_t", C.c_int)]


class _Sap(C.Structure):
    _fields_ = [("ncy", C.c_int), ("nmr", C.c_int), ("storage", C.c_int), ("vecs", C.c_int)]


class _DflParams(C.Structure):
    _fields_ = [("Ns", C.c_int), ("ninv", C.c_int), ("seed", C.c_ulonglong), ("sap", _Sap), ("block", C.c_int * 4),
                ("nref", C.c_int), ("ref_res", C.c_double)]


class _Gcr(C.Structure):
    _fields_ = [("nkv", C.c_int), ("nmx", C.c_int), ("fixed_iters", C.c_int), ("res", C.c_double), ("sap", _Sap),
                ("dfl", C.c_void_p), ("little_tol", C.c_double), ("little_maxit", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("rel_res", C.c_double)]


class _Source(C.Structure):
    _fields_ = [("kind", C.c_int), ("pos", C.c_int * 4), ("seed", C.c_ulonglong), ("index", C.c_longlong),
                ("nvec", C.c_int), ("t_sink", C.c_int), ("mu", C.c_int), ("vec", C.c_void_p)]


class _Ama(C.Structure):
    _fields_ = [("nsrc", C.c_int), ("src", C.POINTER(_Source)), ("exact", C.POINTER(C.c_ubyte)),
                ("sloppy", _Gcr), ("exact_params", _Gcr), ("sloppy_out", C.c_int), ("batch", C.c_int)]


_lib = None


def lib_path() -> str:
    return _SO


def load():
    """Load libdfl.so (building it first only when no build exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        from . import build as _build
        _build.build()
    L = C.CDLL(_SO)
    P, I, D = C.c_void_p, C.c_int, C.c_double
    L.qcd_strerror.restype = C.c_char_p
    L.qcd_strerror.argtypes = [I]
    L.qcd_last_error.restype = C.c_char_p
    L.qcd_field_create.argtypes = [C.POINTER(_Lattice), P, P, C.POINTER(P)]
    L.qcd_field_create_device.argtypes = [C.POINTER(_Lattice), P, P, C.POINTER(P)]
    L.qcd_field_destroy.argtypes = [P]
    L.dirac_apply.argtypes = [P, P, P, I, I, I, P]
    L.dirac_apply_ex.argtypes = [P, P, P, I, I, I, I, I, P]
    L.dirac_apply_noalloc.argtypes = [P, P, P, I, I, I, P]
    L.make_z2_sources.argtypes = [P, C.c_ulonglong, C.c_longlong, I, P, I, P]
    L.qcd_field_tune.argtypes = [P, I, I]
    L.gcr_solve_batched.argtypes = [P, C.POINTER(_Gcr), C.POINTER(P), C.POINTER(P), I, I, I, I, C.POINTER(_Info), P]
    L.make_sequential_sources.argtypes = [P, P, P, I, I, I, I, P]
    L.sap_precond.argtypes = [P, C.POINTER(_Sap), P, P, I, I, P]
    for name, args in [
        ("deflation_setup", [P, C.POINTER(_DflParams), P, C.POINTER(P)]),
        ("deflation_destroy", [P]),
        ("deflation_get_phi", [P, P, P]),
        ("deflation_set_phi", [P, P, P]),
        ("deflation_dims", [P, C.POINTER(I), C.POINTER(I)]),
        ("little_dirac_apply", [P, P, P, I, P]),
        ("little_dirac_solve", [P, P, P, I, D, I, C.POINTER(I), P]),
        ("deflation_restrict", [P, P, P, I, I, P]),
        ("deflation_prolong", [P, P, P, I, I, P]),
        ("gcr_solve", [P, C.POINTER(_Gcr), P, P, I, I, C.POINTER(_Info), P]),
        ("ama_solve", [P, C.POINTER(_Ama), C.POINTER(P), C.POINTER(P), I, C.POINTER(_Info), C.POINTER(_Info), P]),
        ("ama_solve_multi", [I, C.POINTER(P), C.POINTER(_Ama), C.POINTER(C.POINTER(P)), C.POINTER(C.POINTER(P)), I,
                             C.POINTER(C.POINTER(_Info)), C.POINTER(C.POINTER(_Info)), P]),
        ("qcd_field_ape_smear", [P, D, I, P]),
        ("qcd_field_get_ape_links", [P, P, P]),
        ("gauss_smear", [P, P, P, I, I, D, I, P]),
        ("nucleon_2pt", [P, P, I, I, P, P]),
        ("nucleon_seq_sources", [P, P, I, I, P, I, P, P]),
        ("nucleon_3pt", [P, P, P, I, I, P, P, P]),
        ("ama_combine", [C.c_longlong, I, P, I, P, P, P, P]),
        ("qcd_workspace_cached", [I, C.POINTER(C.c_size_t)]),
        ("qcd_workspace_trim", [I]),
        ("qcd_field_trim", [P]),
        ("qcd_prof_enable", [I]),
        ("qcd_prof_reset", []),
        ("qcd_prof_get", [I, C.POINTER(D), C.POINTER(C.c_longlong)]),
        ("qcd_prof_get_work", [I, C.POINTER(D), C.POINTER(D), C.POINTER(D)]),
    ]:
        if hasattr(L, name):
            getattr(L, name).argtypes = args
    _lib = L
    return L


def _check(rc, where, ok_noconv=False):
    if rc == 0 or (ok_noconv and rc == NOCONV):
        return rc
    L = load()
    raise DflError(rc, where, L.qcd_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_1605_00564_amd needs a GPU: no HIP device is visible")
    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _io_of(t) -> int:
    torch = _torch()
    if t.dtype == torch.complex128:
        return F64
    if t.dtype == torch.complex64:
        return F32
    raise TypeError("vectors must be complex128 or complex64 tensors")


def _vec(t, V):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("vectors must be contiguous GPU tensors")
    if t.numel() % (V * 12):
        raise ValueError("vector size is not a multiple of 12 V")
    return t.numel() // (V * 12)


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

@dataclass
class SapParams:
    ncy: int = 5
    nmr: int = 4
    storage: int = F32
    vecs: int = F32     # F16: the sweeps' stored residuals and face half-spinors in FP16

    def c(self):
        return _Sap(self.ncy, self.nmr, self.storage, self.vecs)


@dataclass
class GcrParams:
    nkv: int = 16
    nmx: int = 1000
    fixed_iters: int = 0
    res: float = 1e-10
    sap: SapParams = None
    dfl: "Deflation" = None
    little_tol: float = 1e-6
    little_maxit: int = 24

    def c(self):
        sap = self.sap or SapParams()
        return _Gcr(self.nkv, self.nmx, self.fixed_iters, self.res, sap.c(),
                    self.dfl.handle if self.dfl is not None else None, self.little_tol, self.little_maxit)


@dataclass
class SolveInfo:
    status: int
    iters: int
    rel_res: float


# ---------------------------------------------------------------------------
# handles
# ---------------------------------------------------------------------------

class Field:
    """Gauge field on the device with its packed links and clover term."""

    def __init__(self, dims, block, kappa, csw, U, bc_t: int = -1):
        """U: complex128 [V, 4, 3, 3] as a host numpy array or a GPU tensor."""
        L = load()
        torch = _torch()
        self.dims = tuple(int(d) for d in dims)
        self.block = tuple(int(b) for b in block)
        self.V = int(np.prod(self.dims))
        lat = _Lattice((C.c_int * 4)(*self.dims), (C.c_int * 4)(*self.block), float(kappa), float(csw), int(bc_t))
        h = C.c_void_p()
        if isinstance(U, torch.Tensor):
            if not (U.is_cuda and U.dtype == torch.complex128 and U.is_contiguous()
                    and tuple(U.shape) == (self.V, 4, 3, 3)):
                raise ValueError("device links must be a contiguous complex128 GPU tensor [V, 4, 3, 3]")
            _check(L.qcd_field_create_device(C.byref(lat), C.c_void_p(U.data_ptr()), _stream(), C.byref(h)),
                   "qcd_field_create_device")
        else:
            U = np.ascontiguousarray(U, dtype=np.complex128)
            if U.shape != (self.V, 4, 3, 3):
                raise ValueError("links must be complex128 [V, 4, 3, 3]")
            _check(L.qcd_field_create(C.byref(lat), U.ctypes.data_as(C.c_void_p), _stream(), C.byref(h)),
                   "qcd_field_create")
        self.handle = h
        self.kappa, self.csw, self.bc_t = float(kappa), float(csw), int(bc_t)

    TUNE_STENCIL_BLOCK, TUNE_STENCIL_RG, TUNE_STENCIL_ORDER, TUNE_STENCIL_NR, TUNE_STENCIL_LINKLDS = 0, 1, 2, 3, 4
    TUNE_SAP_PAIR = 5

    def tune(self, knob: int, value: int):
        """Set a launch choice of the Dirac stencil (see include/dfl.h)."""
        _check(load().qcd_field_tune(self.handle, knob, value), "qcd_field_tune")

    def ape_smear(self, alpha: float, n_iter: int):
        """APE-smear the spatial links (kept in the handle for gauss_smear)."""
        _check(load().qcd_field_ape_smear(self.handle, float(alpha), int(n_iter), _stream()), "qcd_field_ape_smear")

    def ape_links(self):
        """The smeared spatial links [V, 3, 3, 3] (complex128, direction mu - 1)."""
        torch = _torch()
        out = torch.empty((self.V, 3, 3, 3), dtype=torch.complex128, device="cuda")
        _check(load().qcd_field_get_ape_links(self.handle, C.c_void_p(out.data_ptr()), _stream()),
               "qcd_field_get_ape_links")
        return out

    def trim(self):
        """Give this handle's scratch buffers to the workspace cache."""
        _check(load().qcd_field_trim(self.handle), "qcd_field_trim")

    def close(self):
        if getattr(self, "handle", None):
            load().qcd_field_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Deflation:
    """Block-local deflation subspace and little Dirac operator.  block: the
    deflation block (default: the field's Schwarz block; else a multiple of
    it); nref rounds of inverse iteration with the deflated solver to
    relative residual ref_res refine the subspace (include/dfl.h,
    deflation_setup)."""

    def __init__(self, field: Field, Ns: int, ninv: int = 5, seed: int = 7, sap: SapParams = None, block=None,
                 nref: int = 0, ref_res: float = 1e-2):
        L = load()
        sap = sap or SapParams()
        blk = (C.c_int * 4)(*([int(b) for b in block] if block is not None else [0, 0, 0, 0]))
        p = _DflParams(int(Ns), int(ninv), int(seed), sap.c(), blk, int(nref), float(ref_res))
        h = C.c_void_p()
        _check(L.deflation_setup(field.handle, C.byref(p), _stream(), C.byref(h)), "deflation_setup")
        self.handle = h
        self.field = field
        nb, ns = C.c_int(), C.c_int()
        _check(L.deflation_dims(h, C.byref(nb), C.byref(ns)), "deflation_dims")
        self.Nb, self.Ns = nb.value, ns.value
        self.Vb = field.V // self.Nb        # deflation-block volume

    def get_phi(self):
        torch = _torch()
        phi = torch.empty((self.Nb, self.Ns, self.Vb, 4, 3), dtype=torch.complex128, device="cuda")
        _check(load().deflation_get_phi(self.handle, C.c_void_p(phi.data_ptr()), _stream()), "deflation_get_phi")
        return phi

    def set_phi(self, phi):
        torch = _torch()
        if phi.dtype != torch.complex128 or not phi.is_cuda or phi.numel() != self.Nb * self.Ns * self.Vb * 12:
            raise ValueError("phi must be a complex128 GPU tensor [Nb, Ns, Vb, 4, 3]")
        phi = phi.contiguous()
        _check(load().deflation_set_phi(self.handle, C.c_void_p(phi.data_ptr()), _stream()), "deflation_set_phi")

    def little_apply(self, v):
        torch = _torch()
        v = v.contiguous()
        n = v.numel() // (self.Nb * self.Ns)
        w = torch.empty_like(v)
        _check(load().little_dirac_apply(self.handle, C.c_void_p(v.data_ptr()), C.c_void_p(w.data_ptr()), n,
                                         _stream()), "little_dirac_apply")
        return w

    def little_solve(self, v, tol=1e-12, maxit=500):
        torch = _torch()
        v = v.contiguous()
        n = v.numel() // (self.Nb * self.Ns)
        w = torch.empty_like(v)
        it = C.c_int()
        rc = load().little_dirac_solve(self.handle, C.c_void_p(v.data_ptr()), C.c_void_p(w.data_ptr()), n, tol,
                                       maxit, C.byref(it), _stream())
        _check(rc, "little_dirac_solve", ok_noconv=True)
        return w, it.value

    def restrict(self, v):
        torch = _torch()
        n = _vec(v, self.field.V)
        u = torch.empty((n, self.Nb, self.Ns), dtype=torch.complex128, device="cuda")
        _check(load().deflation_restrict(self.handle, C.c_void_p(v.data_ptr()), C.c_void_p(u.data_ptr()), n,
                                         _io_of(v), _stream()), "deflation_restrict")
        return u

    def prolong(self, u, dtype=None):
        torch = _torch()
        u = u.contiguous()
        n = u.numel() // (self.Nb * self.Ns)
        v = torch.empty((n, self.field.V, 4, 3), dtype=dtype or torch.complex128, device="cuda")
        _check(load().deflation_prolong(self.handle, C.c_void_p(u.data_ptr()), C.c_void_p(v.data_ptr()), n,
                                        _io_of(v), _stream()), "deflation_prolong")
        return v

    def close(self):
        if getattr(self, "handle", None):
            load().deflation_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# operations
# ---------------------------------------------------------------------------

def dirac_apply(field: Field, x, storage: int = F64, out=None, spinor_in=None, spinor_out=None):
    """out = M x (kappa-normalised Wilson-clover operator).  spinor_in /
    spinor_out select the internal spinor storage on each side (F64, F32,
    or F16 = FP16 with a per-site scale); by default F64 with FP64 storage,
    else F32."""
    torch = _torch()
    n = _vec(x, field.V)
    out = torch.empty_like(x) if out is None else out
    if spinor_in is None and spinor_out is None:
        _check(load().dirac_apply(field.handle, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), n,
                                  _io_of(x), storage, _stream()), "dirac_apply")
        return out
    dflt = F64 if storage == F64 else F32
    si = dflt if spinor_in is None else spinor_in
    so = dflt if spinor_out is None else spinor_out
    _check(load().dirac_apply_ex(field.handle, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), n, _io_of(x),
                                 storage, si, so, _stream()), "dirac_apply_ex")
    return out


def dirac_apply_noalloc(field: Field, x, out, storage: int = F64):
    """out = M x staged in the library's static scratch array (no device
    allocation): x and out are preallocated GPU tensors of one shape."""
    n = _vec(x, field.V)
    if out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor of x's shape and dtype")
    _check(load().dirac_apply_noalloc(field.handle, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), n,
                                      _io_of(x), storage, _stream()), "dirac_apply_noalloc")
    return out


def z2_sources(field: Field, seed: int, n: int, index0: int = 0, dtype=None):
    """n Z2-noise source vectors [n, V, 4, 3] built on the device."""
    torch = _torch()
    dtype = dtype or torch.complex64
    out = torch.empty((n, field.V, 4, 3), dtype=dtype, device="cuda")
    _check(load().make_z2_sources(field.handle, seed, index0, n, C.c_void_p(out.data_ptr()), _io_of(out), _stream()),
           "make_z2_sources")
    return out


def sequential_sources(field: Field, psi, t_sink: int, mu: int = 3, out=None):
    """eta = delta_{t, t_sink} gamma_5 gamma_mu gamma_5 psi for each vector of psi."""
    torch = _torch()
    n = _vec(psi, field.V)
    out = torch.empty_like(psi) if out is None else out
    _check(load().make_sequential_sources(field.handle, C.c_void_p(psi.data_ptr()), C.c_void_p(out.data_ptr()), n,
                                          _io_of(psi), t_sink, mu, _stream()), "make_sequential_sources")
    return out


def sap_precond(field: Field, eta, sap: SapParams = None, out=None):
    """psi = M_SAP eta."""
    torch = _torch()
    n = _vec(eta, field.V)
    out = torch.empty_like(eta) if out is None else out
    p = (sap or SapParams()).c()
    _check(load().sap_precond(field.handle, C.byref(p), C.c_void_p(eta.data_ptr()), C.c_void_p(out.data_ptr()), n,
                              _io_of(eta), _stream()), "sap_precond")
    return out


def gcr_solve(field: Field, b, params: GcrParams = None, x=None):
    """x = M^{-1} b by (deflated) SAP-preconditioned flexible GCR; returns (x, [SolveInfo])."""
    torch = _torch()
    n = _vec(b, field.V)
    x = torch.empty_like(b) if x is None else x
    p = (params or GcrParams()).c()
    info = (_Info * n)()
    rc = load().gcr_solve(field.handle, C.byref(p), C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), n,
                          _io_of(b), info, _stream())
    _check(rc, "gcr_solve", ok_noconv=True)
    return x, [SolveInfo(i.status, i.iters, i.rel_res) for i in info]


def gcr_solve_batched(field: Field, b_list, params: GcrParams, x_list=None, batch: int = 0, graph: bool = False):
    """Solve every vector of b_list (each [V, 4, 3] on the GPU, contiguous)
    in batches; with graph=True (needs params.fixed_iters > 0) the batches
    replay one captured HIP graph per batch size.  Returns (x_list, info)."""
    torch = _torch()
    n = len(b_list)
    x_list = x_list if x_list is not None else [torch.empty_like(v) for v in b_list]
    for v in list(b_list) + list(x_list):
        if not v.is_contiguous() or v.numel() != field.V * 12:
            raise ValueError("vectors must be contiguous [V, 4, 3]")
    bp = (C.c_void_p * n)(*[v.data_ptr() for v in b_list])
    xp = (C.c_void_p * n)(*[v.data_ptr() for v in x_list])
    p = params.c()
    info = (_Info * n)()
    rc = load().gcr_solve_batched(field.handle, C.byref(p), bp, xp, n, _io_of(b_list[0]), batch, 1 if graph else 0,
                                  info, _stream())
    _check(rc, "gcr_solve_batched", ok_noconv=True)
    return x_list, [SolveInfo(i.status, i.iters, i.rel_res) for i in info]


@dataclass
class Source:
    """One source of an AMA set (see ama_solve in include/dfl.h)."""
    kind: int = SRC_POINT
    pos: tuple = (0, 0, 0, 0)
    seed: int = 0
    index: int = 0
    nvec: int = 0
    t_sink: int = 0
    mu: int = 3
    vec: object = None     # SEQ: forward solutions [12, V, 4, 3]; VEC: sources [nvec, V, 4, 3]

    @property
    def count(self):
        return 12 if self.kind in (SRC_POINT, SRC_SEQ) else self.nvec

    def c(self):
        return _Source(self.kind, (C.c_int * 4)(*[int(v) for v in self.pos]), int(self.seed), int(self.index),
                       int(self.nvec), int(self.t_sink), int(self.mu),
                       self.vec.data_ptr() if self.vec is not None else None)


def point(pos) -> Source:
    return Source(SRC_POINT, tuple(pos))


def z2(seed: int, index: int = 0, nvec: int = 1) -> Source:
    return Source(SRC_Z2, seed=seed, index=index, nvec=nvec)


def sequential(fwd, t_sink: int, mu: int = 3) -> Source:
    return Source(SRC_SEQ, t_sink=t_sink, mu=mu, vec=fwd)


def vectors(v) -> Source:
    return Source(SRC_VEC, nvec=int(v.shape[0]), vec=v)


def _ama_struct(field, sources, exact_flags, sloppy, exact, dtype, sloppy_dtype, batch, out_sloppy, out_exact):
    torch = _torch()
    srcs = [s if isinstance(s, Source) else point(s) for s in sources]
    n = len(srcs)
    for s in srcs:
        if s.vec is not None:
            if s.vec.dtype != dtype or not s.vec.is_contiguous() or s.vec.numel() != s.count * field.V * 12:
                raise ValueError("source vectors must be contiguous [n, V, 4, 3] of the io dtype")
    flags = [bool(e) for e in exact_flags] if exact_flags is not None else [False] * n
    xs = out_sloppy if out_sloppy is not None else [
        torch.empty((s.count, field.V, 4, 3), dtype=sloppy_dtype, device="cuda") for s in srcs]
    xe = out_exact if out_exact is not None else [
        torch.empty((s.count, field.V, 4, 3), dtype=dtype, device="cuda") for s, e in zip(srcs, flags) if e]
    ex_srcs = [s for s, e in zip(srcs, flags) if e]
    for t, s in zip(xs, srcs):
        if t.dtype != sloppy_dtype or not t.is_contiguous() or t.numel() != s.count * field.V * 12:
            raise ValueError("sloppy outputs must be contiguous [n, V, 4, 3] of the sloppy dtype")
    for t, s in zip(xe, ex_srcs):
        if t.dtype != dtype or not t.is_contiguous() or t.numel() != s.count * field.V * 12:
            raise ValueError("exact outputs must be contiguous [n, V, 4, 3] of the io dtype")
    if len(xs) != n or len(xe) != len(ex_srcs):
        raise ValueError("one output tensor per source (sloppy) and per flagged source (exact)")
    keep = dict(src=(_Source * n)(*[s.c() for s in srcs]), ex=(C.c_ubyte * n)(*[1 if e else 0 for e in flags]),
                ps=(C.c_void_p * max(n, 1))(*[t.data_ptr() for t in xs]),
                pe=(C.c_void_p * max(len(xe), 1))(*[t.data_ptr() for t in xe]))
    ns = sum(s.count for s in srcs)
    ne = sum(s.count for s in ex_srcs)
    keep["info_s"] = (_Info * max(ns, 1))()
    keep["info_e"] = (_Info * max(ne, 1))()
    a = _Ama(n, C.cast(keep["src"], C.POINTER(_Source)), C.cast(keep["ex"], C.POINTER(C.c_ubyte)), sloppy.c(),
             exact.c(), F64 if sloppy_dtype == torch.complex128 else F32, batch)
    return a, keep, xs, xe, ns, ne


def _infos(arr, n):
    return [SolveInfo(i.status, i.iters, i.rel_res) for i in arr[:n]]


def ama_solve(field: Field, sources, exact_flags, sloppy: GcrParams, exact: GcrParams, dtype=None, batch=0,
              out_sloppy=None, out_exact=None, sloppy_dtype=None):
    """Sloppy solves of every source, exact solves of the flagged ones.
    sources: Source objects (point, z2, sequential, vectors) or (t, x, y, z)
    positions (point sources).  dtype: io precision (exact outputs, source
    vectors); sloppy_dtype: precision of the sloppy outputs (default dtype).
    Returns (x_sloppy[nsrc], x_exact[nexact], info_s, info_e); outputs are
    [count, V, 4, 3] per source and may be passed in to avoid allocation."""
    torch = _torch()
    dtype = dtype or torch.complex64
    sloppy_dtype = sloppy_dtype or dtype
    a, keep, xs, xe, ns, ne = _ama_struct(field, sources, exact_flags, sloppy, exact, dtype, sloppy_dtype, batch,
                                          out_sloppy, out_exact)
    io = F64 if dtype == torch.complex128 else F32
    rc = load().ama_solve(field.handle, C.byref(a), keep["ps"], keep["pe"], io, keep["info_s"], keep["info_e"],
                          _stream())
    _check(rc, "ama_solve", ok_noconv=True)
    return xs, xe, _infos(keep["info_s"], ns), _infos(keep["info_e"], ne)


def ama_solve_multi(fields, sets, dtype=None, sloppy_dtype=None):
    """The AMA sets of several gauge fields in one library call.  sets[k] is
    a dict with keys sources, exact_flags, sloppy, exact and optionally
    batch, out_sloppy, out_exact.  Returns one (x_sloppy, x_exact, info_s,
    info_e) tuple per field."""
    torch = _torch()
    dtype = dtype or torch.complex64
    sloppy_dtype = sloppy_dtype or dtype
    nf = len(fields)
    built = [_ama_struct(f, st["sources"], st.get("exact_flags"), st["sloppy"], st["exact"], dtype, sloppy_dtype,
                         st.get("batch", 0), st.get("out_sloppy"), st.get("out_exact"))
             for f, st in zip(fields, sets)]
    fh = (C.c_void_p * nf)(*[f.handle.value for f in fields])
    amas = (_Ama * nf)(*[b[0] for b in built])
    ps = (C.POINTER(C.c_void_p) * nf)(*[C.cast(b[1]["ps"], C.POINTER(C.c_void_p)) for b in built])
    pe = (C.POINTER(C.c_void_p) * nf)(*[C.cast(b[1]["pe"], C.POINTER(C.c_void_p)) for b in built])
    iS = (C.POINTER(_Info) * nf)(*[C.cast(b[1]["info_s"], C.POINTER(_Info)) for b in built])
    iE = (C.POINTER(_Info) * nf)(*[C.cast(b[1]["info_e"], C.POINTER(_Info)) for b in built])
    io = F64 if dtype == torch.complex128 else F32
    rc = load().ama_solve_multi(nf, fh, amas, ps, pe, io, iS, iE, _stream())
    _check(rc, "ama_solve_multi", ok_noconv=True)
    return [(b[2], b[3], _infos(b[1]["info_s"], b[4]), _infos(b[1]["info_e"], b[5])) for b in built]


def gauss_smear(field: Field, x, kappa_g: float, n_iter: int, out=None):
    """Gaussian smearing of the vectors x [n, V, 4, 3] with the handle's APE links."""
    torch = _torch()
    n = _vec(x, field.V)
    out = torch.empty_like(x) if out is None else out
    _check(load().gauss_smear(field.handle, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), n, _io_of(x),
                              float(kappa_g), int(n_iter), _stream()), "gauss_smear")
    return out


def _prop(field, prop):
    if _vec(prop, field.V) != 12:
        raise ValueError("a propagator is 12 vectors [12, V, 4, 3]")
    return _io_of(prop)


def _spin_matrix(m):
    a = np.ascontiguousarray(np.asarray(m, dtype=np.complex128).reshape(4, 4))
    return a, a.ctypes.data_as(C.c_void_p)


def nucleon_2pt(field: Field, prop, t0: int):
    """G(t)[4, 4] (complex128, [T, 4, 4]) of the point-source propagator prop
    [12, V, 4, 3] with source timeslice t0 (include/dfl.h, nucleon_2pt)."""
    torch = _torch()
    io = _prop(field, prop)
    out = torch.empty((field.dims[0], 4, 4), dtype=torch.complex128, device="cuda")
    _check(load().nucleon_2pt(field.handle, C.c_void_p(prop.data_ptr()), io, int(t0), C.c_void_p(out.data_ptr()),
                              _stream()), "nucleon_2pt")
    return out


def nucleon_seq_sources(field: Field, prop, t_sink: int, proj, flavour: str):
    """The 12 sequential sources [12, V, 4, 3] for a sink on t_sink with the
    spin projector proj, current on the 'u' or 'd' line."""
    torch = _torch()
    io = _prop(field, prop)
    out = torch.empty_like(prop)
    _, pp = keep = _spin_matrix(proj)
    _check(load().nucleon_seq_sources(field.handle, C.c_void_p(prop.data_ptr()), io, int(t_sink), pp,
                                      {"u": 0, "d": 1}[flavour], C.c_void_p(out.data_ptr()), _stream()),
           "nucleon_seq_sources")
    del keep
    return out


def nucleon_3pt(field: Field, seqprop, prop, t0: int, gamma_op):
    """sum_y sum_j (g5 Sigma_j(y))^+ gamma_op x_j(y) per timeslice relative to t0 ([T] complex128)."""
    torch = _torch()
    io = _prop(field, prop)
    if _prop(field, seqprop) != io:
        raise ValueError("sequential propagators and propagator must share the io dtype")
    out = torch.empty((field.dims[0],), dtype=torch.complex128, device="cuda")
    _, gp = keep = _spin_matrix(gamma_op)
    _check(load().nucleon_3pt(field.handle, C.c_void_p(seqprop.data_ptr()), C.c_void_p(prop.data_ptr()), io,
                              int(t0), gp, C.c_void_p(out.data_ptr()), _stream()), "nucleon_3pt")
    del keep
    return out


def ama_combine(appx_g, exact_f=None, appx_f=None):
    """O_AMA = mean_f (exact_f - appx_f) + mean_g appx_g (eqs. caa1, caa2) for
    complex128 GPU tensors [n_g, ...], [n_org, ...], [n_org, ...]."""
    torch = _torch()
    for t in (appx_g, exact_f, appx_f):
        if t is not None and (t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous()):
            raise ValueError("observables must be contiguous complex128 GPU tensors")
    n_g = appx_g.shape[0]
    n_org = 0 if exact_f is None else exact_f.shape[0]
    if n_org and (appx_f is None or appx_f.shape != exact_f.shape or exact_f.shape[1:] != appx_g.shape[1:]):
        raise ValueError("exact_f and appx_f must have one shape, matching appx_g per observable")
    out = torch.empty(appx_g.shape[1:], dtype=torch.complex128, device="cuda")
    ln = out.numel()
    ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
    _check(load().ama_combine(ln, n_g, ptr(appx_g), n_org, ptr(exact_f), ptr(appx_f), ptr(out), _stream()),
           "ama_combine")
    return out


def workspace_cached(device: int = 0) -> int:
    """Bytes the process-wide workspace cache holds on a device (free for
    later handles, but counted as used by the device's free-memory query)."""
    n = C.c_size_t()
    _check(load().qcd_workspace_cached(device, C.byref(n)), "workspace_cached")
    return n.value


def workspace_trim(device: int = -1):
    """Free the cached workspace of a device (-1: every device)."""
    _check(load().qcd_workspace_trim(device), "workspace_trim")


def prof_enable(on: bool = True):
    load().qcd_prof_enable(1 if on else 0)


def prof_reset():
    load().qcd_prof_reset()


def prof_get():
    """{class: dict(ms, launches, flops, bytes, units)} since the last reset."""
    L = load()
    out = {}
    for i, name in enumerate(PROF_CLASSES):
        ms, n = C.c_double(), C.c_longlong()
        fl, by, un = C.c_double(), C.c_double(), C.c_double()
        _check(L.qcd_prof_get(i, C.byref(ms), C.byref(n)), "qcd_prof_get")
        _check(L.qcd_prof_get_work(i, C.byref(fl), C.byref(by), C.byref(un)), "qcd_prof_get_work")
        out[name] = dict(ms=ms.value, launches=n.value, flops=fl.value, bytes=by.value, units=un.value)
    return out
