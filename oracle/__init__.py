"""Oracle: a plain FP64 CPU implementation of the deflated SAP-GCR solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` import this package; the HIP library
never does, and the two share no code.  Site loops (Dirac operator, clover
term, Schwarz sweeps, little-operator assembly) are plain C in
``oracle.c``; the Krylov solver, the deflation subspace and the AMA driver
are numpy, written in the order the paper states them
(von Hippel, Rae, Shintani, Wittig, arXiv:1605.00564, section 2).

Array conventions: gauge field ``U[V, 4, 3, 3]``, spinor ``psi[V, 4, 3]``
(or ``[n, V, 4, 3]``), complex128, lexicographic sites (see ``synth``).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

import synth

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", _SO + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        I = C.c_int
        D = C.c_double
        L.orc_gamma.argtypes = [P, P]
        L.orc_fhat.argtypes = [P, P, P]
        L.orc_dirac.argtypes = [P, D, I, P, P, P, P]
        L.orc_hop.argtypes = [P, I, P, P, P]
        L.orc_clover_inverse.argtypes = [C.c_long, P, P]
        L.orc_clover_inverse.restype = I
        L.orc_clover_matrices.argtypes = [P, D, D, P, P]
        L.orc_dirac_dirichlet.argtypes = [P, D, I, P, P, P, P, P]
        L.orc_dirac_dirichlet.restype = I
        L.orc_sap.argtypes = [P, D, I, P, I, I, P, P, P, P, P]
        L.orc_sap.restype = I
        L.orc_little_op.argtypes = [P, D, I, P, I, P, P, P, P]
        L.orc_little_op.restype = I
        L.orc_block_map.argtypes = [P, P, P, P]
        L.orc_block_map.restype = I
        L.orc_block_neighbours.argtypes = [P, P, P]
        L.orc_block_neighbours.restype = I
        L.orc_block_sites.argtypes = [P, P, P]
        L.orc_block_sites.restype = I
        L.orc_gaussian_fill.argtypes = [C.c_ulonglong, C.c_long, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(C.c_void_p)


def _dims(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


class GeometryError(ValueError):
    pass


def gamma_matrices():
    """(gamma[5,4,4] = gamma_0..3, gamma_5;  sigma[6,4,4] for mu<nu pairs)."""
    g = np.zeros((5, 4, 4), np.complex128)
    s = np.zeros((6, 4, 4), np.complex128)
    lib().orc_gamma(_p(g), _p(s))
    return g, s


SIGMA_PAIRS = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


# --------------------------------------------------------------------------
# The operator  M = A - kappa H  (section 2.2, the Dirac equation D psi = eta)
# --------------------------------------------------------------------------

@dataclass
class Operator:
    """Kappa-normalised O(a)-improved Wilson operator on one gauge field.

    The clover term is held as one 12x12 matrix per site (``Am``), built from
    the clover field strength ``F``; a caller may pass ``Am`` (and ``Ainv``)
    explicitly, e.g. rounded to a storage format, to evaluate the same
    definition on quantised inputs.
    """
    dims: tuple
    U: np.ndarray
    kappa: float
    csw: float
    bc_t: int = -1
    Am: np.ndarray = field(default=None, repr=False)
    _Ainv: np.ndarray = field(default=None, repr=False)

    def __post_init__(self):
        self.dims = tuple(int(d) for d in self.dims)
        self.U = _c128(self.U)
        self.V = synth.volume(self.dims)
        self.F = np.zeros((self.V, 6, 3, 3), np.complex128)
        lib().orc_fhat(_p(_dims(self.dims)), _p(self.U), _p(self.F))
        if self.Am is None:
            self.Am = self.clover_matrices()
        self.Am = _c128(self.Am)

    # -- site-local pieces ------------------------------------------------
    @property
    def Ainv(self):
        if self._Ainv is None:
            A = np.zeros((self.V, 12, 12), np.complex128)
            bad = lib().orc_clover_inverse(self.V, _p(self.Am), _p(A))
            if bad:
                raise ZeroDivisionError(f"clover term singular on {bad} sites")
            self._Ainv = A
        return self._Ainv

    @Ainv.setter
    def Ainv(self, value):
        self._Ainv = _c128(value)

    def clover_matrices(self):
        """A(x) = 1 + i kappa c_sw sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x), 12x12 per site."""
        A = np.zeros((self.V, 12, 12), np.complex128)
        lib().orc_clover_matrices(_p(_dims(self.dims)), self.kappa, self.csw, _p(self.F), _p(A))
        return A

    # -- operators on fields ----------------------------------------------
    def _each(self, psi, fn):
        psi = _c128(psi)
        if psi.ndim == 4:
            return np.stack([fn(p) for p in psi])
        return fn(psi)

    def M(self, psi):
        def one(p):
            out = np.empty_like(p)
            lib().orc_dirac(_p(_dims(self.dims)), self.kappa, self.bc_t, _p(self.U), _p(self.Am), _p(p), _p(out))
            return out
        return self._each(psi, one)

    def H(self, psi):
        def one(p):
            out = np.empty_like(p)
            lib().orc_hop(_p(_dims(self.dims)), self.bc_t, _p(self.U), _p(p), _p(out))
            return out
        return self._each(psi, one)

    def M_dirichlet(self, psi, block):
        """D_Omega + D_Omega*: M with every hop between different blocks dropped."""
        b = _dims(block)

        def one(p):
            out = np.empty_like(p)
            rc = lib().orc_dirac_dirichlet(_p(_dims(self.dims)), self.kappa, self.bc_t, _p(b),
                                           _p(self.U), _p(self.Am), _p(p), _p(out))
            if rc:
                raise GeometryError(f"invalid block {block} for lattice {self.dims}")
            return out
        return self._each(psi, one)

    def sap(self, eta, block, ncy=5, nmr=4):
        """psi = M_SAP eta: n_cy Schwarz cycles from psi = 0 (section 2.2)."""
        b = _dims(block)
        Ainv = self.Ainv

        def one(e):
            out = np.empty_like(e)
            rc = lib().orc_sap(_p(_dims(self.dims)), self.kappa, self.bc_t, _p(b), int(ncy), int(nmr),
                               _p(self.U), _p(self.Am), _p(Ainv), _p(e), _p(out))
            if rc:
                raise GeometryError(f"invalid block {block} for lattice {self.dims}")
            return out
        return self._each(eta, one)

    def dense(self):
        """The full 12V x 12V matrix of M (tiny lattices only)."""
        n = 12 * self.V
        if n > 12 * 4096:
            raise ValueError("dense operator only for tiny lattices")
        Mm = np.zeros((n, n), np.complex128)
        e = np.zeros((self.V, 4, 3), np.complex128)
        for j in range(n):
            e.reshape(-1)[j] = 1.0
            Mm[:, j] = self.M(e).reshape(-1)
            e.reshape(-1)[j] = 0.0
        return Mm


def vdot(a, b):
    """(a, b) = sum conj(a) b."""
    return np.vdot(a.reshape(-1), b.reshape(-1))


def norm(a):
    return float(np.linalg.norm(a.reshape(-1)))


# --------------------------------------------------------------------------
# Flexible GCR with restarts (section 2.2: right-preconditioned GCR on
# D M_SAP phi = eta, psi = M_SAP phi)
# --------------------------------------------------------------------------

@dataclass
class SolveInfo:
    status: int          # 0 converged, 1 not converged (or fixed count reached)
    iters: int
    rel_res: float       # ||b - M x|| / ||b|| recomputed at exit
    history: list


def gcr(apply_M, prec, b, x0=None, nkv=16, nmx=1000, res=1e-10, fixed_iters=0, reorth=True):
    """Solve M x = b by flexible GCR(nkv) with restarts.

    Per iteration k: z_k = prec(r); w_k = M z_k; classical Gram-Schmidt of
    w_k against w_0..w_{k-1} (beta_jk = (w_j, w_k)); a second pass when the
    norm drops by more than 10x; gamma_k = ||w_k||, w_k /= gamma_k;
    c_k = (w_k, r); r -= c_k w_k.  At the end of a cycle, R alpha = c is solved
    (R_jk = beta_jk, R_kk = gamma_k), x += sum_k alpha_k z_k, and the residual
    is recomputed as b - M x.  ``fixed_iters > 0`` stops after exactly that
    many iterations (the truncated solves of all-mode averaging).
    """
    b = _c128(b)
    nb = norm(b)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    r = b - apply_M(x) if x0 is not None else b.copy()
    hist = [norm(r) / nb if nb > 0 else 0.0]
    iters = 0
    if nb == 0:
        return x, SolveInfo(0, 0, 0.0, hist)
    target = res * nb
    limit = fixed_iters if fixed_iters > 0 else nmx
    while True:
        zs, ws = [], []
        R = np.zeros((nkv, nkv), np.complex128)
        c = np.zeros(nkv, np.complex128)
        k = 0
        while k < nkv and iters < limit:
            z = prec(r)
            w = apply_M(z)
            n0 = norm(w)
            for _pass in range(2):
                if not ws:
                    break
                beta = np.array([vdot(wj, w) for wj in ws])
                for j, wj in enumerate(ws):
                    w = w - beta[j] * wj
                R[:len(ws), k] += beta
                if not reorth or norm(w) > 0.1 * n0:
                    break
            gam = norm(w)
            w = w / gam
            R[k, k] = gam
            c[k] = vdot(w, r)
            r = r - c[k] * w
            zs.append(z)
            ws.append(w)
            k += 1
            iters += 1
            hist.append(norm(r) / nb)
            if fixed_iters <= 0 and norm(r) <= target:
                break
        if k:
            alpha = np.linalg.solve(np.triu(R[:k, :k]), c[:k])
            for j in range(k):
                x = x + alpha[j] * zs[j]
        r = b - apply_M(x)
        rel = norm(r) / nb
        hist.append(rel)
        if fixed_iters > 0:
            if iters >= fixed_iters:
                return x, SolveInfo(0 if rel <= res else 1, iters, rel, hist)
        elif rel <= res:
            return x, SolveInfo(0, iters, rel, hist)
        if iters >= limit:
            return x, SolveInfo(1, iters, rel, hist)


# --------------------------------------------------------------------------
# Block-local deflation (section 2.2: P_L, little operator eq. little,
# solution eq. deflsoln, subspace from N_s global fields restricted to the
# N_b blocks and orthonormalised)
# --------------------------------------------------------------------------

def block_sites(dims, block):
    Nb = synth.volume(dims) // synth.volume(block)
    g = np.zeros(Nb * synth.volume(block), np.int64)
    if lib().orc_block_sites(_p(_dims(dims)), _p(_dims(block)), _p(g)):
        raise GeometryError(f"invalid block {block} for lattice {dims}")
    return g.reshape(Nb, -1)


def block_neighbours(dims, block):
    Nb = synth.volume(dims) // synth.volume(block)
    n = np.zeros((Nb, 9), np.int64)
    if lib().orc_block_neighbours(_p(_dims(dims)), _p(_dims(block)), _p(n)):
        raise GeometryError(f"invalid block {block} for lattice {dims}")
    return n


def block_colours(dims, block):
    V = synth.volume(dims)
    Nb = V // synth.volume(block)
    blk = np.zeros(V, np.int64)
    col = np.zeros(Nb, np.int32)
    if lib().orc_block_map(_p(_dims(dims)), _p(_dims(block)), _p(blk), _p(col)):
        raise GeometryError(f"invalid block {block} for lattice {dims}")
    return blk, col


def random_fields(V, Ns, seed):
    """N_s complex-Gaussian global fields from the counter-based generator."""
    key = int(synth.stream_key(seed, synth.STREAM_DFL))
    out = np.zeros((Ns, V, 4, 3), np.complex128)
    lib().orc_gaussian_fill(C.c_ulonglong(key), Ns * V * 12, _p(out))
    return out


def block_mgs(phi, tol=1e-10):
    """Modified Gram-Schmidt, two passes, within each block: phi[Nb, Ns, n]."""
    phi = phi.copy()
    Nb, Ns, _ = phi.shape
    for l in range(Ns):
        n0 = np.linalg.norm(phi[:, l], axis=1)
        for _pass in range(2):
            for k in range(l):
                ov = np.einsum("bi,bi->b", np.conj(phi[:, k]), phi[:, l])
                phi[:, l] -= ov[:, None] * phi[:, k]
        nl = np.linalg.norm(phi[:, l], axis=1)
        if np.any(nl <= tol * np.maximum(n0, 1e-300)):
            raise np.linalg.LinAlgError("deflation fields are linearly dependent on a block")
        phi[:, l] /= nl[:, None]
    return phi


class Deflation:
    """Deflation subspace Phi, little operator A and the projectors.

    block: the deflation block; sap_block: the Schwarz block of the M_SAP
    inverse iteration (default: the deflation block; the paper ties the two,
    the library allows a deflation block made of several Schwarz blocks).
    nref > 0: after the ninv rounds of v <- M_SAP v, nref rounds of the
    inverse iteration v <- M^{-1} v (each field normalised), the solves done
    by the deflated solver on the current subspace to relative residual
    ref_res, each round followed by a new subspace and little operator
    (section 2.2: inverse iteration refined with the deflated solver)."""

    def __init__(self, op: Operator, block, Ns, ninv=5, seed=7, ncy=5, nmr=4, phi=None, sap_block=None,
                 nref=0, ref_res=1e-2):
        self.op = op
        self.block = tuple(int(b) for b in block)
        self.sap_block = tuple(int(b) for b in sap_block) if sap_block is not None else self.block
        self.Ns = int(Ns)
        self.sites = block_sites(op.dims, self.block)       # [Nb, Vb]
        self.nbr = block_neighbours(op.dims, self.block)    # [Nb, 9]
        self.Nb, self.Vb = self.sites.shape
        self.N = self.Nb * self.Ns
        self.fields = None
        if phi is None:
            v = random_fields(op.V, self.Ns, seed)
            for _ in range(ninv):                          # inverse iteration with M_SAP
                v = op.sap(v, self.sap_block, ncy, nmr)
                for l in range(self.Ns):
                    v[l] /= norm(v[l])
            phi = self._orthonormal_blocks(v)
            self.fields = v
        elif nref:
            raise ValueError("refinement starts from generated global fields")
        self._set_phi(phi)
        for _ in range(nref):                              # inverse iteration with the deflated solver
            v = self.fields.copy()
            for l in range(self.Ns):
                x, _ = solve(op, v[l], self.sap_block, ncy, nmr, dfl=self, res=ref_res)
                v[l] = x / norm(x)
            self.fields = v
            self._set_phi(self._orthonormal_blocks(v))

    def _orthonormal_blocks(self, v):
        """Global fields v[Ns, V, 4, 3] restricted to the blocks, then block MGS."""
        vb = v.reshape(self.Ns, self.op.V, 12)[:, self.sites.reshape(-1), :]
        vb = vb.reshape(self.Ns, self.Nb, self.Vb * 12).transpose(1, 0, 2)
        return block_mgs(vb)

    def _set_phi(self, phi):
        op = self.op
        self.phi = np.ascontiguousarray(phi.reshape(self.Nb, self.Ns, self.Vb * 12), np.complex128)
        self.A = np.zeros((self.Nb, 9, self.Ns, self.Ns), np.complex128)
        rc = lib().orc_little_op(_p(_dims(op.dims)), op.kappa, op.bc_t, _p(_dims(self.block)), self.Ns,
                                 _p(op.U), _p(op.Am), _p(self.phi), _p(self.A))
        if rc:
            raise GeometryError("invalid block geometry")
        self._lu = None

    # -- restriction / prolongation --------------------------------------
    def restrict(self, v):
        """u = Phi^+ v, u[Nb, Ns]."""
        vb = v.reshape(self.op.V, 12)[self.sites.reshape(-1)].reshape(self.Nb, self.Vb * 12)
        return np.einsum("bki,bi->bk", np.conj(self.phi), vb)

    def prolong(self, u):
        """Phi u as a global field [V, 4, 3]."""
        vb = np.einsum("bki,bk->bi", self.phi, u.reshape(self.Nb, self.Ns))
        out = np.zeros((self.op.V, 12), np.complex128)
        out[self.sites.reshape(-1)] = vb.reshape(-1, 12)
        return out.reshape(self.op.V, 4, 3)

    # -- little operator --------------------------------------------------
    def little_apply(self, v):
        """w = A v with A[B, d] coupling block B to block nbr[B, d]."""
        v = v.reshape(self.Nb, self.Ns)
        return np.einsum("bdkl,bdl->bk", self.A, v[self.nbr])

    def little_dense(self):
        Ad = np.zeros((self.N, self.N), np.complex128)
        Ns = self.Ns
        for B in range(self.Nb):
            for d in range(9):
                Bp = self.nbr[B, d]
                Ad[B * Ns:(B + 1) * Ns, Bp * Ns:(Bp + 1) * Ns] += self.A[B, d]
        return Ad

    def little_solve(self, u, tol=1e-12):
        """c = A^{-1} u: dense LU for N <= 6144, else GCR on A (block-Jacobi)."""
        u = u.reshape(-1)
        if self.N <= 6144:
            if self._lu is None:
                import scipy.linalg as sl
                self._lu = sl.lu_factor(self.little_dense())
            import scipy.linalg as sl
            return sl.lu_solve(self._lu, u).reshape(self.Nb, self.Ns)
        if self._lu is None:
            self._lu = np.linalg.inv(self.A[:, 0])
        jac = lambda r: np.einsum("bkl,bl->bk", self._lu, r.reshape(self.Nb, self.Ns)).reshape(-1)
        x, info = gcr(lambda v: self.little_apply(v).reshape(-1), jac, u, nkv=32, nmx=5000, res=tol)
        return x.reshape(self.Nb, self.Ns)

    # -- projectors and the deflated solution ----------------------------
    def low_mode(self, eta):
        """Phi A^{-1} Phi^+ eta (the second term of eq. deflsoln)."""
        return self.prolong(self.little_solve(self.restrict(eta)))

    def P_R(self, v):
        """P_R v = v - Phi A^{-1} Phi^+ M v."""
        return v - self.low_mode(self.op.M(v))

    def P_L(self, v):
        """P_L v = v - M Phi A^{-1} Phi^+ v."""
        return v - self.op.M(self.low_mode(v))


# --------------------------------------------------------------------------
# Solver entry points
# --------------------------------------------------------------------------

def solve(op: Operator, b, block=None, ncy=5, nmr=4, dfl: Deflation = None, nkv=16, nmx=1000, res=1e-10,
          fixed_iters=0):
    """psi = M^{-1} b by (deflated) SAP-preconditioned flexible GCR.

    Without deflation: preconditioner M_SAP.  With deflation the solution is
    psi = chi + Phi A^{-1} Phi^+ eta (eq. deflsoln) with chi in the range of
    P_R: GCR starts from Phi A^{-1} Phi^+ eta and every search direction is
    P_R M_SAP r, so that the residual it minimises is P_L eta - P_L D chi.
    """
    if block is None:
        prec = lambda r: r.copy()
    else:
        prec = lambda r: op.sap(r, block, ncy, nmr)
    x0 = None
    if dfl is not None:
        base = prec
        prec = lambda r: dfl.P_R(base(r))
        x0 = dfl.low_mode(b)
    return gcr(op.M, prec, b, x0=x0, nkv=nkv, nmx=nmx, res=res, fixed_iters=fixed_iters)


def sequential_source(psi, dims, t_sink, mu=3):
    """Sequential source for a three-point function (section 2.3): the
    forward solution with the insertion gamma_5 gamma_mu gamma_5 on the sink
    timeslice, zero elsewhere.  psi: [..., V, 4, 3]."""
    g, _ = gamma_matrices()
    G = g[4] @ g[mu] @ g[4]
    V = synth.volume(dims)
    spatial = V // dims[0]
    sel = (np.arange(V) // spatial) == t_sink
    out = np.zeros_like(psi, dtype=np.complex128)
    out[..., sel, :, :] = np.einsum("st,...vtc->...vsc", G, psi[..., sel, :, :])
    return out


def ama_positions(dims, block, x0, steps):
    """Source positions x0 + g for a regular grid of shifts g (all-mode
    averaging, section 2.1) that map the block checkerboard onto itself
    (section 2.2): every component of g is a multiple of the block extent
    and the sum of block steps is even."""
    out = []
    for g in steps:
        nblk = [g[m] // block[m] for m in range(4)]
        if any(g[m] % block[m] for m in range(4)) or sum(nblk) % 2:
            raise GeometryError(f"shift {g} does not preserve the block colouring")
        t, x, y, z = synth.coords(dims, x0)
        out.append(synth.lex(dims, (t + g[0]) % dims[0], (x + g[1]) % dims[1], (y + g[2]) % dims[2],
                             (z + g[3]) % dims[3]))
    return out


def ama_estimate(O_exact, O_appx_f, O_appx_g):
    """O_AMA = (1/N_org) sum_f [O^f - O^(appx) f] + (1/N_G) sum_g O^(appx) g (eqs. caa1-caa2)."""
    rest = np.mean(np.asarray(O_exact) - np.asarray(O_appx_f), axis=0)
    return rest + np.mean(np.asarray(O_appx_g), axis=0)
