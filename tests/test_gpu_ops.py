"""GPU parity of the stencil and the Schwarz preconditioner against the oracle.

FP64 paths must agree to 1e-12 relative per application; reduced-precision
storage (FP32, FP16, BF16 links and clover, FP32 arithmetic) to 1e-5 per
operator application against the oracle evaluated on identically quantised
inputs.  M_SAP eta chains about n_cy (n_mr + 2) = 30 operator applications
with data-dependent minimal-residual coefficients.  Its bound depends on
the storage (SAP_TOL): FP32 storage 1e-6 (FP32 arithmetic on FP32-rounded
inputs; observed about 1e-7); FP16 storage 1e-5 (the per-application
bound: both sides build the clover entries independently in FP64, and the
few entries at an FP16 rounding boundary round to neighbouring values);
BF16 storage 3e-5 (that floor plus the chain bound of about 30 FP32
applications at 1e-6 each; observed about 1.1e-5 on the small lattices).
With the sweeps' own vectors in FP16 (stored block residuals and the
half-spinors handed across block faces, a power-of-two scale per site) each
stored vector carries one FP16 rounding, at most u = 2^-11 of its site's
largest entry; a cycle's stored residual enters the output once, through
that cycle's corrections, so the bound against the same quantised oracle is
n_cy u (SAP_TOL_V16).
"""

import numpy as np
import pytest

import oracle
import synth
from tests import quant

pytestmark = pytest.mark.gpu

F64, F32, F16, BF16 = 0, 1, 2, 3
SAP_TOL = {F32: 1e-6, F16: 1e-5, BF16: 3e-5}
SAP_TOL_V16 = 5 * 2.0 ** -11


def _gpu():
    import torch
    import paper_1605_00564_amd as dfl
    return torch, dfl


def rel(a, b):
    return float(np.linalg.norm((a - b).reshape(-1)) / np.linalg.norm(b.reshape(-1)))


class Case:
    def __init__(self, dims, block, eps, kappa, csw, bc_t=-1, seed=1):
        torch, dfl = _gpu()
        self.dims, self.block = dims, block
        self.U = synth.gauge_field(dims, eps, seed)
        self.op = oracle.Operator(dims, self.U, kappa, csw, bc_t)
        self.field = dfl.Field(dims, block, kappa, csw, self.U, bc_t)
        self._q = {}

    def qop(self, storage):
        """Oracle operator on the storage format's quantised links and clover."""
        if storage not in self._q:
            lk, ck = quant.STORAGE_KIND[storage], quant.CLOVER_KIND[storage]
            q = oracle.Operator(self.dims, quant.quantise_links(self.U, lk), self.op.kappa, self.op.csw, self.op.bc_t,
                                Am=quant.quantise_clover(self.op.Am, ck))
            q.Ainv = quant.quantise_clover(self.op.Ainv, ck)
            self._q[storage] = q
        return self._q[storage]


_cases = {}


def case(*key):
    if key not in _cases:
        _cases[key] = Case(*key)
    return _cases[key]


SMALL = ((8, 4, 4, 8), (2, 2, 2, 2), 0.3, 0.120, 1.0)
MID = ((8, 8, 8, 16), (4, 4, 4, 4), 0.4, 0.124, 1.5)


@pytest.mark.parametrize("key", [SMALL, MID, SMALL + (1,)])
def test_dirac_fp64_matches_oracle(key):
    torch, dfl = _gpu()
    c = case(*key)
    x = synth.gaussian_spinor(c.dims, 5, 1001)
    y = dfl.dirac_apply(c.field, torch.from_numpy(x).cuda(), storage=F64).cpu().numpy()
    ref = c.op.M(x)
    for r in range(5):
        assert rel(y[r], ref[r]) <= 1e-12, r


@pytest.mark.parametrize("storage", [F32, F16, BF16])
@pytest.mark.parametrize("key", [SMALL, MID])
def test_dirac_reduced_precision_matches_quantised_oracle(key, storage):
    torch, dfl = _gpu()
    c = case(*key)
    x = synth.gaussian_spinor(c.dims, 6, 1002).astype(np.complex64)
    y = dfl.dirac_apply(c.field, torch.from_numpy(x).cuda(), storage=storage).cpu().numpy()
    ref = c.qop(storage).M(x.astype(np.complex128))
    unq = c.op.M(x.astype(np.complex128))
    for r in range(6):
        assert rel(y[r], ref[r]) <= 1e-5, (r, rel(y[r], ref[r]))
    # quantisation error against the unquantised operator: reported, bounded loosely
    assert rel(y[0], unq[0]) < {F32: 1e-6, F16: 3e-3, BF16: 2e-2}[storage]


@pytest.mark.parametrize("storage", [F64, F32, F16])
def test_dirac_launch_variants_agree_bit_for_bit(storage):
    """The block-staged stencil with 1, 2 or 4 right-hand sides per
    workgroup, and (FP16 links) the variant holding the block's links in LDS,
    do the same arithmetic per site whatever the lane mapping: outputs are
    identical (so are the site-tile kernel's with 1, 2 or 4 per tile), the
    two kernels agree to rounding, and both match the oracle.  16 right-hand
    sides on 4^4 blocks; FP64 uses at most 2 per workgroup (LDS)."""
    torch, dfl = _gpu()
    c = case(*MID)
    dt = np.complex128 if storage == F64 else np.complex64
    x = torch.from_numpy(synth.gaussian_spinor(c.dims, 16, 1003).astype(dt)).cuda()
    F = dfl.Field
    outs = {}
    try:
        c.field.tune(F.TUNE_STENCIL_LINKLDS, 0)
        for nr in (1, 2, 4):
            c.field.tune(F.TUNE_STENCIL_NR, nr)
            outs[("blk", nr)] = dfl.dirac_apply(c.field, x, storage=storage)
        c.field.tune(F.TUNE_STENCIL_LINKLDS, 1)      # FP16 links: block's links held in LDS
        outs[("blk", "links in LDS")] = dfl.dirac_apply(c.field, x, storage=storage)
        c.field.tune(F.TUNE_STENCIL_BLOCK, 0)
        for rg in (1, 2, 4):
            c.field.tune(F.TUNE_STENCIL_RG, rg)
            outs[("rg", rg)] = dfl.dirac_apply(c.field, x, storage=storage)
    finally:
        c.field.tune(F.TUNE_STENCIL_BLOCK, 1)
        c.field.tune(F.TUNE_STENCIL_RG, 0)
        c.field.tune(F.TUNE_STENCIL_NR, 0)
        c.field.tune(F.TUNE_STENCIL_LINKLDS, 1)
    ref = outs[("blk", 1)]
    for k, y in outs.items():
        if k[0] == "blk":
            assert torch.equal(y, ref), k
        else:
            assert torch.equal(y, outs[("rg", 1)]), k
            d = float((y - ref).abs().max() / ref.abs().max())
            assert d <= (1e-14 if storage == F64 else 1e-6), (k, d)
    qref = (c.op if storage == F64 else c.qop(storage)).M(x.cpu().numpy().astype(np.complex128))
    for r in range(16):
        assert rel(ref[r].cpu().numpy(), qref[r]) <= (1e-12 if storage == F64 else 1e-5), r


@pytest.mark.parametrize("storage", [F16, BF16])
@pytest.mark.parametrize("key", [SMALL, MID])
def test_dirac_fp16_spinors_match_quantised_oracle(key, storage):
    """FP16 spinor storage with a per-site power-of-two scale.  Input side:
    the oracle applies the same operator to the identically quantised input
    (tests/quant.py reproduces the stored values bit for bit), compared
    before any output rounding (FP32 output): 1e-5.  Output side: the FP16
    output is the same FP32 arithmetic stored in the FP16 format, so it must
    equal the format's encoding of the FP32 output (reproduced bit for bit
    by tests/quant.py) up to isolated one-ulp flips where the two kernels'
    FP32 results straddle an FP16 rounding boundary.  The small lattice uses
    2^4 blocks (site-tile kernel), the other 4^4 blocks (block-staged
    kernel); the batch spans 12 right-hand sides with a dynamic range of
    10^6 between sites."""
    torch, dfl = _gpu()
    c = case(*key)
    x = synth.gaussian_spinor(c.dims, 12, 1005)
    x = x * np.exp(np.linspace(-7.0, 7.0, x.shape[1]))[None, :, None, None]
    x = x.astype(np.complex64)
    xq = quant.quantise_spinor_f16(x)
    xt = torch.from_numpy(x).cuda()
    y32 = dfl.dirac_apply(c.field, xt, storage=storage, spinor_in=F16, spinor_out=F32).cpu().numpy()
    y16 = dfl.dirac_apply(c.field, xt, storage=storage, spinor_in=F16, spinor_out=F16).cpu().numpy()
    q = c.qop(storage)
    for r in (0, 5, 11):
        ref = q.M(xq[r])
        err = rel(y32[r], ref)
        print("fp16 spinors, storage", storage, "rhs", r, "rel err (fp32 out)", err)
        assert err <= 1e-5
        enc = quant.quantise_spinor_f16(y32[r])
        differ = float(np.mean(enc != y16[r]))
        m = np.maximum(np.abs(enc.real), np.abs(enc.imag)).reshape(enc.shape[0], -1).max(axis=1)
        dd = y16[r] - enc
        d = np.maximum(np.abs(dd.real), np.abs(dd.imag)).reshape(enc.shape[0], -1).max(axis=1)
        worst = float(np.max(d / np.maximum(m, 1e-300)))
        print("fp16 spinors, storage", storage, "rhs", r, "fp16 out vs encoded fp32 out: differing fraction",
              differ, "worst per-site deviation / site max", worst)
        assert differ < 1e-3
        assert worst <= 2.0 ** -10


@pytest.mark.parametrize("key", [SMALL, MID])
def test_sap_fp64_matches_oracle(key):
    torch, dfl = _gpu()
    c = case(*key)
    eta = synth.gaussian_spinor(c.dims, 3, 1003)
    sp = dfl.SapParams(ncy=5, nmr=4, storage=F64)
    psi = dfl.sap_precond(c.field, torch.from_numpy(eta).cuda(), sp).cpu().numpy()
    ref = c.op.sap(eta, c.block, 5, 4)
    for r in range(3):
        assert rel(psi[r], ref[r]) <= 1e-12, (r, rel(psi[r], ref[r]))


@pytest.mark.parametrize("storage", [F32, F16, BF16])
def test_sap_reduced_precision_matches_quantised_oracle(storage):
    torch, dfl = _gpu()
    c = case(*MID)
    eta = synth.gaussian_spinor(c.dims, 2, 1004).astype(np.complex64)
    sp = dfl.SapParams(ncy=5, nmr=4, storage=storage)
    psi = dfl.sap_precond(c.field, torch.from_numpy(eta).cuda(), sp).cpu().numpy()
    ref = c.qop(storage).sap(eta.astype(np.complex128), c.block, 5, 4)
    for r in range(2):
        print("sap storage", storage, "rhs", r, "rel err", rel(psi[r], ref[r]))
        assert rel(psi[r], ref[r]) <= SAP_TOL[storage], (r, rel(psi[r], ref[r]))


@pytest.mark.parametrize("storage", [F16, BF16])
def test_sap_fp16_vectors_match_quantised_oracle(storage):
    """The sweeps' stored residuals and face half-spinors in FP16 (FP32
    arithmetic, FP32 input and output): the same quantised oracle as the FP32
    vectors, to n_cy u, on both the paired (4 rhs) and the unpaired kernels;
    and the FP32-vector result still to its own bound."""
    torch, dfl = _gpu()
    c = case(*MID)
    eta = torch.from_numpy(synth.gaussian_spinor(c.dims, 4, 1007).astype(np.complex64)).cuda()
    ref = c.qop(storage).sap(eta.cpu().numpy().astype(np.complex128), c.block, 5, 4)
    out = {}
    try:
        for pair in (1, 0):
            c.field.tune(dfl.Field.TUNE_SAP_PAIR, pair)
            for vecs in (F32, F16):
                out[pair, vecs] = dfl.sap_precond(c.field, eta, dfl.SapParams(5, 4, storage, vecs)).cpu().numpy()
    finally:
        c.field.tune(dfl.Field.TUNE_SAP_PAIR, 1)
    for r in range(4):
        for pair in (1, 0):
            e16, e32 = rel(out[pair, F16][r], ref[r]), rel(out[pair, F32][r], ref[r])
            print("sap storage", storage, "pair", pair, "rhs", r, "rel err fp16 vectors", e16, "fp32 vectors", e32)
            assert e16 <= SAP_TOL_V16, (pair, r, e16)
            assert e32 <= SAP_TOL[storage], (pair, r, e32)


def test_sap_fp16_vectors_refused_with_wide_storage():
    torch, dfl = _gpu()
    c = case(*MID)
    eta = torch.from_numpy(synth.gaussian_spinor(c.dims, 1, 1008).astype(np.complex64)).cuda()
    for storage in (F64, F32):
        with pytest.raises(dfl.DflError) as e:
            dfl.sap_precond(c.field, eta, dfl.SapParams(5, 4, storage, F16))
        assert e.value.code == -1 and "FP16 Schwarz vectors" in str(e.value)


@pytest.mark.parametrize("storage", [F32, F16])
def test_sap_paired_right_hand_sides(storage):
    """Schwarz sweeps with two right-hand sides per workgroup (4^4 blocks)
    and with one: the same per-site arithmetic, block reductions in another
    order, so both match the quantised oracle and each other to rounding."""
    torch, dfl = _gpu()
    c = case(*MID)
    eta = torch.from_numpy(synth.gaussian_spinor(c.dims, 4, 1006).astype(np.complex64)).cuda()
    sp = dfl.SapParams(ncy=5, nmr=4, storage=storage)
    try:
        c.field.tune(dfl.Field.TUNE_SAP_PAIR, 1)
        paired = dfl.sap_precond(c.field, eta, sp).cpu().numpy()
        c.field.tune(dfl.Field.TUNE_SAP_PAIR, 0)
        single = dfl.sap_precond(c.field, eta, sp).cpu().numpy()
    finally:
        c.field.tune(dfl.Field.TUNE_SAP_PAIR, 1)
    ref = c.qop(storage).sap(eta.cpu().numpy().astype(np.complex128), c.block, 5, 4)
    for r in range(4):
        assert rel(paired[r], ref[r]) <= SAP_TOL[storage] and rel(single[r], ref[r]) <= SAP_TOL[storage], r
        assert rel(paired[r], single[r]) <= 1e-5, (r, rel(paired[r], single[r]))


@pytest.mark.parametrize("dims,block", [
    ((16, 8, 8, 8), (8, 4, 4, 4)),      # 4^3 x 8 blocks, 256 threads
    ((12, 12, 12, 12), (6, 6, 6, 6)),   # 648 sites per parity: ragged workgroup
    ((16, 16, 16, 16), (8, 8, 8, 8)),   # two sites per thread, global exchange buffers
    ((4, 4, 4, 4), (2, 2, 2, 2)),       # 8 sites per parity in a 64-wide workgroup
])
def test_sap_block_shapes(dims, block):
    """Every launch shape of the Schwarz sweep, with FP32 storage and with
    FP16 storage and FP32 or FP16 sweep vectors, against the quantised
    oracle."""
    torch, dfl = _gpu()
    c = case(dims, block, 0.4, 0.124, 1.5)
    eta = synth.gaussian_spinor(dims, 1, 1005).astype(np.complex64)
    x = torch.from_numpy(eta).cuda()
    psi = dfl.sap_precond(c.field, x, dfl.SapParams(5, 4, F32)).cpu().numpy()
    ref = c.qop(F32).sap(eta.astype(np.complex128), block, 5, 4)
    print("sap block", block, "rel err", rel(psi[0], ref[0]))
    assert rel(psi[0], ref[0]) <= SAP_TOL[F32]
    ref16 = c.qop(F16).sap(eta.astype(np.complex128), block, 5, 4)
    for vecs, tol in ((F32, SAP_TOL[F16]), (F16, SAP_TOL_V16)):
        psi = dfl.sap_precond(c.field, x, dfl.SapParams(5, 4, F16, vecs)).cpu().numpy()
        err = rel(psi[0], ref16[0])
        print("sap block", block, "fp16 storage, vectors", vecs, "rel err", err)
        assert err <= tol, (vecs, err)


def test_sap_point_source_and_single_cycle():
    """Point source: most blocks see a zero residual (alpha guard); ncy = 1."""
    torch, dfl = _gpu()
    c = case(*MID)
    eta = synth.point_source(c.dims, 123, 7)[None]
    psi = dfl.sap_precond(c.field, torch.from_numpy(eta).cuda(), dfl.SapParams(1, 4, F64)).cpu().numpy()
    ref = c.op.sap(eta, c.block, 1, 4)
    assert np.all(np.isfinite(psi))
    assert rel(psi[0], ref[0]) <= 1e-12


def test_geometry_errors_are_reported():
    torch, dfl = _gpu()
    U = synth.gauge_field((4, 4, 4, 4), 0.3, 1)
    with pytest.raises(dfl.DflError) as e:
        dfl.Field((4, 4, 4, 4), (4, 2, 2, 2), 0.12, 1.0, U)
    assert e.value.code == -2
    with pytest.raises(dfl.DflError) as e:
        dfl.Field((4, 4, 4, 4), (3, 2, 2, 2), 0.12, 1.0, U)
    assert e.value.code == -2
