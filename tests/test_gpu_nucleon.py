"""GPU parity of the steps after the solve (section 2.3, eq. Nop; section
2.1, eqs. caa1-caa2; section 3.1, eq. delta_c): the nucleon two-point
contraction, the sequential sources of the three-point functions (forward
and backward sinks, both flavours), the three-point contraction and the AMA
combination, each against the oracle on host-built inputs (FP64
arithmetic on both sides: 1e-12 relative to the largest entry; FP32 inputs
are compared with the oracle on the same rounded values).  End to end, the
three-point function from GPU solves of the GPU's sequential sources must
equal the oracle's direct insertion of the current with the dense inverse
on the 4^4 lattice.  The covariance test evaluates delta_c on the projected
two-point function of truncated solves.
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import nucleon as nuc

pytestmark = pytest.mark.gpu

F64, F32, F16 = 0, 1, 2
DIMS, BLOCK = (8, 4, 4, 4), (2, 2, 2, 2)


def _gpu():
    import torch
    import paper_1605_00564_amd as dfl
    return torch, dfl


def relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


_fld = {}


def field(dims=DIMS, block=BLOCK, eps=0.3, kappa=0.120, csw=1.0):
    key = (dims, block)
    if key not in _fld:
        torch, dfl = _gpu()
        U = synth.gauge_field(dims, eps, 1)
        _fld[key] = (U, dfl.Field(dims, block, kappa, csw, U))
    return _fld[key]


def random_prop(dims, seed, dtype=np.complex128):
    return synth.gaussian_spinor(dims, 12, seed).astype(dtype)


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_two_point_contraction_matches_oracle(dtype):
    torch, dfl = _gpu()
    U, fld = field()
    prop = random_prop(DIMS, 5001, dtype)
    for t0 in (0, 5, DIMS[0] - 1):
        got = dfl.nucleon_2pt(fld, torch.from_numpy(prop).cuda(), t0).cpu().numpy()
        ref = nuc.nucleon_2pt(prop.astype(np.complex128), DIMS, t0)
        err = relmax(got, ref)
        print("2pt", dtype.__name__, "t0", t0, "error", err)
        assert err <= 1e-12


@pytest.mark.parametrize("flavour", ["u", "d"])
@pytest.mark.parametrize("direction,t_s", [("forward", 6), ("backward", 2), ("forward", DIMS[0] - 1),
                                           ("backward", 0)])
def test_sequential_sources_match_oracle(flavour, direction, t_s):
    torch, dfl = _gpu()
    U, fld = field()
    prop = random_prop(DIMS, 5002)
    Pp, Pm = nuc.parity_projectors()
    P = Pp if direction == "forward" else Pm
    got = dfl.nucleon_seq_sources(fld, torch.from_numpy(prop).cuda(), t_s, P, flavour).cpu().numpy()
    ref = nuc.nucleon_seq_sources(prop, DIMS, t_s, P, flavour)
    spatial = synth.volume(DIMS) // DIMS[0]
    off = np.ones(synth.volume(DIMS), bool)
    off[t_s * spatial:(t_s + 1) * spatial] = False
    assert np.all(got[:, off] == 0)
    err = relmax(got, ref)
    print("sequential sources", flavour, direction, "error", err)
    assert err <= 1e-12


def test_three_point_contraction_and_ama_combination_match_oracle():
    torch, dfl = _gpu()
    U, fld = field()
    prop = random_prop(DIMS, 5003)
    seq = random_prop(DIMS, 5004)
    g, _ = oracle.gamma_matrices()
    Gop = g[3] @ g[4]
    got = dfl.nucleon_3pt(fld, torch.from_numpy(seq).cuda(), torch.from_numpy(prop).cuda(), 3, Gop).cpu().numpy()
    assert relmax(got, nuc.nucleon_3pt(seq, prop, DIMS, 3, Gop)) <= 1e-12
    rng = np.random.default_rng(9)
    cplx = lambda *s: rng.normal(size=s) + 1j * rng.normal(size=s)
    ag, ef, af = cplx(7, 8, 4, 4), cplx(2, 8, 4, 4), cplx(2, 8, 4, 4)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = dfl.ama_combine(t(ag), t(ef), t(af)).cpu().numpy()
    assert np.abs(out - oracle.ama_estimate(ef, af, ag)).max() <= 1e-14 * np.abs(ag).max()
    out0 = dfl.ama_combine(t(ag)).cpu().numpy()
    assert np.abs(out0 - ag.mean(axis=0)).max() <= 1e-14 * np.abs(ag).max()


@pytest.mark.parametrize("flavour", ["u", "d"])
def test_three_point_function_end_to_end_matches_direct_insertion(flavour):
    """4^4 lattice (eps 0.3, kappa 0.120, c_sw 1.0), point source at
    (t0 = 1, 2, 3, 0): the propagator and the 12 sequential propagators are
    solved on the GPU to residual 1e-12 (SAP-GCR, 2^4 blocks, FP64), the
    sequential sources (forward sink at t0 + 2, P+) and both contractions
    run on the GPU.  Reference: the current A_3 inserted directly into the
    quark line with the oracle's dense inverse, summed over the insertion
    timeslice (bound: solver residual times the condition number)."""
    torch, dfl = _gpu()
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U, fld = field(dims, block)
    op = oracle.Operator(dims, U, 0.120, 1.0, -1)
    Minv = np.linalg.inv(op.dense())
    V = op.V
    g, _ = oracle.gamma_matrices()
    Gop = g[3] @ g[4]
    Pp, _ = nuc.parity_projectors()
    t0 = 1
    t_s = (t0 + 2) % 4
    x0 = synth.lex(dims, t0, 2, 3, 0)
    p = dfl.GcrParams(nkv=16, nmx=400, res=1e-12, sap=dfl.SapParams(5, 4, F64))
    xs, _, info, _ = dfl.ama_solve(fld, [dfl.point((t0, 2, 3, 0))], None, p, p, dtype=torch.complex128)
    prop = xs[0]
    eta = dfl.nucleon_seq_sources(fld, prop, t_s, Pp, flavour)
    sig, _, info2, _ = dfl.ama_solve(fld, [dfl.vectors(eta)], None, p, p, dtype=torch.complex128)
    assert all(i.status == 0 for i in info + info2)
    got = dfl.nucleon_3pt(fld, sig[0], prop, t0, Gop).cpu().numpy()
    # direct insertion with the dense inverse
    Mi = Minv.reshape(V, 12, V, 12)
    S = nuc.propagator_matrix(Mi[:, :, x0, :].transpose(2, 0, 1).reshape(12, V, 4, 3))
    spatial = V // 4
    sink = np.arange(t_s * spatial, (t_s + 1) * spatial)
    Gfull = np.kron(Gop, np.eye(3))
    ref = np.zeros(4, complex)
    for t in range(4):
        ys = np.arange(t * spatial, (t + 1) * spatial)
        Dp = np.einsum("xiyk,kl,ylj->xij", Mi[np.ix_(sink, range(12), ys, range(12))], Gfull,
                       Mi[ys][:, :, x0, :]).reshape(spatial, 4, 3, 4, 3)
        Ss = S[sink]
        Cx = nuc.contract(Ss, Ss, Dp) if flavour == "d" else nuc.contract(Dp, Ss, Ss) + nuc.contract(Ss, Dp, Ss)
        ref[(t - t0) % 4] = np.einsum("ji,xij->", Pp, Cx)
    err = relmax(got, ref)
    print("end-to-end three-point", flavour, "error", err, "condition number", np.linalg.cond(op.dense()))
    assert err <= 1e-9


@pytest.mark.parametrize("sap_storage,tol", [(F64, 1e-11), (F32, 1e-6)])
def test_covariance_violation_of_the_two_point_function(sap_storage, tol):
    """delta_c (section 3.1, eq. delta_c) of the P+ projected nucleon
    two-point function from truncated solves (one GCR iteration, no
    deflation, as in the paper's test): source shifted by g on the gauge
    field shifted by g against the original.  Shifts that map the Schwarz
    block checkerboard onto itself leave it at rounding level on every
    timeslice; others violate it at the truncation level."""
    torch, dfl = _gpu()
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.4, 1)
    fld = dfl.Field(dims, block, 0.124, 1.5, U)
    # res = 0: pure truncated solves (no residual-stopping rescue of misses)
    p = dfl.GcrParams(nkv=8, fixed_iters=1, res=0.0, sap=dfl.SapParams(5, 4, sap_storage))
    x0 = (1, 2, 3, 1)
    Pp, _ = nuc.parity_projectors()
    Ppt = torch.from_numpy(Pp).cuda()

    def corr(f, pos):
        xs, _, _, _ = dfl.ama_solve(f, [dfl.point(pos)], None, p, p, dtype=torch.complex128)
        G = dfl.nucleon_2pt(f, xs[0], pos[0])
        return torch.einsum("ji,tij->t", Ppt, G).cpu().numpy()

    base = corr(fld, x0)
    for gshift, preserving in [((0, 4, 4, 0), True), ((0, 0, 4, 4), True), ((0, 4, 0, 0), False)]:
        fg = dfl.Field(dims, block, 0.124, 1.5, synth.shift_field(dims, U, gshift))
        pos = tuple((x0[m] + gshift[m]) % dims[m] for m in range(4))
        dc = np.abs(corr(fg, pos) / base - 1)
        print("shift", gshift, "|delta_c(t)|", np.array2string(dc, precision=2))
        if preserving:
            assert dc.max() <= tol
        else:
            assert dc.max() > 1e-6
        fg.close()
    fld.close()
