"""GPU parity of the solver stack: GCR, deflation, little operator, AMA driver.

Tolerances: exact solves at residual 1e-10 agree with the FP64 oracle to
1e-8 relative; FP64-only paths (little operator on a given basis, restriction,
prolongation) to 1e-12; truncated solves are accepted when the oracle's FP64
operator confirms their residual.
"""

import numpy as np
import pytest

import oracle
import synth
from tests import quant

pytestmark = pytest.mark.gpu

F64, F32, F16, BF16 = 0, 1, 2, 3


def _gpu():
    import torch
    import paper_1605_00564_amd as dfl
    return torch, dfl


def rel(a, b):
    return float(np.linalg.norm((a - b).reshape(-1)) / np.linalg.norm(b.reshape(-1)))


def oracle_relres(op, x, b):
    return oracle.norm(b - op.M(x)) / oracle.norm(b)


_fields = {}


def setup(dims, block, eps, kappa, csw, seed=1):
    key = (dims, block, eps, kappa, csw, seed)
    if key not in _fields:
        torch, dfl = _gpu()
        U = synth.gauge_field(dims, eps, seed)
        _fields[key] = (oracle.Operator(dims, U, kappa, csw, -1), dfl.Field(dims, block, kappa, csw, U))
    return _fields[key]


# ---------------------------------------------------------------------------
# GCR
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sap_storage", [F64, F32])
def test_config0_gcr_sap_matches_dense_lu(sap_storage):
    """4^4, eps 0.3, kappa 0.120, c_sw 1.0, point source (seeded site, sc 0),
    GCR + SAP on 2^4 blocks to relative residual 1e-12; dense LU of the
    3072 x 3072 operator is the reference."""
    torch, dfl = _gpu()
    dims = (4, 4, 4, 4)
    op, fld = setup(dims, (2, 2, 2, 2), 0.3, 0.120, 1.0)
    site = synth.seeded_site(dims, 1)
    eta = synth.point_source(dims, site, 0)[None]
    p = dfl.GcrParams(nkv=16, nmx=200, res=1e-12, sap=dfl.SapParams(5, 4, sap_storage))
    x, info = dfl.gcr_solve(fld, torch.from_numpy(eta).cuda(), p)
    x = x.cpu().numpy()
    Md = op.dense()
    ref = np.linalg.solve(Md, eta.reshape(-1))
    cond = np.linalg.cond(Md)
    assert info[0].status == 0 and info[0].rel_res <= 1e-12
    assert oracle_relres(op, x[0], eta[0]) <= 1.5e-12
    assert np.linalg.norm(x.reshape(-1) - ref) <= 10 * cond * 1e-12 * np.linalg.norm(ref)


def test_gcr_matches_oracle_solution_multi_rhs():
    torch, dfl = _gpu()
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    op, fld = setup(dims, block, 0.4, 0.124, 1.5)
    b = synth.gaussian_spinor(dims, 3, 2001)
    p = dfl.GcrParams(nkv=16, nmx=500, res=1e-10, sap=dfl.SapParams(5, 4, F32))
    x, info = dfl.gcr_solve(fld, torch.from_numpy(b).cuda(), p)
    x = x.cpu().numpy()
    ref, rinfo = oracle.solve(op, b[0], block=block, res=1e-13)
    assert rinfo.status == 0
    for r in range(3):
        assert info[r].status == 0
        assert oracle_relres(op, x[r], b[r]) <= 1.05e-10
    assert rel(x[0], ref) <= 1e-8


@pytest.mark.parametrize("storage", [F16, BF16])
def test_sloppy_solve_reduced_storage(storage):
    torch, dfl = _gpu()
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    op, fld = setup(dims, block, 0.4, 0.124, 1.5)
    b = np.stack([synth.point_source(dims, s, sc) for s, sc in [(0, 0), (77, 5)]])
    p = dfl.GcrParams(nkv=8, nmx=20, res=3e-3, sap=dfl.SapParams(5, 4, storage))
    x, info = dfl.gcr_solve(fld, torch.from_numpy(b).to(torch.complex64).cuda(), p)
    x = x.cpu().numpy().astype(np.complex128)
    for r in range(2):
        assert info[r].status == 0
        assert oracle_relres(op, x[r], b[r]) <= 3e-3


def test_fixed_iteration_count_and_noconv():
    torch, dfl = _gpu()
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    op, fld = setup(dims, block, 0.4, 0.124, 1.5)
    b = synth.gaussian_spinor(dims, 1, 2002)
    p = dfl.GcrParams(nkv=8, fixed_iters=2, res=1e-14, sap=dfl.SapParams(5, 4, F32))
    x, info = dfl.gcr_solve(fld, torch.from_numpy(b).cuda(), p)
    assert info[0].iters == 2
    assert info[0].status == dfl.NOCONV
    assert abs(info[0].rel_res - oracle_relres(op, x.cpu().numpy()[0], b[0])) < 1e-6


def test_nan_source_is_rejected():
    torch, dfl = _gpu()
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    op, fld = setup(dims, block, 0.4, 0.124, 1.5)
    b = synth.gaussian_spinor(dims, 1, 2003)
    b[0, 5, 1, 2] = np.nan
    with pytest.raises(dfl.DflError) as e:
        dfl.gcr_solve(fld, torch.from_numpy(b).cuda(), dfl.GcrParams(res=1e-8, sap=dfl.SapParams(5, 4, F32)))
    assert e.value.code == -6


def test_zero_source_gives_zero_solution():
    torch, dfl = _gpu()
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    op, fld = setup(dims, block, 0.4, 0.124, 1.5)
    b = synth.gaussian_spinor(dims, 2, 2004)
    b[1] = 0
    x, info = dfl.gcr_solve(fld, torch.from_numpy(b).cuda(), dfl.GcrParams(res=1e-9, sap=dfl.SapParams(5, 4, F32)))
    x = x.cpu().numpy()
    assert np.all(x[1] == 0) and info[1].status == 0
    assert oracle_relres(op, x[0], b[0]) <= 1.05e-9


# ---------------------------------------------------------------------------
# deflation
# ---------------------------------------------------------------------------

DFL_KEY = ((8, 8, 8, 8), (4, 4, 4, 4), 0.4, 0.124, 1.5)


@pytest.fixture(scope="module")
def dfl_pair():
    torch, dfl = _gpu()
    op, fld = setup(*DFL_KEY)
    d = dfl.Deflation(fld, Ns=8, ninv=3, seed=11, sap=dfl.SapParams(5, 4, F32))
    return op, fld, d


def test_deflation_fields_match_oracle_subspace(dfl_pair):
    """Same counter-based random fields and inverse iteration (FP32 SAP on the
    GPU, FP64 in the oracle).  The fields before orthonormalisation differ by
    the FP32 rounding of the three M_SAP rounds (at most 1e-6 each, the FP32
    Schwarz bound); an orthonormal basis of their span moves by at most that
    perturbation times the condition number of the block's field matrix, so
    the bound is 3e-6 x (largest block condition number)."""
    op, fld, d = dfl_pair
    phi = d.get_phi().cpu().numpy().reshape(d.Nb, d.Ns, -1)
    ref = oracle.Deflation(op, fld.block, Ns=8, ninv=3, seed=11)
    G = np.einsum("bki,bli->bkl", np.conj(phi), phi)
    assert np.abs(G - np.eye(d.Ns)[None]).max() < 1e-5
    # the oracle's fields before Gram-Schmidt, restricted to the blocks
    v = oracle.random_fields(op.V, 8, 11)
    for _ in range(3):
        v = op.sap(v, fld.block, 5, 4)
        for l in range(8):
            v[l] /= oracle.norm(v[l])
    vb = v.reshape(8, op.V, 12)[:, ref.sites.reshape(-1), :].reshape(8, ref.Nb, -1).transpose(1, 0, 2)
    # column scaling does not move the span: condition numbers of the
    # block matrices with unit columns
    vb = vb / np.linalg.norm(vb, axis=2, keepdims=True)
    kappa = max(np.linalg.cond(vb[b].T) for b in range(ref.Nb))
    # subspace distance: residual of projecting the GPU basis onto the oracle's
    proj = np.einsum("bki,bkj,blj->bli", ref.phi, np.conj(ref.phi), phi)
    dist = np.linalg.norm(phi - proj) / np.linalg.norm(phi)
    print("subspace distance", dist, "largest block condition number", kappa)
    assert dist <= 3e-6 * kappa


@pytest.fixture(scope="module")
def dfl_given_phi(dfl_pair):
    """GPU and oracle with the same (FP32-representable) basis."""
    torch, dfl = _gpu()
    op, fld, d = dfl_pair
    ref0 = oracle.Deflation(op, fld.block, Ns=8, ninv=1, seed=12)
    phi32 = ref0.phi.astype(np.complex64).astype(np.complex128)
    d.set_phi(torch.from_numpy(phi32.reshape(d.Nb, d.Ns, -1, 4, 3)).cuda())
    ref = oracle.Deflation(op, fld.block, Ns=8, phi=phi32)
    return op, fld, d, ref


def test_little_operator_apply_matches_oracle(dfl_given_phi):
    torch, dfl = _gpu()
    op, fld, d, ref = dfl_given_phi
    rng = np.random.default_rng(3)
    v = rng.normal(size=(2, d.Nb, d.Ns)) + 1j * rng.normal(size=(2, d.Nb, d.Ns))
    w = d.little_apply(torch.from_numpy(v).cuda()).cpu().numpy()
    for r in range(2):
        wr = ref.little_apply(v[r]).reshape(d.Nb, d.Ns)
        assert rel(w[r], wr) <= 1e-12


def test_restrict_prolong_match_oracle(dfl_given_phi):
    torch, dfl = _gpu()
    op, fld, d, ref = dfl_given_phi
    v = synth.gaussian_spinor(fld.dims, 2, 2101)
    u = d.restrict(torch.from_numpy(v).cuda()).cpu().numpy()
    for r in range(2):
        assert rel(u[r], ref.restrict(v[r])) <= 1e-12
    c = np.ascontiguousarray(u)
    pv = d.prolong(torch.from_numpy(c).cuda()).cpu().numpy()
    for r in range(2):
        assert rel(pv[r], ref.prolong(c[r])) <= 1e-12


@pytest.mark.parametrize("Ns,n", [(8, 10), (20, 3)])
def test_fp32_restrict_prolong_match_oracle(Ns, n):
    """FP32 vectors: the restriction runs as a real GEMM on the matrix cores
    (FP32 accumulation over 12 V_b complex products), the prolongation on the
    vector units.  Tiles: 16 fields x 8 right-hand sides; Ns = 20 needs two
    field tiles, n = 10 a partial rhs tile.  Bound: FP32 rounding of a sum of
    12 V_b = 3072 products, 1e-5 relative."""
    torch, dfl = _gpu()
    op, fld = setup(*DFL_KEY)
    d = dfl.Deflation(fld, Ns=Ns, ninv=1, seed=13, sap=dfl.SapParams(5, 4, F32))
    # the basis comes from the oracle, rounded to FP32 (the GPU's storage),
    # and is loaded into the handle; the oracle uses exactly those values
    ref0 = oracle.Deflation(op, fld.block, Ns=Ns, ninv=1, seed=13)
    phi = ref0.phi.astype(np.complex64).astype(np.complex128)
    d.set_phi(torch.from_numpy(phi.reshape(d.Nb, d.Ns, -1, 4, 3)).cuda())
    ref = oracle.Deflation(op, fld.block, Ns=Ns, phi=phi)
    v = synth.gaussian_spinor(fld.dims, n, 2102).astype(np.complex64)
    u = d.restrict(torch.from_numpy(v).cuda()).cpu().numpy()
    for r in range(n):
        assert rel(u[r], ref.restrict(v[r].astype(np.complex128))) <= 1e-5, r
    c = np.ascontiguousarray(u)
    pv = d.prolong(torch.from_numpy(c).cuda(), dtype=torch.complex64).cpu().numpy()
    for r in range(n):
        assert rel(pv[r], ref.prolong(c[r])) <= 1e-6, r


def test_little_solve_residual(dfl_given_phi):
    torch, dfl = _gpu()
    op, fld, d, ref = dfl_given_phi
    rng = np.random.default_rng(4)
    v = rng.normal(size=(2, d.Nb, d.Ns)) + 1j * rng.normal(size=(2, d.Nb, d.Ns))
    w, its = d.little_solve(torch.from_numpy(v).cuda(), tol=1e-11, maxit=400)
    w = w.cpu().numpy()
    for r in range(2):
        assert rel(ref.little_apply(w[r]).reshape(d.Nb, d.Ns), v[r]) <= 1.1e-11
        assert rel(w[r], ref.little_solve(v[r])) <= 1e-8


def test_little_solve_rejects_more_than_4096_right_hand_sides(dfl_given_phi):
    """Polled little solves read their norms through a pinned buffer of 4096
    values: larger calls are refused before any launch."""
    torch, dfl = _gpu()
    op, fld, d, ref = dfl_given_phi
    v = torch.zeros((4097, d.Nb, d.Ns), dtype=torch.complex128, device="cuda")
    with pytest.raises(dfl.DflError) as e:
        d.little_solve(v)
    assert e.value.code == -1


def test_deflated_exact_solve_matches_oracle(dfl_given_phi):
    torch, dfl = _gpu()
    op, fld, d, ref = dfl_given_phi
    b = synth.point_source(fld.dims, 300, 4)[None]
    p = dfl.GcrParams(nkv=16, nmx=300, res=1e-10, sap=dfl.SapParams(5, 4, F32), dfl=d, little_tol=1e-10,
                      little_maxit=24)
    x, info = dfl.gcr_solve(fld, torch.from_numpy(b).cuda(), p)
    x = x.cpu().numpy()
    p0 = dfl.GcrParams(nkv=16, nmx=300, res=1e-10, sap=dfl.SapParams(5, 4, F32))
    x0, info0 = dfl.gcr_solve(fld, torch.from_numpy(b).cuda(), p0)
    xo, io = oracle.solve(op, b[0], block=fld.block, dfl=ref, res=1e-13)
    assert info[0].status == 0 and oracle_relres(op, x[0], b[0]) <= 1.05e-10
    assert rel(x[0], xo) <= 1e-8
    assert rel(x0.cpu().numpy()[0], xo) <= 1e-8
    print("iterations deflated", info[0].iters, "undeflated", info0[0].iters)


def _sigma_min_estimate(op, block, v, steps=2):
    """Estimate of the smallest singular value of M by inverse iteration on
    M^+ M with oracle solves: (M^+ M)^-1 = M^-1 g5 M^-1 g5 (gamma_5
    hermiticity).  The Rayleigh quotient approaches the largest eigenvalue
    of (M^+ M)^-1 from below, so 1/sqrt of it estimates sigma_min from above."""
    g5 = np.array([1, 1, -1, -1], float)[None, :, None]
    v = v / oracle.norm(v)
    lam = 0.0
    for _ in range(steps):
        y, _ = oracle.solve(op, g5 * v, block=block, res=1e-8)
        w, _ = oracle.solve(op, g5 * y, block=block, res=1e-8)
        lam = float(np.real(oracle.vdot(v, w)))
        v = w / oracle.norm(w)
    return 1.0 / np.sqrt(lam)


def test_config1_exact_deflated_solve():
    """16^3 x 32, eps 0.4, kappa 0.124, c_sw 1.5, SAP 4^4 with 4 MinRes steps,
    deflation Ns = 12 on 4^4 blocks, one point source, exact to 1e-10 with
    FP64 outer and FP32 SAP.  The exact solution has a plain definition,
    x = M^-1 b: the oracle's own FP64 solve to residual 1e-13 (undeflated, so
    nothing of the GPU's subspace enters) is the reference, at 1e-8.  The
    a-posteriori bound ||r|| / (sigma_min ||x||) is reported beside it, with
    sigma_min estimated by two oracle inverse-iteration steps."""
    torch, dfl = _gpu()
    dims, block = (32, 16, 16, 16), (4, 4, 4, 4)
    op, fld = setup(dims, block, 0.4, 0.124, 1.5)
    d = dfl.Deflation(fld, Ns=12, ninv=5, seed=7, sap=dfl.SapParams(5, 4, F32))
    site = synth.seeded_site(dims, 1)
    b = synth.point_source(dims, site, 0)[None]
    p = dfl.GcrParams(nkv=16, nmx=300, res=1e-10, sap=dfl.SapParams(5, 4, F32), dfl=d, little_tol=1e-10)
    x, info = dfl.gcr_solve(fld, torch.from_numpy(b).cuda(), p)
    x = x.cpu().numpy()
    assert info[0].status == 0
    rr = oracle_relres(op, x[0], b[0])
    assert rr <= 1.05e-10
    xo, io = oracle.solve(op, b[0], block=block, res=1e-13)
    assert io.status == 0
    err = rel(x[0], xo)
    smin = _sigma_min_estimate(op, block, synth.gaussian_spinor(dims, 1, 2201)[0])
    bound = oracle.norm(b[0] - op.M(x[0])) / (smin * oracle.norm(x[0]))
    print(f"config1: iterations {info[0].iters}, residual {rr:.2e}, error vs oracle {err:.2e}, "
          f"sigma_min estimate {smin:.3e}, a-posteriori bound {bound:.2e}")
    assert err <= 1e-8
    d.close()


def test_one_and_two_gcr_iterations_match_oracle_steps():
    """Step parity of the flexible GCR (section 2.2): with fixed iteration
    counts 1 and 2, undeflated, FP32 Schwarz preconditioner, the solution
    x = sum_k alpha_k z_k equals the oracle's GCR run with the same steps on
    the identically quantised FP32 operator (the GPU applies M with FP32
    storage inside a cycle).  Each iteration adds one FP32 M_SAP chain (1e-6,
    the FP32 Schwarz bound)."""
    torch, dfl = _gpu()
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    op, fld = setup(dims, block, 0.4, 0.124, 1.5)
    U = op.U
    q = oracle.Operator(dims, quant.quantise_links(U, quant.STORAGE_KIND[F32]), op.kappa, op.csw, op.bc_t,
                        Am=quant.quantise_clover(op.Am, quant.CLOVER_KIND[F32]))
    q.Ainv = quant.quantise_clover(op.Ainv, quant.CLOVER_KIND[F32])
    b = np.stack([synth.point_source(dims, 77, 5), synth.gaussian_spinor(dims, 1, 2202)[0]])
    for it in (1, 2):
        p = dfl.GcrParams(nkv=8, fixed_iters=it, res=1e-14, sap=dfl.SapParams(5, 4, F32))
        x, info = dfl.gcr_solve(fld, torch.from_numpy(b).cuda(), p)
        x = x.cpu().numpy()
        for r in range(2):
            xo, _ = oracle.gcr(q.M, lambda v: q.sap(v, block, 5, 4), b[r], nkv=8, fixed_iters=it)
            err = rel(x[r], xo)
            print("GCR iterations", it, "rhs", r, "error vs oracle steps", err)
            assert info[r].iters == it
            assert err <= it * 1e-6


# ---------------------------------------------------------------------------
# AMA driver
# ---------------------------------------------------------------------------

def test_ama_matches_direct_solves_and_residuals():
    torch, dfl = _gpu()
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    op, fld = setup(dims, block, 0.4, 0.124, 1.5)
    positions = [(1, 2, 3, 0), (5, 6, 3, 0), (1, 2, 7, 4)]       # shifts of whole blocks, even steps
    sloppy = dfl.GcrParams(nkv=8, nmx=30, res=3e-3, sap=dfl.SapParams(5, 4, F16))
    exact = dfl.GcrParams(nkv=16, nmx=300, res=1e-10, sap=dfl.SapParams(5, 4, F32))
    xs, xe, infs, infe = dfl.ama_solve(fld, positions, [True, False, False], sloppy, exact,
                                       dtype=torch.complex128, batch=12)
    assert len(xs) == 3 and len(xe) == 1
    for g, pos in enumerate(positions):
        lex = synth.lex(dims, *pos)
        xg = xs[g].cpu().numpy()
        for sc in (0, 7, 11):
            eta = synth.point_source(dims, lex, sc)
            assert oracle_relres(op, xg[sc], eta) <= 3e-3
    # the same batch through gcr_solve gives the same numbers
    b = np.stack([synth.point_source(dims, synth.lex(dims, *positions[0]), sc) for sc in range(12)])
    xd, _ = dfl.gcr_solve(fld, torch.from_numpy(b).cuda(), sloppy)
    assert rel(xs[0].cpu().numpy(), xd.cpu().numpy()) <= 1e-14
    xo, _ = oracle.solve(op, b[3], block=block, res=1e-13)
    assert rel(xe[0].cpu().numpy()[3], xo) <= 1e-8
    assert all(i.status == 0 for i in infe)


def test_ama_rejects_colour_changing_shift():
    torch, dfl = _gpu()
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    op, fld = setup(dims, block, 0.4, 0.124, 1.5)
    p = dfl.GcrParams(nkv=4, fixed_iters=1, sap=dfl.SapParams(5, 4, F32))
    for bad in ([(0, 0, 0, 0), (4, 0, 0, 0)], [(0, 0, 0, 0), (2, 0, 0, 0)]):
        with pytest.raises(dfl.DflError) as e:
            dfl.ama_solve(fld, bad, [False, False], p, p)
        assert e.value.code == -2


@pytest.mark.parametrize("sap_storage,tol", [(F64, 1e-12), (F32, 1e-9)])
def test_covariance_under_block_preserving_translation(sap_storage, tol):
    """delta_c test (section 3.1): a truncated solve on the shifted field with
    the shifted source equals the shifted truncated solve when the shift maps
    the block checkerboard onto itself; other shifts break it.  Shifts are
    spatial because the antiperiodic time boundary is not translation
    invariant."""
    torch, dfl = _gpu()
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    op, fld = setup(dims, block, 0.4, 0.124, 1.5)
    b = synth.point_source(dims, synth.lex(dims, 1, 2, 3, 1), 2)[None]
    p = dfl.GcrParams(nkv=8, fixed_iters=1, res=1e-14, sap=dfl.SapParams(5, 4, sap_storage))
    x = dfl.gcr_solve(fld, torch.from_numpy(b).cuda(), p)[0].cpu().numpy()[0]
    for g, preserving in [((0, 4, 4, 0), True), ((0, 0, 4, 4), True), ((0, 4, 0, 0), False),
                          ((0, 1, 0, 0), False)]:
        fg = dfl.Field(dims, block, 0.124, 1.5, synth.shift_field(dims, op.U, g))
        bg = synth.shift_field(dims, b[0], g)[None]
        xg = dfl.gcr_solve(fg, torch.from_numpy(bg).cuda(), p)[0].cpu().numpy()[0]
        dc = rel(xg, synth.shift_field(dims, x, g))
        print("shift", g, "delta_c", dc)
        if preserving:
            assert dc <= tol
        else:
            assert dc > 1e-6
