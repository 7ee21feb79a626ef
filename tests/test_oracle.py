"""Pins of the FP64 oracle against facts fixed by the mathematics.

Each test checks the oracle against something other than itself: the Dirac
algebra typed independently here, free-field plane waves (closed form), a
constant abelian background (closed form of the clover term), gauge and
translation covariance, gamma_5-hermiticity, dense LU, the dense Schwarz
kernel K of section 2.2, and the projector identities of the deflation
(section 2.2).  Sizes are tiny so the whole file runs in well under a minute.
"""

import numpy as np
import pytest

import oracle
import synth

DIMS4 = (4, 4, 4, 4)


# ---------------------------------------------------------------------------
# Gamma matrices typed here independently of the oracle (chiral basis)
# ---------------------------------------------------------------------------

def _gammas_typed():
    i = 1j
    Z = np.zeros((2, 2))
    I2 = np.eye(2)
    s = [np.array([[0, 1], [1, 0]]), np.array([[0, -i], [i, 0]]), np.array([[1, 0], [0, -1]])]
    g0 = np.block([[Z, -I2], [-I2, Z]]).astype(complex)
    gk = [np.block([[Z, -i * sk], [i * sk, Z]]) for sk in s]
    g5 = np.diag([1, 1, -1, -1]).astype(complex)
    return [g0] + gk, g5


def spin_apply(m4, psi):
    """Apply a 4x4 spin matrix to psi[..., 4, 3]."""
    return np.einsum("ij,...jc->...ic", m4, psi)


@pytest.fixture(scope="module")
def field4():
    U = synth.gauge_field(DIMS4, 0.3, 1)
    return oracle.Operator(DIMS4, U, 0.120, 1.0, -1)


def test_gamma_algebra_matches_typed_basis():
    g, sig = oracle.gamma_matrices()
    gt, g5t = _gammas_typed()
    for mu in range(4):
        assert np.allclose(g[mu], gt[mu], atol=0)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2 * (mu == nu) * np.eye(4), atol=1e-15)
        assert np.allclose(g[mu], g[mu].conj().T)
    assert np.allclose(g[4], g5t)
    for p, (mu, nu) in enumerate(oracle.SIGMA_PAIRS):
        ref = 0.5j * (gt[mu] @ gt[nu] - gt[nu] @ gt[mu])
        assert np.allclose(sig[p], ref, atol=1e-15)
        # block diagonal in the chiral basis: chiralities do not mix
        assert np.abs(sig[p][:2, 2:]).max() == 0 and np.abs(sig[p][2:, :2]).max() == 0


def test_sequential_source_is_minus_gamma_mu_on_the_sink_timeslice():
    """gamma_5 anticommutes with gamma_mu, so the insertion equals -gamma_mu
    (typed basis) on the sink timeslice and the source vanishes elsewhere."""
    dims = (4, 2, 2, 2)
    gt, _ = _gammas_typed()
    psi = synth.gaussian_spinor(dims, 2, 1007)
    for mu in range(4):
        eta = oracle.sequential_source(psi, dims, 2, mu)
        V = synth.volume(dims)
        t = np.arange(V) // (V // dims[0])
        assert np.abs(eta[:, t != 2]).max() == 0
        ref = -np.einsum("st,rvtc->rvsc", gt[mu], psi[:, t == 2])
        assert np.allclose(eta[:, t == 2], ref, atol=1e-15)


# ---------------------------------------------------------------------------
# Free field: plane waves are eigenvectors with the closed-form symbol
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("bc_t", [-1, 1])
def test_free_field_plane_waves(bc_t):
    dims = (6, 4, 4, 4)
    V = synth.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy()
    kappa, csw = 0.13, 1.7        # the clover term vanishes on U = 1
    op = oracle.Operator(dims, U, kappa, csw, bc_t)
    gt, _ = _gammas_typed()
    t, x, y, z = synth.coords(dims, np.arange(V))
    rng = np.random.default_rng(0)
    for n in [(0, 0, 0, 0), (1, 2, 0, 3), (2, 1, 1, 1), (5, 3, 2, 1)]:
        shift0 = 0.5 if bc_t == -1 else 0.0
        p = [2 * np.pi * (n[0] + shift0) / dims[0]] + [2 * np.pi * n[m] / dims[m] for m in (1, 2, 3)]
        phase = np.exp(1j * (p[0] * t + p[1] * x + p[2] * y + p[3] * z))
        u = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
        psi = phase[:, None, None] * u[None]
        a = 1 - 2 * kappa * sum(np.cos(pm) for pm in p)
        symb = a * np.eye(4) + 2j * kappa * sum(gt[m] * np.sin(p[m]) for m in range(4))
        expect = phase[:, None, None] * (symb @ u)[None]
        got = op.M(psi)
        assert np.abs(got - expect).max() < 1e-13


def test_free_field_inverse_closed_form():
    dims = (4, 4, 4, 4)
    V = synth.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy()
    kappa = 0.1
    op = oracle.Operator(dims, U, kappa, 1.0, -1)
    gt, _ = _gammas_typed()
    # M(p)^{-1} = (a - i b.gamma)/(a^2 + b^2) with a = 1 - 2k sum cos, b_mu = 2k sin p_mu
    p = [np.pi * 3 / 4, 2 * np.pi / 4, 0.0, 2 * np.pi * 3 / 4]
    t, x, y, z = synth.coords(dims, np.arange(V))
    phase = np.exp(1j * (p[0] * t + p[1] * x + p[2] * y + p[3] * z))
    u = np.arange(12).reshape(4, 3) + 1j
    eta = phase[:, None, None] * u[None]
    a = 1 - 2 * kappa * sum(np.cos(pm) for pm in p)
    b = [2 * kappa * np.sin(pm) for pm in p]
    inv = (a * np.eye(4) - 1j * sum(gt[m] * b[m] for m in range(4))) / (a * a + sum(bb * bb for bb in b))
    expect = phase[:, None, None] * (inv @ u)[None]
    x_sol, info = oracle.solve(op, eta, block=None, res=1e-13, nkv=32)
    assert info.status == 0
    assert np.abs(x_sol - expect).max() < 1e-11


# ---------------------------------------------------------------------------
# Clover term: constant abelian background has a closed-form Fhat
# ---------------------------------------------------------------------------

def test_clover_constant_abelian_field():
    dims = (4, 6, 4, 4)
    T, X, Y, Z = dims
    V = synth.volume(dims)
    nflux = 1
    B = 2 * np.pi * nflux / (X * Y)          # flux per plaquette in the x-y plane
    q = np.array([1.0, -1.0, 0.0])           # U(1) charges embedded in SU(3)
    t, x, y, z = synth.coords(dims, np.arange(V))
    U = np.zeros((V, 4, 3, 3), complex)
    for mu in range(4):
        U[:, mu] = np.eye(3)
    # U_y(x) = exp(i q B x);  U_x = exp(-i q B X y) on the last x-slice
    U[:, 2] = np.einsum("v,c->vc", np.ones(V), np.ones(3))[:, :, None] * np.eye(3)
    ph_y = np.exp(1j * np.outer(B * x, q))
    ph_x = np.where((x == X - 1)[:, None], np.exp(-1j * np.outer(B * X * y, q)), 1.0)
    U[:, 2] = ph_y[:, :, None] * np.eye(3)[None]
    U[:, 1] = ph_x[:, :, None] * np.eye(3)[None]
    kappa, csw = 0.125, 1.3
    op = oracle.Operator(dims, U, kappa, csw, -1)
    Am = op.clover_matrices()
    gt, _ = _gammas_typed()
    s12 = 0.5j * (gt[1] @ gt[2] - gt[2] @ gt[1])
    # Fhat_12 = (4 e^{iqB} - 4 e^{-iqB})/8 = i sin(qB); A = 1 + i k csw sigma_12 (x) Fhat_12
    F12 = np.diag(1j * np.sin(q * B))
    expect = np.eye(12) + 1j * kappa * csw * np.kron(s12, F12)
    assert np.abs(Am - expect[None]).max() < 1e-14
    # and every other plane carries no field strength
    assert np.abs(op.F[:, [0, 1, 2, 4, 5]]).max() < 1e-15


def test_clover_hermitian_chiral_blocks(field4):
    Am = field4.clover_matrices()
    assert np.abs(Am - np.conj(np.swapaxes(Am, 1, 2))).max() < 1e-15
    assert np.abs(Am[:, :6, 6:]).max() < 1e-15 and np.abs(Am[:, 6:, :6]).max() < 1e-15
    Ai = field4.Ainv
    assert np.abs(np.einsum("vij,vjk->vik", Am, Ai) - np.eye(12)).max() < 1e-13


def test_csw_zero_is_plain_wilson(field4):
    op0 = oracle.Operator(DIMS4, field4.U, field4.kappa, 0.0, -1)
    psi = synth.gaussian_spinor(DIMS4, 1, 5)[0]
    assert np.abs(op0.M(psi) - (psi - op0.kappa * op0.H(psi))).max() < 1e-14


# ---------------------------------------------------------------------------
# Symmetries of M
# ---------------------------------------------------------------------------

def test_gamma5_hermiticity(field4):
    _, g5 = _gammas_typed()
    psi = synth.gaussian_spinor(DIMS4, 1, 11)[0]
    phi = synth.gaussian_spinor(DIMS4, 1, 12)[0]
    lhs = oracle.vdot(phi, spin_apply(g5, field4.M(spin_apply(g5, psi))))
    rhs = oracle.vdot(field4.M(phi), psi)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_gauge_covariance(field4):
    V = field4.V
    Om = synth.random_su3_field(V, seed=3)
    U = field4.U
    Ug = np.empty_like(U)
    for mu in range(4):
        fwd = np.array([oracle_neighbour(DIMS4, i, mu) for i in range(V)])
        Ug[:, mu] = Om @ U[:, mu] @ np.conj(np.swapaxes(Om[fwd], 1, 2))
    opg = oracle.Operator(DIMS4, Ug, field4.kappa, field4.csw, -1)
    psi = synth.gaussian_spinor(DIMS4, 1, 21)[0]
    Opsi = np.einsum("vab,vsb->vsa", Om, psi)
    lhs = opg.M(Opsi)
    rhs = np.einsum("vab,vsb->vsa", Om, field4.M(psi))
    assert np.abs(lhs - rhs).max() < 1e-13


def oracle_neighbour(dims, i, mu):
    c = list(synth.coords(dims, i))
    c[mu] = (c[mu] + 1) % dims[mu]
    return synth.lex(dims, *c)


@pytest.mark.parametrize("shift,bc", [((0, 1, 2, 3), -1), ((2, 0, 0, 1), 1)])
def test_translation_covariance(field4, shift, bc):
    op = oracle.Operator(DIMS4, field4.U, field4.kappa, field4.csw, bc)
    Us = synth.shift_field(DIMS4, op.U, shift)
    ops = oracle.Operator(DIMS4, Us, op.kappa, op.csw, bc)
    psi = synth.gaussian_spinor(DIMS4, 1, 31)[0]
    lhs = ops.M(synth.shift_field(DIMS4, psi, shift))
    rhs = synth.shift_field(DIMS4, op.M(psi), shift)
    assert np.abs(lhs - rhs).max() < 1e-13


# ---------------------------------------------------------------------------
# Solves against dense LU
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def dense4(field4):
    return field4.dense()


def test_even_odd_schur_matches_dense(field4, dense4):
    """x_e = Mhat^{-1}(b_e + k H_eo A_oo^{-1} b_o), x_o = A_oo^{-1}(b_o + k H_oe x_e)."""
    V = field4.V
    t, x, y, z = synth.coords(DIMS4, np.arange(V))
    par = (t + x + y + z) % 2
    ie = np.repeat(par == 0, 12)
    io = ~ie
    Md = dense4
    Aee, Heo = Md[np.ix_(ie, ie)], Md[np.ix_(ie, io)]
    Hoe, Aoo = Md[np.ix_(io, ie)], Md[np.ix_(io, io)]
    Aoo_i = np.linalg.inv(Aoo)
    Mhat = Aee - Heo @ Aoo_i @ Hoe       # Heo here already carries -kappa
    b = synth.gaussian_spinor(DIMS4, 1, 41)[0].reshape(-1)
    xe = np.linalg.solve(Mhat, b[ie] - Heo @ Aoo_i @ b[io])
    xo = Aoo_i @ (b[io] - Hoe @ xe)
    xs = np.empty_like(b)
    xs[ie], xs[io] = xe, xo
    assert np.linalg.norm(xs - np.linalg.solve(Md, b)) < 1e-12 * np.linalg.norm(xs)
    # the oracle's per-site A^{-1} is the odd-odd block inverse
    Ai = field4.Ainv
    blocks = np.zeros_like(Aoo_i)
    odd_sites = np.where(par == 1)[0]
    for k, s in enumerate(odd_sites):
        blocks[12 * k:12 * k + 12, 12 * k:12 * k + 12] = Ai[s]
    assert np.abs(blocks - Aoo_i).max() < 1e-13


def test_gcr_sap_solve_matches_dense_lu(field4, dense4):
    """The 4^4 configuration: point source, GCR + SAP on 2^4 blocks, residual 1e-12."""
    site = synth.seeded_site(DIMS4, 1)
    eta = synth.point_source(DIMS4, site, 0)
    x_lu = np.linalg.solve(dense4, eta.reshape(-1))
    x, info = oracle.solve(field4, eta, block=(2, 2, 2, 2), ncy=5, nmr=4, res=1e-12)
    assert info.status == 0
    assert info.rel_res <= 1e-12
    cond = np.linalg.cond(dense4)
    assert np.linalg.norm(x.reshape(-1) - x_lu) <= 10 * cond * 1e-12 * np.linalg.norm(x_lu)
    hist = np.array(info.history[1:-1])
    assert np.all(np.diff(hist) <= 1e-15)     # minimal-residual property within the cycle


def test_gcr_exact_preconditioner_one_iteration(field4, dense4):
    b = synth.gaussian_spinor(DIMS4, 1, 51)[0]
    Minv = np.linalg.inv(dense4)
    prec = lambda r: (Minv @ r.reshape(-1)).reshape(r.shape)
    x, info = oracle.gcr(field4.M, prec, b, res=1e-12)
    assert info.iters == 1 and info.rel_res < 1e-12


def test_gcr_identity_preconditioner_full_krylov():
    dims = (2, 2, 2, 2)
    U = synth.gauge_field(dims, 0.5, 4)
    op = oracle.Operator(dims, U, 0.15, 1.2, -1)
    b = synth.gaussian_spinor(dims, 1, 52)[0]
    x, info = oracle.gcr(op.M, lambda r: r.copy(), b, nkv=200, nmx=200, res=1e-13)
    Md = op.dense()
    assert np.linalg.norm(x.reshape(-1) - np.linalg.solve(Md, b.reshape(-1))) < 1e-11 * np.linalg.norm(x)
    assert info.iters <= 192


# ---------------------------------------------------------------------------
# SAP: the Schwarz kernel K and the polynomial M_SAP of section 2.2
# ---------------------------------------------------------------------------

def _dense_sap(Md, colours_of_sites, ncy):
    on = np.repeat(colours_of_sites == 0, 12)
    off = ~on

    def sub_inv(mask):
        out = np.zeros_like(Md)
        idx = np.where(mask)[0]
        out[np.ix_(idx, idx)] = np.linalg.inv(Md[np.ix_(idx, idx)])
        return out

    D_O_inv, D_Os_inv = sub_inv(on), sub_inv(off)
    D_dOs = np.zeros_like(Md)
    D_dOs[np.ix_(off, on)] = Md[np.ix_(off, on)]     # Omega* receives from Omega
    K = D_O_inv + D_Os_inv - D_Os_inv @ D_dOs @ D_O_inv
    n = Md.shape[0]
    S = np.zeros_like(Md)
    Pw = np.eye(n)
    for _ in range(ncy):
        S += Pw
        Pw = Pw @ (np.eye(n) - Md @ K)
    return K, K @ S


def test_sap_converged_blocks_match_schwarz_kernel(field4, dense4):
    blk, col = oracle.block_colours(DIMS4, (2, 2, 2, 2))
    K, Msap = _dense_sap(dense4, col[blk], 5)
    n = dense4.shape[0]
    # the polynomial identity 1 - M M_SAP = (1 - M K)^ncy
    assert np.abs((np.eye(n) - dense4 @ Msap) - np.linalg.matrix_power(np.eye(n) - dense4 @ K, 5)).max() < 1e-12
    eta = synth.gaussian_spinor(DIMS4, 1, 61)[0]
    ref = (Msap @ eta.reshape(-1))
    got = field4.sap(eta, (2, 2, 2, 2), ncy=5, nmr=64).reshape(-1)
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)
    # few MinRes steps: an approximation, but a contraction of the error
    got4 = field4.sap(eta, (2, 2, 2, 2), ncy=5, nmr=4).reshape(-1)
    assert 1e-8 < np.linalg.norm(got4 - ref) / np.linalg.norm(ref) < 1e-2


def _block_ids(dims, block):
    """Block label and site parity of every lexicographic site, from coordinates."""
    V = synth.volume(dims)
    c = np.array([synth.coords(dims, i) for i in range(V)])
    nb = [dims[m] // block[m] for m in range(4)]
    bc = c // np.array(block)
    lab = ((bc[:, 0] * nb[1] + bc[:, 1]) * nb[2] + bc[:, 2]) * nb[3] + bc[:, 3]
    return lab, bc.sum(axis=1) % 2, c.sum(axis=1) % 2


def _dense_minres_sap(Md, dims, block, eta, ncy, nmr):
    """M_SAP eta from the dense operator: per block the Dirichlet restriction
    D_L = [[D_ee, D_eo], [D_oe, D_oo]] of M, the reduced right-hand side
    rho_e - D_eo D_oo^-1 rho_o, nmr minimal-residual steps on the Schur
    complement D_ee - D_eo D_oo^-1 D_oe from zero, the odd sites by back
    substitution; colour 0 blocks first, then colour 1, ncy cycles."""
    lab, colour, par = _block_ids(dims, block)
    psi = np.zeros(Md.shape[0], complex)
    eta = eta.reshape(-1)
    for _ in range(ncy):
        for c in (0, 1):
            rho = eta - Md @ psi
            for B in np.unique(lab[colour == c]):
                e = np.repeat((lab == B) & (par == 0), 12)
                o = np.repeat((lab == B) & (par == 1), 12)
                Dee, Deo = Md[np.ix_(e, e)], Md[np.ix_(e, o)]
                Doe, Doo = Md[np.ix_(o, e)], Md[np.ix_(o, o)]
                Dooi = np.linalg.inv(Doo)
                Dhat = Dee - Deo @ Dooi @ Doe
                r = rho[e] - Deo @ Dooi @ rho[o]
                x = np.zeros_like(r)
                for _it in range(nmr):
                    p = Dhat @ r
                    a = np.vdot(p, r) / np.vdot(p, p)
                    x = x + a * r
                    r = r - a * p
                psi[e] += x
                psi[o] += Dooi @ (rho[o] - Doe @ x)
    return psi


def test_sap_minres_steps_match_dense_block_solves(field4, dense4):
    """The oracle's Schwarz sweeps with four minimal-residual steps (the
    configurations' n_mr) equal the same steps written with dense matrices
    on the 4^4 lattice with 2^4 blocks: Dirichlet block restriction,
    even-odd Schur complement, residual recomputed per colour."""
    eta = synth.gaussian_spinor(DIMS4, 1, 63)[0]
    ref = _dense_minres_sap(dense4, DIMS4, (2, 2, 2, 2), eta, 5, 4)
    got = field4.sap(eta, (2, 2, 2, 2), ncy=5, nmr=4).reshape(-1)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    ref1 = _dense_minres_sap(dense4, DIMS4, (2, 2, 2, 2), eta, 2, 1)
    got1 = field4.sap(eta, (2, 2, 2, 2), ncy=2, nmr=1).reshape(-1)
    assert np.linalg.norm(got1 - ref1) <= 1e-13 * np.linalg.norm(ref1)


def test_dirichlet_operator_drops_every_hop_between_blocks(field4, dense4):
    """D_Omega + D_Omega*: the dense M with every entry coupling two
    different blocks set to zero."""
    lab, _, _ = _block_ids(DIMS4, (2, 2, 2, 2))
    same = np.repeat(lab, 12)[:, None] == np.repeat(lab, 12)[None, :]
    psi = synth.gaussian_spinor(DIMS4, 1, 64)[0]
    ref = (np.where(same, dense4, 0) @ psi.reshape(-1))
    got = field4.M_dirichlet(psi, (2, 2, 2, 2)).reshape(-1)
    assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)


def test_sap_single_colour_sweep_zeroes_residual_on_blocks(field4):
    """After one exact sweep over colour 0 the residual vanishes on colour-0 blocks."""
    blk, col = oracle.block_colours(DIMS4, (2, 2, 2, 2))
    eta = synth.gaussian_spinor(DIMS4, 1, 62)[0]
    # one cycle = colour 0 then colour 1; the colour-1 sweep leaves colour-1 residual zero
    psi = field4.sap(eta, (2, 2, 2, 2), ncy=1, nmr=64)
    r = (eta - field4.M(psi)).reshape(field4.V, 12)
    on1 = col[blk] == 1
    assert np.abs(r[on1]).max() < 1e-12
    assert np.abs(r[~on1]).max() > 1e-3


def test_sap_rejects_bad_geometry(field4):
    with pytest.raises(oracle.GeometryError):
        field4.sap(synth.gaussian_spinor(DIMS4, 1, 1)[0], (4, 2, 2, 2))   # one block in t: odd count
    with pytest.raises(oracle.GeometryError):
        oracle.block_sites((6, 4, 4, 4), (4, 2, 2, 2))                     # does not divide


def test_sap_covariant_under_block_preserving_shift():
    """M_SAP commutes with translations mapping Omega and Omega* onto themselves."""
    dims = (8, 4, 4, 4)
    U = synth.gauge_field(dims, 0.3, 2)
    op = oracle.Operator(dims, U, 0.12, 1.0, -1)
    eta = synth.gaussian_spinor(dims, 1, 71)[0]
    block = (2, 2, 2, 2)
    ref = op.sap(eta, block, 5, 4)
    for g, preserving in [((0, 2, 2, 0), True), ((0, 0, 0, 4), True), ((0, 2, 0, 0), False), ((0, 1, 0, 0), False)]:
        ops = oracle.Operator(dims, synth.shift_field(dims, U, g), 0.12, 1.0, -1)
        got = ops.sap(synth.shift_field(dims, eta, g), block, 5, 4)
        err = np.linalg.norm(got - synth.shift_field(dims, ref, g)) / np.linalg.norm(ref)
        if preserving:
            assert err < 1e-13
        else:
            assert err > 1e-6


# ---------------------------------------------------------------------------
# Deflation: subspace, little operator, projectors (section 2.2)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def dfl8():
    dims = (8, 4, 4, 4)
    U = synth.gauge_field(dims, 0.3, 5)
    op = oracle.Operator(dims, U, 0.12, 1.0, -1)
    return oracle.Deflation(op, (2, 2, 2, 2), Ns=6, ninv=3, seed=9)


def test_deflation_blocks_orthonormal(dfl8):
    G = np.einsum("bki,bli->bkl", np.conj(dfl8.phi), dfl8.phi)
    assert np.abs(G - np.eye(dfl8.Ns)[None]).max() < 1e-14


def test_little_operator_matches_dense_definition(dfl8):
    op = dfl8.op
    N = dfl8.N
    Adense = np.zeros((N, N), complex)
    e = np.zeros(N, complex)
    for j in range(N):
        e[j] = 1.0
        Adense[:, j] = dfl8.restrict(op.M(dfl8.prolong(e))).reshape(-1)
        e[j] = 0.0
    assert np.abs(dfl8.little_dense() - Adense).max() < 1e-13 * np.abs(Adense).max()
    v = synth.gaussian_spinor((1, 1, 1, N // 12 if N % 12 == 0 else 1), 1, 81).reshape(-1)[:N]
    assert np.abs(dfl8.little_apply(v).reshape(-1) - Adense @ v).max() < 1e-12


def test_projector_identities(dfl8):
    op = dfl8.op
    v = synth.gaussian_spinor(op.dims, 1, 82)[0]
    PLv = dfl8.P_L(v)
    assert oracle.norm(dfl8.P_L(PLv) - PLv) < 1e-12 * oracle.norm(v)               # P_L^2 = P_L
    assert oracle.norm(dfl8.P_L(op.M(dfl8.prolong(np.ones((dfl8.Nb, dfl8.Ns)))))) < 1e-12 * oracle.norm(v)
    assert oracle.norm(dfl8.P_L(op.M(v)) - op.M(dfl8.P_R(v))) < 1e-12 * oracle.norm(op.M(v))   # P_L D = D P_R


def test_complete_subspace_deflation_is_exact_inverse(field4, dense4):
    """N_s = 12 V_b: the block subspace spans everything, so Phi A^-1 Phi^+ = M^-1."""
    block = (2, 2, 2, 2)
    Vb = 16
    d = oracle.Deflation(field4, block, Ns=12 * Vb, ninv=0, seed=3)
    eta = synth.gaussian_spinor(DIMS4, 1, 83)[0]
    got = d.low_mode(eta).reshape(-1)
    ref = np.linalg.solve(dense4, eta.reshape(-1))
    assert np.linalg.norm(got - ref) < 1e-10 * np.linalg.norm(ref)


def test_deflated_solve_agrees_with_undeflated(dfl8):
    op = dfl8.op
    eta = synth.point_source(op.dims, 17, 5)
    x1, i1 = oracle.solve(op, eta, block=(2, 2, 2, 2), dfl=dfl8, res=1e-12)
    x0, i0 = oracle.solve(op, eta, block=(2, 2, 2, 2), res=1e-12)
    assert i1.status == 0 and i0.status == 0
    assert oracle.norm(x1 - x0) < 1e-9 * oracle.norm(x0)
    assert i1.iters <= i0.iters


def test_little_solve_gcr_path_matches_lu(dfl8):
    u = synth.gaussian_spinor((1, 1, 1, 1), 8, 84).reshape(-1)[: dfl8.N]
    u = np.resize(u, dfl8.N)
    ref = dfl8.little_solve(u)
    d2 = dfl8
    saved, d2._lu = d2._lu, None
    N0 = d2.N
    try:
        d2.N = 10 ** 9          # force the iterative branch
        got = d2.little_solve(u, tol=1e-13)
    finally:
        d2.N = N0
        d2._lu = saved
    assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()


def test_deflation_blocks_made_of_schwarz_blocks():
    """Deflation block 4x2x2x2 over Schwarz blocks 2^4 (section 2.2 ties the
    two sizes; the library separates them): the inverse iteration runs with
    the Schwarz block (its fields equal those of the tied 2^4 setup with the
    same seed), the subspace is orthonormal per deflation block, the little
    operator equals Phi^+ M Phi built column by column, P_L D = D P_R, and
    the deflated solve agrees with the undeflated one."""
    dims = (8, 4, 4, 4)
    op = oracle.Operator(dims, synth.gauge_field(dims, 0.3, 5), 0.12, 1.0, -1)
    tied = oracle.Deflation(op, (2, 2, 2, 2), Ns=6, ninv=3, seed=9)
    d = oracle.Deflation(op, (4, 2, 2, 2), Ns=6, ninv=3, seed=9, sap_block=(2, 2, 2, 2))
    assert d.Nb == 16 and d.Vb == 32
    assert np.array_equal(d.fields, tied.fields)
    G = np.einsum("bki,bli->bkl", np.conj(d.phi), d.phi)
    assert np.abs(G - np.eye(d.Ns)[None]).max() < 1e-14
    N = d.N
    Adense = np.zeros((N, N), complex)
    e = np.zeros(N, complex)
    for j in range(N):
        e[j] = 1.0
        Adense[:, j] = d.restrict(op.M(d.prolong(e))).reshape(-1)
        e[j] = 0.0
    assert np.abs(d.little_dense() - Adense).max() < 1e-13 * np.abs(Adense).max()
    v = synth.gaussian_spinor(dims, 1, 85)[0]
    assert oracle.norm(d.P_L(op.M(v)) - op.M(d.P_R(v))) < 1e-12 * oracle.norm(op.M(v))
    eta = synth.point_source(dims, 17, 5)
    x1, i1 = oracle.solve(op, eta, block=(2, 2, 2, 2), dfl=d, res=1e-12)
    x0, i0 = oracle.solve(op, eta, block=(2, 2, 2, 2), res=1e-12)
    assert i1.status == 0 and oracle.norm(x1 - x0) < 1e-9 * oracle.norm(x0)


def test_refinement_is_inverse_iteration_with_the_dense_inverse(field4, dense4):
    """Two rounds of refinement with solves to 1e-13 equal two steps of
    v <- M^{-1} v / ||M^{-1} v|| with the dense inverse applied to the fields
    of the unrefined setup, and the subspace is their block
    orthonormalisation."""
    base = oracle.Deflation(field4, (2, 2, 2, 2), Ns=4, ninv=2, seed=9)
    ref = oracle.Deflation(field4, (2, 2, 2, 2), Ns=4, ninv=2, seed=9, nref=2, ref_res=1e-13)
    V = field4.V
    v = base.fields.reshape(4, V * 12).T
    for _ in range(2):
        v = np.linalg.solve(dense4, v)
        v = v / np.linalg.norm(v, axis=0)
    want = v.T.reshape(4, V, 4, 3)
    assert np.abs(ref.fields - want).max() < 1e-10
    assert np.abs(ref.phi - base._orthonormal_blocks(want)).max() < 1e-10


def test_refinement_moves_the_subspace_towards_the_low_modes(field4, dense4):
    """The four eigenvectors of M with the smallest |lambda| (dense
    eigendecomposition) lie closer to the deflation subspace after each
    round of inverse iteration with the deflated solver."""
    w, vecs = np.linalg.eig(dense4)
    low = vecs[:, np.argsort(np.abs(w))[:4]]

    def mean_distance(d):
        out = []
        for k in range(4):
            u = low[:, k].reshape(field4.V, 4, 3)
            out.append(oracle.norm(u - d.prolong(d.restrict(u))) / oracle.norm(u))
        return np.mean(out)

    dist = [mean_distance(oracle.Deflation(field4, (2, 2, 2, 2), Ns=4, ninv=2, seed=9, nref=n, ref_res=1e-12))
            for n in (0, 1, 2)]
    assert dist[1] < 0.97 * dist[0] and dist[2] < dist[1]


# ---------------------------------------------------------------------------
# AMA bookkeeping (section 2.1)
# ---------------------------------------------------------------------------

def test_ama_estimator_reduces_to_sloppy_mean_when_exact_equals_sloppy():
    rng = np.random.default_rng(1)
    appx = rng.normal(size=(8, 5))
    est = oracle.ama_estimate(appx[:2], appx[:2], appx)
    assert np.allclose(est, appx.mean(axis=0))
    ex = appx[:2] + 1.0
    assert np.allclose(oracle.ama_estimate(ex, appx[:2], appx), appx.mean(axis=0) + 1.0)


def test_ama_positions_preserve_block_colouring():
    dims = (16, 8, 8, 8)
    block = (4, 4, 4, 4)
    x0 = 3
    sites = oracle.ama_positions(dims, block, x0, [(0, 0, 0, 0), (8, 0, 0, 0), (4, 4, 0, 0)])
    assert len(set(sites)) == 3
    with pytest.raises(oracle.GeometryError):
        oracle.ama_positions(dims, block, x0, [(4, 0, 0, 0)])
    with pytest.raises(oracle.GeometryError):
        oracle.ama_positions(dims, block, x0, [(2, 2, 0, 0)])


def test_counter_generator_c_matches_python():
    key_seed = 77
    got = oracle.random_fields(16, 2, key_seed)
    key = synth.stream_key(key_seed, synth.STREAM_DFL)
    g = synth.gaussian(key, np.arange(2 * 2 * 16 * 12, dtype=np.uint64))
    ref = (g[0::2] + 1j * g[1::2]).reshape(2, 16, 4, 3)
    assert np.abs(got - ref).max() < 1e-14

