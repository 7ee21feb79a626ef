"""Pins of the nucleon-correlator oracle (section 2.3, eq. Nop) and of the
AMA estimator (section 2.1, eqs. caa1-caa2) against facts fixed elsewhere:

* the charge-conjugation matrix satisfies C gamma_mu C^-1 = -gamma_mu^T;
* the closed-form two-point contraction equals a brute-force evaluation of
  Wick's theorem (a sum over all quark-antiquark matchings with the sign of
  the permutation), written here from the interpolating fields themselves;
* it is gauge invariant, and reduces in closed form for colour-diagonal
  propagators;
* three-point functions from the sequential sources (forward and backward
  sinks, both flavours) equal the direct insertion of the current into the
  quark line computed with the dense inverse of M on the 4^4 lattice;
* the AMA combination reduces to the exact observable with N_G = N_org = 1
  and f = g, and to the sloppy mean when the exact and sloppy evaluations
  coincide.
"""

import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import nucleon as nuc

DIMS4 = (4, 4, 4, 4)


def test_charge_conjugation_matrix():
    g, _ = oracle.gamma_matrices()
    C = nuc.charge_conjugation()
    Ci = np.linalg.inv(C)
    for mu in range(4):
        assert np.allclose(C @ g[mu] @ Ci, -g[mu].T, atol=1e-15)
    # Gamma = C gamma_5 has one nonzero entry per row and column (the GPU
    # kernels rely on it)
    G = nuc.cg5()
    assert np.all((np.abs(G) > 0).sum(axis=0) == 1) and np.all((np.abs(G) > 0).sum(axis=1) == 1)


def _wick(fields, props):
    """<f_0 f_1 ... f_{n-1}> for Grassmann fields (flavour, bar, index) by
    Wick's theorem: the sum over all matchings of each quark with an
    antiquark of its flavour of the product of propagators <q q-bar>, signed
    by the parity of the permutation that brings every matched pair next to
    each other in the order (q, q-bar)."""
    qs = [i for i, f in enumerate(fields) if not f[1]]
    total = 0.0
    for perm in itertools.permutations([i for i, f in enumerate(fields) if f[1]]):
        if any(fields[q][0] != fields[b][0] for q, b in zip(qs, perm)):
            continue
        order = [k for q, b in zip(qs, perm) for k in (q, b)]
        inv = sum(1 for i in range(len(order)) for j in range(i + 1, len(order)) if order[i] > order[j])
        val = (-1) ** inv
        for q, b in zip(qs, perm):
            val = val * props[fields[q][0]][fields[q][2], fields[b][2]]
        total += val
    return total


def test_two_point_contraction_equals_brute_force_wick():
    rng = np.random.default_rng(5)
    Su = rng.normal(size=(12, 12)) + 1j * rng.normal(size=(12, 12))    # index 3 s + c
    Sd = rng.normal(size=(12, 12)) + 1j * rng.normal(size=(12, 12))
    eps = nuc.levi_civita()
    G = nuc.cg5()
    nz = [(b, g) for b in range(4) for g in range(4) if G[b, g] != 0]
    perms = [(a, b, c) for a in range(3) for b in range(3) for c in range(3) if eps[a, b, c] != 0]
    ref = np.zeros((4, 4), complex)
    for al in range(4):
        for alp in range(4):
            acc = 0.0
            for (a, b, c) in perms:
                for (be, ga) in nz:
                    # N_al = eps_abc Gamma_{be ga} u_{a be} d_{b ga} u_{c al}
                    cN = eps[a, b, c] * G[be, ga]
                    for (a2, b2, c2) in perms:
                        for (gp, bp) in nz:
                            # Nbar_alp = eps_a'b'c' Gamma_{g' b'} ubar_{c' alp} dbar_{b' g'} ubar_{a' b'}
                            # (spins g' of the d-bar, b' of the second u-bar)
                            cB = eps[a2, b2, c2] * G[gp, bp]
                            f = [("u", 0, 3 * be + a), ("d", 0, 3 * ga + b), ("u", 0, 3 * al + c),
                                 ("u", 1, 3 * alp + c2), ("d", 1, 3 * gp + b2), ("u", 1, 3 * bp + a2)]
                            acc += cN * cB * _wick(f, {"u": Su, "d": Sd})
            ref[al, alp] = acc
    mat = lambda S: S.reshape(4, 3, 4, 3)[None]
    got = nuc.contract(mat(Su), mat(Su), mat(Sd))[0]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_two_point_contraction_gauge_invariant_and_colour_trivial_form():
    dims = (4, 2, 2, 2)
    V = synth.volume(dims)
    rng = np.random.default_rng(6)
    prop = rng.normal(size=(12, V, 4, 3)) + 1j * rng.normal(size=(12, V, 4, 3))
    G0 = nuc.nucleon_2pt(prop, dims, 1)
    Om = synth.random_su3_field(V, 17)                  # Omega(x)
    Om0 = synth.random_su3_field(1, 18)[0]              # Omega(x0)
    S = nuc.propagator_matrix(prop)
    Sg = np.einsum("xab,xsbtB,CB->xsatC", Om, S, np.conj(Om0))
    propg = Sg.transpose(3, 4, 0, 1, 2).reshape(12, V, 4, 3)
    G1 = nuc.nucleon_2pt(propg, dims, 1)
    assert np.abs(G1 - G0).max() <= 1e-13 * np.abs(G0).max()
    # colour-diagonal propagator S^{aa'} = delta_{aa'} s: the epsilon sums
    # give C = 6 [ s tr(Gamma s Gamma s^T) + s (Gamma s Gamma)^T s ]
    s = rng.normal(size=(V, 4, 4)) + 1j * rng.normal(size=(V, 4, 4))
    Sd = np.einsum("xij,ab->xiajb", s, np.eye(3))
    Gm = nuc.cg5()
    q = np.einsum("ij,xjk,kl->xil", Gm, s, Gm)
    ref = 6 * (s * np.einsum("xij,xij->x", q, s)[:, None, None] + np.einsum("xij,xkj,xkl->xil", s, q, s))
    assert np.abs(nuc.contract(Sd, Sd, Sd) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.fixture(scope="module")
def dense_inverse():
    U = synth.gauge_field(DIMS4, 0.3, 1)
    op = oracle.Operator(DIMS4, U, 0.120, 1.0, -1)
    return op, np.linalg.inv(op.dense())


@pytest.mark.parametrize("flavour", ["d", "u"])
@pytest.mark.parametrize("direction", ["forward", "backward"])
def test_sequential_sources_reproduce_direct_three_point_function(dense_inverse, flavour, direction):
    """The current Gamma_op inserted on timeslice t of a quark line, summed
    over that timeslice, with the nucleon at zero momentum on the sink
    timeslice: direct evaluation with the dense M^-1 (every S(x, y)) against
    the sequential sources, their solutions and the three-point contraction."""
    op, Minv = dense_inverse
    V = op.V
    g, _ = oracle.gamma_matrices()
    Gop = g[3] @ g[4]                                   # axial current A_3
    Pp, Pm = nuc.parity_projectors()
    x0 = synth.lex(DIMS4, 1, 2, 3, 0)
    t0 = 1
    t_s, P = ((t0 + 2) % 4, Pp) if direction == "forward" else ((t0 - 2) % 4, Pm)
    Mi = Minv.reshape(V, 12, V, 12)
    prop = Mi[:, :, x0, :].transpose(2, 0, 1).reshape(12, V, 4, 3)
    S = nuc.propagator_matrix(prop)
    spatial = V // 4
    sink = np.arange(t_s * spatial, (t_s + 1) * spatial)
    direct = np.zeros(4, complex)
    Gfull = np.kron(Gop, np.eye(3))
    for t in range(4):
        ys = np.arange(t * spatial, (t + 1) * spatial)
        # D'(x) = sum_y S(x, y) Gamma_op S(y, x0) for x on the sink timeslice
        Dp = np.einsum("xiyk,kl,ylj->xij", Mi[np.ix_(sink, range(12), ys, range(12))], Gfull,
                       Mi[ys][:, :, x0, :]).reshape(spatial, 4, 3, 4, 3)
        Ss = S[sink]
        if flavour == "d":
            Cx = nuc.contract(Ss, Ss, Dp)
        else:
            Cx = nuc.contract(Dp, Ss, Ss) + nuc.contract(Ss, Dp, Ss)
        direct[(t - t0) % 4] = np.einsum("ji,xij->", P, Cx)
    eta = nuc.nucleon_seq_sources(prop, DIMS4, t_s, P, flavour)
    sig = np.einsum("xiyk,jyk->jxi", Mi, eta.reshape(12, V, 12)).reshape(12, V, 4, 3)
    via_seq = nuc.nucleon_3pt(sig, prop, DIMS4, t0, Gop)
    assert np.abs(direct).max() > 0
    assert np.abs(via_seq - direct).max() <= 1e-10 * np.abs(direct).max()


def test_ama_estimate_reductions():
    rng = np.random.default_rng(7)
    appx = rng.normal(size=(5, 8)) + 1j * rng.normal(size=(5, 8))
    exact = appx[:2] + 0.01 * (rng.normal(size=(2, 8)))
    # N_G = N_org = 1 with f = g: the exact observable
    assert np.allclose(oracle.ama_estimate(exact[:1], appx[:1], appx[:1]), exact[0], rtol=0, atol=1e-15)
    # exact = sloppy: the sloppy mean over G
    assert np.allclose(oracle.ama_estimate(appx[:2], appx[:2], appx), appx.mean(axis=0), rtol=0, atol=1e-15)
    # linear in the bias correction
    est = oracle.ama_estimate(exact, appx[:2], appx)
    assert np.allclose(est - appx.mean(axis=0), (exact - appx[:2]).mean(axis=0), rtol=0, atol=1e-14)
