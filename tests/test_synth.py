"""The seeded input generator: the closed-form SU(3) exponential equals the
eigendecomposition exp(i Q) = V exp(i diag(w)) V^+ (a plain definition) on
random traceless Hermitian matrices over a range of scales, including
degenerate spectra, and the generated links are in SU(3)."""

import numpy as np

import synth


def test_closed_form_exponential_matches_eigendecomposition():
    rng = np.random.default_rng(11)
    lam = synth.gell_mann()
    H = np.einsum("na,aij->nij", rng.normal(size=(20000, 8)).astype(np.complex128), lam) * 0.5
    for eps in (1e-9, 0.05, 0.4, 1.0, 3.0):
        w, vec = np.linalg.eigh(eps * H)
        ref = np.einsum("nik,nk,njk->nij", vec, np.exp(1j * w), np.conj(vec))
        assert np.abs(synth.expi_traceless_hermitian(eps * H) - ref).max() < 1e-13, eps
    Q = np.stack([np.zeros((3, 3)), np.diag([0.3, 0.3, -0.6]), np.diag([-0.3, -0.3, 0.6])]).astype(np.complex128)
    ref = np.stack([np.diag(np.exp(1j * np.diag(q))) for q in Q])
    assert np.abs(synth.expi_traceless_hermitian(Q) - ref).max() < 1e-14


def test_gauge_links_are_su3():
    U = synth.gauge_field((4, 4, 4, 6), 0.4, 2)
    assert np.abs(np.conj(np.swapaxes(U, -1, -2)) @ U - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
