"""Pins of the smearing oracle (section 2.3: Gaussian smearing with
APE-smeared links) against facts fixed elsewhere: the unit gauge field is a
fixed point of APE smearing; smeared links are in SU(3); both smearings are
gauge covariant; alpha = 0 leaves SU(3) links unchanged; in the free field a
spatial plane wave is an eigenvector of one Gaussian step with eigenvalue
(1 + 2 kappa sum_i cos p_i) / (1 + 6 kappa); the smearing operator is
Hermitian and does not couple timeslices."""

import numpy as np

import synth
from oracle import smear

DIMS = (4, 4, 4, 6)


def _gauge_transform(dims, U, Om):
    out = np.empty_like(U)
    V = synth.volume(dims)
    idx = np.arange(V).reshape(dims)
    for mu in range(4):
        fwd = np.roll(idx, -1, axis=mu).reshape(-1)
        out[:, mu] = Om @ U[:, mu] @ np.conj(np.swapaxes(Om[fwd], -1, -2))
    return out


def test_ape_fixed_point_su3_and_alpha_zero():
    V = synth.volume(DIMS)
    one = np.tile(np.eye(3, dtype=complex), (V, 4, 1, 1))
    assert np.abs(smear.ape_smear(DIMS, one, 0.5, 3) - one).max() < 1e-14
    U = synth.gauge_field(DIMS, 0.4, 3)
    assert np.abs(smear.ape_smear(DIMS, U, 0.0, 2) - U).max() < 1e-13
    Us = smear.ape_smear(DIMS, U, 0.5, 4)
    eye = np.eye(3)
    assert np.abs(np.conj(np.swapaxes(Us, -1, -2)) @ Us - eye).max() < 1e-13
    assert np.abs(np.linalg.det(Us) - 1).max() < 1e-13
    assert np.array_equal(Us[:, 0], U[:, 0])                   # time links untouched
    # the projection leaves SU(3) matrices unchanged and is the closest
    # unitary matrix: for a matrix near W it returns W
    W = synth.random_su3_field(8, 5)
    assert np.abs(smear.project_su3(2.5 * W) - W).max() < 1e-14


def test_ape_and_gauss_smearing_are_gauge_covariant():
    V = synth.volume(DIMS)
    U = synth.gauge_field(DIMS, 0.4, 3)
    Om = synth.random_su3_field(V, 9)
    Ug = _gauge_transform(DIMS, U, Om)
    Us, Ugs = smear.ape_smear(DIMS, U, 0.5, 3), smear.ape_smear(DIMS, Ug, 0.5, 3)
    assert np.abs(_gauge_transform(DIMS, Us, Om)[:, 1:] - Ugs[:, 1:]).max() < 1e-13
    psi = synth.gaussian_spinor(DIMS, 1, 77)[0]
    a = smear.gauss_smear(DIMS, Us, psi, 0.4, 5)
    b = smear.gauss_smear(DIMS, Ugs, np.einsum("xab,xsb->xsa", Om, psi), 0.4, 5)
    assert np.abs(np.einsum("xab,xsb->xsa", Om, a) - b).max() < 1e-13 * np.abs(a).max()


def test_gauss_free_field_plane_wave_eigenvalue():
    V = synth.volume(DIMS)
    one = np.tile(np.eye(3, dtype=complex), (V, 4, 1, 1))
    c = np.array([synth.coords(DIMS, i) for i in range(V)])
    n = (0, 1, 3, 2)
    p = 2 * np.pi * np.array(n) / np.array(DIMS)
    phase = np.exp(1j * (c[:, 1:] @ p[1:]))
    chi = np.zeros((V, 4, 3), complex)
    chi[:, 2, 1] = phase * (c[:, 0] == 2)                        # one timeslice, one spin-colour
    kappa, N = 0.3, 7
    lam = ((1 + 2 * kappa * np.cos(p[1:]).sum()) / (1 + 6 * kappa)) ** N
    got = smear.gauss_smear(DIMS, one, chi, kappa, N)
    assert np.abs(got - lam * chi).max() < 1e-14


def test_gauss_smearing_is_hermitian_and_timeslice_local():
    U = smear.ape_smear(DIMS, synth.gauge_field(DIMS, 0.4, 3), 0.5, 2)
    a, b = synth.gaussian_spinor(DIMS, 2, 78)
    Sa, Sb = smear.gauss_smear(DIMS, U, a, 0.25, 4), smear.gauss_smear(DIMS, U, b, 0.25, 4)
    assert abs(np.vdot(a, Sb) - np.vdot(Sa, b)) < 1e-12 * abs(np.vdot(a, Sb))
    V = synth.volume(DIMS)
    t = np.array([synth.coords(DIMS, i)[0] for i in range(V)])
    src = a * (t == 3)[:, None, None]
    out = smear.gauss_smear(DIMS, U, src, 0.25, 4)
    assert np.abs(out[t != 3]).max() == 0 and np.abs(out[t == 3]).max() > 0
