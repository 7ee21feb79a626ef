"""GPU parity of source and sink smearing (section 2.3): APE-smeared spatial
links and Gaussian smearing against the oracle (FP64 on both sides; the GPU
projects onto SU(3) by a Newton iteration, the oracle by a singular value
decomposition), on a synthetic field at 8^4 with several APE steps."""

import numpy as np
import pytest

import synth
from oracle import smear

pytestmark = pytest.mark.gpu

F64, F32 = 0, 1
DIMS, BLOCK = (8, 8, 8, 8), (4, 4, 4, 4)
ALPHA, NAPE = 0.5, 5


def _gpu():
    import torch
    import paper_1605_00564_amd as dfl
    return torch, dfl


_st = {}


def state():
    if not _st:
        torch, dfl = _gpu()
        U = synth.gauge_field(DIMS, 0.4, 2)
        fld = dfl.Field(DIMS, BLOCK, 0.124, 1.5, U)
        _st.update(U=U, fld=fld, Us=smear.ape_smear(DIMS, U, ALPHA, NAPE))
    return _st


def test_ape_links_match_oracle():
    torch, dfl = _gpu()
    s = state()
    with pytest.raises(dfl.DflError) as e:
        s["fld"].ape_links()
    assert e.value.code == -7
    s["fld"].ape_smear(ALPHA, NAPE)
    got = s["fld"].ape_links().cpu().numpy()
    ref = s["Us"][:, 1:]
    err = np.abs(got - ref).max()
    print("APE links: largest deviation", err)
    assert err <= 1e-13
    eye = np.eye(3)
    assert np.abs(np.conj(np.swapaxes(got, -1, -2)) @ got - eye).max() < 1e-14


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_gauss_smearing_matches_oracle(dtype):
    torch, dfl = _gpu()
    s = state()
    s["fld"].ape_smear(ALPHA, NAPE)
    V = synth.volume(DIMS)
    x = np.stack([synth.point_source(DIMS, synth.lex(DIMS, 3, 1, 2, 5), 7),
                  synth.gaussian_spinor(DIMS, 1, 6001)[0]]).astype(dtype)
    got = dfl.gauss_smear(s["fld"], torch.from_numpy(x).cuda(), 0.4, 12).cpu().numpy()
    ref = smear.gauss_smear(DIMS, s["Us"], x.astype(np.complex128), 0.4, 12)
    tol = 1e-12 if dtype == np.complex128 else 1e-6
    for r in range(2):
        err = np.linalg.norm(got[r] - ref[r]) / np.linalg.norm(ref[r])
        print("gauss smearing", np.dtype(dtype).name, "vector", r, "error", err)
        assert err <= tol
    # the smeared point source stays on its timeslice
    t = np.arange(V) // (V // DIMS[0])
    assert np.abs(got[0][t != 3]).max() == 0


def test_smearing_degenerate_parameters():
    """Zero iterations and zero strength are the identity: APE with n = 0 or
    alpha = 0 returns the original spatial links (SU(3) links are their own
    polar factor, to rounding), Gaussian smearing with n = 0 or kappa_G = 0
    returns its input exactly."""
    torch, dfl = _gpu()
    s = state()
    U = s["U"]
    for alpha, n in ((0.5, 0), (0.0, 3)):
        s["fld"].ape_smear(alpha, n)
        got = s["fld"].ape_links().cpu().numpy()
        assert np.abs(got - U[:, 1:]).max() <= 1e-13, (alpha, n)
    x = torch.from_numpy(synth.gaussian_spinor(DIMS, 2, 6002)).cuda()
    for kappa, n in ((0.4, 0), (0.0, 5)):
        assert torch.equal(dfl.gauss_smear(s["fld"], x, kappa, n), x), (kappa, n)
    # back to the parameters the other tests use
    s["fld"].ape_smear(ALPHA, NAPE)
