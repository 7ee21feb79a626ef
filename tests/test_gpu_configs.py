"""GPU parity for the other workloads: device-built sources (Z2 noise,
sequential sources) and the multi-right-hand-side sequential-source workload
(point sources, then sequential sources gamma_5 gamma_mu gamma_5 at t0 + 16,
6^4 Schwarz and deflation blocks, N_s = 20, BF16 link storage and FP16
Schwarz vectors for the sloppy solves, FP64 outer GCR), run at 24^3 x 48 (the smallest lattice of
the uneven multi-field batch) so that the oracle can check it.
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

F64, F32, F16, BF16 = 0, 1, 2, 3


def _gpu():
    import torch
    import paper_1605_00564_amd as dfl
    return torch, dfl


def rel(a, b):
    return float(np.linalg.norm((a - b).reshape(-1)) / np.linalg.norm(b.reshape(-1)))


_st = {}


def small_field():
    if "small" not in _st:
        torch, dfl = _gpu()
        dims, block = (8, 4, 4, 8), (2, 2, 2, 2)
        U = synth.gauge_field(dims, 0.3, 1)
        _st["small"] = (dims, oracle.Operator(dims, U, 0.120, 1.0, -1), dfl.Field(dims, block, 0.120, 1.0, U))
    return _st["small"]


def test_z2_sources_match_counter_generator():
    """Bit for bit: both sides implement SplitMix64 from its definition."""
    torch, dfl = _gpu()
    dims, op, fld = small_field()
    for dt in (torch.complex128, torch.complex64):
        z = dfl.z2_sources(fld, seed=3, n=3, index0=5, dtype=dt).cpu().numpy()
        for r in range(3):
            assert np.array_equal(z[r], synth.z2_source(dims, 3, 5 + r).astype(z.dtype))


@pytest.mark.parametrize("mu", [0, 1, 2, 3])
def test_sequential_sources_match_oracle(mu):
    torch, dfl = _gpu()
    dims, op, fld = small_field()
    psi = synth.gaussian_spinor(dims, 2, 1008)
    eta = dfl.sequential_sources(fld, torch.from_numpy(psi).cuda(), t_sink=5, mu=mu).cpu().numpy()
    ref = oracle.sequential_source(psi, dims, 5, mu)
    assert rel(eta, ref) <= 1e-15


def test_sequential_source_errors():
    torch, dfl = _gpu()
    dims, op, fld = small_field()
    psi = torch.zeros((1, synth.volume(dims), 4, 3), dtype=torch.complex128, device="cuda")
    for t, mu in ((8, 3), (-1, 3), (0, 4)):
        with pytest.raises(dfl.DflError) as e:
            dfl.sequential_sources(fld, psi, t_sink=t, mu=mu)
        assert e.value.code == -1


def test_sequential_workload_6x4_blocks_ns20_bf16():
    """12 point sources at the seeded site, solved sloppily (BF16 links,
    residual 3e-3) and exactly (1e-10); their exact solutions give 12
    sequential sources at t0 + 16 (mu = 3), solved the same two ways.  Every
    sampled solution is checked by the oracle's FP64 residual; one exact
    sequential solution also against the oracle's own solve."""
    torch, dfl = _gpu()
    dims, block = (48, 24, 24, 24), (6, 6, 6, 6)
    kappa, csw = 0.1245, 1.5
    U = synth.gauge_field(dims, 0.4, 1)
    op = oracle.Operator(dims, U, kappa, csw, -1)
    fld = dfl.Field(dims, block, kappa, csw, torch.from_numpy(U).cuda())
    del U
    x0 = synth.seeded_site(dims, 1)
    pos = tuple(int(v) for v in synth.coords(dims, x0))
    sap_bf, sap_32 = dfl.SapParams(5, 4, BF16, F16), dfl.SapParams(5, 4, F32)
    d = dfl.Deflation(fld, Ns=20, ninv=5, seed=7, sap=sap_bf)
    sloppy = dfl.GcrParams(nkv=8, nmx=40, res=3e-3, sap=sap_bf, dfl=d, little_tol=1e-6, little_maxit=8)
    exact = dfl.GcrParams(nkv=16, nmx=400, res=1e-10, sap=sap_32, dfl=d, little_tol=1e-10, little_maxit=16)
    xs, xe, infs, infe = dfl.ama_solve(fld, [pos], [True], sloppy, exact, dtype=torch.complex128)
    assert all(i.status == 0 for i in infs + infe)
    t_sink = (pos[0] + 16) % dims[0]
    seq = dfl.sequential_sources(fld, xe[0], t_sink=t_sink, mu=3)
    ys, info_s = dfl.gcr_solve(fld, seq, sloppy)
    ye, info_e = dfl.gcr_solve(fld, seq, exact)
    assert all(i.status == 0 for i in info_s + info_e)
    print("iterations: point sloppy", infs[0].iters, "exact", infe[0].iters, "sequential sloppy", info_s[0].iters,
          "exact", info_e[0].iters)
    xe0, seq_h, ys_h, ye_h = xe[0].cpu().numpy(), seq.cpu().numpy(), ys.cpu().numpy(), ye.cpu().numpy()
    # the sequential sources are the oracle's insertion on the exact forward solutions
    assert rel(seq_h, oracle.sequential_source(xe0, dims, t_sink, 3)) <= 1e-15
    for sc in (0, 11):
        eta = synth.point_source(dims, x0, sc)
        rr = oracle.norm(eta - op.M(xe0[sc])) / oracle.norm(eta)
        print("forward exact", sc, rr)
        assert rr <= 1.01e-10
        rs = oracle.norm(seq_h[sc] - op.M(ys_h[sc])) / oracle.norm(seq_h[sc])
        re = oracle.norm(seq_h[sc] - op.M(ye_h[sc])) / oracle.norm(seq_h[sc])
        print("sequential sloppy", sc, rs, "exact", re)
        assert rs <= 3e-3 and re <= 1.01e-10
    ref, _ = oracle.solve(op, seq_h[5], block=block, res=1e-12)
    err = rel(ye_h[5], ref)
    print("sequential exact vs oracle solve", err)
    assert err <= 1e-8
    d.close()
    fld.close()
