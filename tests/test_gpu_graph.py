"""Batched fixed-iteration solves replayed from captured HIP graphs.

A replay must reproduce, bit for bit, what the same launches compute when
run eagerly: the first batch of each size is run eagerly (without host
synchronisation) and captured, later batches of that size replay the graph.
A fresh handle solving a replayed batch first (eagerly) is the reference.
The replays are repeated with eager torch work and synchronisations in
between, over an uneven mix of Z2-noise and point sources (batches of 4, 4
and 2), and the residuals they report are checked with the oracle.  Both
storage formats of the Schwarz sweeps' own vectors are covered (FP32, and
the FP16 format of the benchmark's sloppy solves).
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

F32, F16 = 1, 2
DIMS, BLOCK = (8, 8, 8, 8), (4, 4, 4, 4)


def _gpu():
    import torch
    import paper_1605_00564_amd as dfl
    return torch, dfl


def make(U, torch, dfl, vecs=F32):
    fld = dfl.Field(DIMS, BLOCK, 0.124, 1.5, U)
    sap = dfl.SapParams(5, 4, F16, vecs)
    d = dfl.Deflation(fld, Ns=8, ninv=3, seed=7, sap=sap)
    p = dfl.GcrParams(nkv=4, fixed_iters=2, res=3e-3, sap=sap, dfl=d, little_tol=1e-6, little_maxit=6)
    return fld, d, p


def sources(torch, dfl, fld):
    z = dfl.z2_sources(fld, seed=2, n=5, dtype=torch.complex128)
    V = synth.volume(DIMS)
    pts = []
    for k in range(5):
        e = np.zeros((V, 4, 3), np.complex128)
        e[(37 * k + 11) % V, k % 4, k % 3] = 1.0
        pts.append(torch.from_numpy(e).cuda())
    # uneven mix: Z2 and point sources interleaved
    return [z[0], pts[0], z[1], pts[1], z[2], pts[2], z[3], pts[3], z[4], pts[4]]


@pytest.mark.parametrize("vecs", [F32, F16])
def test_graph_replay_matches_eager_solves(vecs):
    torch, dfl = _gpu()
    U = synth.gauge_field(DIMS, 0.4, 1)
    op = oracle.Operator(DIMS, U, 0.124, 1.5, -1)
    fld, d, p = make(U, torch, dfl, vecs)
    b = sources(torch, dfl, fld)
    runs = []
    for rep in range(3):
        x, info = dfl.gcr_solve_batched(fld, b, p, batch=4, graph=True)
        runs.append(([v.cpu().numpy() for v in x], info))
        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        _ = float(junk.square().sum())
        torch.cuda.synchronize()
    for rep in (1, 2):
        for r in range(10):
            assert np.array_equal(runs[rep][0][r], runs[0][0][r]), (rep, r)
    # reference: a fresh handle computes batch 1 (sources 4..7) eagerly first
    fld2, d2, p2 = make(U, torch, dfl, vecs)
    b2 = [b[k].clone() for k in (4, 5, 6, 7)]
    x2, info2 = dfl.gcr_solve_batched(fld2, b2, p2, batch=4, graph=True)
    for k, r in enumerate((4, 5, 6, 7)):
        assert np.array_equal(x2[k].cpu().numpy(), runs[0][0][r]), r
        assert info2[k].rel_res == runs[0][1][r].rel_res
    # reported residuals are the FP64 residuals of the returned solutions
    for r in (0, 1, 8, 9):
        bb = b[r].cpu().numpy()
        rr = oracle.norm(bb - op.M(runs[0][0][r])) / oracle.norm(bb)
        assert abs(rr - runs[0][1][r].rel_res) <= 1e-9 * rr, (r, rr, runs[0][1][r].rel_res)
        assert runs[0][1][r].iters == 2
    for h in (d2, fld2, d, fld):
        h.close()


def test_graph_mode_requires_fixed_iterations():
    torch, dfl = _gpu()
    U = synth.gauge_field(DIMS, 0.4, 1)
    fld, d, p = make(U, torch, dfl)
    p.fixed_iters = 0
    b = sources(torch, dfl, fld)[:2]
    with pytest.raises(dfl.DflError) as e:
        dfl.gcr_solve_batched(fld, b, p, batch=2, graph=True)
    assert e.value.code == -1
    d.close()
    fld.close()


def test_autotuner_choice_solves():
    """The autotuner times the valid block shapes (4^4 and 8 x 4^3 here) on
    a trial batch of 4, picks the outer iteration count per shape, times
    batch 8 for the winner, then the stencil variants, and returns ready
    handles.  Solves with its choice report the FP64 residual the oracle
    recomputes, and flag it against the target."""
    torch, dfl = _gpu()
    from paper_1605_00564_amd import tune
    dims = (16, 8, 8, 8)
    U = synth.gauge_field(dims, 0.4, 1)
    choice, fld, d = tune.tune_solver(dims, U, 0.124, 1.5, nsrc=16, batches=(4, 8), Ns=8, ninv=3)
    assert choice.block in ((4, 4, 4, 4), (8, 4, 4, 4)) and choice.batch in (4, 8)
    assert [(t["block"], t["batch"]) for t in choice.table][:2] == [((4, 4, 4, 4), 4), ((8, 4, 4, 4), 4)]
    assert len(choice.table) == 3 and choice.table[2]["batch"] == 8
    assert 2 <= choice.fixed_iters <= 8 and choice.trial_rel_res <= 0.8 * 3e-3
    p = tune.sloppy_params(d, choice.fixed_iters)
    b = list(dfl.z2_sources(fld, seed=5, n=4, dtype=torch.complex128))
    x, info = dfl.gcr_solve_batched(fld, b, p, batch=choice.batch, graph=True)
    op = oracle.Operator(dims, U, 0.124, 1.5, -1)
    for r in range(4):
        bb = b[r].cpu().numpy()
        rr = oracle.norm(bb - op.M(x[r].cpu().numpy())) / oracle.norm(bb)
        assert abs(rr - info[r].rel_res) <= 1e-9 * rr, (r, rr, info[r].rel_res)
        assert (info[r].status == 0) == (rr <= 3e-3) and rr < 1e-2, (r, rr)
    d.close()
    fld.close()


def test_workspace_cache_keeps_and_trims_closed_handles_buffers():
    torch, dfl = _gpu()
    U = synth.gauge_field(DIMS, 0.4, 1)
    dfl.workspace_trim()
    fld, d, p = make(U, torch, dfl)
    b = sources(torch, dfl, fld)[:4]
    dfl.gcr_solve_batched(fld, b, p, batch=4, graph=False)
    outgrown = dfl.workspace_cached(0)     # buffers the handle replaced by larger ones
    d.close()
    fld.close()
    held = dfl.workspace_cached(0)
    assert held > outgrown
    # a new handle of the same size takes the cached buffers back
    fld, d, p = make(U, torch, dfl)
    x, info = dfl.gcr_solve_batched(fld, b, p, batch=4, graph=False)
    assert dfl.workspace_cached(0) < held
    # trimming a live handle gives its buffers back; it allocates again later
    before = dfl.workspace_cached(0)
    fld.trim()
    assert dfl.workspace_cached(0) > before
    x2, _ = dfl.gcr_solve_batched(fld, b, p, batch=4, graph=False)
    for r in range(4):
        assert torch.equal(x2[r], x[r])
    # graphs captured before a trim are dropped: capture, trim, capture again
    xg1, _ = dfl.gcr_solve_batched(fld, b, p, batch=4, graph=True)
    xg2, _ = dfl.gcr_solve_batched(fld, b, p, batch=4, graph=True)      # replay
    fld.trim()
    xg3, _ = dfl.gcr_solve_batched(fld, b, p, batch=4, graph=True)      # eager run and a new capture
    xg4, _ = dfl.gcr_solve_batched(fld, b, p, batch=4, graph=True)      # its replay
    for r in range(4):
        for y in (xg2, xg3, xg4):
            assert torch.equal(y[r], xg1[r])
    d.close()
    fld.close()
    dfl.workspace_trim(0)
    assert dfl.workspace_cached(0) == 0


def test_stencil_knobs_reject_bad_values():
    torch, dfl = _gpu()
    U = synth.gauge_field(DIMS, 0.4, 1)
    fld = dfl.Field(DIMS, BLOCK, 0.124, 1.5, U)
    F = dfl.Field
    for knob, value in ((F.TUNE_STENCIL_RG, 3), (F.TUNE_STENCIL_NR, 3), (99, 1)):
        with pytest.raises(dfl.DflError) as e:
            fld.tune(knob, value)
        assert e.value.code == -1
    for knob, value in ((F.TUNE_STENCIL_RG, 4), (F.TUNE_STENCIL_NR, 4), (F.TUNE_STENCIL_LINKLDS, 0),
                        (F.TUNE_STENCIL_ORDER, 0), (F.TUNE_STENCIL_BLOCK, 1)):
        fld.tune(knob, value)
    fld.close()


def test_graph_cache_follows_the_workspace_layout():
    """A graph captured for batches of 2 inside a 4-wide workspace (the tail
    of 10 sources in batches of 4) writes its solutions at the 4-wide
    layout's address; a later call with 2 sources lays the workspace out
    2-wide, so it must capture its own graph rather than replay that one.
    Both calls on one handle must give exactly what a fresh handle gives."""
    torch, dfl = _gpu()
    U = synth.gauge_field(DIMS, 0.4, 1)
    fld, d, p = make(U, torch, dfl)
    b = sources(torch, dfl, fld)
    dfl.gcr_solve_batched(fld, b, p, batch=4, graph=True)
    two = [b[3].clone(), b[6].clone()]
    x, info = dfl.gcr_solve_batched(fld, two, p, graph=True)
    fld2, d2, p2 = make(U, torch, dfl)
    xr, infor = dfl.gcr_solve_batched(fld2, [v.clone() for v in two], p2, graph=True)
    for k in range(2):
        assert torch.equal(x[k], xr[k]), k
        assert info[k].rel_res == infor[k].rel_res
    # and a replay of the 2-wide graph on the first handle
    x3, _ = dfl.gcr_solve_batched(fld, two, p, graph=True)
    for k in range(2):
        assert torch.equal(x3[k], xr[k]), k
    for h in (d2, fld2, d, fld):
        h.close()
