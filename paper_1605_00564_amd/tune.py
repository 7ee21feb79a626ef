"""Autotuner for the solver's launch and layout choices on one gauge field.

Four choices are made by measurement on the device, never by formula:

* the Schwarz block shape, which is also the deflation block shape (the
  paper ties the two together, section 2.2): every valid candidate shape gets
  its own handle and deflation subspace, and the one with the least time per
  source of a short fixed-iteration batched solve wins;
* the number of outer GCR iterations of the graph-replayed sloppy solves:
  the smallest count whose trial batch stays below a margin of the target
  residual (callers still check every reported residual);
* the number of right-hand sides per solver launch, among the candidates
  that fit the device memory;
* the Dirac stencil's launch variant (block-staged with 1, 2 or 4
  right-hand sides per workgroup, or with the block's links held in LDS, or
  site tiles with 1, 2 or 4 per tile), timed at the chosen batch and set on
  the handle.

The trial solves use Z2-noise sources built on the device and replay a
captured graph, as the production sloppy solves do.  Timings are wall-clock
after device synchronisation, so they include launch overheads.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field as dfield

from . import _lib as L

F16 = L.F16


def valid_blocks(dims, candidates):
    """Shapes b with L_mu divisible by b_mu and an even number of blocks in
    every direction (the block checkerboard must close)."""
    out = []
    for b in candidates:
        if all(Lm % bm == 0 and bm % 2 == 0 and (Lm // bm) % 2 == 0 for Lm, bm in zip(dims, b)):
            out.append(tuple(b))
    return out


def _sync():
    import torch
    torch.cuda.synchronize()


def tune_stencil(fld: L.Field, nrhs: int, storage: int = F16, reps: int = 5):
    """Time the stencil variants on nrhs vectors; set and return the fastest.
    A variant is (block-staged, right-hand sides per site tile, right-hand
    sides per block workgroup, links held in LDS)."""
    import torch
    x = torch.randn((nrhs, fld.V, 4, 3), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    variants = [(1, 0, 1, 0), (1, 0, 2, 0), (1, 0, 4, 0), (1, 0, 2, 1), (0, 1, 0, 0), (0, 2, 0, 0), (0, 4, 0, 0)]
    times = {}
    for blk, rg, nr, llds in variants:
        fld.tune(L.Field.TUNE_STENCIL_BLOCK, blk)
        fld.tune(L.Field.TUNE_STENCIL_RG, rg)
        fld.tune(L.Field.TUNE_STENCIL_NR, nr)
        fld.tune(L.Field.TUNE_STENCIL_LINKLDS, llds)
        L.dirac_apply(fld, x, storage=storage, out=y)
        _sync()
        t = time.perf_counter()
        for _ in range(reps):
            L.dirac_apply(fld, x, storage=storage, out=y)
        _sync()
        times[(blk, rg, nr, llds)] = (time.perf_counter() - t) / reps
    best = min(times, key=times.get)
    fld.tune(L.Field.TUNE_STENCIL_BLOCK, best[0])
    fld.tune(L.Field.TUNE_STENCIL_RG, best[1])
    fld.tune(L.Field.TUNE_STENCIL_NR, best[2])
    fld.tune(L.Field.TUNE_STENCIL_LINKLDS, best[3])
    return best, times


@dataclass
class Choice:
    block: tuple
    batch: int
    fixed_iters: int
    stencil: tuple
    setup_s: float
    per_source_s: float
    trial_rel_res: float
    table: list = dfield(default_factory=list)


def memory_batch_limit(V: int, nkv: int) -> int:
    """Largest batch whose Krylov space (FP32) and FP64 io fit 75% of the
    memory that is free or held by the library's workspace cache (cached
    buffers too small for this lattice are freed when an allocation needs
    their room), rounded down to an even count."""
    import torch
    free, _ = torch.cuda.mem_get_info()
    free += L.workspace_cached(torch.cuda.current_device())
    per = V * (96 * (2 * nkv + 3) + 192 * 5)
    nb = max(1, int(0.75 * free) // per)
    # the Schwarz and stencil kernels take right-hand sides in pairs
    return nb - nb % 2 if nb > 1 else nb


def sloppy_params(d, fixed_iters: int, res: float = 3e-3) -> L.GcrParams:
    """The sloppy solve the tuner times: FP16 storage and FP16 sweep vectors
    in SAP, a fixed number of outer iterations (no host decisions, so it can
    be graph-replayed)."""
    sap = L.SapParams(5, 4, F16, F16)
    return L.GcrParams(nkv=max(2, fixed_iters), fixed_iters=fixed_iters, res=res, sap=sap, dfl=d,
                       little_tol=1e-6, little_maxit=4)


def _trial(fld, d, srcs, nb, iters, res):
    """Capture (first call) and time one replay of a batch of nb sources;
    returns (seconds per source, worst reported FP64 residual)."""
    p = sloppy_params(d, iters, res)
    L.gcr_solve_batched(fld, srcs, p, batch=nb, graph=True)       # eager + capture
    _sync()
    t = time.perf_counter()
    _, info = L.gcr_solve_batched(fld, srcs, p, batch=nb, graph=True)   # replay
    _sync()
    return (time.perf_counter() - t) / nb, max(i.rel_res for i in info)


def rank_by_prior(cands, prior):
    """Order candidate block shapes by a previous tuning's time per source
    per site (shapes it did not time go last, in their given order)."""
    seen = {}
    for row in prior or []:
        b = tuple(row["block"])
        v = row["per_source_s"] / row["volume"]
        seen[b] = min(v, seen.get(b, v))
    return sorted(cands, key=lambda b: (b not in seen, seen.get(b, 0.0)))


def tune_solver(dims, U, kappa, csw, nsrc, blocks=((4, 4, 4, 4), (8, 4, 4, 4), (6, 6, 6, 6), (8, 8, 8, 8)),
                batches=(8, 12, 16, 24), Ns=12, ninv=5, fixed_iters=2, res=3e-3, margin=0.8, max_iters=8,
                prior=None, keep=2, log=None):
    """Pick block shape, outer iteration count and batch for a field with
    nsrc sloppy sources; returns (Choice, field handle, deflation handle) for
    the winner, the handles ready to use (the others are closed).

    Per valid block shape: build the handles (timed as setup), then replay a
    trial batch of Z2-noise sources at fixed_iters outer iterations, adding
    one iteration while the worst FP64 residual exceeds margin x res.  Every
    candidate's setup has been paid by the time the choice is made, so the
    shape with the least time per source wins (its remaining cost is
    nsrc x that time); setup times are reported, not ranked.  For the winner
    alone the other batch sizes are timed, then the stencil variant.

    prior: the table of an earlier tuning with the same kappa, c_sw and
    field recipe (another lattice size).  Its ranking (time per source per
    site) orders the valid shapes, only the best `keep` of them are timed,
    and the search for N_iter starts at the prior winner's count."""
    log = log or (lambda *a: None)
    sap = L.SapParams(5, 4, F16, F16)
    V = 1
    for d in dims:
        V *= d
    cands = valid_blocks(dims, blocks)
    if not cands:
        raise ValueError(f"no valid block shape for {dims}")
    if prior:
        cands = rank_by_prior(cands, prior)[:max(1, keep)]
        known = [r for r in prior if "fixed_iters" in r]
        if known:
            best_prior = min(known, key=lambda r: r["per_source_s"] / r["volume"])
            fixed_iters = max(fixed_iters, int(best_prior["fixed_iters"]) - 1)
    best = None
    table = []
    nb = None
    for b in cands:
        # untimed: free the previous candidate's scratch, so that every
        # candidate's setup makes the same allocations
        L.workspace_trim()
        fld = d = None
        try:
            t0 = time.perf_counter()
            fld = L.Field(dims, b, kappa, csw, U)
            d = L.Deflation(fld, Ns=Ns, ninv=ninv, seed=7, sap=sap)
            _sync()
            setup = time.perf_counter() - t0
            if nb is None:
                # one trial batch size for every shape, so that they compare fairly
                fld.trim()
                nb = max(1, min(nsrc, memory_batch_limit(V, fixed_iters + 2), batches[0]))
            srcs = list(L.z2_sources(fld, seed=99, n=nb))
            iters = fixed_iters
            while True:
                per, worst = _trial(fld, d, srcs, nb, iters, res)
                if worst <= margin * res or iters >= max_iters:
                    break
                iters += 1
            del srcs
            fld.trim()
        except L.DflError as e:
            # a shape whose buffers do not fit beside the handles already held
            # (the best candidate so far, other fields' handles) is no choice
            if e.code != L.QCD_ENOMEM or best is None:
                raise
            log(f"[tune] block {b}: skipped, out of device memory ({e})")
            for h in (d, fld):
                if h is not None:
                    h.close()
            continue
        cost = nsrc * per
        table.append({"block": b, "batch": nb, "fixed_iters": iters, "setup_s": setup, "per_source_s": per,
                      "trial_rel_res": worst, "solve_cost_s": cost, "volume": V})
        log(f"[tune] block {b} batch {nb} N_iter {iters}: setup {setup:.2f} s, {per * 1e3:.1f} ms/source, "
            f"residual {worst:.2e}, solve cost {cost:.2f} s")
        if best is None or cost < best[0]:
            if best is not None:
                best[3].close()
                best[2].close()
            best = (cost, Choice(b, nb, iters, (1, 0, 0, 1), setup, per, worst), fld, d)
        else:
            d.close()
            fld.close()
    _, choice, fld, d = best
    limit = memory_batch_limit(V, max(2, choice.fixed_iters) + 1)
    for nb in [n for n in batches if choice.batch < n <= min(limit, nsrc)]:
        srcs = list(L.z2_sources(fld, seed=99, n=nb))
        per, worst = _trial(fld, d, srcs, nb, choice.fixed_iters, res)
        del srcs
        table.append({"block": choice.block, "batch": nb, "fixed_iters": choice.fixed_iters,
                      "setup_s": choice.setup_s, "per_source_s": per, "trial_rel_res": worst,
                      "solve_cost_s": nsrc * per, "volume": V})
        log(f"[tune] block {choice.block} batch {nb}: {per * 1e3:.1f} ms/source")
        if per < choice.per_source_s and worst <= margin * res:
            choice.batch, choice.per_source_s, choice.trial_rel_res = nb, per, worst
    choice.stencil, stimes = tune_stencil(fld, choice.batch)
    log(f"[tune] stencil variant {choice.stencil}: " +
        ", ".join(f"{k}: {v * 1e3:.2f} ms" for k, v in stimes.items()))
    choice.table = table
    return choice, fld, d
