"""pmCIMb with the saturation remedy.

Beyn's extraction on a disk recovers at most L eigenvalues: with L probe columns the
moment matrix C0 has rank <= L, and when a disk holds more eigenvalues the rank test
returns p = L and the eigenvalues of D are not those of T (the end of Section 3.2;
the paper's remedy is smaller cells or a larger l).  This driver applies the first:

  level 0   the plan's cover: indicators and moments in one sweep, Beyn on the
            flagged disks;
  level k   every cell whose disk came back saturated (p = L) is split 2 x 2 and its
            four children are swept (one plan over all of them, the coefficients
            shared on the device), their flagged disks extracted;

until no flagged disk is saturated or `max_depth` levels have run (extractions after
level 0 use N_beyn = 64 nodes, see pmcimb_adaptive).  The candidates of
the unsaturated disks of every level are filtered by ownership across all of them
(Step 2.f's rule, extended over cells of different parents: a value within
1e-6 max(1, |lambda|) of cells' shared edges belongs to the cell with the smallest
(x0, y0); nep_own), verified (sigma_min(T(lambda)) < tol_ver) and merged (nep_dedup).
Every sweep, extraction and verification runs in the library's kernels, the ownership
and merge rules in its host routines; only the cell bookkeeping is Python.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import nep as N


@dataclass(frozen=True)
class Cell:
    x0: float
    x1: float
    y0: float
    y1: float
    level: int


@dataclass
class AdaptiveResult:
    eigs: np.ndarray                 # verified, merged, sorted by (Re, Im)
    sigma: np.ndarray                # sigma_min of each returned eigenvalue
    levels: int                      # levels run (0 = the initial cover only)
    disks_swept: List[int]           # per level
    saturated: List[int]             # saturated flagged disks per level
    unresolved: int                  # cells still saturated after max_depth
    node_solves: int
    seconds: float
    per_level_candidates: List[int] = field(default_factory=list)


def _key(c):
    return (c.x0, c.x1, c.y0, c.y1)


def _cells_of(region, level):
    hx = (region.x1 - region.x0) / region.nx
    hy = (region.y1 - region.y0) / region.ny
    out = []
    for ix in range(region.nx):          # disk order of the library: ix * ny + iy
        for iy in range(region.ny):
            x0 = region.x0 + ix * hx
            y0 = region.y0 + iy * hy
            out.append(Cell(x0, x0 + hx, y0, y0 + hy, level))
    return out


def _extract(plan, flags, L):
    """Beyn on the flagged disks: (candidates [(disk, lambda)], saturated disk ids)."""
    flagged = np.nonzero(flags)[0]
    cand, sat = [], []
    if len(flagged) == 0:
        return cand, sat
    eig, p, sv, keep, _, _ = N.nep_beyn(plan, flagged)
    for i, d in enumerate(flagged):
        if int(p[i]) >= L:
            sat.append(int(d))
            continue
        for k in range(int(p[i])):
            if keep[i, k]:
                cand.append((int(d), eig[i, k]))
    return cand, sat


def pmcimb_adaptive(problem, region, opts, F, V, max_depth: int = 5, N_beyn: int = 64,
                    refine_iters: int = 2, log=None) -> AdaptiveResult:
    """problem: gen.Problem; region: gen.Region (the initial cover); opts: gen.Options
    with L > 0; F (n x s), V (n x L) host or device probe blocks.

    Level 0 screens the cover with opts.N nodes (indicators and moments of one sweep).
    Every extraction after that sweeps its cells with N_beyn nodes (the paper's split:
    a cheap indicator rule, a finer rule for Beyn): the flagged, unsaturated cells of
    level 0 again as they are, the saturated ones split 2 x 2.  On a circumscribed
    circle an eigenvalue on a cell edge sits at 0.71 r from the centre, where 32 nodes
    leave a quadrature error of ~1e-5 r and 64 nodes ~1e-10 r.  Eigenvalues of
    neighbouring cells just outside the circle still perturb the moments, so every
    candidate is moved onto its eigenvalue (nep_refine, refine_iters Rayleigh-functional
    updates) before ownership is decided and sigma_min is checked."""
    import copy
    import gen
    import torch
    if opts.L < 1:
        raise ValueError("the saturation remedy needs Beyn columns (L > 0)")
    t0 = time.perf_counter()
    devp = N.upload_problem(problem)
    Fd = N._dev_complex(F, torch)
    Vd = N._dev_complex(V, torch)
    L = opts.L
    ob = copy.copy(opts)
    ob.N = max(opts.N, N_beyn)
    cands = []
    disks_swept, saturated, per_level = [], [], []
    solves = 0

    # level 0: the given cover; this plan also serves the verification
    plan0 = N.nep_plan([devp], [region], opts)
    try:
        _, flags, _, _ = N.nep_indicator(plan0, [Fd], [Vd])
        solves += plan0.total_disks * opts.N
        disks_swept.append(plan0.total_disks)
        cells = _cells_of(region, 0)
        cand, sat = _extract(plan0, flags, L)
        saturated.append(len(sat))
        if ob.N == opts.N:
            cands += [(_key(cells[d]), lam) for d, lam in cand]
            redo = []
        else:
            # every flagged, unsaturated cell (also one whose candidates all fell outside it)
            redo = sorted({_key(cells[d]): cells[d] for d in np.nonzero(flags)[0] if d not in sat}.values(),
                          key=_key)
        per_level.append(len(cand) if ob.N == opts.N else 0)
        pending = [(cells[d], 2) for d in sat] + [(c, 1) for c in redo]
        level = 0
        while pending and level < max_depth:
            level += 1
            regs = [gen.Region(c.x0, c.x1, c.y0, c.y1, k, k) for c, k in pending]
            plan = N.nep_plan([devp] * len(regs), regs, ob)
            try:
                _, flags, _, _ = N.nep_indicator(plan, [Fd] * len(regs), [Vd] * len(regs))
                solves += plan.total_disks * ob.N
                disks_swept.append(plan.total_disks)
                children = [ch for r in regs for ch in _cells_of(r, level)]
                cand, sat = _extract(plan, flags, L)
            finally:
                N.nep_destroy(plan)
            cands += [(_key(children[d]), lam) for d, lam in cand]
            per_level.append(len(cand))
            saturated.append(len(sat))
            pending = [(children[d], 2) for d in sat]
            if log:
                log(f"level {level}: {len(regs)} cells swept with {ob.N} nodes, {int(flags.sum())} flagged, "
                    f"{len(cand)} candidates, {len(sat)} saturated")
        # refinement onto the eigenvalues, ownership across cells, verification, merge
        if cands:
            lam = np.asarray([l for _, l in cands], dtype=np.complex128)
            lam, sig, acc, _ = N.nep_refine(plan0, np.zeros(len(lam), np.int32), lam, refine_iters)
            cands = [(c, l) for (c, _), l in zip(cands, lam)]
            sel = N.nep_own(np.asarray([c for c, _ in cands], dtype=np.float64), lam) & acc
            al, asg = lam[sel], sig[sel]
            keep = N.nep_dedup(al, asg) if len(al) else np.zeros(0, bool)
            eigs, sg = al[keep], asg[keep]
        else:
            eigs, sg = np.zeros(0, np.complex128), np.zeros(0)
    finally:
        N.nep_destroy(plan0)
    torch.cuda.synchronize()
    order = np.lexsort((eigs.imag, eigs.real))
    return AdaptiveResult(eigs[order], sg[order], len(disks_swept) - 1, disks_swept, saturated, len(pending),
                          solves, time.perf_counter() - t0, per_level)
