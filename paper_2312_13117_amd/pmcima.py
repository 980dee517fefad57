"""pmCIMa (Section 3.1) on the library's kernels.

Step 1   the cover's disks are screened with the ratio indicator (eq (3.1); N = 16
         nodes and tol_ind = 0.1 by default); every flagged cell is split into its four
         quadrants and the quadrants are screened at the next level, for
         ceil(log2(r / tol_eps)) + 2 levels (Step 1.a and the appendix routine's two
         extra levels: the last cells have radius at most tol_eps / 2).  Each level is
         one plan over all its cells (every flagged cell a 2 x 2 region), so a level's
         node systems run as one batched sweep.  The centres of the cells flagged at
         the last level, merged where closer than tol_eps, approximate the eigenvalues.
Step 2   for every merged value, the right singular vector of sigma_min(T(lambda)) on
         the device (nep_refine): the eigenvector in place of the paper's shifted
         sparse eigensolver.  With refine_iters > 0 the values are also moved onto the
         eigenvalues by the two-sided Rayleigh functional and duplicates merged
         (not part of the paper's method; reported separately).

Only the cell bookkeeping is Python; the merge is the library's host routine
(nep_merge), and every node system, sum and indicator, and Step 2, run in the
library's kernels.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from . import nep as N

Cell = Tuple[float, float, float, float]          # x0, x1, y0, y1


def level_count(r: float, tol_eps: float) -> int:
    """Levels of Step 1: ceil(log2(r / tol_eps)) + 2."""
    return int(math.ceil(math.log2(r / tol_eps))) + 2


def region_cells(x0: float, x1: float, y0: float, y1: float, nx: int, ny: int):
    """(cell, centre, radius) of the disks the library builds for a region, in its disk
    order (ix * ny + iy), with the library's arithmetic for centres and half-widths."""
    hx = (x1 - x0) / nx / 2.0
    hy = (y1 - y0) / ny / 2.0
    r = math.hypot(hx, hy)
    out = []
    for ix in range(nx):
        for iy in range(ny):
            cx = x0 + (2 * ix + 1) * hx
            cy = y0 + (2 * iy + 1) * hy
            out.append(((cx - hx, cx + hx, cy - hy, cy + hy), complex(cx, cy), r))
    return out


@dataclass
class PmcimaResult:
    levels: int
    disks: List[List[Tuple[Cell, complex, float]]]   # per level: the disks swept
    ind: List[np.ndarray]                            # per level: indicator per disk
    flags: List[np.ndarray]                          # per level: flag per disk
    centres: np.ndarray                              # flagged at the last level
    eigs: np.ndarray                                 # merged centres (Step 1.c)
    sigma: Optional[np.ndarray] = None               # sigma_min(T) at each value of eigs
    vectors: Optional[np.ndarray] = None             # Step 2, m x n
    refined: Optional[np.ndarray] = None             # refine_iters > 0: refined, merged
    refined_sigma: Optional[np.ndarray] = None
    node_solves: int = 0
    seconds: float = 0.0
    level_seconds: List[float] = field(default_factory=list)


def pmcima(problem, region, F, N_nodes: int = 16, tol_ind: float = 0.1, tol_eps: float = 1e-6,
           precision: int = 0, vectors: bool = True, refine_iters: int = 0, log=None) -> PmcimaResult:
    """problem: gen.Problem; region: gen.Region (the initial cover); F: n x s probes."""
    import gen
    import torch
    t0 = time.perf_counter()
    devp = N.upload_problem(problem)
    Fd = N._dev_complex(F, torch)
    s = int(Fd.shape[1])
    opts = gen.Options(N=N_nodes, s=s, L=0, tol_ind=tol_ind, precision=precision)
    disks = region_cells(region.x0, region.x1, region.y0, region.y1, region.nx, region.ny)
    L = level_count(disks[0][2], tol_eps)
    all_disks, all_ind, all_flags, lsec = [], [], [], []
    solves = 0
    flagged = []
    plan0 = N.nep_plan([devp], [region], opts)
    try:
        regs = [region]
        for level in range(1, L + 1):
            tl = time.perf_counter()
            plan = plan0 if level == 1 else N.nep_plan([devp] * len(regs), regs, opts)
            try:
                ind, flags, _, _ = N.nep_indicator(plan, [Fd] * len(regs))
            finally:
                if plan is not plan0:
                    N.nep_destroy(plan)
            assert len(flags) == len(disks)
            solves += len(disks) * N_nodes
            ind = ind.max(axis=1)
            all_disks.append(disks)
            all_ind.append(ind)
            all_flags.append(flags)
            flagged = [disks[i] for i in np.nonzero(flags)[0]]
            lsec.append(time.perf_counter() - tl)
            if log:
                log(f"level {level}: {len(disks)} disks, {len(flagged)} flagged, {lsec[-1] * 1e3:.1f} ms")
            if not flagged:
                break
            if level < L:
                regs = [gen.Region(c[0], c[1], c[2], c[3], 2, 2) for c, _, _ in flagged]
                disks = [d for c, _, _ in flagged for d in region_cells(c[0], c[1], c[2], c[3], 2, 2)]
        centres = np.asarray([c for _, c, _ in flagged], dtype=np.complex128)
        eigs, _ = N.nep_merge(centres, tol_eps)
        res = PmcimaResult(len(all_disks), all_disks, all_ind, all_flags, centres, eigs)
        if len(eigs) and (vectors or refine_iters > 0):
            pid = np.zeros(len(eigs), np.int32)
            _, sig, _, vec = N.nep_refine(plan0, pid, eigs, 0, want_vectors=vectors)
            res.sigma, res.vectors = sig, vec
            if refine_iters > 0:
                lam, sg, acc, _ = N.nep_refine(plan0, pid, eigs, refine_iters)
                keep = N.nep_dedup(lam, sg)
                res.refined, res.refined_sigma = lam[keep & acc], sg[keep & acc]
    finally:
        N.nep_destroy(plan0)
    torch.cuda.synchronize()
    res.node_solves = solves
    res.level_seconds = lsec
    res.seconds = time.perf_counter() - t0
    return res
