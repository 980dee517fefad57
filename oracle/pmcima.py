"""pmCIMa (Section 3.1) in plain complex128 numpy (TEST INFRASTRUCTURE ONLY).

Step 1 screens the disks of a cover with the ratio indicator (eq (3.1), N = 16 nodes,
tol_ind = 0.1) and splits every flagged cell into its four quadrants, level after
level, until the cells are smaller than the requested precision tol_eps; the centres
of the cells flagged at the last level approximate the eigenvalues, and centres closer
than tol_eps are merged (the remark after the algorithm).  Step 2 computes, for each
merged value, the vector belonging to the smallest singular value of T(lambda).

Readings (listed with the design notes as well):
* Levels.  Step 1.a gives ceil(log2(r / tol_eps)); the appendix routine runs two more.
  The two extra levels are kept: with them the last cells have radius at most
  tol_eps / 2.
* Children.  A flagged cell [x0, x1] x [y0, y1] is split by the same cover as any
  region (2 x 2 equal cells, listed x-major), so the child disks are the disks of
  Region(x0, x1, y0, y1, 2, 2).
* A level that flags nothing ends the search with no eigenvalue.
* Merge.  Star clusters in list order: the first centre not yet merged takes every
  other unmerged centre closer than tol_eps (absolute, as in the appendix routine),
  and the cluster's mean (each centre counted once) is one eigenvalue.
* Step 2.  The paper takes the eigenvector of the eigenvalue of T(lambda) nearest 0
  (a shifted sparse eigensolver); here it is the right singular vector of
  sigma_min(T(lambda)), which is the null vector of T at an exact eigenvalue, with
  unit 2-norm and its largest-modulus entry real and positive.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

from gen import Problem, Region
from .nep import assemble, cover, sweep_disk

Cell = Tuple[float, float, float, float]          # x0, x1, y0, y1


def level_count(r: float, tol_eps: float) -> int:
    """Step 1.a with the appendix's two extra levels."""
    return int(math.ceil(math.log2(r / tol_eps))) + 2


def disks_of(region: Region):
    """(cell, centre, radius) of every disk of a region's cover, in cover order."""
    out = []
    for d in cover(region):
        out.append(((d.cx - d.hx, d.cx + d.hx, d.cy - d.hy, d.cy + d.hy), d.c, d.r))
    return out


def children(cell: Cell):
    """The four quadrant disks of a flagged cell (the cover of its 2 x 2 split)."""
    return disks_of(Region(cell[0], cell[1], cell[2], cell[3], 2, 2))


def merge(centres: Sequence[complex], tol_eps: float) -> np.ndarray:
    """Star clusters in list order, each centre counted once; cluster means, the real
    and imaginary parts each summed in list order and divided by the member count."""
    z = [complex(v) for v in centres]
    used = [False] * len(z)
    out = []
    for i in range(len(z)):
        if used[i]:
            continue
        members = [j for j in range(len(z)) if not used[j] and abs(z[j] - z[i]) < tol_eps]
        for j in members:
            used[j] = True
        re = sum(z[j].real for j in members)
        im = sum(z[j].imag for j in members)
        out.append(complex(re / len(members), im / len(members)))
    return np.asarray(out, dtype=np.complex128)


def null_vector(prob: Problem, lam: complex) -> Tuple[np.ndarray, float]:
    """Right singular vector of sigma_min(T(lambda)) (full SVD) with the phase fixed so
    that its largest-modulus entry is real and positive; and sigma_min itself."""
    _, s, Vh = np.linalg.svd(assemble(prob, lam))
    v = Vh[-1].conj()
    k = int(np.argmax(np.abs(v)))
    v = v * (abs(v[k]) / v[k])
    return v / np.linalg.norm(v), float(s[-1])


@dataclass
class PmcimaResult:
    levels: int                                    # levels run
    disks: List[List[Tuple[Cell, complex, float]]]  # per level: the disks swept
    ind: List[np.ndarray]                          # per level: indicator per disk
    flags: List[np.ndarray]                        # per level: flag per disk
    centres: np.ndarray                            # centres flagged at the last level
    eigs: np.ndarray                               # merged
    vectors: np.ndarray = field(default=None)      # m x n (Step 2)
    sigma: np.ndarray = field(default=None)        # sigma_min at each merged value


def pmcima(prob: Problem, region: Region, F: np.ndarray, N: int = 16, tol_ind: float = 0.1,
           tol_eps: float = 1e-6, vectors: bool = True) -> PmcimaResult:
    """pmCIMa of Section 3.1 on the cover of `region` with probe block F (n x s)."""
    disks = disks_of(region)
    L = level_count(disks[0][2], tol_eps)
    all_disks, all_ind, all_flags = [], [], []
    flagged = []
    for level in range(1, L + 1):
        ind = np.zeros(len(disks))
        for i, (_, c, r) in enumerate(disks):
            sw = sweep_disk(prob, c, r, N, F, None)
            ind[i] = sw.indicator()[0]
        flags = ind > tol_ind
        all_disks.append(disks)
        all_ind.append(ind)
        all_flags.append(flags)
        flagged = [disks[i] for i in range(len(disks)) if flags[i]]
        if not flagged:
            break
        if level < L:
            disks = [ch for cell, _, _ in flagged for ch in children(cell)]
    centres = np.asarray([c for _, c, _ in flagged], dtype=np.complex128)
    eigs = merge(centres, tol_eps)
    res = PmcimaResult(len(all_disks), all_disks, all_ind, all_flags, centres, eigs)
    if vectors:
        vs = [null_vector(prob, lam) for lam in eigs]
        res.vectors = np.asarray([v for v, _ in vs]).reshape(len(eigs), prob.n)
        res.sigma = np.asarray([s for _, s in vs])
    return res


def sim_quadtree_labels(prob: Problem, root: Cell, depth: int, F: np.ndarray, N: int = 32,
                        tol_ind: float = 0.1) -> List[Tuple[int, Cell, np.ndarray]]:
    """The SIM recursion of Section 2.1 (Step 1.b of pmCIMa) over a quadtree below
    `root`: every flagged cell is split into its four quadrants (cover order of a 2 x 2
    split) and each quadrant's disk is screened with the indicator of eq (3.1), down to
    `depth` levels below the root.  The root itself is always split: for a matrix
    polynomial of degree >= 2 a circle around the whole spectrum gives P f = 0, so its
    indicator says nothing.  Returns one record per split cell, level by level and in
    cover order within a level: (level of the split cell, the cell, indicators of its
    four quadrants); a quadrant is flagged iff its indicator exceeds tol_ind."""
    out = []
    parents = [root]
    for level in range(depth):
        nxt = []
        for cell in parents:
            ch = children(cell)
            ind = np.array([sweep_disk(prob, c, r, N, F, None).indicator()[0] for _, c, r in ch])
            fl = ind > tol_ind
            out.append((level, cell, ind))
            if level + 1 < depth:
                nxt.extend(ch[k][0] for k in range(4) if fl[k])
        parents = nxt
    return out
