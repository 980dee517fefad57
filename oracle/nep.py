"""Plain FP64 reference of the pmCIMb path (Section 3.2 of the paper).

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the benchmark's
CPU-baseline leg.  Numbers are complex128 throughout.

Readings of silent or garbled passages are listed with each function; the same
list is kept in the design notes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.linalg as sla

from gen import (PHI_ONE, PHI_Z, PHI_Z2, PHI_NEG_Z, PHI_EXP_NEG_TAU_Z, Problem,
                 Region, Options, ElementwiseDelay, CircleDoubleLayer)

# ---------------------------------------------------------------- T(z)


def phi(kind: int, param: float, z: complex) -> complex:
    """Scalar function multiplying coefficient A_k in the split form of T(z)."""
    if kind == PHI_ONE:
        return 1.0 + 0j
    if kind == PHI_Z:
        return complex(z)
    if kind == PHI_Z2:
        return complex(z) * complex(z)
    if kind == PHI_NEG_Z:
        return -complex(z)
    if kind == PHI_EXP_NEG_TAU_Z:
        return complex(np.exp(-param * complex(z)))
    raise ValueError(f"unknown phi kind {kind}")


def dphi(kind: int, param: float, z: complex) -> complex:
    """d phi / dz (used only by the argument-principle count)."""
    if kind == PHI_ONE:
        return 0j
    if kind == PHI_Z:
        return 1.0 + 0j
    if kind == PHI_Z2:
        return 2.0 * complex(z)
    if kind == PHI_NEG_Z:
        return -1.0 + 0j
    if kind == PHI_EXP_NEG_TAU_Z:
        return complex(-param * np.exp(-param * complex(z)))
    raise ValueError(f"unknown phi kind {kind}")


def circle_double_layer(n: int, k: complex) -> np.ndarray:
    """T(k) = (I + K_n(k)) / 2 on n equispaced points t_j = 2 pi j / n of the unit
    circle.  The kernel of K is 2 dPhi(x(t), y(s))/dnu(y) = -(i k r / 4) H1(k r),
    r = |x - y| = 2 |sin((t - s)/2)|; it is split as L1 ln(4 sin^2((t - s)/2)) + L2
    with L1 = (k r / (4 pi)) J1(k r) and L2 the rest (L2 = -1/(2 pi) on the diagonal),
    and integrated by Kress's rule: the logarithmic part with the weights
    R_j(t) = -(2 pi / m) sum_{l=1}^{m-1} cos(l (t - t_j)) / l - (pi / m^2) cos(m (t - t_j))
    (m = n / 2), the smooth part by the trapezoid rule (pi / m) sum_j."""
    import scipy.special as ssp
    m = n // 2
    t = 2.0 * np.pi * np.arange(n) / n
    d = t[:, None] - t[None, :]
    l = np.arange(1, m)
    R = -(2.0 * np.pi / m) * (np.cos(d[..., None] * l) / l).sum(axis=-1) - (np.pi / m ** 2) * np.cos(m * d)
    r = 2.0 * np.abs(np.sin(d / 2.0))
    off = ~np.eye(n, dtype=bool)
    z = complex(k) * r
    K = np.zeros((n, n), dtype=np.complex128)
    K[off] = -(1j * z[off] / 4.0) * ssp.hankel1(1, z[off])
    L1 = np.zeros((n, n), dtype=np.complex128)
    L1[off] = (z[off] / (4.0 * np.pi)) * ssp.jv(1, z[off])
    L2 = np.full((n, n), -1.0 / (2.0 * np.pi), dtype=np.complex128)
    L2[off] = K[off] - L1[off] * np.log(4.0 * np.sin(d[off] / 2.0) ** 2)
    Kn = R * L1 + (np.pi / m) * L2
    return 0.5 * (np.eye(n) + Kn)


def assemble(prob: Problem, z: complex) -> np.ndarray:
    """T(z) = sum_k phi_k(z) A_k: the matrix function of eq (1.1), in the split form of
    the appendix routine that generates T(z); an ElementwiseDelay problem is written out
    entry by entry, -z I + A0 + A1 .* exp(-tau .* z)."""
    if isinstance(prob, ElementwiseDelay):
        T = prob.A0 + prob.A1 * np.exp(-prob.tau * complex(z))
        T[np.diag_indices(prob.n)] -= complex(z)
        return T
    if isinstance(prob, CircleDoubleLayer):
        return circle_double_layer(prob.n, z)
    T = np.zeros((prob.n, prob.n), dtype=np.complex128)
    for A, kind, par in zip(prob.coeffs, prob.phi_kind, prob.phi_param):
        f = phi(kind, par, z)
        if A is None:
            T[np.diag_indices(prob.n)] += f
        else:
            T += f * A
    return T


def assemble_derivative(prob: Problem, z: complex) -> np.ndarray:
    if isinstance(prob, ElementwiseDelay):
        T = -prob.tau * prob.A1 * np.exp(-prob.tau * complex(z))
        T[np.diag_indices(prob.n)] -= 1.0
        return T
    T = np.zeros((prob.n, prob.n), dtype=np.complex128)
    for A, kind, par in zip(prob.coeffs, prob.phi_kind, prob.phi_param):
        f = dphi(kind, par, z)
        if A is None:
            T[np.diag_indices(prob.n)] += f
        else:
            T += f * A
    return T


# ---------------------------------------------------------------- cover and nodes


@dataclass
class Disk:
    ix: int
    iy: int
    cx: float
    cy: float
    hx: float
    hy: float

    @property
    def r(self) -> float:
        # circumscribed circle of the cell (Section 3: squares replaced by the disks
        # circumscribing them)
        return math.hypot(self.hx, self.hy)

    @property
    def c(self) -> complex:
        return complex(self.cx, self.cy)


def cover(reg: Region) -> List[Disk]:
    """Split the rectangle into nx x ny equal cells, listed x-major (disk index
    ix*ny + iy), as the driver of the appendix builds its centre list."""
    hx = (reg.x1 - reg.x0) / reg.nx / 2.0
    hy = (reg.y1 - reg.y0) / reg.ny / 2.0
    out = []
    for ix in range(reg.nx):
        for iy in range(reg.ny):
            out.append(Disk(ix, iy, reg.x0 + (2 * ix + 1) * hx, reg.y0 + (2 * iy + 1) * hy, hx, hy))
    return out


def nodes_weights(c: complex, r: float, N: int) -> Tuple[np.ndarray, np.ndarray]:
    """Trapezoidal rule for (1/2 pi i) \\oint g(z) dz on |z - c| = r, eq (2.3):
    theta_j = 2 pi (j-1)/N for j = 1..N, z_j = c + r e^{i theta_j}, and
    w_j = (1/2 pi i) * (2 pi / N) * i r e^{i theta_j} = (r/N) e^{i theta_j}."""
    theta = 2.0 * np.pi * np.arange(N) / N
    e = np.exp(1j * theta)
    return c + r * e, (r / N) * e


# ---------------------------------------------------------------- sweep (Step 1, Step 2.b)


@dataclass
class DiskSweep:
    PfN: np.ndarray          # n x s : N-point rule of P f, eq (2.3)
    PfN2: np.ndarray         # n x s : N/2-point rule on the 1-based even nodes
    C0: Optional[np.ndarray]  # n x L : eq (3.2)
    C1: Optional[np.ndarray]  # n x L : eq (3.3)
    profile: np.ndarray      # N x s : ||x_j|| per node and probe column
    scale: np.ndarray        # s : sum_j |w_j| ||x_j[:, q]||, the size of the summands of P f|_N
    scale_half: np.ndarray   # s : sum_{j even} 2 |w_j| ||x_j[:, q]||, the same for P f|_{N/2}

    @property
    def scales(self) -> Tuple[np.ndarray, np.ndarray]:
        return self.scale, self.scale_half

    def indicator(self) -> Tuple[float, np.ndarray]:
        """eq (3.1) of this disk, with the rounding-noise floor (see ``indicator``)."""
        return indicator(self.PfN, self.PfN2, self.scales)


def sweep_disk(prob: Problem, c: complex, r: float, N: int, F: np.ndarray,
               V: Optional[np.ndarray]) -> DiskSweep:
    """Solve T(z_j) X_j = [F | V] at every node (eq (2.4)) and form the weighted sums.

    * P f|_N    = sum_{j=1..N} w_j x_j                        (eq (2.3))
    * P f|_{N/2} = sum_{j even, 1-based} 2 w_j x_j             (the half rule of Section 3.1)
    * C_{0,N}  = sum_j w_j X^V_j,  C_{1,N} = sum_j w_j z_j X^V_j  (eqs (3.2)-(3.3); the
      garbled factor "(z + r theta_j)" of eq (3.3) is read as the node z_j, and the
      normalisation is the exact trapezoid (r/N) e^{i theta_j} of (1/2 pi i) \\oint).
    """
    n = prob.n
    z, w = nodes_weights(c, r, N)
    s = F.shape[1]
    B = F if V is None else np.concatenate([F, V], axis=1)
    PfN = np.zeros((n, s), dtype=np.complex128)
    PfN2 = np.zeros((n, s), dtype=np.complex128)
    C0 = None if V is None else np.zeros((n, V.shape[1]), dtype=np.complex128)
    C1 = None if V is None else np.zeros((n, V.shape[1]), dtype=np.complex128)
    profile = np.zeros((N, s))
    for j in range(N):          # j is 0-based here; node j+1 in the paper's numbering
        X = sla.solve(assemble(prob, z[j]), B)   # LU with partial pivoting (LAPACK gesv)
        x = X[:, :s]
        PfN += w[j] * x
        if (j + 1) % 2 == 0:
            PfN2 += 2.0 * w[j] * x
        if V is not None:
            XV = X[:, s:]
            C0 += w[j] * XV
            C1 += (w[j] * z[j]) * XV
        profile[j] = [norm2(x[:, q]) for q in range(s)]
    scale = (np.abs(w)[:, None] * profile).sum(axis=0)
    scale_half = (2.0 * np.abs(w[1::2])[:, None] * profile[1::2]).sum(axis=0)
    return DiskSweep(PfN, PfN2, C0, C1, profile, scale, scale_half)


def norm2(v: np.ndarray) -> float:
    """Euclidean norm of a vector, scaled by its largest modulus so that entries far
    outside 1e+-154 neither overflow nor underflow when squared."""
    a = np.abs(np.asarray(v).ravel())
    m = float(a.max()) if a.size else 0.0
    if m == 0.0 or not math.isfinite(m):
        return m
    return m * math.sqrt(float(np.sum((a / m) ** 2)))


# Rounding-noise floor of a quadrature sum relative to the size of its summands.
# A sum of N node solutions, each with a normwise relative error eps, lies within
# (eps + gamma_N) * S of the exact sum, S = sum_j |weight_j| ||x_j||.  A backward-stable
# LU gives eps <= c n u kappa; with n <= 2^12, u = 2^-53 and kappa <= 2^10 (the floor
# can only matter on disks far from every eigenvalue, where the node matrices are well
# conditioned) n u kappa <= 2^-31, and the floor is twice that.
NOISE_FLOOR = 2.0 ** -30


def indicator(PfN: np.ndarray, PfN2: np.ndarray, scales=None,
              floor: float = NOISE_FLOOR) -> Tuple[float, np.ndarray]:
    """Ratio indicator of eq (3.1), read as in the appendix's indicator routine: the
    elementwise ratio P f|_N ./ P f|_{N/2}, its 2-norm, divided by sqrt(n).  With s > 1
    probe columns the disk's indicator is the maximum over columns.  A non-finite
    column (0/0 or x/0) gives +inf, which flags the disk.

    Reading (floating point): far from every eigenvalue both quadrature errors fall
    below the rounding level of their summands and their ratio is noise of order one,
    where the paper states I ~ e^{-CN/2}.  ``scales`` = (S_N, S_half) per column, the
    summand sizes of the two rules (sum_j |w_j| ||x_j||, and over the 1-based even
    nodes with weights 2|w_j|).  A column whose sums are both at most ``floor`` times
    their own summand size, all four numbers finite, has I_q = 0.  A node next to an
    eigenvalue outside the circle dominates its rule's summands and that rule's sum
    alike, so it never brings a column under the floor."""
    n = PfN.shape[0]
    s = PfN.shape[1]
    Iq = np.empty(s)
    for q in range(s):
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            ratio = PfN[:, q] / PfN2[:, q]      # complex division, scaled by numpy
        v = norm2(ratio) / math.sqrt(n) if np.all(np.isfinite(ratio)) else math.inf
        Iq[q] = v if math.isfinite(v) else math.inf
        if scales is not None:
            SN, SH = float(scales[0][q]), float(scales[1][q])
            a, b = norm2(PfN[:, q]), norm2(PfN2[:, q])
            if all(math.isfinite(t) for t in (a, b, SN, SH)) and a <= floor * SN and b <= floor * SH:
                Iq[q] = 0.0
    return float(np.max(Iq)), Iq


# ---------------------------------------------------------------- Beyn (Step 2.c-2.e)


@dataclass
class BeynResult:
    sv: np.ndarray           # singular values of C0 (length L, descending)
    p: int                   # rank kept: #{sigma > tol_svd}
    lam: np.ndarray          # eigenvalues of D (length p)
    vec: np.ndarray          # n x p eigenvectors V_0 s_i, unit 2-norm
    D: np.ndarray            # p x p


def beyn(C0: np.ndarray, C1: np.ndarray, tol_svd: float) -> BeynResult:
    """Beyn's extraction (eq (2.8) with the truncation of Step 2.d):
    C0 = U S W^H (economy SVD), p = #{sigma_i > tol_svd},
    D = U_0^H C1 W_0 S_0^{-1}, eig(D) -> lambda_i, s_i, eigenvectors U_0 s_i."""
    U, sv, Wh = np.linalg.svd(C0, full_matrices=False)
    p = int(np.sum(sv > tol_svd))
    if p == 0:
        return BeynResult(sv, 0, np.zeros(0, np.complex128),
                          np.zeros((C0.shape[0], 0), np.complex128), np.zeros((0, 0), np.complex128))
    U0 = U[:, :p]
    W0 = Wh[:p, :].conj().T
    D = U0.conj().T @ C1 @ W0 @ np.diag(1.0 / sv[:p])
    lam, S = np.linalg.eig(D)
    vec = U0 @ S
    vec = vec / np.linalg.norm(vec, axis=0, keepdims=True)
    return BeynResult(sv, p, lam, vec, D)


# ---------------------------------------------------------------- Step 2.f ownership


def owner_cell(lam: complex, reg: Region, rel_band: float = 1e-6) -> Optional[Tuple[int, int]]:
    """Cell that keeps an eigenvalue (Step 2.f: drop values outside the square).

    The strict test |Re l - cx| < hx, |Im l - cy| < hy leaves a value that lies on an
    edge shared by two cells to neither of them, and a value computed from each side
    of the edge to both.  Reading: a value within rel_band*max(1,|l|) of a cell edge
    belongs to the neighbour with the smaller index on that axis; values outside the
    closed region (beyond the band) belong to no cell.  The band (1e-6) exceeds the
    quadrature error that edge eigenvalues carry with N = 32 nodes on circumscribed
    circles (up to ~2e-7 relative on the small workload)."""
    band = rel_band * max(1.0, abs(lam))

    def axis(v, lo, hi, cells):
        if v < lo - band or v > hi + band:
            return None
        h = (hi - lo) / cells
        t = (v - lo) / h
        k = int(round(t))
        if abs(v - (lo + k * h)) <= band:      # on (or within the band of) grid line k
            return min(max(k - 1, 0), cells - 1)
        return min(max(int(math.floor(t)), 0), cells - 1)

    ix = axis(lam.real, reg.x0, reg.x1, reg.nx)
    iy = axis(lam.imag, reg.y0, reg.y1, reg.ny)
    if ix is None or iy is None:
        return None
    return ix, iy


# ---------------------------------------------------------------- Step 3 verification


def sigma_min(prob: Problem, lam: complex) -> float:
    """Smallest singular value of T(lambda) from a full SVD."""
    return float(np.linalg.svd(assemble(prob, lam), compute_uv=False)[-1])


def min_abs_eig(prob: Problem, lam: complex) -> float:
    """The paper's Step 3 statistic: the eigenvalue of T(lambda) of smallest modulus."""
    return float(np.min(np.abs(np.linalg.eigvals(assemble(prob, lam)))))


def dedup(lams: Sequence[complex], sig: Sequence[float], rel: float = 1e-8) -> List[int]:
    """Indices to keep after merging values closer than rel*max(1,|l|); of a close pair
    the one with the smaller sigma_min is kept."""
    order = sorted(range(len(lams)), key=lambda i: (sig[i], i))
    kept: List[int] = []
    for i in order:
        if all(abs(lams[i] - lams[k]) > rel * max(1.0, abs(lams[i])) for k in kept):
            kept.append(i)
    return sorted(kept, key=lambda i: (lams[i].real, lams[i].imag))


# ---------------------------------------------------------------- the whole path


@dataclass
class PmcimbResult:
    disks: List[Disk]
    ind: np.ndarray                  # per disk
    ind_cols: np.ndarray             # per disk x s
    flags: np.ndarray                # per disk, bool
    sweeps: List[DiskSweep]
    beyn: dict                       # disk index -> BeynResult (flagged disks)
    cand: List[Tuple[int, complex]]  # (disk, lambda) kept by Step 2.f
    sigma: np.ndarray                # sigma_min per candidate
    accepted: np.ndarray             # bool per candidate
    eigs: np.ndarray                 # verified, deduplicated, sorted by (Re, Im)


def pmcimb(prob: Problem, reg: Region, opts: Options, F: np.ndarray,
           V: Optional[np.ndarray], disk_subset: Optional[Sequence[int]] = None) -> PmcimbResult:
    """pmCIMb, Section 3.2: Step 1 (indicators, flag I > tol_ind), Step 2 (Beyn on the
    flagged disks with the moments of the same sweep, since both use the same nodes),
    Step 2.f (ownership filter), Step 3 (sigma_min(T(lambda)) < tol_ver), then
    de-duplication.  ``disk_subset`` restricts the sweep to some disks (sampling)."""
    disks = cover(reg)
    idx = list(range(len(disks))) if disk_subset is None else list(disk_subset)
    sweeps, ind, ind_cols = [], [], []
    for d in idx:
        dk = disks[d]
        sw = sweep_disk(prob, dk.c, dk.r, opts.N, F, V)
        I, Iq = sw.indicator()
        sweeps.append(sw)
        ind.append(I)
        ind_cols.append(Iq)
    ind = np.array(ind)
    flags = ind > opts.tol_ind
    by = {}
    cand = []
    if V is not None:
        for k, d in enumerate(idx):
            if not flags[k]:
                continue
            br = beyn(sweeps[k].C0, sweeps[k].C1, opts.tol_svd)
            by[d] = br
            for lam in br.lam:
                if owner_cell(lam, reg) == (disks[d].ix, disks[d].iy):
                    cand.append((d, complex(lam)))
    sig = np.array([sigma_min(prob, l) for _, l in cand])
    acc = sig < opts.tol_ver
    acc_l = [l for (d, l), a in zip(cand, acc) if a]
    acc_s = [s for s, a in zip(sig, acc) if a]
    keep = dedup(acc_l, acc_s)
    eigs = np.array([acc_l[i] for i in keep], dtype=np.complex128)
    return PmcimbResult([disks[d] for d in idx], ind, np.array(ind_cols), flags, sweeps, by,
                        cand, sig, acc, eigs)
