"""Seeded synthetic inputs for the contour-integral eigensolver workloads.

This module is shared by the CPU oracle and the GPU path.  It holds input
recipes only (seeded Gaussian matrices, probe blocks, region grids and the
split form of T(z)); none of the eigensolver's arithmetic lives here.

The split form of a problem is T(z) = sum_k phi_k(z) A_k (the structure of the
paper's test matrix function in the appendix routine that generates T(z): a
quadratic T0 + z T1 + z^2 T2).  A coefficient of ``None`` stands for the
identity matrix, which is never materialised.

phi kinds (names shared with the C header):
  ONE            phi(z) = 1
  Z              phi(z) = z
  Z2             phi(z) = z^2
  NEG_Z          phi(z) = -z
  EXP_NEG_TAU_Z  phi(z) = exp(-tau z), tau = param
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

PHI_ONE, PHI_Z, PHI_Z2, PHI_NEG_Z, PHI_EXP_NEG_TAU_Z = 0, 1, 2, 3, 4
PHI_NAMES = {PHI_ONE: "ONE", PHI_Z: "Z", PHI_Z2: "Z2", PHI_NEG_Z: "NEG_Z",
             PHI_EXP_NEG_TAU_Z: "EXP_NEG_TAU_Z"}


@dataclass
class Problem:
    """T(z) = sum_k phi_k(z) A_k with A_k complex128 n x n (row-major) or None (= I)."""
    n: int
    coeffs: List[Optional[np.ndarray]]
    phi_kind: List[int]
    phi_param: List[float] = field(default_factory=list)

    def __post_init__(self):
        if not self.phi_param:
            self.phi_param = [0.0] * len(self.coeffs)
        assert len(self.coeffs) == len(self.phi_kind) == len(self.phi_param)
        for A in self.coeffs:
            if A is not None:
                assert A.shape == (self.n, self.n) and A.dtype == np.complex128


@dataclass
class ElementwiseDelay:
    """T(z) = -z I + A0 + A1 .* exp(-tau .* z): every entry of A1 with a delay of its
    own (tau real n x n, >= 0).  With n^2 distinct delays T has no short split form, so
    the GPU path assembles it by a caller-supplied assembler (the generic T(z) of the
    paper's appendix routine that generates T) instead of the split coefficients."""
    n: int
    A0: np.ndarray
    A1: np.ndarray
    tau: np.ndarray

    def __post_init__(self):
        for X in (self.A0, self.A1):
            assert X.shape == (self.n, self.n) and X.dtype == np.complex128
        assert self.tau.shape == (self.n, self.n) and self.tau.dtype == np.float64


@dataclass
class CircleDoubleLayer:
    """Scattering poles of the sound-soft unit disk: T(k) = (I + K_n(k)) / 2 with K the
    double-layer operator (kernel 2 dPhi/dnu(y), Phi = (i/4) H0(k|x-y|)) on the unit
    circle, discretised by the Nystrom rule with the logarithmic splitting of Kress on
    n equispaced points (n even).  No split form: assembled by a device assembler."""
    n: int

    def __post_init__(self):
        assert self.n >= 4 and self.n % 2 == 0


@dataclass
class Region:
    """Rectangle [x0,x1] x [y0,y1] split into nx x ny equal cells."""
    x0: float
    x1: float
    y0: float
    y1: float
    nx: int
    ny: int


@dataclass
class Options:
    N: int = 32          # trapezoidal nodes per circle
    s: int = 1           # indicator probe columns
    L: int = 8           # Beyn probe columns
    tol_ind: float = 0.1
    tol_svd: float = 1e-6
    tol_ver: float = 1e-6
    precision: int = 0   # 0 = complex128 LU, 1 = complex64 LU + complex128 refinement
    max_refine: int = 3
    batch: int = 0       # node matrices per batch (0 = library default)
    streams: int = 0     # worker streams (0 = library default)
    pivot: int = 0       # 0 = partial pivoting, 1 = tournament pivoting
    graph: int = 0       # 1 = capture the indicator sweep in a HIP graph and replay it


@dataclass
class Workload:
    name: str
    problems: List[Problem]
    regions: List[Region]
    opts: Options
    F: List[np.ndarray]              # per problem n x s, unit-norm columns
    V: List[Optional[np.ndarray]]    # per problem n x L, unit-norm columns (or None)


def gaussian(seed: int, n: int, m: Optional[int] = None) -> np.ndarray:
    """Real N(0,1) draws from numpy's default_rng(seed), row-major fill, divided by sqrt(n)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n if m is None else m)) / np.sqrt(n)


def probes(seed: int, n: int, cols: int) -> np.ndarray:
    """Real N(0,1) probe block with unit 2-norm columns, stored complex128."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, cols))
    X /= np.linalg.norm(X, axis=0, keepdims=True)
    return np.ascontiguousarray(X.astype(np.complex128))


def qep(K: np.ndarray, C: np.ndarray, M: Optional[np.ndarray]) -> Problem:
    """T(z) = K + z C + z^2 M (M None = identity)."""
    n = K.shape[0]
    c = lambda X: None if X is None else np.ascontiguousarray(X.astype(np.complex128))
    return Problem(n, [c(K), c(C), c(M)], [PHI_ONE, PHI_Z, PHI_Z2])


def delay(A0: np.ndarray, A1: np.ndarray, tau: float) -> Problem:
    """T(z) = -z I + A0 + A1 exp(-tau z)."""
    n = A0.shape[0]
    c = lambda X: np.ascontiguousarray(X.astype(np.complex128))
    return Problem(n, [None, c(A0), c(A1)], [PHI_NEG_Z, PHI_ONE, PHI_EXP_NEG_TAU_Z],
                   [0.0, 0.0, float(tau)])


# ----------------------------------------------------------------- workloads
def qep_c1(n: int = 64) -> Problem:
    A = gaussian(0, n)
    B = gaussian(1, n)
    return qep(A + A.T, 0.1 * B, None)


def workload_small_qep(n: int = 64) -> Workload:
    """n=64 QEP, [-2,2]^2 split 4x4, N=32, s=1 probe, L=8 (the small configuration)."""
    prob = qep_c1(n)
    opts = Options(N=32, s=1, L=8)
    return Workload("qep_n64_4x4", [prob], [Region(-2, 2, -2, 2, 4, 4)], opts,
                    [probes(2, n, 1)], [probes(3, n, 8)])


def workload_dense_qep(n: int = 1024, precision: int = 0, nx: int = 16, ny: int = 16,
                       half_width: float = 4.0) -> Workload:
    """n=1024 QEP, M = I + 0.1 G G^T, [-4,4]^2 split 16x16, N=32, s=4, L=16."""
    A = gaussian(0, n)
    B = gaussian(1, n)
    G = gaussian(2, n)
    M = np.eye(n) + 0.1 * (G @ G.T)
    prob = qep(A + A.T, 0.1 * B, M)
    opts = Options(N=32, s=4, L=16, precision=precision)
    hw = half_width
    return Workload(f"qep_n{n}_{nx}x{ny}" + ("_mixed" if precision else ""), [prob],
                    [Region(-hw, hw, -hw, hw, nx, ny)], opts,
                    [probes(3, n, 4)], [probes(4, n, 16)])


def delay_family(count: int = 64, sizes: Sequence[int] = (128, 256, 512, 1024, 2048)):
    """Uneven batch of delay problems: n_p ~ U{sizes}, tau_p ~ U[0.5,2] from rng(40)."""
    rng = np.random.default_rng(40)
    ns = rng.choice(np.asarray(sizes), size=count)
    taus = rng.uniform(0.5, 2.0, size=count)
    out = []
    for p in range(count):
        n = int(ns[p])
        out.append(delay(gaussian(1000 + 2 * p, n), gaussian(1001 + 2 * p, n), float(taus[p])))
    return out


def workload_delay(count: int = 64, sizes: Sequence[int] = (128, 256, 512, 1024, 2048),
                   precision: int = 1) -> Workload:
    probs = delay_family(count, sizes)
    reg = Region(-3.0, 1.0, -6.0, 6.0, 8, 16)
    opts = Options(N=48, s=1, L=8, precision=precision)
    F = [probes(2000 + p, pr.n, 1) for p, pr in enumerate(probs)]
    return Workload("delay_uneven", probs, [reg] * len(probs), opts, F, [None] * len(probs))


def delay_sampled_rectangles(p: int, count: int = 8, cells: int = 128) -> List[int]:
    """The rectangles of delay problem p checked one by one when the problem is too
    large to check whole: `count` distinct cover indices from default_rng(4000 + p)."""
    rng = np.random.default_rng(4000 + p)
    return sorted(int(i) for i in rng.choice(cells, size=count, replace=False))


def elementwise_delay(n: int, seed: int, tau_lo: float = 0.5, tau_hi: float = 2.0) -> ElementwiseDelay:
    """A0 = G0, A1 = G1 (Gaussian / sqrt(n), seeds `seed`, `seed` + 1), tau_ij ~
    U[tau_lo, tau_hi] from rng(seed + 2)."""
    c = lambda X: np.ascontiguousarray(X.astype(np.complex128))
    tau = np.random.default_rng(seed + 2).uniform(tau_lo, tau_hi, size=(n, n))
    return ElementwiseDelay(n, c(gaussian(seed, n)), c(gaussian(seed + 1, n)), np.ascontiguousarray(tau))


def screener_problem(p: int, n: int = 256) -> Problem:
    """Member p of the parametrised QEP family: K = A + A^T + s_p I, C = c_p B, M = I."""
    rng = np.random.default_rng(5000 + p)
    A = rng.standard_normal((n, n)) / np.sqrt(n)
    B = rng.standard_normal((n, n)) / np.sqrt(n)
    s_p = rng.uniform(-2.0, 2.0)
    c_p = rng.uniform(0.01, 0.5)
    return qep(A + A.T + s_p * np.eye(n), c_p * B, None)


def rotated_diagonal(roots: Sequence[complex], seed: int, n: Optional[int] = None,
                     quadratic_partner: Optional[Sequence[complex]] = None) -> Problem:
    """Q diag(z - a_i) Q^H (linear) or Q diag((z-a_i)(z-b_i)) Q^H (quadratic) with a
    seeded random unitary Q: a problem whose eigenvalues are known exactly."""
    a = np.asarray(roots, dtype=np.complex128)
    n = len(a) if n is None else n
    assert len(a) == n
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    Q = Q * (np.diag(R) / np.abs(np.diag(R)))
    rot = lambda d: np.ascontiguousarray(Q @ np.diag(d) @ Q.conj().T)
    if quadratic_partner is None:
        return Problem(n, [rot(-a), None], [PHI_ONE, PHI_Z])
    b = np.asarray(quadratic_partner, dtype=np.complex128)
    return Problem(n, [rot(a * b), rot(-(a + b)), None], [PHI_ONE, PHI_Z, PHI_Z2])


def paper_demo_problem() -> Problem:
    """The 4x4 quadratic T0 + z T1 + z^2 T2 printed in the paper's appendix routine
    that generates T(z)."""
    T2 = np.diag([3.0, 1.0, 3.0, 1.0])
    T1 = np.array([[0.4, 0, -0.3, 0], [0, 0, 0, 0], [-0.3, 0, 0.5, -0.2], [0, 0, -0.2, 0.2]])
    T0 = np.array([[-7.0, 2, 4, 0], [2, -4, 2, 0], [4, 2, -9, 3], [0, 0, 3, -3]])
    return qep(T0, T1, T2)


# ---------------------------------------------------------------- screener MLP inputs
MLP_LAYERS = [(32, 128), (128, 128), (128, 4)]   # in x out per dense layer


def mlp_param_count() -> int:
    return sum(i * o + o for i, o in MLP_LAYERS)


def mlp_init(seed: int = 7) -> np.ndarray:
    """Initial screener parameters, flat float32: for each layer W (in x out, row-major)
    then b (out), each entry uniform in [-1/sqrt(in), 1/sqrt(in)] from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in MLP_LAYERS:
        bound = 1.0 / np.sqrt(i)
        parts.append(rng.uniform(-bound, bound, size=(i, o)).ravel())
        parts.append(rng.uniform(-bound, bound, size=o))
    return np.concatenate(parts).astype(np.float32)
