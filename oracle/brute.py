"""Independent references used to pin the oracle (TEST INFRASTRUCTURE ONLY).

* companion linearisation of a quadratic eigenvalue problem (a library eig),
* argument-principle eigenvalue counts (1/2 pi i) \\oint tr(T^{-1} T') dz,
* roots of scalar delay equations via the Lambert W function,
* the closed forms of the trapezoidal rule for simple poles.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np
import scipy.linalg as sla
import scipy.special as ssp

from gen import Problem, PHI_ONE, PHI_Z, PHI_Z2
from .nep import assemble, assemble_derivative


def qep_coefficients(prob: Problem):
    """(K, C, M) of a quadratic T(z) = K + z C + z^2 M given in split form."""
    K = C = M = None
    for A, kind in zip(prob.coeffs, prob.phi_kind):
        A = np.eye(prob.n, dtype=np.complex128) if A is None else A
        if kind == PHI_ONE:
            K = A if K is None else K + A
        elif kind == PHI_Z:
            C = A if C is None else C + A
        elif kind == PHI_Z2:
            M = A if M is None else M + A
        else:
            raise ValueError("not a quadratic problem")
    z = np.zeros((prob.n, prob.n), dtype=np.complex128)
    return (z if K is None else K), (z if C is None else C), (z if M is None else M)


def companion_eigs(prob: Problem) -> np.ndarray:
    """All 2n eigenvalues of K + z C + z^2 M from the first companion pencil
    [[0, I], [-K, -C]] - z [[I, 0], [0, M]]."""
    K, C, M = qep_coefficients(prob)
    n = prob.n
    I = np.eye(n)
    Z = np.zeros((n, n))
    A = np.block([[Z, I], [-K, -C]])
    B = np.block([[I, Z], [Z, M]])
    return sla.eig(A, B, right=False)


def argument_principle_count(prob: Problem, c: complex, r: float, nodes: int = 512) -> float:
    """(1/2 pi i) \\oint_{|z-c|=r} tr(T(z)^{-1} T'(z)) dz by a fine trapezoid: the number
    of eigenvalues (with multiplicity) inside the circle.  Returned unrounded."""
    theta = 2.0 * np.pi * np.arange(nodes) / nodes
    acc = 0j
    for t in theta:
        z = c + r * np.exp(1j * t)
        acc += (r / nodes) * np.exp(1j * t) * np.trace(np.linalg.solve(assemble(prob, z),
                                                                     assemble_derivative(prob, z)))
    return acc.real


def delay_scalar_roots(a: complex, b: complex, tau: float, branches: Sequence[int]) -> np.ndarray:
    """Roots of -z + a + b e^{-tau z} = 0: z = a + W_k(tau b e^{-a tau}) / tau."""
    arg = tau * b * np.exp(-a * tau)
    return np.array([a + ssp.lambertw(arg, k) / tau for k in branches])


def trapezoid_pole_full(delta: complex, N: int) -> complex:
    """Exact value of sum_j w_j / (z_j - a) for the N-point rule, delta = (a - c)/r:
    1/(1 - delta^N) inside the circle, -q^N/(1 - q^N) outside (q = 1/delta)."""
    if abs(delta) < 1:
        return 1.0 / (1.0 - delta ** N)
    q = 1.0 / delta
    return -q ** N / (1.0 - q ** N)


def trapezoid_pole_half(delta: complex, N: int) -> complex:
    """Exact value of the half rule on the 1-based even nodes (a rule shifted by half a
    step): 1/(1 + delta^{N/2}) inside, q^{N/2}/(1 + q^{N/2}) outside."""
    h = N // 2
    if abs(delta) < 1:
        return 1.0 / (1.0 + delta ** h)
    q = 1.0 / delta
    return q ** h / (1.0 + q ** h)


def hankel_zeros(m: int, x0: float, x1: float, y0: float, y1: float, grid: int = 24) -> np.ndarray:
    """Zeros of H_m^(1) in the rectangle: Newton (H_m' = (H_{m-1} - H_{m+1}) / 2) from a
    grid of starts, duplicates merged; the count is checked against the argument
    principle (1/2 pi i) oint H_m'/H_m on the rectangle's boundary."""
    h = lambda z: ssp.hankel1(m, z)
    dh = lambda z: 0.5 * (ssp.hankel1(m - 1, z) - ssp.hankel1(m + 1, z))
    found: List[complex] = []
    for a in np.linspace(x0, x1, grid):
        for b in np.linspace(y0, y1, grid):
            z = complex(a, b)
            for _ in range(60):
                step = h(z) / dh(z)
                z -= step
                if not np.isfinite(z) or abs(step) < 1e-15 * max(1.0, abs(z)):
                    break
            if np.isfinite(z) and x0 < z.real < x1 and y0 < z.imag < y1 and abs(h(z)) < 1e-10:
                if all(abs(z - w) > 1e-8 for w in found):
                    found.append(z)
    # argument principle on the boundary (a fine trapezoid rule per side)
    pts = np.concatenate([np.linspace(complex(x0, y0), complex(x1, y0), 4000, endpoint=False),
                          np.linspace(complex(x1, y0), complex(x1, y1), 4000, endpoint=False),
                          np.linspace(complex(x1, y1), complex(x0, y1), 4000, endpoint=False),
                          np.linspace(complex(x0, y1), complex(x0, y0), 4000, endpoint=False)])
    nxt = np.roll(pts, -1)
    mid = 0.5 * (pts + nxt)
    count = np.sum(dh(mid) / h(mid) * (nxt - pts)) / (2j * np.pi)
    assert abs(count - round(count.real)) < 1e-3 and round(count.real) == len(found), (m, count, found)
    return np.asarray(found, dtype=np.complex128)
