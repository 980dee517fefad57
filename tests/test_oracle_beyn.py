"""Pins of the oracle's Beyn extraction, ownership filter, verification and the
whole pmCIMb driver against independent references (companion linearisation,
library eigenvalues, Lambert-W delay roots, argument-principle counts, and the
paper's printed 4x4 example)."""
import os

import numpy as np
import pytest

import gen
import oracle
from oracle import brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _match(a, b):
    a = np.sort_complex(np.asarray(a))
    b = np.asarray(b)
    err = 0.0
    for v in a:
        err = max(err, np.min(np.abs(b - v)) / max(1.0, abs(v)))
    return err


def test_beyn_linear_matches_library_eig():
    # T(z) = A - z I with a non-normal A: the eigenvalues inside the circle are the
    # library eig(A) there.  Inside values within 0.5 r and outside ones beyond 1.6 r
    # keep the quadrature error below 0.5^N + 1.6^-N.
    n, c, r = 40, 0.1 + 0.1j, 0.45
    rng = np.random.default_rng(11)
    k_in = 6
    lam = np.empty(n, np.complex128)
    lam[:k_in] = c + 0.5 * r * rng.uniform(0, 1, k_in) * np.exp(2j * np.pi * rng.uniform(0, 1, k_in))
    lam[k_in:] = c + r * rng.uniform(1.6, 4, n - k_in) * np.exp(2j * np.pi * rng.uniform(0, 1, n - k_in))
    S = np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    A = S @ np.diag(lam) @ np.linalg.inv(S)
    prob = gen.Problem(n, [A.astype(np.complex128), None], [gen.PHI_ONE, gen.PHI_NEG_Z])
    ev = np.linalg.eigvals(A)
    inside = ev[np.abs(ev - c) < r]
    assert len(inside) == k_in
    sw = oracle.sweep_disk(prob, c, r, 64, gen.probes(1, n, 1), gen.probes(2, n, 12))
    br = oracle.beyn(sw.C0, sw.C1, 1e-8)
    assert br.p == k_in
    assert _match(br.lam, inside) < 1e-10
    # eigenvectors: A v = lambda v
    for k in range(br.p):
        v = br.vec[:, k]
        assert np.linalg.norm(A @ v - br.lam[k] * v) < 1e-9


def test_beyn_rotated_quadratic_exact_roots():
    # inside roots within 0.4 r, partner roots beyond 2.5 r: quadrature error ~ 0.4^N
    n, N = 10, 32
    rng = np.random.default_rng(3)
    c, r = 0.2 - 0.1j, 1.0
    a = c + 0.4 * r * rng.uniform(0, 1, n) * np.exp(2j * np.pi * rng.uniform(0, 1, n))
    b = c + r * (2.5 + rng.uniform(0, 1, n)) * np.exp(2j * np.pi * rng.uniform(0, 1, n))
    prob = gen.rotated_diagonal(a[:4].tolist() + (c + 3.0 + np.arange(n - 4)).tolist(), 8,
                                quadratic_partner=b)
    inside = a[:4]
    sw = oracle.sweep_disk(prob, c, r, N, gen.probes(1, n, 1), gen.probes(2, n, 6))
    br = oracle.beyn(sw.C0, sw.C1, 1e-6)
    assert br.p == 4
    assert _match(br.lam, inside) < 1e-11


def test_beyn_delay_lambert_w():
    # commuting diagonal (rotated) delay problem -zI + A0 + A1 e^{-tau z}; its
    # eigenvalues are the scalar roots a_i + W_k(tau b_i e^{-a_i tau}) / tau.
    tau = 1.3
    a = np.array([-0.4, 0.1, -1.2, 0.3, -0.8, 0.6])
    b = np.array([0.9, -0.5, 0.3, 0.2, -0.7, 0.4])
    n = len(a)
    r2 = np.random.default_rng(21)
    Z = r2.standard_normal((n, n)) + 1j * r2.standard_normal((n, n))
    Q, _ = np.linalg.qr(Z)
    A0 = Q @ np.diag(a) @ Q.conj().T
    A1 = Q @ np.diag(b) @ Q.conj().T
    prob = gen.delay(A0, A1, tau)
    roots = np.concatenate([brute.delay_scalar_roots(a[i], b[i], tau, range(-4, 5)) for i in range(n)])
    assert np.max(np.abs(-roots + np.repeat(a, 9) + np.repeat(b, 9) * np.exp(-tau * roots))) < 1e-12
    c = -0.2 + 0.1j
    d = np.sort(np.abs(roots - c))
    k = int(np.argmax(d[1:5] - d[0:4]))             # widest gap among the 5 nearest
    r = 0.5 * (d[k] + d[k + 1])
    inside = roots[np.abs(roots - c) < r]
    assert 1 <= len(inside) <= n
    sw = oracle.sweep_disk(prob, c, r, 128, gen.probes(1, n, 1), gen.probes(2, n, n))
    br = oracle.beyn(sw.C0, sw.C1, 1e-8)
    assert br.p == len(inside)
    # trapezoidal error bound on a circle: (max inside |a-c|/r)^N + (r / min outside |a-c|)^N
    dist = np.abs(roots - c)
    bound = np.max(dist[dist < r] / r) ** 128 + (r / np.min(dist[dist > r])) ** 128
    assert _match(br.lam, inside) < 1e3 * bound + 1e-11


def test_paper_demo_recovers_all_eigenvalues():
    # The paper's worked input: 4x4 quadratic, [-3,3]^2 split 9x9, N = 64, l = 10.
    ref = np.loadtxt(os.path.join(GOLD, "paper_demo_qep.txt"))
    prob = gen.paper_demo_problem()
    res = oracle.pmcimb(prob, gen.Region(-3, 3, -3, 3, 9, 9), gen.Options(N=64, s=1, L=10),
                       gen.probes(11, 4, 1), gen.probes(12, 4, 10))
    assert len(res.eigs) == 8
    assert np.max(np.abs(np.sort(res.eigs.real) - ref) / np.abs(ref)) < 1e-12
    assert np.max(np.abs(res.eigs.imag)) < 1e-12
    # independent of the probes (Section 2.1: P f = 0 iff no eigenvalue, w.p. 1)
    res2 = oracle.pmcimb(prob, gen.Region(-3, 3, -3, 3, 9, 9), gen.Options(N=64, s=1, L=10),
                        gen.probes(21, 4, 1), gen.probes(22, 4, 10))
    assert np.max(np.abs(np.sort(res2.eigs.real) - ref)) < 1e-11
    # each stored value is a root of det T
    for v in ref:
        assert oracle.sigma_min(prob, v) < 1e-12


def test_flags_agree_with_argument_principle_small_qep():
    w = gen.workload_small_qep()
    prob, reg = w.problems[0], w.regions[0]
    ev = brute.companion_eigs(prob)
    assert len(ev) == 128
    res = oracle.pmcimb(prob, reg, w.opts, w.F[0], None)
    for k, dk in enumerate(res.disks):
        dist = np.abs(ev - dk.c)
        count_geom = int(np.sum(dist < dk.r))
        if np.min(np.abs(dist - dk.r)) > 0.1 * dk.r:
            # clear of the contour: flag iff the disk holds eigenvalues
            assert res.flags[k] == (count_geom > 0)
    # argument-principle count on two disks equals the companion count
    clear = [np.min(np.abs(np.abs(ev - d.c) - d.r)) / d.r for d in res.disks]
    holding = [k for k in range(16) if np.sum(np.abs(ev - res.disks[k].c) < res.disks[k].r) > 0]
    for k in (0, max(holding, key=lambda k: clear[k])):
        dk = res.disks[k]
        cnt = brute.argument_principle_count(prob, dk.c, dk.r, 1024)
        assert abs(cnt - round(cnt)) < 1e-3
        assert round(cnt) == int(np.sum(np.abs(ev - dk.c) < dk.r))


def test_owner_cell_edges():
    reg = gen.Region(-2, 2, -2, 2, 4, 4)
    assert oracle.owner_cell(0.3 + 0.3j, reg) == (2, 2)
    assert oracle.owner_cell(0.0 + 0.3j, reg) == (1, 2)      # on x = 0: the smaller neighbour
    assert oracle.owner_cell(1e-13 + 0.3j, reg) == (1, 2)    # inside the tie band
    assert oracle.owner_cell(5e-7 + 0.3j, reg) == (1, 2)     # inside the 1e-6 band
    assert oracle.owner_cell(1e-5 + 0.3j, reg) == (2, 2)     # outside the band
    assert oracle.owner_cell(-2.0 - 2.0j, reg) == (0, 0)      # closed region corner
    assert oracle.owner_cell(2.0 + 2.0j, reg) == (3, 3)
    assert oracle.owner_cell(2.1 + 0j, reg) is None


def test_sigma_min_and_dedup():
    prob = gen.paper_demo_problem()
    ev = brute.companion_eigs(prob)
    for v in ev:
        assert oracle.sigma_min(prob, v) < 1e-12
    z = 0.7 + 0.2j
    assert oracle.sigma_min(prob, z) <= oracle.min_abs_eig(prob, z) + 1e-15
    keep = oracle.dedup([1.0 + 0j, 1.0 + 1e-12j, 2.0 + 0j], [1e-9, 1e-12, 1e-10])
    assert keep == [1, 2]


def test_small_qep_structure():
    # The small configuration's spectrum: 128 eigenvalues, 12 of 16 disks flagged.
    w = gen.workload_small_qep()
    prob = w.problems[0]
    ev = brute.companion_eigs(prob)
    assert np.max(np.abs(ev)) < 2.0
    res = oracle.pmcimb(prob, w.regions[0], w.opts, w.F[0], w.V[0])
    assert int(res.flags.sum()) == 12
    # every accepted value is a true eigenvalue
    for v in res.eigs:
        assert np.min(np.abs(ev - v)) < 1e-6 * max(1, abs(v))
