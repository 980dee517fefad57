"""Pins of the oracle's quadrature sweep and indicator against closed forms.

Nothing here calls the GPU.  The closed forms are the exact discrete sums of the
trapezoidal rule for simple poles (derived from the geometric series of
1/(1 - delta e^{-i theta}) over the N-th roots of unity), so a dropped term, a wrong
sign, a wrong node set for the half rule or a wrong weight fails them.
"""
import numpy as np
import pytest

import gen
import oracle
from oracle import brute


@pytest.mark.parametrize("N", [8, 16, 32, 48])
def test_weights_sum_to_zero(N):
    z, w = oracle.nodes_weights(0.3 - 0.2j, 0.7, N)
    assert abs(w.sum()) < 1e-15
    assert np.allclose(np.abs(z - (0.3 - 0.2j)), 0.7, atol=1e-15)
    # first node at theta = 0 (theta_j = 2 pi (j-1)/N, j = 1..N)
    assert abs(z[0] - (0.3 - 0.2j + 0.7)) < 1e-15


@pytest.mark.parametrize("N", [16, 32, 48, 64])
@pytest.mark.parametrize("delta", [0.0, 0.3 + 0.4j, -0.85, 0.9j, 1.3 - 0.2j, -2.5, 4j])
def test_pole_sums_match_closed_form(N, delta):
    c, r = 0.5 + 0.25j, 0.8
    a = c + r * delta
    z, w = oracle.nodes_weights(c, r, N)
    full = np.sum(w / (z - a))
    half = np.sum(2.0 * w[1::2] / (z[1::2] - a))     # 1-based even nodes j = 2, 4, ..., N
    assert abs(full - brute.trapezoid_pole_full(delta, N)) < 1e-14
    assert abs(half - brute.trapezoid_pole_half(delta, N)) < 1e-14
    # z-weighted sum: sum w_j z_j/(z_j - a) = a * sum w_j/(z_j - a)  (sum w_j = 0)
    assert abs(np.sum(w * z / (z - a)) - a * brute.trapezoid_pole_full(delta, N)) < 1e-13


def test_sweep_linear_closed_form():
    n = 12
    rng = np.random.default_rng(7)
    roots = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    seed = 77
    prob = gen.rotated_diagonal(roots, seed)
    # the same unitary as the generator (seeded), rebuilt here for the closed form
    r2 = np.random.default_rng(seed)
    Z = r2.standard_normal((n, n)) + 1j * r2.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    Q = Q * (np.diag(R) / np.abs(np.diag(R)))
    F = gen.probes(1, n, 2)
    V = gen.probes(2, n, 3)
    c, r, N = 0.1 + 0.05j, 0.6, 32
    sw = oracle.sweep_disk(prob, c, r, N, F, V)
    delta = (roots - c) / r
    g = np.array([brute.trapezoid_pole_full(d, N) for d in delta])
    h = np.array([brute.trapezoid_pole_half(d, N) for d in delta])
    QH = Q.conj().T
    assert np.allclose(sw.PfN, Q @ np.diag(g) @ QH @ F, rtol=0, atol=1e-13)
    assert np.allclose(sw.PfN2, Q @ np.diag(h) @ QH @ F, rtol=0, atol=1e-13)
    assert np.allclose(sw.C0, Q @ np.diag(g) @ QH @ V, rtol=0, atol=1e-13)
    assert np.allclose(sw.C1, Q @ np.diag(roots * g) @ QH @ V, rtol=0, atol=1e-13)
    # indicator from the exact vectors
    I, Iq = oracle.indicator(sw.PfN, sw.PfN2)
    ex = Q @ np.diag(g) @ QH @ F
    eh = Q @ np.diag(h) @ QH @ F
    exact = np.max(np.linalg.norm(ex / eh, axis=0) / np.sqrt(n))
    assert abs(I - exact) < 1e-10 * max(1, exact)
    # profile = per-node solution norms
    z, _ = oracle.nodes_weights(c, r, N)
    for j in (0, 5, 31):
        x = Q @ np.diag(1.0 / (z[j] - roots)) @ QH @ F
        assert np.allclose(sw.profile[j], np.linalg.norm(x, axis=0), rtol=1e-12)


def test_sweep_quadratic_partial_fractions():
    n = 8
    rng = np.random.default_rng(9)
    a = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    b = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n) + 3.0
    seed = 31
    prob = gen.rotated_diagonal(a, seed, quadratic_partner=b)
    r2 = np.random.default_rng(seed)
    Z = r2.standard_normal((n, n)) + 1j * r2.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    Q = Q * (np.diag(R) / np.abs(np.diag(R)))
    F = gen.probes(3, n, 1)
    V = gen.probes(4, n, 4)
    c, r, N = -0.1 + 0.2j, 1.1, 48
    sw = oracle.sweep_disk(prob, c, r, N, F, V)
    g = lambda x: brute.trapezoid_pole_full((x - c) / r, N)
    # 1/((z-a)(z-b)) = (1/(z-a) - 1/(z-b)) / (a - b)
    ga = np.array([(g(ai) - g(bi)) / (ai - bi) for ai, bi in zip(a, b)])
    za = np.array([(ai * g(ai) - bi * g(bi)) / (ai - bi) for ai, bi in zip(a, b)])
    QH = Q.conj().T
    assert np.allclose(sw.PfN, Q @ np.diag(ga) @ QH @ F, rtol=0, atol=1e-12)
    assert np.allclose(sw.C0, Q @ np.diag(ga) @ QH @ V, rtol=0, atol=1e-12)
    assert np.allclose(sw.C1, Q @ np.diag(za) @ QH @ V, rtol=0, atol=1e-12)


def test_indicator_inside_vs_outside():
    # one root inside a rotated problem: I ~ 1; all roots far outside: I ~ q^{N/2}
    n = 16
    roots = np.concatenate([[0.05 + 0.02j], 3.0 + np.arange(n - 1) * 0.1])
    prob = gen.rotated_diagonal(roots, 3)
    F = gen.probes(5, n, 1)
    sw = oracle.sweep_disk(prob, 0j, 0.5, 32, F, None)
    I_in, _ = oracle.indicator(sw.PfN, sw.PfN2)
    assert 0.5 < I_in < 2.0
    sw2 = oracle.sweep_disk(prob, 1.2 + 0j, 0.3, 32, F, None)
    I_out, _ = oracle.indicator(sw2.PfN, sw2.PfN2)
    assert I_out < 1e-3


def test_indicator_nonfinite_flags():
    PfN = np.ones((4, 2), np.complex128)
    PfN2 = np.ones((4, 2), np.complex128)
    PfN2[1, 1] = 0
    I, Iq = oracle.indicator(PfN, PfN2)
    assert np.isinf(I) and Iq[0] == pytest.approx(1.0)


def test_solve_residual_small_qep():
    w = gen.workload_small_qep()
    prob = w.problems[0]
    z = 0.3 + 0.7j
    T = oracle.assemble(prob, z)
    B = np.concatenate([w.F[0], w.V[0]], axis=1)
    import scipy.linalg as sla
    X = sla.solve(T, B)
    res = np.linalg.norm(T @ X - B) / (np.linalg.norm(T) * np.linalg.norm(X))
    assert res < 1e-15
    # assembly: K + z C + z^2 I
    K, C, M = brute.qep_coefficients(prob)
    assert np.allclose(T, K + z * C + z * z * M, atol=1e-15)


def test_cover_geometry():
    reg = gen.Region(-3.0, 1.0, -6.0, 6.0, 8, 16)
    d = oracle.cover(reg)
    assert len(d) == 128
    assert d[0].hx == pytest.approx(0.25) and d[0].hy == pytest.approx(0.375)
    assert d[0].r == pytest.approx(np.hypot(0.25, 0.375))
    assert (d[17].ix, d[17].iy) == (1, 1)
    assert d[17].cx == pytest.approx(-3 + 0.75) and d[17].cy == pytest.approx(-6 + 0.375 * 3)


def _rotated(n, roots, seed):
    """The generator's rotated diagonal problem Q diag(z - a_i) Q^H and its unitary Q
    (rebuilt here from the same seed for the closed forms)."""
    prob = gen.rotated_diagonal(roots, seed)
    r2 = np.random.default_rng(seed)
    Z = r2.standard_normal((n, n)) + 1j * r2.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    return prob, Q * (np.diag(R) / np.abs(np.diag(R)))


def test_summand_scales_closed_form():
    # x_j = Q diag(1/(z_j - a_i)) Q^H f, so ||x_j||^2 = sum_i |g_i|^2 / |z_j - a_i|^2 with
    # g = Q^H f (Q unitary): S_N = sum_j (r/N) ||x_j||, S_half = sum_{j even} 2 (r/N) ||x_j||
    n = 10
    rng = np.random.default_rng(12)
    roots = 2.0 * (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n))
    prob, Q = _rotated(n, roots, 13)
    F = gen.probes(14, n, 3)
    c, r, N = 0.2 - 0.1j, 0.7, 16
    sw = oracle.sweep_disk(prob, c, r, N, F, None)
    theta = 2.0 * np.pi * np.arange(N) / N
    z = c + r * np.exp(1j * theta)
    g = Q.conj().T @ F
    xn = np.sqrt((np.abs(g)[None, :, :] ** 2 / np.abs(z[:, None, None] - roots[None, :, None]) ** 2).sum(axis=1))
    SN = (r / N) * xn.sum(axis=0)
    SH = 2.0 * (r / N) * xn[1::2].sum(axis=0)          # 1-based even nodes 2, 4, ..., N
    assert np.allclose(sw.profile, xn, rtol=1e-12, atol=0)
    assert np.allclose(sw.scale, SN, rtol=1e-12, atol=0)
    assert np.allclose(sw.scale_half, SH, rtol=1e-12, atol=0)


def test_noise_floor_is_above_the_rounding_of_an_empty_disk():
    # poles far outside (q = 0.25 / 4 -> q^{N/2} ~ 1e-19): both computed sums are
    # rounding noise, far below the floor times their summand sizes
    n = 12
    roots = 4.0 + 0.3 * np.arange(n) + 0.1j
    prob, _ = _rotated(n, roots, 5)
    sw = oracle.sweep_disk(prob, 0j, 0.25, 32, gen.probes(6, n, 2), None)
    a = np.array([oracle.norm2(sw.PfN[:, q]) for q in range(2)]) / sw.scale
    b = np.array([oracle.norm2(sw.PfN2[:, q]) for q in range(2)]) / sw.scale_half
    assert np.all(a < 1e-3 * oracle.NOISE_FLOOR) and np.all(b < 1e-3 * oracle.NOISE_FLOOR)


@pytest.mark.parametrize("dist", [0.6, 0.75])
def test_indicator_above_the_floor_matches_closed_form(dist):
    # every pole outside at |a - c| = r / q with q^{N/2} ~ 1e-4 .. 1e-2: the half-rule sum
    # is far above the floor, so the indicator is the ratio of the exact closed-form
    # vectors, q^{N/2}-small and unflagged
    n, N = 8, 32
    c, r = 0.1 + 0.1j, 0.5
    ang = 2.0 * np.pi * np.arange(n) / n + 0.3
    roots = c + (r / dist) * np.exp(1j * ang) * (1.0 + 0.05 * np.arange(n))
    prob, Q = _rotated(n, roots, 21)
    F = gen.probes(22, n, 1)
    sw = oracle.sweep_disk(prob, c, r, N, F, None)
    delta = (roots - c) / r
    gN = np.array([brute.trapezoid_pole_full(d, N) for d in delta])
    gH = np.array([brute.trapezoid_pole_half(d, N) for d in delta])
    ex = Q @ np.diag(gN) @ Q.conj().T @ F
    eh = Q @ np.diag(gH) @ Q.conj().T @ F
    exact = np.linalg.norm(ex / eh) / np.sqrt(n)
    assert oracle.norm2(sw.PfN2[:, 0]) > 1e3 * oracle.NOISE_FLOOR * sw.scale_half[0]
    I, _ = sw.indicator()
    assert abs(I - exact) <= 1e-6 * exact
    assert 0 < I < 0.1


@pytest.mark.parametrize("node", [0, 1, 6, 7])
@pytest.mark.parametrize("delta", [1e-8, 1e-12])
def test_outside_eigenvalue_next_to_a_node_keeps_the_disk_flagged(node, delta):
    # an eigenvalue inside the disk and one just outside the circle, delta * r from node
    # `node` (0-based; odd and even nodes of the half rule): that node's solution
    # dominates the summands of its rule(s) and P f|_N alike, so neither rule's sum can
    # fall under the noise floor and the disk stays flagged
    n, N = 12, 16
    c, r = 0.0j, 1.0
    zk = c + r * np.exp(2j * np.pi * node / N)
    roots = np.concatenate([[0.3 * np.exp(0.7j), zk + delta * r * (zk - c) / r], 5.0 + 0.5 * np.arange(n - 2)])
    prob, _ = _rotated(n, roots, 31)
    sw = oracle.sweep_disk(prob, c, r, N, gen.probes(32, n, 1), None)
    I, _ = sw.indicator()
    assert I > 0.1
    # the disk with the inside eigenvalue alone is flagged too, with I ~ 1
    roots2 = roots.copy()
    roots2[1] = 7.0
    prob2, _ = _rotated(n, roots2, 31)
    I2, _ = oracle.sweep_disk(prob2, c, r, N, gen.probes(32, n, 1), None).indicator()
    assert 0.5 < I2 < 2.0


def test_indicator_is_scale_invariant():
    # T scaled by 1e+-160 scales every sum by the inverse; the ratio is unchanged and no
    # square of an entry may overflow or underflow
    n = 16
    roots = np.concatenate([[0.05 + 0.02j], 0.4 + 0.1j * np.arange(n - 1)])
    prob, _ = _rotated(n, roots, 41)
    F = gen.probes(42, n, 1)
    sw = oracle.sweep_disk(prob, 0j, 0.5, 32, F, None)
    I0, _ = sw.indicator()
    for f in (1e-160, 1e160):
        I, _ = oracle.indicator(f * sw.PfN, f * sw.PfN2, (f * sw.scale, f * sw.scale_half))
        assert I == pytest.approx(I0, rel=1e-13)


def test_indicator_noise_floor():
    # all roots far outside: both sums sink below the rounding level of the summands
    # (q^N ~ 1e-40), their raw ratio is noise of order one, the floor reports 0; a disk
    # with a root inside is unaffected by the floor
    n = 12
    roots = 4.0 + 0.3 * np.arange(n) + 0.1j
    prob = gen.rotated_diagonal(roots, 5)
    F = gen.probes(6, n, 2)
    sw = oracle.sweep_disk(prob, 0j, 0.25, 32, F, None)
    assert np.all(np.linalg.norm(sw.PfN2, axis=0) < 1e-12 * sw.scale_half)
    assert np.all(np.linalg.norm(sw.PfN, axis=0) < 1e-12 * sw.scale)
    I, Iq = sw.indicator()
    assert I == 0.0 and np.all(Iq == 0.0)
    roots2 = roots.copy()
    roots2[0] = 0.05 - 0.02j
    prob2 = gen.rotated_diagonal(roots2, 5)
    sw2 = oracle.sweep_disk(prob2, 0j, 0.25, 32, F, None)
    a, _ = oracle.indicator(sw2.PfN, sw2.PfN2)
    b, _ = sw2.indicator()
    assert a == b and b > 0.1
