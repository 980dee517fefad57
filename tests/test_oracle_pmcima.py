"""Pins of the oracle's pmCIMa (Section 3.1): the level count and the last cells'
size in closed form, the quadrant geometry, the merge on constructed centres, and
the whole recursion against independent references (the paper's printed 4x4
quadratic and its companion eigenvalues; a rotated diagonal linear problem whose
eigenvalues and null vectors are known exactly; Lambert-W roots of a delay problem)."""
import math
import os

import numpy as np

import gen
from oracle import brute
from oracle import pmcima as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_level_count_and_last_radius():
    for r, tol in ((math.sqrt(2) / 2, 1e-6), (0.3, 1e-6), (1.0, 1e-3), (0.25 * math.sqrt(2), 1e-8)):
        L = P.level_count(r, tol)
        # each level halves the radius: the last cells are tol/4 .. tol/2 in radius
        rl = r / 2 ** (L - 1)
        assert tol / 4 < rl <= tol / 2, (r, tol, L, rl)
    assert P.level_count(math.sqrt(2) / 2, 1e-6) == 22


def test_children_are_quadrants():
    ch = P.children((0.0, 1.0, -1.0, 0.0))
    cells = [c for c, _, _ in ch]
    assert cells == [(0.0, 0.5, -1.0, -0.5), (0.0, 0.5, -0.5, 0.0), (0.5, 1.0, -1.0, -0.5), (0.5, 1.0, -0.5, 0.0)]
    for cell, c, r in ch:
        assert c == complex((cell[0] + cell[1]) / 2, (cell[2] + cell[3]) / 2)
        assert abs(r - math.sqrt(2) / 4) < 1e-15


def test_merge_star_clusters():
    t = 1e-6
    z = [0.0, 0.6e-6, 1.3e-6, 5.0, 5.0 + 0.5e-6j, 2.0]
    # 0 takes 0.6e-6 but not 1.3e-6 (1.3e-6 from 0), which then starts its own cluster
    out = P.merge(z, t)
    assert np.allclose(out, [0.3e-6, 1.3e-6, 5.0 + 0.25e-6j, 2.0], rtol=0, atol=1e-15)
    assert P.merge([], t).shape == (0,)


def _one_to_one(found, exact, tol):
    d = np.abs(found[:, None] - exact[None, :])
    near = np.argmin(d, axis=0)
    assert len(set(near.tolist())) == len(exact)
    return d[near, np.arange(len(exact))].max()


def test_paper_demo_all_eigenvalues():
    # the paper's printed 4x4 quadratic: 8 real eigenvalues, every one in [-3,3] x [-1,1]
    gold = np.loadtxt(os.path.join(GOLD, "paper_demo_qep.txt"))
    prob = gen.paper_demo_problem()
    res = P.pmcima(prob, gen.Region(-3, 3, -1, 1, 6, 2), gen.probes(2, 4, 1))
    assert res.levels == P.level_count(math.sqrt(2) / 2, 1e-6)
    assert len(res.eigs) == 8
    assert _one_to_one(res.eigs, gold, 1e-6) <= 0.5e-6
    # Step 2: the vector is the eigenvector of the companion pencil to O(|lambda - lambda*|)
    K, Cm, M = brute.qep_coefficients(prob)
    for lam, v, s in zip(res.eigs, res.vectors, res.sigma):
        ex = gold[np.argmin(np.abs(gold - lam))]
        T = K + ex * Cm + ex * ex * M
        x = np.linalg.svd(T)[2][-1].conj()
        assert abs(abs(np.vdot(x, v)) - 1.0) < 1e-5
        assert abs(np.linalg.norm(v) - 1.0) < 1e-14
        k = np.argmax(np.abs(v))
        assert v[k].imag == 0 and v[k].real > 0
        assert s < 1e-5


def test_rotated_linear_values_and_null_vectors():
    # T(z) = Q diag(z - a_i) Q^H: eigenvalues a_i; at any lambda the singular vectors are
    # the columns of Q, so the returned vector is the exact null vector of T(a_i)
    a = np.array([0.31 + 0.22j, -0.55 + 0.61j, 0.47 + 0.013j, -0.2 - 0.7j, 0.8 - 0.45j, 1.7 + 1.1j])
    prob = gen.rotated_diagonal(a, seed=17)
    res = P.pmcima(prob, gen.Region(-1, 1, -1, 1, 2, 2), gen.probes(5, len(a), 1))
    inside = a[(np.abs(a.real) < 1) & (np.abs(a.imag) < 1)]
    assert len(res.eigs) == len(inside)
    assert _one_to_one(res.eigs, inside, 1e-6) <= 0.5e-6
    for lam, v in zip(res.eigs, res.vectors):
        ex = inside[np.argmin(np.abs(inside - lam))]
        T = prob.coeffs[0] + ex * np.eye(len(a))
        assert np.linalg.norm(T @ v) < 1e-13


def test_delay_lambert_roots():
    # rotated diagonal delay problem: the eigenvalues are the Lambert-W roots of the
    # scalar equations -z + a_i + b_i exp(-tau z) = 0
    n, tau = 4, 1.0
    a = np.array([-0.5 + 0.2j, 0.1 - 0.3j, -0.2 + 0.0j, 0.3 + 0.4j])
    b = np.array([0.3, -0.2 + 0.1j, 0.25, -0.1])
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    prob = gen.delay(Q @ np.diag(a) @ Q.conj().T, Q @ np.diag(b) @ Q.conj().T, tau)
    roots = np.concatenate([brute.delay_scalar_roots(a[i], b[i], tau, range(-3, 4)) for i in range(n)])
    reg = gen.Region(-1.5, 1.0, -1.0, 1.0, 5, 4)
    inside = roots[(roots.real > reg.x0) & (roots.real < reg.x1) & (roots.imag > reg.y0) & (roots.imag < reg.y1)]
    assert len(inside) >= 4
    res = P.pmcima(prob, reg, gen.probes(6, n, 1), vectors=False)
    assert len(res.eigs) == len(inside)
    assert _one_to_one(res.eigs, inside, 1e-6) <= 0.5e-6


def test_sim_quadtree_labels_against_root_positions():
    # a rotated diagonal linear problem with known roots: a child's disk is flagged
    # exactly when it holds a root, for roots kept at least 0.15 r away from every
    # child circle (inside: I ~ 1 per root; outside: I ~ q^{N/2} << tol_ind); the root
    # is always split, and only flagged children are split again, in cover order
    roots = np.array([0.61 + 0.37j, -1.22 - 1.41j, 2.63 - 0.52j, -2.9 + 2.7j, 3.55 + 3.45j])
    n = len(roots)
    prob = gen.rotated_diagonal(roots, 19)
    F = gen.probes(23, n, 1)
    recs = P.sim_quadtree_labels(prob, (-4.0, 4.0, -4.0, 4.0), 3, F, N=32)

    def holds(c, r):
        return np.abs(roots - c) < r

    parents = {(-4.0, 4.0, -4.0, 4.0)}
    for level, cell, ind in recs:
        assert cell in parents, (level, cell)
        for (ch, c, r), I in zip(P.children(cell), ind):
            d = np.abs(np.abs(roots - c) - r)
            if np.all(d > 0.15 * r):
                assert (I > 0.1) == bool(holds(c, r).any()), (level, ch, I)
            if I > 0.1 and level < 2:
                parents.add(ch)
    # level 0 has one record; each later record's cell was a flagged child of the previous level
    assert [lv for lv, _, _ in recs].count(0) == 1
