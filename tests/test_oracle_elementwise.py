"""Pins of the oracle on a problem without a short split form: the elementwise delay
T(z) = -z I + A0 + A1 .* exp(-tau .* z).  Its assembly reduces to the split delay
problem when every delay is equal; its derivative matches finite differences; with
upper-triangular A0, A1 its eigenvalues are the Lambert-W roots of the diagonal
entries (each with its own delay), which Beyn's extraction on one disk recovers; and
the whole driver's flags agree with argument-principle counts."""
import numpy as np

import gen
import oracle
from oracle import brute


def test_equal_delays_reduce_to_split_form():
    p = gen.elementwise_delay(9, seed=50)
    p.tau[:] = 1.3
    q = gen.delay(p.A0, p.A1, 1.3)
    for z in (0.3 - 0.2j, -1.1 + 2.0j, 0.0):
        assert np.allclose(oracle.assemble(p, z), oracle.assemble(q, z), rtol=0, atol=1e-14)
        assert np.allclose(oracle.assemble_derivative(p, z), oracle.assemble_derivative(q, z), rtol=0, atol=1e-14)


def test_derivative_by_finite_differences():
    p = gen.elementwise_delay(7, seed=60)
    z, h = 0.4 - 0.7j, 1e-6
    fd = (oracle.assemble(p, z + h) - oracle.assemble(p, z - h)) / (2 * h)
    fdi = (oracle.assemble(p, z + 1j * h) - oracle.assemble(p, z - 1j * h)) / (2j * h)
    d = oracle.assemble_derivative(p, z)
    assert np.max(np.abs(fd - d)) < 1e-8 and np.max(np.abs(fdi - d)) < 1e-8


def _triangular(n, seed):
    p = gen.elementwise_delay(n, seed=seed)
    p.A0[:] = np.triu(p.A0)
    p.A1[:] = np.triu(p.A1)
    return p


def test_beyn_recovers_lambert_roots_of_triangular_problem():
    # det T(z) = prod_i (-z + a_i + b_i exp(-tau_ii z)): the roots of each diagonal entry
    n = 6
    p = _triangular(n, seed=70)
    a, b, t = np.diag(p.A0), np.diag(p.A1), np.diag(p.tau)
    roots = np.concatenate([brute.delay_scalar_roots(a[i], b[i], t[i], range(-4, 5)) for i in range(n)])
    # a disk around the two closest principal-branch roots, every other root well
    # outside it (quadrature error below 1e-12 with 128 nodes)
    prin = np.array([brute.delay_scalar_roots(a[i], b[i], t[i], [0])[0] for i in range(n)])
    d = np.abs(prin[:, None] - prin[None, :]) + np.eye(n) * 1e9
    i, j = np.unravel_index(np.argmin(d), d.shape)
    c = 0.5 * (prin[i] + prin[j])
    r = 0.8 * d[i, j]
    inside = roots[np.abs(roots - c) < r]
    assert len(inside) >= 2
    assert np.all(np.abs(inside - c) < 0.7 * r)
    assert np.all(np.abs(roots[np.abs(roots - c) >= r] - c) > 1.3 * r)
    F = gen.probes(71, n, 1)
    V = gen.probes(72, n, 6)
    sw = oracle.sweep_disk(p, c, r, 128, F, V)
    br = oracle.beyn(sw.C0, sw.C1, 1e-8)
    assert br.p == len(inside)
    for v in inside:
        assert np.min(np.abs(br.lam - v)) < 1e-9


def test_driver_flags_match_argument_principle():
    p = gen.elementwise_delay(10, seed=80)
    reg = gen.Region(-2.0, 1.0, -3.0, 3.0, 3, 6)
    opts = gen.Options(N=32, s=1, L=0)
    F = gen.probes(81, p.n, 1)
    res = oracle.pmcimb(p, reg, opts, F, None)
    checked = 0
    for d, flag in zip(res.disks, res.flags):
        cnt = brute.argument_principle_count(p, d.c, d.r, nodes=256)
        k = int(round(cnt))
        near = brute.argument_principle_count(p, d.c, 1.2 * d.r, nodes=256)
        inner = brute.argument_principle_count(p, d.c, 0.8 * d.r, nodes=256)
        if round(near) == round(inner):        # no eigenvalue close to the circle
            assert abs(cnt - k) < 1e-6
            assert bool(flag) == (k > 0), (d, cnt)
            checked += 1
    assert checked >= 6
