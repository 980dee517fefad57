"""Pins of the oracle's scattering-pole problem (Section 4.2's sound-soft unit disk): the
Nystrom matrix of (I + K(k)) / 2 acts on the sampled Fourier modes e^{i m t} with the
exact eigenvalues (i pi k / 2) J_m'(k) H_m(k) of the continuous operator (library
Bessel functions), so its singular points in the lower half-plane are the zeros of
the Hankel functions; the zeros themselves are checked by their residual and an
argument-principle count, and the whole pmCIMb driver over the paper's region (100
squares) returns exactly them."""
import functools

import numpy as np
import scipy.special as ssp

import gen
import oracle
from oracle import brute

REGION = (0.2, 3.2, -3.2, -0.2)


@functools.lru_cache(maxsize=1)
def _all_zeros():
    return np.concatenate([brute.hankel_zeros(m, *REGION) for m in range(0, 11)])


def test_fourier_modes_are_eigenvectors():
    n = 64
    t = 2 * np.pi * np.arange(n) / n
    for k in (1.3 - 0.7j, 2.2 - 1.9j, 0.5 - 0.3j, 3.0 - 2.9j):
        T = oracle.assemble(gen.CircleDoubleLayer(n), k)
        for m in range(-12, 13):
            e = np.exp(1j * m * t)
            mu = (1j * np.pi * k / 2) * 0.5 * (ssp.jv(m - 1, k) - ssp.jv(m + 1, k)) * ssp.hankel1(m, k)
            assert np.linalg.norm(T @ e - mu * e) <= 1e-12 * np.linalg.norm(e), (k, m)


def test_hankel_zeros_are_double_singular_points():
    zs = _all_zeros()
    assert len(zs) == 6                      # m = 2, 3, 4 (two), 5 (two); none for m <= 1 or m >= 6
    T = gen.CircleDoubleLayer(64)
    for z in zs:
        s = np.linalg.svd(oracle.assemble(T, z), compute_uv=False)
        # modes m and -m: two singular values at rounding level, the third well away
        assert s[-1] < 1e-12 and s[-2] < 1e-12 and s[-3] > 1e-3, (z, s[-3:])


def test_driver_finds_the_poles():
    x0, x1, y0, y1 = REGION
    reg = gen.Region(x0, x1, y0, y1, 10, 10)
    opts = gen.Options(N=32, s=1, L=4)
    prob = gen.CircleDoubleLayer(64)
    res = oracle.pmcimb(prob, reg, opts, gen.probes(11, 64, 1), gen.probes(12, 64, 4))
    zs = _all_zeros()
    assert len(res.eigs) == len(zs)
    for z in zs:
        assert np.min(np.abs(res.eigs - z)) < 1e-9 * abs(z)
