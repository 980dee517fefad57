"""Writes the stored expected values under tests/golden/ from the oracle only.

paper_demo_qep.txt: the 4x4 quadratic printed in the paper's appendix routine that
generates T(z) (T2 = diag(3,1,3,1), T1, T0 as printed there), and its 8 eigenvalues
from the companion linearisation (a library generalized eigensolver).

small_qep_n64_eigs.txt: the 128 eigenvalues of the n = 64 QEP (K = A + A^T, C = 0.1 B,
M = I, seeds 0, 1) from its companion pencil, sorted by (Re, Im).

hankel_zeros_scattering.txt: the zeros of the Hankel functions H_m^(1), m = 0..10, in
[0.2, 3.2] x [-3.2, -0.2] (the scattering poles of the sound-soft unit disk in the
region of the paper's scattering experiment), by Newton and argument-principle count.

dense_qep_n1024_eigs.txt (with --dense; minutes of CPU): the 2048 eigenvalues of the
dense n = 1024 QEP (K = A + A^T, C = 0.1 B, M = I + 0.1 G G^T, seeds 0, 1, 2) from
its companion pencil, sorted by (Re, Im).

dense_qep_n1024_indicators.txt (with --dense-sweep; ~15 min on 8 cores): the oracle's
indicator sweep of the dense n = 1024 workload (256 disks x 32 nodes, 4 probe columns):
per disk the flag, I_q and the sizes of both sums relative to their summands.

delay_uneven_indicators.txt (with --delay; ~30 min on 8 cores): the oracle's indicator
of every rectangle of every delay problem with n <= 512 and of 8 seeded rectangles of
each larger one (48 nodes, one probe column).

screener_labels_n256.txt (with --screener): the SIM quadtree labels (child flags of
every split cell, three levels below [-4, 4]^2) of 16 held-out members of the n = 256
screener family.
"""
import os
import sys

import multiprocessing as mp

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
import oracle  # noqa: E402
from oracle import brute  # noqa: E402
from oracle import pmcima  # noqa: E402

_JOB = {}


def _single_thread():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _disk_indicator(args):
    """Oracle indicator sweep of one disk of the problem in _JOB (fork-shared)."""
    key, c, r = args
    prob, F, N = _JOB[key]
    sw = oracle.sweep_disk(prob, c, r, N, F, None)
    I, Iq = sw.indicator()
    rn = [oracle.norm2(sw.PfN[:, q]) / sw.scale[q] for q in range(F.shape[1])]
    rh = [oracle.norm2(sw.PfN2[:, q]) / sw.scale_half[q] for q in range(F.shape[1])]
    return I, Iq, rn, rh


def _pool(jobs, workers):
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_single_thread) as pool:
        return pool.map(_disk_indicator, jobs, chunksize=1)


def dense_sweep(workers=7):
    w = gen.workload_dense_qep(1024)
    _JOB["dense"] = (w.problems[0], w.F[0], w.opts.N)
    cov = oracle.cover(w.regions[0])
    res = _pool([("dense", d.c, d.r) for d in cov], workers)
    with open(os.path.join(HERE, "dense_qep_n1024_indicators.txt"), "w") as f:
        f.write("# Oracle indicator sweep of the dense n = 1024 QEP workload (K = A + A^T, C = 0.1 B,\n")
        f.write("# M = I + 0.1 G G^T, seeds 0, 1, 2; [-4, 4]^2 split 16 x 16, N = 32, F seed 3, s = 4):\n")
        f.write("# eq (3.1) per probe column with the rounding-noise floor, flag iff max_q I_q > 0.1.\n")
        f.write("# columns: disk flag I_q[0..3] |PfN_q|/S_N[0..3] |PfN2_q|/S_half[0..3]\n")
        f.write("# Written by tests/golden/make_golden.py --dense-sweep (oracle only).\n")
        for d, (I, Iq, rn, rh) in enumerate(res):
            f.write(f"{d} {int(I > w.opts.tol_ind)} " + " ".join(f"{v:.17e}" for v in list(Iq) + rn + rh) + "\n")


def delay(workers=7):
    w = gen.workload_delay(64)
    jobs, meta = [], []
    for p, prob in enumerate(w.problems):
        _JOB[p] = (prob, w.F[p], w.opts.N)
        cov = oracle.cover(w.regions[p])
        rects = range(len(cov)) if prob.n <= 512 else gen.delay_sampled_rectangles(p)
        for i in rects:
            jobs.append((p, cov[i].c, cov[i].r))
            meta.append((p, prob.n, i))
    # largest systems first so that the pool's tail is short
    order = sorted(range(len(jobs)), key=lambda k: -meta[k][1])
    out = _pool([jobs[k] for k in order], workers)
    res = [None] * len(jobs)
    for k, r in zip(order, out):
        res[k] = r
    with open(os.path.join(HERE, "delay_uneven_indicators.txt"), "w") as f:
        f.write("# Oracle indicators of the uneven delay family (64 problems T(z) = -z I + A0 + A1 exp(-tau z),\n")
        f.write("# n ~ U{128..2048}, tau ~ U[0.5, 2] from rng(40); [-3, 1] x [-6, 6] split 8 x 16, N = 48,\n")
        f.write("# F seed 2000 + p, s = 1): every rectangle of the problems with n <= 512, and the 8\n")
        f.write("# rectangles gen.delay_sampled_rectangles(p) of the larger ones.\n")
        f.write("# columns: problem n rectangle flag I |PfN|/S_N |PfN2|/S_half\n")
        f.write("# Written by tests/golden/make_golden.py --delay (oracle only).\n")
        for (p, n, i), (I, Iq, rn, rh) in zip(meta, res):
            f.write(f"{p} {n} {i} {int(I > w.opts.tol_ind)} {I:.17e} {rn[0]:.17e} {rh[0]:.17e}\n")


SCREENER_SAMPLE = [1600 + 25 * k for k in range(16)]


def _labels(p):
    prob = gen.screener_problem(p, 256)
    return pmcima.sim_quadtree_labels(prob, (-4.0, 4.0, -4.0, 4.0), 3, gen.probes(2, 256, 1), N=32)


def screener(workers=7):
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_single_thread) as pool:
        res = pool.map(_labels, SCREENER_SAMPLE, chunksize=1)
    with open(os.path.join(HERE, "screener_labels_n256.txt"), "w") as f:
        f.write("# SIM quadtree labels of held-out members of the n = 256 screener QEP family\n")
        f.write("# (gen.screener_problem(p), probe seed 2, N = 32, tol_ind 0.1, three levels below\n")
        f.write("# [-4, 4]^2, the root always split): one line per split cell.\n")
        f.write("# columns: problem level x0 x1 y0 y1 I[0..3] of its quadrants (cover order)\n")
        f.write("# Written by tests/golden/make_golden.py --screener (oracle only).\n")
        for p, recs in zip(SCREENER_SAMPLE, res):
            for level, cell, ind in recs:
                f.write(f"{p} {level} " + " ".join(f"{v:.17g}" for v in cell) + " "
                        + " ".join(f"{v:.17e}" for v in ind) + "\n")


def dense():
    w = gen.workload_dense_qep(1024)
    ev = brute.companion_eigs(w.problems[0])
    ev = ev[np.lexsort((ev.imag, ev.real))]
    with open(os.path.join(HERE, "dense_qep_n1024_eigs.txt"), "w") as f:
        f.write("# All 2n = 2048 eigenvalues of the dense n = 1024 QEP K + z C + z^2 M with\n")
        f.write("# K = A + A^T, C = 0.1 B, M = I + 0.1 G G^T (Gaussian entries / sqrt(n), seeds 0, 1, 2),\n")
        f.write("# from the companion pencil; columns: Re Im, sorted by (Re, Im).\n")
        f.write("# Written by tests/golden/make_golden.py --dense (oracle only).\n")
        for v in ev:
            f.write(f"{v.real:.17e} {v.imag:.17e}\n")


def small():
    w = gen.workload_small_qep()
    ev = brute.companion_eigs(w.problems[0])
    ev = ev[np.lexsort((ev.imag, ev.real))]
    with open(os.path.join(HERE, "small_qep_n64_eigs.txt"), "w") as f:
        f.write("# All 2n = 128 eigenvalues of the n = 64 QEP K + z C + z^2 I with K = A + A^T,\n")
        f.write("# C = 0.1 B (Gaussian entries / sqrt(n), seeds 0, 1), from the companion pencil;\n")
        f.write("# columns: Re Im, sorted by (Re, Im).  Written by tests/golden/make_golden.py (oracle only).\n")
        for v in ev:
            f.write(f"{v.real:.17e} {v.imag:.17e}\n")


def hankel():
    zs = np.concatenate([brute.hankel_zeros(m, 0.2, 3.2, -3.2, -0.2) for m in range(0, 11)])
    ms = np.concatenate([[m] * len(brute.hankel_zeros(m, 0.2, 3.2, -3.2, -0.2)) for m in range(0, 11)])
    with open(os.path.join(HERE, "hankel_zeros_scattering.txt"), "w") as f:
        f.write("# Zeros of H_m^(1) in [0.2, 3.2] x [-3.2, -0.2], m = 0..10 (each a double scattering pole of\n")
        f.write("# the sound-soft unit disk); columns: m Re Im.  Written by tests/golden/make_golden.py (oracle only).\n")
        for m, z in zip(ms, zs):
            f.write(f"{int(m)} {z.real:.17e} {z.imag:.17e}\n")


def main():
    if "--dense" in sys.argv:
        dense()
        return
    if "--dense-sweep" in sys.argv:
        dense_sweep()
        return
    if "--delay" in sys.argv:
        delay()
        return
    if "--screener" in sys.argv:
        screener()
        return
    small()
    hankel()
    p = gen.paper_demo_problem()
    ev = brute.companion_eigs(p)
    ev = np.sort(ev.real[np.argsort(ev.real)])
    with open(os.path.join(HERE, "paper_demo_qep.txt"), "w") as f:
        f.write("# Eigenvalues of the 4x4 quadratic of the paper's appendix (T0 + z T1 + z^2 T2,\n")
        f.write("# matrices as printed in the routine that generates T(z)); all 8 are real.\n")
        f.write("# Written by tests/golden/make_golden.py (companion linearisation, oracle only).\n")
        for v in ev:
            f.write(f"{v:.17e}\n")


if __name__ == "__main__":
    main()
