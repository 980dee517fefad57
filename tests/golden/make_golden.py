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
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
from oracle import brute  # noqa: E402


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
