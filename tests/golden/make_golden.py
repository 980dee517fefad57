"""Writes the stored expected values under tests/golden/ from the oracle only.

paper_demo_qep.txt: the 4x4 quadratic printed in the paper's appendix routine that
generates T(z) (T2 = diag(3,1,3,1), T1, T0 as printed there), and its 8 eigenvalues
from the companion linearisation (a library generalized eigensolver).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
from oracle import brute  # noqa: E402


def main():
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
