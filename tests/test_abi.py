"""CPU-side checks of the C ABI: the library loads, exports every entry point that
include/nep.h declares, rejects invalid arguments before touching a device, and its
host-only merge routine behaves.  No compute calls (no GPU here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nep.h")


def _lib():
    from paper_2312_13117_amd import nep as N
    if not os.path.exists(N.LIB_PATH):
        pytest.skip("libnep.so not built")
    return N, N.lib()


def test_header_symbols_exported():
    N, L = _lib()
    text = open(HEADER).read()
    names = sorted(set(re.findall(r"\b(nep_[a-z_]+)\s*\(", text)))
    assert "nep_plan" in names and "nep_indicator" in names and "nep_beyn" in names and "nep_verify" in names
    for name in names:
        assert hasattr(L, name), f"{name} declared in nep.h but not exported"


def test_plan_rejects_bad_options():
    N, L = _lib()
    import gen
    prob = N.nep_problem(16, 1, None, None, None)
    reg = N.nep_region(-1, 1, -1, 1, 2, 2)
    h = C.c_void_p()
    for o in (gen.Options(N=7), gen.Options(N=2), gen.Options(s=0), gen.Options(L=40), gen.Options(precision=5),
              gen.Options(max_refine=-1), gen.Options(tol_ind=float("nan")), gen.Options(streams=4),
              gen.Options(pivot=2), gen.Options(graph=2)):
        co = N.nep_options(o.N, o.s, o.L, o.tol_ind, o.tol_svd, o.tol_ver, o.precision, o.max_refine, o.batch,
                           o.streams, o.pivot, o.graph)
        st = L.nep_plan(C.byref(prob), 1, C.byref(reg), C.byref(co), None, C.byref(h))
        assert st == -1 and not h.value
        assert L.nep_last_error(None).decode()
    # null arguments and a bad region
    co = N.nep_options(32, 1, 8, 0.1, 1e-6, 1e-6, 0, 3, 0, 0, 0, 0)
    assert L.nep_plan(None, 1, C.byref(reg), C.byref(co), None, C.byref(h)) == -1
    kinds = (C.c_int * 1)(0)
    ptrs = (C.c_void_p * 1)(None)
    prob = N.nep_problem(16, 1, ptrs, kinds, None)
    bad = N.nep_region(1, -1, -1, 1, 2, 2)
    assert L.nep_plan(C.byref(prob), 1, C.byref(bad), C.byref(co), None, C.byref(h)) == -1
    prob_big = N.nep_problem(5000, 1, ptrs, kinds, None)
    assert L.nep_plan(C.byref(prob_big), 1, C.byref(reg), C.byref(co), None, C.byref(h)) == -1
    # a problem without split terms (assembled by a caller function) needs complex128
    co_mixed = N.nep_options(32, 1, 8, 0.1, 1e-6, 1e-6, 1, 3, 0, 0, 0, 0)
    assert L.nep_plan(C.byref(N.nep_problem(16, 0, None, None, None)), 1, C.byref(reg), C.byref(co_mixed), None,
                      C.byref(h)) == -1
    assert "NEP_FP64" in L.nep_last_error(None).decode()
    kinds_bad = (C.c_int * 1)(9)
    assert L.nep_plan(C.byref(N.nep_problem(16, 1, ptrs, kinds_bad, None)), 1, C.byref(reg), C.byref(co), None,
                      C.byref(h)) == -1


def test_null_plan_calls():
    N, L = _lib()
    assert L.nep_indicator(None, None, None, None, None, None) == -1
    assert L.nep_verify(None, None, None, 0, None, None) == -1
    assert L.nep_refine(None, None, None, 0, 2, None, None, None, 0) == -1
    assert L.nep_set_assembler(None, 0, None, None) == -1
    # the shipped assembler rejects a missing context or a wrong order without launching
    assert L.nep_assemble_elementwise_delay(None, 4, None, 1, None, 16, None) != 0
    ctx = N.nep_elementwise_delay(4, None, None, None)
    assert L.nep_assemble_elementwise_delay(C.byref(ctx), 4, None, 1, None, 16, None) != 0
    assert L.nep_total_disks(None) == 0
    L.nep_destroy(None)
    for s in (0, 1, 2, 3, -1, -2, -3, -4, -5, -6, 99):
        assert L.nep_status_str(s)


def test_dedup_keeps_smaller_sigma():
    N, L = _lib()
    lam = np.array([1.0 + 0j, 1.0 + 5e-9j, 2.0, 2.0 + 1e-3j, -3.0 + 1e-12j], np.complex128)
    sig = np.array([1e-9, 1e-12, 1e-10, 1e-10, 1e-11])
    keep = N.nep_dedup(lam, sig, 1e-8)
    assert keep.tolist() == [False, True, True, True, True]
    assert N.nep_dedup(np.zeros(0, np.complex128), np.zeros(0)).shape == (0,)


def test_merge_matches_the_oracle_merge():
    # pmCIMa's merge (Section 3.1): star groups in list order, means summed in list order
    N, L = _lib()
    from oracle import pmcima as opm
    rng = np.random.default_rng(5)
    base = rng.uniform(-1, 1, 12) + 1j * rng.uniform(-1, 1, 12)
    z = np.concatenate([base + 3e-7 * (rng.uniform(-1, 1, 12) + 1j * rng.uniform(-1, 1, 12)) for _ in range(4)])
    z = z[rng.permutation(len(z))]
    got, grp = N.nep_merge(z, 1e-6)
    want = opm.merge(z, 1e-6)
    assert len(got) == len(want) == 12
    assert np.array_equal(got, want)                       # same sums in the same order
    for k in range(len(got)):
        assert np.all(np.abs(z[grp == k] - z[np.argmax(grp == k)]) < 1e-6)
    assert N.nep_merge(np.zeros(0, np.complex128), 1e-6)[0].shape == (0,)


def test_ownership_across_cells_of_different_sizes():
    N, L = _lib()
    big = (0.0, 1.0, 0.0, 1.0)                 # a level-0 cell
    s1 = (1.0, 1.5, 0.0, 0.5)                  # two children of its right neighbour
    s2 = (1.0, 1.5, 0.5, 1.0)
    cells = [big, s1, big, s1, s2, s2, big]
    lam = np.array([0.5 + 0.5j,                # inside big: kept
                    1.0 + 0.25j,               # on the edge big | s1, produced by s1: big owns it
                    1.0 + 0.25j,               # the same value produced by big: kept
                    1.2 + 0.5j,                # on the edge s1 | s2, produced by s1: s1 comes first
                    1.2 + 0.5j,                # produced by s2: dropped
                    1.3 + 0.7j,                # inside s2: kept
                    2.0 + 0.0j], np.complex128)  # outside every cell: dropped
    keep = N.nep_own(np.asarray(cells), lam)
    assert keep.tolist() == [True, False, True, True, False, True, False]
    # within the band of an edge counts as on it
    keep = N.nep_own(np.asarray([s1, big]), np.array([1.0 + 5e-7 + 0.25j, 1.0 + 5e-7 + 0.25j]))
    assert keep.tolist() == [False, True]
