"""Graph mode of the indicator sweep: the captured HIP graph, replayed several times
with the program's own eager GPU work and synchronisations between the replays,
gives the eager path's results bit for bit (flags, indicators, profiles and the
four quadrature sums), also when the mixed-precision refinement asks for complex128
re-solves after the replay, and on a plan of uneven problem sizes."""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def N():
    import torch
    assert torch.cuda.is_available()
    from paper_2312_13117_amd import nep
    nep.lib()
    return nep


def _run(N, problems, regions, opts, F, V, calls):
    import torch
    plan = N.nep_plan(problems, regions, opts)
    outs = []
    try:
        for c in range(calls):
            ind, flags, prof, st = N.nep_indicator(plan, F, V, want_profiles=True)
            sums = N.nep_copy_sums(plan, 0, plan.total_disks)
            outs.append((ind, flags, prof, st, sums, N.nep_get_stats(plan)))
            # eager work of the program between replays
            x = torch.randn(1 << 20, device="cuda")
            (x * 2 + 1).sum().item()
            torch.cuda.synchronize()
    finally:
        N.nep_destroy(plan)
    return outs


def _same(a, b):
    ia, fa, pa, sa, ua, _ = a
    ib, fb, pb, sb, ub, _ = b
    assert sa == sb
    assert np.array_equal(fa, fb)
    assert np.array_equal(ia, ib)
    assert np.array_equal(pa, pb)
    for x, y in zip(ua, ub):
        if x is None:
            assert y is None
        elif isinstance(x, list):     # multi-problem plan: one array per disk
            assert len(x) == len(y) and all(np.array_equal(u, v) for u, v in zip(x, y))
        else:
            assert np.array_equal(x, y)


@pytest.mark.parametrize("prec,max_refine", [(0, 3), (1, 3), (1, 0)])
def test_graph_replays_equal_eager(N, prec, max_refine):
    say(f"case graph small workload precision={prec} max_refine={max_refine}")
    w = gen.workload_small_qep()
    base = dict(N=32, s=1, L=8, precision=prec, max_refine=max_refine)
    eager = _run(N, w.problems, w.regions, gen.Options(**base), w.F, w.V, 1)[0]
    reps = _run(N, w.problems, w.regions, gen.Options(**base, graph=1), w.F, w.V, 3)
    for r in reps:
        _same(eager, r)
    if prec == 1 and max_refine == 0:
        # no refinement sweeps: every node takes the complex128 re-solve (gathered in
        # batches of 32), which must give the complex128 sweep's bits
        assert eager[3] == N.NEP_WARN_REFINE_FALLBACK
        assert all(r[5]["refine_fallbacks"] == 16 * 32 for r in reps)
        fp64 = _run(N, w.problems, w.regions, gen.Options(N=32, s=1, L=8, precision=0), w.F, w.V, 1)[0]
        assert np.array_equal(fp64[1], eager[1])
        for x, y in zip(fp64[4], eager[4]):
            assert np.array_equal(x, y)


def test_graph_uneven_plan_and_beyn_between(N):
    # three delay problems of different orders in one plan (largest-first issue
    # order); a Beyn re-sweep of two disks between replays rewrites the shared
    # layout buffers, which every replay uploads again
    say("case graph uneven delay plan")
    probs = gen.delay_family(3, sizes=(200, 96, 64))     # orders 96, 64, 200: reordered
    say("  orders", [p.n for p in probs])
    regs = [gen.Region(-3.0, 1.0, -6.0, 6.0, 2, 4)] * 3
    F = [gen.probes(2000 + i, p.n, 1) for i, p in enumerate(probs)]
    V = [gen.probes(70 + i, p.n, 4) for i, p in enumerate(probs)]
    opts = dict(N=16, s=1, L=4, precision=1)
    eager = _run(N, probs, regs, gen.Options(**opts), F, V, 1)[0]
    plan = N.nep_plan(probs, regs, gen.Options(**opts, graph=1))
    try:
        a = N.nep_indicator(plan, F, V, want_profiles=True)
        sa = N.nep_copy_sums(plan, 0, plan.total_disks)
        N.nep_beyn(plan, np.array([0, 3], dtype=np.int32), V)
        b = N.nep_indicator(plan, F, V, want_profiles=True)
        sb = N.nep_copy_sums(plan, 0, plan.total_disks)
        for out, sums in ((a, sa), (b, sb)):
            _same(eager, (*out, sums, None))
    finally:
        N.nep_destroy(plan)
