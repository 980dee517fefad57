"""Failure handling forced from the host (every kernel still runs to completion):
a non-finite coefficient flags every disk conservatively; a node 1e-10 from an
eigenvalue defeats complex64 refinement and is re-solved in complex128 (with a
warning, counted), giving the complex128 sweep's result; a workspace larger than the
device returns NEP_ERR_NOMEM without leaving a plan behind."""
import numpy as np
import pytest

import gen
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def N():
    import torch
    assert torch.cuda.is_available()
    from paper_2312_13117_amd import nep
    nep.lib()
    return nep


def test_nan_coefficient_flags_every_disk(N):
    say("case NaN in a coefficient")
    n = 24
    A = gen.gaussian(900, n)
    K = (A + A.T).astype(np.complex128)
    K[3, 5] = np.nan
    prob = gen.qep(K, 0.1 * gen.gaussian(901, n), None)
    reg = gen.Region(-1.0, 1.0, -1.0, 1.0, 2, 2)
    plan = N.nep_plan([prob], [reg], gen.Options(N=16, s=1, L=0))
    try:
        ind, flags, _, st = N.nep_indicator(plan, [gen.probes(902, n, 1)])
        assert st in (0, 1)
        assert flags.all()                     # a non-finite indicator flags its disk
    finally:
        N.nep_destroy(plan)


def test_node_next_to_an_eigenvalue_falls_back_to_complex128(N):
    n = 32
    reg = gen.Region(-1.0, 1.0, -1.0, 1.0, 1, 1)
    c, r = 0.0, np.hypot(1.0, 1.0)
    rng = np.random.default_rng(910)
    roots = 0.5 * (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n))
    roots[0] = c + r + 1e-10                   # 1e-10 outside node 1 (theta = 0)
    prob = gen.rotated_diagonal(roots, seed=911)
    F, V = gen.probes(912, n, 1), gen.probes(913, n, 4)
    say("case node 1e-10 from an eigenvalue, mixed precision")
    sums = {}
    for prec in (0, 1):
        plan = N.nep_plan([prob], [reg], gen.Options(N=16, s=1, L=4, precision=prec))
        try:
            _, _, _, st = N.nep_indicator(plan, [F], [V])
            stats = N.nep_get_stats(plan)
            sums[prec] = N.nep_copy_sums(plan, 0, 1)
        finally:
            N.nep_destroy(plan)
        if prec == 1:
            say(f"  status {st}, re-solved nodes {stats['refine_fallbacks']}")
            assert st == 2 and stats["refine_fallbacks"] >= 1
    for a, b in zip(sums[0], sums[1]):
        a, b = np.asarray(a), np.asarray(b)
        # the near-singular node dominates every sum and is identical in both runs
        assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(a)


def test_workspace_beyond_the_device_is_nomem(N):
    say("case workspace beyond device memory")
    import torch
    n = 4096
    total = torch.cuda.get_device_properties(0).total_memory
    batch = 2048                               # 2048 x 4096^2 x 16 B = 550 GB
    assert batch * n * n * 16 > 1.5 * total
    prob = gen.Problem(n, [None], [gen.PHI_NEG_Z])          # T(z) = -z I, nothing to upload
    reg = gen.Region(-1.0, 1.0, -1.0, 1.0, 8, 8)            # 64 disks x 32 nodes = 2048 tasks
    with pytest.raises(N.NepError) as e:
        N.nep_plan([prob], [reg], gen.Options(N=32, s=1, L=0, batch=batch))
    assert e.value.status == -2                             # NEP_ERR_NOMEM
