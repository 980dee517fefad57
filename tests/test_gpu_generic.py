"""A problem without a short split form through the whole path: the elementwise delay
T(z) = -z I + A0 + A1 .* exp(-tau .* z), written at every node by the library's
nep_assemble_elementwise_delay (registered with nep_set_assembler), against the
oracle's entry-by-entry T(z): sums, flags, verified eigenvalues, graph replays, and
the argument checks of problems without split terms."""
import numpy as np
import pytest

import gen
import oracle
from test_gpu_parity import check_sums, say, _eig_match

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def N():
    import torch
    assert torch.cuda.is_available()
    from paper_2312_13117_amd import nep
    nep.lib()
    return nep


# orders through the register panel (37), the recursive panel (300, one workgroup per
# matrix and the step-parallel solve) and several batches
@pytest.mark.parametrize("n,Nn,s,L", [(5, 8, 1, 2), (37, 16, 2, 4), (300, 8, 1, 4)])
def test_sums_elementwise_delay(N, n, Nn, s, L):
    say(f"case elementwise delay sums n={n} N={Nn} s={s} L={L}")
    prob = gen.elementwise_delay(n, seed=300 + n)
    reg = gen.Region(-1.5, 0.5, -1.0, 1.0, 2, 2)
    opts = gen.Options(N=Nn, s=s, L=L)
    F, V = gen.probes(1, n, s), gen.probes(2, n, L)
    plan = N.nep_plan([prob], [reg], opts)
    try:
        ind, flags, _, st = N.nep_indicator(plan, [F], [V])
        assert st in (0, 2)
        check_sums(N, plan, prob, reg, opts, F, V, 1e-12)
        ref = oracle.pmcimb(prob, reg, opts, F, None)
        assert np.array_equal(flags, ref.flags)
    finally:
        N.nep_destroy(plan)


def test_pmcimb_elementwise_delay_matches_oracle(N):
    n = 40
    prob = gen.elementwise_delay(n, seed=410)
    reg = gen.Region(-2.0, 1.0, -3.0, 3.0, 3, 6)
    opts = gen.Options(N=32, s=1, L=12)
    F, V = gen.probes(3, n, 1), gen.probes(4, n, 12)
    say(f"case pmcimb elementwise delay n={n}")
    ref = oracle.pmcimb(prob, reg, opts, F, V)
    plan = N.nep_plan([prob], [reg], opts)
    try:
        res = N.pmcimb(plan, [F], [V])
        assert np.array_equal(res.flags, ref.flags)
        say(f"  {int(ref.flags.sum())} flagged, {len(ref.eigs)} verified eigenvalues")
        assert len(ref.eigs) >= 3
        _eig_match(res.eigs, ref.eigs, 1e-10)
        # verification works on an assembled problem; refinement needs the split form
        sig, acc = N.nep_verify(plan, [0] * len(ref.eigs), ref.eigs)
        assert np.all(acc) and np.all(sig < opts.tol_ver)
        for l, sv in zip(ref.eigs, sig):              # the estimate never undershoots sigma_min
            assert sv >= oracle.sigma_min(prob, l) * (1 - 1e-8)
        with pytest.raises(N.NepError):
            N.nep_refine(plan, [0], ref.eigs[:1], 2)
        lam, sg, ac, vec = N.nep_refine(plan, [0] * len(ref.eigs), ref.eigs, 0, want_vectors=True)
        assert np.array_equal(sg, sig)
        for l, v, sv in zip(ref.eigs, vec, sg):
            # the right singular vector of sigma_min: ||T(lambda) v|| = sigma_min
            assert abs(np.linalg.norm(v[:n]) - 1) < 1e-12
            assert np.linalg.norm(oracle.assemble(prob, l) @ v[:n]) <= 1.05 * sv + 1e-14
    finally:
        N.nep_destroy(plan)


def test_graph_replay_with_assembler(N):
    n = 64
    prob = gen.elementwise_delay(n, seed=520)
    reg = gen.Region(-1.0, 1.0, -1.0, 1.0, 2, 2)
    F, V = gen.probes(5, n, 2), gen.probes(6, n, 4)
    say("case elementwise delay graph replay")
    out = []
    for graph in (0, 1):
        plan = N.nep_plan([prob], [reg], gen.Options(N=16, s=2, L=4, graph=graph))
        try:
            for _ in range(1 + graph):             # the second graph call replays
                N.nep_indicator(plan, [F], [V])
            out.append(N.nep_copy_sums(plan, 0, plan.total_disks))
        finally:
            N.nep_destroy(plan)
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def test_assembled_problem_needs_complex128(N):
    prob = gen.elementwise_delay(8, seed=600)
    with pytest.raises(N.NepError):
        N.nep_plan([prob], [gen.Region(-1, 1, -1, 1, 1, 1)], gen.Options(N=8, precision=1))


def test_dense_elementwise_delay_sampled(N):
    """n = 1024 over the delay workload's rectangle (8 x 16 cells, 48 nodes): two disks
    checked against the oracle in the plan's full launch configuration."""
    n = 1024
    prob = gen.elementwise_delay(n, seed=700)
    reg = gen.Region(-3.0, 1.0, -6.0, 6.0, 8, 16)
    opts = gen.Options(N=48, s=1, L=0)
    F = gen.probes(7, n, 1)
    say("case elementwise delay n=1024 sampled")
    plan = N.nep_plan([prob], [reg], opts)
    try:
        N.nep_indicator(plan, [F])
        check_sums(N, plan, prob, reg, opts, F, None, 1e-12, disks=[0, 77])
    finally:
        N.nep_destroy(plan)
