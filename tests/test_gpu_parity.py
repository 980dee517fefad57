"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on the
same seeded inputs.

Tolerances (derived in the design notes):
  * quadrature sums: ||gpu - oracle|| <= 1e-12 * S (complex128 LU) or 1e-11 * S
    (complex64 LU + complex128 refinement; raised to 4 * 2^-26 * kappa * u32, the
    refinement stopping rule's bound at the disk's worst-conditioned node, where that
    is larger), S = sum_j |w_j| ||X_j||, the size of the summands, because the sums of
    an empty disk cancel down to the quadrature error and a relative test on the sum
    itself would measure the cancellation, not the solver;
  * flags identical (disks with |I - tol_ind| <= 1e-6 tol_ind excluded, none occur);
  * verified eigenvalues: same count, each within 1e-10 (FP64) / 1e-8 (mixed)
    relative to the oracle's;
  * sigma_min: estimate >= true value (it is an upper bound by construction) and
    accept flags identical outside [tol/10, 10 tol].
"""
import os
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


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


def summand_scale(prob, dk, Nn, X_cols):
    z, w = oracle.nodes_weights(dk.c, dk.r, Nn)
    import scipy.linalg as sla
    tot = 0.0
    for j in range(Nn):
        x = sla.solve(oracle.assemble(prob, z[j]), X_cols)
        tot += abs(w[j]) * max(1.0, abs(z[j])) * np.linalg.norm(x)
    return tot


def refine_bound(prob, dk, Nn):
    # the mixed-precision stopping rule leaves an error below 2^-26 kappa u32 per node
    # (kappa = the node matrix's 2-norm condition number): four times that at the
    # worst node of the disk
    z, _ = oracle.nodes_weights(dk.c, dk.r, Nn)
    kappa = max(np.linalg.cond(oracle.assemble(prob, zj)) for zj in z)
    return 4.0 * 2.0 ** -26 * 2.0 ** -24 * kappa


def fp64_bound(prob, dk, Nn):
    # two backward-stable complex128 solves differ by about kappa u64 (kappa = the node
    # matrix's condition number, LAPACK's 1-norm estimate): eight times that at the
    # worst node of the disk
    from scipy.linalg import lapack
    z, _ = oracle.nodes_weights(dk.c, dk.r, Nn)
    kappa = 0.0
    for zj in z:
        T = oracle.assemble(prob, zj)
        lu, _, info = lapack.zgetrf(T)
        assert info == 0
        rc, _ = lapack.zgecon(lu, np.linalg.norm(T, 1), norm="1")
        kappa = max(kappa, 1.0 / rc)
    return 8.0 * 2.0 ** -53 * kappa


def check_sums(N, plan, prob, reg, opts, F, V, tol, disks=None):
    nd = plan.total_disks
    PfN, PfN2, C0, C1 = N.nep_copy_sums(plan, 0, nd)
    cov = oracle.cover(reg)
    for d in (range(nd) if disks is None else disks):
        dk = cov[d]
        sw = oracle.sweep_disk(prob, dk.c, dk.r, opts.N, F, V)
        B = F if V is None else np.concatenate([F, V], axis=1)
        S = summand_scale(prob, dk, opts.N, B)
        if opts.precision == 1:
            tol = max(tol, refine_bound(prob, dk, opts.N))
        assert np.linalg.norm(PfN[d] - sw.PfN) <= tol * S, (d, "PfN")
        assert np.linalg.norm(PfN2[d] - sw.PfN2) <= tol * S, (d, "PfN2")
        if V is not None:
            assert np.linalg.norm(C0[d] - sw.C0) <= tol * S, (d, "C0")
            assert np.linalg.norm(C1[d] - sw.C1) <= tol * S, (d, "C1")


# pivot 0 = partial pivoting, 1 = tournament (panels of > 128 rows go through the
# chunk/merge tree: n = 300 and 700 take one and two merge levels).  Panel kernels by
# rows: <= 128 in registers (<= 256 under tournament pivoting); <= 1024 recursive
# leaves of 8 columns in pairs; 1025 to
# 2048 in complex64 leaves of 16 columns, two rows per thread; more: the streaming
# panel (n = 1100, complex128; the largest orders below).  Orders >= 256 with <= 8
# columns take the step-parallel solve; orders >= 512 with 9 to 32 columns the
# step-parallel solve with its row tiles on the matrix cores (m = 12: one 16-column
# block; 20, 29 and 32: two; n = 600, 777 and 1030 end in a ragged block).
@pytest.mark.parametrize("n,Nn,s,L,prec,pivot", [(4, 8, 1, 2, 0, 0), (37, 8, 1, 4, 0, 0), (100, 16, 2, 6, 0, 0),
                                                 (600, 8, 4, 8, 0, 0), (777, 8, 4, 16, 1, 0),
                                                 (1030, 4, 3, 26, 0, 0), (520, 8, 2, 30, 1, 0),
                                                 (200, 16, 1, 8, 0, 0), (200, 16, 1, 8, 1, 0),
                                                 (130, 12, 3, 5, 1, 0), (300, 8, 1, 4, 0, 0), (700, 8, 1, 4, 1, 0),
                                                 (4, 8, 1, 2, 0, 1), (200, 16, 1, 8, 0, 1), (130, 12, 3, 5, 1, 1),
                                                 (300, 8, 1, 4, 0, 1), (700, 8, 1, 4, 1, 1),
                                                 (1100, 4, 1, 2, 0, 0), (1100, 4, 1, 2, 1, 0)])
def test_sums_ragged_sizes(N, n, Nn, s, L, prec, pivot):
    say(f"case sums n={n} N={Nn} s={s} L={L} precision={prec} pivot={pivot}")
    A = gen.gaussian(100 + n, n)
    B = gen.gaussian(200 + n, n)
    prob = gen.qep(A + A.T, 0.1 * B, None)
    reg = gen.Region(-1.0, 1.0, -0.5, 0.5, 2, 1)
    opts = gen.Options(N=Nn, s=s, L=L, precision=prec, pivot=pivot)
    F, V = gen.probes(1, n, s), gen.probes(2, n, L)
    plan = N.nep_plan([prob], [reg], opts)
    try:
        ind, flags, prof, st = N.nep_indicator(plan, [F], [V], want_profiles=True)
        assert st in (0, 2)
        check_sums(N, plan, prob, reg, opts, F, V, 1e-12 if prec == 0 else 1e-11)
        for d, dk in enumerate(oracle.cover(reg)):
            sw = oracle.sweep_disk(prob, dk.c, dk.r, Nn, F, None)
            I, Iq = sw.indicator()
            assert flags[d] == (I > opts.tol_ind)
            assert np.allclose(prof[d], sw.profile, rtol=1e-10 if prec == 0 else 1e-9)
    finally:
        N.nep_destroy(plan)


@pytest.mark.parametrize("n,prec", [(1600, 0), (2048, 0), (2048, 1), (3000, 1), (4096, 0)])
def test_largest_orders_sampled(N, n, prec):
    # up to the library's largest order: panels of more than 1024 (complex128) or 2048
    # (complex64) rows take the streaming panel; one disk of four nodes.  Orders from
    # 1600 on also keep many workgroups of the LDS-loaded updates in flight at once
    # (where waiting for the vector-memory count alone before a barrier gave wrong
    # sums now and then)
    say(f"case largest orders n={n} precision={prec}")
    A = gen.gaussian(100 + n, n)
    B = gen.gaussian(200 + n, n)
    prob = gen.qep(A + A.T, 0.1 * B, None)
    reg = gen.Region(-1.0, 1.0, -0.5, 0.5, 1, 1)
    opts = gen.Options(N=4, s=1, L=2, precision=prec)
    F, V = gen.probes(1, n, 1), gen.probes(2, n, 2)
    plan = N.nep_plan([prob], [reg], opts)
    try:
        _, _, _, st = N.nep_indicator(plan, [F], [V])
        assert st in (0, 2)
        # at these orders the rounding of either solver reaches the 1e-12 of the
        # smaller cases: the bound follows the node matrices' conditioning
        tol = max(1e-12, fp64_bound(prob, oracle.cover(reg)[0], opts.N)) if prec == 0 else 1e-11
        check_sums(N, plan, prob, reg, opts, F, V, tol)
    finally:
        N.nep_destroy(plan)


def test_small_workload_flags_indicators(N):
    w = gen.workload_small_qep()
    say("case small workload: n=64, 4x4 disks, N=32, s=1, L=8")
    plan = N.nep_plan(w.problems, w.regions, w.opts)
    try:
        ind, flags, prof, st = N.nep_indicator(plan, w.F, w.V, want_profiles=True)
        ref = oracle.pmcimb(w.problems[0], w.regions[0], w.opts, w.F[0], None)
        assert np.array_equal(flags, ref.flags)
        assert int(flags.sum()) == 12
        assert np.all(np.abs(ind[:, 0] - ref.ind) <= 1e-6 * np.maximum(ref.ind, 1.0))
        check_sums(N, plan, w.problems[0], w.regions[0], w.opts, w.F[0], w.V[0], 1e-12, disks=[0, 5, 10])
    finally:
        N.nep_destroy(plan)


def _eig_match(a, b, tol):
    a = np.asarray(a)
    b = np.asarray(b)
    assert len(a) == len(b), (len(a), len(b))
    for v in a:
        assert np.min(np.abs(b - v)) <= tol * max(1.0, abs(v)), v


@pytest.mark.parametrize("prec", [0, 1])
def test_small_workload_unsaturated_eigenvalues(N, prec):
    # the small workload with 31 Beyn columns: every flagged disk holds < 31 values
    w = gen.workload_small_qep()
    opts = gen.Options(N=32, s=1, L=31, precision=prec)
    V = gen.probes(3, 64, 31)
    say(f"case small workload L=31 precision={prec}")
    plan = N.nep_plan(w.problems, w.regions, opts)
    try:
        res = N.pmcimb(plan, w.F, [V])
        ref = oracle.pmcimb(w.problems[0], w.regions[0], opts, w.F[0], V)
        assert np.array_equal(res.flags, ref.flags)
        assert len(ref.eigs) > 60
        _eig_match(res.eigs, ref.eigs, 1e-10 if prec == 0 else 1e-8)
        # each verified value is an eigenvalue of the quadratic (companion pencil)
        from oracle import brute
        ev = brute.companion_eigs(w.problems[0])
        for v in res.eigs:   # accuracy of the N = 32 rule for values near the circles
            assert np.min(np.abs(ev - v)) < 1e-6 * max(1, abs(v))
    finally:
        N.nep_destroy(plan)


def test_paper_demo(N):
    ref = np.loadtxt(os.path.join(GOLD, "paper_demo_qep.txt"))
    prob = gen.paper_demo_problem()
    say("case paper demo: n=4, 9x9 disks, N=64, L=3")
    # n = 4 allows at most 4 probe columns (Beyn needs L <= n to be meaningful)
    opts = gen.Options(N=64, s=1, L=4)
    plan = N.nep_plan([prob], [gen.Region(-3, 3, -3, 3, 9, 9)], opts)
    try:
        res = N.pmcimb(plan, [gen.probes(11, 4, 1)], [gen.probes(12, 4, 4)])
        assert len(res.eigs) == 8
        assert np.max(np.abs(np.sort(res.eigs.real) - ref) / np.abs(ref)) < 1e-12
    finally:
        N.nep_destroy(plan)


def test_sigma_min_upper_bound_and_accept(N):
    w = gen.workload_small_qep()
    say("case sigma_min on the small workload's candidates")
    plan = N.nep_plan(w.problems, w.regions, w.opts)
    try:
        res = N.pmcimb(plan, w.F, w.V)
        assert len(res.cand) > 20
        ratios = []
        for lam, s, acc in zip(res.cand, res.sigma, res.accepted):
            ref = oracle.sigma_min(w.problems[0], lam)
            assert s >= ref * (1 - 1e-10)              # inverse iteration never undershoots
            assert acc == (ref < w.opts.tol_ver)        # same accept decision as the full SVD
            ratios.append(s / ref)
        # 4 iterations of inverse iteration on T^H T: close to the SVD value for most
        assert np.median(ratios) < 1.05 and np.max(ratios) < 2.0
        # exact eigenvalues give sigma ~ 0
        from oracle import brute
        ev = brute.companion_eigs(w.problems[0])[:6]
        sig, acc = N.nep_verify(plan, [0] * 6, ev)
        assert np.all(acc) and np.all(sig < 1e-10)
    finally:
        N.nep_destroy(plan)


def test_beyn_eigenvectors(N):
    # rotated diagonal quadratic with 3 roots inside one disk: vectors are null vectors
    n = 24
    rng = np.random.default_rng(4)
    a = np.concatenate([[0.1 + 0.05j, -0.2 - 0.1j, 0.05 - 0.2j], 3 + rng.uniform(0, 1, n - 3)])
    b = 5 + rng.uniform(0, 1, n) + 1j
    prob = gen.rotated_diagonal(a, 9, quadratic_partner=b)
    say("case Beyn eigenvectors: rotated diagonal n=24")
    opts = gen.Options(N=32, s=1, L=6)
    plan = N.nep_plan([prob], [gen.Region(-0.5, 0.5, -0.5, 0.5, 1, 1)], opts)
    try:
        import torch
        N.nep_indicator(plan, [gen.probes(1, n, 1)], [gen.probes(2, n, 6)])
        eig, p, sv, keep, vec, st = N.nep_beyn(plan, [0], want_vectors=True)
        assert p[0] == 3
        v = vec[0].cpu().numpy()
        got = sorted(eig[0, :3], key=lambda x: (x.real, x.imag))
        exp = sorted(a[:3], key=lambda x: (x.real, x.imag))
        assert np.max(np.abs(np.array(got) - np.array(exp))) < 1e-12
        for k in range(3):
            T = oracle.assemble(prob, eig[0, k])
            assert abs(np.linalg.norm(v[:, k]) - 1) < 1e-12
            assert np.linalg.norm(T @ v[:, k]) < 1e-10
    finally:
        N.nep_destroy(plan)


def test_uneven_delay_plan(N):
    # two delay problems of different order in one plan, against the oracle and the
    # Lambert-W roots of its scalar (rotated diagonal) member
    tau = 1.3
    a = np.array([-0.4, 0.1, -1.2, 0.3, -0.8])
    b = np.array([0.9, -0.5, 0.3, 0.2, -0.7])
    r2 = np.random.default_rng(21)
    Z = r2.standard_normal((5, 5)) + 1j * r2.standard_normal((5, 5))
    Q, _ = np.linalg.qr(Z)
    p0 = gen.delay(Q @ np.diag(a) @ Q.conj().T, Q @ np.diag(b) @ Q.conj().T, tau)
    p1 = gen.delay(gen.gaussian(3, 70), gen.gaussian(4, 70), 0.8)
    regs = [gen.Region(-1.5, 0.5, -1.0, 1.0, 2, 2), gen.Region(-3, 1, -2, 2, 2, 2)]
    opts = gen.Options(N=48, s=1, L=5)
    say("case uneven delay plan: n=5 and n=70")
    plan = N.nep_plan([p0, p1], regs, opts)
    try:
        F = [gen.probes(7, 5, 1), gen.probes(8, 70, 1)]
        V = [gen.probes(9, 5, 5), gen.probes(10, 70, 5)]
        ind, flags, _, st = N.nep_indicator(plan, F, V)
        for p, prob in enumerate([p0, p1]):
            off = N.lib().nep_disk_offset(plan.handle, p)
            ref = oracle.pmcimb(prob, regs[p], opts, F[p], V[p])
            assert np.array_equal(flags[off:off + 4], ref.flags)
        roots = np.concatenate([oracle.brute.delay_scalar_roots(a[i], b[i], tau, range(-3, 4)) for i in range(5)])
        dp = np.array([0] * 4 + [1] * 4, np.int32)
        fl = np.nonzero(flags[:4])[0]
        eig, p, sv, keep, _, _ = N.nep_beyn(plan, fl)
        found = [eig[i, k] for i in range(len(fl)) for k in range(p[i]) if keep[i, k]]
        sig, acc = N.nep_verify(plan, [0] * len(found), found)
        inside = roots[(roots.real >= -1.5) & (roots.real <= 0.5) & (np.abs(roots.imag) <= 1.0)]
        got = np.array(found)[acc]
        assert len(got) == len(inside)
        _eig_match(got, inside, 1e-9)
    finally:
        N.nep_destroy(plan)


@pytest.mark.parametrize("prec", [0, 1])
def test_singular_node_flags_disk(N, prec):
    # unrotated diagonal problem with a root exactly on node 1 of disk 0: exact zero pivot
    # (in complex64 too: the node and the root are the same double, so the assembled
    # entry is 0 before rounding; the complex128 re-solve meets the same zero pivot)
    n = 8
    r = float(np.hypot(1.0, 1.0))            # radius of the disk of the cell [-1,1]^2
    roots = np.array([r, 2.5, 3.0, 3.5, 4.0, 4.5, 5.0, 5.5], np.complex128)
    prob = gen.Problem(n, [np.ascontiguousarray(np.diag(-roots)), None], [gen.PHI_ONE, gen.PHI_Z])
    say(f"case singular node precision={prec}")
    opts = gen.Options(N=8, s=1, L=2, precision=prec)
    # disk 0: centre 0, radius sqrt(2) -> node 1 (theta = 0) at z = sqrt(2) hits the root
    reg = gen.Region(-1.0, 1.0, -1.0, 1.0, 1, 1)
    plan = N.nep_plan([prob], [reg], opts)
    try:
        ind, flags, _, st = N.nep_indicator(plan, [gen.probes(1, n, 1)], [gen.probes(2, n, 2)])
        assert st == N.NEP_WARN_SINGULAR_NODE
        assert flags[0]
        assert N.nep_get_stats(plan)["singular_nodes"] >= 1
    finally:
        N.nep_destroy(plan)


@pytest.mark.parametrize("scale", [1e160, 1e-160])
def test_scaled_coefficients(N, scale):
    # T scaled by 1e+-160 scales every solution and sum by the inverse; the indicator is a
    # ratio and must not change, although squares of the entries leave the double range
    n = 48
    A = gen.gaussian(120, n)
    base = gen.qep(A + A.T, 0.1 * gen.gaussian(121, n), None)
    reg = gen.Region(-4.0, 4.0, -3.0, 3.0, 4, 3)          # 8 flagged disks, 4 empty (I ~ 0.01)
    opts = gen.Options(N=16, s=2, L=0)
    F = gen.probes(122, n, 2)
    say(f"case coefficients scaled by {scale:g}")
    out = []
    for f in (1.0, scale):
        M = np.ascontiguousarray(f * np.eye(n, dtype=np.complex128))
        prob = gen.Problem(n, [f * base.coeffs[0], f * base.coeffs[1], M], base.phi_kind)
        plan = N.nep_plan([prob], [reg], opts)
        try:
            ind, flags, prof, st = N.nep_indicator(plan, [F], None, want_profiles=True)
            assert st == 0
            out.append((ind.copy(), flags.copy(), prof.copy()))
        finally:
            N.nep_destroy(plan)
    assert np.array_equal(out[0][1], out[1][1]) and out[0][1].any() and not out[0][1].all()
    # indicators: unchanged where resolved (empty disks under the floor report 0 both times)
    assert np.allclose(out[1][0], out[0][0], rtol=1e-9, atol=0)
    assert np.allclose(out[1][2] * scale, out[0][2], rtol=1e-10, atol=0)
    cov = oracle.cover(reg)
    for d in range(len(cov)):
        I, _ = oracle.sweep_disk(prob, cov[d].c, cov[d].r, opts.N, F, None).indicator()
        assert bool(out[1][1][d]) == (I > opts.tol_ind)


def test_sweep_is_deterministic(N):
    w = gen.workload_small_qep()
    say("case determinism")
    plan = N.nep_plan(w.problems, w.regions, w.opts)
    try:
        N.nep_indicator(plan, w.F, w.V)
        a = N.nep_copy_sums(plan, 0, plan.total_disks)
        N.nep_indicator(plan, w.F, w.V)
        b = N.nep_copy_sums(plan, 0, plan.total_disks)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    finally:
        N.nep_destroy(plan)
    # one or three worker streams and small batches give the same bits (batches are
    # independent)
    for streams, batch in ((1, 24), (3, 40)):
        o1 = gen.Options(N=32, s=1, L=8, streams=streams, batch=batch)
        plan = N.nep_plan(w.problems, w.regions, o1)
        try:
            N.nep_indicator(plan, w.F, w.V)
            c = N.nep_copy_sums(plan, 0, plan.total_disks)
            for x, y in zip(a, c):
                assert np.array_equal(x, y)
        finally:
            N.nep_destroy(plan)


def test_dense_workload_sampled(N):
    # the benchmark's configuration at full size (n = 1024, 16 x 16 disks, N = 32,
    # s = 4, L = 16), checked on two sampled disks that the oracle computes one by one
    w = gen.workload_dense_qep(1024)
    say("case dense workload n=1024 full sweep, 2 sampled disks")
    plan = N.nep_plan(w.problems, w.regions, w.opts)
    try:
        ind, flags, _, st = N.nep_indicator(plan, w.F, w.V)
        assert plan.total_disks == 256
        sample = [119, 0, 255, 15]   # next to the origin (flagged) and the four far corners
        check_sums(N, plan, w.problems[0], w.regions[0], w.opts, w.F[0], w.V[0], 1e-12, disks=sample[:2])
        cov = oracle.cover(w.regions[0])
        for d in sample:
            sw = oracle.sweep_disk(w.problems[0], cov[d].c, cov[d].r, 32, w.F[0], None)
            I, _ = sw.indicator()
            assert flags[d] == (I > 0.1)
    finally:
        N.nep_destroy(plan)


def test_results_do_not_depend_on_the_probes(N):
    """Flags and eigenvalues are properties of T (P f = 0 exactly when a disk holds no
    eigenvalue, for almost every probe): other probe draws give the same flags on the
    n = 64 workload, and with 31 Beyn columns the same verified eigenvalues (to the
    quadrature error; to rounding after refinement)."""
    w = gen.workload_small_qep()
    say("case probe independence")
    out = []
    for fs, vs in ((2, 3), (20, 30)):
        o = gen.Options(N=32, s=1, L=31)
        plan = N.nep_plan(w.problems, w.regions, o)
        try:
            res = N.pmcimb(plan, [gen.probes(fs, 64, 1)], [gen.probes(vs, 64, 31)])
            lam, sig, acc, _ = N.nep_refine(plan, [0] * len(res.eigs), res.eigs, 2)
            out.append((res.flags, np.sort_complex(res.eigs), np.sort_complex(lam)))
        finally:
            N.nep_destroy(plan)
    assert np.array_equal(out[0][0], out[1][0])
    a, b = out[0][1], out[1][1]
    assert len(a) == len(b) and len(a) > 20
    assert max(np.min(np.abs(b - v)) for v in a) < 1e-5
    ra, rb = out[0][2], out[1][2]
    assert max(np.min(np.abs(rb - v)) / max(1, abs(v)) for v in ra) < 1e-12


def test_update_timers(N):
    # the paired update's event timers: on one stream the launches cannot overlap, so
    # the union of their intervals is their sum; on two streams it lies between half
    # the sum and the sum
    n = 600
    A = gen.gaussian(610, n)
    prob = gen.qep(A + A.T, 0.1 * gen.gaussian(611, n), None)
    reg = gen.Region(-1.0, 1.0, -1.0, 1.0, 2, 2)
    F, V = gen.probes(612, n, 1), gen.probes(613, n, 4)
    say("case update timers n=600, one and two streams")
    for streams in (1, 2):
        plan = N.nep_plan([prob], [reg], gen.Options(N=16, s=1, L=4, streams=streams, batch=16))
        try:
            N.nep_indicator(plan, [F], [V])
            st = N.nep_get_stats(plan)
        finally:
            N.nep_destroy(plan)
        # 64 node solves in 4 batches, 4 pairs of panels each (n = 600: k0 = 0, 128, 256, 384)
        assert st["gemm_launches"] == 16 and st["gemm_flops"] > 0
        tot, busy = st["ms_gemm"], st["ms_gemm_busy"]
        assert 0 < busy <= tot * (1 + 1e-4) + 1e-3
        if streams == 1:
            assert busy >= tot * (1 - 1e-4) - 1e-3
        else:
            assert busy >= 0.5 * tot - 1e-3
