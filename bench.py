"""Benchmark of the pmCIMb quadrature sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dense|dense_mixed|small|delay]

A step is one pass of the whole path over the workload:
- assembly + LU + block solve + quadrature sums + indicators for every (disk, node);
- Beyn's extraction on the flagged disks;
- sigma_min verification of the kept candidates, then the merge.
Inputs are seeded synthetic matrices already resident in HBM when the timed region
starts.

Prints ONE JSON line.
- `value` = node solves per second of the whole step on the dense n = 1024 QEP in
  complex128.
- `mixed` = the same workload with complex64 LUs and complex128 refinement: its
  rate, speedup, and agreement with the complex128 sweep.
- `eigenpairs_unsaturated` = eigenpairs/s where the rank test is not cut by the probe
  count (the workload as configured saturates every flagged disk).
- `generic_assembly` = the whole step on a problem without a short split form (an
  elementwise delay, n = 1024, written at every node by an assembler callback).
- `scattering` = the paper's scattering-pole experiment (sound-soft unit disk, 100
  squares) by pmCIMb and pmCIMa, poles against the Hankel-function zeros.
- `pmcima` = pmCIMa (indicator levels down to tol_eps = 1e-6, merge, Step 2 vectors,
  then refinement) on the n = 64 workload: time, node solves and accuracy.
- `eigenpairs_complete` = the complete spectrum of the dense workload (2048
  eigenvalues) by the saturation remedy (cells split 2 x 2 until no flagged disk
  saturates, candidates refined and verified), complex128 and mixed sweeps: wall time,
  eigenpairs/s, and the worst relative error against the companion pencil stored
  under tests/golden/.
- `roofline` = the dominant kernel (trailing-update kernel of the batched LU). Its
  durations come from the library's own HIP events recorded on the stream the
  kernel runs on; the average launch duration is the union of the launches'
  intervals over their number (launches of the two worker streams may overlap).
- `delay_family` = the uneven delay family in full (64 problems, n 128..2048, 393,216
  node systems in one plan, complex64 + refinement): one pass.
- `screener` = the learned screener on the n = 256 family (2000 problems): miss rate,
  solves a skip policy would save, ordering gain.
- `peak_measured` = the matrix-core rate of the update's MFMA shape on this device.
- `cpu_baseline` = the FP64 CPU oracle on a bounded sample of the same workload, one
  single-threaded LAPACK worker per host core over disks.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12}


def build_workload(name: str, delay_count: int = 8, pivot: int = 0):
    w = _workload(name, delay_count)
    w.opts.pivot = pivot
    return w


def _workload(name: str, delay_count: int):
    import gen
    if name == "dense":
        return gen.workload_dense_qep(1024, precision=0)
    if name == "dense_mixed":
        return gen.workload_dense_qep(1024, precision=1)
    if name == "small":
        return gen.workload_small_qep()
    if name == "small_L31":
        w = gen.workload_small_qep()
        w.opts = gen.Options(N=32, s=1, L=31)
        w.V = [gen.probes(3, 64, 31)]
        w.name = "qep_n64_4x4_L31"
        return w
    if name == "delay":
        full = gen.workload_delay(64, precision=1)
        full.problems = full.problems[:delay_count]
        full.regions = full.regions[:delay_count]
        full.F = full.F[:delay_count]
        full.V = full.V[:delay_count]
        full.name = f"delay_uneven_first{delay_count}"
        return full
    raise SystemExit(f"unknown workload {name}")


class Runner:
    """Plan + device inputs for one workload; step() runs the whole path once."""

    def __init__(self, w):
        import torch
        from paper_2312_13117_amd import nep as N
        self.N, self.w = N, w
        self.plan = N.nep_plan(w.problems, w.regions, w.opts)
        self.F = [N._dev_complex(f, torch) for f in w.F]
        V = [N._dev_complex(v, torch) if v is not None else None for v in w.V]
        self.V = V if all(v is not None for v in V) else None
        self.disk_prob = np.zeros(self.plan.total_disks, np.int32)
        for p in range(len(w.problems)):
            first = N.lib().nep_disk_offset(self.plan.handle, p)
            last = N.lib().nep_disk_offset(self.plan.handle, p + 1) if p + 1 < len(w.problems) else \
                self.plan.total_disks
            self.disk_prob[first:last] = p

    def step(self):
        N = self.N
        ind, flags, _, _ = N.nep_indicator(self.plan, self.F, self.V)
        st = N.nep_get_stats(self.plan)
        flagged = np.nonzero(flags)[0]
        cand, cdisk = [], []
        if self.V is not None and len(flagged):
            eig, p, sv, keep, _, _ = N.nep_beyn(self.plan, flagged)
            for i, d in enumerate(flagged):
                for k in range(int(p[i])):
                    if keep[i, k]:
                        cand.append(eig[i, k])
                        cdisk.append(d)
        eigs = np.zeros(0, np.complex128)
        if cand:
            sig, acc = N.nep_verify(self.plan, self.disk_prob[np.asarray(cdisk)], cand)
            al = np.asarray(cand)[acc]
            if len(al):
                eigs = al[N.nep_dedup(al, sig[acc])]
        return {"flags": flags, "ind": ind, "ncand": len(cand), "eigs": eigs, "stats": st}

    def sums(self):
        if len(self.w.problems) != 1:
            return None
        return self.N.nep_copy_sums(self.plan, 0, self.plan.total_disks)

    def close(self):
        self.N.nep_destroy(self.plan)


VERBOSE = False


def _log(msg):
    if VERBOSE:
        print(msg, file=sys.stderr, flush=True)


def _progress(msg):
    """One stderr line per block of the benchmark (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def timed(runner, steps: int, warmup: int):
    import torch
    for i in range(warmup):
        t0 = time.perf_counter()
        runner.step()
        torch.cuda.synchronize()
        _log(f"{runner.w.name}: warm-up step {i + 1}/{warmup} {time.perf_counter() - t0:.2f} s")
    torch.cuda.synchronize()
    times, outs = [], []
    for i in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = runner.step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        outs.append(o)
        _log(f"{runner.w.name}: step {i + 1}/{steps} {times[-1]:.2f} s")
    k = int(np.argsort(times)[len(times) // 2])
    return float(np.median(times)), outs[k]


_CPU_JOB = {}


def _cpu_worker_init():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _cpu_disk(d):
    import oracle
    prob, reg, opts, F, V = _CPU_JOB["w"]
    dk = oracle.cover(reg)[d]
    t0 = time.perf_counter()
    oracle.sweep_disk(prob, dk.c, dk.r, opts.N, F, V)
    return time.perf_counter() - t0


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, disks_per_worker: int = 2):
    """The FP64 CPU oracle on a bounded sample of the same workload, the analogue of the
    paper's parfor over disks: one single-threaded LAPACK worker process per host core
    (the GPU machine's CPU share: OMP_NUM_THREADS, at most 16), each sweeping whole disks of
    problem 0.  Runs before the GPU is touched (the workers are forked)."""
    import multiprocessing as mp
    import oracle  # noqa: F401  (imported before the fork: the workers must not import scipy themselves)
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
    cores = max(1, min(cores, 16, os.cpu_count() or 1))
    prob, reg = w.problems[0], w.regions[0]
    _CPU_JOB["w"] = (prob, reg, w.opts, w.F[0], w.V[0])
    nd = reg.nx * reg.ny
    idx = np.linspace(0, nd - 1, min(nd, cores * disks_per_worker)).round().astype(int).tolist()
    ctx = mp.get_context("fork")
    with ctx.Pool(cores, initializer=_cpu_worker_init) as pool:
        pool.map(_cpu_disk, idx[:cores], chunksize=1)          # page in, start the pool
        t0 = time.perf_counter()
        per = pool.map(_cpu_disk, idx, chunksize=1)
        dt = time.perf_counter() - t0
    solves = len(idx) * w.opts.N
    nrhs = w.F[0].shape[1] + (0 if w.V[0] is None else w.V[0].shape[1])
    return {"value": solves / dt, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{len(idx)} disks x {w.opts.N} nodes of problem 0 (n={prob.n}, {nrhs} right-hand sides, "
                      f"complex128 LAPACK gesv per node), one single-threaded worker process per core over "
                      f"disks; {dt:.1f} s wall, {float(np.mean(per)):.2f} s per disk"}


def copy_calibration(nbytes: int = 1 << 30, reps: int = 3):
    """A plain device-to-device copy of `nbytes` (torch's copy kernel), for scaling
    the FETCH_SIZE / WRITE_SIZE counters of a profiled run to bytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps, "GBps": 2 * nbytes / dt / 1e9}


def golden_eigs(name: str):
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    a = np.loadtxt(path)
    return a[:, 0] + 1j * a[:, 1]


def _match_err(found, ref):
    """(worst relative error of found values against their nearest reference, whether
    the nearest references are all different)."""
    if ref is None or not len(found):
        return None, None
    d = np.abs(found[:, None] - ref[None, :])
    near = np.argmin(d, axis=1)
    err = float(np.max(d[np.arange(len(found)), near] / np.maximum(1.0, np.abs(ref[near]))))
    return err, bool(len(set(near.tolist())) == len(found))


def pmcima_run():
    """pmCIMa (Section 3.1) on the n = 64 workload's cover with N = 16, tol_eps = 1e-6,
    then two refinement updates: time, node solves, and accuracy of the merged and the
    refined values against the companion pencil."""
    import gen
    from paper_2312_13117_amd import pmcima
    w = gen.workload_small_qep()
    ref = golden_eigs("small_qep_n64_eigs.txt")
    run = lambda: pmcima.pmcima(w.problems[0], w.regions[0], w.F[0], refine_iters=2)
    run()
    r = run()
    e_m, _ = _match_err(r.eigs, ref)
    e_r, one = _match_err(r.refined, ref)
    return {"workload": "qep_n64_4x4_pmcima_N16_tol1e-6", "levels": r.levels,
            "disks": int(sum(len(d) for d in r.disks)), "node_solves": int(r.node_solves), "seconds": r.seconds,
            "solves_per_s": r.node_solves / r.seconds, "merged_values": int(len(r.eigs)),
            "max_rel_err_merged": e_m, "refined_eigenpairs": int(len(r.refined)), "max_rel_err_refined": e_r,
            "refined_one_to_one": one, "eigenpairs_per_s": len(r.refined) / r.seconds}


def generic_run(steps: int):
    """A problem without a short split form: the elementwise delay T(z) = -zI + A0 +
    A1 .* exp(-tau .* z) at n = 1024 over the delay workload's rectangle (8 x 16 cells,
    48 nodes, s = 1, L = 8), assembled at every node by the library's assembler
    callback: the whole pmCIMb step in complex128."""
    import gen
    prob = gen.elementwise_delay(1024, seed=700)
    w = gen.Workload("elementwise_delay_n1024_8x16", [prob], [gen.Region(-3.0, 1.0, -6.0, 6.0, 8, 16)],
                     gen.Options(N=48, s=1, L=8), [gen.probes(7, 1024, 1)], [gen.probes(8, 1024, 8)])
    r = Runner(w)
    T, o = timed(r, steps, 1)
    r.close()
    st = o["stats"]
    return {"workload": w.name, "value": st["node_solves"] / T, "unit": "solves/s", "ms_per_step": T * 1e3,
            "flagged_disks": int(np.sum(o["flags"])), "verified_eigenpairs": int(len(o["eigs"])),
            "phase_ms": phase_dict(st)}


def scattering_run():
    """Scattering poles of the sound-soft unit disk (the paper's second experiment, with
    a self-written discretisation: the double-layer Nystrom matrix on 64 points of the
    circle, assembled on the device): pmCIMb and pmCIMa over [0.2, 3.2] x [-3.2, -0.2]
    split into 100 squares, poles against the stored Hankel-function zeros."""
    import gen
    import torch
    from paper_2312_13117_amd import nep as N, pmcima
    a = np.loadtxt(os.path.join(ROOT, "tests", "golden", "hankel_zeros_scattering.txt"))
    ref = a[:, 1] + 1j * a[:, 2]
    prob = gen.CircleDoubleLayer(64)
    reg = gen.Region(0.2, 3.2, -3.2, -0.2, 10, 10)
    w = gen.Workload("scattering_unit_disk_10x10", [prob], [reg], gen.Options(N=32, s=1, L=4),
                     [gen.probes(11, 64, 1)], [gen.probes(12, 64, 4)])
    r = Runner(w)
    T, o = timed(r, 3, 1)
    r.close()
    e_b, one_b = _match_err(o["eigs"], ref)
    pmcima.pmcima(prob, reg, w.F[0])
    torch.cuda.synchronize()
    pa = pmcima.pmcima(prob, reg, w.F[0])
    e_a, _ = _match_err(pa.eigs, ref)
    return {"workload": w.name, "hankel_zeros": int(len(ref)),
            "pmcimb": {"ms_per_step": T * 1e3, "poles": int(len(o["eigs"])), "max_rel_err": e_b,
                       "one_to_one": one_b, "node_solves": int(o["stats"]["node_solves"])},
            "pmcima": {"seconds": pa.seconds, "poles": int(len(pa.eigs)), "max_rel_err": e_a,
                       "levels": pa.levels, "node_solves": int(pa.node_solves)}}


def complete_spectrum(pivot: int, reps: int = 2):
    """The saturation remedy on the dense workload (cells split until no flagged disk
    saturates, candidates refined and verified): eigenpairs/s of the complete spectrum
    and the worst relative error against the companion pencil, per precision."""
    import torch
    from paper_2312_13117_amd import adaptive
    ref = golden_eigs("dense_qep_n1024_eigs.txt")
    res = {}
    for tag, precision in (("fp64", 0), ("mixed", 1)):
        w = build_workload("dense" if precision == 0 else "dense_mixed", pivot=pivot)
        run = lambda: adaptive.pmcimb_adaptive(w.problems[0], w.regions[0], w.opts, w.F[0], w.V[0], max_depth=8)
        ts, r = [], None                  # the library is warm from the sweep benchmark
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = run()
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        e = {"eigenpairs": int(len(r.eigs)), "seconds": t, "eigenpairs_per_s": len(r.eigs) / t,
             "node_solves": int(r.node_solves), "levels": r.levels, "disks_swept": r.disks_swept,
             "unresolved": r.unresolved}
        if ref is not None:
            e["max_rel_err_vs_companion"], e["one_to_one"] = _match_err(r.eigs, ref)
            e["companion_eigenvalues"] = int(len(ref))
            if len(r.eigs):
                # every eigenvalue's relative error against its nearest companion eigenvalue
                d = np.abs(r.eigs[:, None] - ref[None, :])
                near = np.argmin(d, axis=1)
                err = d[np.arange(len(r.eigs)), near] / np.maximum(1.0, np.abs(ref[near]))
                e["rel_err_quantiles"] = {q: float(np.quantile(err, float(q))) for q in ("0.5", "0.9", "0.99", "1.0")}
                e["eigenvalues_above_1e-8"] = int(np.sum(err > 1e-8))
        res[tag] = e
        _log(f"complete spectrum {tag}: {e}")
    res["speedup_mixed_vs_fp64"] = res["fp64"]["seconds"] / res["mixed"]["seconds"]
    return res


def delay_run():
    """The uneven delay family in full: 64 problems T(z) = -z I + A0 + A1 exp(-tau z) with
    n drawn from {128, ..., 2048}, 8 x 16 rectangles x 48 nodes each (393,216 node
    systems), complex64 LUs with complex128 refinement, all in one plan (largest n
    first over two worker streams); one pass after the other blocks warmed the kernels."""
    w = build_workload("delay", 64)
    r = Runner(w)
    T, o = timed(r, 1, 0)
    r.close()
    st = o["stats"]
    return {"workload": "delay_uneven_64problems_8x16_N48", "problems": len(w.problems),
            "n": sorted(set(p.n for p in w.problems)), "node_solves": int(st["node_solves"]), "seconds": T,
            "value": st["node_solves"] / T, "unit": "solves/s", "lu_pflop": st["lu_flops"] / 1e15,
            "lu_tflops_over_wall": st["lu_flops"] / T / 1e12,
            "lu_frac_of_fp32_peak_over_wall": st["lu_flops"] / T / PEAK["fp32"],
            "flagged_rectangles": int(np.sum(o["flags"])), "refine_sweeps": st["refine_sweeps"],
            "refine_fallbacks": st["refine_fallbacks"], "phase_ms_stream_summed": phase_dict(st)}


def screener_run():
    """The learned screener on the n = 256 QEP family: SIM labels of 2000 problems on a
    three-level quadtree (complex64 LUs with complex128 refinement), training on 1600,
    test metrics on 400 (miss rate against the method's own flags, child solves a skip
    policy would save, child evaluations until every positive child is screened in
    network order against raster and random order), the held-out problems screened in
    ranked rounds, and the labels of 400 problems again in complex128 (time, identity)."""
    from paper_2312_13117_amd import screener
    rep = screener.run(2000, 1600, 256, log=_log, precision=1, compare_fp64=400)
    t = rep["test"]
    return {"workload": "screener_qep_n256_2000problems_depth3", "label_solves": rep["dataset"]["solves"],
            "label_seconds": rep["dataset"]["seconds"], "train_seconds": rep["training"]["seconds"],
            "miss_rate": t["miss_rate"], "solves_saved": t["solves_saved"], "solves_total": t["solves_total"],
            "evals_until_all_positive": t["evals_until_all_positive"], "per_level": t["per_level"],
            "trivial_all_positive": rep["trivial_all_positive"],
            "label_precision": "complex64 + complex128 refinement",
            "labels_mixed_vs_fp64": rep["labels_mixed_vs_fp64"],
            "ranked_rounds": {o: {"seconds": v["seconds"],
                                  "positive_children_known_after_round": [lv["known_after_round"] for lv in v["levels"]],
                                  "mean_sweeps_until_all_positive": [lv["mean_sweeps_until_all_positive"]
                                                                     for lv in v["levels"]]}
                              for o, v in rep["ranked_rounds"].items()}}


def peak_measured():
    """The matrix-core rate of the update's MFMA shape on this device (TFLOP/s)."""
    from paper_2312_13117_amd import nep as N
    return {"fp64": N.nep_mfma_peak(N.NEP_FP64), "fp32": N.nep_mfma_peak(N.NEP_FP32_REFINE),
            "unit": "TFLOP/s", "kernel": "independent chains of the 16x16x4 MFMA, 1024 workgroups x 4 waves"}


def phase_dict(st):
    return {k: st[k] for k in ("ms_assemble", "ms_lu", "ms_solve", "ms_refine", "ms_sums", "ms_total")}


def measured_traffic(workload: str, prec: str, flops_per_launch: float = None):
    """HBM bytes per launch of the update kernel from the committed counter summary, or
    None when there is none for this workload and precision, the LU source has changed
    since, or the launches now have another shape (a different batch: flops per launch
    differ)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "lu_kernels_counters_dense_n1024.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    for block in text.split("```")[1::2]:
        kv = {}
        for line in block.splitlines():
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        try:
            if kv.get("workload") != workload or kv.get("precision") != prec:
                continue
            src = os.path.join(ROOT, kv["kernel_source"])
            if hashlib.sha256(open(src, "rb").read()).hexdigest() != kv["kernel_source_sha256"]:
                return None
            if flops_per_launch is not None and \
                    abs(float(kv["flops_per_launch"]) - flops_per_launch) > 0.005 * flops_per_launch:
                return None
            return float(kv["traffic_bytes_per_launch"])
        except (OSError, KeyError, ValueError):
            return None
    return None


def roofline(st, prec, workload=None):
    # The worker streams' update launches can run at the same time; each launch's own
    # event interval then includes the time it shares the CUs with the other one, and
    # the kernel's rate is its flops over the time any of its launches runs (the union
    # of the intervals), which equals the plain sum when no two launches overlap.
    busy = st["ms_gemm_busy"]
    achieved = st["gemm_flops"] / (busy * 1e-3) if busy > 0 else 0.0
    fpl = st["gemm_flops"] / max(1, st["gemm_launches"])
    traffic = measured_traffic(workload, prec, fpl) if workload else None
    # complex128 products are formed from 3 real products (3M): the matrix cores execute
    # 6 of the 8 credited flops per complex multiply-add; complex64 uses all 4 (8 of 8)
    executed = 0.75 if prec == "fp64" else 1.0
    return {"kernel": "lu_gemm_dma_kernel<UPDATE2> (trailing update of the batched LU, two panels per pass, K = 128, operands loaded straight into LDS)",
            "bound": "mfma",
            "achieved": achieved / 1e12, "peak": PEAK[prec] / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK[prec], "traffic": traffic, "traffic_unit": "bytes per launch (HBM, counters)",
            "executed_frac": executed * achieved / PEAK[prec],
            "credit": "8 real flops per complex multiply-add" + (" (3M: 6 executed)" if prec == "fp64" else ""),
            "launches": st["gemm_launches"],
            "avg_launch_ms": busy / max(1, st["gemm_launches"]),
            "avg_launch_ms_own_interval": st["ms_gemm"] / max(1, st["gemm_launches"]),
            "flops_per_launch": st["gemm_flops"] / max(1, st["gemm_launches"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="dense")
    ap.add_argument("--delay-count", type=int, default=8)
    ap.add_argument("--cpu-disks-per-core", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-eigen", action="store_true")
    ap.add_argument("--no-delay", action="store_true", help="skip the full delay-family pass")
    ap.add_argument("--no-screener", action="store_true", help="skip the screener block")
    ap.add_argument("--precision", choices=("default", "fp64", "mixed"), default="default",
                    help="override the workload's LU arithmetic (complex128, or complex64 + refinement)")
    ap.add_argument("--graph", action="store_true",
                    help="capture the indicator sweep in a HIP graph on its first call and replay it")
    ap.add_argument("--pivot", choices=("partial", "tournament"), default="partial",
                    help="pivot choice of the node LU panels")
    ap.add_argument("--verbose", action="store_true", help="one stderr line per step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and print its sizes")
    args = ap.parse_args()
    global VERBOSE
    VERBOSE = args.verbose
    pivot = 0 if args.pivot == "partial" else 1
    if args.copy_calibration:
        print(json.dumps(copy_calibration()))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    w = build_workload(args.workload, args.delay_count, pivot)
    w.opts.graph = 1 if args.graph else 0
    if args.precision != "default":
        w.opts.precision = 0 if args.precision == "fp64" else 1
        w.name += "_" + args.precision
    prec = "fp32" if w.opts.precision == 1 else "fp64"
    # the CPU oracle first: its worker processes are forked before the GPU is touched
    cpu = None if args.no_cpu_baseline else cpu_baseline(w, args.cpu_disks_per_core)
    if cpu is not None:
        _progress(f"cpu baseline {cpu['value']:.1f} solves/s on {cpu['cores']} cores")
    r = Runner(w)
    T, o = timed(r, args.steps, args.warmup)
    sums64 = r.sums() if (args.workload == "dense" and not args.no_mixed) else None
    r.close()
    st = o["stats"]
    out = {
        "metric": "quadrature solves/s (node assembly + LU + block solve + sums per (disk, node)) over the "
                  "whole pmCIMb step; eigenpairs/s alongside",
        "value": st["node_solves"] / T,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if prec == "fp64" else "c64+c128",
        "data": "synthetic (seeded Gaussian coefficients and probes)",
        "config": {"workload": w.name, "n": sorted(set(p.n for p in w.problems)), "disks": int(len(o["flags"])),
                   "nodes_per_disk": w.opts.N, "probes": w.opts.s, "beyn_columns": w.opts.L, "precision": prec,
                   "problems": len(w.problems), "pivot": args.pivot},
        "eigenpairs_per_s": len(o["eigs"]) / T,
        "verified_eigenpairs": int(len(o["eigs"])),
        "flagged_disks": int(np.sum(o["flags"])),
        "candidates": o["ncand"],
        "phase_ms": phase_dict(st),
        "refine_sweeps": st["refine_sweeps"],
        "refine_fallbacks": st["refine_fallbacks"],
        "lu_flops_per_step": st["lu_flops"],
        # the whole LU's algorithmic flops (sum of 8 n^3 / 3) over the wall time of the
        # indicator sweep (assembly, LU, solves, sums; both worker streams) and of the step
        "lu_frac_of_peak_over_sweep_wall": st["lu_flops"] / (st["ms_total"] * 1e-3) / PEAK[prec],
        "lu_frac_of_peak_over_step_wall": st["lu_flops"] / T / PEAK[prec],
        "sweep_ms": st["ms_total"],
        "roofline": roofline(st, prec, w.name),
    }
    _progress(f"{w.name}: {out['value']:.0f} solves/s, {T * 1e3:.0f} ms per step")
    out["peak_measured"] = peak_measured()
    if args.workload == "dense" and not args.no_mixed:
        wm = build_workload("dense_mixed", pivot=pivot)
        rm = Runner(wm)
        Tm, om = timed(rm, args.steps, args.warmup)
        sm = rm.sums()
        rm.close()
        stm = om["stats"]
        # agreement of the mixed sweep with the complex128 sweep: moments of flagged
        # disks (no cancellation there) and identical flags
        fl = np.nonzero(o["flags"])[0]
        rel = 0.0
        for d in fl:
            for a, b in ((sm[2][d], sums64[2][d]), (sm[3][d], sums64[3][d])):
                rel = max(rel, float(np.linalg.norm(a - b) / np.linalg.norm(b)))
        _progress(f"{wm.name}: {stm['node_solves'] / Tm:.0f} solves/s")
        out["mixed"] = {"workload": wm.name, "value": stm["node_solves"] / Tm, "ms_per_step": Tm * 1e3,
                        "speedup_vs_fp64": T / Tm, "flags_identical": bool(np.array_equal(om["flags"], o["flags"])),
                        "max_rel_moment_diff_vs_fp64_flagged": rel, "refine_sweeps": stm["refine_sweeps"],
                        "refine_fallbacks": stm["refine_fallbacks"], "phase_ms": phase_dict(stm),
                        "sweep_ms": stm["ms_total"], "sweep_speedup_vs_fp64": st["ms_total"] / stm["ms_total"],
                        "lu_frac_of_fp32_peak_over_sweep_wall": stm["lu_flops"] / (stm["ms_total"] * 1e-3) / PEAK["fp32"],
                        "roofline": roofline(stm, "fp32", wm.name), "verified_eigenpairs": int(len(om["eigs"]))}
    if args.workload in ("dense", "dense_mixed") and not args.no_eigen:
        # eigenpairs where the rank test is not saturated (31 probe columns, n = 64)
        eo = {}
        for tag, precision in (("fp64", 0), ("mixed", 1)):
            we = build_workload("small_L31", pivot=pivot)
            we.opts.precision = precision
            re_ = Runner(we)
            Te, oe = timed(re_, max(3, args.steps), 1)
            re_.close()
            eo[tag] = {"eigenpairs": int(len(oe["eigs"])), "ms_per_step": Te * 1e3,
                       "eigenpairs_per_s": len(oe["eigs"]) / Te}
        out["eigenpairs_unsaturated"] = {"workload": "qep_n64_4x4_L31", **eo}
        _progress("unsaturated eigenpairs done")
    if args.workload == "dense" and not args.no_eigen and not args.no_mixed:
        out["eigenpairs_complete"] = {"workload": w.name + "_adaptive", **complete_spectrum(pivot)}
        _progress("complete spectrum done")
    if args.workload == "dense" and not args.no_eigen:
        out["pmcima"] = pmcima_run()
        out["generic_assembly"] = generic_run(max(2, min(args.steps, 3)))
        out["scattering"] = scattering_run()
        _progress("pmCIMa, generic assembly and scattering done")
    if args.workload == "dense" and not args.no_delay:
        out["delay_family"] = delay_run()
        _progress(f"delay family: {out['delay_family']['value']:.0f} solves/s")
    if args.workload == "dense" and not args.no_screener:
        out["screener"] = screener_run()
        _progress("screener done")
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
