"""Benchmark of the pmCIMb quadrature sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dense|small|...]

A step is one pass of the whole path over the workload: assembly + LU + block solve
+ quadrature sums + indicators for every (disk, node), Beyn's extraction on the
flagged disks, and sigma_min verification of the kept candidates.  Inputs are seeded
synthetic matrices already resident in HBM when the timed region starts.

Prints ONE JSON line (rank 0).  `value` = node solves per second of the whole step.
`roofline` reports the dominant kernel (the trailing-update kernel of the batched LU)
from the library's own per-launch HIP events on the stream it runs on.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same workload.
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


def build_workload(name: str):
    import gen
    if name == "dense":
        return gen.workload_dense_qep(1024, precision=0)
    if name == "dense_mixed":
        return gen.workload_dense_qep(1024, precision=1)
    if name == "small":
        return gen.workload_small_qep()
    raise SystemExit(f"unknown workload {name}")


def run_gpu(w, steps: int, warmup: int):
    import torch
    from paper_2312_13117_amd import nep as N
    plan = N.nep_plan(w.problems, w.regions, w.opts)
    F = [N._dev_complex(f, torch) for f in w.F]
    V = [N._dev_complex(v, torch) if v is not None else None for v in w.V]
    Vl = V if all(v is not None for v in V) else None
    disk_prob = np.zeros(plan.total_disks, np.int32)
    for p in range(len(w.problems)):
        first = N.lib().nep_disk_offset(plan.handle, p)
        last = N.lib().nep_disk_offset(plan.handle, p + 1) if p + 1 < len(w.problems) else plan.total_disks
        disk_prob[first:last] = p
    res = None
    for _ in range(warmup):
        res = N.pmcimb(plan, F, Vl, disk_prob)
    torch.cuda.synchronize()
    times, sweep_stats = [], []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ind, flags, _, _ = N.nep_indicator(plan, F, Vl)
        st_sweep = N.nep_get_stats(plan)
        flagged = np.nonzero(flags)[0]
        cand, cdisk = [], []
        if Vl is not None and len(flagged):
            eig, p, sv, keep, _, _ = N.nep_beyn(plan, flagged)
            for i, d in enumerate(flagged):
                for k in range(int(p[i])):
                    if keep[i, k]:
                        cand.append(eig[i, k])
                        cdisk.append(d)
        nver = 0
        if cand:
            sig, acc = N.nep_verify(plan, disk_prob[np.asarray(cdisk)], cand)
            al = np.asarray(cand)[acc]
            nver = int(N.nep_dedup(al, sig[acc]).sum()) if len(al) else 0
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        sweep_stats.append(st_sweep)
        res = (flags, len(cand), nver)
    N.nep_destroy(plan)
    return times, sweep_stats, res


def cpu_baseline(w, max_disks: int):
    """FP64 CPU oracle on a bounded sample: the first `max_disks` disks of problem 0."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    prob, reg = w.problems[0], w.regions[0]
    disks = oracle.cover(reg)
    # sample disks spread over the region
    idx = np.linspace(0, len(disks) - 1, max_disks).round().astype(int)
    t0 = time.perf_counter()
    for d in idx:
        dk = disks[d]
        oracle.sweep_disk(prob, dk.c, dk.r, w.opts.N, w.F[0], w.V[0])
    dt = time.perf_counter() - t0
    solves = len(idx) * w.opts.N
    return {"value": solves / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(idx)} disks x {w.opts.N} nodes of problem 0 (n={prob.n}, "
                      f"{w.F[0].shape[1]}+{0 if w.V[0] is None else w.V[0].shape[1]} right-hand sides), "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="dense")
    ap.add_argument("--cpu-disks", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    w = build_workload(args.workload)
    times, stats, (flags, ncand, nver) = run_gpu(w, args.steps, args.warmup)
    T = float(np.median(times))
    st = stats[len(stats) // 2]
    nsolves = st["node_solves"]
    prec = "fp32" if w.opts.precision == 1 else "fp64"
    achieved = st["gemm_flops"] / (st["ms_gemm"] * 1e-3) if st["ms_gemm"] > 0 else 0.0
    lu_rate = st["lu_flops"] / (st["ms_lu"] * 1e-3) if st["ms_lu"] > 0 else 0.0
    out = {
        "metric": "quadrature solves/s (node LU + block solve + sums) of the whole pmCIMb step",
        "value": nsolves / T,
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
        "config": {"workload": w.name, "n": w.problems[0].n, "disks": int(len(flags)), "nodes_per_disk": w.opts.N,
                   "probes": w.opts.s, "beyn_columns": w.opts.L, "precision": prec},
        "eigenpairs_per_s": nver / T,
        "verified_eigenpairs": nver,
        "flagged_disks": int(np.sum(flags)),
        "candidates": ncand,
        "phase_ms": {k: st[k] for k in ("ms_assemble", "ms_lu", "ms_solve", "ms_refine", "ms_sums", "ms_total")},
        "lu_tflops": lu_rate / 1e12,
        "lu_frac_of_peak": lu_rate / PEAK[prec],
        "roofline": {"kernel": "lu_gemm_kernel<update> (trailing update of the batched LU)", "bound": "mfma",
                     "achieved": achieved / 1e12, "peak": PEAK[prec] / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK[prec], "traffic": None,
                     "launches": st["gemm_launches"], "avg_launch_ms": st["ms_gemm"] / max(1, st["gemm_launches"])},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_disks)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
