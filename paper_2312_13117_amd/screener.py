"""Learned screening of child subregions (an extension, not part of the paper).

The spectral indicator method recursively quadrisects flagged squares (the SIM
recursion of Section 2.1, the level loop of pmCIMa in Section 3.1).  For a parametrised
family of problems this driver

  1. runs that recursion on a quadtree over a square (levels 1..depth below the root),
     sweeping every child of every flagged parent through the C ABI, and records for
     each flagged parent its node profile ||T(z_j)^{-1} f|| (j = 1..N) and the four
     child flags;
  2. trains the screener network (32 -> 128 -> 128 -> 4) on the GPU with the library's
     forward/backward/Adam kernels, features log10(profile) z-scored with training
     statistics;
  3. evaluates it on held-out problems: miss rate against the method's own flags,
     solves saved by the counterfactual "skip predicted-negative children" policy, and
     the ordering gain (child evaluations until every positive child has been screened,
     network order vs raster and random order);
  4. screens the held-out problems again with each level's children swept in ranked
     rounds (screen_ordered): round r sweeps every parent's child of rank r, ranked by
     the network or in cover order, and the positive children known after each round
     are counted.

The network only orders the screening; every child is still swept by the method, so
the flags (and the eigenvalues) never depend on it.

    python -m paper_2312_13117_amd.screener --problems 2000 --train 1600
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import nep as N


@dataclass
class Rect:
    x0: float
    x1: float
    y0: float
    y1: float


def _children(r: Rect) -> List[Rect]:
    """Children in the library's cell order (ix-major: ix*2 + iy)."""
    xm, ym = 0.5 * (r.x0 + r.x1), 0.5 * (r.y0 + r.y1)
    return [Rect(r.x0, xm, r.y0, ym), Rect(r.x0, xm, ym, r.y1), Rect(xm, r.x1, r.y0, ym), Rect(xm, r.x1, ym, r.y1)]


def _sweep(dev_problems, entries, split: int, opts, F):
    """One plan over `entries` = [(problem index, rect)], each rect split split x split;
    returns (flags [len(entries), split^2], profiles [len(entries), split^2, N])."""
    import gen
    probs = [dev_problems[p] for p, _ in entries]
    regs = [gen.Region(r.x0, r.x1, r.y0, r.y1, split, split) for _, r in entries]
    plan = N.nep_plan(probs, regs, opts)
    try:
        Fl = [F[p] for p, _ in entries]
        ind, flags, prof, st = N.nep_indicator(plan, Fl, None, want_profiles=True)
    finally:
        N.nep_destroy(plan)
    k = split * split
    return flags.reshape(len(entries), k), prof[:, :, 0].reshape(len(entries), k, opts.N)


@dataclass
class Dataset:
    problem: np.ndarray    # parent's problem index
    level: np.ndarray      # parent's level (0 = root)
    profile: np.ndarray    # parent's node profile [rows, N]
    labels: np.ndarray     # child flags [rows, 4]
    sweeps: int            # disks swept
    seconds: float
    cell: np.ndarray = None  # parent cell (x0, x1, y0, y1) [rows, 4]


def build_dataset(problems, depth: int = 3, root: Rect = Rect(-4, 4, -4, 4), N_nodes: int = 32,
                  probe_seed: int = 2, chunk: int = 1000, log=print, precision: int = 0) -> Dataset:
    """SIM recursion over the quadtree for every problem; one record per flagged parent.
    precision: 0 = complex128 LU, 1 = complex64 LU with complex128 refinement."""
    import gen
    import torch
    opts = gen.Options(N=N_nodes, s=1, L=0, precision=precision)
    devp = [N.upload_problem(p) for p in problems]
    F = [N._dev_complex(gen.probes(probe_seed, p.n, 1), torch) for p in problems]
    t0 = time.perf_counter()
    rows_p, rows_l, rows_prof, rows_lab, rows_cell = [], [], [], [], []
    sweeps = 0
    # level 0: the root disk of every problem (for its profile)
    ent = [(p, root) for p in range(len(problems))]
    fl, pr = [], []
    for c in range(0, len(ent), chunk):
        f, q = _sweep(devp, ent[c:c + chunk], 1, opts, F)
        fl.append(f[:, 0])
        pr.append(q[:, 0])
    fl, pr = np.concatenate(fl), np.concatenate(pr)
    sweeps += len(ent)
    # The root is always subdivided: a circle that encloses the whole spectrum of a
    # matrix polynomial of degree >= 2 gives P f = 0 (T(z)^{-1} decays like z^-2), so
    # the root's indicator carries no information and the level-1 cells form the
    # initial cover.  The root's sweep still provides its node profile.
    parents = [(p, r, prof) for (p, r), prof in zip(ent, pr)]
    for level in range(1, depth + 1):
        if not parents:
            break
        ent = [(p, r) for p, r, _ in parents]
        flags, prof = [], []
        for c in range(0, len(ent), chunk):
            f, q = _sweep(devp, ent[c:c + chunk], 2, opts, F)
            flags.append(f)
            prof.append(q)
        flags, prof = np.concatenate(flags), np.concatenate(prof)
        sweeps += 4 * len(ent)
        nxt = []
        for i, (p, r, pprof) in enumerate(parents):
            rows_p.append(p)
            rows_l.append(level - 1)
            rows_prof.append(pprof)
            rows_lab.append(flags[i].astype(np.float32))
            rows_cell.append((r.x0, r.x1, r.y0, r.y1))
            if level < depth:
                for k, cr in enumerate(_children(r)):
                    if flags[i, k]:
                        nxt.append((p, cr, prof[i, k]))
        log(f"level {level}: {len(parents)} parents, {int(flags.sum())} positive children")
        parents = nxt
    return Dataset(np.asarray(rows_p), np.asarray(rows_l), np.asarray(rows_prof), np.asarray(rows_lab), sweeps,
                   time.perf_counter() - t0, np.asarray(rows_cell))


def train(ds: Dataset, train_mask: np.ndarray, epochs: int = 200, batch: int = 256, lr: float = 1e-3,
          init_seed: int = 7, shuffle_seed: int = 11, log=print):
    """Adam on the mean BCE with the library's kernels; returns (params, X, stats)."""
    import gen
    import torch
    dev = "cuda"
    rows = len(ds.labels)
    prof = torch.from_numpy(np.ascontiguousarray(ds.profile, dtype=np.float64)).to(dev)
    X = torch.empty((rows, ds.profile.shape[1]), dtype=torch.float32, device=dev)
    mean = torch.empty(ds.profile.shape[1], dtype=torch.float32, device=dev)
    sd = torch.empty_like(mean)
    tr = np.nonzero(train_mask)[0].astype(np.int32)
    trd = torch.from_numpy(tr).to(dev)
    N.nep_mlp_features(prof, rows, ds.profile.shape[1], trd, mean, sd, X)
    Y = torch.from_numpy(np.ascontiguousarray(ds.labels, dtype=np.float32)).to(dev)
    params = torch.from_numpy(gen.mlp_init(init_seed)).to(dev)
    grad = torch.zeros_like(params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    work = torch.empty(N.nep_mlp_workspace_floats(batch), dtype=torch.float32, device=dev)
    rng = np.random.default_rng(shuffle_seed)
    perms = np.concatenate([rng.permutation(tr) for _ in range(epochs)]).astype(np.int32)
    permd = torch.from_numpy(perms).to(dev)
    nb = max(1, len(tr) // batch)
    step = 0
    losses = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        base = ep * len(tr)
        for b in range(nb):
            idx = permd[base + b * batch: base + (b + 1) * batch]
            want = (b == nb - 1)
            L = N.nep_mlp_grad(params, X, Y, idx, int(idx.numel()), grad, work, want_loss=want)
            step += 1
            N.nep_mlp_adam(params, grad, m, v, step, lr)
            if want:
                losses.append(L)
        if ep % 50 == 0 or ep == epochs - 1:
            log(f"epoch {ep}: batch loss {losses[-1]:.4f}")
    torch.cuda.synchronize()
    return params, X, {"epochs": epochs, "steps": step, "seconds": time.perf_counter() - t0,
                       "loss_first": losses[0], "loss_last": losses[-1],
                       "feature_mean": mean.cpu().tolist(), "feature_sd": sd.cpu().tolist()}


def predict(params, X, rows: np.ndarray) -> np.ndarray:
    import torch
    B = len(rows)
    idx = torch.from_numpy(np.ascontiguousarray(rows, dtype=np.int32)).to("cuda")
    probs = torch.empty((B, 4), dtype=torch.float32, device="cuda")
    work = torch.empty(N.nep_mlp_workspace_floats(B), dtype=torch.float32, device="cuda")
    N.nep_mlp_forward(params, X, idx, B, probs, work)
    return probs.cpu().numpy()


def screen_ordered(problems, params, feature_mean, feature_sd, depth: int = 3, order: str = "network",
                   root: Rect = Rect(-4, 4, -4, 4), N_nodes: int = 32, probe_seed: int = 2) -> dict:
    """The SIM recursion of build_dataset with the children screened in ranked rounds:
    at every level, round r sweeps, for every flagged parent, its child of rank r --
    by descending network probability (order "network"; features of the parent's
    profile standardised with the training statistics, probabilities from the
    allocation-free forward pass) or in cover order ("raster").  Every child is still
    swept, so the flags are the method's; the ranking only decides which children are
    known first.  Returns, per level, the positive children known after each round, the
    mean number of child sweeps per parent until its positive children are all known,
    the wall time, and the labels (problem, level, cell, flags) for comparison."""
    import gen
    import torch
    opts = gen.Options(N=N_nodes, s=1, L=0)
    devp = [N.upload_problem(p) for p in problems]
    F = [N._dev_complex(gen.probes(probe_seed, p.n, 1), torch) for p in problems]
    mean = torch.tensor(feature_mean, dtype=torch.float32, device="cuda")
    sd = torch.tensor(feature_sd, dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    f, pr = _sweep(devp, [(p, root) for p in range(len(problems))], 1, opts, F)
    parents = [(p, root, pr[p, 0]) for p in range(len(problems))]
    levels, labels = [], []
    for level in range(1, depth + 1):
        if not parents:
            break
        P = len(parents)
        if order == "network":
            prof = torch.from_numpy(np.ascontiguousarray(np.stack([q for _, _, q in parents]), dtype=np.float64))
            prof = prof.to("cuda")
            X = torch.empty((P, N_nodes), dtype=torch.float32, device="cuda")
            N.nep_mlp_features(prof, P, N_nodes, None, mean, sd, X)
            probs = torch.empty((P, 4), dtype=torch.float32, device="cuda")
            for c0 in range(0, P, N.NEP_MLP_NOALLOC_MAX_B):
                B = min(N.NEP_MLP_NOALLOC_MAX_B, P - c0)
                idx = torch.arange(c0, c0 + B, dtype=torch.int32, device="cuda")
                N.nep_mlp_forward_noalloc(params, X, idx, B, probs[c0:c0 + B])
            rank = np.argsort(-probs.cpu().numpy(), axis=1, kind="stable")
        else:
            rank = np.tile(np.arange(4), (P, 1))
        flags = np.zeros((P, 4), dtype=bool)
        cprof = np.zeros((P, 4, N_nodes))
        known = []
        kids = [_children(r) for _, r, _ in parents]
        for rnd in range(4):
            ent = [(p, kids[i][rank[i, rnd]]) for i, (p, _, _) in enumerate(parents)]
            fl, q = _sweep(devp, ent, 1, opts, F)
            flags[np.arange(P), rank[:, rnd]] = fl[:, 0].astype(bool)
            cprof[np.arange(P), rank[:, rnd]] = q[:, 0]
            known.append(int(flags.sum()))
        # child sweeps per parent until all of its positive children were known
        pos_rank = np.where(np.take_along_axis(flags, rank, axis=1), np.arange(4)[None, :] + 1, 0)
        until = pos_rank.max(axis=1)
        has = until > 0
        levels.append({"level": level, "parents": P, "positive_children": known[-1],
                       "known_after_round": known, "mean_sweeps_until_all_positive":
                       float(until[has].mean()) if has.any() else 0.0})
        nxt = []
        for i, (p, r, _) in enumerate(parents):
            labels.append((p, level - 1, (r.x0, r.x1, r.y0, r.y1), flags[i].copy()))
            if level < depth:
                nxt.extend((p, kids[i][k], cprof[i, k]) for k in range(4) if flags[i, k])
        parents = nxt
    torch.cuda.synchronize()
    return {"order": order, "problems": len(problems), "seconds": time.perf_counter() - t0, "levels": levels,
            "labels": labels}


def evaluate(prob: np.ndarray, labels: np.ndarray, levels: np.ndarray, nodes: int = 32, seed: int = 13) -> dict:
    """Screening metrics of predicted child probabilities against the method's flags."""
    y = labels > 0.5
    pred = prob >= 0.5
    pos = y.sum()
    out = {
        "parents": int(len(y)),
        "children": int(y.size),
        "positive_children": int(pos),
        "miss_rate": float(((~pred) & y).sum() / max(1, pos)),
        "solves_saved": int(nodes * ((~pred) & (~y)).sum()),
        "solves_total": int(nodes * y.size),
        "false_skip_solves": int(nodes * ((~pred) & y).sum()),
    }
    # ordering: evaluations until every positive child has been screened
    def until_all(order_scores):
        cnt = []
        for i in range(len(y)):
            if not y[i].any():
                continue
            order = np.argsort(-order_scores[i], kind="stable")
            last = max(np.nonzero(y[i][order])[0])
            cnt.append(last + 1)
        return float(np.mean(cnt)) if cnt else 0.0
    raster = np.tile(-np.arange(4, dtype=float), (len(y), 1))   # children 0,1,2,3 in order
    rng = np.random.default_rng(seed)
    rnd = np.mean([until_all(rng.uniform(size=y.shape)) for _ in range(20)])
    out["evals_until_all_positive"] = {"network": until_all(prob), "raster": until_all(raster), "random": rnd,
                                       "oracle_best": until_all(y.astype(float))}
    out["per_level"] = {}
    for lv in sorted(set(levels.tolist())):
        mk = levels == lv
        yl, pl = y[mk], pred[mk]
        out["per_level"][int(lv + 1)] = {"children": int(yl.size), "label_rate": float(yl.mean()),
                                         "miss_rate": float(((~pl) & yl).sum() / max(1, yl.sum())),
                                         "accuracy": float((pl == yl).mean())}
    return out


def run(n_problems: int = 2000, n_train: int = 1600, n: int = 256, depth: int = 3, epochs: int = 200,
        log=print, precision: int = 0, compare_fp64: int = 0) -> dict:
    """The whole pipeline; the labels' sweeps in the given precision.  With
    compare_fp64 > 0 (and precision 1) the first compare_fp64 held-out problems are
    labelled again in complex128 for the time ratio and label identity."""
    import gen
    t0 = time.perf_counter()
    problems = [gen.screener_problem(p, n) for p in range(n_problems)]
    log(f"generated {n_problems} problems (n={n}) in {time.perf_counter() - t0:.1f} s")
    ds = build_dataset(problems, depth=depth, log=log, precision=precision)
    versus = None
    if precision == 1 and compare_fp64 > 0:
        sub = problems[n_train:n_train + compare_fp64]
        d64 = build_dataset(sub, depth=depth, log=lambda *a: None, precision=0)
        d32 = build_dataset(sub, depth=depth, log=lambda *a: None, precision=1)
        same = (len(d64.labels) == len(d32.labels) and np.array_equal(d64.labels, d32.labels)
                and np.array_equal(d64.cell, d32.cell))
        versus = {"problems": len(sub), "seconds_fp64": d64.seconds, "seconds_mixed": d32.seconds,
                  "speedup_mixed_vs_fp64": d64.seconds / d32.seconds, "labels_identical": bool(same)}
        log(f"labels of {len(sub)} problems: complex128 {d64.seconds:.2f} s, mixed {d32.seconds:.2f} s, "
            f"identical {same}")
    log(f"dataset: {len(ds.labels)} parents from {ds.sweeps} disk sweeps ({ds.sweeps * 32} solves) "
        f"in {ds.seconds:.1f} s")
    train_mask = ds.problem < n_train
    params, X, tstats = train(ds, train_mask, epochs=epochs, log=log)
    test_rows = np.nonzero(~train_mask)[0]
    probs = predict(params, X, test_rows)
    ev = evaluate(probs, ds.labels[test_rows], ds.level[test_rows])
    trivial = evaluate(np.ones_like(probs), ds.labels[test_rows], ds.level[test_rows])
    # the held-out problems screened again with the children in ranked rounds
    live = {}
    for order in ("network", "raster"):
        r = screen_ordered(problems[n_train:], params, tstats["feature_mean"], tstats["feature_sd"], depth=depth,
                           order=order)
        live[order] = {k: r[k] for k in ("seconds", "levels")}
    log(f"ranked rounds: {live}")
    return {"problems": n_problems, "train_problems": n_train, "n": n, "depth": depth,
            "dataset": {"parents": int(len(ds.labels)), "disk_sweeps": ds.sweeps, "solves": ds.sweeps * 32,
                        "seconds": ds.seconds},
            "training": {k: v for k, v in tstats.items() if not k.startswith("feature_")}, "test": ev,
            "trivial_all_positive": {k: trivial[k] for k in ("miss_rate", "solves_saved")},
            "ranked_rounds": live, "precision": precision, "labels_mixed_vs_fp64": versus}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--problems", type=int, default=2000)
    ap.add_argument("--train", type=int, default=1600)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--precision", type=int, default=0, help="0: complex128 LU, 1: complex64 + refinement")
    ap.add_argument("--compare-fp64", type=int, default=0)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    rep = run(a.problems, a.train, a.n, epochs=a.epochs, log=lambda *x: print(*x, file=sys.stderr, flush=True),
              precision=a.precision, compare_fp64=a.compare_fp64)
    js = json.dumps(rep)
    print(js)
    if a.out:
        with open(a.out, "w") as f:
            f.write(js + "\n")


if __name__ == "__main__":
    main()
