"""GPU checks of the screener network kernels against the FP64 oracle, and of the
screening pipeline (labels from the method's own sweeps, training, evaluation)."""
import sys

import numpy as np
import pytest

import gen
import oracle
from oracle import mlp as omlp

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


def _batch(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, 32)).astype(np.float32)
    Y = (rng.uniform(size=(B, 4)) > 0.6).astype(np.float32)
    return X, Y


def test_forward_and_gradient_match_oracle(N):
    import torch
    say("case screener gradient B=37")
    B = 37
    X, Y = _batch(B, 1)
    th = gen.mlp_init(7)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    P, Xd, Yd = d(th), d(X), d(Y)
    grad = torch.zeros_like(P)
    work = torch.empty(N.nep_mlp_workspace_floats(B), dtype=torch.float32, device="cuda")
    loss = N.nep_mlp_grad(P, Xd, Yd, None, B, grad, work, want_loss=True)
    Lr, gr = omlp.loss_and_grad(th.astype(np.float64), X.astype(np.float64), Y.astype(np.float64))
    g = grad.cpu().numpy().astype(np.float64)
    assert abs(loss - Lr) <= 1e-5 * abs(Lr)
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)
    # per layer too (the small output layer must not hide in the norm)
    offs = [0, 4096, 4224, 20608, 20736, 21248, 21252]
    for a, b in zip(offs[:-1], offs[1:]):
        assert np.linalg.norm(g[a:b] - gr[a:b]) <= 1e-4 * np.linalg.norm(gr[a:b]) + 1e-9
    probs = torch.empty((B, 4), dtype=torch.float32, device="cuda")
    N.nep_mlp_forward(P, Xd, None, B, probs, work)
    _, _, pr = omlp.forward(th.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(probs.cpu().numpy() - pr)) < 1e-5
    # gathered rows: idx selects rows of X and Y
    idx = np.array([5, 0, 36, 12], np.int32)
    N.nep_mlp_grad(P, Xd, Yd, d(idx), 4, grad, work)
    _, gi = omlp.loss_and_grad(th.astype(np.float64), X[idx].astype(np.float64), Y[idx].astype(np.float64))
    assert np.linalg.norm(grad.cpu().numpy() - gi) <= 1e-4 * np.linalg.norm(gi)


def test_adam_matches_oracle(N):
    import torch
    say("case screener adam")
    rng = np.random.default_rng(2)
    th = gen.mlp_init(7)
    g = rng.standard_normal(th.size).astype(np.float32) * 1e-2
    m = rng.standard_normal(th.size).astype(np.float32) * 1e-3
    v = np.abs(rng.standard_normal(th.size).astype(np.float32)) * 1e-5
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    P, G, M, V = d(th), d(g), d(m), d(v)
    N.nep_mlp_adam(P, G, M, V, 3, 1e-3)
    ref, mr, vr = omlp.adam_step(th.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                                 v.astype(np.float64), 3)
    assert np.max(np.abs(P.cpu().numpy() - ref)) < 1e-6
    assert np.allclose(M.cpu().numpy(), mr, rtol=1e-5, atol=1e-9)


def test_screener_labels_training_and_gain(N):
    from paper_2312_13117_amd import screener
    say("case screener pipeline: 240 problems n=48, depth 3")
    problems = [gen.screener_problem(p, 48) for p in range(240)]
    ds = screener.build_dataset(problems, depth=3, log=say)
    assert len(ds.labels) > 240
    # labels are the method's own flags: recompute two parents' children with the oracle
    F = gen.probes(2, 48, 1)
    checked = 0
    for row in (0, len(ds.labels) // 2):
        p, lvl = int(ds.problem[row]), int(ds.level[row])
        # find the parent rectangle by replaying the recursion for this problem
        rect = screener.Rect(-4, 4, -4, 4)
        if lvl == 0:
            kids = screener._children(rect)
            for k, r in enumerate(kids):
                dk = oracle.Disk(0, 0, 0.5 * (r.x0 + r.x1), 0.5 * (r.y0 + r.y1), 0.5 * (r.x1 - r.x0),
                                 0.5 * (r.y1 - r.y0))
                sw = oracle.sweep_disk(problems[p], dk.c, dk.r, 32, F, None)
                I, _ = sw.indicator()
                assert bool(ds.labels[row, k]) == (I > 0.1)
            checked += 1
    assert checked >= 1
    train_mask = ds.problem < 180
    params, X, tstats = screener.train(ds, train_mask, epochs=60, log=say)
    assert tstats["loss_last"] < tstats["loss_first"]
    test_rows = np.nonzero(~train_mask)[0]
    probs = screener.predict(params, X, test_rows)
    ev = screener.evaluate(probs, ds.labels[test_rows], ds.level[test_rows])
    say(ev)
    e = ev["evals_until_all_positive"]
    # the trained network orders the children better than a random order
    assert e["network"] < e["random"]
    assert 0.0 <= ev["miss_rate"] <= 1.0
    # a live screen of the held-out problems in ranked rounds: every child is swept, so
    # the labels are the method's; network ranking knows more positive children after
    # the first round than cover order
    held = problems[180:]
    runs = {o: screener.screen_ordered(held, params, tstats["feature_mean"], tstats["feature_sd"], depth=3,
                                       order=o) for o in ("network", "raster")}
    want = {}
    for i in test_rows:
        key = (int(ds.problem[i]) - 180, int(ds.level[i])) + tuple(np.round(ds.cell[i], 12))
        want[key] = ds.labels[i] > 0.5
    for o, r in runs.items():
        got = {(p, lv) + tuple(np.round(c, 12)): f for p, lv, c, f in r["labels"]}
        assert set(got) == set(want), o
        for k in want:
            assert np.array_equal(got[k], want[k]), (o, k)
    first = {o: sum(lv["known_after_round"][0] for lv in r["levels"]) for o, r in runs.items()}
    tot = sum(lv["positive_children"] for lv in runs["network"]["levels"])
    say(f"positive children known after the first round: network {first['network']}, raster {first['raster']} "
        f"of {tot}")
    assert first["network"] > first["raster"]
