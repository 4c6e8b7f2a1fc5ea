"""Workgroup-tile autotuning of the forward products of a batched plan over an
uneven problem list: every tile gives results identical bit for bit to the
shape heuristic's, a plan tuned on its first execute matches the untuned
plan bit for bit, and the tuning table is written to RSVD_TUNE_CACHE and
reused by a later plan with the same shapes."""
import json
import os

import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu

TILES = [(64, 64), (128, 64), (64, 128), (128, 128)]
SHAPES = [  # m, n, k, p, q, alpha: triangular-factor (n >= 4 l) and plain problems, m < n and m > n
    (700, 300, 40, 16, 2, 0.05),
    (300, 200, 80, 16, 1, 0.03),
    (90, 1100, 24, 8, 2, 0.08),
    (1030, 130, 30, 10, 2, 0.1),
    (257, 257, 64, 16, 2, 0.02),
]
MODES = [(np.float64, torch.float64, "f64"), (np.float32, torch.float32, "f32"),
         (np.float32, torch.float32, "bf16")]


def problems(npdt):
    out = []
    for i, (m, n, k, p, q, alpha) in enumerate(SHAPES):
        A = wl.make_matrix(m, n, np.exp(-alpha * np.arange(1, min(m, n) + 1)), 300 + i).astype(npdt)
        out.append((A, dict(m=m, n=n, k=k, p=p, q=q, seed=400 + i)))
    return out


def snapshot(plan, As):
    outs, w, kk, info = plan.execute(As)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    return [tuple(t.clone() for t in o) for o in outs], w.clone(), kk.clone()


def same(a, b):
    (oa, wa, ka), (ob, wb, kb) = a, b
    assert torch.equal(wa, wb) and torch.equal(ka, kb)
    for x, y in zip(oa, ob):
        for s, t in zip(x, y):
            assert torch.equal(s, t)


@pytest.mark.parametrize("npdt,tdt,prec", MODES, ids=[m[2] for m in MODES])
def test_every_tile_gives_identical_results(npdt, tdt, prec):
    import paper_1710_01463_amd as P
    probs = problems(npdt)
    As = [torch.from_numpy(A).cuda() for A, _ in probs]
    plan = P.Plan([pr for _, pr in probs], tdt, prec, graph=True)
    ref = snapshot(plan, As)
    n = len(plan.tiles())
    assert n >= 3  # the sketch products of every stage and the projections
    for tile in TILES:
        plan.set_tiles([tile] * n)
        assert plan.tiles() == [tile] * n
        same(ref, snapshot(plan, As))
        same(ref, snapshot(plan, As))  # graph replay with the same descriptors
    mixed = [TILES[i % 4] for i in range(n)]
    plan.set_tiles(mixed)
    same(ref, snapshot(plan, As))
    with pytest.raises(RuntimeError):
        plan.set_tiles([(32, 64)] * n)
    with pytest.raises(RuntimeError):
        plan.set_tiles([(64, 64)] * (n + 1))
    plan.close()


def test_tuned_plan_matches_and_table_is_reused(tmp_path, monkeypatch):
    import paper_1710_01463_amd as P
    cache = tmp_path / "tiles.json"
    monkeypatch.setenv("RSVD_TUNE_CACHE", str(cache))
    probs = problems(np.float32)
    As = [torch.from_numpy(A).cuda() for A, _ in probs]
    base = P.Plan([pr for _, pr in probs], torch.float32, "f32", graph=True)
    ref = snapshot(base, As)
    base.close()
    tuned = P.Plan([pr for _, pr in probs], torch.float32, "f32", graph=True, tune=True)
    same(ref, snapshot(tuned, As))  # the tuning execute, then the first graph launch
    same(ref, snapshot(tuned, As))
    chosen = tuned.tiles()
    assert all(t in TILES for t in chosen)
    table = json.loads(cache.read_text())
    assert len(table) >= 1 and set(table.values()) <= {f"{a}x{b}" for a, b in TILES}
    again = P.Plan([pr for _, pr in probs], torch.float32, "f32", graph=True, tune=True)
    same(ref, snapshot(again, As))
    assert again.tiles() == chosen  # every signature found in the table, nothing re-measured
    tuned.close()
    again.close()
