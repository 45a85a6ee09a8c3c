"""Batched rounds (lv_batch_*): many views of uneven n, k and rank updated in
one graph-replayed round must equal the same views updated one by one with
lv_view_update, bit for bit, and the FP64 oracle within tolerance.

The batch autotunes the tile rows of every level pass at creation and
stores them in the views; the one-by-one twins take the same tile rows.
A batch stages every update at its view's full width r_max (unused columns
zero).  Zero columns leave every value exact but a different width selects
a different reduction order, so the one-by-one twins receive the same
zero-padded factors."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import dev, host, need_gpu, note, read_all

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    note(f"start {request.node.nodeid}")
    yield


# (n, k, r): ragged orders, k from 1 to 16, ranks 1..8 (level ranks up to 64)
SHAPES = [(256, 16, 1), (300, 8, 3), (700, 16, 2), (513, 1, 2), (1100, 4, 5), (384, 16, 4),
          (640, 2, 8), (256, 16, 8), (900, 16, 1), (128, 8, 7)]


@pytest.mark.parametrize("dtype_name", ["f32", "f64", "bf16"])
def test_batch_rounds_match_single_views_and_oracle(dtype_name):
    need_gpu()
    import torch
    from paper_1403_6968_amd import linview as lv
    td, nd = (torch.float64, np.float64) if dtype_name == "f64" else (torch.float32, np.float32)
    mode = {"f32": lv.LV_FP32, "f64": lv.LV_FP64, "bf16": lv.LV_FP32_BF16SHADOW}[dtype_name]
    rounds = 4
    views, twins, ref, staged = [], [], [], []
    for v, (n, k, r) in enumerate(SHAPES):
        A = synth.gaussian_matrix(n, seed=30, config=4, view=v).astype(nd).astype(np.float64)
        views.append(lv.View(dev(A, td), k, r_max=r, mode=mode))
        twins.append(lv.View(dev(A, td), k, r_max=r, mode=mode))
        ref.append(O.reeval(A, k))
    batch = lv.Batch(views)
    tun = batch.tuning()
    note(f"autotuning {dtype_name}: {tun}; tiles {[v.tile_rows() for v in views]}")
    assert tun["tuned_groups"] + tun["cache_hits"] > 0
    for v, tw in zip(views, twins):
        tw.set_tile_rows(v.tile_rows())      # the twins reduce in the same order
    # the zero round of the autotuner left every view unchanged
    for v in range(len(SHAPES)):
        got, twin = read_all(views[v]), read_all(twins[v])
        for i in got:
            np.testing.assert_array_equal(got[i], twin[i])
    for t in range(rounds):
        for v, (n, k, r) in enumerate(SHAPES):
            if (v + t) % 4 == 3:                      # some views sit a round out
                batch.stage(v)
                z = torch.zeros(n, r, dtype=td, device="cuda")
                twins[v].update(z, z)
                continue
            rr = 1 + (v + t) % r                       # ranks vary between rounds
            U, V = synth.update_factors(n, rr, 1, seed=31 + t, config=4, view=v)
            U = U[0].astype(nd).astype(np.float64)
            V = V[0].astype(nd).astype(np.float64)
            Ud, Vd = dev(U, td), dev(V, td)
            batch.stage(v, Ud, Vd)
            Up = np.zeros((n, r)); Up[:, :rr] = U
            Vp = np.zeros((n, r)); Vp[:, :rr] = V
            twins[v].update(dev(Up, td), dev(Vp, td))
            ref[v] = O.incr_update(ref[v], U, V)
        batch.update()
    tol = {"f64": 1e-10, "f32": 1e-4, "bf16": 5e-3}[dtype_name]
    worst = 0.0
    for v in range(len(SHAPES)):
        got, twin = read_all(views[v]), read_all(twins[v])
        for i in got:
            np.testing.assert_array_equal(got[i], twin[i])
            worst = max(worst, O.maxrel(got[i], ref[v][i]))
    note(f"batch {dtype_name}: worst maxrel vs oracle {worst:.2e}")
    assert worst < tol
    assert views[0].stats()["updates"] == rounds
    batch.close()
    for x in views + twins:
        x.close()


def test_batch_errors():
    need_gpu()
    import torch
    from paper_1403_6968_amd import linview as lv
    a = lv.View(torch.zeros(64, 64, dtype=torch.float32, device="cuda"), 4)
    b = lv.View(torch.zeros(64, 64, dtype=torch.float64, device="cuda"), 4)
    with pytest.raises(lv.LinviewError):
        lv.Batch([a, b])                               # mixed modes
    batch = lv.Batch([a])
    U = torch.zeros(64, 2, dtype=torch.float32, device="cuda")
    with pytest.raises(lv.LinviewError):
        batch.stage(0, U, U)                           # rank above r_max
    with pytest.raises(lv.LinviewError):
        batch.stage(1)                                 # no such view
    batch.close(); a.close(); b.close()


def test_batched_workload_full_size_against_oracle():
    """The batched benchmark's workload at its real size: 64 views, n in
    {512, 1024, 2048, 4096}, k in {8, 16}, ranks 1..8, FP32, drawn by the
    same generator as bench.py; three rounds through one batch (autotuned
    tiles, the round planner's lane split at 64 views), then every element of
    every stored power of every view against the FP64 oracle."""
    need_gpu()
    import torch
    from paper_1403_6968_amd import linview as lv
    g = synth.rng(0, 4, 0)
    ns = g.choice([512, 1024, 2048, 4096], size=64)
    ks = g.choice([8, 16], size=64)
    rs = g.integers(1, 9, size=64)
    rounds = 3
    views, ref = [], []
    for v in range(64):
        n, k, r = int(ns[v]), int(ks[v]), int(rs[v])
        A = synth.gaussian_matrix(n, seed=0, config=4, view=v).astype(np.float32).astype(np.float64)
        views.append(lv.View(dev(A, torch.float32), k, r_max=r))
        ref.append(O.reeval(A, k))
    note("64 views created")
    batch = lv.Batch(views)
    for t in range(rounds):
        for v in range(64):
            n, r = int(ns[v]), int(rs[v])
            U, V = synth.update_factors(n, r, rounds, seed=0, config=4, view=v)
            U = U[t].astype(np.float32).astype(np.float64)
            V = V[t].astype(np.float32).astype(np.float64)
            batch.stage(v, dev(U, torch.float32), dev(V, torch.float32))
            ref[v] = O.incr_update(ref[v], U, V)
        batch.update()
    torch.cuda.synchronize()
    worst = 0.0
    for v in range(64):
        got = read_all(views[v])
        for i in ref[v]:
            err = O.maxrel(got[i], ref[v][i])
            worst = max(worst, err)
            assert err < 1e-4, f"view {v} (n={ns[v]}, k={ks[v]}, r={rs[v]}) A^{i}: maxrel {err:.2e}"
    note(f"64 views after {rounds} rounds: worst maxrel {worst:.2e}")
    batch.close()
    for x in views:
        x.close()


def test_autotune_cache_persists_through_json(tmp_path):
    """Tile rows chosen by the autotuner, saved as JSON, cleared from the
    process and loaded again, serve a second batch of the same shapes
    without timing anything."""
    need_gpu()
    import torch
    from paper_1403_6968_amd import linview as lv
    shapes = [(700, 16, 2), (1500, 8, 4), (3000, 16, 1)]
    mk = lambda: [lv.View(dev(synth.gaussian_matrix(n, seed=50, config=4, view=v).astype(np.float32), torch.float32),
                          k, r_max=r) for v, (n, k, r) in enumerate(shapes)]
    lv.lv_tune_cache_clear()
    a = mk()
    ba = lv.Batch(a)
    t1 = ba.tuning()
    assert t1["tuned_groups"] > 0 and t1["cache_hits"] == 0
    path = str(tmp_path / "tune.json")
    lv.lv_tune_cache_save(path)
    lv.lv_tune_cache_clear()
    assert lv.lv_tune_cache_load(path) == t1["tuned_groups"]
    b = mk()
    bb = lv.Batch(b)
    t2 = bb.tuning()
    note(f"first {t1}, after reload {t2}; tiles {[v.tile_rows() for v in a]}")
    assert t2["tuned_groups"] == 0 and t2["cache_hits"] == t1["tuned_groups"]
    assert [v.tile_rows() for v in a] == [v.tile_rows() for v in b]
    for x in (ba, bb):
        x.close()
    for v in a + b:
        v.close()
