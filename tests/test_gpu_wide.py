"""Top factors 512 columns wide (k = 16, r_max = 32): plain float views reach
level rank 256 below the top and a rank-512 update of the top power (App. A:
the level-j factors are 2^j r columns wide).  Each stored power equals the
FP64 oracle's re-evaluation of the accumulated matrix within the mode's
tolerance (FP32 1e-4, bfloat16 shadows 5e-3); a pipelined batch equals the
sequential updates bit for bit; a batched round equals one-by-one twins bit
for bit; a server coalescing up to 32 requests per update equals the oracle."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import dev, host, need_gpu, note, read_all

pytestmark = pytest.mark.gpu

MiB = 1 << 20
TOL = {"fp32": 1e-4, "bf16": 5e-3}


@pytest.fixture(autouse=True)
def _announce(request):
    note(f"start {request.node.nodeid}")
    yield


def _lv():
    need_gpu()
    from paper_1403_6968_amd import linview
    return linview


@pytest.mark.parametrize("mode_name", ["fp32", "bf16"])
def test_wide_view_updates_match_oracle(mode_name):
    """n = 700 (ragged), k = 16, rank-32 updates: level ranks 32 .. 256,
    top 512; six updates one at a time on one view, the same six as a
    pipelined batch on a twin."""
    lv = _lv()
    import torch
    mode = {"fp32": lv.LV_FP32, "bf16": lv.LV_FP32_BF16SHADOW}[mode_name]
    n, k, r, T = 700, 16, 32, 6
    A = synth.gaussian_matrix(n, seed=61, config=7).astype(np.float32)
    Us, Vs = synth.update_factors(n, r, T, seed=61, config=7)
    Us, Vs = Us.astype(np.float32), Vs.astype(np.float32)
    Ad, Ud, Vd = dev(A, torch.float32), dev(Us, torch.float32), dev(Vs, torch.float32)
    a = lv.View(Ad, k, r_max=r, mode=mode)
    b = lv.View(Ad, k, r_max=r, mode=mode)
    b.set_pipeline(False)
    for t in range(T):
        a.update(Ud[t], Vd[t])
    c = lv.View(Ad, k, r_max=r, mode=mode)
    c.update_batch(Ud, Vd)                       # pipelined over the level stages
    b.update_batch(Ud, Vd)                       # the same batch run sequentially
    torch.cuda.synchronize()
    At = A.astype(np.float64) + np.einsum("tir,tjr->ij", Us.astype(np.float64), Vs.astype(np.float64))
    ref = O.reeval(At, k)
    worst = 0.0
    for p in a.powers():
        pa, pb, pc = a.read(p), b.read(p), c.read(p)
        assert torch.equal(pb, pc), f"P{p}: pipelined != sequential"
        for got in (pa, pc):
            err = O.maxrel(host(got), ref[p])
            worst = max(worst, err)
            assert err < TOL[mode_name], (p, err)
    note(f"wide {mode_name}: maxrel vs oracle {worst:.2e}")
    for x in (a, b, c):
        x.close()


def test_wide_batched_round_matches_twins():
    """A batch of a width-512 view and a narrow one: three rounds equal the
    one-by-one twins bit for bit (same tile rows) and the oracle."""
    lv = _lv()
    import torch
    shapes = [(600, 16, 32), (520, 8, 8)]
    views, twins, ref = [], [], []
    for v, (n, k, r) in enumerate(shapes):
        A = synth.gaussian_matrix(n, seed=62, config=4, view=v).astype(np.float32).astype(np.float64)
        views.append(lv.View(dev(A, torch.float32), k, r_max=r))
        twins.append(lv.View(dev(A, torch.float32), k, r_max=r))
        ref.append(O.reeval(A, k))
    batch = lv.Batch(views)
    for v, tw in zip(views, twins):
        tw.set_tile_rows(v.tile_rows())
    for t in range(3):
        for v, (n, k, r) in enumerate(shapes):
            U, V = synth.update_factors(n, r, 1, seed=63 + t, config=4, view=v)
            U = U[0].astype(np.float32).astype(np.float64)
            V = V[0].astype(np.float32).astype(np.float64)
            batch.stage(v, dev(U, torch.float32), dev(V, torch.float32))
            twins[v].update(dev(U, torch.float32), dev(V, torch.float32))
            ref[v] = O.incr_update(ref[v], U, V)
        batch.update()
    worst = 0.0
    for v in range(len(shapes)):
        got, twin = read_all(views[v]), read_all(twins[v])
        for i in got:
            np.testing.assert_array_equal(got[i], twin[i])
            worst = max(worst, O.maxrel(got[i], ref[v][i]))
    note(f"wide batch: worst maxrel vs oracle {worst:.2e}")
    assert worst < 1e-4
    batch.close()
    for x in views + twins:
        x.close()


def test_wide_server_coalesces_32_and_matches_oracle():
    """BF16-shadow server with r_coalesce 32 over three views: every request
    is queued before the first round is formed, so each view's requests are
    applied as ceil(count / 32) coalesced updates of up to rank 32; every
    view equals the FP64 oracle."""
    lv = _lv()
    import torch
    mode = lv.LV_FP32_BF16SHADOW
    views = [(1500, 16), (1100, 16), (2100, 8)]
    per_view = (70, 50, 40)
    probe = lv.Server(8 * MiB, mode=mode, r_coalesce=32)
    total = sum(probe.view_bytes(n, k) for n, k in views)
    probe.close()
    srv = lv.Server(8 * MiB + total, mode=mode, r_coalesce=32)
    ids, reqs = {}, []
    for v, (n, k) in enumerate(views):
        A = synth.gaussian_matrix(n, seed=64, config=5, view=v).astype(np.float32)
        ids[v] = srv.add_view(dev(A, torch.float32), k)
        U, V = synth.update_factors(n, 1, per_view[v], seed=65, config=5, view=v)
        reqs += [(v, U[t, :, 0].astype(np.float32), V[t, :, 0].astype(np.float32)) for t in range(per_view[v])]
    order = synth.rng(65, 5, 1).permutation(len(reqs))
    reqs = [reqs[i] for i in order]
    for v, u, w in reqs:
        srv.submit(ids[v], u, w)
    while srv.step() > 0:
        pass
    srv.drain()
    st = srv.stats()
    note(f"wide server stats {st}")
    assert st["submitted"] == st["completed"] == len(reqs)
    assert st["coalesced_updates"] == sum(-(-c // 32) for c in per_view)   # 3 + 2 + 2
    for v, (n, k) in enumerate(views):
        A = synth.gaussian_matrix(n, seed=64, config=5, view=v).astype(np.float32).astype(np.float64)
        U = np.array([u for vv, u, _ in reqs if vv == v], dtype=np.float64)
        W = np.array([w for vv, _, w in reqs if vv == v], dtype=np.float64)
        ref = O.reeval(A + U.T @ W, k)
        worst = 0.0
        for p in ref:
            err = O.maxrel(host(srv.read(ids[v], p)), ref[p])
            worst = max(worst, err)
            assert err < 5e-3, (v, p, err)
        note(f"wide server view {v} n={n}: maxrel vs oracle {worst:.2e}")
    srv.close()
