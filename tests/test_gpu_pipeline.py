"""Pipelined update_batch: the levels of successive updates run as stages on
streams of their own (App. A: level j of update t needs only P_j after
update t-1 and the factors level j-1 of update t assembled).  Every kernel
sees the inputs of the sequential order, so a pipelined batch must equal the
same batch run sequentially bit for bit, and both must equal the FP64
oracle's re-evaluation of the accumulated matrix within the mode's
tolerance (FP32 1e-4, FP64 1e-10, bfloat16 shadows 5e-3)."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import dev, host, need_gpu, note

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    note(f"start {request.node.nodeid}")
    yield


def _setup(mode_name, n, k, r, T, seed):
    torch = need_gpu()
    from paper_1403_6968_amd import linview as lv
    mode = {"fp32": lv.LV_FP32, "fp64": lv.LV_FP64, "bf16": lv.LV_FP32_BF16SHADOW}[mode_name]
    dt = torch.float64 if mode_name == "fp64" else torch.float32
    npdt = np.float64 if mode_name == "fp64" else np.float32
    A = synth.gaussian_matrix(n, seed=seed, config=7).astype(npdt)
    Us, Vs = synth.update_factors(n, r, T, seed=seed, config=7)
    Us, Vs = Us.astype(npdt), Vs.astype(npdt)
    return torch, lv, mode, dt, A, Us, Vs


def _oracle(A, Us, Vs, k):
    At = A.astype(np.float64) + np.einsum("tir,tjr->ij", Us.astype(np.float64), Vs.astype(np.float64))
    return O.reeval(At, k)


TOL = {"fp32": 1e-4, "fp64": 1e-10, "bf16": 5e-3}


@pytest.mark.parametrize("mode_name,n,k,r", [
    ("fp32", 1000, 16, 1),     # four levels: four stages, five slabs
    ("fp64", 700, 8, 2),       # three stages
    ("bf16", 1100, 16, 1),     # shadows: skinny / update passes per stage
    ("fp32", 513, 4, 4),       # two stages, ragged n
    ("fp32", 2100, 32, 1),     # five levels on four stages (levels 3, 4 share one)
    ("fp32", 600, 16, 4),      # float R = 16 / 32 levels on the matrix cores
])
def test_pipelined_equals_sequential_and_oracle(mode_name, n, k, r):
    torch, lv, mode, dt, A, Us, Vs = _setup(mode_name, n, k, r, 23, seed=11)
    Ad, Ud, Vd = dev(A, dt), dev(Us, dt), dev(Vs, dt)
    a = lv.View(Ad, k, r_max=r, mode=mode)
    b = lv.View(Ad, k, r_max=r, mode=mode)
    b.set_pipeline(False)
    a.update_batch(Ud, Vd)
    b.update_batch(Ud, Vd)
    torch.cuda.synchronize()
    ref = _oracle(A, Us, Vs, k)
    worst = 0.0
    for p in a.powers():
        pa, pb = a.read(p), b.read(p)
        assert torch.equal(pa, pb), f"P{p}: pipelined != sequential"
        err = O.maxrel(host(pa), ref[p])
        worst = max(worst, err)
        assert err < TOL[mode_name], (p, err)
    note(f"{mode_name} n={n} k={k} r={r}: bit-equal, maxrel vs oracle {worst:.2e}")
    assert a.stats()["updates"] == b.stats()["updates"] == 23
    a.close()
    b.close()


def test_pipelined_with_drift_checks_singles_and_other_stream():
    """Periodic drift checks inside a pipelined batch (the stages join and
    fork again), single updates between batches, and a batch on a non-default
    stream: all equal the sequential view bit for bit."""
    torch, lv, mode, dt, A, Us, Vs = _setup("fp32", 900, 16, 1, 40, seed=12)
    Ad, Ud, Vd = dev(A, dt), dev(Us, dt), dev(Vs, dt)
    k = 16
    a = lv.View(Ad, k, r_max=1)
    b = lv.View(Ad, k, r_max=1)
    b.set_pipeline(False)
    for v in (a, b):
        v.set_drift_check(7)
    s = torch.cuda.Stream()
    for v in (a, b):
        v.update_batch(Ud[:17], Vd[:17])
        v.update(Ud[17], Vd[17])
        v.update(Ud[18], Vd[18])
        s.wait_stream(torch.cuda.current_stream())     # the view's earlier work first
        with torch.cuda.stream(s):
            v.update_batch(Ud[19:], Vd[19:], stream=s)
        torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    sa, sb = a.stats(), b.stats()
    assert sa["drift_checks"] == sb["drift_checks"] == 40 // 7
    assert sa["drift_reanchors"] == sb["drift_reanchors"] == 0
    ref = _oracle(A, Us, Vs, k)
    for p in a.powers():
        pa = a.read(p)
        assert torch.equal(pa, b.read(p)), p
        assert O.maxrel(host(pa), ref[p]) < 1e-4, p
    a.close()
    b.close()


def test_two_views_pipelined_concurrently():
    """Two views pipelining batches at the same time on two streams (each
    view's own stage streams): each equals its sequential result."""
    torch, lv, mode, dt, A, Us, Vs = _setup("fp32", 800, 16, 1, 30, seed=13)
    A2 = synth.gaussian_matrix(800, seed=14, config=7).astype(np.float32)
    Ad, A2d, Ud, Vd = dev(A, dt), dev(A2, dt), dev(Us, dt), dev(Vs, dt)
    views = [lv.View(Ad, 16), lv.View(A2d, 16)]
    refs = [lv.View(Ad, 16), lv.View(A2d, 16)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for v, s in zip(views, streams):
        v.update_batch(Ud, Vd, stream=s)
    for v in refs:
        v.set_pipeline(False)
        v.update_batch(Ud, Vd)
    torch.cuda.synchronize()
    for v, w in zip(views, refs):
        for p in v.powers():
            assert torch.equal(v.read(p), w.read(p)), p
        v.close()
        w.close()


@pytest.mark.parametrize("pipelined", [True, False])
def test_autotune_leaves_view_unchanged(pipelined):
    """lv_view_autotune times zero updates only: every stored power and the
    update count are unchanged bit for bit, the chosen height is an allowed
    one and is set on every level; updates after it still equal the
    sequential order with the same tiles and the oracle."""
    torch, lv, mode, dt, A, Us, Vs = _setup("fp32", 1300, 16, 1, 12, seed=15)
    Ad, Ud, Vd = dev(A, dt), dev(Us, dt), dev(Vs, dt)
    a = lv.View(Ad, 16)
    a.update_batch(Ud[:4], Vd[:4])
    torch.cuda.synchronize()
    before = {p: a.read(p) for p in a.powers()}
    rows = a.autotune(pipelined=pipelined, trial_updates=4)
    note(f"pipelined={pipelined}: chose {rows} tile rows")
    assert rows in range(256, 1025, 128)
    assert a.tile_rows() == [rows] * 4
    assert a.stats()["updates"] == 4
    for p in a.powers():
        assert torch.equal(a.read(p), before[p]), p
    b = lv.View(Ad, 16)                      # the same tile history as a: 512, then the chosen rows
    b.set_pipeline(False)
    b.update_batch(Ud[:4], Vd[:4])
    b.set_tile_rows([rows] * 4)
    a.update_batch(Ud[4:], Vd[4:])
    b.update_batch(Ud[4:], Vd[4:])
    ref = _oracle(A, Us, Vs, 16)
    for p in a.powers():
        pa = a.read(p)
        assert torch.equal(pa, b.read(p)), p
        assert O.maxrel(host(pa), ref[p]) < 1e-4
    a.close()
    b.close()


@pytest.mark.parametrize("mode_name,n,k,r", [("fp64", 700, 16, 1), ("bf16", 900, 8, 2), ("fp32", 600, 2, 1)])
def test_autotune_other_modes_and_short_chains(mode_name, n, k, r):
    """The autotuner leaves FP64 and bfloat16-shadow views unchanged bit for
    bit (shadows included: later updates still equal the sequential order),
    and a view with one level (k = 2, no pipeline) takes it as well."""
    torch, lv, mode, dt, A, Us, Vs = _setup(mode_name, n, k, r, 8, seed=16)
    Ad, Ud, Vd = dev(A, dt), dev(Us, dt), dev(Vs, dt)
    a = lv.View(Ad, k, r_max=r, mode=mode)
    a.update_batch(Ud[:3], Vd[:3])
    torch.cuda.synchronize()
    before = {p: a.read(p) for p in a.powers()}
    rows = a.autotune(pipelined=True, trial_updates=3)
    assert rows in range(256, 1025, 128)
    assert a.stats()["updates"] == 3
    for p in a.powers():
        assert torch.equal(a.read(p), before[p]), p
    b = lv.View(Ad, k, r_max=r, mode=mode)
    b.set_pipeline(False)
    b.update_batch(Ud[:3], Vd[:3])
    b.set_tile_rows([rows] * (len(b.powers()) - 1))
    a.update_batch(Ud[3:], Vd[3:])
    b.update_batch(Ud[3:], Vd[3:])
    ref = _oracle(A, Us, Vs, k)
    for p in a.powers():
        pa = a.read(p)
        assert torch.equal(pa, b.read(p)), p
        assert O.maxrel(host(pa), ref[p]) < TOL[mode_name], p
    a.close()
    b.close()
