"""Matrix-power views under the linear, skip-s and exponential models
(lv_chain_*, IncrLin / IncrSkip-s / IncrExp of App. A) against the FP64
oracle (`oracle.reeval_model`, `oracle.incr_update_model`).

Tolerances as for the exponential view: maxrel FP64 1e-10, FP32 1e-4;
deltarel d + 4 sqrt(t) u max|P_t| / max|P_t - P_0| (d = 1e-7 / 1e-2)."""

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


def _lv():
    need_gpu()
    from paper_1403_6968_amd import linview
    return linview


MODEL = {"lin": 1, "exp": 0, "skip": 2}


@pytest.mark.parametrize("model,k,s,n,r,dtype", [
    ("lin", 16, 0, 300, 1, "f64"), ("lin", 8, 0, 1000, 2, "f32"), ("lin", 12, 0, 257, 3, "f32"),
    ("skip", 16, 4, 600, 1, "f32"), ("skip", 16, 2, 300, 2, "f64"), ("skip", 32, 4, 520, 4, "f32"),
    ("exp", 16, 0, 700, 2, "f32"), ("lin", 1, 0, 130, 2, "f32"), ("skip", 8, 8, 384, 1, "f64"),
    ("lin", 32, 0, 256, 4, "f32"), ("skip", 64, 8, 512, 2, "f32")])
def test_models_track_oracle(model, k, s, n, r, dtype):
    lv = _lv()
    import torch
    td, nd = (torch.float64, np.float64) if dtype == "f64" else (torch.float32, np.float32)
    tol, dbase = (1e-10, 1e-7) if dtype == "f64" else (1e-4, 1e-2)
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    T = 6
    sm = s if model == "skip" else None
    A = np.asarray(synth.gaussian_matrix(n, seed=80 + n, config=4), dtype=nd).astype(np.float64)
    Us, Vs = synth.update_factors(n, r, T, seed=80 + n, config=4)
    Us, Vs = (np.asarray(x, dtype=nd).astype(np.float64) for x in (Us, Vs))
    ch = lv.Chain(dev(A, td), k, r_max=r, model=MODEL[model], s=s)
    assert ch.powers() == O.stored_powers(model, k, sm)
    P = O.reeval_model(A, model, k, sm)
    base_ref = P
    base_got = {i: host(ch.read(i)) for i in P}
    create = max(O.maxrel(base_got[i], P[i]) for i in P)
    assert create < (1e-13 if dtype == "f64" else 1e-6)
    for t in range(T):
        ch.update(dev(Us[t], td), dev(Vs[t], td))
        P = O.incr_update_model(P, Us[t], Vs[t], model, k, sm)
    got = {i: host(ch.read(i)) for i in P}
    worst = max(O.maxrel(got[i], P[i]) for i in P)
    wdr = 0.0
    for i in P:
        dr = O.deltarel(got[i], base_got[i], P[i], base_ref[i])
        dtol = dbase + 4 * np.sqrt(T) * u * np.abs(P[i]).max() / np.abs(P[i] - base_ref[i]).max()
        assert dr < dtol, f"P_{i} deltarel {dr:.3e} >= {dtol:.3e}"
        wdr = max(wdr, dr)
    note(f"{model} k={k} s={s} n={n} r={r} {dtype}: create {create:.1e}, maxrel {worst:.2e}, "
         f"worst deltarel {wdr:.2e} over {len(P)} stored")
    assert worst < tol
    ch.close()


def test_models_agree_with_exp_view():
    """P_16 of the linear, skip-4 and exponential chains and of the
    exponential view after the same updates, FP64."""
    lv = _lv()
    import torch
    n, k, T = 400, 16, 5
    A = synth.gaussian_matrix(n, seed=81)
    Us, Vs = synth.update_factors(n, 2, T, seed=81)
    view = lv.View(dev(A, torch.float64), k, r_max=2)
    chains = [lv.Chain(dev(A, torch.float64), k, r_max=2, model=m, s=s)
              for m, s in [(lv.LV_MODEL_LIN, 0), (lv.LV_MODEL_SKIP, 4), (lv.LV_MODEL_EXP, 0)]]
    for t in range(T):
        view.update(dev(Us[t], torch.float64), dev(Vs[t], torch.float64))
        for c in chains:
            c.update(dev(Us[t], torch.float64), dev(Vs[t], torch.float64))
    ref = read_all(view)
    for c in chains:
        for i in c.powers():
            if i in ref:
                assert O.maxrel(host(c.read(i)), ref[i]) < 1e-12
    view.close()
    for c in chains:
        c.close()


def test_models_integer_exact():
    """A DAG adjacency with edge insertions: every stored power is an
    integer matrix below 2^24 (FP32 exact) under all models."""
    lv = _lv()
    import torch
    n, k = 256, 12
    adj = synth.random_dag(n, 0.03, seed=9)
    g = synth.rng(9, 0, 79)
    cur = adj.copy()
    ups = []
    while len(ups) < 4:
        a, b = sorted(g.integers(0, n, size=2))
        if a != b and cur[a, b] == 0:
            cur[a, b] = 1.0
            uu = np.zeros((n, 1)); uu[a] = 1.0
            vv = np.zeros((n, 1)); vv[b] = 1.0
            ups.append((uu, vv))
    for model, s in [("lin", 0), ("skip", 4)]:
        sm = s if model == "skip" else None
        ch = lv.Chain(dev(adj, torch.float32), k, model=MODEL[model], s=s)
        for uu, vv in ups:
            ch.update(dev(uu, torch.float32), dev(vv, torch.float32))
        ref = O.reeval_model(cur, model, k, sm)
        assert max(np.abs(ref[i]).max() for i in ref) < 2 ** 24
        for i in ref:
            np.testing.assert_array_equal(host(ch.read(i)), ref[i], err_msg=f"{model} P_{i}")
        ch.close()


def test_models_errors():
    lv = _lv()
    import torch
    A = dev(synth.gaussian_matrix(64, seed=82), torch.float32)
    with pytest.raises(lv.LinviewError):
        lv.Chain(A, 12, model=lv.LV_MODEL_SKIP, s=8)
    ch = lv.Chain(A, 6, model=lv.LV_MODEL_LIN)
    with pytest.raises(lv.LinviewError):
        ch.read(7)
    with pytest.raises(lv.LinviewError):
        ch.update(dev(np.zeros((64, 2)), torch.float32), dev(np.zeros((64, 2)), torch.float32))  # r > r_max
    ch.close()


@pytest.mark.parametrize("model,k,s,n", [("lin", 5, 0, 3), ("skip", 8, 2, 1), ("exp", 4, 0, 7)])
def test_models_tiny_orders(model, k, s, n):
    """Orders far below one tile (all padding) under every model, FP64."""
    lv = _lv()
    import torch
    sm = s if model == "skip" else None
    A = synth.gaussian_matrix(n, seed=83 + n)
    Us, Vs = synth.update_factors(n, 1, 3, seed=83 + n)
    ch = lv.Chain(dev(A, torch.float64), k, model=MODEL[model], s=s)
    P = O.reeval_model(A, model, k, sm)
    for t in range(3):
        ch.update(dev(Us[t], torch.float64), dev(Vs[t], torch.float64))
        P = O.incr_update_model(P, Us[t], Vs[t], model, k, sm)
    for i in P:
        assert O.maxrel(host(ch.read(i)), P[i]) < 1e-12
    ch.close()
