"""The general form T_{i+1} = A T_i + B under the linear model (lv_glin_*):
every T_1 .. T_k kept current by re-evaluation, hybrid or incremental
evaluation (App. B, linear model), against the FP64 oracle
(`oracle.reeval_general_lin` of the final A, and the oracle's HybridLin /
IncrLin steps).

Tolerances: maxrel FP64 1e-10, FP32 1e-4; deltarel d + 4 sqrt(t) u max|T_t|
/ max|T_t - T_0| with d = 1e-7 / 1e-2, as for the other views."""

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


def _lv():
    need_gpu()
    from paper_1403_6968_amd import linview
    return linview


def _rounded(x, nd):
    return np.asarray(x, dtype=nd).astype(np.float64)


@pytest.mark.parametrize("strategy", [0, 1, 2])
@pytest.mark.parametrize("n,k,r,p,dtype", [(300, 16, 2, 3, "f64"), (1000, 8, 1, 1, "f32"), (600, 12, 4, 16, "f32"),
                                           (257, 5, 3, 130, "f32"), (384, 16, 1, 64, "f64"), (130, 1, 2, 2, "f32")])
def test_glin_tracks_oracle(strategy, n, k, r, p, dtype):
    lv = _lv()
    import torch
    td, nd = (torch.float64, np.float64) if dtype == "f64" else (torch.float32, np.float32)
    tol, dbase = (1e-10, 1e-7) if dtype == "f64" else (1e-4, 1e-2)
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    T = 6
    A = _rounded(synth.gaussian_matrix(n, seed=90 + n, config=5), nd)
    T0, B = (_rounded(x, nd) for x in synth.general_operands(n, p, seed=90 + n, config=5))
    Us, Vs = (_rounded(x, nd) for x in synth.update_factors(n, r, T, seed=90 + n, config=5))
    g = lv.GLin(dev(A, td), k, dev(T0, td), dev(B, td), r_max=r, strategy=strategy)
    ref0 = O.reeval_general_lin(A, T0, B, k)
    got0 = {i: host(g.read(i)) for i in ref0}
    create = max(O.maxrel(got0[i], ref0[i]) for i in ref0)
    assert create < (1e-13 if dtype == "f64" else 1e-6), create
    Tcur, Acur = dict(ref0), A.copy()
    step = {0: None, 1: O.incr_update_general_hybrid_lin, 2: O.incr_update_general_factored_lin}[strategy]
    for t in range(T):
        g.update(dev(Us[t], td), dev(Vs[t], td))
        if step is not None:
            Acur, Tcur = step(Acur, Tcur, T0, Us[t], Vs[t])
        else:
            Acur = Acur + Us[t] @ Vs[t].T
            Tcur = O.reeval_general_lin(Acur, T0, B, k)
    got = {i: host(g.read(i)) for i in Tcur}
    worst = max(O.maxrel(got[i], Tcur[i]) for i in Tcur)
    wdr = 0.0
    for i in Tcur:
        change = np.abs(Tcur[i] - ref0[i]).max()
        dr = O.deltarel(got[i], got0[i], Tcur[i], ref0[i])
        dtol = dbase + 4 * np.sqrt(T) * u * np.abs(Tcur[i]).max() / change
        assert dr < dtol, f"T_{i} deltarel {dr:.3e} >= {dtol:.3e}"
        wdr = max(wdr, dr)
    note(f"glin strategy={strategy} n={n} k={k} r={r} p={p} {dtype}: create {create:.1e}, maxrel {worst:.2e}, "
         f"worst deltarel {wdr:.2e}")
    assert worst < tol
    np.testing.assert_array_equal(host(g.read(0)), T0)
    g.close()


def test_glin_strategies_agree_b0():
    """B = 0 (the p-sweep setting of the general-form experiment): the three
    strategies give the same T_i in FP64 after the same updates."""
    lv = _lv()
    import torch
    n, k, p = 500, 16, 8
    A = synth.gaussian_matrix(n, seed=91)
    T0 = synth.general_operands(n, p, seed=91)[0]
    B = np.zeros((n, p))
    Us, Vs = synth.update_factors(n, 1, 4, seed=91)
    gs = [lv.GLin(dev(A, torch.float64), k, dev(T0, torch.float64), dev(B, torch.float64), strategy=s)
          for s in (0, 1, 2)]
    for t in range(4):
        for g in gs:
            g.update(dev(Us[t], torch.float64), dev(Vs[t], torch.float64))
    ref = O.reeval_general_lin(A + np.einsum("tir,tjr->ij", Us, Vs), T0, B, k)
    for g in gs:
        for i in ref:
            assert O.maxrel(host(g.read(i)), ref[i]) < 1e-12
        g.close()


def test_glin_errors():
    lv = _lv()
    import torch
    A = dev(synth.gaussian_matrix(64, seed=92), torch.float32)
    T0 = dev(np.zeros((64, 3)), torch.float32)
    with pytest.raises(lv.LinviewError):
        lv.GLin(A, 16, T0, T0, r_max=16, strategy=lv.LV_GLIN_INCR)
    g = lv.GLin(A, 4, T0, T0)
    with pytest.raises(lv.LinviewError):
        g.read(5)
    with pytest.raises(lv.LinviewError):
        g.update(dev(np.zeros((64, 2)), torch.float32), dev(np.zeros((64, 2)), torch.float32))
    g.close()
