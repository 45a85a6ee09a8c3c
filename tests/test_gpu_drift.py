"""Drift check and re-anchoring (lv_view_drift_check) against the oracle.

Integer workloads make every quantity exact (FP32 storage of walk counts
below 2^24, double sums of integers below 2^53), so the device residuals
must equal the oracle's chain_residuals bit for bit, and a triggered
re-anchor must restore the exact chain."""

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


def test_fresh_views_have_small_residuals():
    lv = _lv()
    import torch
    for n, dtype, tol in ((1000, torch.float32, 1e-5), (300, torch.float64, 1e-12)):
        A = synth.gaussian_matrix(n, seed=21)
        view = lv.View(dev(A, dtype), 16)
        z = dev(synth.rng(21, 0, 5).standard_normal(n), torch.float64)
        res = host(view.drift_check(z, tau=1e-3))
        note(f"fresh n={n} {dtype}: residuals {res}")
        assert res.shape == (4,) and res.max() < tol
        st = view.stats()
        assert st["drift_reanchors"] == 0 and st["last_residual"] == pytest.approx(res.max())
        view.close()


def test_exact_residuals_and_reanchor_on_integer_chain():
    lv = _lv()
    import torch
    n, k = 384, 16
    adj = synth.random_dag(n, 0.05, seed=6)
    P = O.reeval(adj, k)
    view = lv.View(dev(adj, torch.float32), k)
    for i, M in read_all(view).items():
        np.testing.assert_array_equal(M, P[i])
    # perturb the stored A^2 by 8 at (a, b)
    a, b = 17, 301
    Q = {i: M.copy() for i, M in P.items()}
    Q[2][a, b] += 8.0
    view.write(2, dev(Q[2], torch.float32))
    z_np = (np.arange(n) % 2).astype(np.float64)
    z = dev(z_np, torch.float64)
    want = O.chain_residuals(Q, z_np)
    # a bound it cannot trip: residuals only, no re-anchor
    got = host(view.drift_check(z, tau=1e30))
    note(f"perturbed residuals gpu {got} oracle {want}")
    np.testing.assert_array_equal(got, np.array(want))
    np.testing.assert_array_equal(host(view.read(2)), Q[2])
    assert view.stats()["drift_reanchors"] == 0
    # a bound it trips: the chain is recomputed on the device
    got = host(view.drift_check(z, tau=1e-3))
    np.testing.assert_array_equal(got, np.array(want))
    st = view.stats()
    assert st["drift_reanchors"] == 1
    for i, M in read_all(view).items():
        np.testing.assert_array_equal(M, P[i])
    # clean chain: nothing more happens
    got = host(view.drift_check(z, tau=1e-3))
    assert got.max() == 0.0 and view.stats()["drift_reanchors"] == 1
    view.close()


def test_reanchor_after_perturbation_fp64():
    lv = _lv()
    import torch
    n, k, T = 300, 8, 10
    A = synth.gaussian_matrix(n, seed=22)
    Us, Vs = synth.update_factors(n, 2, T, seed=22)
    view = lv.View(dev(A, torch.float64), k, r_max=2)
    view.update_batch(dev(Us, torch.float64), dev(Vs, torch.float64))
    P = O.apply_updates(O.reeval(A, k), Us, Vs)
    bad = host(view.read(4))
    bad[5, 7] += 1e-3
    view.write(4, dev(bad, torch.float64))
    z = dev(synth.rng(22, 0, 5).standard_normal(n), torch.float64)
    res = host(view.drift_check(z, tau=1e-8))
    note(f"fp64 perturbed residuals {res}")
    assert res.max() > 1e-6 and view.stats()["drift_reanchors"] == 1
    for i, M in read_all(view).items():
        assert O.maxrel(M, P[i]) < 1e-10
    view.close()


def _perturb(lv, torch, view, power, rel, seed):
    """Add a relative perturbation of size rel to stored power `power`."""
    M = host(view.read(power))
    g = synth.rng(seed, 0, 11)
    M = M + rel * np.abs(M).max() * g.standard_normal(M.shape)
    view.write(power, dev(M, view.dtype))


@pytest.mark.parametrize("modename", ["fp32", "bf16shadow", "fp64"])
def test_periodic_check_reanchors_within_interval(modename):
    """Every D-th update runs the check with the mode's default bound: a
    clean chain passes, a perturbed A^k written between two checks is caught
    by the next one and the chain is re-evaluated from the stored A, after
    which the view follows the oracle again."""
    lv = _lv()
    import torch
    mode = {"fp32": lv.LV_FP32, "bf16shadow": lv.LV_FP32_BF16SHADOW, "fp64": lv.LV_FP64}[modename]
    dtype = torch.float64 if mode == lv.LV_FP64 else torch.float32
    np_t = np.float64 if mode == lv.LV_FP64 else np.float32
    n, k, r, D, T = 700, 16, 2, 5, 13
    A = np.asarray(synth.gaussian_matrix(n, seed=23), dtype=np_t).astype(np.float64)
    Us, Vs = synth.update_factors(n, r, T, seed=23)
    Us = np.asarray(Us, dtype=np_t).astype(np.float64)
    Vs = np.asarray(Vs, dtype=np_t).astype(np.float64)
    view = lv.View(dev(A, dtype), k, r_max=r, mode=mode)
    view.set_drift_check(D)
    st = view.stats()
    assert st["drift_every"] == D
    assert st["drift_tau"] == {lv.LV_FP32: 1e-5, lv.LV_FP32_BF16SHADOW: 5e-4, lv.LV_FP64: 1e-11}[mode]
    # updates 1..7 (a check after update 5 finds the chain clean)
    view.update_batch(dev(Us[:7], dtype), dev(Vs[:7], dtype))
    st = view.stats()
    note(f"{modename}: after 7 updates checks={st['drift_checks']} residual={st['last_residual']:.2e}")
    assert st["drift_checks"] == 1 and st["drift_reanchors"] == 0
    assert st["last_residual"] < st["drift_tau"]
    # corrupt A^k: the check after update 10 must catch it and re-anchor
    _perturb(lv, torch, view, k, 1e-2, 24)
    for t in range(7, T):
        view.update(dev(Us[t], dtype), dev(Vs[t], dtype))
    st = view.stats()
    note(f"{modename}: after {T} updates checks={st['drift_checks']} reanchors={st['drift_reanchors']}")
    assert st["drift_checks"] == 2 and st["drift_reanchors"] == 1
    P = O.apply_updates(O.reeval(A, k), Us, Vs)
    tol = {lv.LV_FP32: 1e-4, lv.LV_FP32_BF16SHADOW: 5e-3, lv.LV_FP64: 1e-10}[mode]
    got = read_all(view)
    for i in P:
        err = O.maxrel(got[i], P[i])
        assert err < tol, f"A^{i}: maxrel {err:.2e}"
    view.close()


def test_periodic_check_in_batch_rounds():
    """Batched rounds count as updates of every view and run each view's
    periodic check after the round."""
    lv = _lv()
    import torch
    ns, k, r, D = (512, 768), 8, 1, 3
    views, refs = [], []
    for q, n in enumerate(ns):
        A = np.asarray(synth.gaussian_matrix(n, seed=30 + q), dtype=np.float32).astype(np.float64)
        v = lv.View(dev(A, torch.float32), k, r_max=r)
        v.set_drift_check(D)
        views.append(v)
        refs.append(O.reeval(A, k))
    batch = lv.Batch(views)
    for t in range(7):
        for q, n in enumerate(ns):
            U, V = synth.update_factors(n, r, 1, seed=40 + 10 * t + q)
            U = np.asarray(U[0], dtype=np.float32).astype(np.float64)
            V = np.asarray(V[0], dtype=np.float32).astype(np.float64)
            batch.stage(q, dev(U, torch.float32), dev(V, torch.float32))
            refs[q] = O.incr_update(refs[q], U, V)
        if t == 4:
            _perturb(lv, torch, views[1], k, 1e-2, 25)     # between the checks after rounds 3 and 6
        batch.update()
    torch.cuda.synchronize()
    for q, v in enumerate(views):
        st = v.stats()
        note(f"view {q}: checks={st['drift_checks']} reanchors={st['drift_reanchors']}")
        assert st["drift_checks"] == 2
        assert st["drift_reanchors"] == (1 if q == 1 else 0)
        got = read_all(v)
        for i in refs[q]:
            assert O.maxrel(got[i], refs[q][i]) < 1e-4
    batch.close()
    for v in views:
        v.close()


def test_set_drift_check_arguments():
    lv = _lv()
    import torch
    view = lv.View(torch.zeros(256, 256, device="cuda"), 4)
    with pytest.raises(lv.LinviewError):
        view.set_drift_check(-1)
    with pytest.raises(lv.LinviewError):
        view.set_drift_check(4, float("nan"))
    view.set_drift_check(4, 0.25, dev(np.ones(256), torch.float64))
    st = view.stats()
    assert st["drift_every"] == 4 and st["drift_tau"] == 0.25
    view.set_drift_check(0)
    assert view.stats()["drift_every"] == 0
    view.close()
