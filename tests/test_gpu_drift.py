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
