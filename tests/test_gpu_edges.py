"""Degenerate and boundary cases of the powers view, against closed forms
rather than the oracle's own recurrences:

* order n = 1: every stored power and sum is a scalar power or a geometric
  sum of the updated entry;
* A = I under a rank-1 update: (I + u v^T)^i = I + c_i u v^T with
  c_i = ((1 + v^T u)^i - 1) / (v^T u) (expand the binomial, (u v^T)^j =
  (v^T u)^(j-1) u v^T);
* a nilpotent update (A = 0, u = e_1, v = e_2, so (u v^T)^2 = 0): P_1 = u v^T
  and every higher power is exactly zero, also after the factors of the
  update have been formed in floating point;
* an empty batch (count 0) leaves the view bit-identical and its update
  count unchanged; a rank-0 update is rejected.
"""

from __future__ import annotations

import ctypes

import numpy as np
import pytest

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


def test_order_one_scalar_powers_and_sums():
    lv = _lv()
    import torch
    k, T = 16, 5
    g = synth.rng(90, 0, 1)
    a = 0.9
    us, vs = 0.05 * g.standard_normal(T), 0.05 * g.standard_normal(T)
    view = lv.View(dev(np.array([[a]]), torch.float64), k, sums=True)
    for t in range(T):
        view.update(dev(np.array([[us[t]]]), torch.float64), dev(np.array([[vs[t]]]), torch.float64))
    afin = a + float(np.dot(us, vs))
    for i in view.powers():
        got = host(view.read(i))[0, 0]
        assert abs(got - afin ** i) <= 1e-13 * abs(afin ** i), (i, got, afin ** i)
        s = host(view.read_sum(i))[0, 0]
        ref = sum(afin ** e for e in range(i))
        assert abs(s - ref) <= 1e-13 * abs(ref), (i, s, ref)
    view.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_identity_rank1_closed_form(dtype):
    lv = _lv()
    import torch
    n, k = 300, 32
    td, tol = (torch.float64, 1e-12) if dtype == "f64" else (torch.float32, 2e-6)
    g = synth.rng(91, 0, 1)
    u = (g.standard_normal(n) / np.sqrt(n)).astype(np.float64)
    v = (0.03 * g.standard_normal(n) / np.sqrt(n)).astype(np.float64)
    if dtype == "f32":
        u, v = u.astype(np.float32).astype(np.float64), v.astype(np.float32).astype(np.float64)
    view = lv.View(dev(np.eye(n), td), k)
    view.update(dev(u[:, None], td), dev(v[:, None], td))
    s = float(v @ u)
    uvt = np.outer(u, v)
    for i in view.powers():
        c = ((1.0 + s) ** i - 1.0) / s
        ref = np.eye(n) + c * uvt
        err = np.abs(host(view.read(i)) - ref).max() / np.abs(ref).max()
        assert err < tol, (i, err)
    view.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_nilpotent_update_stays_exactly_zero(dtype):
    lv = _lv()
    import torch
    n, k = 200, 16
    td = torch.float64 if dtype == "f64" else torch.float32
    u, v = np.zeros((n, 1)), np.zeros((n, 1))
    u[0, 0], v[1, 0] = 1.0, 1.0
    view = lv.View(dev(np.zeros((n, n)), td), k)
    view.update(dev(u, td), dev(v, td))
    got = read_all(view)
    np.testing.assert_array_equal(got[1], u @ v.T)
    for i in view.powers()[1:]:
        np.testing.assert_array_equal(got[i], np.zeros((n, n)))
    view.close()


def test_empty_batch_and_rank_zero():
    lv = _lv()
    import torch
    n, k = 400, 8
    A = synth.gaussian_matrix(n, seed=92, config=2)
    Us, Vs = synth.update_factors(n, 2, 3, seed=92, config=2)
    view = lv.View(dev(A, torch.float32), k, r_max=2)
    view.update_batch(dev(Us, torch.float32), dev(Vs, torch.float32))
    before = read_all(view)
    count = view.stats()["updates"]
    empty = torch.zeros(0, n, 2, dtype=torch.float32, device="cuda")
    view.update_batch(empty, empty)
    torch.cuda.synchronize()
    after = read_all(view)
    for i in before:
        np.testing.assert_array_equal(after[i], before[i])
    assert view.stats()["updates"] == count
    buf = torch.zeros(n, 2, dtype=torch.float32, device="cuda")
    st = lv.load().lv_view_update(view.handle, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(buf.data_ptr()), 0,
                                  2, 2, None)
    assert st == lv.LV_EINVAL and "rank" in lv.lv_last_error()
    view.close()
