"""Least squares kept current under rank-1 changes of the data (lv_ols_*,
Sec. 5.1 with Sherman-Morrison) against the FP64 oracle
(`oracle.incr_update_ols`, `oracle.reeval_ols`) and numpy's lstsq.

Tolerances: FP64 maxrel 1e-10; FP32 1e-4 for W and beta (X^T X of these
workloads has a condition number near 35, so FP32 storage of W alone
contributes about 35 * 2^-24 ~ 2e-6 per update)."""

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


def _data(m, n, p, seed, nd):
    g = synth.rng(seed, 0, 93)
    X = np.asarray(g.standard_normal((m, n)), dtype=nd).astype(np.float64)
    Y = np.asarray(g.standard_normal((m, p)), dtype=nd).astype(np.float64)
    return X, Y, g


@pytest.mark.parametrize("m,n,p,dtype", [(600, 300, 3, "f64"), (2000, 1000, 1, "f32"), (520, 257, 64, "f32"),
                                         (1024, 512, 8, "f64"), (300, 130, 5, "f32")])
def test_ols_tracks_oracle(m, n, p, dtype):
    lv = _lv()
    import torch
    td, nd = (torch.float64, np.float64) if dtype == "f64" else (torch.float32, np.float32)
    tol = 1e-10 if dtype == "f64" else 1e-4
    X, Y, g = _data(m, n, p, 100 + n, nd)
    ols = lv.Ols(dev(X, td), dev(Y, td))
    W, beta = O.reeval_ols(X, Y)
    cW = O.maxrel(host(ols.read(lv.LV_OLS_INVERSE)), W)
    cb = O.maxrel(host(ols.read(lv.LV_OLS_BETA)), beta)
    assert cW < (1e-11 if dtype == "f64" else 1e-5) and cb < (1e-11 if dtype == "f64" else 1e-5), (cW, cb)
    T = 8
    for t in range(T):
        if t % 2:
            row = int(g.integers(0, m))
            dx = np.asarray(g.standard_normal((n, 1)) * 0.3, dtype=nd).astype(np.float64)
            u = np.zeros((m, 1)); u[row] = 1.0
            ols.update_row(row, dev(dx[:, 0], td))
            X, W, beta = O.incr_update_ols(X, Y, W, beta, u, dx)
        else:
            u = np.asarray(g.standard_normal((m, 1)) * 0.05, dtype=nd).astype(np.float64)
            v = np.asarray(g.standard_normal((n, 1)) * 0.3, dtype=nd).astype(np.float64)
            ols.update(dev(u[:, 0], td), dev(v[:, 0], td))
            X, W, beta = O.incr_update_ols(X, Y, W, beta, u, v)
    gW, gb, gX = host(ols.read(lv.LV_OLS_INVERSE)), host(ols.read(lv.LV_OLS_BETA)), host(ols.read(lv.LV_OLS_X))
    eW, eb, eX = O.maxrel(gW, W), O.maxrel(gb, beta), O.maxrel(gX, X)
    note(f"ols m={m} n={n} p={p} {dtype}: newton-schulz {ols.info()}, create W {cW:.1e} beta {cb:.1e}; "
         f"after {T} updates W {eW:.2e} beta {eb:.2e} X {eX:.1e}")
    assert eW < tol and eb < tol and eX < (1e-15 if dtype == "f64" else 1e-6)
    ols.close()


def test_ols_against_lstsq_full_size():
    """n = 4096, m = 8192, p = 16, FP32, 10 row changes: beta against numpy's
    least-squares solution of the final data (a different method)."""
    lv = _lv()
    import torch
    m, n, p, T = 8192, 4096, 16, 10
    X, Y, g = _data(m, n, p, 7, np.float32)
    ols = lv.Ols(dev(X, torch.float32), dev(Y, torch.float32))
    for t in range(T):
        row = int(g.integers(0, m))
        dx = np.asarray(g.standard_normal(n) * 0.3, dtype=np.float32)
        ols.update_row(row, dev(dx, torch.float32))
        X[row] += dx.astype(np.float64)
    ref = np.linalg.lstsq(X, Y, rcond=None)[0]
    got = host(ols.read(lv.LV_OLS_BETA))
    err = O.maxrel(got, ref)
    note(f"ols full size m={m} n={n} p={p}: beta maxrel vs lstsq {err:.2e}, {ols.info()}")
    assert err < 1e-4
    ols.close()


def test_ols_row_update_equals_dense_form_bitwise():
    lv = _lv()
    import torch
    m, n, p = 700, 300, 4
    X, Y, g = _data(m, n, p, 8, np.float32)
    a = lv.Ols(dev(X, torch.float32), dev(Y, torch.float32))
    b = lv.Ols(dev(X, torch.float32), dev(Y, torch.float32))
    for t in range(4):
        row = int(g.integers(0, m))
        dx = np.asarray(g.standard_normal(n) * 0.3, dtype=np.float32)
        u = np.zeros(m, dtype=np.float32); u[row] = 1.0
        a.update_row(row, dev(dx, torch.float32))
        b.update(dev(u, torch.float32), dev(dx, torch.float32))
    for what in (lv.LV_OLS_BETA, lv.LV_OLS_INVERSE, lv.LV_OLS_X):
        np.testing.assert_array_equal(host(a.read(what)), host(b.read(what)))
    a.close()
    b.close()


def test_ols_errors():
    lv = _lv()
    import torch
    m, n = 400, 100
    X, Y, _ = _data(m, n, 2, 9, np.float64)
    X[:, 5] = X[:, 7]                                           # rank deficient: X^T X singular
    with pytest.raises(lv.LinviewError):
        lv.Ols(dev(X, torch.float64), dev(Y, torch.float64))
    X, Y, _ = _data(m, n, 2, 9, np.float64)
    ols = lv.Ols(dev(X, torch.float64), dev(Y, torch.float64))
    with pytest.raises(lv.LinviewError):
        ols.update_row(m, dev(np.zeros(n), torch.float64))
    with pytest.raises(ValueError):
        ols.update(dev(np.zeros(m - 1), torch.float64), dev(np.zeros(n), torch.float64))
    ols.close()


@pytest.mark.parametrize("m,n,p", [(9, 3, 2), (5, 1, 1)])
def test_ols_tiny(m, n, p):
    """Orders far below one tile (all padding), FP64, dense and row changes."""
    lv = _lv()
    import torch
    X, Y, g = _data(m, n, p, 20 + m, np.float64)
    ols = lv.Ols(dev(X, torch.float64), dev(Y, torch.float64))
    W, beta = O.reeval_ols(X, Y)
    for t in range(4):
        if t % 2:
            row = int(g.integers(0, m))
            dx = g.standard_normal((n, 1)) * 0.3
            u = np.zeros((m, 1)); u[row] = 1.0
            ols.update_row(row, dev(dx[:, 0], torch.float64))
            X, W, beta = O.incr_update_ols(X, Y, W, beta, u, dx)
        else:
            u, v = g.standard_normal((m, 1)) * 0.1, g.standard_normal((n, 1)) * 0.3
            ols.update(dev(u[:, 0], torch.float64), dev(v[:, 0], torch.float64))
            X, W, beta = O.incr_update_ols(X, Y, W, beta, u, v)
    assert O.maxrel(host(ols.read(lv.LV_OLS_BETA)), beta) < 1e-10
    assert O.maxrel(host(ols.read(lv.LV_OLS_INVERSE)), W) < 1e-10
    ols.close()
