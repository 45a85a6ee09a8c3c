"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Sizes span several tiles and a ragged edge (n not a multiple of the 256
padding order).  Tolerances (normwise max-norm, `oracle.maxrel`):
  FP64 views       1e-10  (rounding of n-term double sums, k = 16)
  FP32 views       1e-4   (the stated FP32 tolerance)
  FP32 deltarel    1e-2   (accumulated change vs the reference change)
Integer-valued workloads (DAG walk counts) must match bit for bit.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import dev, host, need_gpu, note, read_all, report, storage_inputs

pytestmark = pytest.mark.gpu


def _lv():
    need_gpu()
    from paper_1403_6968_amd import linview
    return linview


@pytest.fixture(autouse=True)
def _announce(request):
    note(f"start {request.node.nodeid}")
    yield


# ---------------------------------------------------------------- creation

@pytest.mark.parametrize("n,k,dtype", [(256, 16, "f64"), (1000, 16, "f32"), (300, 8, "f64"),
                                       (5, 4, "f32"), (1, 2, "f64"), (513, 1, "f32")])
def test_create_matches_reeval(n, k, dtype):
    lv = _lv()
    import torch
    td, nd = (torch.float64, np.float64) if dtype == "f64" else (torch.float32, np.float32)
    A64 = synth.gaussian_matrix(n, seed=1, config=1)
    A = np.asarray(A64, dtype=nd)
    view = lv.View(dev(A, td), k)
    ref = O.reeval(A.astype(np.float64), k)
    got = read_all(view)
    tol = 1e-12 if dtype == "f64" else 1e-6
    res = report(f"create n={n} k={k} {dtype}", got, ref)
    for i, (mr, _) in res.items():
        assert mr < tol, f"P_{i}"
    view.close()


# ---------------------------------------------------------------- updates

def _run_updates(lv, n, k, r, T, dtype, seed, check_every, tol, dtol=None, batch=False, tiles=None):
    import torch
    td, nd = (torch.float64, np.float64) if dtype == "f64" else (torch.float32, np.float32)
    A64 = synth.gaussian_matrix(n, seed=seed, config=2)
    Us64, Vs64 = synth.update_factors(n, r, T, seed=seed, config=2)
    A, Us, Vs = storage_inputs(A64, Us64, Vs64, nd)
    view = lv.View(dev(A, td), k, r_max=r)
    if tiles is not None:
        view.set_tile_rows([tiles] * (len(view.powers()) - 1))
    P0_ref = O.reeval(A, k)
    P0_got = read_all(view)
    P = dict(P0_ref)
    Ud, Vd = dev(Us, td), dev(Vs, td)
    t = 0
    while t < T:
        step = min(check_every, T - t)
        if batch:
            view.update_batch(Ud[t:t + step], Vd[t:t + step])
        else:
            for s in range(t, t + step):
                view.update(Ud[s], Vd[s])
        P = O.apply_updates(P, Us[t:t + step], Vs[t:t + step])
        t += step
        got = read_all(view)
        res = report(f"n={n} k={k} r={r} {dtype} after {t}", got, P, P0_got, P0_ref)
        for i, (mr, dr) in res.items():
            assert mr < tol, f"P_{i} maxrel {mr:.3e} after {t} updates"
            if dtol is not None:
                assert dr < dtol, f"P_{i} deltarel {dr:.3e} after {t} updates"
    # the incremental oracle itself agrees with re-evaluation of the final A
    Afin = A + np.einsum("tir,tjr->ij", Us, Vs)
    R = O.reeval(Afin, k)
    for i in P:
        assert O.maxrel(P[i], R[i]) < 1e-11
    assert view.stats()["updates"] == T
    return view


def test_cfg1_fp64_n256_k16_100_updates():
    """Matrix-power view A^16, n = 256, FP64, 100 rank-1 updates."""
    lv = _lv()
    v = _run_updates(lv, 256, 16, 1, 100, "f64", seed=0, check_every=25, tol=1e-10, dtol=1e-7)
    v.close()


def test_fp32_ragged_n1000():
    lv = _lv()
    v = _run_updates(lv, 1000, 16, 1, 40, "f32", seed=1, check_every=20, tol=1e-4, dtol=1e-2)
    v.close()


@pytest.mark.parametrize("n,k,r,dtype", [(600, 8, 2, "f32"), (300, 4, 3, "f64"), (257, 2, 1, "f32"),
                                         (70, 16, 1, "f64"), (130, 1, 4, "f64"), (1024, 16, 1, "f32"),
                                         (520, 4, 4, "f64"), (256, 2, 8, "f32"),
                                         # level ranks above 16: chunked skinny passes + Gram kernel
                                         (600, 16, 4, "f32"), (520, 16, 8, "f64"), (300, 256, 1, "f64"),
                                         (777, 32, 3, "f32")])
def test_updates_shapes(n, k, r, dtype):
    lv = _lv()
    tol = 1e-10 if dtype == "f64" else 1e-4
    dtol = 1e-7 if dtype == "f64" else 2e-2
    v = _run_updates(lv, n, k, r, 12, dtype, seed=n + k + r, check_every=6, tol=tol, dtol=dtol)
    v.close()


@pytest.mark.parametrize("tiles,dtype,r", [(256, "f32", 1), (1024, "f32", 4), (256, "f64", 2), (1024, "f64", 1)])
def test_tile_rows_settings(tiles, dtype, r):
    """Every allowed tile height gives a correct update (the partial counts of
    the tail follow the tile height); n = 1300 leaves a ragged last tile."""
    lv = _lv()
    tol = 1e-10 if dtype == "f64" else 1e-4
    v = _run_updates(lv, 1300, 16, r, 6, dtype, seed=77 + tiles, check_every=3, tol=tol, tiles=tiles)
    assert v.tile_rows() == [tiles] * 4
    with pytest.raises(lv.LinviewError):
        lv.lv_view_set_tile_rows(v.handle, 0, 200)
    with pytest.raises(lv.LinviewError):
        lv.lv_view_set_tile_rows(v.handle, 4, 512)      # the top level has no level pass
    v.close()


def test_update_batch_equals_sequential_bitwise():
    lv = _lv()
    import torch
    n, k, T = 700, 16, 9
    A64 = synth.gaussian_matrix(n, seed=4)
    Us64, Vs64 = synth.update_factors(n, 1, T, seed=4)
    A, Us, Vs = storage_inputs(A64, Us64, Vs64, np.float32)
    a = lv.View(dev(A, torch.float32), k)
    b = lv.View(dev(A, torch.float32), k)
    Ud, Vd = dev(Us, torch.float32), dev(Vs, torch.float32)
    for t in range(T):
        a.update(Ud[t], Vd[t])
    b.update_batch(Ud, Vd)
    for i in a.powers():
        assert torch.equal(a.read(i), b.read(i)), f"P_{i}"
    a.close(); b.close()


def test_deterministic_bitwise():
    lv = _lv()
    import torch
    n, k, T = 800, 16, 5
    A64 = synth.gaussian_matrix(n, seed=5)
    Us64, Vs64 = synth.update_factors(n, 2, T, seed=5)
    A, Us, Vs = storage_inputs(A64, Us64, Vs64, np.float32)
    outs = []
    for _ in range(2):
        v = lv.View(dev(A, torch.float32), k, r_max=2)
        v.update_batch(dev(Us, torch.float32), dev(Vs, torch.float32))
        outs.append([v.read(i) for i in v.powers()])
        v.close()
    for x, y in zip(*outs):
        assert torch.equal(x, y)


def test_dag_walk_counts_bit_exact_fp32():
    """Edge insertions into a DAG: every stored power holds integer walk
    counts; FP32 arithmetic is exact below 2^24, so the GPU must match the
    oracle bit for bit."""
    lv = _lv()
    import torch
    n, k = 384, 16
    adj = synth.random_dag(n, 0.05, seed=6)
    g = synth.rng(6, 0, 77)
    edges = []
    while len(edges) < 6:
        a, b = sorted(g.integers(0, n, size=2))
        if a != b and adj[a, b] == 0:
            edges.append((a, b))
    view = lv.View(dev(adj, torch.float32), k)
    P = O.reeval(adj, k)
    for a, b in edges:
        u = np.zeros((n, 1)); u[a] = 1.0
        v = np.zeros((n, 1)); v[b] = 1.0
        view.update(dev(u, torch.float32), dev(v, torch.float32))
        P = O.incr_update(P, u, v)
    assert max(np.abs(P[i]).max() for i in P) < 2 ** 24
    got = read_all(view)
    for i in P:
        np.testing.assert_array_equal(got[i], P[i])
    view.close()


def test_zero_update_leaves_view_unchanged():
    lv = _lv()
    import torch
    n, k = 500, 16
    A = np.asarray(synth.gaussian_matrix(n, seed=7), dtype=np.float32)
    view = lv.View(dev(A, torch.float32), k)
    before = [view.read(i) for i in view.powers()]
    V = dev(synth.update_factors(n, 1, 1, seed=7)[1][0], torch.float32)
    view.update(torch.zeros_like(V), V)
    for i, b in zip(view.powers(), before):
        assert torch.equal(view.read(i), b)
    view.close()


def test_rank_r_update_equals_r_rank1_updates_fp64():
    lv = _lv()
    import torch
    n, k, r = 400, 8, 4
    A = synth.gaussian_matrix(n, seed=8)
    U, V = synth.update_factors(n, r, 1, seed=8)
    a = lv.View(dev(A, torch.float64), k, r_max=r)
    b = lv.View(dev(A, torch.float64), k, r_max=r)
    a.update(dev(U[0], torch.float64), dev(V[0], torch.float64))
    for c in range(r):
        b.update(dev(U[0][:, [c]], torch.float64), dev(V[0][:, [c]], torch.float64))
    ref = O.reeval(A + U[0] @ V[0].T, k)
    for i in a.powers():
        assert O.maxrel(host(a.read(i)), ref[i]) < 1e-11
        assert O.maxrel(host(b.read(i)), ref[i]) < 1e-11
    a.close(); b.close()


def test_reanchor_restores_chain():
    lv = _lv()
    import torch
    n, k, T = 512, 16, 20
    A64 = synth.gaussian_matrix(n, seed=9)
    Us64, Vs64 = synth.update_factors(n, 1, T, seed=9)
    A, Us, Vs = storage_inputs(A64, Us64, Vs64, np.float32)
    view = lv.View(dev(A, torch.float32), k)
    view.update_batch(dev(Us, torch.float32), dev(Vs, torch.float32))
    view.reanchor()
    P1 = host(view.read(1))
    ref = O.reeval(P1, k)             # exact chain of the stored A
    for i in view.powers():
        assert O.maxrel(host(view.read(i)), ref[i]) < 1e-6
    assert view.stats()["reanchors"] == 1
    view.close()


# ---------------------------------------------------------------- re-evaluation baseline

@pytest.mark.parametrize("n,k,dtype", [(256, 16, "f64"), (1000, 16, "f32"), (384, 4, "f32")])
def test_reeval_baseline(n, k, dtype):
    lv = _lv()
    import torch
    td, nd = (torch.float64, np.float64) if dtype == "f64" else (torch.float32, np.float32)
    A64 = synth.gaussian_matrix(n, seed=10)
    Us64, Vs64 = synth.update_factors(n, 1, 1, seed=10)
    A, Us, Vs = storage_inputs(A64, Us64, Vs64, nd)
    out = lv.reeval(dev(A, td), k, dev(Us[0], td), dev(Vs[0], td))
    ref = O.reeval(A + Us[0] @ Vs[0].T, k)[k]
    mr = O.maxrel(host(out), ref)
    note(f"reeval n={n} k={k} {dtype}: maxrel={mr:.2e}")
    assert mr < (1e-12 if dtype == "f64" else 1e-4)


# ---------------------------------------------------------------- errors on device calls

def test_bad_arguments_raise():
    lv = _lv()
    import torch
    A = torch.zeros(64, 64, dtype=torch.float32, device="cuda")
    with pytest.raises(lv.LinviewError):
        lv.View(A, 3)
    with pytest.raises(lv.LinviewError):
        lv.View(A, 16, r_max=0)
    view = lv.View(A, 4, r_max=1)
    U = torch.zeros(64, 2, dtype=torch.float32, device="cuda")
    with pytest.raises(lv.LinviewError):
        view.update(U, U)                       # rank above r_max
    with pytest.raises(lv.LinviewError):
        view.read(3)
    with pytest.raises(TypeError):
        view.update(U[:, :1].double(), U[:, :1].double())
    view.close()
