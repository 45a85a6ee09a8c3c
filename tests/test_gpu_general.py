"""General-form views: T_i of T_{i+1} = A T_i + B (i in {1, 2, 4, ..., k})
kept current under updates of A by hybrid evaluation, against the FP64
oracle (`oracle.reeval_general`, `oracle.incr_update_general`) and, at full
size, against the defining iteration (`oracle.iterate_general`).

Tolerances as for the powers and sums: maxrel FP64 1e-10, FP32 1e-4,
BF16-shadow mode 5e-3; deltarel d + 4 sqrt(t) u max|T_t| / max|T_t - T_0|
with the storage unit roundoff u and d = 1e-7 / 1e-2 / 5e-2; integer
results of a DAG bit for bit."""

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


def _ts(view):
    return {i: host(view.read_general(i)) for i in view.powers()}


def _rounded(x, nd):
    return np.asarray(x, dtype=nd).astype(np.float64)


@pytest.mark.parametrize("n,k,r,p,dtype,mode", [
    (300, 16, 2, 3, "f64", "f64"), (1000, 16, 1, 1, "f32", "f32"), (600, 16, 4, 16, "f32", "f32"),
    (257, 32, 3, 5, "f32", "f32"), (520, 8, 8, 64, "f64", "f64"), (700, 16, 2, 8, "f32", "bf16"),
    (130, 1, 2, 2, "f32", "f32"), (400, 4, 1, 32, "f32", "f32"), (384, 16, 1, 64, "f32", "f32")])
def test_general_tracks_oracle(n, k, r, p, dtype, mode):
    lv = _lv()
    import torch
    td, nd = (torch.float64, np.float64) if dtype == "f64" else (torch.float32, np.float32)
    lvmode = {"f64": lv.LV_FP64, "f32": lv.LV_FP32, "bf16": lv.LV_FP32_BF16SHADOW}[mode]
    tol = {"f64": 1e-10, "f32": 1e-4, "bf16": 5e-3}[mode]
    dbase = {"f64": 1e-7, "f32": 1e-2, "bf16": 5e-2}[mode]
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    T = 8
    A = _rounded(synth.gaussian_matrix(n, seed=60 + n, config=3), nd)
    T0, B = (_rounded(x, nd) for x in synth.general_operands(n, p, seed=60 + n, config=3))
    Us, Vs = (_rounded(x, nd) for x in synth.update_factors(n, r, T, seed=60 + n, config=3))
    view = lv.View(dev(A, td), k, r_max=r, mode=lvmode, general=(dev(T0, td), dev(B, td)))
    plain = lv.View(dev(A, td), k, r_max=r, mode=lvmode, sums=True)
    P, S, Tr = O.reeval(A, k), O.reeval_sums(A, k), O.reeval_general(A, T0, B, k)
    T_ref0, T_got0 = Tr, _ts(view)
    create_err = max(O.maxrel(T_got0[i], Tr[i]) for i in Tr)
    assert create_err < (1e-13 if dtype == "f64" else 1e-6), create_err
    for t in range(T):
        view.update(dev(Us[t], td), dev(Vs[t], td))
        plain.update(dev(Us[t], td), dev(Vs[t], td))
        P, S, Tr = O.incr_update_general(P, S, Tr, T0, B, Us[t], Vs[t])
    got = _ts(view)
    worst = max(O.maxrel(got[i], Tr[i]) for i in Tr)
    msg = []
    for i in Tr:
        dr = O.deltarel(got[i], T_got0[i], Tr[i], T_ref0[i])
        dtol = dbase + 4 * np.sqrt(T) * u * np.abs(Tr[i]).max() / np.abs(Tr[i] - T_ref0[i]).max()
        msg.append(f"T{i}: {dr:.1e}(<{dtol:.1e})")
        assert dr < dtol, f"T_{i} deltarel {dr:.3e} >= {dtol:.3e}"
    note(f"general n={n} k={k} r={r} p={p} {mode}: create {create_err:.1e}, after {T} updates maxrel "
         f"{worst:.2e}; " + " ".join(msg))
    assert worst < tol
    # powers and sums of a general-form view equal those of a sums view bit for bit
    pw, pp = read_all(view), read_all(plain)
    for i in pw:
        np.testing.assert_array_equal(pw[i], pp[i])
    for i in view.powers():
        np.testing.assert_array_equal(host(view.read_sum(i)), host(plain.read_sum(i)))
    view.close()
    plain.close()


def test_general_dag_exact():
    """A DAG adjacency with 0/1 T_0 and B: every T_i is an integer below
    2^24 under edge insertions, so FP32 is exact."""
    lv = _lv()
    import torch
    n, k, p = 384, 16, 3
    adj = synth.random_dag(n, 0.03, seed=8)
    g = synth.rng(8, 0, 78)
    T0 = g.integers(0, 2, size=(n, p)).astype(np.float64)
    B = g.integers(0, 2, size=(n, p)).astype(np.float64)
    cur = adj.copy()
    ups = []
    while len(ups) < 5:
        a, b = sorted(g.integers(0, n, size=2))
        if a != b and cur[a, b] == 0:
            cur[a, b] = 1.0
            uu = np.zeros((n, 1)); uu[a] = 1.0
            vv = np.zeros((n, 1)); vv[b] = 1.0
            ups.append((uu, vv))
    view = lv.View(dev(adj, torch.float32), k, general=(dev(T0, torch.float32), dev(B, torch.float32)))
    P, S, Tr = O.reeval(adj, k), O.reeval_sums(adj, k), O.reeval_general(adj, T0, B, k)
    for uu, vv in ups:
        view.update(dev(uu, torch.float32), dev(vv, torch.float32))
        P, S, Tr = O.incr_update_general(P, S, Tr, T0, B, uu, vv)
    top = max(np.abs(Tr[i]).max() for i in Tr)
    assert top < 2 ** 24
    got = _ts(view)
    for i in Tr:
        np.testing.assert_array_equal(got[i], Tr[i], err_msg=f"T_{i}")
    note(f"dag general: max entry {top:.0f}")
    view.close()


def test_general_regression_workload():
    """Gradient-descent regression (A = I - eta X^T X, B = eta X^T Y) with
    new training rows as rank-1 changes of A, FP32, against the oracle."""
    lv = _lv()
    import torch
    n, p, k, T = 512, 4, 16, 6
    A, B, eta = synth.regression_problem(n, p, 2 * n, seed=5)
    A, B = _rounded(A, np.float32), _rounded(B, np.float32)
    T0 = np.zeros((n, p))
    Us, Vs = (_rounded(x, np.float32) for x in synth.regression_rows(n, T, eta, seed=5))
    view = lv.View(dev(A, torch.float32), k, general=(dev(T0, torch.float32), dev(B, torch.float32)))
    P, S, Tr = O.reeval(A, k), O.reeval_sums(A, k), O.reeval_general(A, T0, B, k)
    for t in range(T):
        view.update(dev(Us[t], torch.float32), dev(Vs[t], torch.float32))
        P, S, Tr = O.incr_update_general(P, S, Tr, T0, B, Us[t], Vs[t])
    got = _ts(view)
    worst = max(O.maxrel(got[i], Tr[i]) for i in Tr)
    note(f"regression n={n} p={p}: maxrel {worst:.2e}")
    assert worst < 1e-4
    view.close()


@pytest.mark.parametrize("n,p,mode", [(8192, 16, "f32"), (8192, 1, "bf16"), (8192, 1, "f32")])
def test_general_full_size_against_iteration(n, p, mode):
    """n = 8192, k = 16, rank 1, 12 updates; every stored T_i against the
    defining iteration on the final A (no powers formed on the host)."""
    lv = _lv()
    import torch
    k, T = 16, 12
    lvmode = lv.LV_FP32 if mode == "f32" else lv.LV_FP32_BF16SHADOW
    A = _rounded(synth.gaussian_matrix(n, seed=61, config=3), np.float32)
    T0, B = (_rounded(x, np.float32) for x in synth.general_operands(n, p, seed=61, config=3))
    Us, Vs = (_rounded(x, np.float32) for x in synth.update_factors(n, 1, T, seed=61, config=3))
    view = lv.View(dev(A, torch.float32), k, mode=lvmode, general=(dev(T0, torch.float32), dev(B, torch.float32)))
    base_got = _ts(view)
    base_ref = O.iterate_general(A, T0, B, k)
    for t in range(T):
        view.update(dev(Us[t], torch.float32), dev(Vs[t], torch.float32))
    Afin = A + np.einsum("tir,tjr->ij", Us, Vs)
    ref = O.iterate_general(Afin, T0, B, k)
    got = _ts(view)
    u = 2.0 ** -24
    tol, dbase = (1e-4, 1e-2) if mode == "f32" else (5e-3, 5e-2)
    msg = []
    for i in ref:
        mr = O.maxrel(got[i], ref[i])
        dr = O.deltarel(got[i], base_got[i], ref[i], base_ref[i])
        dtol = dbase + 4 * np.sqrt(T) * u * np.abs(ref[i]).max() / np.abs(ref[i] - base_ref[i]).max()
        msg.append(f"T{i}: {mr:.1e}/{dr:.1e}(<{dtol:.1e})")
        assert mr < tol, f"T_{i} maxrel {mr:.3e}"
        assert dr < dtol, f"T_{i} deltarel {dr:.3e} >= {dtol:.3e}"
    note(f"general full size n={n} p={p} {mode}: " + " ".join(msg))
    view.close()


def test_general_reanchor_and_errors():
    lv = _lv()
    import torch
    n, k, p = 400, 8, 6
    A = _rounded(synth.gaussian_matrix(n, seed=62), np.float32)
    T0, B = (_rounded(x, np.float32) for x in synth.general_operands(n, p, seed=62))
    Us, Vs = (_rounded(x, np.float32) for x in synth.update_factors(n, 1, 3, seed=62))
    view = lv.View(dev(A, torch.float32), k, general=(dev(T0, torch.float32), dev(B, torch.float32)))
    for t in range(3):
        view.update(dev(Us[t], torch.float32), dev(Vs[t], torch.float32))
    view.reanchor()
    Afin = host(view.read(1))
    ref = O.reeval_general(Afin, T0, B, k)
    got = _ts(view)
    assert max(O.maxrel(got[i], ref[i]) for i in ref) < 1e-6
    # batched updates give the same T bit for bit as single updates
    twin = lv.View(dev(A, torch.float32), k, general=(dev(T0, torch.float32), dev(B, torch.float32)))
    twin.update_batch(dev(Us, torch.float32), dev(Vs, torch.float32))
    single = lv.View(dev(A, torch.float32), k, general=(dev(T0, torch.float32), dev(B, torch.float32)))
    for t in range(3):
        single.update(dev(Us[t], torch.float32), dev(Vs[t], torch.float32))
    g1, g2 = _ts(twin), _ts(single)
    for i in g1:
        np.testing.assert_array_equal(g1[i], g2[i])
    plain = lv.View(dev(A, torch.float32), k, sums=True)
    with pytest.raises(lv.LinviewError) as e:
        plain.read_general(2)
    assert e.value.status == lv.LV_ESTATE
    with pytest.raises(lv.LinviewError):
        lv.Batch([view])                                  # general views are single-view only
    with pytest.raises(lv.LinviewError):
        view.read_general(3)
    with pytest.raises(lv.LinviewError):
        lv.View(dev(A, torch.float32), k, general=(dev(np.zeros((n, 65)), torch.float32),
                                                    dev(np.zeros((n, 65)), torch.float32)))
    for x in (view, twin, single, plain):
        x.close()


# ---- factored (incremental) deltas, App. B


@pytest.mark.parametrize("n,k,r,p,dtype,mode", [
    (300, 16, 2, 3, "f64", "f64"), (1000, 16, 1, 1, "f32", "f32"), (600, 8, 4, 200, "f32", "f32"),
    (257, 32, 3, 5, "f32", "f32"), (520, 8, 8, 130, "f64", "f64"), (700, 16, 2, 8, "f32", "bf16"),
    (130, 1, 2, 2, "f32", "f32"), (384, 16, 1, 1000, "f32", "f32")])
def test_general_factored_tracks_oracle(n, k, r, p, dtype, mode):
    lv = _lv()
    import torch
    td, nd = (torch.float64, np.float64) if dtype == "f64" else (torch.float32, np.float32)
    lvmode = {"f64": lv.LV_FP64, "f32": lv.LV_FP32, "bf16": lv.LV_FP32_BF16SHADOW}[mode]
    tol = {"f64": 1e-10, "f32": 1e-4, "bf16": 5e-3}[mode]
    dbase = {"f64": 1e-7, "f32": 1e-2, "bf16": 5e-2}[mode]
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    T = 8
    A = _rounded(synth.gaussian_matrix(n, seed=70 + n, config=3), nd)
    T0, B = (_rounded(x, nd) for x in synth.general_operands(n, p, seed=70 + n, config=3))
    Us, Vs = (_rounded(x, nd) for x in synth.update_factors(n, r, T, seed=70 + n, config=3))
    view = lv.View(dev(A, td), k, r_max=r, mode=lvmode, general=(dev(T0, td), dev(B, td)),
                   strategy=lv.LV_GENERAL_FACTORED)
    plain = lv.View(dev(A, td), k, r_max=r, mode=lvmode, sums=True)
    P, S, Tr = O.reeval(A, k), O.reeval_sums(A, k), O.reeval_general(A, T0, B, k)
    T_ref0, T_got0 = Tr, _ts(view)
    create_err = max(O.maxrel(T_got0[i], Tr[i]) for i in Tr)
    assert create_err < (1e-13 if dtype == "f64" else 1e-6), create_err
    for t in range(T):
        view.update(dev(Us[t], td), dev(Vs[t], td))
        plain.update(dev(Us[t], td), dev(Vs[t], td))
        P, S, Tr = O.incr_update_general_factored(P, S, Tr, T0, B, Us[t], Vs[t])
    got = _ts(view)
    worst = max(O.maxrel(got[i], Tr[i]) for i in Tr)
    msg = []
    for i in Tr:
        dr = O.deltarel(got[i], T_got0[i], Tr[i], T_ref0[i])
        dtol = dbase + 4 * np.sqrt(T) * u * np.abs(Tr[i]).max() / np.abs(Tr[i] - T_ref0[i]).max()
        msg.append(f"T{i}: {dr:.1e}(<{dtol:.1e})")
        assert dr < dtol, f"T_{i} deltarel {dr:.3e} >= {dtol:.3e}"
    note(f"general factored n={n} k={k} r={r} p={p} {mode}: create {create_err:.1e}, after {T} updates maxrel "
         f"{worst:.2e}; " + " ".join(msg))
    assert worst < tol
    pw, pp = read_all(view), read_all(plain)
    for i in pw:
        np.testing.assert_array_equal(pw[i], pp[i])
    view.close()
    plain.close()


def test_general_factored_equals_hybrid_fp64():
    lv = _lv()
    import torch
    n, k, r, p = 400, 16, 2, 6
    A = synth.gaussian_matrix(n, seed=71)
    T0, B = synth.general_operands(n, p, seed=71)
    Us, Vs = synth.update_factors(n, r, 5, seed=71)
    vh = lv.View(dev(A, torch.float64), k, r_max=r, general=(dev(T0, torch.float64), dev(B, torch.float64)))
    vf = lv.View(dev(A, torch.float64), k, r_max=r, general=(dev(T0, torch.float64), dev(B, torch.float64)),
                 strategy=lv.LV_GENERAL_FACTORED)
    for t in range(5):
        vh.update(dev(Us[t], torch.float64), dev(Vs[t], torch.float64))
        vf.update(dev(Us[t], torch.float64), dev(Vs[t], torch.float64))
    gh, gf = _ts(vh), _ts(vf)
    for i in gh:
        assert O.maxrel(gf[i], gh[i]) < 1e-12
    vh.close()
    vf.close()


def test_general_factored_regression_p1000_full_size():
    """The regression workload at the paper's p = 1000 with n = 8192, FP32,
    factored deltas, rank-1 row additions; sampled columns of every T_i
    against the defining iteration on the final A (columns of T evolve
    independently)."""
    lv = _lv()
    import torch
    n, p, k, T = 8192, 1000, 16, 6
    A, B, eta = synth.regression_problem(n, p, n + n // 2, seed=9)
    A, B = _rounded(A, np.float32), _rounded(B, np.float32)
    T0 = np.zeros((n, p))
    Us, Vs = (_rounded(x, np.float32) for x in synth.regression_rows(n, T, eta, seed=9))
    view = lv.View(dev(A, torch.float32), k, general=(dev(T0, torch.float32), dev(B, torch.float32)),
                   strategy=lv.LV_GENERAL_FACTORED)
    cols = synth.rng(9, 0, 95).choice(p, size=8, replace=False)
    base_got = {i: host(view.read_general(i))[:, cols] for i in view.powers()}
    base_ref = O.iterate_general(A, T0[:, cols], B[:, cols], k)
    for t in range(T):
        view.update(dev(Us[t], torch.float32), dev(Vs[t], torch.float32))
    Afin = A + np.einsum("tir,tjr->ij", Us, Vs)
    ref = O.iterate_general(Afin, T0[:, cols], B[:, cols], k)
    got = {i: host(view.read_general(i))[:, cols] for i in view.powers()}
    u = 2.0 ** -24
    msg = []
    for i in ref:
        mr = O.maxrel(got[i], ref[i])
        assert mr < 1e-4, f"T_{i} maxrel {mr:.3e}"
        change = np.abs(ref[i] - base_ref[i]).max()
        if change == 0.0:
            # T_1 = A T_0 + B with T_0 = 0 does not depend on A: it must not move
            np.testing.assert_array_equal(got[i], base_got[i])
            msg.append(f"T{i}: {mr:.1e}/unchanged")
            continue
        dr = O.deltarel(got[i], base_got[i], ref[i], base_ref[i])
        dtol = 1e-2 + 4 * np.sqrt(T) * u * np.abs(ref[i]).max() / change
        msg.append(f"T{i}: {mr:.1e}/{dr:.1e}(<{dtol:.1e})")
        assert dr < dtol, f"T_{i} deltarel {dr:.3e} >= {dtol:.3e}"
    note(f"regression factored n={n} p={p}: " + " ".join(msg))
    view.close()


@pytest.mark.parametrize("strategy", [0, 1])
def test_general_tiny_order(strategy):
    """n = 5 (all padding), k = 8, FP64, both strategies."""
    lv = _lv()
    import torch
    n, k, p = 5, 8, 3
    A = synth.gaussian_matrix(n, seed=72)
    T0, B = synth.general_operands(n, p, seed=72)
    Us, Vs = synth.update_factors(n, 1, 3, seed=72)
    view = lv.View(dev(A, torch.float64), k, general=(dev(T0, torch.float64), dev(B, torch.float64)),
                   strategy=strategy)
    P, S, Tr = O.reeval(A, k), O.reeval_sums(A, k), O.reeval_general(A, T0, B, k)
    for t in range(3):
        view.update(dev(Us[t], torch.float64), dev(Vs[t], torch.float64))
        P, S, Tr = O.incr_update_general(P, S, Tr, T0, B, Us[t], Vs[t])
    got = _ts(view)
    assert max(O.maxrel(got[i], Tr[i]) for i in Tr) < 1e-12
    view.close()


# ---- skip-s model with factored deltas (Table 1, App. B); updates of rank
# below r_max exercise the factor widths of the update's own rank


@pytest.mark.parametrize("n,k,s,r_max,r_upd,p,dtype", [
    (300, 16, 4, 2, 2, 3, "f64"), (1000, 16, 4, 1, 1, 1, "f32"), (600, 8, 2, 4, 2, 40, "f32"),
    (257, 8, 1, 2, 1, 5, "f32"), (520, 16, 8, 2, 1, 130, "f64"), (130, 4, 2, 1, 1, 2, "f32"),
    (400, 8, 8, 4, 1, 6, "f32"), (333, 16, 16, 8, 3, 9, "f64")])
def test_general_skip_tracks_oracle(n, k, s, r_max, r_upd, p, dtype):
    lv = _lv()
    import torch
    td, nd = (torch.float64, np.float64) if dtype == "f64" else (torch.float32, np.float32)
    mode = lv.LV_FP64 if dtype == "f64" else lv.LV_FP32
    tol, dbase = (1e-10, 1e-7) if dtype == "f64" else (1e-4, 1e-2)
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    T = 6
    A = _rounded(synth.gaussian_matrix(n, seed=75 + n, config=3), nd)
    T0, B = (_rounded(x, nd) for x in synth.general_operands(n, p, seed=75 + n, config=3))
    Us, Vs = (_rounded(x, nd) for x in synth.update_factors(n, r_upd, T, seed=75 + n, config=3))
    view = lv.View(dev(A, td), k, r_max=r_max, mode=mode, general=(dev(T0, td), dev(B, td)),
                   strategy=lv.LV_GENERAL_FACTORED, skip=s)
    plain = lv.View(dev(A, td), s, r_max=r_max, mode=mode, sums=True)
    idx = O.skip_indices(k, s)
    assert view.general_indices() == idx
    P, S, Tr = O.reeval(A, s), O.reeval_sums(A, s), O.reeval_general_skip(A, T0, B, k, s)
    T_ref0 = Tr
    T_got0 = {i: host(view.read_general(i)) for i in idx}
    create_err = max(O.maxrel(T_got0[i], Tr[i]) for i in idx)
    assert create_err < (1e-13 if dtype == "f64" else 1e-6), create_err
    for t in range(T):
        view.update(dev(Us[t], td), dev(Vs[t], td))
        plain.update(dev(Us[t], td), dev(Vs[t], td))
        P, S, Tr = O.incr_update_general_factored_skip(P, S, Tr, T0, B, Us[t], Vs[t], s)
    got = {i: host(view.read_general(i)) for i in idx}
    worst = max(O.maxrel(got[i], Tr[i]) for i in idx)
    msg = []
    for i in idx:
        dr = O.deltarel(got[i], T_got0[i], Tr[i], T_ref0[i])
        dtol = dbase + 4 * np.sqrt(T) * u * np.abs(Tr[i]).max() / np.abs(Tr[i] - T_ref0[i]).max()
        msg.append(f"T{i}: {dr:.1e}(<{dtol:.1e})")
        assert dr < dtol, f"T_{i} deltarel {dr:.3e} >= {dtol:.3e}"
    note(f"general skip n={n} k={k} s={s} r={r_upd}/{r_max} p={p} {dtype}: create {create_err:.1e}, after {T} "
         f"updates maxrel {worst:.2e}; " + " ".join(msg))
    assert worst < tol
    # the stored powers and sums (up to P_s) are those of a plain view with sums
    pw, pp = read_all(view), read_all(plain)
    assert sorted(pw) == sorted(pp)
    for i in pw:
        np.testing.assert_array_equal(pw[i], pp[i])
    for i in view.powers():
        np.testing.assert_array_equal(host(view.read_sum(i)), host(plain.read_sum(i)))
    # the skip model's indices are the only T stored
    with pytest.raises(lv.LinviewError):
        view.read_general(3 if s != 1 else k + 1)
    view.close()
    plain.close()


def test_general_skip_full_size_against_iteration():
    """Skip-4 model with factored deltas at n = 8192, k = 16, p = 16, FP32,
    rank 1, 8 updates: every stored T_i (1, 2, 4, 8, 12, 16) against the
    defining iteration T_{i+1} = A T_i + B on the final A."""
    lv = _lv()
    import torch
    n, k, s, p, T = 8192, 16, 4, 16, 8
    A = _rounded(synth.gaussian_matrix(n, seed=63, config=3), np.float32)
    T0, B = (_rounded(x, np.float32) for x in synth.general_operands(n, p, seed=63, config=3))
    Us, Vs = (_rounded(x, np.float32) for x in synth.update_factors(n, 1, T, seed=63, config=3))
    view = lv.View(dev(A, torch.float32), k, general=(dev(T0, torch.float32), dev(B, torch.float32)),
                   strategy=lv.LV_GENERAL_FACTORED, skip=s)
    idx = O.skip_indices(k, s)

    def iterate(Am):
        out, Tm = {}, T0
        for i in range(1, k + 1):
            Tm = Am @ Tm + B
            if i in idx:
                out[i] = Tm
        return out

    base_got = {i: host(view.read_general(i)) for i in idx}
    base_ref = iterate(A)
    for t in range(T):
        view.update(dev(Us[t], torch.float32), dev(Vs[t], torch.float32))
    ref = iterate(A + np.einsum("tir,tjr->ij", Us, Vs))
    got = {i: host(view.read_general(i)) for i in idx}
    u = 2.0 ** -24
    msg = []
    for i in idx:
        mr = O.maxrel(got[i], ref[i])
        dr = O.deltarel(got[i], base_got[i], ref[i], base_ref[i])
        dtol = 1e-2 + 4 * np.sqrt(T) * u * np.abs(ref[i]).max() / np.abs(ref[i] - base_ref[i]).max()
        msg.append(f"T{i}: {mr:.1e}/{dr:.1e}(<{dtol:.1e})")
        assert mr < 1e-4, f"T_{i} maxrel {mr:.3e}"
        assert dr < dtol, f"T_{i} deltarel {dr:.3e} >= {dtol:.3e}"
    note("general skip-4 full size: " + " ".join(msg))
    view.close()


def test_general_skip_reanchor_and_batch():
    """Skip-4 view (k = 16): re-anchoring rebuilds every stored T from the
    current A (T_8, T_12, T_16 included); batched updates give the same T bit
    for bit as single updates."""
    lv = _lv()
    import torch
    n, k, s, p = 400, 16, 4, 6
    A = _rounded(synth.gaussian_matrix(n, seed=64), np.float32)
    T0, B = (_rounded(x, np.float32) for x in synth.general_operands(n, p, seed=64))
    Us, Vs = (_rounded(x, np.float32) for x in synth.update_factors(n, 1, 3, seed=64))

    def make():
        return lv.View(dev(A, torch.float32), k, general=(dev(T0, torch.float32), dev(B, torch.float32)),
                       strategy=lv.LV_GENERAL_FACTORED, skip=s)

    view, twin = make(), make()
    for t in range(3):
        view.update(dev(Us[t], torch.float32), dev(Vs[t], torch.float32))
    twin.update_batch(dev(Us, torch.float32), dev(Vs, torch.float32))
    idx = view.general_indices()
    for i in idx:
        np.testing.assert_array_equal(host(view.read_general(i)), host(twin.read_general(i)))
    view.reanchor()
    ref = O.reeval_general_skip(host(view.read(1)), T0, B, k, s)
    assert max(O.maxrel(host(view.read_general(i)), ref[i]) for i in idx) < 1e-6
    with pytest.raises(lv.LinviewError):
        view.read(8)                                       # the powers stop at P_4
    view.close()
    twin.close()
