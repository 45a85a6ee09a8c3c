"""Views with sums of powers (LV_WITH_SUMS): S_i = I + A + ... + A^(i-1) for
i in {1, 2, 4, ..., k} kept current under updates, against the FP64 oracle
(`oracle.reeval_sums`, `oracle.incr_update_sums`).

Tolerances as for the powers: maxrel FP64 1e-10, FP32 1e-4, BF16-shadow mode
5e-3; deltarel d + 4 sqrt(t) u max|S_t| / max|S_t - S_0| with the storage
unit roundoff u and d = 1e-7 / 1e-2 / 5e-2 (the storage term is the bound
derived for the powers: S holds the identity, so its entries are large next
to their change and float storage rounds away a visible part of it);
integer walk counts of a DAG bit for bit."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import dev, host, need_gpu, note, read_all, storage_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    note(f"start {request.node.nodeid}")
    yield


def _lv():
    need_gpu()
    from paper_1403_6968_amd import linview
    return linview


def _sums(view):
    return {i: host(view.read_sum(i)) for i in view.powers()}


@pytest.mark.parametrize("n,k,r,dtype,mode", [
    (300, 16, 2, "f64", "f64"), (1000, 16, 1, "f32", "f32"), (600, 16, 4, "f32", "f32"),
    (257, 32, 3, "f32", "f32"), (520, 8, 8, "f64", "f64"), (700, 16, 2, "f32", "bf16"), (130, 1, 2, "f32", "f32")])
def test_sums_track_oracle(n, k, r, dtype, mode):
    lv = _lv()
    import torch
    td, nd = (torch.float64, np.float64) if dtype == "f64" else (torch.float32, np.float32)
    lvmode = {"f64": lv.LV_FP64, "f32": lv.LV_FP32, "bf16": lv.LV_FP32_BF16SHADOW}[mode]
    tol = {"f64": 1e-10, "f32": 1e-4, "bf16": 5e-3}[mode]
    dbase = {"f64": 1e-7, "f32": 1e-2, "bf16": 5e-2}[mode]
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    T = 8
    A64 = synth.gaussian_matrix(n, seed=50 + n, config=2)
    Us, Vs = synth.update_factors(n, r, T, seed=50 + n, config=2)
    A, Us, Vs = storage_inputs(A64, Us, Vs, nd)
    view = lv.View(dev(A, td), k, r_max=r, mode=lvmode, sums=True)
    plain = lv.View(dev(A, td), k, r_max=r, mode=lvmode)
    P, S = O.reeval(A, k), O.reeval_sums(A, k)
    S0_ref, S0_got = S, _sums(view)
    create_err = max(O.maxrel(S0_got[i], S[i]) for i in S)
    assert create_err < (1e-13 if dtype == "f64" else 1e-6), create_err
    for t in range(T):
        view.update(dev(Us[t], td), dev(Vs[t], td))
        plain.update(dev(Us[t], td), dev(Vs[t], td))
        P, S = O.incr_update_sums(P, S, Us[t], Vs[t])
    got = _sums(view)
    worst = max(O.maxrel(got[i], S[i]) for i in S)
    msg = []
    for i in S:
        if i == 1:
            continue
        dr = O.deltarel(got[i], S0_got[i], S[i], S0_ref[i])
        dtol = dbase + 4 * np.sqrt(T) * u * np.abs(S[i]).max() / np.abs(S[i] - S0_ref[i]).max()
        msg.append(f"S{i}: {dr:.1e}(<{dtol:.1e})")
        assert dr < dtol, f"S_{i} deltarel {dr:.3e} >= {dtol:.3e}"
    note(f"sums n={n} k={k} r={r} {mode}: create {create_err:.1e}, after {T} updates maxrel {worst:.2e}; "
         + " ".join(msg))
    assert worst < tol
    np.testing.assert_array_equal(got[1], np.eye(n))                       # S_1 = I stays
    # the powers of a view with sums equal those of a plain view bit for bit
    pw, pp = read_all(view), read_all(plain)
    for i in pw:
        np.testing.assert_array_equal(pw[i], pp[i])
    view.close()
    plain.close()


def test_sums_dag_walk_counts_exact():
    """S_i of a DAG adjacency counts the walks of length < i; edge insertions
    keep every value an integer below 2^24, so FP32 is exact."""
    lv = _lv()
    import torch
    n, k = 384, 16
    adj = synth.random_dag(n, 0.03, seed=8)
    g = synth.rng(8, 0, 77)
    cur = adj.copy()
    ups = []
    while len(ups) < 5:
        a, b = sorted(g.integers(0, n, size=2))
        if a != b and cur[a, b] == 0:
            cur[a, b] = 1.0
            u = np.zeros((n, 1)); u[a] = 1.0
            v = np.zeros((n, 1)); v[b] = 1.0
            ups.append((u, v))
    view = lv.View(dev(adj, torch.float32), k, sums=True)
    P, S = O.reeval(adj, k), O.reeval_sums(adj, k)
    for u, v in ups:
        view.update(dev(u, torch.float32), dev(v, torch.float32))
        P, S = O.incr_update_sums(P, S, u, v)
    assert max(np.abs(S[i]).max() for i in S) < 2 ** 24
    got = _sums(view)
    for i in S:
        np.testing.assert_array_equal(got[i], S[i], err_msg=f"S_{i}")
    note(f"dag sums: max entry {max(np.abs(S[i]).max() for i in S):.0f}")
    view.close()


def test_sums_reanchor_and_errors():
    lv = _lv()
    import torch
    n, k = 400, 8
    A = np.asarray(synth.gaussian_matrix(n, seed=51), dtype=np.float32).astype(np.float64)
    Us, Vs = synth.update_factors(n, 1, 3, seed=51)
    Us, Vs = Us.astype(np.float32).astype(np.float64), Vs.astype(np.float32).astype(np.float64)
    view = lv.View(dev(A, torch.float32), k, sums=True)
    for t in range(3):
        view.update(dev(Us[t], torch.float32), dev(Vs[t], torch.float32))
    view.reanchor()
    Afin = host(view.read(1))
    ref = O.reeval_sums(Afin, k)
    got = _sums(view)
    assert max(O.maxrel(got[i], ref[i]) for i in ref) < 1e-6
    plain = lv.View(dev(A, torch.float32), k)
    with pytest.raises(lv.LinviewError) as e:
        plain.read_sum(2)
    assert e.value.status == lv.LV_ESTATE
    with pytest.raises(lv.LinviewError):
        lv.Batch([view])                                  # sums views are single-view only
    with pytest.raises(lv.LinviewError):
        view.read_sum(3)
    view.close()
    plain.close()
