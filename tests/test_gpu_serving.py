"""Serving loop (lv_server_*): admission by footprint, coalescing, continuous
batching.  Each view's result after serving a mixed request stream equals
the FP64 oracle and the same view served alone (different coalescing)
within the FP32 tolerance 1e-4 (5e-3 with bfloat16 shadows)."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import dev, host, need_gpu, note

pytestmark = pytest.mark.gpu

MiB = 1 << 20


@pytest.fixture(autouse=True)
def _announce(request):
    note(f"start {request.node.nodeid}")
    yield


def _lv():
    need_gpu()
    from paper_1403_6968_amd import linview
    return linview


def test_admission_by_footprint():
    lv = _lv()
    import torch
    probe = lv.Server(8 * MiB, r_coalesce=4)
    one = probe.view_bytes(1024, 16)
    probe.close()
    srv = lv.Server(4 * MiB + 2 * one + one // 2, r_coalesce=4)
    A = dev(synth.gaussian_matrix(1024, seed=40), torch.float32)
    a = srv.add_view(A, 16)
    b = srv.add_view(A, 16)
    with pytest.raises(lv.LinviewError) as e:
        srv.add_view(A, 16)
    assert e.value.status == lv.LV_ENOMEM and "admission" in str(e.value)
    srv.remove_view(a)
    c = srv.add_view(A, 16)                       # the freed block is reused
    assert srv.stats()["views"] == 2 and c == a
    srv.remove_view(b)
    srv.remove_view(c)
    assert srv.stats()["arena_free"] == 2 * one + one // 2
    srv.close()


SHAPES = [(300, 16), (700, 8), (1000, 16), (1500, 4)]
PER_VIEW = 24


def _requests():
    reqs = []
    for v, (n, _) in enumerate(SHAPES):
        U, V = synth.update_factors(n, 1, PER_VIEW, seed=41, config=5, view=v)
        for t in range(PER_VIEW):
            reqs.append((v, U[t, :, 0].astype(np.float32), V[t, :, 0].astype(np.float32)))
    order = synth.rng(41, 5, 9).permutation(len(reqs))
    return [reqs[i] for i in order]


def _serve(lv, views_subset, reqs, step_every, mode=None, hold=None):
    import torch
    mode = lv.LV_FP32 if mode is None else mode
    probe = lv.Server(8 * MiB, mode=mode)
    total = sum(probe.view_bytes(SHAPES[v][0], SHAPES[v][1]) for v in views_subset)
    probe.close()
    srv = lv.Server(8 * MiB + total, mode=mode, r_coalesce=4)
    if hold is not None:
        srv.set_hold(*hold)
    ids = {}
    for v in views_subset:
        n, k = SHAPES[v]
        A = synth.gaussian_matrix(n, seed=42, config=5, view=v).astype(np.float32)
        ids[v] = srv.add_view(dev(A, torch.float32), k)
    cnt = 0
    for v, u, w in reqs:
        if v not in ids:
            continue
        srv.submit(ids[v], u, w)
        cnt += 1
        if cnt % step_every == 0:
            srv.step()
    while srv.step() > 0:
        pass
    srv.drain()
    out = {v: {p: host(srv.read(ids[v], p)) for p in [2 ** j for j in range(int(np.log2(SHAPES[v][1])) + 1)]}
           for v in ids}
    st = srv.stats()
    srv.close()
    return out, st


@pytest.mark.parametrize("shadow", [False, True])
def test_mix_equals_alone_and_oracle(shadow):
    lv = _lv()
    mode = lv.LV_FP32_BF16SHADOW if shadow else lv.LV_FP32
    tol = 5e-3 if shadow else 1e-4
    reqs = _requests()
    mix, st = _serve(lv, range(len(SHAPES)), reqs, step_every=5, mode=mode)
    note(f"mix stats {st}")
    assert st["submitted"] == st["completed"] == len(reqs)
    assert st["coalesced_updates"] < len(reqs)          # some requests were coalesced
    assert 0 < st["latency_p50_s"] <= st["latency_p99_s"] <= st["latency_max_s"]
    for v, (n, k) in enumerate(SHAPES):
        A = synth.gaussian_matrix(n, seed=42, config=5, view=v).astype(np.float32).astype(np.float64)
        for vv, u, w in reqs:
            if vv == v:
                A += np.outer(u.astype(np.float64), w.astype(np.float64))
        ref = O.reeval(A, k)
        alone, _ = _serve(lv, [v], reqs, step_every=2, mode=mode)
        for p in ref:
            mr = O.maxrel(mix[v][p], ref[p])
            ma = O.maxrel(alone[v][p], mix[v][p])
            assert mr < tol, (v, p, mr)
            assert ma < tol, (v, p, ma)
        note(f"view {v} n={n} k={k}: maxrel vs oracle {max(O.maxrel(mix[v][p], ref[p]) for p in ref):.2e}")


def test_hold_policy_applies_every_request():
    """With a hold policy (a view waits for a full rank-4 update, or for the
    device to run idle) every request is still applied, the updates are
    fuller, and the views equal the ones served without holding and the
    oracle."""
    lv = _lv()
    reqs = _requests()
    base, st0 = _serve(lv, range(len(SHAPES)), reqs, step_every=5)
    held, st1 = _serve(lv, range(len(SHAPES)), reqs, step_every=5, hold=(4, 10.0))
    note(f"no hold {st0}; hold {st1}")
    assert st1["submitted"] == st1["completed"] == len(reqs)
    assert st1["coalesced_updates"] <= st0["coalesced_updates"]
    for v, (n, k) in enumerate(SHAPES):
        A = synth.gaussian_matrix(n, seed=42, config=5, view=v).astype(np.float32).astype(np.float64)
        for vv, u, w in reqs:
            if vv == v:
                A += np.outer(u.astype(np.float64), w.astype(np.float64))
        ref = O.reeval(A, k)
        for p in ref:
            assert O.maxrel(held[v][p], ref[p]) < 1e-4, (v, p)
            assert O.maxrel(held[v][p], base[v][p]) < 1e-4, (v, p)
    srv = lv.Server(8 * MiB, r_coalesce=4)
    with pytest.raises(lv.LinviewError):
        srv.set_hold(0, 0.0)
    with pytest.raises(lv.LinviewError):
        srv.set_hold(1, -1.0)
    srv.close()
