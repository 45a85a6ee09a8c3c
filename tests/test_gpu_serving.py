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


LARGE = [(8192, 16), (4096, 16), (2048, 16), (3000, 16)]
LARGE_PER_VIEW = (48, 40, 32, 32)


def _serve_large(lv, subset, reqs, step_every, rc=16):
    """BF16-shadow server with r_coalesce rc over the views in subset."""
    import torch
    mode = lv.LV_FP32_BF16SHADOW
    probe = lv.Server(8 * MiB, mode=mode, r_coalesce=rc)
    total = sum(probe.view_bytes(LARGE[v][0], LARGE[v][1]) for v in subset)
    probe.close()
    srv = lv.Server(8 * MiB + total, mode=mode, r_coalesce=rc)
    ids = {}
    for v in subset:
        n, k = LARGE[v]
        A = synth.gaussian_matrix(n, seed=43, config=5, view=v).astype(np.float32)
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
    out = {v: {p: host(srv.read(ids[v], p)) for p in [2 ** j for j in range(int(np.log2(LARGE[v][1])) + 1)]}
           for v in ids}
    st = srv.stats()
    srv.close()
    return out, st


@pytest.mark.parametrize("rc", [16, 32])
def test_mix_equals_alone_and_oracle_large_shadow(rc):
    """The serving configuration's mode and coalescing widths at realistic
    orders: bfloat16 shadows, r_coalesce 16 and 32 (top factors 512 wide),
    views of n = 2048 .. 8192 served together (coalesced ranks up to rc) and
    each alone with another cadence; both equal the FP64 oracle within 5e-3
    and each other."""
    lv = _lv()
    reqs = []
    for v, (n, _) in enumerate(LARGE):
        U, V = synth.update_factors(n, 1, LARGE_PER_VIEW[v], seed=44, config=5, view=v)
        for t in range(LARGE_PER_VIEW[v]):
            reqs.append((v, U[t, :, 0].astype(np.float32), V[t, :, 0].astype(np.float32)))
    order = synth.rng(44, 5, 9).permutation(len(reqs))
    reqs = [reqs[i] for i in order]
    mix, st = _serve_large(lv, range(len(LARGE)), reqs, step_every=24 * rc // 16, rc=rc)
    note(f"large mix stats {st}")
    assert st["submitted"] == st["completed"] == len(reqs)
    assert st["coalesced_updates"] < len(reqs) / 4        # wide coalesced updates
    for v, (n, k) in enumerate(LARGE):
        A = synth.gaussian_matrix(n, seed=43, config=5, view=v).astype(np.float32).astype(np.float64)
        U = np.array([u for vv, u, _ in reqs if vv == v], dtype=np.float64)
        W = np.array([w for vv, _, w in reqs if vv == v], dtype=np.float64)
        A += U.T @ W
        ref = O.reeval(A, k)
        alone, _ = _serve_large(lv, [v], reqs, step_every=3, rc=rc)
        worst = 0.0
        for p in ref:
            mr = O.maxrel(mix[v][p], ref[p])
            ma = O.maxrel(alone[v][p], mix[v][p])
            worst = max(worst, mr)
            assert mr < 5e-3, (v, p, mr)
            assert ma < 5e-3, (v, p, ma)
        note(f"large view {v} n={n}: maxrel vs oracle {worst:.2e}")


def test_admission_queue_admits_when_memory_frees():
    """With the admission queue on, a view that does not fit waits (its
    requests queue), is admitted when a removal frees room, and then serves
    its queued requests: its result equals the oracle with all of them."""
    lv = _lv()
    import torch
    n, k = 1024, 16
    probe = lv.Server(8 * MiB, r_coalesce=4)
    one = probe.view_bytes(n, k)
    probe.close()
    srv = lv.Server(4 * MiB + 2 * one + one // 2, r_coalesce=4)
    srv.set_admission_queue(True)
    As = [synth.gaussian_matrix(n, seed=45, config=5, view=v).astype(np.float32) for v in range(3)]
    ids = [srv.add_view(dev(A, torch.float32), k) for A in As]
    st = srv.stats()
    assert st["views"] == 2 and st["views_waiting"] == 1
    waiting = ids[2]
    U, V = synth.update_factors(n, 1, 10, seed=46, config=5)
    Uf, Vf = U[:, :, 0].astype(np.float32), V[:, :, 0].astype(np.float32)
    for t in range(10):                                  # queued while waiting
        srv.submit(waiting, Uf[t], Vf[t])
        srv.submit(ids[0], Uf[t], Vf[t])
    for _ in range(3):
        srv.step()
    with pytest.raises(lv.LinviewError):
        srv.read(waiting, 1)                             # not admitted yet
    srv.remove_view(ids[1])                              # frees a block: the waiting view is admitted
    st = srv.stats()
    assert st["views"] == 2 and st["views_waiting"] == 0 and st["admitted_late"] == 1
    srv.drain()
    st = srv.stats()
    assert st["submitted"] == st["completed"] == 20
    A = As[2].astype(np.float64) + Uf.astype(np.float64).T @ Vf.astype(np.float64)
    ref = O.reeval(A, k)
    for p in ref:
        err = O.maxrel(host(srv.read(waiting, p)), ref[p])
        assert err < 1e-4, (p, err)
    # a view larger than the whole arena is refused even with the queue on
    with pytest.raises(lv.LinviewError):
        srv.add_view(dev(np.zeros((4096, 4096), np.float32), torch.float32), k)
    # the arena is full again: a third view waits, and can be dropped with its requests
    w = srv.add_view(dev(As[1], torch.float32), k)
    assert srv.stats()["views_waiting"] == 1
    srv.submit(w, Uf[0], Vf[0])
    assert srv.stats()["submitted"] == 21
    srv.remove_view(w)
    st = srv.stats()
    assert st["views_waiting"] == 0 and st["submitted"] == 20 and st["views"] == 2
    srv.close()
