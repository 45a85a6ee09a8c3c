"""Full-size parity: the benchmark's workload (A^16, n = 8192, FP32, 1000
rank-1 updates applied with lv_view_update_batch as bench.py does), checked
every 100 updates element by element on every stored power against the
oracle's re-evaluation of the accumulated A_t (oracle.reeval, FP64), and on
sampled rows and columns against the definition: each sampled row / column
of A_t^(2^j) by repeated vector-matrix products with the FP64 accumulated
A_t (oracle.power_rows / power_cols), no n x n power formed.

Tolerances over the samples: maxrel 1e-4 (FP32).  deltarel (error of the
accumulated change) is bounded by FP32 storage itself: every update adds a
term about 2e-6 of the stored entries, so each addition rounds away a few
percent of it.  The bound is derived from the arithmetic,
    deltarel <= 1e-2 + 4 * sqrt(t) * u * max|R_t| / max|R_t - R_0|,
u = 2^-24 the FP32 unit roundoff (each addition rounds by at most one ulp,
the roundings accumulate as a random walk over t updates, and 4 covers the
maximum over the samples); a view that missed the last tenth of the updates
(its change is short by a random walk of T/10 steps, about a third of the
total) exceeds it."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import dev, need_gpu, note

pytestmark = pytest.mark.gpu


def test_bench_workload_sampled_every_100_updates():
    need_gpu()
    import torch
    from paper_1403_6968_amd import linview as lv

    n, k, T, every = 8192, 16, 1000, 100
    note(f"full-size n={n} k={k} T={T}: generating inputs")
    A = synth.gaussian_matrix(n, seed=0, config=2).astype(np.float32)
    Us, Vs = synth.update_factors(n, 1, T, seed=0, config=2)
    Us, Vs = Us.astype(np.float32), Vs.astype(np.float32)
    rows = np.array([0, 1, 4097, 5000, n - 1])
    cols = np.array([0, 777, 4096, n - 2, n - 1])

    view = lv.View(dev(A, torch.float32), k)
    Ud, Vd = dev(Us, torch.float32), dev(Vs, torch.float32)
    powers = view.powers()

    def gpu_samples():
        out = {}
        for i in powers:
            P = view.read(i)
            out[i] = (P[torch.as_tensor(rows, device="cuda")].double().cpu().numpy(),
                      P[:, torch.as_tensor(cols, device="cuda")].double().cpu().numpy())
            del P
        return out

    def ref_samples(At):
        out = {}
        R = At[rows, :].copy()
        C = At[:, cols].copy()
        for i in range(1, k + 1):
            if i in powers:
                out[i] = (R.copy(), C.copy())
            R = R @ At
            C = At @ C
        return out

    def gpu_full():
        return {i: view.read(i).double().cpu().numpy() for i in powers}

    A64 = A.astype(np.float64)
    full0, rfull0 = gpu_full(), O.reeval(A64, k)
    for i in powers:      # creation: one rounding of the FP64 chain
        assert O.maxrel(full0[i], rfull0[i]) < 1e-6
    g0, r0 = gpu_samples(), ref_samples(A64)
    # ref_samples' recurrence agrees with the oracle's definition-based routine
    assert O.maxrel(r0[16][0], O.power_rows(A64, 16, rows)) < 1e-12
    At = A64.copy()
    worst = {}
    g = g0
    for t0 in range(0, T, every):
        view.update_batch(Ud[t0:t0 + every], Vd[t0:t0 + every])
        At += Us[t0:t0 + every, :, 0].astype(np.float64).T @ Vs[t0:t0 + every, :, 0].astype(np.float64)
        g_prev = g if t0 > 0 else g0
        g, r = gpu_samples(), ref_samples(At)
        msg = []
        for i in powers:
            got = np.concatenate([g[i][0].ravel(), g[i][1].ravel()])
            ref = np.concatenate([r[i][0].ravel(), r[i][1].ravel()])
            got0 = np.concatenate([g0[i][0].ravel(), g0[i][1].ravel()])
            ref0 = np.concatenate([r0[i][0].ravel(), r0[i][1].ravel()])
            mr = O.maxrel(got, ref)
            dr = O.deltarel(got, got0, ref, ref0)
            t = t0 + every
            dtol = 1e-2 + 4 * np.sqrt(t) * 2.0 ** -24 * np.abs(ref).max() / np.abs(ref - ref0).max()
            worst[i] = max(worst.get(i, 0.0), mr)
            msg.append(f"P{i}: {mr:.2e}/{dr:.2e}(<{dtol:.1e})")
            assert mr < 1e-4, f"P_{i} maxrel {mr:.3e} after {t}"
            assert dr < dtol, f"P_{i} deltarel {dr:.3e} >= {dtol:.3e} after {t}"
        note(f"after {t0 + every}: maxrel/deltarel " + " ".join(msg))
        # every element of every stored power against the oracle's re-evaluation
        full, rfull = gpu_full(), O.reeval(At, k)
        msg = []
        for i in powers:
            mr = O.maxrel(full[i], rfull[i])
            dr = O.deltarel(full[i], full0[i], rfull[i], rfull0[i])
            dtol = 1e-2 + 4 * np.sqrt(t) * 2.0 ** -24 * np.abs(rfull[i]).max() / np.abs(rfull[i] - rfull0[i]).max()
            msg.append(f"P{i}: {mr:.2e}/{dr:.2e}(<{dtol:.1e})")
            assert mr < 1e-4, f"P_{i} full maxrel {mr:.3e} after {t}"
            assert dr < dtol, f"P_{i} full deltarel {dr:.3e} >= {dtol:.3e} after {t}"
        del full, rfull
        note(f"after {t0 + every}, every element: " + " ".join(msg))
    # the stored chain after 1000 FP32 updates still satisfies P_{2i} = P_i P_i
    z = dev(synth.rng(0, 2, 9).standard_normal(n), torch.float64)
    res = view.drift_check(z, tau=1e-3).cpu().numpy()
    note(f"drift residuals after {T} updates: {res}")
    assert res.max() < 1e-3 and view.stats()["drift_reanchors"] == 0
    # a stale view (the last 100 updates missed) fails the bound
    for i in powers:
        ref = r[i][0].ravel()
        ref0 = r0[i][0].ravel()
        dtol = 1e-2 + 4 * np.sqrt(T) * 2.0 ** -24 * np.abs(ref).max() / np.abs(ref - ref0).max()
        dr = O.deltarel(g_prev[i][0].ravel(), g0[i][0].ravel(), ref, ref0)
        note(f"stale P{i}: deltarel {dr:.2e} vs bound {dtol:.2e}")
        assert dr > dtol
    view.close()


def _lowrank_samples(A0, Uc, Vc, rows, cols, powers):
    """Sampled rows and columns of (A0 + Uc Vc^T)^i for i in powers, by the
    definition: repeated vector-matrix products, with the accumulated update
    applied in factored form (no n x n matrix besides A0 is formed)."""
    out = {}
    R = A0[rows, :] + Uc[rows, :] @ Vc.T
    C = A0[:, cols] + Uc @ Vc[cols, :].T
    for i in range(1, max(powers) + 1):
        if i in powers:
            out[i] = (R.copy(), C.copy())
        R = R @ A0 + (R @ Uc) @ Vc.T
        C = A0 @ C + Uc @ (Vc.T @ C)
    return out


@pytest.mark.timeout(900)
def test_rank4_n16384_fp32_and_bf16_shadow_every_100_updates():
    """A^16 at n = 16384, 500 rank-4 updates, the plain FP32 path and the
    BF16-shadow path on the same inputs; sampled rows / columns of every
    stored power against the FP64 oracle after every 100 updates.
    Bounds: FP32 maxrel 1e-4, BF16 path maxrel 5e-3; deltarel 1e-2 (FP32)
    and 5e-2 (BF16 path) plus the FP32 storage term derived for the rank-1
    workload above; a view that missed the last 100 updates fails both."""
    need_gpu()
    import torch
    from paper_1403_6968_amd import linview as lv

    n, k, r, T, every = 16384, 16, 4, 500, 100
    note(f"n={n} k={k} r={r} T={T}: generating inputs")
    A = synth.gaussian_matrix(n, seed=0, config=3).astype(np.float32)
    Us, Vs = synth.update_factors(n, r, T, seed=0, config=3)
    Us, Vs = Us.astype(np.float32), Vs.astype(np.float32)
    rows = np.array([0, 3, 8191, 12000, n - 1])
    cols = np.array([1, 4096, 9999, n - 3, n - 1])
    A64 = A.astype(np.float64)
    modes = {"fp32": lv.LV_FP32, "bf16": lv.LV_FP32_BF16SHADOW}
    views = {name: lv.View(dev(A, torch.float32), k, r_max=r, mode=m) for name, m in modes.items()}
    powers = views["fp32"].powers()
    Ud, Vd = dev(Us, torch.float32), dev(Vs, torch.float32)

    def gpu_samples(view):
        out = {}
        ri = torch.as_tensor(rows, device="cuda")
        ci = torch.as_tensor(cols, device="cuda")
        for i in powers:
            P = view.read(i)
            out[i] = (P[ri].double().cpu().numpy(), P[:, ci].double().cpu().numpy())
            del P
        return out

    def flat(x):
        return np.concatenate([x[0].ravel(), x[1].ravel()])

    # the factored recurrence agrees with the oracle's definition-based rows / columns
    g = synth.rng(1, 3, 5)
    a_s, u_s, v_s = g.standard_normal((64, 64)) / 8, g.standard_normal((64, 6)) / 8, g.standard_normal((64, 6)) / 8
    chk = _lowrank_samples(a_s, u_s, v_s, np.array([0, 5, 63]), np.array([2, 7]), [1, 2, 4, 8, 16])
    assert O.maxrel(chk[16][0], O.power_rows(a_s + u_s @ v_s.T, 16, np.array([0, 5, 63]))) < 1e-12
    assert O.maxrel(chk[8][1], O.power_cols(a_s + u_s @ v_s.T, 8, np.array([2, 7]))) < 1e-12
    zero = np.zeros((n, 0))
    r0 = _lowrank_samples(A64, zero, zero, rows, cols, powers)
    g0 = {name: gpu_samples(v) for name, v in views.items()}
    g_prev = None
    bounds = {"fp32": (1e-4, 1e-2), "bf16": (5e-3, 5e-2)}
    for t0 in range(0, T, every):
        t = t0 + every
        g_prev = {name: gpu_samples(v) for name, v in views.items()} if t == T else g_prev
        for v in views.values():
            v.update_batch(Ud[t0:t], Vd[t0:t])
        Uc = Us[:t].astype(np.float64).transpose(1, 0, 2).reshape(n, t * r)
        Vc = Vs[:t].astype(np.float64).transpose(1, 0, 2).reshape(n, t * r)
        ref = _lowrank_samples(A64, Uc, Vc, rows, cols, powers)
        for name, v in views.items():
            g = gpu_samples(v)
            msg = []
            for i in powers:
                got, want = flat(g[i]), flat(ref[i])
                mr = O.maxrel(got, want)
                dr = O.deltarel(got, flat(g0[name][i]), want, flat(r0[i]))
                mtol, dbase = bounds[name]
                dtol = dbase + 4 * np.sqrt(t) * 2.0 ** -24 * np.abs(want).max() / np.abs(want - flat(r0[i])).max()
                msg.append(f"P{i}: {mr:.2e}/{dr:.2e}")
                assert mr < mtol, f"{name} P_{i} maxrel {mr:.3e} after {t}"
                assert dr < dtol, f"{name} P_{i} deltarel {dr:.3e} >= {dtol:.3e} after {t}"
            note(f"{name} after {t}: maxrel/deltarel " + " ".join(msg))
    # a view that missed the last 100 updates fails the bounds
    for name in views:
        for i in powers:
            want = flat(ref[i])
            dtol = bounds[name][1] + 4 * np.sqrt(T) * 2.0 ** -24 * np.abs(want).max() / np.abs(want - flat(r0[i])).max()
            dr = O.deltarel(flat(g_prev[name][i]), flat(g0[name][i]), want, flat(r0[i]))
            assert dr > dtol, f"stale {name} P_{i}: deltarel {dr:.3e} within {dtol:.3e}"
    for v in views.values():
        v.close()
