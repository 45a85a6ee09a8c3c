"""Full-size parity: the benchmark's workload (A^16, n = 8192, FP32, 1000
rank-1 updates applied with lv_view_update_batch as bench.py does), checked
every 100 updates on sampled rows and columns of every stored power.

The oracle computes each sampled row / column of A_t^(2^j) by definition
(repeated vector-matrix products with the FP64 accumulated A_t, see
oracle.power_rows / power_cols), so no n x n power is formed on the host.

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

    A64 = A.astype(np.float64)
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
