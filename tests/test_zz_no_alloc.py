"""The allocation-free update entry point (lv_powers_update_noalloc): caller-
held stored powers updated with the library's static device scratch must
equal what lv_view_update gives a view of the same shape (same kernels, same
reduction order: bit for bit), and follow the FP64 oracle.  Two shapes run in
a row in one process, the second smaller, so the second call works on a
scratch array that still holds the first call's contents."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import dev, need_gpu, note, storage_inputs

pytestmark = pytest.mark.gpu


def _run(lv, torch, n, k, r, mode, T, seed):
    note(f"noalloc: n={n} k={k} r={r} mode={mode} updates={T}")
    np_t, t_t = (np.float64, torch.float64) if mode == lv.LV_FP64 else (np.float32, torch.float32)
    A64 = synth.gaussian_matrix(n, seed=seed, config=1)
    Us, Vs = synth.update_factors(n, r, T, seed=seed, config=1)
    A, Us, Vs = storage_inputs(A64, Us, Vs, np_t)
    view = lv.View(dev(A, t_t), k, r_max=r, mode=mode)
    powers = [view.read(i).clone() for i in view.powers()]   # caller-held copies
    P = O.reeval(A, k)
    for t in range(T):
        U, V = dev(Us[t], t_t), dev(Vs[t], t_t)
        view.update(U, V)
        lv.lv_powers_update_noalloc(powers, U, V, mode)
        P = O.incr_update(P, Us[t], Vs[t])
    torch.cuda.synchronize()
    tol = 1e-10 if mode == lv.LV_FP64 else 1e-4
    for j, i in enumerate(view.powers()):
        ref = view.read(i)
        assert torch.equal(powers[j], ref), f"A^{i} differs from lv_view_update"
        err = O.maxrel(powers[j].double().cpu().numpy(), P[i])
        assert err < tol, f"A^{i}: maxrel {err:.2e}"
    view.close()


@pytest.mark.parametrize("modename", ["fp32", "fp64"])
def test_noalloc_equals_view_update_twice(modename):
    need_gpu()
    import torch
    from paper_1403_6968_amd import linview as lv
    mode = lv.LV_FP32 if modename == "fp32" else lv.LV_FP64
    _run(lv, torch, 1024, 16, 2, mode, 4, 61)     # first call: the larger shape
    _run(lv, torch, 512, 8, 1, mode, 3, 62)       # then a smaller one on the same scratch


def test_noalloc_rejects_bad_shapes():
    need_gpu()
    import torch
    from paper_1403_6968_amd import linview as lv
    P = [torch.zeros(300, 300, device="cuda") for _ in range(3)]
    u = torch.zeros(300, 1, device="cuda")
    with pytest.raises(lv.LinviewError):          # n not a multiple of 256
        lv.lv_powers_update_noalloc(P, u, u, lv.LV_FP32)
    P = [torch.zeros(16384, 16384, device="cuda") for _ in range(2)]
    u = torch.zeros(16384, 64, device="cuda")
    with pytest.raises(lv.LinviewError, match="scratch"):   # beyond the static array
        lv.lv_powers_update_noalloc(P, u, u, lv.LV_FP32)
