"""Helpers for the GPU tests: device availability, tensor transfer and the
oracle-side reference state for a sequence of updates."""

from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle as O


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1403_6968_amd import linview
    linview.load()          # raises if the HIP library is missing: no fallback
    return torch


def note(msg: str) -> None:
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def dev(x: np.ndarray, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t) -> np.ndarray:
    return t.detach().to("cpu").double().numpy()


def read_all(view) -> dict:
    return {i: host(view.read(i)) for i in view.powers()}


def storage_inputs(A64, Us, Vs, np_dtype):
    """Round the FP64 inputs once to the storage type; the oracle then uses
    the float64 values of the rounded numbers (both sides see identical
    inputs)."""
    A = np.asarray(A64, dtype=np_dtype).astype(np.float64)
    U = np.asarray(Us, dtype=np_dtype).astype(np.float64)
    V = np.asarray(Vs, dtype=np_dtype).astype(np.float64)
    return A, U, V


def report(tag, got: dict, ref: dict, base_got=None, base_ref=None):
    out = {}
    for i in ref:
        mr = O.maxrel(got[i], ref[i])
        dr = None
        if base_got is not None:
            dr = O.deltarel(got[i], base_got[i], ref[i], base_ref[i])
        out[i] = (mr, dr)
    note(f"{tag}: " + ", ".join(f"P{i}: maxrel={v[0]:.2e}" + (f" deltarel={v[1]:.2e}" if v[1] is not None else "")
                                  for i, v in out.items()))
    return out
