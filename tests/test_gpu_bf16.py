"""BF16-shadow mode (LV_FP32_BF16SHADOW): the tall-skinny products read a
bfloat16 copy of every stored power below the top and multiply on the matrix
cores with float accumulation; storage, rank updates, Gram and factor
assembly stay FP32 (Gram in FP64).

Pins:
  * exactness on integers: walk counts of a DAG and of a permutation plus
    inserted edges are integers below 2^8 in every shadowed power and every
    factor, so bfloat16 holds them exactly and the float sums stay below
    2^24: the result must equal the oracle bit for bit.  This fixes the
    matrix-core operand and result layouts (a transposed or shifted operand
    changes the counts), for 1, 2 and 4 factor blocks of 32 columns.
  * random workloads: maxrel <= 5e-3 (BF16-path tolerance) and deltarel
    <= 5e-2 against the FP64 oracle, and the FP32 view of the same inputs
    is at least as close.
  * shadow refresh on write / re-anchor: an update after replacing A must
    follow the new powers, which the skinny products only see through a
    rewritten shadow."""

from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import dev, need_gpu, note, read_all, storage_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    note(f"start {request.node.nodeid}")
    yield


def _lv():
    need_gpu()
    from paper_1403_6968_amd import linview
    return linview


def _edges(n, r, count, cur, g):
    """count rank-r updates, each inserting r new edges a -> b (U e_a, V e_b)."""
    out = []
    for _ in range(count):
        U = np.zeros((n, r)); V = np.zeros((n, r))
        c = 0
        while c < r:
            a, b = g.integers(0, n, size=2)
            if a != b and cur[a, b] == 0:
                cur[a, b] = 1.0; U[a, c] = 1.0; V[b, c] = 1.0; c += 1
        out.append((U, V))
    return out


def _exact_case(A, k, r, updates, tiles=None):
    lv = _lv()
    import torch
    n = A.shape[0]
    P = O.reeval(A, k)
    big = max(np.abs(P[i]).max() for i in P if i < k)
    for U, V in updates:
        dU, dV = O.incr_factors(P, U, V)
        big = max(big, max(np.abs(x).max() for x in dU.values()), max(np.abs(x).max() for x in dV.values()))
        P = O.incr_update(P, U, V)
        big = max(big, max(np.abs(P[i]).max() for i in P if i < k))
    assert big < 256, "precondition: shadowed powers and factors exact in bfloat16"
    assert np.abs(P[k]).max() < 2 ** 24
    view = lv.View(dev(A, torch.float32), k, r_max=r, mode=lv.LV_FP32_BF16SHADOW)
    if tiles is not None:
        view.set_tile_rows([tiles] * (len(view.powers()) - 1))
    for U, V in updates:
        view.update(dev(U, torch.float32), dev(V, torch.float32))
    got = read_all(view)
    for i in P:
        np.testing.assert_array_equal(got[i], P[i], err_msg=f"P_{i} (tile rows {tiles})")
    note(f"exact: n={n} k={k} r={r}: max entry {max(np.abs(P[i]).max() for i in P):.0f}, "
         f"nonzeros of P_k {int((P[k] != 0).sum())}")
    view.close()


def test_integer_dag_walk_counts_exact():
    n, k = 384, 16
    adj = synth.random_dag(n, 0.028, seed=6)
    g = synth.rng(6, 0, 78)
    cur = adj.copy()
    ups = []
    while len(ups) < 6:
        a, b = sorted(g.integers(0, n, size=2))
        if a != b and cur[a, b] == 0:
            cur[a, b] = 1.0
            u = np.zeros((n, 1)); u[a] = 1.0
            v = np.zeros((n, 1)); v[b] = 1.0
            ups.append((u, v))
    _exact_case(adj, k, 1, ups)


@pytest.mark.parametrize("n,k,r", [(512, 16, 16), (320, 64, 4), (1024, 32, 8)])
def test_integer_permutation_high_rank_exact(n, k, r):
    """Level ranks up to 128 on shadowed levels (1, 2 and 4 factor blocks)."""
    g = synth.rng(7, 0, 79, n)
    A = np.zeros((n, n))
    A[np.arange(n), g.permutation(n)] = 1.0
    cur = A.copy()
    _exact_case(A, k, r, _edges(n, r, 2, cur, g))


# Tile heights whose tiles hold an odd number of 64-row chunks (320, 448,
# 576) or end in a ragged tile with an odd count (n = 1300 pads to 1536:
# 1536 = 3 x 448 + 192).  The skinny pass from the shadow pairs chunks at
# level ranks up to 32; an unguarded second chunk would re-add stale rows
# into Y and write X rows beyond the tile, which the exact integer counts
# expose.
@pytest.mark.parametrize("tiles", [320, 448, 576, 960])
def test_odd_chunk_tiles_exact(tiles):
    n, k, r = 1300, 16, 2
    g = synth.rng(8, 0, 80, tiles)
    A = np.zeros((n, n))
    A[np.arange(n), g.permutation(n)] = 1.0
    cur = A.copy()
    _exact_case(A, k, r, _edges(n, r, 3, cur, g), tiles=tiles)


@pytest.mark.parametrize("tiles", [320, 448])
def test_odd_chunk_tiles_random(tiles):
    lv = _lv()
    import torch
    n, k, r, T = 1300, 16, 4, 6
    A64 = synth.gaussian_matrix(n, seed=44, config=3)
    Us, Vs = synth.update_factors(n, r, T, seed=44, config=3)
    A, Us, Vs = storage_inputs(A64, Us, Vs, np.float32)
    view = lv.View(dev(A, torch.float32), k, r_max=r, mode=lv.LV_FP32_BF16SHADOW)
    view.set_tile_rows([tiles] * 4)
    base = read_all(view)
    P0 = O.reeval(A, k)
    P = P0
    for t in range(T):
        P = O.incr_update(P, Us[t], Vs[t])
        view.update(dev(Us[t], torch.float32), dev(Vs[t], torch.float32))
    got = read_all(view)
    view.close()
    for i in P:
        mr, dr = O.maxrel(got[i], P[i]), O.deltarel(got[i], base[i], P[i], P0[i])
        note(f"tiles {tiles} P{i}: maxrel {mr:.2e} deltarel {dr:.2e}")
        assert mr < 5e-3 and dr < 5e-2, f"P_{i}"


# (n, k, r): ragged orders; level ranks from 1 to 128 on shadowed levels
SHAPES = [(300, 16, 1), (777, 16, 3), (520, 8, 16), (256, 64, 4), (1000, 16, 2)]


@pytest.mark.parametrize("n,k,r", SHAPES)
def test_random_updates_within_bf16_tolerance(n, k, r):
    lv = _lv()
    import torch
    T = 12
    A64 = synth.gaussian_matrix(n, seed=40, config=3)
    Us, Vs = synth.update_factors(n, r, T, seed=40, config=3)
    A, Us, Vs = storage_inputs(A64, Us, Vs, np.float32)
    views = {m: lv.View(dev(A, torch.float32), k, r_max=r, mode=m) for m in (lv.LV_FP32, lv.LV_FP32_BF16SHADOW)}
    base = {m: read_all(v) for m, v in views.items()}
    P0 = O.reeval(A, k)
    P = P0
    for t in range(T):
        P = O.incr_update(P, Us[t], Vs[t])
        for v in views.values():
            v.update(dev(Us[t], torch.float32), dev(Vs[t], torch.float32))
    err = {}
    for m, v in views.items():
        got = read_all(v)
        err[m] = {i: (O.maxrel(got[i], P[i]), O.deltarel(got[i], base[m][i], P[i], P0[i])) for i in P}
        v.close()
    bf, fp = err[lv.LV_FP32_BF16SHADOW], err[lv.LV_FP32]
    note(f"n={n} k={k} r={r}: " + " ".join(f"P{i}: bf16 {bf[i][0]:.1e}/{bf[i][1]:.1e} fp32 {fp[i][0]:.1e}/{fp[i][1]:.1e}"
                                           for i in P))
    for i in P:
        assert bf[i][0] < 5e-3, f"P_{i} maxrel {bf[i][0]:.3e}"
        assert bf[i][1] < 5e-2, f"P_{i} deltarel {bf[i][1]:.3e}"
        assert fp[i][0] < 1e-4
    # the shadow path is an approximation: its top-level change error is not
    # smaller than the FP32 path's by more than rounding noise
    assert bf[k][1] >= 0.5 * fp[k][1]


def test_write_and_reanchor_refresh_the_shadows():
    lv = _lv()
    import torch
    n, k, r = 640, 16, 2
    A64 = synth.gaussian_matrix(n, seed=41, config=3)
    Us, Vs = synth.update_factors(n, r, 4, seed=41, config=3)
    A, Us, Vs = storage_inputs(A64, Us, Vs, np.float32)
    B, C = (np.asarray(synth.gaussian_matrix(n, seed=s, config=3), dtype=np.float32).astype(np.float64)
            for s in (42, 43))
    view = lv.View(dev(A, torch.float32), k, r_max=r, mode=lv.LV_FP32_BF16SHADOW)
    view.update(dev(Us[0], torch.float32), dev(Vs[0], torch.float32))

    def check(tag, ref):
        got = read_all(view)
        worst = max(O.maxrel(got[i], ref[i]) for i in ref)
        note(f"{tag}: worst maxrel {worst:.2e}")
        assert worst < 5e-3, tag
        return got

    # checkpoint restore: every stored power written (FP32 values of B's chain)
    PB = {i: np.asarray(x, dtype=np.float32).astype(np.float64) for i, x in O.reeval(B, k).items()}
    for i, x in PB.items():
        view.write(i, dev(x, torch.float32))
    view.update(dev(Us[1], torch.float32), dev(Vs[1], torch.float32))
    check("write all + update", O.incr_update(PB, Us[1], Vs[1]))
    # A replaced by C, chain re-evaluated from it
    view.write(1, dev(C, torch.float32))
    view.reanchor()
    view.update(dev(Us[2], torch.float32), dev(Vs[2], torch.float32))
    got = check("write A + re-anchor + update", O.incr_update(O.reeval(C, k), Us[2], Vs[2]))
    # drift check with tau = 0 re-anchors on the device (gated chain + shadows)
    z = dev(synth.rng(41, 3, 9).standard_normal(n), torch.float64)
    view.drift_check(z, tau=0.0)
    view.update(dev(Us[3], torch.float32), dev(Vs[3], torch.float32))
    check("device re-anchor + update", O.incr_update(O.reeval(got[1], k), Us[3], Vs[3]))
    assert view.stats()["drift_reanchors"] == 1
    view.close()


def test_reeval_rejects_shadow_mode():
    lv = _lv()
    import torch
    A = torch.zeros(64, 64, dtype=torch.float32, device="cuda")
    with pytest.raises(lv.LinviewError):
        lv.lv_reeval(A, 4, None, None, lv.LV_FP32_BF16SHADOW, torch.empty_like(A),
                     torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
