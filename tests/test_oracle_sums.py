"""Pins of the sums-of-powers oracle (S_k = I + A + ... + A^(k-1), Sec. 5.2.3,
Table 1) against facts other than itself: exact rational brute-force sums,
closed forms (geometric series of a diagonal matrix, the band of a shift
matrix), the telescoping identity (I - A) S_k = I - A^k, the factor widths
r (i - 1), and planted mistakes in copies of the incremental step."""

from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import synth


def _frac(M):
    M = np.asarray(M, dtype=np.float64)
    assert np.all(M == np.round(M))
    return np.array([[Fraction(int(x)) for x in row] for row in M], dtype=object)


def _brute_sum(Af, k):
    """sum_{i<k} A^i in exact rationals, by repeated multiplication."""
    n = Af.shape[0]
    term = np.array([[Fraction(int(a == b)) for b in range(n)] for a in range(n)], dtype=object)
    total = term.copy()
    for _ in range(k - 1):
        term = term.dot(Af)
        total = total + term
    return total


@pytest.mark.parametrize("n,k", [(3, 1), (4, 2), (4, 8), (5, 16)])
def test_reeval_sums_exact_rational(n, k):
    A = synth.integer_matrix((n, n), -1, 1, seed=20 + n + k)
    S = O.reeval_sums(A, k)
    for i in S:
        assert (_frac(S[i]) == _brute_sum(_frac(A), i)).all(), i


@pytest.mark.parametrize("k", [2, 8, 32])
def test_reeval_sums_diagonal_geometric_series(k):
    d = np.array([0.5, -0.3, 0.9, 0.0, 2.0])
    S = O.reeval_sums(np.diag(d), k)
    want = np.where(d == 1.0, k, (1.0 - d ** k) / (1.0 - d))
    assert np.allclose(np.diag(S[k]), want, rtol=1e-13, atol=0)
    assert np.count_nonzero(S[k] - np.diag(np.diag(S[k]))) == 0


@pytest.mark.parametrize("n,k", [(6, 4), (6, 8), (10, 4)])
def test_reeval_sums_shift_band(n, k):
    N = np.eye(n, k=1)                           # N^i has ones on diagonal i
    S = O.reeval_sums(N, k)
    a, b = np.indices((n, n))
    assert np.array_equal(S[k], ((b - a >= 0) & (b - a < k)).astype(float))


def test_reeval_sums_telescoping():
    A = synth.gaussian_matrix(40, seed=21)
    k = 16
    S, P = O.reeval_sums(A, k), O.reeval(A, k)
    I = np.eye(40)
    assert np.abs((I - A) @ S[k] - (I - P[k])).max() < 1e-13


def _exact_incr_sums(fn, n, k, r, seed):
    A = synth.integer_matrix((n, n), -1, 1, seed=seed)
    U = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=1)
    V = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=2)
    P, S = O.reeval(A, k), O.reeval_sums(A, k)
    Pn, Sn = fn(P, S, U, V)
    Anew = _frac(A + U @ V.T)
    for i in Sn:
        if not (_frac(Sn[i]) == _brute_sum(Anew, i)).all():
            return False
    return True


@pytest.mark.parametrize("seed", range(5))
def test_incr_sums_exact_rational(seed):
    assert _exact_incr_sums(O.incr_update_sums, n=4, k=8, r=1 + seed % 3, seed=seed)


def test_incr_sums_widths():
    n, k, r = 12, 32, 3
    A = synth.gaussian_matrix(n, seed=22)
    U, V = synth.update_factors(n, r, 1, seed=22)
    dQ, dW, dU, dV = O.incr_sums_factors(O.reeval(A, k), O.reeval_sums(A, k), U[0], V[0])
    for i in dQ:
        assert dQ[i].shape == (n, r * (i - 1)) and dW[i].shape == (n, r * (i - 1))
        assert dU[i].shape == (n, r * i)


def test_incr_sums_many_updates_and_path_independence():
    n, k, T = 30, 16, 8
    A = synth.gaussian_matrix(n, seed=23)
    Us, Vs = synth.update_factors(n, 2, T, seed=23)
    P, S = O.reeval(A, k), O.reeval_sums(A, k)
    for t in range(T):
        P, S = O.incr_update_sums(P, S, Us[t], Vs[t])
    Afin = A + np.einsum("tir,tjr->ij", Us, Vs)
    R = O.reeval_sums(Afin, k)
    assert max(O.maxrel(S[i], R[i]) for i in R) < 1e-12
    # the same total change as one rank-2T update
    P1, S1 = O.incr_update_sums(O.reeval(A, k), O.reeval_sums(A, k),
                                np.concatenate(list(Us), axis=1), np.concatenate(list(Vs), axis=1))
    assert max(O.maxrel(S1[i], R[i]) for i in R) < 1e-12


def _mutant(kind):
    """Copies of the sums step, each with one planted mistake."""
    def fn(P, S, U, V):
        dU, dV = O.incr_factors(P, U, V)
        n = P[1].shape[0]
        dQ, dW = {1: np.zeros((n, 0))}, {1: np.zeros((n, 0))}
        for i in O.levels(max(P))[1:]:
            h = i // 2
            Uh, Vh, Qh, Wh = dU[h], dV[h], dQ[h], dW[h]
            Sh = S[h] + Qh @ Wh.T if kind == "new_sums" else S[h]
            left = P[h] @ Qh + Qh
            if kind == "drop_identity":
                left = P[h] @ Qh
            right = Sh.T @ Vh + Wh @ (Qh.T @ Vh)
            if kind == "drop_cross":
                right = Sh.T @ Vh
            if kind == "transposed_sum":
                right = Sh @ Vh + Wh @ (Qh.T @ Vh)
            dQ[i] = np.hstack([Uh, left])
            dW[i] = np.hstack([right, Wh])
        return ({i: P[i] + dU[i] @ dV[i].T for i in P}, {i: S[i] + dQ[i] @ dW[i].T for i in S})
    return fn


@pytest.mark.parametrize("kind", ["new_sums", "drop_identity", "drop_cross", "transposed_sum"])
def test_sums_pins_catch_planted_mistakes(kind):
    caught = not all(_exact_incr_sums(_mutant(kind), n=4, k=8, r=1 + s % 2, seed=s) for s in range(4))
    assert caught, f"exact pin did not catch mutant {kind}"


def test_sums_unmutated_copy_passes():
    assert all(_exact_incr_sums(_mutant("none"), n=4, k=8, r=1 + s % 2, seed=s) for s in range(4))
