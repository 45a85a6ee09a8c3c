"""Pins of the general-form oracle (T_{i+1} = A T_i + B, Sec. 5.3, Table 1)
against facts other than itself: the plain iteration T_{i+1} = A T_i + B
run step by step (exact rationals on integers, and in floating point), the
B = 0 case T_k = A^k T_0, the unrolled identity T_k = A^k T_0 + S_k B, the
hybrid deltas against re-evaluation, and planted mistakes."""

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


def _iterate(Af, T0f, Bf, k):
    """T_1 .. T_k by the plain iteration, in exact rationals."""
    out, T = {}, T0f
    for i in range(1, k + 1):
        T = Af.dot(T) + Bf
        out[i] = T
    return out


def _case(n, p, seed):
    A = synth.integer_matrix((n, n), -1, 1, seed=seed)
    T0 = synth.integer_matrix((n, p), -2, 2, seed=seed, tag=3)
    B = synth.integer_matrix((n, p), -2, 2, seed=seed, tag=4)
    return A, T0, B


@pytest.mark.parametrize("n,p,k", [(3, 1, 1), (4, 2, 4), (4, 3, 8), (5, 1, 16)])
def test_reeval_general_exact_iteration(n, p, k):
    A, T0, B = _case(n, p, 30 + n + k)
    T = O.reeval_general(A, T0, B, k)
    ref = _iterate(_frac(A), _frac(T0), _frac(B), k)
    for i in T:
        assert (_frac(T[i]) == ref[i]).all(), i


def test_reeval_general_zero_b_is_power_times_t0():
    A = synth.gaussian_matrix(30, seed=31)
    T0 = synth.rng(31, 0, 5).standard_normal((30, 4))
    T = O.reeval_general(A, T0, np.zeros((30, 4)), 16)
    P = O.reeval(A, 16)
    assert max(np.abs(T[i] - P[i] @ T0).max() for i in T) < 1e-13


def test_reeval_general_unrolled_identity():
    A = synth.gaussian_matrix(40, seed=32)
    g = synth.rng(32, 0, 5)
    T0, B = g.standard_normal((40, 3)), g.standard_normal((40, 3))
    k = 16
    T, P, S = O.reeval_general(A, T0, B, k), O.reeval(A, k), O.reeval_sums(A, k)
    assert np.abs(T[k] - (P[k] @ T0 + S[k] @ B)).max() < 1e-12


def _exact_incr(fn, n, p, k, r, seed):
    A, T0, B = _case(n, p, seed)
    U = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=1)
    V = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=2)
    P, S, T = O.reeval(A, k), O.reeval_sums(A, k), O.reeval_general(A, T0, B, k)
    _, _, Tn = fn(P, S, T, T0, B, U, V)
    ref = _iterate(_frac(A + U @ V.T), _frac(T0), _frac(B), k)
    return all((_frac(Tn[i]) == ref[i]).all() for i in Tn)


@pytest.mark.parametrize("seed", range(4))
def test_incr_general_exact(seed):
    assert _exact_incr(O.incr_update_general, n=4, p=1 + seed % 3, k=8, r=1 + seed % 2, seed=seed)


def test_incr_general_many_updates():
    n, p, k, T_ = 25, 3, 16, 6
    A = synth.gaussian_matrix(n, seed=33)
    g = synth.rng(33, 0, 5)
    T0, B = g.standard_normal((n, p)), g.standard_normal((n, p))
    Us, Vs = synth.update_factors(n, 2, T_, seed=33)
    P, S, T = O.reeval(A, k), O.reeval_sums(A, k), O.reeval_general(A, T0, B, k)
    for t in range(T_):
        P, S, T = O.incr_update_general(P, S, T, T0, B, Us[t], Vs[t])
    R = O.reeval_general(A + np.einsum("tir,tjr->ij", Us, Vs), T0, B, k)
    assert max(O.maxrel(T[i], R[i]) for i in R) < 1e-12


def _mutant(kind):
    def fn(P, S, T, T0, B, U, V):
        dQ, dW, dU, dV = O.incr_sums_factors(P, S, U, V)
        D = {1: U @ (V.T @ T0)}
        for i in O.levels(max(P))[1:]:
            h = i // 2
            Th = T[h] if kind == "old_t" else T[h] + D[h]
            term_p = P[h] @ D[h]
            if kind == "new_power":
                term_p = (P[h] + dU[h] @ dV[h].T) @ D[h]
            term_s = dQ[h] @ (dW[h].T @ B)
            if kind == "drop_sums":
                term_s = 0
            D[i] = term_p + dU[h] @ (dV[h].T @ Th) + term_s
        return P, S, {i: T[i] + D[i] for i in T}
    return fn


@pytest.mark.parametrize("kind", ["old_t", "new_power", "drop_sums"])
def test_general_pins_catch_planted_mistakes(kind):
    caught = not all(_exact_incr(_mutant(kind), n=4, p=2, k=8, r=1 + s % 2, seed=s) for s in range(4))
    assert caught, kind


def test_general_unmutated_copy_passes():
    assert all(_exact_incr(_mutant("none"), n=4, p=2, k=8, r=1 + s % 2, seed=s) for s in range(4))


def test_iterate_general_matches_exact_iteration():
    """The floating-point defining iteration (used for full-size checks)
    agrees with the exact rational iteration on integer inputs."""
    A, T0, B = _case(5, 2, 41)
    it = O.iterate_general(A, T0, B, 8)
    ref = _iterate(_frac(A), _frac(T0), _frac(B), 8)
    assert sorted(it) == [1, 2, 4, 8]
    for i in it:
        assert (_frac(it[i]) == ref[i]).all(), i


# ---- factored (incremental) deltas of App. B


@pytest.mark.parametrize("n,p,k,r,seed", [(4, 2, 8, 1, 50), (5, 1, 16, 2, 51), (4, 3, 4, 1, 52), (3, 2, 2, 2, 53)])
def test_factored_general_exact_iteration(n, p, k, r, seed):
    A, T0, B = _case(n, p, seed)
    U = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=5)
    V = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=6)
    _, _, Tn = O.incr_update_general_factored(O.reeval(A, k), O.reeval_sums(A, k), O.reeval_general(A, T0, B, k),
                                              T0, B, U, V)
    ref = _iterate(_frac(A + U @ V.T), _frac(T0), _frac(B), k)
    for i in Tn:
        assert (_frac(Tn[i]) == ref[i]).all(), i


def test_factored_widths_and_agreement_with_hybrid():
    n, p, k, r = 20, 3, 16, 2
    A = synth.gaussian_matrix(n, seed=54)
    T0, B = synth.general_operands(n, p, seed=54)
    U, V = synth.update_factors(n, r, 1, seed=54)
    P, S, T = O.reeval(A, k), O.reeval_sums(A, k), O.reeval_general(A, T0, B, k)
    Y, Z = O.incr_general_factors(P, S, T, T0, B, U[0], V[0])
    c = {1: r}
    for i in O.levels(k)[1:]:
        h = i // 2
        c[i] = h * r + c[h] + max(h - 1, 1) * r
    for i in Y:
        assert Y[i].shape == (n, c[i]) and Z[i].shape == (p, c[i])
    _, _, Th = O.incr_update_general(P, S, T, T0, B, U[0], V[0])
    _, _, Tf = O.incr_update_general_factored(P, S, T, T0, B, U[0], V[0])
    for i in Th:
        assert O.maxrel(Tf[i], Th[i]) < 1e-13


def _factored_mutant(kind):
    def fn(P, S, T, T0, B, U, V):
        dQ, dW, dU, dV = O.incr_sums_factors(P, S, U, V)
        n, r = U.shape
        dQ, dW = dict(dQ), dict(dW)
        dQ[1], dW[1] = np.zeros((n, r)), np.zeros((n, r))
        Y, Z = {1: U}, {1: T0.T @ V}
        for i in O.levels(max(P))[1:]:
            h = i // 2
            Th = T[h] + Y[h] @ Z[h].T if kind == "new_t" else T[h]
            cross = 0 if kind == "drop_cross" else dU[h] @ (dV[h].T @ Y[h])
            Y[i] = np.hstack([dU[h], P[h] @ Y[h] + cross, dQ[h]])
            Bt = T0.T if kind == "t0_for_b" else B.T
            Z[i] = np.hstack([Th.T @ dV[h], Z[h], Bt @ dW[h]])
        return {i: T[i] + Y[i] @ Z[i].T for i in T}
    return fn


@pytest.mark.parametrize("kind", ["new_t", "drop_cross", "t0_for_b"])
def test_factored_pins_catch_planted_mistakes(kind):
    caught = False
    for seed in range(3):
        A, T0, B = _case(4, 2, 60 + seed)
        U = synth.integer_matrix((4, 1), -1, 1, seed=60 + seed, tag=5)
        V = synth.integer_matrix((4, 1), -1, 1, seed=60 + seed, tag=6)
        k = 8
        Tn = _factored_mutant(kind)(O.reeval(A, k), O.reeval_sums(A, k), O.reeval_general(A, T0, B, k), T0, B, U, V)
        ref = _iterate(_frac(A + U @ V.T), _frac(T0), _frac(B), k)
        if not all((_frac(Tn[i]) == ref[i]).all() for i in Tn):
            caught = True
    assert caught, kind


def test_factored_unmutated_copy_passes():
    for seed in range(3):
        A, T0, B = _case(4, 2, 60 + seed)
        U = synth.integer_matrix((4, 1), -1, 1, seed=60 + seed, tag=5)
        V = synth.integer_matrix((4, 1), -1, 1, seed=60 + seed, tag=6)
        Tn = _factored_mutant("none")(O.reeval(A, 8), O.reeval_sums(A, 8), O.reeval_general(A, T0, B, 8), T0, B, U, V)
        ref = _iterate(_frac(A + U @ V.T), _frac(T0), _frac(B), 8)
        assert all((_frac(Tn[i]) == ref[i]).all() for i in Tn)


# ---- linear model (App. B): ReevalLin, HybridLin, IncrLin


def _lin_exact(fn, n, p, k, r, seed):
    A, T0, B = _case(n, p, seed)
    U = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=7)
    V = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=8)
    T = O.reeval_general_lin(A, T0, B, k)
    An, Tn = fn(A, T, T0, U, V)
    ref = _iterate(_frac(A + U @ V.T), _frac(T0), _frac(B), k)
    return (_frac(An) == _frac(A + U @ V.T)).all() and all((_frac(Tn[i]) == ref[i]).all() for i in Tn)


def test_reeval_general_lin_is_the_iteration():
    A, T0, B = _case(4, 2, 80)
    T = O.reeval_general_lin(A, T0, B, 7)
    ref = _iterate(_frac(A), _frac(T0), _frac(B), 7)
    assert sorted(T) == list(range(1, 8))
    for i in T:
        assert (_frac(T[i]) == ref[i]).all()


@pytest.mark.parametrize("k,r,seed", [(6, 1, 81), (8, 2, 82), (3, 1, 83)])
def test_general_lin_steps_exact(k, r, seed):
    assert _lin_exact(O.incr_update_general_hybrid_lin, 4, 2, k, r, seed)
    assert _lin_exact(O.incr_update_general_factored_lin, 4, 2, k, r, seed)


@pytest.mark.parametrize("n,p,k", [(5, 1, 8), (7, 3, 16), (4, 6, 4)])
def test_general_lin_operation_counts_match_appendix_b(n, p, k):
    """App. B, linear model, rank-1 updates: incremental evaluation costs
    2np + sum_{i=2..k} (n^2 (i-1) + 3n (i-1) + np (i+1)); hybrid evaluation
    costs 2np + (k - 1)(p n^2 + 6np); re-evaluation k (p n^2 + np)."""
    A = synth.gaussian_matrix(n, seed=84)
    T0, B = synth.general_operands(n, p, seed=84)
    U, V = synth.update_factors(n, 1, 1, seed=84)
    T = O.reeval_general_lin(A, T0, B, k)
    ci, ch, cr = O.OpCounter(), O.OpCounter(), O.OpCounter()
    O.incr_update_general_factored_lin(A, T, T0, U[0], V[0], ci)
    O.incr_update_general_hybrid_lin(A, T, T0, U[0], V[0], ch)
    O.reeval_general_lin(A, T0, B, k, cr)
    assert ci.ops == 2 * n * p + sum(n * n * (i - 1) + 3 * n * (i - 1) + n * p * (i + 1) for i in range(2, k + 1))
    assert ch.ops == 2 * n * p + (k - 1) * (p * n * n + 6 * n * p)
    assert cr.ops == k * (p * n * n + n * p)


def _lin_mutant(kind):
    def fn(A, T, T0, U, V):
        An = A + U @ V.T
        D = {1: U @ (V.T @ T0)}
        for i in range(2, max(T) + 1):
            Am = An if kind == "new_a" else A
            t3 = 0 if kind == "drop_cross" else U @ (V.T @ D[i - 1])
            Tp = T[i - 1] + D[i - 1] if kind == "new_t" else T[i - 1]
            D[i] = U @ (V.T @ Tp) + Am @ D[i - 1] + t3
        return An, {i: T[i] + D[i] for i in T}
    return fn


@pytest.mark.parametrize("kind", ["new_a", "drop_cross", "new_t"])
def test_general_lin_pins_catch_planted_mistakes(kind):
    assert not all(_lin_exact(_lin_mutant(kind), 4, 2, 6, 1, s) for s in range(85, 88)), kind


def test_general_lin_unmutated_copy_passes():
    assert all(_lin_exact(_lin_mutant("none"), 4, 2, 6, 1, s) for s in range(85, 88))


# ---- skip-s model (Table 1, App. B): exponential up to T_s, then steps of s


def _skip_state(A, T0, B, k, s):
    return O.reeval(A, s), O.reeval_sums(A, s), O.reeval_general_skip(A, T0, B, k, s)


@pytest.mark.parametrize("k,s", [(8, 2), (8, 1), (16, 4), (4, 4), (12, 4)])
def test_reeval_general_skip_is_the_iteration(k, s):
    A, T0, B = _case(4, 2, 70 + k + s)
    T = O.reeval_general_skip(A, T0, B, k, s)
    assert sorted(T) == O.skip_indices(k, s)
    ref = _iterate(_frac(A), _frac(T0), _frac(B), k)
    for i in T:
        assert (_frac(T[i]) == ref[i]).all(), i


def test_skip_indices_and_validation():
    assert O.skip_indices(16, 4) == [1, 2, 4, 8, 12, 16]
    assert O.skip_indices(8, 1) == [1, 2, 3, 4, 5, 6, 7, 8]
    assert O.skip_indices(8, 8) == [1, 2, 4, 8]
    for k, s in [(8, 3), (8, 16), (6, 4)]:
        with pytest.raises(ValueError):
            O.skip_indices(k, s)


def _skip_exact(fn, n, p, k, s, r, seed):
    A, T0, B = _case(n, p, seed)
    U = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=8)
    V = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=9)
    P, S, T = _skip_state(A, T0, B, k, s)
    Tn = fn(P, S, T, T0, B, U, V, s)
    ref = _iterate(_frac(A + U @ V.T), _frac(T0), _frac(B), k)
    return all((_frac(Tn[i]) == ref[i]).all() for i in Tn)


def _skip_update(P, S, T, T0, B, U, V, s):
    return O.incr_update_general_factored_skip(P, S, T, T0, B, U, V, s)[2]


@pytest.mark.parametrize("k,s,r,seed", [(8, 2, 1, 0), (8, 1, 2, 1), (16, 4, 1, 2), (12, 4, 2, 3), (8, 4, 1, 4)])
def test_skip_factored_exact(k, s, r, seed):
    assert _skip_exact(_skip_update, 4, 2, k, s, r, 80 + seed)


def test_skip_factored_widths_and_many_updates():
    n, p, k, s, r = 30, 3, 16, 4, 2
    A = synth.gaussian_matrix(n, seed=34)
    g = synth.rng(34, 0, 5)
    T0, B = g.standard_normal((n, p)), g.standard_normal((n, p))
    Us, Vs = synth.update_factors(n, r, 5, seed=34)
    P, S, T = _skip_state(A, T0, B, k, s)
    Y, Z = O.incr_general_factors_skip(P, S, T, T0, B, Us[0], Vs[0], s)
    c = {1: r}
    for i in O.levels(s)[1:]:
        c[i] = (i // 2) * r + c[i // 2] + max(i // 2 - 1, 1) * r      # Q_1: a zero block of width r
    for i in range(2 * s, k + 1, s):
        c[i] = c[i - s] + s * r + max(s - 1, 1) * r
    for i in T:
        assert Y[i].shape == (n, c[i]) and Z[i].shape == (p, c[i]), i
    for t in range(5):
        P, S, T = O.incr_update_general_factored_skip(P, S, T, T0, B, Us[t], Vs[t], s)
    R = O.reeval_general_skip(A + np.einsum("tir,tjr->ij", Us, Vs), T0, B, k, s)
    assert max(O.maxrel(T[i], R[i]) for i in R) < 1e-12


def _skip_mutant(kind):
    def fn(P, S, T, T0, B, U, V, s):
        Y, Z = O.incr_general_factors(P, S, {i: T[i] for i in O.levels(s)}, T0, B, U, V)
        dQ, dW, dU, dV = O.incr_sums_factors(P, S, U, V)
        n, r = U.shape
        Qs, Ws = (dQ[s], dW[s]) if s > 1 else (np.zeros((n, r)), np.zeros((n, r)))
        for i in range(2 * s, max(T) + 1, s):
            h = i - s
            Ps = P[s] + dU[s] @ dV[s].T if kind == "new_power" else P[s]
            cross = 0 if kind == "drop_cross" else dU[s] @ (dV[s].T @ Y[h])
            Th = T[h] + Y[h] @ Z[h].T if kind == "new_t" else T[h]
            Y[i] = np.hstack([dU[s], Ps @ Y[h] + cross, Qs])
            Wb = np.zeros_like(Ws) if kind == "drop_sums" else Ws
            Z[i] = np.hstack([Th.T @ dV[s], Z[h], B.T @ Wb])
        return {i: T[i] + Y[i] @ Z[i].T for i in T}
    return fn


@pytest.mark.parametrize("kind", ["new_power", "drop_cross", "new_t", "drop_sums"])
def test_skip_pins_catch_planted_mistakes(kind):
    cases = [(8, 2, 1, 90), (16, 4, 1, 91), (8, 2, 2, 92)]
    assert not all(_skip_exact(_skip_mutant(kind), 4, 2, k, s, r, seed) for k, s, r, seed in cases), kind


def test_skip_unmutated_copy_passes():
    cases = [(8, 2, 1, 90), (16, 4, 1, 91), (8, 2, 2, 92)]
    assert all(_skip_exact(_skip_mutant("none"), 4, 2, k, s, r, seed) for k, s, r, seed in cases)
