"""Pins of the linear / skip-s model oracle (Sec. 3.2, Table 1, App. A)
against facts other than itself: exact rational powers by brute force, the
stored-matrix counts of Table 2 (space), App. A's operation counts in closed
form, the degenerate cases (skip-1 is linear, skip-k is exponential), and
planted mistakes."""

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


MODELS = [("lin", 6, None), ("lin", 8, None), ("exp", 8, None), ("skip", 8, 2), ("skip", 12, 4),
          ("skip", 16, 4), ("skip", 8, 1), ("skip", 8, 8)]


@pytest.mark.parametrize("model,k,s", MODELS)
def test_reeval_model_exact_powers(model, k, s):
    A = synth.integer_matrix((4, 4), -1, 1, seed=70 + k)
    P = O.reeval_model(A, model, k, s)
    Af = _frac(A)
    for i in P:
        assert (_frac(P[i]) == O.brute_power(Af, i)).all(), i


def _exact_incr(fn, model, k, s, n, r, seed):
    A = synth.integer_matrix((n, n), -1, 1, seed=seed)
    U = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=1)
    V = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=2)
    P = O.reeval_model(A, model, k, s)
    Pn = fn(P, U, V, model, k, s)
    Anew = _frac(A + U @ V.T)
    return all((_frac(Pn[i]) == O.brute_power(Anew, i)).all() for i in Pn)


@pytest.mark.parametrize("model,k,s", MODELS)
@pytest.mark.parametrize("r", [1, 2])
def test_incr_model_exact_rational(model, k, s, r):
    assert _exact_incr(O.incr_update_model, model, k, s, n=4, r=r, seed=71 + r + k)


def test_stored_matrices_match_table2_space():
    """Table 2 (space, incremental matrix powers): linear keeps k matrices,
    exponential log k + 1, skip-s log s + k/s."""
    assert O.stored_powers("lin", 16) == list(range(1, 17))
    assert O.stored_powers("exp", 16) == [1, 2, 4, 8, 16]
    assert O.stored_powers("skip", 16, 4) == [1, 2, 4, 8, 12, 16]
    for k, s in [(16, 4), (32, 8), (64, 2)]:
        assert len(O.stored_powers("skip", k, s)) == int(np.log2(s)) + k // s
    with pytest.raises(ValueError):
        O.model_steps("skip", 12, 8)
    with pytest.raises(ValueError):
        O.model_steps("exp", 12)


@pytest.mark.parametrize("model,k,s", MODELS)
def test_factor_widths(model, k, s):
    n, r = 7, 3
    A = synth.gaussian_matrix(n, seed=72)
    U, V = synth.update_factors(n, r, 1, seed=72)
    dU, dV = O.incr_model_factors(O.reeval_model(A, model, k, s), U[0], V[0], model, k, s)
    for i in dU:
        assert dU[i].shape == (n, r * i) and dV[i].shape == (n, r * i)


def _lin_closed(n, k):
    return n * n * (k * k + k - 1) + Fraction(3, 2) * n * k * (k - 1)


def _exp_closed(n, k):
    return n * n * (4 * k - 3) + Fraction(n * (k - 1) * (2 * k + 5), 3)


def _skip_closed(n, k, s):
    # the exact form App. A sums to (exponential part to s, then k/s - 1 skip products)
    return (Fraction(k * k, s) + k + 2 * s - 3) * n * n + \
        (Fraction((s - 1) * (2 * s + 5), 3) + Fraction((2 * s + 1) * k * (k - s), 2 * s)) * n


@pytest.mark.parametrize("model,k,s", MODELS)
@pytest.mark.parametrize("n", [3, 6])
def test_operation_counts_match_appendix_a(model, k, s, n):
    A = synth.gaussian_matrix(n, seed=73)
    U, V = synth.update_factors(n, 1, 1, seed=73)
    cnt = O.OpCounter()
    O.incr_update_model(O.reeval_model(A, model, k, s), U[0], V[0], model, k, s, counter=cnt)
    want = {"lin": lambda: _lin_closed(n, k), "exp": lambda: _exp_closed(n, k),
            "skip": lambda: _skip_closed(n, k, s)}[model]()
    assert cnt.ops == want
    assert O.paper_cost(model, n, k, s) == want


def test_models_agree_and_exp_matches_increxp():
    n, k = 20, 16
    A = synth.gaussian_matrix(n, seed=74)
    U, V = synth.update_factors(n, 2, 1, seed=74)
    out = {}
    for model, s in [("lin", None), ("exp", None), ("skip", 4)]:
        P = O.incr_update_model(O.reeval_model(A, model, k, s), U[0], V[0], model, k, s)
        out[model] = P[k]
    ref = O.reeval(A + U[0] @ V[0].T, k)[k]
    for m in out:
        assert O.maxrel(out[m], ref) < 1e-13, m
    Pe = O.incr_update(O.reeval(A, k), U[0], V[0])
    Pm = O.incr_update_model(O.reeval_model(A, "exp", k), U[0], V[0], "exp", k)
    for i in Pe:
        np.testing.assert_array_equal(Pe[i], Pm[i])


def _mutant(kind):
    def fn(P, U, V, model, k, s):
        dU, dV = {1: U}, {1: V}
        for i, a, b in O.model_steps(model, k, s):
            Pa = P[a] + dU[a] @ dV[a].T if kind == "new_pa" else P[a]
            Ua, Va, Ub, Vb = dU[a], dV[a], dU[b], dV[b]
            Z = Pa @ Ub + (0 if kind == "drop_cross" else Ua @ (Va.T @ Ub))
            Y = (P[a].T @ Va) if kind == "y_from_pa" else ((P[b] if kind == "y_untransposed" else P[b].T) @ Va)
            dU[i] = np.hstack([Ua, Z])
            dV[i] = np.hstack([Y, Vb])
        return {i: P[i] + dU[i] @ dV[i].T for i in P}
    return fn


@pytest.mark.parametrize("kind", ["new_pa", "drop_cross", "y_from_pa", "y_untransposed"])
def test_model_pins_catch_planted_mistakes(kind):
    caught = False
    for model, k, s in [("lin", 6, None), ("skip", 8, 2)]:
        for seed in range(3):
            if not _exact_incr(_mutant(kind), model, k, s, n=4, r=1, seed=seed):
                caught = True
    assert caught, f"exact pin did not catch mutant {kind}"


def test_model_unmutated_copy_passes():
    for model, k, s in [("lin", 6, None), ("skip", 8, 2)]:
        for seed in range(3):
            assert _exact_incr(_mutant("none"), model, k, s, n=4, r=1, seed=seed)
