"""Pins of the OLS oracle (Sec. 5.1 with the Sherman-Morrison formula of
Sec. 4) against facts other than itself: least squares by a different
method (numpy.linalg.lstsq), the factorisation of Delta Z checked exactly on
integers, Sherman-Morrison against an exact rational inverse, long update
sequences against re-evaluation of the final data, and planted mistakes."""

from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import synth


def _exact_inverse(M):
    """Gauss-Jordan elimination in exact rationals."""
    n = len(M)
    A = [[Fraction(int(M[i][j])) for j in range(n)] + [Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        d = A[c][c]
        A[c] = [x / d for x in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return np.array([[float(A[i][n + j]) for j in range(n)] for i in range(n)])


def _problem(m, n, p, seed):
    g = synth.rng(seed, 0, 90)
    return g.standard_normal((m, n)), g.standard_normal((m, p))


def test_reeval_matches_lstsq():
    X, Y = _problem(60, 12, 3, 1)
    W, beta = O.reeval_ols(X, Y)
    ref = np.linalg.lstsq(X, Y, rcond=None)[0]
    assert np.abs(beta - ref).max() < 1e-12 * np.abs(ref).max() * 10
    assert np.abs(W @ (X.T @ X) - np.eye(12)).max() < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_delta_z_factorisation_exact(seed):
    X = synth.integer_matrix((7, 4), -3, 3, seed=seed)
    u = synth.integer_matrix((7, 1), -2, 2, seed=seed, tag=1)
    v = synth.integer_matrix((4, 1), -2, 2, seed=seed, tag=2)
    p1, q1, p2, q2 = O.ols_delta_z(X, u, v)
    Xn = X + u @ v.T
    assert np.array_equal(p1 @ q1.T + p2 @ q2.T, Xn.T @ Xn - X.T @ X)


def test_sherman_morrison_against_exact_inverse():
    E = np.array([[4.0, 1, 0], [1, 3, 1], [0, 1, 2]])
    p = np.array([[1.0], [0], [2]])
    q = np.array([[0.0], [1], [1]])
    r, s = O.sherman_morrison(_exact_inverse(E), p, q)
    assert np.abs(_exact_inverse(E) + r @ s.T - _exact_inverse(E + p @ q.T)).max() < 1e-15


@pytest.mark.parametrize("seed", range(3))
def test_incremental_step_against_exact_inverse(seed):
    X = synth.integer_matrix((9, 4), -3, 3, seed=10 + seed)
    Y = synth.integer_matrix((9, 2), -3, 3, seed=10 + seed, tag=3)
    u = synth.integer_matrix((9, 1), -1, 1, seed=10 + seed, tag=1)
    v = synth.integer_matrix((4, 1), -1, 1, seed=10 + seed, tag=2)
    Z = X.T @ X
    Xn = X + u @ v.T
    Wex = _exact_inverse(Z)
    _, Wn, bn = O.incr_update_ols(X, Y, Wex, Wex @ (X.T @ Y), u, v)
    Wref = _exact_inverse(Xn.T @ Xn)
    assert np.abs(Wn - Wref).max() < 1e-12 * np.abs(Wref).max()
    bref = Wref @ (Xn.T @ Y)
    assert np.abs(bn - bref).max() < 1e-11 * np.abs(bref).max()


def test_update_sequence_against_reeval():
    m, n, p, T = 80, 16, 4, 12
    X, Y = _problem(m, n, p, 2)
    W, beta = O.reeval_ols(X, Y)
    g = synth.rng(2, 0, 91)
    for t in range(T):
        if t % 2:
            u = np.zeros((m, 1)); u[g.integers(0, m)] = 1.0      # one sample's features change
        else:
            u = g.standard_normal((m, 1)) * 0.3
        v = g.standard_normal((n, 1)) * 0.3
        X, W, beta = O.incr_update_ols(X, Y, W, beta, u, v)
    Wr, br = O.reeval_ols(X, Y)
    assert np.abs(W - Wr).max() < 1e-10 * np.abs(Wr).max()
    assert np.abs(beta - br).max() < 1e-10 * np.abs(br).max()


def _mutant(kind):
    def fn(X, Y, W, beta, u, v):
        u = u.reshape(-1, 1)
        v = v.reshape(-1, 1)
        Xtu = X.T @ u
        p1, q1 = v, Xtu
        p2 = Xtu if kind == "drop_uu" else Xtu + v * (u.T @ u).item()
        q2 = v

        def sm(Wm, p, q):
            Wp = Wm @ p
            lam = (1.0 if kind == "sign" else -1.0) / (1.0 + (q.T @ Wp).item())
            return lam * Wp, Wm.T @ q
        r1, s1 = sm(W, p1, q1)
        W1 = W if kind == "old_w_second" else W + r1 @ s1.T
        r2, s2 = sm(W1, p2, q2)
        R, S = np.hstack([r1, r2]), np.hstack([s1, s2])
        uY = u.T @ Y
        Wmid = W + R @ S.T if kind == "new_w_middle" else W
        cross = 0 if kind == "drop_cross" else R @ ((S.T @ v) @ uY)
        dbeta = R @ (S.T @ (X.T @ Y)) + (Wmid @ v) @ uY + cross
        return X + u @ v.T, W + R @ S.T, beta + dbeta
    return fn


def _mutant_ok(kind):
    m, n, p = 40, 8, 2
    X, Y = _problem(m, n, p, 3)
    W, beta = O.reeval_ols(X, Y)
    g = synth.rng(3, 0, 92)
    u, v = g.standard_normal((m, 1)), g.standard_normal((n, 1))
    Xn, Wn, bn = _mutant(kind)(X, Y, W, beta, u, v)
    Wr, br = O.reeval_ols(Xn, Y)
    return np.abs(Wn - Wr).max() < 1e-9 * np.abs(Wr).max() and np.abs(bn - br).max() < 1e-9 * np.abs(br).max()


@pytest.mark.parametrize("kind", ["sign", "old_w_second", "drop_uu", "new_w_middle", "drop_cross"])
def test_ols_pins_catch_planted_mistakes(kind):
    assert not _mutant_ok(kind), f"pin did not catch mutant {kind}"


def test_ols_unmutated_copy_passes():
    assert _mutant_ok("none")
