"""Pins of the FP64 oracle against facts the paper and mathematics fix.

Every function of `oracle` is checked against something other than itself:
exact rational arithmetic, closed forms, graph path counts found by
enumeration, the paper's printed widths, operation count and memory table,
and invariants.  The mutation tests at the end plant plausible mistakes in
copies of the oracle's IncrExp step and check that the pins catch each one.
"""

from __future__ import annotations

import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return rows


def _frac(M):
    return np.array([[Fraction(int(x)) for x in row] for row in np.asarray(M)], dtype=object)


def _exact_int(M):
    """float64 array of exact integers -> object array of Fractions."""
    M = np.asarray(M, dtype=np.float64)
    assert np.all(M == np.round(M))
    return _frac(M)


# ----------------------------------------------------------------- levels

def test_levels_powers_of_two():
    assert O.levels(1) == [1]
    assert O.levels(16) == [1, 2, 4, 8, 16]
    assert O.levels(256)[-1] == 256 and len(O.levels(256)) == 9
    for bad in (0, 3, 6, 12, -4):
        with pytest.raises(ValueError):
            O.levels(bad)


# ----------------------------------------------------------------- reeval

@pytest.mark.parametrize("n,k", [(1, 8), (3, 2), (4, 4), (4, 8), (2, 16)])
def test_reeval_exact_rational(n, k):
    """Small-integer A: float64 repeated squaring equals exact rational
    brute-force powers (all intermediate integers are far below 2^53)."""
    A = synth.integer_matrix((n, n), -2, 2, seed=n * 100 + k)
    P = O.reeval(A, k)
    Af = _frac(A)
    for i in O.levels(k):
        ref = O.brute_power(Af, i)
        got = _exact_int(P[i])
        assert (got == ref).all(), f"P_{i} differs from the exact power"


@pytest.mark.parametrize("n", [5, 8])
def test_reeval_brute_float(n):
    A = synth.gaussian_matrix(n, seed=3)
    P = O.reeval(A, 16)
    for i in O.levels(16):
        assert O.maxrel(P[i], O.brute_power(A, i)) < 1e-13


@pytest.mark.parametrize("n", [64, 200, 512])
def test_reeval_matches_library_power(n):
    A = synth.gaussian_matrix(n, seed=1)
    P = O.reeval(A, 16)
    for i in O.levels(16):
        assert O.maxrel(P[i], np.linalg.matrix_power(A, i)) < 1e-12


def test_reeval_diagonal():
    d = np.array([0.5, -1.25, 2.0, 0.0, 1.0, -0.75])
    P = O.reeval(np.diag(d), 16)
    for i in O.levels(16):
        np.testing.assert_array_equal(P[i], np.diag(d ** i))


def test_reeval_nilpotent_and_shift():
    n = 7
    J = np.eye(n, k=1)
    P = O.reeval(J, 8)
    for i in O.levels(8):
        np.testing.assert_array_equal(P[i], np.eye(n, k=i))  # zero when i >= n
    T = np.triu(synth.gaussian_matrix(n, seed=4), 1)          # strictly upper
    P = O.reeval(T, 8)
    assert np.all(P[8] == 0.0)


# ----------------------------------------------------------------- incremental

def _exact_incr_check(incr_fn, n=4, k=8, r=2, seed=0):
    """Integer A, U, V: the incremental result must equal the exact rational
    power of A + U V^T at every stored level."""
    A = synth.integer_matrix((n, n), -1, 1, seed=seed)
    U = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=1)
    V = synth.integer_matrix((n, r), -1, 1, seed=seed, tag=2)
    P = O.reeval(A, k)
    Pn = incr_fn(P, U, V)
    Anew = _frac(A) + _frac(U).dot(_frac(V).T)
    for i in O.levels(k):
        if not (np.asarray(Pn[i]) == np.round(np.asarray(Pn[i]))).all():
            return False
        if not (_exact_int(Pn[i]) == O.brute_power(Anew, i)).all():
            return False
    return True


@pytest.mark.parametrize("seed", range(6))
def test_incr_exact_rational(seed):
    assert _exact_incr_check(O.incr_update, n=4, k=8, r=1 + seed % 3, seed=seed)


def test_incr_exact_rational_two_updates():
    n, k = 4, 8
    A = synth.integer_matrix((n, n), -1, 1, seed=11)
    P = O.reeval(A, k)
    Af = _frac(A)
    for t in range(3):
        U = synth.integer_matrix((n, 1), -1, 1, seed=20 + t, tag=1)
        V = synth.integer_matrix((n, 1), -1, 1, seed=20 + t, tag=2)
        P = O.incr_update(P, U, V)
        Af = Af + _frac(U).dot(_frac(V).T)
    for i in O.levels(k):
        assert (_exact_int(P[i]) == O.brute_power(Af, i)).all()


def test_incr_widths_match_paper():
    """Sec. 4.3: rank-1 deltas of A^2, A^4, A^8 have width 2, 4, 8, not the
    uncompacted 3, 9, 27."""
    rows = _read_golden("compact_widths.txt")
    n = 10
    A = synth.gaussian_matrix(n, seed=2)
    U, V = synth.update_factors(n, 1, 1, seed=2)
    dU, dV = O.incr_factors(O.reeval(A, 8), U[0], V[0])
    for power, compact, uncompacted in rows:
        assert dU[int(power)].shape == (n, int(compact))
        assert dV[int(power)].shape == (n, int(compact))
        assert dU[int(power)].shape[1] != int(uncompacted)
    for r in (2, 3):
        U, V = synth.update_factors(n, r, 1, seed=5)
        dU, dV = O.incr_factors(O.reeval(A, 16), U[0], V[0])
        for i in O.levels(16):
            assert dU[i].shape == (n, i * r) and dV[i].shape == (n, i * r)


@pytest.mark.parametrize("c", [0.7, -0.3, 1.1])
def test_incr_closed_form_scaled_identity(c):
    """(cI + u v^T)^k = c^k I + ((c + lam)^k - c^k) / lam * u v^T, lam = v^T u."""
    n, k = 12, 16
    g = synth.rng(7, 0, 9)
    u = g.standard_normal((n, 1)) * 0.3
    v = g.standard_normal((n, 1)) * 0.3
    lam = float((v.T @ u)[0, 0])
    P = O.incr_update(O.reeval(c * np.eye(n), k), u, v)
    for i in O.levels(k):
        ref = c ** i * np.eye(n) + ((c + lam) ** i - c ** i) / lam * (u @ v.T)
        assert O.maxrel(P[i], ref) < 1e-13


def test_incr_closed_form_zero_matrix():
    """A = 0: (u v^T)^k = lam^(k-1) u v^T."""
    n, k = 9, 16
    g = synth.rng(8, 0, 9)
    u = g.standard_normal((n, 1))
    v = g.standard_normal((n, 1)) * 0.2
    lam = float((v.T @ u)[0, 0])
    P = O.incr_update(O.reeval(np.zeros((n, n)), k), u, v)
    for i in O.levels(k):
        assert O.maxrel(P[i], lam ** (i - 1) * (u @ v.T)) < 1e-13


def test_incr_diagonal_update_stays_diagonal():
    n, k = 8, 16
    d = np.linspace(-0.9, 0.9, n)
    e = np.zeros((n, 1)); e[3, 0] = 1.0
    delta = 0.25
    P = O.incr_update(O.reeval(np.diag(d), k), delta * e, e)
    d2 = d.copy(); d2[3] += delta
    for i in O.levels(k):
        assert O.maxrel(P[i], np.diag(d2 ** i)) < 1e-14


def _walk_count(adj, a, b, length):
    """Number of walks of exactly `length` edges from a to b, by explicit
    enumeration of vertex sequences (no matrix products)."""
    n = adj.shape[0]
    count = 0
    for mid in itertools.product(range(n), repeat=length - 1):
        seq = (a,) + mid + (b,)
        if all(adj[seq[t], seq[t + 1]] for t in range(length)):
            count += 1
    return count


def test_incr_dag_edge_insertion_path_counts():
    """Graph reachability (Sec. 5.2 use of matrix powers): inserting edge
    a->b into a DAG is the update u = e_a, v = e_b; every stored power then
    holds exact walk counts, checked against enumeration."""
    n, k = 6, 4
    adj = synth.random_dag(n, 0.5, seed=3)
    a, b = 1, 4
    adj0 = adj.copy(); adj0[a, b] = 0.0
    u = np.zeros((n, 1)); u[a] = 1.0
    v = np.zeros((n, 1)); v[b] = 1.0
    P = O.incr_update(O.reeval(adj0, k), u, v)
    for i in O.levels(k):
        for s in range(n):
            for t in range(n):
                want = adj[s, t] if i == 1 else _walk_count(adj, s, t, i)
                assert P[i][s, t] == want


def test_incr_shift_restore():
    """Remove one superdiagonal entry of the shift matrix J, then restore it
    by a rank-1 update: every P_i becomes J^i exactly."""
    n, k, p = 9, 8, 4
    J = np.eye(n, k=1)
    Jm = J.copy(); Jm[p, p + 1] = 0.0
    u = np.zeros((n, 1)); u[p] = 1.0
    v = np.zeros((n, 1)); v[p + 1] = 1.0
    P = O.incr_update(O.reeval(Jm, k), u, v)
    for i in O.levels(k):
        np.testing.assert_array_equal(P[i], np.eye(n, k=i))


def test_incr_zero_update_is_identity():
    n, k = 16, 16
    A = synth.gaussian_matrix(n, seed=5)
    P = O.reeval(A, k)
    V = synth.update_factors(n, 2, 1, seed=5)[1][0]
    Pn = O.incr_update(P, np.zeros((n, 2)), V)
    for i in O.levels(k):
        np.testing.assert_array_equal(Pn[i], P[i])


def test_incr_agrees_with_reeval_after_many_updates():
    n, k, T = 96, 16, 60
    A = synth.gaussian_matrix(n, seed=6)
    Us, Vs = synth.update_factors(n, 1, T, seed=6)
    P = O.apply_updates(O.reeval(A, k), Us, Vs)
    Acc = A + np.einsum("tir,tjr->ij", Us, Vs)
    R = O.reeval(Acc, k)
    for i in O.levels(k):
        assert O.maxrel(P[i], R[i]) < 1e-12
        # consistency of the stored chain: P_{2i} = P_i P_i
        if 2 * i <= k:
            assert O.maxrel(P[2 * i], P[i] @ P[i]) < 1e-12


def test_incr_delta_rank_bound():
    """rank(Delta P_i) <= i * r (Sec. 4.2/4.3 factored form)."""
    n, k, r = 40, 8, 1
    A = synth.gaussian_matrix(n, seed=7)
    U, V = synth.update_factors(n, r, 1, seed=7, sigma=0.1)
    P0 = O.reeval(A, k)
    P1 = O.incr_update(P0, U[0], V[0])
    for i in O.levels(k):
        s = np.linalg.svd(P1[i] - P0[i], compute_uv=False)
        assert np.sum(s > 1e-12 * s[0]) <= i * r


def test_path_independence():
    """One rank-r update == r rank-1 updates == re-evaluation (Sec. 4.1: the
    delta depends only on A and A + Delta A)."""
    n, k, r = 48, 16, 4
    A = synth.gaussian_matrix(n, seed=8)
    U, V = synth.update_factors(n, r, 1, seed=8, sigma=0.05)
    P0 = O.reeval(A, k)
    one = O.incr_update(P0, U[0], V[0])
    seq = O.apply_updates(P0, [U[0][:, [c]] for c in range(r)], [V[0][:, [c]] for c in range(r)])
    ref = O.reeval(A + U[0] @ V[0].T, k)
    for i in O.levels(k):
        assert O.maxrel(one[i], ref[i]) < 1e-12
        assert O.maxrel(seq[i], ref[i]) < 1e-12


# ----------------------------------------------------------------- op count

def _paper_exp_cost(n, k):
    """App. A closed form for IncrExp under a rank-1 update."""
    return n * n * (4 * k - 3) + (n * (k - 1) * (2 * k + 5)) // 3


@pytest.mark.parametrize("n,k", [(100, 16), (64, 2), (30, 64), (200, 256)])
def test_opcount_matches_paper(n, k):
    """The instrumented oracle performs exactly the paper's operation count
    n^2 (4k - 3) + n (k - 1)(2k + 5) / 3 (App. A), which holds only for the
    compact two-block factors."""
    A = synth.gaussian_matrix(n, seed=9, target_norm=0.9)
    U, V = synth.update_factors(n, 1, 1, seed=9)
    P = O.reeval(A, k)
    cnt = O.OpCounter()
    O.incr_update(P, U[0], V[0], counter=cnt)
    assert cnt.ops == _paper_exp_cost(n, k)


def test_table5_memory_stored_matrices():
    """Table 5: IncrExp memory for A^16 is 10 float64 n x n matrices (the
    m + 1 = 5 stored powers, row and column partitioned), re-evaluation 3."""
    stored = len(O.reeval(np.eye(2), 16))
    for n, reeval_gb, incr_gb in _read_golden("table5_memory.txt"):
        gib = n * n * 8 / 2 ** 30
        assert round(2 * stored * gib, 1) == incr_gb
        assert round(3 * gib, 1) == reeval_gb


# ----------------------------------------------------------------- rows/cols, metrics

def test_power_rows_cols():
    n, k = 50, 16
    A = synth.gaussian_matrix(n, seed=10)
    R = O.reeval(A, k)
    rows, cols = [0, 7, 49], [3, 3, 20]
    for i in O.levels(k):
        assert O.maxrel(O.power_rows(A, i, rows), R[i][rows, :]) < 1e-13
        assert O.maxrel(O.power_cols(A, i, cols), R[i][:, cols]) < 1e-13
    # exact on integer data
    Ai = synth.integer_matrix((5, 5), -1, 1, seed=12)
    ref = O.brute_power(_frac(Ai), 4)
    assert (_exact_int(O.power_rows(Ai, 4, [0, 1, 2, 3, 4])) == ref).all()
    assert (_exact_int(O.power_cols(Ai, 4, [0, 1, 2, 3, 4])) == ref).all()


def test_metrics():
    R = np.array([[1.0, -4.0], [2.0, 0.0]])
    X = R.copy(); X[1, 1] = 0.5
    assert O.maxrel(X, R) == pytest.approx(0.5 / 4.0)
    assert O.maxrel(R, R) == 0.0
    assert O.maxrel(np.zeros(2), np.zeros(2)) == 0.0
    assert math.isinf(O.maxrel(np.ones(2), np.zeros(2)))
    R0 = np.zeros((2, 2)); X0 = np.zeros((2, 2))
    assert O.deltarel(X, X0, R, R0) == pytest.approx(0.125)
    # a stale view (skipped the change) has deltarel 1
    assert O.deltarel(X0, X0, R, R0) == pytest.approx(1.0)


def test_stale_view_caught_by_deltarel_not_maxrel():
    """At the workload's scale, skipping the last 20% of the updates leaves
    maxrel tiny but deltarel large: deltarel is the check that sees it."""
    n, k, T = 128, 16, 50
    A = synth.gaussian_matrix(n, seed=13)
    Us, Vs = synth.update_factors(n, 1, T, seed=13)
    P0 = O.reeval(A, k)
    full = O.apply_updates(P0, Us, Vs)
    stale = O.apply_updates(P0, Us[:40], Vs[:40])
    assert O.maxrel(stale[16], full[16]) < 5e-3
    assert O.deltarel(stale[16], P0[16], full[16], P0[16]) > 0.05


# ----------------------------------------------------------------- mutation tests

def _mutant(kind):
    """Copies of the IncrExp step, each with one planted mistake."""
    def fn(P, U, V):
        k = max(P)
        dU, dV = {1: U}, {1: V}
        Pw = dict(P)
        for i in O.levels(k)[1:]:
            h = i // 2
            Uh, Vh = dU[h], dV[h]
            Ph = Pw[h]
            if kind == "new_powers":      # uses P_{i/2} after its own update
                Ph = P[h] + Uh @ Vh.T
            G = Vh.T @ Uh
            if kind == "gram_transposed":
                G = Uh.T @ Vh
            X = Ph @ Uh
            Z = X + Uh @ G
            if kind == "drop_gram_term":
                Z = X
            if kind == "sign":
                Z = X - Uh @ G
            Y = Ph.T @ Vh
            if kind == "transposed_operand":
                Y = Ph @ Vh
            if kind == "swap_blocks":
                dU[i] = np.hstack([Z, Uh]); dV[i] = np.hstack([Y, Vh])
            else:
                dU[i] = np.hstack([Uh, Z]); dV[i] = np.hstack([Y, Vh])
        return {i: P[i] + dU[i] @ dV[i].T for i in P}
    return fn


@pytest.mark.parametrize("kind", ["new_powers", "gram_transposed", "drop_gram_term",
                                  "sign", "transposed_operand", "swap_blocks"])
def test_pins_catch_planted_mistakes(kind):
    caught = not all(_exact_incr_check(_mutant(kind), n=4, k=8, r=1 + s % 2, seed=s)
                     for s in range(4))
    assert caught, f"exact pin did not catch mutant {kind}"


def test_unmutated_copy_passes():
    assert all(_exact_incr_check(_mutant("none"), n=4, k=8, r=1 + s % 2, seed=s) for s in range(4))


# ----------------------------------------------------------------- chain residuals

def test_chain_residuals_pins():
    """Residuals of the defining relation P_{2i} = P_i P_i: zero (to rounding)
    for a re-evaluated chain, exactly zero on integers, and for a
    perturbation delta * e_a e_b^T of P_i probed with z = e_b the closed form
    of the two residuals that see it."""
    n, k = 30, 16
    A = synth.gaussian_matrix(n, seed=14)
    P = O.reeval(A, k)
    assert max(O.chain_residuals(P, np.ones(n))) < 1e-14
    Ai = synth.integer_matrix((6, 6), -1, 1, seed=15)
    Pi = O.reeval(Ai, 8)
    assert O.chain_residuals(Pi, np.arange(6.0)) == [0.0, 0.0, 0.0]
    # perturb P_2 at (a, b) by delta; z = e_b
    a, b, delta = 2, 5, 0.5
    Q = {i: M.copy() for i, M in P.items()}
    Q[2][a, b] += delta
    z = np.zeros(n); z[b] = 1.0
    res = O.chain_residuals(Q, z)
    c0 = Q[2] @ z                       # rho_1: P_2' z vs A (A z)
    assert res[0] == pytest.approx(delta / np.max(np.abs(c0)), rel=1e-12)
    assert res[2] < 1e-13               # P_8 / P_4 relation untouched
    assert res[1] > 1e-3                # P_4 vs P_2' P_2' sees it
