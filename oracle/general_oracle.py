"""FP64 oracle: the general iterative form T_{i+1} = A T_i + B.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 5.3 and Table 1 (general form column, exponential model):

    T_1 = A T_0 + B,    T_i = P_{i/2} T_{i/2} + S_{i/2} B   for i = 2, 4, ..., k,

with the powers P_i and the sums S_i of the exponential model; T is n x p.

Hybrid evaluation (Sec. 5.3.2, "Hybrid evaluation") keeps the change of every
T_i as one n x p matrix D_i instead of factors.  By the delta rule of
Sec. 4.1 with old operands (the same expansion as the factored form of
App. B, multiplied out), for Delta A = U V^T, Delta P_i = U_i V_i^T and
Delta S_i = Q_i W_i^T:

    D_1 = U (V^T T_0),
    D_i = P_h D_h + U_h (V_h^T (T_h + D_h)) + Q_h (W_h^T B),   h = i/2,

where P_h and T_h are the old values.

Incremental evaluation keeps the change of T_i factored instead,
Delta T_i = Y_i Z_i^T (App. B, exponential model, in our names):

    Y_1 = U,  Z_1 = T_0^T V,
    Y_i = [U_h, P_h Y_h + U_h (V_h^T Y_h), Q_h],
    Z_i = [T_h^T V_h, Z_h, B^T W_h],                     h = i/2,

all from the old values, with Q_1 = W_1 = 0 taken as blocks of width r (as
the paper counts them) and Q_h of its own width r (h - 1) above: widths
c_1 = r, c_2 = 3r, c_{2h} = h r + c_h + (h - 1) r; every T_i then takes
T_i += Y_i Z_i^T.  (The paper's count (2i - 1) r also takes Q_h as h r wide;
zero columns change no product.)

Skip-s model (Table 1, general form column; App. B): the exponential model
up to T_s, then T_{js} = P_s T_{(j-1)s} + S_s B for j = 2 .. k/s, so that
the same expansion with h = (j - 1)s and the top-level factors gives

    Y_{js} = [U_s, P_s Y_h + U_s (V_s^T Y_h), Q_s],
    Z_{js} = [T_h^T V_s, Z_h, B^T W_s],

widths c_{js} = c_h + s r + (s - 1) r (Q_1 again a zero block of width r).
"""

from __future__ import annotations

import numpy as np

from .linview_oracle import OpCounter, levels, reeval
from .sums_oracle import incr_sums_factors, reeval_sums


def iterate_general(A: np.ndarray, T0: np.ndarray, B: np.ndarray, k: int) -> dict[int, np.ndarray]:
    """T_1, T_2, T_4, ..., T_k by the defining iteration T_{i+1} = A T_i + B
    (Sec. 5.3), one step at a time: k products of A with an n x p matrix,
    cheap enough for full-size checks where the powers are not formed."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    want = set(levels(k))
    out, T = {}, np.asarray(T0, dtype=np.float64)
    for i in range(1, k + 1):
        T = A @ T + B
        if i in want:
            out[i] = T
    return out


def reeval_general(A: np.ndarray, T0: np.ndarray, B: np.ndarray, k: int) -> dict[int, np.ndarray]:
    """T_1, T_2, T_4, ..., T_k by the exponential model of Table 1."""
    A = np.asarray(A, dtype=np.float64)
    P, S = reeval(A, k), reeval_sums(A, k)
    T = {1: A @ T0 + B}
    for i in levels(k)[1:]:
        h = i // 2
        T[i] = P[h] @ T[h] + S[h] @ B
    return T


def incr_update_general(P, S, T, T0, B, U, V):
    """Hybrid IncrExp step for the powers, the sums and T (module
    docstring).  All deltas from the old values, then every stored matrix
    takes its delta.  Returns (P', S', T')."""
    dQ, dW, dU, dV = incr_sums_factors(P, S, U, V)
    D = {1: U @ (V.T @ T0)}
    for i in levels(max(P))[1:]:
        h = i // 2
        D[i] = P[h] @ D[h] + dU[h] @ (dV[h].T @ (T[h] + D[h])) + dQ[h] @ (dW[h].T @ B)
    Pn = {i: P[i] + dU[i] @ dV[i].T for i in P}
    Sn = {i: S[i] + dQ[i] @ dW[i].T for i in S}
    Tn = {i: T[i] + D[i] for i in T}
    return Pn, Sn, Tn


def incr_general_factors(P, S, T, T0, B, U, V):
    """Factored deltas Delta T_i = Y_i Z_i^T of the general form (module
    docstring, App. B), from the old powers, sums and T.  Q_1 and W_1 are
    zero blocks of width r, as the paper counts them.  Returns (Y, Z)."""
    dQ, dW, dU, dV = incr_sums_factors(P, S, U, V)
    n, r = np.asarray(U).shape
    dQ = dict(dQ)
    dW = dict(dW)
    dQ[1], dW[1] = np.zeros((n, r)), np.zeros((n, r))
    Y = {1: np.asarray(U, dtype=np.float64)}
    Z = {1: np.asarray(T0, dtype=np.float64).T @ np.asarray(V, dtype=np.float64)}
    for i in levels(max(P))[1:]:
        h = i // 2
        Y[i] = np.hstack([dU[h], P[h] @ Y[h] + dU[h] @ (dV[h].T @ Y[h]), dQ[h]])
        Z[i] = np.hstack([T[h].T @ dV[h], Z[h], np.asarray(B).T @ dW[h]])
    return Y, Z


def incr_update_general_factored(P, S, T, T0, B, U, V):
    """Incremental (factored) step for the powers, the sums and T: all
    factors from the old values, then every stored matrix takes its delta.
    Returns (P', S', T')."""
    dQ, dW, dU, dV = incr_sums_factors(P, S, U, V)
    Y, Z = incr_general_factors(P, S, T, T0, B, U, V)
    Pn = {i: P[i] + dU[i] @ dV[i].T for i in P}
    Sn = {i: S[i] + dQ[i] @ dW[i].T for i in S}
    Tn = {i: T[i] + Y[i] @ Z[i].T for i in T}
    return Pn, Sn, Tn


def _check_skip(k: int, s: int) -> None:
    if s < 1 or s & (s - 1) or k % s:
        raise ValueError(f"skip model needs s a power of two dividing k, got s={s}, k={k}")


def skip_indices(k: int, s: int) -> list[int]:
    """Indices of the stored T under the skip-s model: 1, 2, 4, .., s, 2s, .., k."""
    _check_skip(k, s)
    return levels(s) + list(range(2 * s, k + 1, s))


def reeval_general_skip(A: np.ndarray, T0: np.ndarray, B: np.ndarray, k: int, s: int) -> dict[int, np.ndarray]:
    """T_1, T_2, .., T_s by the exponential model, then T_2s, .., T_k by
    T_{js} = P_s T_{(j-1)s} + S_s B (skip-s model of Table 1)."""
    _check_skip(k, s)
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    T = reeval_general(A, T0, B, s)
    Ps, Ss = reeval(A, s)[s], reeval_sums(A, s)[s]
    for i in range(2 * s, k + 1, s):
        T[i] = Ps @ T[i - s] + Ss @ B
    return T


def incr_general_factors_skip(P, S, T, T0, B, U, V, s: int):
    """Factored deltas of every stored T under the skip-s model (module
    docstring), from the old powers and sums up to s and the old T.
    Returns (Y, Z)."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    Y, Z = incr_general_factors(P, S, {i: T[i] for i in levels(s)}, T0, B, U, V)
    dQ, dW, dU, dV = incr_sums_factors(P, S, U, V)
    n, r = U.shape
    Qs, Ws = (dQ[s], dW[s]) if s > 1 else (np.zeros((n, r)), np.zeros((n, r)))
    for i in range(2 * s, max(T) + 1, s):
        h = i - s
        Y[i] = np.hstack([dU[s], P[s] @ Y[h] + dU[s] @ (dV[s].T @ Y[h]), Qs])
        Z[i] = np.hstack([T[h].T @ dV[s], Z[h], B.T @ Ws])
    return Y, Z


def incr_update_general_factored_skip(P, S, T, T0, B, U, V, s: int):
    """IncrSkip-s step for the powers and sums up to s and every stored T:
    all factors from the old values, then every stored matrix takes its
    delta.  Returns (P', S', T')."""
    dQ, dW, dU, dV = incr_sums_factors(P, S, U, V)
    Y, Z = incr_general_factors_skip(P, S, T, T0, B, U, V, s)
    Pn = {i: P[i] + dU[i] @ dV[i].T for i in P}
    Sn = {i: S[i] + dQ[i] @ dW[i].T for i in S}
    Tn = {i: T[i] + Y[i] @ Z[i].T for i in T}
    return Pn, Sn, Tn


# ---- the linear model (Sec. 3.2, Table 1): T_{i+1} = A T_i + B stored for
# every i = 1 .. k (App. B, linear model)


def reeval_general_lin(A: np.ndarray, T0: np.ndarray, B: np.ndarray, k: int,
                       counter: OpCounter | None = None) -> dict[int, np.ndarray]:
    """ReevalLin: T_1 .. T_k by the iteration itself (k products with A)."""
    c = counter if counter is not None else OpCounter()
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    out, T = {}, np.asarray(T0, dtype=np.float64)
    for i in range(1, k + 1):
        T = c.add(c.mm(A, T), B)
        out[i] = T
    return out


def incr_update_general_hybrid_lin(A, T, T0, U, V, counter: OpCounter | None = None):
    """HybridLin step (App. B, hybrid evaluation of the linear model): with
    Delta A = U V^T and the old A and T,
        Delta T_1 = U (V^T T_0),
        Delta T_i = U (V^T T_{i-1}) + A Delta T_{i-1} + U (V^T Delta T_{i-1}),
    each Delta T_i one n x p matrix; then T_i += Delta T_i and A += U V^T.
    Returns (A', T')."""
    c = counter if counter is not None else OpCounter()
    A = np.asarray(A, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    D = {1: c.mm(U, c.mm(V.T, np.asarray(T0, dtype=np.float64)))}
    for i in range(2, max(T) + 1):
        t1 = c.mm(U, c.mm(V.T, T[i - 1]))
        t2 = c.mm(A, D[i - 1])
        t3 = c.mm(U, c.mm(V.T, D[i - 1]))
        D[i] = c.add(c.add(t1, t2), t3)
    return A + U @ V.T, {i: T[i] + D[i] for i in T}


def incr_update_general_factored_lin(A, T, T0, U, V, counter: OpCounter | None = None):
    """IncrLin step for the general form (App. B, linear model): factored
    Delta T_i = Y_i Z_i^T with
        Y_1 = U,  Z_1 = T_0^T V,
        Y_i = [U, A Y_{i-1} + U (V^T Y_{i-1})],  Z_i = [T_{i-1}^T V, Z_{i-1}],
    old A and T; widths i r.  Then T_i += Y_i Z_i^T and A += U V^T.
    Returns (A', T')."""
    c = counter if counter is not None else OpCounter()
    A = np.asarray(A, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    Y = {1: U}
    Z = {1: c.mm(np.asarray(T0, dtype=np.float64).T, V)}
    for i in range(2, max(T) + 1):
        Y[i] = np.hstack([U, c.add(c.mm(A, Y[i - 1]), c.mm(U, c.mm(V.T, Y[i - 1])))])
        Z[i] = np.hstack([c.mm(T[i - 1].T, V), Z[i - 1]])
    Tn = {}
    for i in T:
        Tn[i] = T[i] + c.mm(Y[i], Z[i].T)
    return A + U @ V.T, Tn
