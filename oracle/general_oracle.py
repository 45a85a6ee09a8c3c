"""FP64 oracle: the general iterative form T_{i+1} = A T_i + B.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 5.4 and Table 1 (general form column, exponential model):

    T_1 = A T_0 + B,    T_i = P_{i/2} T_{i/2} + S_{i/2} B   for i = 2, 4, ..., k,

with the powers P_i and the sums S_i of the exponential model; T is n x p.

Hybrid evaluation (Sec. 5.4, "Hybrid evaluation") keeps the change of every
T_i as one n x p matrix D_i instead of factors.  By the delta rule of
Sec. 4.1 with old operands (the same expansion as the factored form of
App. B, multiplied out), for Delta A = U V^T, Delta P_i = U_i V_i^T and
Delta S_i = Q_i W_i^T:

    D_1 = U (V^T T_0),
    D_i = P_h D_h + U_h (V_h^T (T_h + D_h)) + Q_h (W_h^T B),   h = i/2,

where P_h and T_h are the old values.
"""

from __future__ import annotations

import numpy as np

from .linview_oracle import levels, reeval
from .sums_oracle import incr_sums_factors, reeval_sums


def iterate_general(A: np.ndarray, T0: np.ndarray, B: np.ndarray, k: int) -> dict[int, np.ndarray]:
    """T_1, T_2, T_4, ..., T_k by the defining iteration T_{i+1} = A T_i + B
    (Sec. 5.4), one step at a time: k products of A with an n x p matrix,
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
