"""FP64 oracle: sums of matrix powers S_k = I + A + ... + A^(k-1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 5.2.3 ("Sums of Matrix Powers") and Table 1 give the exponential model

    S_1 = I,     S_i = P_{i/2} S_{i/2} + S_{i/2}   for i = 2, 4, ..., k,

with the powers P_i of the exponential model.  The paper states that the
incremental cost matches that of the powers but omits the derivation.  The
delta rule of Sec. 4.1 (Delta E = E(A + Delta A) - E(A), all operands OLD)
applied to this recurrence, with the power deltas Delta P_i = U_i V_i^T of
App. A and the sum deltas kept factored as Delta S_i = Q_i W_i^T, gives

    Delta S_i = Delta P_h (S_h + Delta S_h) + (P_h + I) Delta S_h,  h = i/2
              = U_h (S_h^T V_h + W_h (Q_h^T V_h))^T + (P_h Q_h + Q_h) W_h^T

so the factors of level i are

    Q_i = [ U_h ,  P_h Q_h + Q_h ],
    W_i = [ S_h^T V_h + W_h (Q_h^T V_h) ,  W_h ],

starting from Delta S_1 = 0 (Q_1, W_1 with no columns): Q_2 = U, W_2 = V,
and the width of Q_i, W_i is r (i - 1).
"""

from __future__ import annotations

import numpy as np

from .linview_oracle import incr_factors, levels, reeval


def reeval_sums(A: np.ndarray, k: int) -> dict[int, np.ndarray]:
    """Re-evaluation of S_1, S_2, S_4, ..., S_k by the exponential model of
    Table 1 (sums of powers column).  Returns {i: S_i}."""
    A = np.asarray(A, dtype=np.float64)
    P = reeval(A, k)
    S = {1: np.eye(A.shape[0])}
    for i in levels(k)[1:]:
        h = i // 2
        S[i] = P[h] @ S[h] + S[h]
    return S


def incr_sums_factors(P: dict[int, np.ndarray], S: dict[int, np.ndarray], U: np.ndarray, V: np.ndarray):
    """Factored deltas Delta S_i = Q_i W_i^T of every stored sum for
    Delta A = U V^T, from the OLD powers and sums (module docstring).
    Returns (dQ, dW, dU, dV): the sum factors and the power factors."""
    dU, dV = incr_factors(P, U, V)
    n = P[1].shape[0]
    dQ = {1: np.zeros((n, 0))}
    dW = {1: np.zeros((n, 0))}
    for i in levels(max(P))[1:]:
        h = i // 2
        Uh, Vh, Qh, Wh = dU[h], dV[h], dQ[h], dW[h]
        dQ[i] = np.hstack([Uh, P[h] @ Qh + Qh])
        dW[i] = np.hstack([S[h].T @ Vh + Wh @ (Qh.T @ Vh), Wh])
    return dQ, dW, dU, dV


def incr_update_sums(P: dict[int, np.ndarray], S: dict[int, np.ndarray], U: np.ndarray, V: np.ndarray):
    """IncrExp for the powers and the sums: all factors from the old values,
    then P_i += U_i V_i^T and S_i += Q_i W_i^T.  Returns (P', S')."""
    dQ, dW, dU, dV = incr_sums_factors(P, S, U, V)
    Pn = {i: P[i] + dU[i] @ dV[i].T for i in P}
    Sn = {i: S[i] + dQ[i] @ dW[i].T for i in S}
    return Pn, Sn
