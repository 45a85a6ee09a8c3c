"""FP64 oracle: matrix powers by re-evaluation and by IncrExp.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation follows the paper.  k = 2^m is the target power; the exponential
model stores P_1 = A, P_2, P_4, ..., P_k with P_i = P_{i/2} P_{i/2}
(Table 1, "Exponential" row of the matrix-powers column).  An update of A is
a low-rank product Delta A = U V^T (Sec. 4.2, factored representation).  The
change of every stored power is kept in factored form
Delta P_i = U_i V_i^T with U_i, V_i of width i * r (Sec. 4.3 and App. A,
exponential model):

    U_1 = U,  V_1 = V
    U_i = [ U_{i/2} ,  P_{i/2} U_{i/2} + U_{i/2} (V_{i/2}^T U_{i/2}) ]
    V_i = [ P_{i/2}^T V_{i/2} ,  V_{i/2} ]

All factors are computed from the OLD powers (the delta of an expression E
is E(A + Delta A) - E(A), Sec. 4.1), and only then is every stored power
updated, P_i += U_i V_i^T (the trigger for A^4 in Sec. 4.4 first assigns
all factors and then applies all "+=" statements).
"""

from __future__ import annotations

import math

import numpy as np


def levels(k: int) -> list[int]:
    """The stored powers 1, 2, 4, ..., k of the exponential model.

    The paper assumes log2(k) is an integer (Table 1 caption); any other k is
    rejected.
    """
    if k < 1 or (k & (k - 1)) != 0:
        raise ValueError(f"k must be a power of two, got {k}")
    out = [1]
    while out[-1] < k:
        out.append(out[-1] * 2)
    return out


class OpCounter:
    """Counts arithmetic operations under the paper's convention (App. A):
    a product of an (a x b) and a (b x c) matrix costs a*b*c, an elementwise
    sum of two (a x b) matrices costs a*b, and "P += U V^T" of rank w on an
    n x n matrix costs n*n*w (the accumulation into P is not counted
    separately, so the rank-1 change of A costs n^2)."""

    def __init__(self) -> None:
        self.ops = 0

    def mm(self, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
        self.ops += X.shape[0] * X.shape[1] * Y.shape[1]
        return X @ Y

    def add(self, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
        self.ops += X.size
        return X + Y

    def rank_update(self, P: np.ndarray, U: np.ndarray, V: np.ndarray) -> np.ndarray:
        self.ops += P.shape[0] * P.shape[1] * U.shape[1]
        return P + U @ V.T


def reeval(A: np.ndarray, k: int) -> dict[int, np.ndarray]:
    """ReevalExp: all stored powers of A by repeated squaring.

    Table 1, exponential model: P_1 = A, P_i = P_{i/2} P_{i/2} for
    i = 2, 4, ..., k (Sec. 5.2).  Returns {i: P_i}.
    """
    A = np.asarray(A, dtype=np.float64)
    P = {1: A.copy()}
    for i in levels(k)[1:]:
        P[i] = P[i // 2] @ P[i // 2]
    return P


def incr_factors(P: dict[int, np.ndarray], U: np.ndarray, V: np.ndarray,
                 counter: OpCounter | None = None):
    """Factored deltas of every stored power for Delta A = U V^T.

    App. A, exponential model, with the compact two-block factors of Sec. 4.3:
    for i = 2, 4, ..., k (all with the OLD powers P_{i/2})

        G   = V_{i/2}^T U_{i/2}
        U_i = [ U_{i/2},  P_{i/2} U_{i/2} + U_{i/2} G ]
        V_i = [ P_{i/2}^T V_{i/2},  V_{i/2} ]

    Returns (dU, dV): dicts {i: U_i}, {i: V_i}, U_i and V_i of width i * r.
    """
    c = counter if counter is not None else OpCounter()
    k = max(P)
    dU = {1: np.asarray(U, dtype=np.float64)}
    dV = {1: np.asarray(V, dtype=np.float64)}
    for i in levels(k)[1:]:
        h = i // 2
        Uh, Vh, Ph = dU[h], dV[h], P[h]
        G = c.mm(Vh.T, Uh)                       # V_{i/2}^T U_{i/2}
        X = c.mm(Ph, Uh)                         # P_{i/2} U_{i/2}
        Z = c.add(X, c.mm(Uh, G))                # P U + U (V^T U)
        Y = c.mm(Ph.T, Vh)                       # P_{i/2}^T V_{i/2}
        dU[i] = np.hstack([Uh, Z])
        dV[i] = np.hstack([Y, Vh])
    return dU, dV


def incr_update(P: dict[int, np.ndarray], U: np.ndarray, V: np.ndarray,
                counter: OpCounter | None = None) -> dict[int, np.ndarray]:
    """IncrExp trigger for one update Delta A = U V^T.

    First all factors from the old powers (incr_factors), then every stored
    power is updated, P_i += U_i V_i^T (trigger of Sec. 4.4; cost accounting
    of App. A).  Returns the new {i: P_i}; the input dict is not modified.
    """
    c = counter if counter is not None else OpCounter()
    dU, dV = incr_factors(P, U, V, c)
    return {i: c.rank_update(P[i], dU[i], dV[i]) for i in P}


def apply_updates(P: dict[int, np.ndarray], Us, Vs) -> dict[int, np.ndarray]:
    """Apply a sequence of updates (U_t, V_t) in order with incr_update."""
    for U, V in zip(Us, Vs):
        P = incr_update(P, U, V)
    return P


def power_rows(A: np.ndarray, k: int, rows) -> np.ndarray:
    """Rows `rows` of A^k by definition: e_i^T A A ... A (k factors),
    evaluated as k - 1 successive vector-matrix products."""
    A = np.asarray(A, dtype=np.float64)
    R = A[np.asarray(rows), :].copy()
    for _ in range(k - 1):
        R = R @ A
    return R


def power_cols(A: np.ndarray, k: int, cols) -> np.ndarray:
    """Columns `cols` of A^k by definition: A A ... A e_l, as k - 1 successive
    matrix-vector products.  Returns an (n x len(cols)) array."""
    A = np.asarray(A, dtype=np.float64)
    C = A[:, np.asarray(cols)].copy()
    for _ in range(k - 1):
        C = A @ C
    return C


def brute_power(A, k: int):
    """A^k as k - 1 successive products A (A (... A)).  Works for float arrays
    and for object arrays of fractions.Fraction (exact arithmetic)."""
    A = np.asarray(A)
    R = A.copy()
    for _ in range(k - 1):
        R = R.dot(A)
    return R


def chain_residuals(P: dict[int, np.ndarray], z: np.ndarray) -> list[float]:
    """How far stored powers are from the exponential model's defining
    relation P_{2i} = P_i P_i (Table 1), probed with a vector z:
    rho_i = max|P_{2i} z - P_i (P_i z)| / max|P_{2i} z| for i = 1, 2, ..., k/2."""
    out = []
    z = np.asarray(z, dtype=np.float64)
    for i in levels(max(P))[:-1]:
        c = P[2 * i] @ z
        b = P[i] @ (P[i] @ z)
        den = float(np.max(np.abs(c)))
        num = float(np.max(np.abs(c - b)))
        out.append(num / den if den > 0 else (math.inf if num > 0 else 0.0))
    return out


def maxrel(X: np.ndarray, R: np.ndarray) -> float:
    """Normwise max-norm relative error max|X - R| / max|R|."""
    X = np.asarray(X, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    den = float(np.max(np.abs(R))) if R.size else 0.0
    num = float(np.max(np.abs(X - R))) if R.size else 0.0
    if den == 0.0:
        return 0.0 if num == 0.0 else math.inf
    return num / den


def deltarel(Xt: np.ndarray, X0: np.ndarray, Rt: np.ndarray, R0: np.ndarray) -> float:
    """Relative error of the accumulated change:
    max|(X_t - X_0) - (R_t - R_0)| / max|R_t - R_0|.  A view that skipped
    updates has a change far from the reference change even when its
    maxrel is small."""
    dX = np.asarray(Xt, dtype=np.float64) - np.asarray(X0, dtype=np.float64)
    dR = np.asarray(Rt, dtype=np.float64) - np.asarray(R0, dtype=np.float64)
    return maxrel(dX, dR)
