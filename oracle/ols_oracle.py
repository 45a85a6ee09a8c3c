"""FP64 oracle: ordinary least squares maintained under rank-1 changes of
the data (Sherman-Morrison).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 5.1 ("Ordinary Least Squares") with the incremental treatment of
Sec. 4 (the Sherman-Morrison formula and the OLS example): X is m x n
(predictors), Y is m x p (responses), Z = X^T X, W = Z^{-1} and the
estimate beta* = W X^T Y.  For Delta X = u v^T (u: m, v: n),

    Delta Z = [v, X^T u + v (u^T u)] [u^T X; v^T] = p1 q1^T + p2 q2^T
    p1 = v,  q1 = X^T u,  p2 = X^T u + v (u^T u),  q2 = v.

The inverse takes the two outer products in turn by Sherman-Morrison,

    Delta_1(W) = -(W p1)(q1^T W) / (1 + q1^T W p1),        W1 = W + Delta_1(W)
    Delta_2(W) = -(W1 p2)(q2^T W1) / (1 + q2^T W1 p2),

so Delta W = r1 s1^T + r2 s2^T = R S^T with s1 = W^T q1, s2 = W1^T q2 and
r1, r2 the rest.  With the old X and W,

    Delta beta* = R S^T X^T Y + W v u^T Y + R S^T v u^T Y.

Both E = Z and E + Delta Z are assumed nonsingular (as the formula
requires).
"""

from __future__ import annotations

import numpy as np


def reeval_ols(X: np.ndarray, Y: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Re-evaluation: W = (X^T X)^{-1} (library inverse) and
    beta* = W X^T Y.  Returns (W, beta)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    W = np.linalg.inv(X.T @ X)
    return W, W @ (X.T @ Y)


def ols_delta_z(X: np.ndarray, u: np.ndarray, v: np.ndarray):
    """The two outer products of Delta Z for Delta X = u v^T (Sec. 5.1):
    returns (p1, q1, p2, q2), each n x 1."""
    u = np.asarray(u, dtype=np.float64).reshape(-1, 1)
    v = np.asarray(v, dtype=np.float64).reshape(-1, 1)
    Xtu = X.T @ u
    return v, Xtu, Xtu + v * (u.T @ u).item(), v


def sherman_morrison(W: np.ndarray, p: np.ndarray, q: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Delta(E^{-1}) for Delta E = p q^T (Sec. 4, Sherman-Morrison) as an
    outer product r s^T: s = W^T q, r = -(W p) / (1 + q^T W p).  Returns
    (r, s)."""
    Wp = W @ p
    lam = -1.0 / (1.0 + (q.T @ Wp).item())
    return lam * Wp, W.T @ q


def incr_update_ols(X: np.ndarray, Y: np.ndarray, W: np.ndarray, beta: np.ndarray,
                    u: np.ndarray, v: np.ndarray):
    """One incremental step for Delta X = u v^T (module docstring): the two
    Sherman-Morrison steps in order, then Delta beta* from the old X and W.
    Returns (X', W', beta')."""
    X = np.asarray(X, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64).reshape(-1, 1)
    v = np.asarray(v, dtype=np.float64).reshape(-1, 1)
    p1, q1, p2, q2 = ols_delta_z(X, u, v)
    r1, s1 = sherman_morrison(W, p1, q1)
    W1 = W + r1 @ s1.T
    r2, s2 = sherman_morrison(W1, p2, q2)
    R = np.hstack([r1, r2])
    S = np.hstack([s1, s2])
    uY = u.T @ Y
    dbeta = R @ (S.T @ (X.T @ Y)) + (W @ v) @ uY + R @ ((S.T @ v) @ uY)
    return X + u @ v.T, W + R @ S.T, beta + dbeta
